"""Write tests/golden/cavity128_oracle.json: the FP64 oracle's run of the
128^3 natural-convection melting cavity (Sec. 3.3 geometry; Ra 1e5, Pr 0.02,
Ste 0.1 with the Mach-0.1 lattice mapping), sampled every 2000 steps up to
20,000: the mean liquid fraction, the hot-wall Nusselt number of Eq. (65)
(from the enthalpy the next step lets in through the x- face) and the liquid
fraction and temperature at 256 seeded cells.

Calls only the oracle (about 90 minutes on 8 host threads):
    python tests/golden/make_cavity128_golden.py [--steps 20000] [--every 2000] [--fields F]
With --fields, the whole liquid-fraction field at every sample and the
temperature field at the last one are also saved to F (numpy .npz, FP64), for
comparisons of a whole recorded run that the JSON's sampled cells cannot make.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "cavity128_oracle.json")


def sample_cells(n, count=256, seed=128):
    """Cells (flat index x + n (y + n z)) drawn without replacement; half of
    them in the eight columns next to the hot wall, where the melt is."""
    rng = np.random.default_rng(seed)
    near = rng.choice(8 * n * n, size=count // 2, replace=False)
    x, yz = near % 8, near // 8
    near = x + n * yz
    rest = rng.choice(n ** 3, size=count - count // 2, replace=False)
    return np.unique(np.concatenate([near, rest]))


def nusselt(cfg, st):
    """Eq. (65): the x- inflow of the next step (the same step with every other
    face adiabatic; the collision is local) per wall node, over the conductive
    flux chi_l C_p,ref dT / nx."""
    one_face = dict(cfg, face_bc=[W.DIRICHLET] + [W.ADIABATIC] * 5)
    _, hist = oracle.run(one_face, st, 1, history=True)
    chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
    dT = cfg["face_T"][0] - cfg["T_m"]
    return hist[0, 3] / (cfg["ny"] * cfg["nz"]) * cfg["nx"] / (chi * cfg["cp_ref"] * dT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=2000)
    ap.add_argument("--fields", default=None)
    args = ap.parse_args()
    n = 128
    cfg = W.melting_cavity(n, 1e5, 0.02, 0.1, precision=W.FP64)
    cells = sample_cells(n)
    st = oracle.init_state(cfg)
    t0 = time.time()
    rows, done, fls = [], 0, []
    for k in range(args.every, args.steps + 1, args.every):
        st = oracle.run(cfg, st, k - done)
        done = k
        f = oracle.fields(cfg, st)
        fl, T = f["fl"].reshape(-1), f["T"].reshape(-1)
        if args.fields:
            fls.append(f["fl"].copy())
        rows.append(dict(step=k, mean_fl=float(fl.mean()), nusselt=float(nusselt(cfg, st)),
                         fl=[float(v) for v in fl[cells]], T=[float(v) for v in T[cells]]))
        print(json.dumps(dict(step=k, mean_fl=rows[-1]["mean_fl"], nusselt=rows[-1]["nusselt"],
                              elapsed_s=round(time.time() - t0, 1))), flush=True)
    doc = dict(
        what="FP64 oracle, 128^3 melting cavity (Sec. 3.3 geometry), Ra 1e5, Pr 0.02, "
             "Ste 0.1, Mach-0.1 lattice mapping; mean liquid fraction, hot-wall Nusselt "
             "number (Eq. (65)) and liquid fraction / temperature at sampled cells",
        writer="tests/golden/make_cavity128_golden.py (oracle only)",
        n=n, every=args.every, cells=[int(c) for c in cells], samples=rows)
    with open(OUT, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {OUT}")
    if args.fields:
        np.savez_compressed(args.fields, steps=np.array([r["step"] for r in rows]),
                            fl=np.stack(fls), T=f["T"], nu=np.array([r["nusselt"] for r in rows]))
        print(f"wrote {args.fields}")


if __name__ == "__main__":
    main()
