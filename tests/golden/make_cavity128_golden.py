"""Write tests/golden/cavity128_oracle.json: the FP64 oracle's run of the
128^3 natural-convection melting cavity (Sec. 3.3 geometry; Ra 1e5, Pr 0.02,
Ste 0.1 with the Mach-0.1 lattice mapping), sampled every 2000 steps up to
20,000: the mean liquid fraction, the hot-wall Nusselt number of Eq. (65)
(from the enthalpy the next step lets in through the x- face) and the liquid
fraction and temperature at 256 seeded cells.  With --workload table2_case1,
the same for case 1 of Table 2 on its 160 x 160 x 80 grid, every 1000 steps up
to 6000, into tests/golden/table2_case1_oracle.json.

Calls only the oracle (about 90 minutes on 8 host threads for the 128^3 run,
30 for the Table 2 one):
    python tests/golden/make_cavity128_golden.py [--workload W] [--steps S] [--every E] [--fields F]
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

WORKLOADS = {
    # name: (configuration, default steps, default sampling interval, output)
    "cavity128": (lambda: W.melting_cavity(128, 1e5, 0.02, 0.1, precision=W.FP64), 20000, 2000,
                  "cavity128_oracle.json"),
    "table2_case1": (lambda: W.table2_case(1, precision=W.FP64), 6000, 1000,
                     "table2_case1_oracle.json"),
}


def sample_cells(nx, ny, nz, count=256, seed=128):
    """Cells (flat index x + nx (y + ny z)) drawn without replacement; half of
    them in the eight columns next to the hot wall, where the melt is."""
    rng = np.random.default_rng(seed)
    near = rng.choice(8 * ny * nz, size=count // 2, replace=False)
    x, yz = near % 8, near // 8
    near = x + nx * yz
    rest = rng.choice(nx * ny * nz, size=count - count // 2, replace=False)
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
    ap.add_argument("--workload", default="cavity128", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--fields", default=None)
    args = ap.parse_args()
    make, steps, every, out_name = WORKLOADS[args.workload]
    args.steps = args.steps or steps
    args.every = args.every or every
    cfg = make()
    n = cfg["nx"]
    cells = sample_cells(cfg["nx"], cfg["ny"], cfg["nz"])
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
    what = ("128^3 melting cavity (Sec. 3.3 geometry), Ra 1e5, Pr 0.02, Ste 0.1"
            if args.workload == "cavity128" else
            "Table 2 case 1 on its 160 x 160 x 80 grid (Ra 2.5e4, Pr 0.02, Ste 0.4)")
    doc = dict(
        what=f"FP64 oracle, {what}, Mach-0.1 lattice mapping; mean liquid fraction, "
             "hot-wall Nusselt number (Eq. (65)) and liquid fraction / temperature at "
             "sampled cells",
        writer="tests/golden/make_cavity128_golden.py (oracle only)",
        n=n, every=args.every, cells=[int(c) for c in cells], samples=rows)
    if args.workload != "cavity128":
        doc.update(shape=[cfg["nx"], cfg["ny"], cfg["nz"]], workload=args.workload)
    out = os.path.join(HERE, out_name)
    with open(out, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {out}")
    if args.fields:
        np.savez_compressed(args.fields, steps=np.array([r["step"] for r in rows]),
                            fl=np.stack(fls), T=f["T"], nu=np.array([r["nusselt"] for r in rows]))
        print(f"wrote {args.fields}")


if __name__ == "__main__":
    main()
