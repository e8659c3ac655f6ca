"""Long-run parity of the 128^3 melting cavity (Ra 1e5, Pr 0.02, Ste 0.1):
the FP32 GPU run against the FP64 CPU oracle over many steps.

Not collected by pytest (minutes to an hour of oracle time).  Three ways to
run it:
    python tests/long_parity_cavity128.py --steps 10000 --every 1000
        GPU and oracle in lockstep on a machine with the GPU;
    python tests/long_parity_cavity128.py --steps 20000 --every 1000 --record run.npz
        the GPU run alone, saving the mean liquid fraction and the liquid
        fraction field (float32) every `every` steps and the temperature
        field every `t_every` steps;
    python tests/long_parity_cavity128.py --against run.npz
        the oracle alone (no GPU needed), compared with a recorded GPU run.
Prints, every `every` steps, the mean liquid fraction of both, the largest
pointwise liquid-fraction difference, (where recorded) the largest
temperature difference, and the hot-wall Nusselt number of Eq. (65) of both:
the library's (lbpc_budgets) and the oracle's, from the enthalpy its next
step lets in through the x- face.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def _row(k, fl_gpu, fl_ref, T_gpu, T_ref, t0, nu_gpu=None, nu_ref=None):
    row = dict(step=k, mean_fl_gpu=float(np.mean(fl_gpu, dtype=np.float64)),
               mean_fl_oracle=float(fl_ref.mean()),
               max_dfl=float(np.abs(fl_gpu.astype(np.float64) - fl_ref).max()),
               elapsed_s=round(time.time() - t0, 1))
    if T_gpu is not None:
        row["max_dT"] = float(np.abs(T_gpu.astype(np.float64) - T_ref).max())
    if nu_gpu is not None and nu_ref is not None:
        row["nu_gpu"], row["nu_oracle"] = float(nu_gpu), float(nu_ref)
    return row


def _oracle_nusselt(cfg64, st):
    """Eq. (65) on the oracle's state: the enthalpy its next step lets in
    through the x- face (the same step with every other face adiabatic; the
    collision is local, so the x- links see the same post-collision state),
    per wall node, over the conductive flux chi_l C_p,ref dT / nx."""
    one_face = dict(cfg64, face_bc=[W.DIRICHLET] + [W.ADIABATIC] * 5)
    _, hist = oracle.run(one_face, st, 1, history=True)
    chi = cfg64["lambda_l"] / (cfg64["rho0"] * cfg64["cp_ref"])
    dT = cfg64["face_T"][0] - cfg64["T_m"]
    return hist[0, 3] / (cfg64["ny"] * cfg64["nz"]) * cfg64["nx"] / (chi * cfg64["cp_ref"] * dT)


def _summary(args_n, steps, rows):
    return dict(summary="long parity", n=args_n, steps=steps, threads=oracle.threads(),
                max_dfl=max(r["max_dfl"] for r in rows),
                max_d_mean_fl=max(abs(r["mean_fl_gpu"] - r["mean_fl_oracle"]) for r in rows),
                max_rel_dnu=max((abs(r["nu_gpu"] / r["nu_oracle"] - 1.0) for r in rows
                                 if "nu_gpu" in r), default=None))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--t-every", type=int, default=5000)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--record", default=None)
    ap.add_argument("--against", default=None)
    args = ap.parse_args()
    t0 = time.time()
    rows = []

    if args.against:
        rec = np.load(args.against)  # arrays written by --record (no pickles)
        n, every = int(rec["n"]), int(rec["every"])
        steps = rec["steps"]
        cfg64 = W.melting_cavity(n, 1e5, 0.02, 0.1, precision=W.FP64)
        st = oracle.init_state(cfg64)
        done = 0
        for i, k in enumerate(steps):
            st = oracle.run(cfg64, st, int(k) - done)
            done = int(k)
            r = oracle.fields(cfg64, st)
            key = f"T_{int(k)}"
            T_gpu = rec[key] if key in rec.files else None
            nu_gpu = rec["nu"][i] if "nu" in rec.files else None
            nu_ref = _oracle_nusselt(cfg64, st) if nu_gpu is not None else None
            row = _row(int(k), rec["fl"][i], r["fl"], T_gpu, r["T"], t0, nu_gpu, nu_ref)
            rows.append(row)
            print(json.dumps(row), flush=True)
        print(json.dumps(_summary(n, done, rows)), flush=True)
        return

    from paper_1703_02652_amd import Cavity
    cfg64 = W.melting_cavity(args.n, 1e5, 0.02, 0.1, precision=W.FP64)
    cav = Cavity(dict(cfg64, precision=W.FP32), device="cuda")
    if args.record:
        steps, fls, Ts, nus = [], [], {}, []
        for k in range(args.every, args.steps + 1, args.every):
            cav.step(args.every)
            g = cav.fields(names=("T", "fl"))
            nus.append(cav.nusselt())
            steps.append(k)
            fls.append(g["fl"].cpu().numpy().astype(np.float32))
            if k % args.t_every == 0:
                Ts[f"T_{k}"] = g["T"].cpu().numpy().astype(np.float32)
            print(json.dumps(dict(step=k, mean_fl_gpu=float(g["fl"].mean()),
                                  elapsed_s=round(time.time() - t0, 1))), flush=True)
        np.savez_compressed(args.record, n=args.n, every=args.every, steps=np.array(steps),
                            fl=np.stack(fls), nu=np.array(nus), **Ts)
        return

    st = oracle.init_state(cfg64)
    for k in range(args.every, args.steps + 1, args.every):
        cav.step(args.every)
        st = oracle.run(cfg64, st, args.every)
        g = cav.fields(names=("T", "fl"))
        r = oracle.fields(cfg64, st)
        row = _row(k, g["fl"].cpu().numpy(), r["fl"], g["T"].cpu().numpy(), r["T"], t0,
                   cav.nusselt(), _oracle_nusselt(cfg64, st))
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(json.dumps(_summary(args.n, args.steps, rows)), flush=True)


if __name__ == "__main__":
    main()
