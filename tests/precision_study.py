"""Storage-precision study on the Ra = 1e6 melting cavity (Pr 0.02 and 6.2):
FP32, shifted FP16 and shifted BF16 GPU runs against the FP64 CPU oracle.

Not collected by pytest (about a minute of oracle time per Prandtl number);
run on a machine with the GPU:
    python tests/precision_study.py --n 64 --steps 2000 --every 500
Prints, every `every` steps and for each storage format, the largest and RMS
differences of T, f_l and |u| from the oracle and the difference of the mean
liquid fraction.  These are reported numbers, not pass/fail checks.
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

FORMATS = ((W.FP32, "fp32"), (W.FP16S, "fp16s"), (W.BF16S, "bf16s"))


def _errors(got, ref):
    out = {}
    for key in ("T", "fl"):
        d = got[key] - ref[key]
        out[f"max_{key}"] = float(np.abs(d).max())
        out[f"rms_{key}"] = float(np.sqrt(np.mean(d * d)))
    um_g = np.sqrt(got["ux"] ** 2 + got["uy"] ** 2 + got["uz"] ** 2)
    um_r = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2 + ref["uz"] ** 2)
    out["max_u"] = float(np.abs(um_g - um_r).max())
    out["max_u_ref"] = float(um_r.max())
    out["d_mean_fl"] = float(abs(got["fl"].mean() - ref["fl"].mean()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--Pr", type=float, nargs="+", default=[0.02, 6.2])
    args = ap.parse_args()
    from paper_1703_02652_amd import Cavity
    t0 = time.time()
    summary = {}
    for Pr in args.Pr:
        cfg64 = W.precision_cavity(args.n, Pr, precision=W.FP64)
        cavs = {name: Cavity(dict(cfg64, precision=p), device="cuda") for p, name in FORMATS}
        st = oracle.init_state(cfg64)
        for k in range(args.every, args.steps + 1, args.every):
            st = oracle.run(cfg64, st, args.every)
            ref = oracle.fields(cfg64, st)
            for name, cav in cavs.items():
                cav.step(args.every)
                got = {key: v.cpu().numpy() for key, v in
                       cav.fields(names=("T", "fl", "u")).items()}
                row = dict(Pr=Pr, n=args.n, step=k, storage=name, **_errors(got, ref),
                           elapsed_s=round(time.time() - t0, 1))
                print(json.dumps(row), flush=True)
                summary[f"Pr{Pr}_{name}"] = row
        for cav in cavs.values():
            cav.close()
    print(json.dumps(dict(summary="precision study", threads=oracle.threads(), final=summary)),
          flush=True)


if __name__ == "__main__":
    main()
