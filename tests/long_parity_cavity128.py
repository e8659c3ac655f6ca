"""Long-run parity of the 128^3 melting cavity (Ra 1e5, Pr 0.02, Ste 0.1):
the FP32 GPU run against the FP64 CPU oracle over many steps.

Not collected by pytest (minutes of oracle time); run on a machine with the GPU:
    python tests/long_parity_cavity128.py --steps 10000 --every 1000
Prints, every `every` steps, the mean liquid fraction of both, the largest
pointwise liquid-fraction difference and the largest temperature difference.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--n", type=int, default=128)
    args = ap.parse_args()
    from paper_1703_02652_amd import Cavity
    cfg64 = W.melting_cavity(args.n, 1e5, 0.02, 0.1, precision=W.FP64)
    cav = Cavity(dict(cfg64, precision=W.FP32), device="cuda")
    st = oracle.init_state(cfg64)
    rows = []
    t0 = time.time()
    for k in range(args.every, args.steps + 1, args.every):
        cav.step(args.every)
        st = oracle.run(cfg64, st, args.every)
        g = cav.fields(names=("T", "fl"))
        r = oracle.fields(cfg64, st)
        row = dict(step=k, mean_fl_gpu=float(g["fl"].mean()), mean_fl_oracle=float(r["fl"].mean()),
                   max_dfl=float(np.abs(g["fl"].cpu().numpy() - r["fl"]).max()),
                   max_dT=float(np.abs(g["T"].cpu().numpy() - r["T"]).max()),
                   elapsed_s=round(time.time() - t0, 1))
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(json.dumps(dict(summary="long parity", n=args.n, steps=args.steps, threads=oracle.threads(),
                          max_dfl=max(r["max_dfl"] for r in rows),
                          max_d_mean_fl=max(abs(r["mean_fl_gpu"] - r["mean_fl_oracle"]) for r in rows))),
          flush=True)


if __name__ == "__main__":
    main()
