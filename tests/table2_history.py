"""The three 3D melting cases of Sec. 3.3 (Table 2) run to the Fourier numbers
the paper shows (cases 1 and 2 to Fo = 0.8, case 3 to Fo = 0.4), printing the
average Nusselt number on the hot wall (Eq. (65)) and the mean liquid fraction
against Fo (the quantities of the paper's Fig. 12).  FP32 storage, autotuned
launch.

Not collected by pytest (about ten minutes of GPU time, most of it case 3,
whose small diffusivity needs 4.4 million steps); run on a machine with the GPU:
    python tests/table2_history.py [--cases 1,2,3] [--samples 40]
Prints one JSON line per sample and one summary line per case.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import workloads as W  # noqa: E402

FO_END = {1: 0.8, 2: 0.8, 3: 0.4}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="1,2,3")
    ap.add_argument("--samples", type=int, default=40)
    args = ap.parse_args()
    from paper_1703_02652_amd import Cavity
    for case in [int(c) for c in args.cases.split(",")]:
        cfg = W.table2_case(case, precision=W.FP32)
        n = cfg["nx"] * cfg["ny"] * cfg["nz"]
        chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
        lc = cfg["nx"]
        total = int(round(FO_END[case] * lc * lc / chi))
        per = max(16, total // args.samples // 16 * 16)
        cav = Cavity(cfg, device="cuda")
        cav.autotune(10)
        t0 = time.time()
        done, rows = 0, []
        while done < total:
            k = min(per, total - done)
            cav.step(k)
            done += k
            b = cav.budgets()
            row = dict(case=case, step=done, fo=round(chi * done / lc ** 2, 4),
                       nusselt=round(float(cav.nusselt(b=b)), 4),
                       mean_fl=round(float(b[0, 2]) / n, 6), elapsed_s=round(time.time() - t0, 1))
            rows.append(row)
            print(json.dumps(row), flush=True)
        st = int(cav.status().max())
        print(json.dumps(dict(summary="table2", case=case, steps=total, fo_end=FO_END[case],
                              launch=list(cav.get_launch()), unstable=st,
                              mlups=round(n * total / (time.time() - t0) / 1e6),
                              final=rows[-1])), flush=True)
        cav.close()


if __name__ == "__main__":
    main()
