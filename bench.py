"""Throughput of the coupled D3Q19 / D3Q7 phase-change step on one MI355X.

Headline workload: natural-convection melting in a 128^3 cavity (Ra = 1e5,
Pr = 0.02, Ste = 0.1), D3Q19 MRT flow + D3Q7 MRT enthalpy, FP32 storage and
arithmetic, synthetic initial state (solid at T_m, hot wall at T_h = 1).
One step = the whole fused step for every cell (collisions, buoyancy and
solid-region forcing, streaming with walls, enthalpy -> (T, f_l)) plus its
FP64 budget partials; reductions of the partials run inside the timed region.

Prints one JSON line.  value = MLUPS (million cell updates per second).
Extra figures (256^3 16-bit storage, the 64-cavity batch, the adjoint/forward
cost ratio at 96^3) go into "extras".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell update: the 26 populations read once and written
# once in the storage type (FP64 416, FP32 208, 16-bit populations with an FP32
# g_0 108).  The roofline fraction uses these.
BYTES_PER_CELL = {0: 416, 1: 208, 2: 108, 3: 108}
# Bytes the storage format actually moves: the FP32 format keeps g_0 as an FP32
# value and a 16-bit correction (25 x 4 + 6 = 106 B per copy), the others
# match the algorithmic count.
FORMAT_BYTES_PER_CELL = {0: 416, 1: 212, 2: 108, 3: 108}


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_step_fp32_cavity128.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, rec["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return rec["traffic_bytes_per_launch"] if sha == rec["source_sha256_prefix"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(cav, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cav.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_cavity(cfg, steps, warmup, launch=None, label=""):
    from paper_1703_02652_amd import Cavity
    cav = Cavity(cfg, device="cuda")
    best = None
    if launch:
        cav.set_launch(*launch)
    else:
        best = cav.autotune(10)
    cav.step(warmup)
    dt = timed_steps(cav, steps)
    kern_ms = cav.time_step_kernel(20)
    cells = sum(c["nx"] * c["ny"] * c["nz"] for c in (cfg if isinstance(cfg, list) else [cfg]))
    mlups = cells * steps / dt / 1e6
    log(f"[bench] {label}: {mlups:.0f} MLUPS, {1e3 * dt / steps:.4f} ms/step, kernel "
        f"{kern_ms:.4f} ms, launch {cav.get_launch()} (tuned {best})")
    st = cav.status()
    return cav, dict(mlups=mlups, ms_per_step=1e3 * dt / steps, kernel_ms=kern_ms,
                     launch=list(cav.get_launch()), unstable=int(st.max()))


def precision_errors(n=256, steps=5000):
    """Shifted FP16 / BF16 storage against the FP32 GPU run of the same cavity
    (Ra 1e6, Pr 0.02 and 6.2): max and RMS errors of T, |u| and f_l, and the
    difference of the mean liquid fraction."""
    import torch
    import workloads as W
    from paper_1703_02652_amd import Cavity
    out = {}
    for Pr in (0.02, 6.2):
        ref = None
        for name, prec in (("fp32", W.FP32), ("fp16s", W.FP16S), ("bf16s", W.BF16S)):
            cav = Cavity(W.precision_cavity(n, Pr, precision=prec), device="cuda")
            cav.step(steps)
            f = cav.fields(names=("T", "fl", "u"))
            umag = torch.sqrt(f["ux"] ** 2 + f["uy"] ** 2 + f["uz"] ** 2)
            cur = dict(T=f["T"], fl=f["fl"], u=umag)
            if ref is None:
                ref = cur
            else:
                e = {}
                for k in ("T", "fl", "u"):
                    d = (cur[k] - ref[k]).abs()
                    e[f"max_{k}"] = float(d.max())
                    e[f"rms_{k}"] = float(torch.sqrt((d * d).mean()))
                e["d_mean_fl"] = float((cur["fl"].mean() - ref["fl"].mean()).abs())
                e["max_u_ref"] = float(ref["u"].max())
                out[f"Pr{Pr}_{name}_vs_fp32"] = e
            cav.close()
            del cav
            torch.cuda.empty_cache()
        del ref
    return dict(cells=n**3, steps=steps, errors=out)


def cpu_baseline(cfg, target_s=15.0, max_steps=400):
    """The FP64 CPU oracle on the same workload, a bounded number of steps
    (about target_s seconds, sized from a short probe after one warm-up step)."""
    import oracle
    st = oracle.run(cfg, oracle.init_state(cfg), 1)
    probe = []
    for k in (2, 6):   # per-step cost without the per-call state conversion
        t = time.perf_counter()
        st = oracle.run(cfg, st, k)
        probe.append(time.perf_counter() - t)
    t1 = max((probe[1] - probe[0]) / 4, 1e-3)
    n = int(max(1, min(max_steps, target_s / t1)))
    t = time.perf_counter()
    oracle.run(cfg, st, n)
    dt = time.perf_counter() - t
    cells = cfg["nx"] * cfg["ny"] * cfg["nz"]
    return dict(value=cells * n / dt / 1e6, unit="MLUPS", cores=oracle.threads(), kind="oracle",
                sample=f"{cfg['nx']}x{cfg['ny']}x{cfg['nz']} coupled FP64 oracle, {n} steps "
                       f"from the same initial state ({dt:.1f} s)")


def cpu_scaled():
    """The oracle on the scaled configurations: the 64^3 coupled cavity and the
    1D melting case (64 x 4 x 4, 2000 steps, MRT) in full, on all host cores and
    on one core."""
    import oracle
    import workloads as W
    out = {}
    n_all = oracle.threads()
    try:
        for threads in (n_all, 1):
            oracle.set_threads(threads)
            cfg = W.melting_cavity(64, 1e5, 0.02, 0.1, precision=W.FP64)
            st = oracle.run(cfg, oracle.init_state(cfg), 1)
            steps = 40 if threads > 1 else 8
            t = time.perf_counter()
            oracle.run(cfg, st, steps)
            dt = time.perf_counter() - t
            out[f"cavity64_coupled_{threads}threads"] = dict(
                mlups=64**3 * steps / dt / 1e6, steps=steps, seconds=round(dt, 3))
            c1 = W.stefan_1d(W.MRT)
            t = time.perf_counter()
            oracle.run(c1, oracle.init_state(c1), 2000)
            dt = time.perf_counter() - t
            out[f"melting1d_2000steps_{threads}threads"] = dict(
                mlups=64 * 16 * 2000 / dt / 1e6, seconds=round(dt, 3))
    finally:
        oracle.set_threads(n_all)
    return out


def full_run_128(launch, steps=20000):
    """The 128^3 cavity over its whole run (Fo = 0.2) in one timed call, with the
    liquid fraction and the hot-wall Nusselt number at the end."""
    import torch
    import workloads as W
    from paper_1703_02652_amd import Cavity
    cfg = W.cavity_128(precision=W.FP32)
    cav = Cavity(cfg, device="cuda")
    cav.set_launch(*launch)
    dt = timed_steps(cav, steps)
    b = cav.budgets()
    r = dict(steps=steps, seconds=round(dt, 3), mlups=128**3 * steps / dt / 1e6,
             mean_fl=round(float(b[0, 2]) / 128**3, 6), nusselt_hot_wall=round(float(cav.nusselt(b=b)), 4),
             unstable=int(cav.status().max()))
    cav.close()
    del cav
    # the same run again, untimed, with the budgets every tenth of it: f_l and
    # Nu against Fo, mass drift and the enthalpy balance H(t) - H(0) = inflow
    cav = Cavity(cfg, device="cuda")
    cav.set_launch(*launch)
    b0 = cav.budgets()[0]
    chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
    hist = []
    for k in range(1, 11):
        cav.step(steps // 10)
        b = cav.budgets()
        inflow = float(b[0, 3] - b0[3])
        hist.append(dict(step=k * (steps // 10), fo=round(chi * k * (steps // 10) / 128**2, 5),
                         mean_fl=round(float(b[0, 2]) / 128**3, 6),
                         nusselt=round(float(cav.nusselt(b=b)), 4),
                         mass_drift=float(b[0, 1] / b0[1] - 1.0),
                         enthalpy_balance=float((b[0, 0] - b0[0] - inflow) / max(abs(inflow), 1.0))))
    r["history"] = hist
    cav.close()
    del cav
    torch.cuda.empty_cache()
    return r


def adjoint_ratio(prec, n=96, steps=2000, every=100):
    import torch
    import workloads as W
    from paper_1703_02652_amd import Cavity
    cfg = W.adjoint_cavity(n, precision=prec)
    cav = Cavity(cfg, device="cuda")
    cav.set_wall_T(0, W.hot_wall_field(n, n))
    cav.autotune(5)
    state = cav.save()
    t_fwd = timed_steps(cav, steps)
    cav.load(state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cav.adjoint_forward(steps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cav.adjoint_backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return dict(precision=["fp64", "fp32"][prec], cells=n**3, steps=steps, ckpt_every=every,
                forward_ms_per_step=1e3 * t_fwd / steps,
                backward_ms_per_step=1e3 * (t2 - t1) / steps,
                backward_over_forward=(t2 - t1) / t_fwd,
                total_over_forward=(t2 - t0) / t_fwd)


def table2_history(case=1, fo_end=0.8, samples=8):
    """Sec. 3.3, Table 2 case 1 (160 x 160 x 80, Ra 2.5e4, Pr 0.02, Ste 0.4,
    FP32) run to Fo = 0.8, as the paper's Fig. 12 shows it: the library's
    hot-wall Nusselt number (Eq. (65)) and the mean liquid fraction at eight
    Fourier numbers.  The paper's curves are figures, so this is a record of
    the run, not a comparison."""
    import workloads as W
    from paper_1703_02652_amd import Cavity
    cfg = W.table2_case(case, precision=W.FP32)
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
    lc = cfg["nx"]
    cav = Cavity(cfg, device="cuda")
    cav.autotune(5)
    rows, done, t_run = [], 0, 0.0
    for k in range(1, samples + 1):
        target = int(round(fo_end * k / samples * lc * lc / chi))
        t_run += timed_steps(cav, target - done)
        done = target
        b = cav.budgets()
        rows.append(dict(fo=round(chi * done / lc ** 2, 4), steps=done,
                         nusselt=round(float(b[0, 6]), 4), mean_fl=round(float(b[0, 2]) / n, 6)))
    r = dict(case=case, cells=n, steps=done, mlups=round(n * done / t_run / 1e6, 1),
             launch=list(cav.get_launch()), unstable=int(cav.status().max()), history=rows)
    cav.close()
    return r


def adjoint_line(args):
    """The differentiation workload (96^3, Ra 1e4, Pr 1, Ste 0.1, checkpoint
    every 100 steps) over --steps steps as the main line: backward / forward
    time per step, with the adjoint kernel's roofline."""
    import workloads as W
    prec = W.FP32 if args.workload.endswith("fp32") else W.FP64
    r = adjoint_ratio(prec, steps=args.steps)
    log(f"[bench] adjoint: {r}")
    out = dict(metric=f"adjoint/forward cost ratio ({args.workload})",
               value=round(r["backward_over_forward"], 4), unit="backward time / forward time",
               n_gpus=1, steps=args.steps, warmup=0, ms_per_step=round(r["backward_ms_per_step"], 5),
               higher_is_better=False, scaling="weak", vs_baseline=None,
               dtype="f32" if prec == W.FP32 else "f64", data="synthetic",
               config=dict(workload="adjoint96_Ra1e4_Pr1_Ste0.1_ckpt100", cells=96**3),
               extras=r)
    print(json.dumps(out), flush=True)


def two_d_validations():
    """Sec. 3.2 at the paper's sizes on y-periodic slabs, FP32: solidification
    in a corner (400 x 400, to Fo = 0.25 with l_c = 400) and melting with
    convection (Table 1 on a 128 x 128 slab, Nu of Eq. (65) at the hot wall
    averaged over ten samples in the last 2 % of the steps before Fo = 4, 10,
    20, and the mean liquid fraction)."""
    import math

    import numpy as np
    import torch
    import workloads as W
    from paper_1703_02652_amd import Cavity
    out = {}
    n, chi = 400, 0.2
    cfg = W.corner_solidification(n, chi=chi, precision=W.FP32)
    cav = Cavity(cfg, T0=np.full((n, 1, n), 0.3), device="cuda")
    cav.autotune(5)
    steps = int(round(0.25 * n * n / chi))
    dt = timed_steps(cav, steps)
    fl = cav.fields(names=("fl",))["fl"][:, 0, :].cpu().numpy()   # [z][x]
    diag = float(sum(1.0 - fl[i, i] for i in range(n))) * math.sqrt(2.0)
    out["corner400_fp32"] = dict(
        cells=n * n, steps=steps, fo=0.25, mlups=n * n * steps / dt / 1e6,
        launch=list(cav.get_launch()), liquid_fraction=round(float(fl.mean()), 5),
        solid_depth_mid_row=round(float((1.0 - fl[n // 2]).sum()), 3),
        solid_depth_bisector=round(diag, 3),
        symmetry_max_dfl=float(np.abs(fl - fl.T).max()))
    cav.close()
    del cav
    torch.cuda.empty_cache()

    n = 128
    cfg = W.convection_2d(n, precision=W.FP32)
    chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
    cav = Cavity(cfg, device="cuda")
    cav.autotune(5)
    rec, done, t_run = [], 0, 0.0
    for fo in (4.0, 10.0, 20.0):
        t = int(round(fo * n * n / chi))
        w = max(10, t // 50) // 10 * 10
        t_run += timed_steps(cav, t - w - done)
        nus = []
        for _ in range(10):   # hot-wall inflow only (the cold face may see outflow)
            t_run += timed_steps(cav, w // 10)
            nus.append(cav.nusselt())
        done = t
        rec.append(dict(fo=fo, steps=t, nusselt=round(float(np.mean(nus)), 4),
                        mean_fl=round(float(cav.budgets()[0, 2]) / (n * n), 5)))
    out["convection2d128_fp32"] = dict(cells=n * n, mlups=n * n * done / t_run / 1e6,
                                       launch=list(cav.get_launch()), history=rec,
                                       unstable=int(cav.status().max()))
    cav.close()
    del cav
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="cavity128_fp32",
                    choices=["cavity128_fp32", "cavity256_fp32", "cavity256_fp16s", "cavity256_bf16s",
                             "cavity128_fp64", "batch64_fp32", "adjoint96_fp32", "adjoint96_fp64"],
                    help="cavity timed for the main line (profiling of the other kernels)")
    ap.add_argument("--launch", default=None,
                    help="block,grid,graph_steps,xcd_run instead of autotuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 10 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the lbpc library runs on one GPU (asked for --gpus {args.gpus}); "
              "a multi-GPU decomposition is not implemented", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.calibrate_copy:
        # a plain 1 GiB device copy, 10 times: the counter calibration, and
        # the bandwidth a copy reaches on this GPU (read + write bytes / time)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps(dict(calibrate_copy_bytes=a.numel() * 4, dispatches=11,
                              copy_ms=round(ms, 4),
                              copy_gbs_read_plus_write=round(2 * a.numel() * 4 / (ms * 1e-3) / 1e9, 1))))
        return
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    if args.workload.startswith("adjoint96"):
        adjoint_line(args)
        return

    prec = {"fp32": W.FP32, "fp16s": W.FP16S, "bf16s": W.BF16S, "fp64": W.FP64}[
        args.workload.split("_")[1]]
    if args.workload.startswith("cavity128"):
        cfg = W.cavity_128(precision=prec)
        wl_name = "cavity128_Ra1e5_Pr0.02_Ste0.1"
    elif args.workload.startswith("batch64"):
        cfg, _ = W.batch_cavities(precision=prec)
        wl_name = "batch64_N32-96_Ra1e3-1e6_Pr0.02-50_Ste0.05-0.5"
    else:
        cfg = W.precision_cavity(256, 0.02, precision=prec)
        wl_name = "cavity256_Ra1e6_Pr0.02_Ste0.1"
    cells = sum(c["nx"] * c["ny"] * c["nz"] for c in (cfg if isinstance(cfg, list) else [cfg]))
    cav, main_r = run_cavity(cfg, args.steps, args.warmup, launch=launch, label=args.workload)
    alg_bytes = BYTES_PER_CELL[prec] * cells
    achieved = alg_bytes / (main_r["kernel_ms"] * 1e-3) / 1e9
    step_gbs = alg_bytes / (main_r["ms_per_step"] * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic() if args.workload == "cavity128_fp32" else None,
                    kernel=f"k_step<{args.workload.split('_')[1]}, flow, MRT, wall-inflow partials>",
                    bytes_per_cell=BYTES_PER_CELL[prec], bytes_per_launch=alg_bytes,
                    format_bytes_per_cell=FORMAT_BYTES_PER_CELL[prec],
                    kernel_ms=round(main_r["kernel_ms"], 5),
                    time_source="mean time per step kernel over a captured graph of 14 "
                                "back-to-back wall-inflow-partials steps, HIP events around "
                                "each replay on the library's stream",
                    frac_of_step=round(step_gbs / HBM_PEAK_GBS, 4))
    cav.close()
    del cav

    extras = {}

    def extra(key, fn, *a, **kw):
        """One extra figure: a failure is logged and recorded under its key, so
        that it never costs the main line."""
        try:
            val = fn(*a, **kw)
        except Exception as e:  # noqa: BLE001 - any failure of a side figure
            val = {"error": f"{type(e).__name__}: {e}"}
        finally:
            torch.cuda.empty_cache()
        if isinstance(val, dict) and key is None:
            extras.update(val)
        else:
            extras[key] = val
        log(f"[bench] {key or fn.__name__}: {val}")

    def cavity_extra(c, xs, label):
        cv, r = run_cavity(c, xs, 20, label=label)
        try:
            n = c["nx"] * c["ny"] * c["nz"]
            r["hbm_frac"] = round(BYTES_PER_CELL[c["precision"]] * n / (r["kernel_ms"] * 1e-3)
                                  / 1e9 / HBM_PEAK_GBS, 4)
        finally:
            cv.close()
        return r

    def table2(case, xs):
        c = W.table2_case(case)
        cv, r = run_cavity(c, xs, 20, label=f"table2 case {case}")
        try:
            cv.step(200)
            b = cv.budgets()[0]
            r["after_steps"] = int(b[4])
            r["nusselt_hot_wall"] = round(float(cv.nusselt()), 4)
            r["mean_fl"] = round(float(b[2]) / (c["nx"] * c["ny"] * c["nz"]), 6)
        finally:
            cv.close()
        return r

    def batch64():
        from paper_1703_02652_amd import Cavity
        bcfgs, _ = W.batch_cavities()
        bc = Cavity(bcfgs, device="cuda")
        try:
            bc.autotune(5)
            bc.step(20)
            bsteps = 5000   # the whole run of the batch workload, timed in one call
            dt = timed_steps(bc, bsteps)
            cells = np.array([c["nx"] * c["ny"] * c["nz"] for c in bcfgs], dtype=np.float64)
            bb = bc.budgets()
            fl = bb[:, 2] / cells
            return dict(cells=int(cells.sum()), steps=bsteps,
                        mlups=float(cells.sum()) * bsteps / dt / 1e6, ms_per_step=1e3 * dt / bsteps,
                        launch=list(bc.get_launch()), unstable_cavities=int(bc.status().sum()),
                        mean_fl_min=round(float(fl.min()), 6), mean_fl_max=round(float(fl.max()), 6))
        finally:
            bc.close()

    if not args.no_extras:
        xs = max(50, args.steps // 5)
        for name, xprec in (("cavity256_fp32", W.FP32), ("cavity256_fp16s", W.FP16S),
                            ("cavity256_bf16s", W.BF16S)):
            extra(name, cavity_extra, W.precision_cavity(256, 0.02, precision=xprec), xs, name)
        extra("cavity128_fp64", cavity_extra, W.cavity_128(precision=W.FP64), xs, "cavity128_fp64")
        for case in (1, 2, 3):
            extra(f"table2_case{case}_fp32", table2, case, xs)
        extra("table2_case1_history_fp32", table2_history)
        extra("batch64_fp32", batch64)
        extra("precision256_errors", precision_errors)
        extra("adjoint96_fp32", adjoint_ratio, W.FP32)
        extra("adjoint96_fp64", adjoint_ratio, W.FP64)
        extra("cavity128_full_run_fp32", full_run_128, main_r["launch"])
        extra("adjoint96_fp32_every_step", adjoint_ratio, W.FP32, steps=200, every=1)
        extra(None, two_d_validations)

    cpu = None
    if not args.no_cpu and not isinstance(cfg, list):
        cpu = cpu_baseline(dict(cfg, precision=W.FP64))
        log(f"[bench] cpu baseline: {cpu}")
        if not args.no_extras:
            extra("cpu_oracle_scaled", cpu_scaled)

    out = dict(
        metric=f"coupled flow+enthalpy MLUPS ({args.workload})",
        value=round(main_r["mlups"], 1), unit="MLUPS", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(main_r["ms_per_step"], 5), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64" if prec == W.FP64 else "f32",
        data="synthetic",
        config=dict(workload=wl_name,
                    lattice="D3Q19 MRT + D3Q7 MRT", cells=cells,
                    storage=args.workload.split("_")[1], launch=main_r["launch"]),
        roofline=roofline, cpu_baseline=cpu, extras=extras,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
