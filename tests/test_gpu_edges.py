"""Edge cases on the GPU: degenerate lattices (one cell, one-cell-thick
dimensions with walls or periodic wrap) against the oracle from arbitrary
states, and the full-size 256^3 cavity in the launch shape the benchmark
tunes, in FP32 and shifted FP16 storage."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import W19, absdiff, make_cavity, random_walls, rel

pytestmark = pytest.mark.gpu

D, A, P = W.DIRICHLET, W.ADIABATIC, W.PERIODIC
# (nx, ny, nz, faces): every link of a 1x1x1 cell hits a wall; thin dimensions
# with walls on both sides; thin periodic dimensions wrap onto the cell itself
DEGENERATE = [
    (1, 1, 1, [D, A, D, A, A, D]),
    (1, 5, 1, [D, D, P, P, A, A]),
    (2, 1, 3, [A, D, P, P, D, A]),
    (3, 2, 1, [P, P, D, D, A, A]),
    (1, 1, 9, [P, P, P, P, D, A]),
]


@pytest.mark.parametrize("case", range(len(DEGENERATE)))
@pytest.mark.parametrize("flow", [0, 1])
def test_degenerate_lattices_match_oracle(case, flow):
    nx, ny, nz, bc = DEGENERATE[case]
    cfg = W.base_config(nx, ny, nz, flow=flow, enth_model=W.MRT, precision=W.FP64, face_bc=bc,
                        face_T=[1.0, -0.4, 0.3, 0.7, 0.9, -0.2], g_beta=4e-3, latent=1.5,
                        lambda_s=0.09, lambda_l=0.09, nu=0.04, cp_l=1.4)
    f, g = W.random_populations(cfg, seed=300 + case, f_scale=W19)
    walls = random_walls(cfg, seed=400 + case)
    tw = W.wall_fields(cfg, walls)
    cav = make_cavity(cfg, walls=walls)
    cav.set_state(f, g)
    cav.step(7)
    st = oracle.run(cfg, (f if flow else None, g), 7, tw=tw)
    fg, gg = cav.state()
    print(f"{nx}x{ny}x{nz} flow={flow}: g {rel(gg, st[1]):.2e}"
          + (f" f {rel(fg, st[0]):.2e}" if flow else ""))
    assert rel(gg, st[1]) < 1e-12
    if flow:
        assert rel(fg, st[0]) < 1e-12


@pytest.mark.parametrize("prec", [W.FP32, W.FP16S, W.BF16S])
def test_cavity256_full_size_one_step_against_oracle(prec):
    """Full-size 256^3 precision cavity (Ra 1e6, Pr 0.02) in the launch shape the
    benchmark tunes: after 100 steps the oracle's FP64 step from the GPU state
    (decoded) agrees with the GPU's next state to the storage rounding."""
    cfg = W.precision_cavity(256, 0.02, precision=prec)
    cav = make_cavity(cfg)
    cav.autotune(3)
    cav.step(100)
    f, g = cav.state()
    st = (f.cpu().numpy(), g.cpu().numpy())
    del f, g
    cav.step(1)
    f1, g1 = cav.state()
    ref = oracle.run(dict(cfg, precision=W.FP64), st, 1)
    dev = np.abs(ref[0] - W19.reshape(19, 1, 1, 1) * cfg["rho0"]).max()
    ef, eg = absdiff(f1, ref[0]), absdiff(g1, ref[1])
    print(f"256^3 {['fp64', 'fp32', 'fp16s', 'bf16s'][prec]} one step (launch {cav.get_launch()}): "
          f"max|df| {ef:.2e} (max deviation {dev:.2e}), max|dg| {eg:.2e}")
    # shifted storage rounds the deviation f - w rho0 (FP32: 24 bits, FP16: 11,
    # BF16: 8) and g_1..6; deviations near 2e-5 are FP16 subnormals (spacing
    # 2^-24, below the smallest normal 6.1e-5): observed FP32 6.7e-12, FP16
    # 3.0e-8 = 2^-25
    bits = {W.FP32: 20, W.FP16S: 10, W.BF16S: 7}[prec]
    floor = {W.FP32: 1e-13, W.FP16S: 2.0 ** -25, W.BF16S: 0.0}[prec]
    assert ef < 2.0 ** -bits * dev + floor
    assert eg < 2.0 ** -bits * np.abs(ref[1][1:]).max()
    assert abs(cav.budgets()[0, 1] / 256**3 - 1.0) < 1e-5


def _storage_step_error(cfg, prec, flow, t_shift, f1, g1, ref):
    """Largest ratio of error to bound after one step in a storage format:
    each population plane within the storage rounding of its own deviation
    from rest (f - w rho0, g_a - (omega_T / 2) C_p,ref T_shift) plus FP32
    arithmetic on the largest deviation; g_0 within its own FP32 rounding."""
    bits = {W.FP32: 20, W.FP16S: 10, W.BF16S: 7}[prec]
    floor = 2.0 ** -24 if prec == W.FP16S else 0.0   # FP16 subnormal spacing
    worst = 0.0
    if flow:
        rest = W19.reshape(19, 1, 1, 1) * cfg["rho0"]
        dev = np.abs(ref[0] - rest).reshape(19, -1).max(axis=1)
        err = np.abs(f1.cpu().numpy() - ref[0]).reshape(19, -1).max(axis=1)
        bound = 2.0 ** -bits * dev + 2.0 ** -18 * dev.max() + floor
        worst = max(worst, float((err / bound).max()))
    gshift = 0.5 * cfg["omega_T"] * cfg["cp_ref"] * t_shift
    gdev = np.abs(ref[1][1:] - gshift).reshape(6, -1).max(axis=1)
    gerr = np.abs(g1.cpu().numpy()[1:] - ref[1][1:]).reshape(6, -1).max(axis=1)
    gbound = 2.0 ** -bits * gdev + 2.0 ** -18 * gdev.max() + floor
    e0 = absdiff(g1[0], ref[1][0])
    b0 = 2.0 ** -22 * np.abs(ref[1][0]).max() + 2.0 ** -18 * gdev.max()
    return max(worst, float((gerr / gbound).max()), e0 / b0)


# (flow, enthalpy model, faces) on a ragged 13 x 11 x 9 lattice: walls only,
# mixed walls and periodic pairs, fully periodic
FORMAT_CASES = [
    (1, W.MRT, [D, D, A, A, A, A]),
    (1, W.SRT, [D, A, P, P, D, A]),
    (1, W.MRT, [P] * 6),
    (0, W.MRT, [D, A, P, P, P, P]),
    (1, W.MRT, [A, D, D, A, D, D]),
]


@pytest.mark.parametrize("case", range(len(FORMAT_CASES)))
@pytest.mark.parametrize("prec", [W.FP32, W.FP16S, W.BF16S])
def test_random_state_one_step_in_every_storage_format(case, prec):
    """One step from an arbitrary state held in FP32, shifted FP16 or shifted
    BF16 storage (per-node wall temperatures; the 16-bit formats with a
    reference temperature of 0.3) against the oracle's FP64 step from the same
    decoded state: each population plane within the storage rounding of its
    own deviation from rest (f - w rho0, g_a - (omega_T / 2) C_p,ref T_shift)
    plus FP32 arithmetic on the largest deviation."""
    flow, model, bc = FORMAT_CASES[case]
    t_shift = 0.3 if prec in (W.FP16S, W.BF16S) else 0.0
    cfg = W.base_config(13, 11, 9, flow=flow, enth_model=model, precision=prec, face_bc=list(bc),
                        face_T=[1.0, -0.4, 0.3, 0.7, 0.9, -0.2], g_beta=4e-3, latent=1.5,
                        lambda_s=0.09, lambda_l=0.09, nu=0.04, T_shift=t_shift)
    f, g = W.random_populations(cfg, seed=500 + case, f_scale=W19)
    walls = random_walls(cfg, seed=600 + case)
    tw = W.wall_fields(cfg, walls)
    cav = make_cavity(cfg, walls=walls)
    cav.set_state(f, g)
    f0, g0 = cav.state()               # the stored state, decoded
    st = (f0.cpu().numpy() if flow else None, g0.cpu().numpy())
    cav.step(1)
    f1, g1 = cav.state()
    ref = oracle.run(dict(cfg, precision=W.FP64), st, 1, tw=tw)
    worst = _storage_step_error(cfg, prec, flow, t_shift, f1, g1, ref)
    print(f"case {case} {['fp64', 'fp32', 'fp16s', 'bf16s'][prec]}: largest error / bound {worst:.3f}")
    assert worst < 1.0


@pytest.mark.parametrize("seed", range(12))
def test_random_shapes_faces_and_launches_match_oracle(seed):
    """Seeded sweep: lattice dimensions from 1 to 40 (up to 24,000 cells, so
    tiles cross rows and planes at arbitrary places), random face types
    (periodic in pairs), flow on or off, SRT or MRT, and a random launch shape
    (tile size, persistent grid, XCD order, graph length); three steps from an
    arbitrary state equal the oracle's to 1e-12 of each population plane."""
    rng = np.random.default_rng(9000 + seed)
    while True:
        nx, ny, nz = (int(v) for v in rng.integers(1, 41, size=3))
        if nx * ny * nz <= 24000:
            break
    bc = [int(v) for v in rng.choice([D, A, P], size=6)]
    for d in range(3):
        if P in (bc[2 * d], bc[2 * d + 1]):
            bc[2 * d] = bc[2 * d + 1] = P
    flow = int(rng.integers(0, 2))
    model = W.MRT if rng.uniform() < 0.5 else W.SRT
    cfg = W.base_config(nx, ny, nz, flow=flow, enth_model=model, precision=W.FP64, face_bc=bc,
                        face_T=[float(v) for v in rng.uniform(-0.5, 1.0, size=6)], g_beta=4e-3,
                        latent=1.5, lambda_s=0.09, lambda_l=0.12, cp_l=1.3, nu=0.04)
    launch = (int(rng.choice([64, 128, 192, 256])), int(rng.choice([0, 8, 24])),
              int(rng.integers(0, 17)), int(rng.choice([0, 1, 3, 16, 1 << 20])))
    f, g = W.random_populations(cfg, seed=9100 + seed, f_scale=W19)
    walls = random_walls(cfg, seed=9200 + seed)
    tw = W.wall_fields(cfg, walls)
    cav = make_cavity(cfg, walls=walls)
    cav.set_launch(*launch)
    cav.set_state(f, g)
    cav.step(3)
    st = oracle.run(cfg, (f if flow else None, g), 3, tw=tw)
    fg, gg = cav.state()
    print(f"seed {seed}: {nx}x{ny}x{nz} faces {bc} flow {flow} model {model} launch {launch}: "
          f"g {rel(gg, st[1]):.1e}" + (f" f {rel(fg, st[0]):.1e}" if flow else ""))
    assert rel(gg, st[1]) < 1e-12
    if flow:
        assert rel(fg, st[0]) < 1e-12


@pytest.mark.parametrize("seed", range(9))
def test_random_shapes_in_storage_formats_one_step(seed):
    """Seeded sweep in the FP32, FP16 and BF16 storage formats: random lattice
    dimensions (1 to 40), face types, flow, enthalpy model and launch shape;
    one step from an arbitrary stored state against the oracle's FP64 step
    from the decoded state, within the storage rounding."""
    rng = np.random.default_rng(9500 + seed)
    while True:
        nx, ny, nz = (int(v) for v in rng.integers(1, 41, size=3))
        if nx * ny * nz <= 24000:
            break
    bc = [int(v) for v in rng.choice([D, A, P], size=6)]
    for d in range(3):
        if P in (bc[2 * d], bc[2 * d + 1]):
            bc[2 * d] = bc[2 * d + 1] = P
    prec = (W.FP32, W.FP16S, W.BF16S)[seed % 3]
    flow = int(rng.integers(0, 2))
    model = W.MRT if rng.uniform() < 0.5 else W.SRT
    t_shift = 0.3 if prec != W.FP32 else 0.0
    cfg = W.base_config(nx, ny, nz, flow=flow, enth_model=model, precision=prec, face_bc=bc,
                        face_T=[float(v) for v in rng.uniform(-0.5, 1.0, size=6)], g_beta=4e-3,
                        latent=1.5, lambda_s=0.09, lambda_l=0.12, cp_l=1.3, nu=0.04,
                        T_shift=t_shift)
    launch = (int(rng.choice([64, 128, 192, 256])), int(rng.choice([0, 8, 24])),
              int(rng.integers(0, 17)), int(rng.choice([0, 1, 3, 16, 1 << 20])))
    f, g = W.random_populations(cfg, seed=9600 + seed, f_scale=W19)
    walls = random_walls(cfg, seed=9700 + seed)
    tw = W.wall_fields(cfg, walls)
    cav = make_cavity(cfg, walls=walls)
    cav.set_launch(*launch)
    cav.set_state(f, g)
    f0, g0 = cav.state()
    st = (f0.cpu().numpy() if flow else None, g0.cpu().numpy())
    cav.step(1)
    f1, g1 = cav.state()
    ref = oracle.run(dict(cfg, precision=W.FP64), st, 1, tw=tw)
    worst = _storage_step_error(cfg, prec, flow, t_shift, f1, g1, ref)
    print(f"seed {seed}: {nx}x{ny}x{nz} {['fp64', 'fp32', 'fp16s', 'bf16s'][prec]} faces {bc} "
          f"flow {flow} launch {launch}: largest error / bound {worst:.3f}")
    assert worst < 1.0
