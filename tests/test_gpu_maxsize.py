"""The largest cavity the library accepts (812^3 cells: planes of up to 2^29
cells are addressed with 32-bit byte offsets) on the GPU, checked through
properties that hold exactly at any size: a problem that is uniform across y
and z evolves every (y, z) row of the cavity exactly like a one-row lattice,
so the 812^3 run must equal, bit for bit, an 812 x 1 x 1 run, and that in
turn the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import make_cavity

pytestmark = pytest.mark.gpu

N = 812   # 812^3 + 384 <= 2^29 < 813^3


def _rows_equal(big, small):
    """Every (z, y) row of big (nz, ny, nx) equals small's single row."""
    import torch
    return bool(torch.equal(big, small.expand_as(big)))


def test_max_size_fp64_walls_on_all_faces_equals_one_row_and_the_oracle():
    """Enthalpy only, FP64, walls on every face (hot and cold x walls,
    adiabatic y and z walls: the walls-only push path), 812^3 cells, whose g_0
    plane ends 1 KiB below 2^32 bytes.  With u = 0 and a y,z-uniform state the
    adiabatic bounce-back returns what a neighbouring row would have sent, so
    every row equals an 812 x 1 x 1 periodic lattice bit for bit, and that
    equals the oracle to 1e-12."""
    import torch
    cfg = W.base_config(N, N, N, flow=0, enth_model=W.MRT, precision=W.FP64,
                        face_bc=[W.DIRICHLET, W.DIRICHLET] + [W.ADIABATIC] * 4,
                        face_T=[1.0, -0.5, 0, 0, 0, 0], lambda_s=0.12, lambda_l=0.12,
                        latent=2.0, T_m=0.0)
    one = dict(cfg, ny=1, nz=1, face_bc=[W.DIRICHLET, W.DIRICHLET] + [W.PERIODIC] * 4)
    steps = 150
    big = make_cavity(cfg)
    big.set_launch(256, 0, 16, 0)
    big.step(steps)
    b = big.budgets()[0]
    small = make_cavity(one)
    small.step(steps)
    for name in ("h", "T", "fl"):
        fb = big.fields(names=(name,))[name]
        fs = small.fields(names=(name,))[name]
        assert _rows_equal(fb, fs), name
        del fb
        torch.cuda.empty_cache()
    ref = oracle.run(one, oracle.init_state(one), steps)
    _, g = small.state()
    err = float(np.abs(g.cpu().numpy() - ref[1]).max() / np.abs(ref[1]).max())
    print(f"{N}^3 FP64 enthalpy: rows equal the one-row run; one-row vs oracle {err:.2e}; "
          f"liquid {b[2] / N**3:.4f} of the cavity")
    assert err < 1e-12
    assert 0.0 < b[2] / N**3 < 1.0
    big.close()


def test_max_size_fp32_coupled_periodic_equals_one_row():
    """Coupled D3Q19 + D3Q7, FP32 storage (113 GB of state), 812^3 cells,
    hot and cold x walls, periodic y and z (the general link path), buoyancy
    along z: the x-dependent buoyancy drives a flow along z that is uniform in
    y and z, and every row equals an 812 x 1 x 1 run bit for bit; mass is
    conserved."""
    import torch
    cfg = W.melting_cavity(N, 1e5, 0.02, 0.1, precision=W.FP32)
    cfg.update(face_bc=[W.DIRICHLET, W.DIRICHLET] + [W.PERIODIC] * 4, g_beta=2e-4, nu=0.02,
               lambda_s=0.05, lambda_l=0.05, latent=2.0)
    one = dict(cfg, ny=1, nz=1)
    steps = 60
    big = make_cavity(cfg)
    big.set_launch(256, 0, 16, 0)
    m0 = big.budgets()[0, 1]
    big.step(steps)
    m1 = big.budgets()[0, 1]
    small = make_cavity(one)
    small.step(steps)
    for name in ("T", "fl", "u"):
        fb = big.fields(names=(name,))
        fs = small.fields(names=(name,))
        for k in fb:
            assert _rows_equal(fb[k], fs[k]), k
        del fb
        torch.cuda.empty_cache()
    uz = small.fields(names=("u",))["uz"]
    print(f"{N}^3 FP32 coupled: rows equal the one-row run; max |u_z| {float(uz.abs().max()):.2e}; "
          f"mass drift {m1 / m0 - 1:.1e}")
    assert float(uz.abs().max()) > 1e-6
    assert abs(m1 / m0 - 1.0) < 1e-10
    big.close()
