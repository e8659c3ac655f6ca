"""The 2D validations of Sec. 3.2 on the GPU, run as y-periodic slabs: against
the oracle, and against exact properties of the two problems."""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
import workloads as W
from analytic import neumann_melting_k
from gpu_util import make_cavity, rel
from test_oracle_conditioning import DRIFT_PER_1000

pytestmark = pytest.mark.gpu


def test_corner_solidification_matches_oracle_and_is_symmetric():
    """Sec. 3.2.1 corner on a 56 x 1 x 56 slab (ragged against the tiles), FP64,
    800 steps: the GPU state equals the oracle's, and f_l is symmetric under
    x <-> z."""
    n, steps = 56, 800
    cfg = W.corner_solidification(n=n, chi=0.2)
    T0 = np.full((n, 1, n), 0.3)
    cav = make_cavity(cfg, T0=T0)
    cav.step(steps)
    _, g = cav.state()
    ref = oracle.run(cfg, oracle.init_state(cfg, T0), steps)
    err = rel(g, ref[1])
    fl = cav.fields(names=("fl",))["fl"][:, 0, :].cpu().numpy()
    sym = np.abs(fl - fl.T).max()
    print(f"corner: rel g {err:.2e}, symmetry {sym:.2e}, mean f_l {fl.mean():.4f}")
    assert 0.05 < fl.mean() < 0.95
    assert err < max(1e-12, DRIFT_PER_1000 * steps / 1000)
    assert sym < 1e-10
    # the step map at the end of the run: one oracle step from the GPU state
    # equals the GPU's next step to 1e-12
    st = (None, g.cpu().numpy())
    cav.step(1)
    _, g1 = cav.state()
    one = oracle.run(cfg, st, 1)
    print(f"corner: one step from the GPU state, rel g {rel(g1, one[1]):.2e}")
    assert rel(g1, one[1]) < 1e-12


def test_convection_slab_matches_oracle():
    """Sec. 3.2.2 slab (40 x 1 x 40, Table 1 groups with l_c = 40, faster latent
    release and a random mixed-phase start so that buoyant flow and all phases
    are present), FP64, 500 steps: f and g equal the oracle's."""
    n, steps = 40, 500
    cfg = W.convection_2d(n, precision=W.FP64)
    cfg.update(latent=2.0)
    T0 = W.random_temperature(cfg, seed=33, lo=-0.3, hi=1.0)
    cav = make_cavity(cfg, T0=T0)
    cav.step(steps)
    f, g = cav.state()
    ref = oracle.run(cfg, oracle.init_state(cfg, T0), steps)
    ef, eg = rel(f, ref[0]), rel(g, ref[1])
    u = cav.fields(names=("u",))
    umax = float(max(u["ux"].abs().max(), u["uz"].abs().max()))
    print(f"convection slab: rel f {ef:.2e}, rel g {eg:.2e}, max |u| {umax:.2e}")
    assert umax > 1e-4
    tol = max(1e-12, DRIFT_PER_1000 * steps / 1000)
    assert ef < tol and eg < tol
    st = (f.cpu().numpy(), g.cpu().numpy())
    cav.step(1)
    f1, g1 = cav.state()
    one = oracle.run(cfg, st, 1)
    e1f, e1g = rel(f1, one[0]), rel(g1, one[1])
    print(f"convection slab: one step from the GPU state, rel f {e1f:.2e}, rel g {e1g:.2e}")
    assert e1f < 1e-12 and e1g < 1e-12


def test_slab_is_y_invariant_bitwise():
    """A one-cell-thick periodic slab and a three-cell one with the same
    y-independent state evolve identically, bit for bit (FP32 storage)."""
    cfg1 = W.convection_2d(48, precision=W.FP32)
    cfg1.update(nu=0.02, lambda_s=0.05, lambda_l=0.05, g_beta=2e-3, latent=2.0)
    cfg3 = dict(cfg1, ny=3)
    T0 = W.random_temperature(cfg1, seed=21, lo=-0.3, hi=1.0)
    a = make_cavity(cfg1, T0=T0)
    b = make_cavity(cfg3, T0=np.repeat(T0, 3, axis=1))
    a.step(400)
    b.step(400)
    fa = a.fields(names=("h", "T", "fl", "rho", "u"))
    fb = b.fields(names=("h", "T", "fl", "rho", "u"))
    assert float(fa["uz"].abs().max()) > 1e-4
    for key in ("h", "T", "fl", "rho", "ux", "uz"):
        for y in range(3):
            assert bool((fa[key][:, 0, :] == fb[key][:, y, :]).all()), key


def test_conduction_slab_mean_nusselt_matches_neumann():
    """Table 1 slab without buoyancy (one-phase Neumann melting along x), FP64:
    the mean of Eq. (65) from the GPU's cumulative wall inflow while the front
    moves from 10 to 25 cells equals the exact mean within 1e-4."""
    n = 64
    cfg = W.convection_2d(n, precision=W.FP64, buoyancy=False)
    cfg.update(nz=2, flow=0)
    chi = cfg["lambda_l"]
    k = neumann_melting_k(0.01)
    t1, t2 = (int(round((X / (2.0 * k)) ** 2 / chi)) for X in (10.0, 25.0))
    cav = make_cavity(cfg)
    cav.step(t1)
    q1 = cav.budgets()[0, 3]
    cav.step(t2 - t1)
    q2 = cav.budgets()[0, 3]
    nu_num = (q2 - q1) / (t2 - t1) / (cfg["ny"] * cfg["nz"]) * n / (chi * cfg["cp_ref"])
    fo1, fo2 = chi * t1 / n ** 2, chi * t2 / n ** 2
    nu_ex = 2.0 * (math.sqrt(fo2) - math.sqrt(fo1)) / (erf(k) * math.sqrt(math.pi) * (fo2 - fo1))
    print(f"conduction slab: mean Nu {nu_num:.6f} vs exact {nu_ex:.6f}")
    assert abs(nu_num / nu_ex - 1.0) < 1e-4
