"""The seeded workloads (host logic, no GPU): the dimensionless groups of the
paper's problems map onto lattice units as the readings state, and the named
workloads have the shapes, boundaries and draws the benchmark and the tests
rely on."""
import math

import numpy as np
import pytest

import workloads as W


def _groups(cfg, l_c):
    """Ra, Pr, Ste and the velocity scale of a cavity, from its lattice values
    (Eq. (64): Ra = g beta dT l_c^3 / (nu chi), Pr = nu / chi, Ste = C_p dT / L)."""
    chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
    dT = cfg["face_T"][0] - cfg["T_m"]
    Ra = cfg["g_beta"] * dT * l_c ** 3 / (cfg["nu"] * chi)
    Pr = cfg["nu"] / chi
    Ste = cfg["cp_l"] * dT / cfg["latent"]
    U = math.sqrt(cfg["g_beta"] * dT * l_c)          # free-fall velocity
    return Ra, Pr, Ste, U


@pytest.mark.parametrize("n,Ra,Pr,Ste", [(128, 1e5, 0.02, 0.1), (256, 1e6, 6.2, 0.1),
                                         (96, 1e4, 1.0, 0.1), (40, 2.5e4, 10.0, 0.4)])
def test_melting_cavity_reproduces_its_groups(n, Ra, Pr, Ste):
    cfg = W.melting_cavity(n, Ra, Pr, Ste, precision=W.FP64)
    Ra2, Pr2, Ste2, U = _groups(cfg, n)
    assert Ra2 == pytest.approx(Ra, rel=1e-12)
    assert Pr2 == pytest.approx(Pr, rel=1e-12)
    assert Ste2 == pytest.approx(Ste, rel=1e-12)
    assert U == pytest.approx(0.1 / math.sqrt(3.0), rel=1e-12)   # Mach 0.1
    # the geometry of Sec. 3.3: hot x- face at 1, cold x+ face at T_m, the rest
    # adiabatic; all solid at T_m; buoyancy referenced to T_m
    assert cfg["face_bc"] == [W.DIRICHLET, W.DIRICHLET] + [W.ADIABATIC] * 4
    assert cfg["face_T"][:2] == [1.0, cfg["T_m"]] and cfg["T_m"] == 0.0 == cfg["T_ref"]
    assert (cfg["nx"], cfg["ny"], cfg["nz"]) == (n, n, n)
    # stable relaxation: tau_g = chi / omega_T + 1/2 > 1/2, s_nu in (0, 2)
    chi = cfg["lambda_l"] / (cfg["rho0"] * cfg["cp_ref"])
    assert chi / cfg["omega_T"] > 0.0 and 0.0 < 1.0 / (3 * cfg["nu"] + 0.5) < 2.0


@pytest.mark.parametrize("case", [1, 2, 3])
def test_table2_cases_on_their_grids(case):
    (nx, ny, nz), Pr, Ra = W.TABLE2[case]
    cfg = W.table2_case(case, precision=W.FP64)
    assert (cfg["nx"], cfg["ny"], cfg["nz"]) == (nx, ny, nz) and nz == 80
    Ra2, Pr2, Ste2, _ = _groups(cfg, nx)     # l_c = nx, the hot-to-cold length
    assert Ra2 == pytest.approx(Ra, rel=1e-12) and Pr2 == pytest.approx(Pr, rel=1e-12)
    assert Ste2 == pytest.approx(0.4, rel=1e-12)


def test_corner_and_slab_problems():
    c = W.corner_solidification()
    assert (c["nx"], c["ny"], c["nz"]) == (400, 1, 400) and c["flow"] == 0
    assert c["face_bc"][2:4] == [W.PERIODIC, W.PERIODIC]
    # Ste_s = C_p (T_m - T_wall) / L = 4 with the walls at -1 and T0 = 0.3 far away
    assert c["cp_s"] * (c["T_m"] - c["face_T"][0]) / c["latent"] == pytest.approx(4.0)
    assert c["face_T"][0] == c["face_T"][4] == -1.0 and c["face_T"][1] == c["face_T"][5] == 0.3
    s = W.convection_2d()
    assert (s["nx"], s["ny"], s["nz"]) == (128, 1, 128)
    Ra, Pr, Ste, _ = _groups(s, 128)
    assert Ra == pytest.approx(2.5e4) and Pr == pytest.approx(0.02) and Ste == pytest.approx(0.01)


def test_batch_draw_is_seeded_and_in_range():
    cfgs, draws = W.batch_cavities()
    again, draws2 = W.batch_cavities()
    assert len(cfgs) == 64 and draws == draws2

    def same(a, b):        # NaN entries (sigma_override) compare equal
        return np.array_equal(np.asarray(a, dtype=float), np.asarray(b, dtype=float),
                              equal_nan=True) if isinstance(a, list) else a == b
    assert all(same(c[k], d[k]) for c, d in zip(cfgs, again) for k in c)
    sizes = [d["n"] for d in draws]
    assert set(sizes) <= {32, 48, 64, 96} and len(set(sizes)) == 4
    assert sum(n ** 3 for n in sizes) == 17_227_776          # the benchmark's 17.2 M cells
    for c, d in zip(cfgs, draws):
        assert 1e3 <= d["Ra"] <= 1e6 and 0.02 <= d["Pr"] <= 50 and 0.05 <= d["Ste"] <= 0.5
        Ra, Pr, Ste, _ = _groups(c, d["n"])
        assert (Ra, Pr, Ste) == pytest.approx((d["Ra"], d["Pr"], d["Ste"]), rel=1e-12)
    assert len({c["precision"] for c in cfgs}) == 1


def test_random_states_are_seeded_and_span_the_phases():
    cfg = W.base_config(9, 7, 5)
    f1, g1 = W.random_populations(cfg, seed=3, f_scale=np.ones(19))
    f2, g2 = W.random_populations(cfg, seed=3, f_scale=np.ones(19))
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2)
    h = g1.sum(axis=0)
    hs = cfg["cp_s"] * cfg["T_m"]
    hl = cfg["cp_l"] * cfg["T_m"] + cfg["latent"]
    assert (h <= hs).any() and ((h > hs) & (h < hl)).any() and (h >= hl).any()
