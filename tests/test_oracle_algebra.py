"""Pins of the oracle's cell-level algebra against what the paper and textbook
lattice Boltzmann fix independently (no GPU)."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W

RNG = np.random.default_rng(20170308)


def cfg_default(**kw):
    return W.base_config(4, 4, 4, **kw)


@pytest.fixture(scope="module")
def tab():
    return oracle.tables()


# ---------------------------------------------------------------- lattices --
def test_d3q7_velocity_moments(tab):
    """Eq. (4): sum e_i = 0 and sum e_i e_j = 2 delta_ij (c = 1)."""
    e = tab["e7"]
    assert np.allclose(e.sum(0), 0)
    assert np.allclose(e.T @ e, 2 * np.eye(3))


def test_d3q19_velocity_set(tab):
    """Eq. (48): the 19 velocities are the rest vector, the 6 axis vectors and the
    12 face diagonals, each once."""
    e = tab["e19"].astype(int)
    want = {(0, 0, 0)}
    want |= {v for v in itertools.product((-1, 0, 1), repeat=3) if 1 <= sum(map(abs, v)) <= 2}
    assert {tuple(v) for v in e} == want and len(e) == 19


def _basis7(e):
    """D3Q7 moment basis written from its physical meaning: density, flux,
    energy-like (6 - 7 e^2) and the two second-order anisotropies."""
    ex, ey, ez = e.T
    e2 = ex**2 + ey**2 + ez**2
    return np.stack([np.ones_like(ex), ex, ey, ez, 6 - 7 * e2, 3 * ex**2 - e2, ey**2 - ez**2])


def _basis19(e):
    """Gram-Schmidt polynomial basis of d'Humieres et al. (2002)."""
    ex, ey, ez = e.T
    e2 = ex**2 + ey**2 + ez**2
    q = 5 * e2 - 9
    p = 3 * e2 - 5
    return np.stack([
        np.ones_like(ex), 19 * e2 - 30, (21 * e2**2 - 53 * e2 + 24) / 2,
        ex, q * ex, ey, q * ey, ez, q * ez,
        3 * ex**2 - e2, p * (3 * ex**2 - e2), ey**2 - ez**2, p * (ey**2 - ez**2),
        ex * ey, ey * ez, ex * ez,
        ex * (ey**2 - ez**2), ey * (ez**2 - ex**2), ez * (ex**2 - ey**2)])


def test_N_matches_polynomial_basis(tab):
    """Eq. (24) as transcribed equals the moment polynomials evaluated on Eq. (3)."""
    assert np.array_equal(tab["N"], _basis7(tab["e7"]))


def test_M_matches_polynomial_basis(tab):
    """Eq. (51) as transcribed equals the standard D3Q19 polynomial basis on Eq. (48)."""
    assert np.array_equal(tab["M"], _basis19(tab["e19"]))


def test_rows_orthogonal_and_inverses(tab):
    N, M = tab["N"], tab["M"]
    dN = N @ N.T
    dM = M @ M.T
    assert np.allclose(dN, np.diag(np.diag(dN)))
    assert np.allclose(dM, np.diag(np.diag(dM)))
    assert np.array_equal(np.diag(dN), [7, 2, 2, 2, 42, 12, 4])
    assert np.array_equal(np.diag(dM), [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12,
                                        24, 4, 4, 4, 8, 8, 8])
    assert np.allclose(tab["Ninv"] @ N, np.eye(7), atol=1e-14)
    assert np.allclose(tab["Minv"] @ M, np.eye(19), atol=1e-14)


# ----------------------------------------------------------- equilibria --
@pytest.mark.parametrize("omega_T", [0.25, 0.2, 1 / 3])
def test_geq_moments_eq9(tab, omega_T):
    """Eq. (9): zeroth, first and second moments of g^eq."""
    cfg = cfg_default(omega_T=omega_T, cp_ref=1.3)
    e = tab["e7"]
    for _ in range(20):
        h, T, cp = RNG.uniform(-2, 12), RNG.uniform(-1, 2), RNG.uniform(0.5, 2)
        u = RNG.uniform(-0.1, 0.1, 3)
        g = oracle.g_eq(cfg, h, T, cp, u)
        assert g.sum() == pytest.approx(h, abs=1e-13)
        assert np.allclose(e.T @ g, cp * T * u, atol=1e-14)
        second = (e[:, :, None] * e[:, None, :] * g[:, None, None]).sum(0)
        assert np.allclose(second, 1.3 * T * omega_T * np.eye(3), atol=1e-14)


def test_neq_equals_N_geq(tab):
    """Eq. (25) is the moment image of Eq. (7)."""
    cfg = cfg_default(omega_T=0.22, cp_ref=0.9)
    for _ in range(20):
        h, T, cp = RNG.uniform(-2, 12), RNG.uniform(-1, 2), RNG.uniform(0.5, 2)
        u = RNG.uniform(-0.1, 0.1, 3)
        assert np.allclose(tab["N"] @ oracle.g_eq(cfg, h, T, cp, u),
                           oracle.n_eq(cfg, h, T, cp, u), atol=1e-13)


def _feq_textbook(rho, u, e):
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    eu = e @ u
    return w * rho * (1 + 3 * eu + 4.5 * eu**2 - 1.5 * (u @ u))


def _guo_textbook(F, u, e):
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    return w * (3 * ((e - u) @ F) + 9 * (e @ u) * (e @ F))


def test_meq_is_moment_image_of_second_order_feq(tab):
    """Eq. (53) (with the 11th entry read as -1/2 of the 10th) equals M f^eq for the
    usual second-order D3Q19 equilibrium; every entry is checked."""
    for _ in range(20):
        rho, u = RNG.uniform(0.8, 1.2), RNG.uniform(-0.1, 0.1, 3)
        assert np.allclose(tab["M"] @ _feq_textbook(rho, u, tab["e19"]), oracle.m_eq(rho, u),
                           atol=1e-13)


def test_printed_pi_xx_entry_is_not_the_moment_image(tab):
    """The literal 11th entry of Eq. (53) (u_z^2 not halved) is not M f^eq: the
    reading of that entry is forced."""
    rho, u = 1.0, np.array([0.02, 0.03, 0.05])
    literal = rho * (-u[0]**2 + 0.5 * u[1]**2 + u[2]**2)
    assert abs(literal - (tab["M"] @ _feq_textbook(rho, u, tab["e19"]))[10]) > 1e-4


def test_FF_is_moment_image_of_guo_forcing(tab):
    """Eq. (54) (10th entry read as 6 F_x u_x - 2 F.u) equals M F_Guo."""
    for _ in range(20):
        F, u = RNG.uniform(-1e-3, 1e-3, 3), RNG.uniform(-0.1, 0.1, 3)
        assert np.allclose(tab["M"] @ _guo_textbook(F, u, tab["e19"]),
                           oracle.force_moments(F, u), atol=1e-15)


# ------------------------------------------------------------ phase rule --
def test_phase_rule_inverts_eq2():
    """h -> (T, f_l) inverts h = C_p T + f_l L (Eq. (2)) in each range, with the
    lever rule in the mushy range, for T_m != 0 and C_p,s != C_p,l."""
    cfg = cfg_default(cp_s=1.0, cp_l=2.0, latent=3.0, T_m=0.5)
    hs, hl = 0.5, 2.0 * 0.5 + 3.0
    for h in np.concatenate([np.linspace(-3, hs, 7), np.linspace(hs, hl, 9), np.linspace(hl, 9, 7)]):
        T, fl = oracle.phase(cfg, h)
        assert 0.0 <= fl <= 1.0
        cp = (1 - fl) * 1.0 + fl * 2.0
        assert cp * T + fl * 3.0 == pytest.approx(h, abs=1e-13)
        if h <= hs:
            assert fl == 0.0
        if h >= hl:
            assert fl == 1.0
        if hs < h < hl:
            assert T == 0.5


# ------------------------------------------------------------- collisions --
def _random_cell(cfg):
    f = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12) * (1 + 0.2 * RNG.uniform(-1, 1, 19))
    g = np.concatenate([[RNG.uniform(-1, 12)], 0.15 * RNG.uniform(-1, 2, 6)])
    return f, g


@pytest.mark.parametrize("tau", [0.564, 0.7, 1.012, 1.5, 6.9])
def test_d3q7_mrt_with_equal_rates_is_srt(tau):
    """With every sigma equal to 1/tau_g the MRT collision (Eq. (21)) is the BGK
    collision (Eq. (6))."""
    lam = (tau - 0.5) * 0.25
    base = dict(lambda_s=lam, lambda_l=lam, g_beta=1e-3)
    srt = cfg_default(enth_model=W.SRT, **base)
    mrt = cfg_default(enth_model=W.MRT, sigma_override=[1 / tau] * 7, **base)
    for _ in range(30):
        f, g = _random_cell(srt)
        _, gs1, _ = oracle.collide_cell(srt, f, g)
        _, gs2, _ = oracle.collide_cell(mrt, f, g)
        assert np.allclose(gs1, gs2, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 1.7])
def test_d3q19_mrt_with_equal_rates_is_bgk_guo(tab, tau):
    """With every non-conserved rate equal to 1/tau the MRT collision with forcing
    (Eq. (49)-(50)) is BGK with Guo's forcing term, written here in velocity space."""
    s = 1 / tau
    nu = (tau - 0.5) / 3
    cfg = cfg_default(nu=nu, s_e=s, s_eps=s, s_q=s, s_pi=s, s_t=s, g_beta=2e-3)
    e = tab["e19"]
    for _ in range(30):
        f, g = _random_cell(cfg)
        fs, _, aux = oracle.collide_cell(cfg, f, g)
        u = np.array([aux["ux"], aux["uy"], aux["uz"]])
        F = np.array([aux["Fx"], aux["Fy"], aux["Fz"]])
        rho = f.sum()
        ref = f - (f - _feq_textbook(rho, u, e)) / tau + (1 - 0.5 / tau) * _guo_textbook(F, u, e)
        assert np.allclose(fs, ref, rtol=1e-14, atol=1e-15)


def test_eq56_momentum_with_forcing(tab):
    """Eq. (56) with the local density: rho u = sum f e + F/2; conserved moments of
    Eq. (49): rho and j are changed only by the force."""
    cfg = cfg_default(g_beta=3e-3)
    e = tab["e19"]
    for _ in range(30):
        f, g = _random_cell(cfg)
        fs, _, aux = oracle.collide_cell(cfg, f, g)
        u = np.array([aux["ux"], aux["uy"], aux["uz"]])
        F = np.array([aux["Fx"], aux["Fy"], aux["Fz"]])
        rho = f.sum()
        assert np.allclose(rho * u, e.T @ f + F / 2, atol=1e-15)
        assert fs.sum() == pytest.approx(rho, abs=1e-14)
        assert np.allclose(e.T @ fs, e.T @ f + F, atol=1e-15)


def test_solid_forcing_limits():
    """f_l = 0: u = 0 and the force cancels the momentum; f_l = 1: the force is the
    buoyancy of Eq. (55)."""
    cfg = cfg_default(g_beta=2e-3, latent=10.0)
    f = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12) * (1 + 0.1 * RNG.uniform(-1, 1, 19))
    e = oracle.tables()["e19"]
    g_solid = np.array([-0.5, 0.01, 0, 0, 0, 0, 0])
    _, _, a = oracle.collide_cell(cfg, f, g_solid)
    assert a["fl"] == 0 and a["ux"] == a["uy"] == a["uz"] == 0
    assert np.allclose([a["Fx"], a["Fy"], a["Fz"]], -2 * (e.T @ f), atol=1e-16)
    g_liq = np.array([11.0, 0.1, 0, 0.05, 0, 0, 0.02])
    _, _, a = oracle.collide_cell(cfg, f, g_liq)
    T = g_liq.sum() - 10.0
    assert a["fl"] == 1 and a["T"] == pytest.approx(T)
    assert np.allclose([a["Fx"], a["Fy"], a["Fz"]], [0, 0, 2e-3 * T], atol=1e-16)


def _rates(cfg, s1, s4, s5, s6):
    c = dict(cfg)
    c["sigma_override"] = [s1, s1, s1, s1, s4, s5, s6]
    return c


@pytest.mark.parametrize("s1,s4", [(1.14, 1.9), (1.14, 0.1), (1.4, 0.6), (0.7, 1.3)])
def test_interface_error_eq45(s1, s4):
    """Sec. 2.4: at an interface cell (T = T_m, u = 0) whose +x neighbour is solid
    at T_m, so that g_2 = w C_p,ref T_m arrives from it (Eq. (42)), the
    post-collision g_1 sent into the solid differs from (1/2) omega_T C_p,ref T_m by
    (sigma_1 + sigma_4 - 2)/2 (g_0 + g_3 + ... + g_6 - h + omega_T C_p,ref T_m),
    Eq. (45), with sigma_4 = sigma_5 (Sec. 3.1.2)."""
    cfg = cfg_default(flow=0, T_m=0.3, latent=5.0, cp_s=1.0, cp_l=1.0, omega_T=0.25)
    cfg = _rates(cfg, s1, s4, s4, 1.0)
    wT = 0.25 * cfg["T_m"]
    for _ in range(20):
        h = RNG.uniform(0.3 + 0.1, 0.3 + 4.9)  # mushy
        g = np.empty(7)
        g[[0, 3, 4, 5, 6]] = RNG.uniform(-0.2, 0.4, 5) + np.array([h / 2, 0, 0, 0, 0])
        g[2] = 0.5 * wT
        g[1] = h - g[[0, 2, 3, 4, 5, 6]].sum()
        _, gs, aux = oracle.collide_cell(cfg, None, g)
        assert aux["T"] == cfg["T_m"]
        rhs = (s1 + s4 - 2) / 2 * (g[[0, 3, 4, 5, 6]].sum() - h + wT)
        assert gs[1] - 0.5 * wT == pytest.approx(rhs, abs=1e-13)


def test_relaxation_rule_cancels_interface_error_on_all_axes():
    """With the default rates (sigma_4 = sigma_5 = sigma_6 = 2 - sigma_chi) an
    interface cell at T_m with u = 0 sends exactly (1/2) omega_T C_p,ref T_m into a
    neighbour that returned that value, along x, y and z (Sec. 2.4, Eq. (47))."""
    cfg = cfg_default(flow=0, T_m=0.0, latent=5.0, lambda_s=0.13, lambda_l=0.13)
    for axis in range(3):
        out, back = 1 + 2 * axis, 2 + 2 * axis
        for _ in range(20):
            h = RNG.uniform(0.1, 4.9)
            g = RNG.uniform(-0.2, 0.4, 7)
            g[back] = 0.0
            g[out] = 0.0
            g[0] += h - g.sum()
            _, gs, _ = oracle.collide_cell(cfg, None, g)
            assert abs(gs[out]) < 1e-14


def test_eq36_rest_and_transverse_sum():
    """Eq. (36) for u = 0 and sigma_4 = sigma_5: the sum g_0 + g_3 + ... + g_6 relaxes
    toward h - omega_T C_p,ref T with rate sigma_5."""
    cfg = cfg_default(flow=0, T_m=0.0, latent=5.0)
    for s5 in (0.3, 1.0, 1.7):
        c = _rates(cfg, 1.2, s5, s5, 0.9)
        for _ in range(10):
            g = RNG.uniform(-0.2, 2.0, 7)
            _, gs, aux = oracle.collide_cell(c, None, g)
            S, Spost = g[[0, 3, 4, 5, 6]].sum(), gs[[0, 3, 4, 5, 6]].sum()
            want = (1 - s5) * S + s5 * (aux["h"] - 0.25 * aux["T"])
            assert Spost == pytest.approx(want, abs=1e-13)
