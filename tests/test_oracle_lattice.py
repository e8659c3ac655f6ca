"""Pins of the oracle's full time step against closed forms, conservation laws,
symmetries, a linear-stability analysis and the paper's printed values (no GPU)."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from analytic import neumann_melting_front, neumann_melting_k, solidification_k

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].split()
        if len(line) == 2:
            out[line[0]] = float(line[1])
    return out


# ------------------------------------------------------------ closed forms --
def test_neumann_front_matches_paper_value():
    """Sec. 3.1.1: chi_l = 0.001, Ste_l = 0.1 puts the interface at 0.44 at t = 1000."""
    g = _golden("neumann_melting.txt")
    X = neumann_melting_front(g["t"], g["chi_l"], g["Ste_l"])
    assert round(X, int(g["X_digits"])) == g["X"]


def test_two_phase_k_reduces_to_one_phase():
    """Eq. (63) with Ste_l -> 0 (no superheat) is the one-phase Eq. (61) relation."""
    k1 = neumann_melting_k(0.05)
    k2 = solidification_k(0.05, 1e-14, 0.3, 0.3)
    assert k2 == pytest.approx(k1, rel=1e-9)


def _front(cfg, state):
    fl = oracle.fields(cfg, state)["fl"]
    axis = [cfg["nx"], cfg["ny"], cfg["nz"]].index(max(cfg["nx"], cfg["ny"], cfg["nz"]))
    area = cfg["nx"] * cfg["ny"] * cfg["nz"] / [cfg["nx"], cfg["ny"], cfg["nz"]][axis]
    return fl.sum() / area


def test_stefan_melting_mrt_matches_neumann():
    """1D melting (Sec. 3.1.1) on a 64x4x4 lattice, chi = 0.05, Ste = 0.1, 2000 steps:
    sum of f_l along x (walls half a cell outside the nodes) against Eq. (61)."""
    cfg = W.stefan_1d(W.MRT)
    st = oracle.run(cfg, oracle.init_state(cfg), 2000)
    X = _front(cfg, st)
    Xa = neumann_melting_front(2000, 0.05, 0.1)
    assert abs(X - Xa) <= 0.05


def test_stefan_error_shrinks_with_resolution():
    """Doubling the front distance (t x 4 at the same chi) halves the relative
    front error or better."""
    cfg = W.stefan_1d(W.MRT)
    st = oracle.init_state(cfg)
    st = oracle.run(cfg, st, 500)
    e1 = abs(_front(cfg, st) / neumann_melting_front(500, 0.05, 0.1) - 1)
    st = oracle.run(cfg, st, 1500)
    e2 = abs(_front(cfg, st) / neumann_melting_front(2000, 0.05, 0.1) - 1)
    assert e2 < 0.6 * e1


def test_srt_leaks_into_solid_mrt_does_not():
    """Sec. 3.1.1 and Sec. 2.4: with tau below 1 the SRT model drives the solid below
    T_m (negative, as the paper's -0.00152 at tau = 0.564), while the MRT model with
    the rule of Eq. (47) keeps every solid cell ahead of the front at h_s."""
    g = _golden("neumann_melting.txt")
    chi = (0.564 - 0.5) * 0.25
    out = {}
    for model in (W.SRT, W.MRT):
        cfg = W.stefan_1d(model, chi=chi)
        st = oracle.run(cfg, oracle.init_state(cfg), 3000)
        fl = oracle.fields(cfg, st)
        T = fl["T"][0, 0]
        front = int(math.ceil(fl["fl"][0, 0].sum()))
        out[model] = T[front + 1:]
    assert np.sign(out[W.SRT].min()) == g["srt_leak_sign"]
    assert out[W.SRT].min() < -1e-6
    assert np.abs(out[W.MRT]).max() < 1e-13


def test_rule_holds_in_solid_for_all_steps():
    """Sec. 2.4 invariant over time: with MRT and T_m = 0, every cell beyond the first
    non-liquid neighbour of the front keeps |h - h_s| < 1e-13 at every step."""
    cfg = W.stefan_1d(W.MRT)
    st = oracle.init_state(cfg)
    for _ in range(20):
        st = oracle.run(cfg, st, 50)
        h = oracle.fields(cfg, st)["h"][0, 0]
        first_solid = int(np.argmax(h <= 0.0))
        assert np.abs(h[first_solid + 1:]).max() < 1e-13


@pytest.mark.parametrize("model", [W.SRT, W.MRT])
def test_symmetry_x_y_z(model):
    """Sec. 3.1.1: the 1D problem solved along x, y or z gives the same fields."""
    res = []
    for axis in range(3):
        cfg = W.stefan_1d(model, axis=axis, n=32)
        st = oracle.run(cfg, oracle.init_state(cfg), 400)
        T = oracle.fields(cfg, st)["T"]  # [z][y][x]
        prof = np.moveaxis(T, 2 - axis, 0).reshape(32, -1)
        assert np.allclose(prof, prof[:, :1], atol=1e-15)
        res.append(prof[:, 0])
    assert np.allclose(res[0], res[1], atol=1e-13, rtol=0)
    assert np.allclose(res[0], res[2], atol=1e-13, rtol=0)


def _rotate_z(state, e19, e7, n):
    """Rotate a state by 90 degrees about z: the cell (x, y, z) goes to
    (n - 1 - y, x, z) and the population along e to the one along R e, with
    R (ex, ey, ez) = (-ey, ex, ez)."""
    def perm(e):
        key = {tuple(v): i for i, v in enumerate(e.astype(int))}
        return [key[(-int(v[1]), int(v[0]), int(v[2]))] for v in e]

    def planes(p, e):
        out = np.empty_like(p)
        for a, b in enumerate(perm(e)):
            out[b] = np.swapaxes(p[a][:, ::-1, :], 1, 2)
        return out

    f, g = state
    assert f.shape[2] == f.shape[3] == n
    return planes(f, e19), planes(g, e7)


@pytest.mark.parametrize("model", [W.SRT, W.MRT])
def test_quarter_turn_about_gravity_commutes_with_the_step(model):
    """Isotropy of the coupled step: on a square-based box (walls of the same
    kind on the four side faces, fixed temperatures on the bottom and top,
    gravity along -z) rotating an arbitrary mixed-phase state by 90 degrees
    about z and stepping gives the rotation of the stepped state.  A wrong sign,
    index or transposed entry in the D3Q19 moments, the forcing, the D3Q7 rates
    or the streaming of one direction breaks this."""
    n = 8
    cfg = W.base_config(n, n, 6, flow=1, enth_model=model, precision=W.FP64,
                        face_bc=[W.ADIABATIC] * 4 + [W.DIRICHLET] * 2,
                        face_T=[0.0] * 4 + [1.0, -0.2], g_beta=3e-3, latent=1.0,
                        cp_s=1.0, cp_l=1.4, lambda_s=0.12, lambda_l=0.05, nu=0.04)
    tab = oracle.tables()
    w19 = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int(round(v @ v))] for v in tab["e19"]])
    f, g = W.random_populations(cfg, seed=90, f_scale=w19 * cfg["rho0"], g_rest_range=(-0.6, 1.6))
    st = (f, g)
    a = oracle.run(cfg, _rotate_z(st, tab["e19"], tab["e7"], n), 25)
    b = _rotate_z(oracle.run(cfg, st, 25), tab["e19"], tab["e7"], n)
    fl = oracle.fields(cfg, b)["fl"]
    assert 0.05 < fl.mean() < 0.95 and np.abs(oracle.fields(cfg, b)["ux"]).max() > 1e-4
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-13 * np.abs(y).max()


# --------------------------------------------------------- conservation --
def _closed_box(n=(10, 8, 6), **kw):
    return W.base_config(*n, flow=1, face_bc=[W.ADIABATIC] * 6, face_T=[0.0] * 6,
                         g_beta=2e-3, latent=1.0, lambda_s=0.08, lambda_l=0.08, nu=0.05, **kw)


def test_mass_and_enthalpy_conserved_in_adiabatic_box():
    cfg = _closed_box()
    T0 = W.random_temperature(cfg, seed=1, lo=-0.5, hi=2.0)
    st = oracle.init_state(cfg, T0)
    _, hist = oracle.run(cfg, st, 300, history=True)
    H, mass, flux = hist[:, 0], hist[:, 1], hist[:, 3]
    assert np.all(flux == 0.0)
    assert np.abs(mass / mass[0] - 1).max() < 1e-13
    assert np.abs(H - H[0]).max() < 1e-13 * np.abs(H).max()


def test_enthalpy_budget_with_fixed_temperature_walls():
    """H(t+1) - H(t) equals the enthalpy entering through the anti-bounce-back links."""
    cfg = W.base_config(9, 7, 6, flow=1, face_bc=[W.DIRICHLET, W.DIRICHLET, W.ADIABATIC,
                                                  W.ADIABATIC, W.DIRICHLET, W.PERIODIC * 0 + W.ADIABATIC],
                        face_T=[1.0, -0.3, 0, 0, 0.4, 0], g_beta=3e-3, latent=2.0,
                        lambda_s=0.1, lambda_l=0.1, nu=0.04)
    tw = W.wall_fields(cfg, {0: 1.0 + 0.1 * np.random.default_rng(3).uniform(-1, 1, 7 * 6)})
    st = oracle.init_state(cfg, W.random_temperature(cfg, seed=2))
    _, hist = oracle.run(cfg, st, 200, tw=tw, history=True)
    dH = np.diff(hist[:, 0])
    assert np.abs(dH - hist[:-1, 3]).max() < 1e-13 * np.abs(hist[:, 0]).max()
    assert np.abs(hist[:, 3]).max() > 1e-3


def test_fixed_point_at_melting_temperature():
    """All walls at T_m and the solid at T_m: nothing changes (T_ref = T_m, so no
    buoyancy; g = 0 and f at rest)."""
    cfg = W.melting_cavity(8, 1e5, 0.02, 0.1, precision=W.FP64)
    cfg["face_T"] = [0.0] * 6
    st0 = oracle.init_state(cfg)
    st = oracle.run(cfg, st0, 50)
    assert np.array_equal(st[1], st0[1])
    assert np.abs(st[0] - st0[0]).max() < 1e-15


# ------------------------------------------------ linear-stability pins --
def _d3q7_operator(k, cfg):
    """Per-wavenumber D3Q7 step for an all-liquid medium at rest, built from the
    polynomial moment basis: one step multiplies the Fourier amplitude by
    A = diag(exp(-i k.e)) C."""
    e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    ex, ey, ez = e.T
    e2 = (e**2).sum(1)
    N = np.stack([np.ones(7), ex, ey, ez, 6 - 7 * e2, 3 * ex**2 - e2, ey**2 - ez**2]).astype(float)
    sig = 1 / (cfg["lambda_l"] / (cfg["omega_T"]) + 0.5)
    R = np.diag([sig, sig, sig, sig, 2 - sig, 2 - sig, 2 - sig])
    # n^eq perturbation for u = 0: (dh, 0, 0, 0, 6 dh - 21 omega_T dT, 0, 0), dT = dh / C_p,l
    Q = np.zeros((7, 7))
    Q[0, :] = 1
    Q[4, :] = 6 - 21 * cfg["omega_T"] / cfg["cp_l"]
    C = np.eye(7) - np.linalg.inv(N) @ R @ (N - Q)
    return np.diag(np.exp(-1j * (e @ k))) @ C


def test_diffusion_mode_decay_matches_lattice_eigenvalue_and_eq34():
    """A sine temperature mode in a periodic all-liquid box decays per step by the
    dominant eigenvalue of the linear step operator, and that rate is
    chi k^2 with chi from Eq. (34) up to O(k^4)."""
    n = 32
    lam = 0.07
    cfg = W.base_config(n, 4, 4, flow=0, face_bc=[W.PERIODIC] * 6, lambda_s=lam,
                        lambda_l=lam, latent=1.0)
    kx = 2 * math.pi / n
    x = np.arange(n)
    T0 = 1.0 + 1e-3 * np.cos(kx * x)
    T0 = np.broadcast_to(T0, (4, 4, n)).copy()
    st = oracle.init_state(cfg, T0)
    steps = 200
    st = oracle.run(cfg, st, 100)        # let the non-hydrodynamic modes die out
    a0 = np.abs(np.fft.fft(oracle.fields(cfg, st)["T"][0, 0])[1])
    st = oracle.run(cfg, st, steps)
    a1 = np.abs(np.fft.fft(oracle.fields(cfg, st)["T"][0, 0])[1])
    rate = (a1 / a0) ** (1 / steps)
    ev = np.linalg.eigvals(_d3q7_operator(np.array([kx, 0, 0]), cfg))
    lead = ev[np.argmax(np.abs(ev))]
    assert abs(lead.imag) < 1e-12
    assert rate == pytest.approx(lead.real, abs=1e-12)
    chi = (1 / (1 / (lam / 0.25 + 0.5)) - 0.5) * 0.25   # Eq. (34)
    assert -math.log(rate) == pytest.approx(chi * kx**2, rel=5 * kx**2)


def _d3q19_operator(k, cfg):
    e = oracle.tables()["e19"]
    ex, ey, ez = e.T
    e2 = (e**2).sum(1)
    q, p = 5 * e2 - 9, 3 * e2 - 5
    M = np.stack([np.ones(19), 19 * e2 - 30, (21 * e2**2 - 53 * e2 + 24) / 2, ex, q * ex, ey,
                  q * ey, ez, q * ez, 3 * ex**2 - e2, p * (3 * ex**2 - e2), ey**2 - ez**2,
                  p * (ey**2 - ez**2), ex * ey, ey * ez, ex * ez, ex * (ey**2 - ez**2),
                  ey * (ez**2 - ex**2), ez * (ex**2 - ey**2)])
    s_nu = 1 / (3 * cfg["nu"] + 0.5)
    L = np.diag([0, cfg["s_e"], cfg["s_eps"], 0, cfg["s_q"], 0, cfg["s_q"], 0, cfg["s_q"], s_nu,
                 cfg["s_pi"], s_nu, cfg["s_pi"], s_nu, s_nu, s_nu, cfg["s_t"], cfg["s_t"], cfg["s_t"]])
    # linear part of m^eq about rest: rho (1, -11, 3), j (1, -2/3) per axis
    Q = np.zeros((19, 19))
    Q[0], Q[1], Q[2] = M[0], -11 * M[0], 3 * M[0]
    for a, b in ((3, 4), (5, 6), (7, 8)):
        Q[a] = M[a]
        Q[b] = -2 / 3 * M[a]
    C = np.eye(19) - np.linalg.inv(M) @ L @ (M - Q)
    return np.diag(np.exp(-1j * (e @ k))) @ C


def test_shear_wave_decay_matches_lattice_eigenvalue_and_eq59():
    """Seed the shear eigenvector of the linear D3Q19 MRT operator (built here from
    the polynomial moment basis) as a small transverse wave u_z(x): the oracle must
    keep it an eigenvector and scale it by the eigenvalue each step; that rate is
    nu k^2 with nu from Eq. (59) up to O(k^4)."""
    n = 32
    nu = 0.04
    cfg = W.base_config(n, 4, 4, flow=1, face_bc=[W.PERIODIC] * 6, nu=nu, g_beta=0.0,
                        latent=1.0, lambda_s=0.05, lambda_l=0.05)
    kx = 2 * math.pi / n
    ev, vec = np.linalg.eig(_d3q19_operator(np.array([kx, 0, 0]), cfg))
    e = oracle.tables()["e19"]
    # the shear mode: real eigenvalue near 1 - nu k^2 whose eigenvector carries j_z
    jz = np.abs(e[:, 2] @ vec)
    cand = [i for i in range(19) if abs(ev[i].imag) < 1e-12 and jz[i] > 1e-3]
    i = min(cand, key=lambda i: abs(ev[i].real - (1 - nu * kx**2)))
    lam, v = ev[i].real, vec[:, i]
    v = v / (e[:, 2] @ v)                      # unit momentum amplitude
    T0 = np.full((4, 4, n), 1.5)               # all liquid
    f, g = oracle.init_state(cfg, T0)
    eps = 1e-5
    phase = np.exp(1j * kx * np.arange(n))
    wave = eps * np.real(v[:, None] * phase[None, :])
    d0 = np.broadcast_to(wave[:, None, None, :], f.shape)
    steps = 200
    st = oracle.run(cfg, (f + d0, g), steps)

    def amp(d):  # complex amplitude of the e^{ikx} component of each population
        return 2 * (d * np.conj(phase)).mean(axis=(1, 2, 3))
    c0, c1 = amp(d0), amp(st[0] - f)
    assert np.abs(c1 - lam**steps * c0).max() < 1e-9 * np.abs(c0).max()
    rate = (np.vdot(c0, c1).real / np.vdot(c0, c0).real) ** (1 / steps)
    assert rate == pytest.approx(lam, abs=1e-12)
    assert -math.log(rate) == pytest.approx(nu * kx**2, rel=5 * kx**2)


def test_body_force_poiseuille_is_exact():
    """Flow between halfway bounce-back walls driven by a uniform buoyancy force
    (all liquid, uniform T, low Mach so that the O(u^2) density variation is
    negligible): with (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16 and the same
    for s_t, the steady profile is the parabola F x (H - x) / (2 rho nu), walls at
    x = 0 and x = H, nodes at i + 1/2."""
    H = 8
    nu = 0.1
    s_nu = 1 / (3 * nu + 0.5)
    s_magic = 1 / (3 / 16 / (1 / s_nu - 0.5) + 0.5)
    cfg = W.base_config(H, 2, 2, flow=1, face_bc=[W.ADIABATIC, W.ADIABATIC] + [W.PERIODIC] * 4,
                        face_T=[0.0] * 6, nu=nu, s_q=s_magic, s_t=s_magic, g_beta=1e-7,
                        latent=1.0, lambda_s=0.1, lambda_l=0.1, T_ref=0.0)
    T0 = np.full((2, 2, H), 2.0)     # liquid, T - T_ref = 2
    st = oracle.init_state(cfg, T0)
    st = oracle.run(cfg, st, 4000)
    fl = oracle.fields(cfg, st)
    x = np.arange(H) + 0.5
    F = 1e-7 * 2.0
    want = F * x * (H - x) / (2 * 1.0 * nu)
    assert np.allclose(fl["uz"][0, 0], want, rtol=1e-9, atol=1e-14)
    assert np.abs(fl["ux"]).max() < 1e-15


# ----------------------------------------------------------- tangent mode --
def test_tangent_matches_central_difference():
    """The dual-number tangent of the final liquid fraction w.r.t. one hot-wall node
    equals a central difference of the FP64 runs."""
    cfg = W.melting_cavity(6, 1e4, 1.0, 0.1, precision=W.FP64)
    tw = W.wall_fields(cfg, {0: W.hot_wall_field(6, 6)})
    st = oracle.init_state(cfg)
    st = oracle.run(cfg, st, 30, tw=tw)
    node = 7
    dtw = np.zeros_like(tw)
    dtw[node] = 1.0
    L, dL = oracle.run_tangent(cfg, st, 40, tw=tw, dtw=dtw)
    d = 1e-5
    Lp = oracle.loss(cfg, oracle.run(cfg, st, 40, tw=tw + d * dtw))
    Lm = oracle.loss(cfg, oracle.run(cfg, st, 40, tw=tw - d * dtw))
    assert L == pytest.approx(oracle.loss(cfg, oracle.run(cfg, st, 40, tw=tw)), rel=1e-15)
    assert dL == pytest.approx((Lp - Lm) / (2 * d), rel=1e-6)
    assert abs(dL) > 1e-3
