"""Pins of the oracle on the 2D validations of Sec. 3.2, run as one-cell-thick
slabs in the xz plane with y periodic: solidification in a corner (Sec. 3.2.1)
and melting with convection (Sec. 3.2.2, Table 1, Eq. (65))."""
import math

import numpy as np
from scipy.special import erf, erfc

import oracle
import workloads as W
from analytic import neumann_melting_k, solidification_k


def _corner(n, steps, chi=0.2):
    cfg = W.corner_solidification(n=n, chi=chi)
    st = oracle.init_state(cfg, np.full((n, 1, n), 0.3))
    st = oracle.run(cfg, st, steps)
    f = oracle.fields(cfg, st)
    return cfg, f["fl"][:, 0, :], f["T"][:, 0, :]   # [z][x]


def test_corner_solidification_is_symmetric_in_x_and_z():
    """Both cooled faces are equal and the D3Q7 MRT operator with
    sigma_4 = sigma_5 = sigma_6 is isotropic, so the solution is symmetric
    under x <-> z (up to rounding of the summation order)."""
    _, fl, T = _corner(40, 500)
    assert 0.05 < fl.mean() < 0.95
    assert np.abs(fl - fl.T).max() < 1e-10
    assert np.abs(T - T.T).max() < 1e-10


def test_corner_far_from_the_corner_is_the_1d_two_phase_solution():
    """Away from the corner (rows around z = n/2, where the z = 0 face has not
    been felt) the front along x and the temperature follow the two-phase
    Neumann solution, Eq. (62)-(63), with Ste_s = C_p (T_f - T_l) / L = 4 and
    Ste_l = C_p (T0 - T_f) / L = 1.2; near the corner the solid is thicker."""
    n, chi = 128, 0.2
    k = solidification_k(4.0, 1.2, chi, chi)
    t = int(round((16.0 / (2.0 * k)) ** 2 / chi))      # front near 16 cells
    _, fl, T = _corner(n, t, chi)
    rows = slice(n // 2 - 8, n // 2 + 8)
    X_num = (1.0 - fl[rows]).sum(axis=1).mean()
    X_ex = 2.0 * k * math.sqrt(chi * t)
    assert abs(X_num / X_ex - 1.0) < 0.03
    x = np.arange(n) + 0.5
    s = 2.0 * math.sqrt(chi * t)
    T_ex = np.where(x <= X_ex, -1.0 + erf(x / s) / erf(k),
                    0.3 - 0.3 * erfc(x / s) / erfc(k))
    assert np.abs(T[rows] - T_ex).max() < 0.03
    # along the bisector the two cold faces together freeze further
    d = np.array([1.0 - fl[i, i] for i in range(n)]).sum() * math.sqrt(2.0)
    assert d > 1.2 * X_ex


def test_slab_is_y_invariant():
    """A slab one cell thick along periodic y evolves exactly like a thicker
    periodic slab with the same y-independent initial state (flow on)."""
    cfg1 = W.convection_2d(16, precision=W.FP64)
    cfg1.update(nu=0.02, lambda_s=0.05, lambda_l=0.05, g_beta=2e-3, latent=2.0)
    cfg3 = dict(cfg1, ny=3)
    T0 = W.random_temperature(cfg1, seed=21, lo=-0.3, hi=1.0)
    a = oracle.fields(cfg1, oracle.run(cfg1, oracle.init_state(cfg1, T0), 150))
    b = oracle.fields(cfg3, oracle.run(cfg3, oracle.init_state(cfg3, np.repeat(T0, 3, axis=1)), 150))
    assert np.abs(a["uz"]).max() > 1e-4
    for key in ("h", "T", "fl", "rho", "ux", "uz"):
        for y in range(3):
            assert np.array_equal(a[key][:, 0, :], b[key][:, y, :]), key
        assert np.abs(b["uy"]).max() < 1e-14    # y -> -y mirror holds to rounding


def _conduction_nu_mean(n_x, X1, X2):
    """Mean of Eq. (65) over the steps in which the front moves from X1 to X2
    cells, from the lattice wall flux, and the same mean of the exact
    one-phase Neumann value Nu = 1 / (erf(k) sqrt(pi Fo))."""
    cfg = W.convection_2d(n_x, precision=W.FP64, buoyancy=False)
    cfg.update(nz=2, flow=0)   # u stays 0 without buoyancy
    chi = cfg["lambda_l"]
    k = neumann_melting_k(0.01)
    t1, t2 = (int(round((X / (2.0 * k)) ** 2 / chi)) for X in (X1, X2))
    st = oracle.run(cfg, oracle.init_state(cfg), t1)
    _, hist = oracle.run(cfg, st, t2 - t1, history=True)
    q = hist[:, 3].mean() / (cfg["ny"] * cfg["nz"])       # inflow through x- per step
    nu_num = q * n_x / (chi * cfg["cp_ref"] * 1.0)
    fo1, fo2 = chi * t1 / n_x ** 2, chi * t2 / n_x ** 2
    nu_ex = 2.0 * (math.sqrt(fo2) - math.sqrt(fo1)) / (erf(k) * math.sqrt(math.pi) * (fo2 - fo1))
    return nu_num, nu_ex


def test_conduction_melting_nusselt_follows_neumann():
    """With g beta = 0 the Table 1 slab is the one-phase Neumann problem along
    x.  At Ste = 0.01 the lattice Nu is a staircase n_x / (m + 1/2) (m cells
    melted: the mushy cell pins T_m at its centre); its mean over the melting
    of many cells equals the mean of the exact Nu, and the error falls as the
    front moves away from the wall."""
    e = []
    for X1, X2 in ((4.0, 10.0), (10.0, 25.0)):
        nu_num, nu_ex = _conduction_nu_mean(64, X1, X2)
        e.append(abs(nu_num / nu_ex - 1.0))
    assert e[0] < 1e-3 and e[1] < 1e-4      # observed 3e-5 and 6e-6
    assert e[1] < 0.6 * e[0]
