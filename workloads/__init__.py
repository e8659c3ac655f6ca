"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module only builds inputs: cavity descriptions (plain dicts of lattice-unit
numbers), wall-temperature fields, initial temperature fields and random
population states.  It holds none of the lattice Boltzmann arithmetic: no
equilibria, no collision, no streaming.  Both the product binding and the oracle
binding marshal the same dict into their own C structs.

Units: every number is in lattice units, delta_x = delta_t = c = 1.

Mapping from dimensionless groups (Eq. (64), Sec. 3.2.2): the characteristic
length is the hot-to-cold distance in cells, l_c = nx, and Delta T = T_h - T_m.
The velocity scale is U = Ma * c_s with c_s = 1/sqrt(3).  From Ra, Pr and the
definitions of Eq. (64):
    nu   = U * l_c * sqrt(Pr / Ra)
    chi  = nu / Pr
    g_beta = U**2 / (Delta T * l_c)        (so that Ra = g_beta dT l_c^3 / (nu chi))
    L    = C_p * Delta T / Ste
The thermal relaxation is given by the conductivity lambda = rho0 * C_p,ref * chi,
from which each side derives its own relaxation rates.
"""
from __future__ import annotations

import math

import numpy as np

# face order used everywhere: x-, x+, y-, y+, z-, z+
PERIODIC = 0
DIRICHLET = 1    # fixed temperature, no-slip
ADIABATIC = 2    # zero heat flux, no-slip

FP64, FP32, FP16S, BF16S = 0, 1, 2, 3
SRT, MRT = 0, 1

# Free D3Q19 relaxation rates that the paper leaves open (Eq. (52)): the common
# set of d'Humieres et al. (2002), the paper's Ref. [20].
DEFAULT_RATES = dict(s_e=1.19, s_eps=1.4, s_q=1.2, s_pi=1.4, s_t=1.98)

CONFIG_KEYS = (
    "nx", "ny", "nz", "flow", "enth_model", "precision", "face_bc", "face_T",
    "omega_T", "cp_s", "cp_l", "cp_ref", "lambda_s", "lambda_l", "latent", "T_m",
    "rho0", "nu", "s_e", "s_eps", "s_q", "s_pi", "s_t", "g_beta", "T_ref",
    "sigma_override", "T_shift",
)


def base_config(nx, ny, nz, **kw):
    """A cavity description with neutral defaults; keyword arguments override."""
    cfg = dict(
        nx=int(nx), ny=int(ny), nz=int(nz), flow=1, enth_model=MRT, precision=FP64,
        face_bc=[DIRICHLET, DIRICHLET, ADIABATIC, ADIABATIC, ADIABATIC, ADIABATIC],
        face_T=[1.0, 0.0, 0.0, 0.0, 0.0, 0.0],
        omega_T=0.25, cp_s=1.0, cp_l=1.0, cp_ref=1.0, lambda_s=0.1, lambda_l=0.1,
        latent=10.0, T_m=0.0, rho0=1.0, nu=0.05, g_beta=0.0, T_ref=0.0,
        sigma_override=[float("nan")] * 7, T_shift=0.0,
    )
    cfg.update(DEFAULT_RATES)
    for k, v in kw.items():
        if k not in CONFIG_KEYS:
            raise KeyError(f"unknown cavity key {k!r}")
        cfg[k] = v
    cfg["face_bc"] = [int(b) for b in cfg["face_bc"]]
    cfg["face_T"] = [float(t) for t in cfg["face_T"]]
    cfg["sigma_override"] = [float(s) for s in cfg["sigma_override"]]
    return cfg


def lattice_from_groups(n_hot_cold, Ra, Pr, Ste, Ma=0.1, dT=1.0, cp=1.0):
    """Eq. (64) solved for lattice-unit nu, chi, g*beta and L (see module doc)."""
    U = Ma / math.sqrt(3.0)
    nu = U * n_hot_cold * math.sqrt(Pr / Ra)
    chi = nu / Pr
    g_beta = U * U / (dT * n_hot_cold)
    latent = cp * dT / Ste
    return dict(nu=nu, chi=chi, g_beta=g_beta, latent=latent)


def melting_cavity(n, Ra, Pr, Ste, precision=FP32, Ma=0.1, enth_model=MRT):
    """Cubic cavity melting (Sec. 3.3): solid at T_m = 0, hot wall x- at T_h = 1,
    cold wall x+ at T_m, the four other faces adiabatic; all walls no-slip;
    buoyancy along +z with T_ref = T_m.  The 16-bit formats store the moving
    enthalpy populations relative to the mid temperature of the two walls."""
    p = lattice_from_groups(n, Ra, Pr, Ste, Ma)
    chi = p["chi"]
    return base_config(
        n, n, n, flow=1, enth_model=enth_model, precision=precision,
        face_bc=[DIRICHLET, DIRICHLET, ADIABATIC, ADIABATIC, ADIABATIC, ADIABATIC],
        face_T=[1.0, 0.0, 0.0, 0.0, 0.0, 0.0],
        lambda_s=chi, lambda_l=chi, latent=p["latent"], nu=p["nu"], g_beta=p["g_beta"],
        T_shift=0.5,
    )


# --------------------------------------------------------------------------- #
# The named workloads
# --------------------------------------------------------------------------- #
def stefan_1d(enth_model=MRT, axis=0, n=64, width=4, chi=0.05, Ste=0.1):
    """1D conduction melting (Sec. 3.1.1) on an n x width x width lattice along
    `axis`, periodic across it, Dirichlet T_h = 1 at the low face, adiabatic at
    the high face; enthalpy distribution only, FP64.  Solid starts at T_m = 0."""
    dims = [width, width, width]
    dims[axis] = n
    bc = [PERIODIC] * 6
    bc[2 * axis] = DIRICHLET
    bc[2 * axis + 1] = ADIABATIC
    fT = [0.0] * 6
    fT[2 * axis] = 1.0
    return base_config(*dims, flow=0, enth_model=enth_model, precision=FP64,
                       face_bc=bc, face_T=fT, lambda_s=chi, lambda_l=chi,
                       latent=1.0 / Ste, nu=0.1, g_beta=0.0)


def cavity_128(precision=FP32):
    """Natural-convection melting at 128^3: Ra = 1e5, Pr = 0.02, Ste = 0.1."""
    return melting_cavity(128, 1e5, 0.02, 0.1, precision=precision)


def precision_cavity(n=256, Pr=0.02, precision=FP16S):
    """Precision variant: Ra = 1e6, Pr in {0.02, 6.2}, Ste = 0.1."""
    return melting_cavity(n, 1e6, Pr, 0.1, precision=precision)


def adjoint_cavity(n=96, precision=FP64):
    """Differentiation workload: Ra = 1e4, Pr = 1, Ste = 0.1."""
    return melting_cavity(n, 1e4, 1.0, 0.1, precision=precision)


# Sec. 3.3, Table 2: grid (x, y, z), Pr, Ra; Ste = 0.4 for all three cases.
TABLE2 = {1: ((160, 160, 80), 0.02, 2.5e4), 2: ((160, 160, 80), 10.0, 2.5e4),
          3: ((200, 200, 80), 10.0, 1.0e6)}


def table2_case(case, precision=FP32, Ma=0.1):
    """The paper's 3D melting cases on their printed grids (x hot-to-cold), with
    l_c = nx for the lattice mapping; otherwise as melting_cavity."""
    (nx, ny, nz), Pr, Ra = TABLE2[case]
    cfg = melting_cavity(nx, Ra, Pr, 0.4, precision=precision, Ma=Ma)
    cfg.update(ny=ny, nz=nz)
    return cfg


def corner_solidification(n=400, chi=0.2, precision=FP64, T0=0.3, T_wall=-1.0, Ste=4.0):
    """2D solidification in a corner (Sec. 3.2.1) on an n x 1 x n slab in the xz
    plane, periodic along y: liquid at T0 = 0.3 above T_f = T_m = 0, the faces
    x = 0 and z = 0 held at T_l = -1 from t = 0, Ste = C_p (T_f - T_l) / L = 4,
    equal solid and liquid properties, enthalpy only.  The quarter-infinite
    domain is truncated at x = n and z = n with the far faces held at T0."""
    latent = 1.0 * (0.0 - T_wall) / Ste
    return base_config(n, 1, n, flow=0, enth_model=MRT, precision=precision,
                       face_bc=[DIRICHLET, DIRICHLET, PERIODIC, PERIODIC, DIRICHLET, DIRICHLET],
                       face_T=[T_wall, T0, 0.0, 0.0, T_wall, T0],
                       lambda_s=chi, lambda_l=chi, latent=latent, T_m=0.0, nu=0.1, g_beta=0.0)


def convection_2d(n=128, precision=FP32, Ra=2.5e4, Pr=0.02, Ste=0.01, Ma=0.1, buoyancy=True):
    """2D melting with convection (Sec. 3.2.2, Table 1) on an n x 1 x n slab in
    the xz plane, periodic along y: solid at T_m = 0, x = 0 at T_h = 1, x = n at
    T_m, z faces adiabatic, no-slip; l_c = n.  buoyancy=False keeps g beta = 0
    (pure conduction, the one-phase Neumann problem along x)."""
    cfg = melting_cavity(n, Ra, Pr, Ste, precision=precision, Ma=Ma)
    cfg.update(ny=1, face_bc=[DIRICHLET, DIRICHLET, PERIODIC, PERIODIC, ADIABATIC, ADIABATIC])
    if not buoyancy:
        cfg["g_beta"] = 0.0
    return cfg


def hot_wall_field(ny, nz, seed=1703, amp=0.05):
    """Hot-wall temperature field T_w(y, z) = 1 + U(-amp, amp); layout [z][y]."""
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amp, amp, size=(nz, ny))


def fd_nodes(ny, nz, count=16, seed=2652):
    """Wall nodes (flat index y + ny*z) drawn without replacement."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(ny * nz, size=count, replace=False))


def batch_cavities(count=64, seed=355, precision=FP32, sizes=(32, 48, 64, 96)):
    """Uneven batch: N ~ U{sizes}, log10 Ra ~ U(3, 6), log10 Pr ~ U(log10 .02,
    log10 50), Ste ~ U(.05, .5).  Returns (configs, draws)."""
    rng = np.random.default_rng(seed)
    cfgs, draws = [], []
    for _ in range(count):
        n = int(rng.choice(sizes))
        Ra = 10.0 ** rng.uniform(3.0, 6.0)
        Pr = 10.0 ** rng.uniform(math.log10(0.02), math.log10(50.0))
        Ste = rng.uniform(0.05, 0.5)
        cfgs.append(melting_cavity(n, Ra, Pr, Ste, precision=precision))
        draws.append(dict(n=n, Ra=Ra, Pr=Pr, Ste=Ste))
    return cfgs, draws


# --------------------------------------------------------------------------- #
# Random states and fields for parity tests
# --------------------------------------------------------------------------- #
def random_populations(cfg, seed, f_scale, g_rest_range=(-1.0, 12.0), g_amp=0.15,
                       f_amp=0.2):
    """Random pre-collision populations in SoA layout [q][z][y][x] (FP64).

    f_alpha = f_scale[alpha] * (1 + f_amp * U(-1, 1)); the caller passes the
    per-direction scale.  g_0 is drawn from `g_rest_range` so that h = sum(g)
    lands in the solid, mushy and liquid ranges; g_1..6 = g_amp * U(-1, 2).
    No equilibrium is involved: these are arbitrary states."""
    rng = np.random.default_rng(seed)
    shp = (cfg["nz"], cfg["ny"], cfg["nx"])
    f_scale = np.asarray(f_scale, dtype=np.float64).reshape(19, 1, 1, 1)
    f = f_scale * (1.0 + f_amp * rng.uniform(-1.0, 1.0, size=(19,) + shp))
    g = np.empty((7,) + shp)
    g[0] = rng.uniform(*g_rest_range, size=shp)
    g[1:] = g_amp * rng.uniform(-1.0, 2.0, size=(6,) + shp)
    return f, g


def random_temperature(cfg, seed, lo=-0.5, hi=1.5, frac_at_melt=0.2):
    """Initial temperature field [z][y][x] with a fraction of cells exactly at T_m."""
    rng = np.random.default_rng(seed)
    shp = (cfg["nz"], cfg["ny"], cfg["nx"])
    T = rng.uniform(lo, hi, size=shp)
    T[rng.uniform(size=shp) < frac_at_melt] = cfg["T_m"]
    return T


def face_shapes(cfg):
    """(rows, cols) of each face's node field: x faces [nz][ny], y faces [nz][nx],
    z faces [ny][nx]."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    return [(nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)]


def wall_fields(cfg, overrides=None):
    """Concatenated per-node wall temperatures of the six faces (FP64, flat).
    Faces without an override take their constant face_T."""
    parts = []
    for face, shp in enumerate(face_shapes(cfg)):
        if overrides is not None and face in overrides:
            a = np.asarray(overrides[face], dtype=np.float64).reshape(shp)
        else:
            a = np.full(shp, cfg["face_T"][face], dtype=np.float64)
        parts.append(a.ravel())
    return np.concatenate(parts)
