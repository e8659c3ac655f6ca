"""Helpers shared by the GPU tests (test side only)."""
from __future__ import annotations

import numpy as np

import workloads as W

# D3Q19 rest weights, used only to scale random test states
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _np(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def rel(a, b):
    """Largest relative difference.  Population arrays ([q][z][y][x], q = 7 or
    19) are compared plane by plane, each against its own largest value, so
    that the small moving populations are held to the same relative bound as
    the large rest populations; other arrays against their largest value."""
    a, b = _np(a), _np(b)
    if a.ndim == 4 and a.shape[0] in (7, 19):
        return max(rel(a[q], b[q]) for q in range(a.shape[0]))
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def rel_from(a, b, b0, frac=1e-2):
    """rel() for runs that relax toward rest: each population plane of a
    against b, with the plane's scale floored at frac times its largest value
    in the starting state b0 (the moving populations of a box that settles to
    a uniform state shrink by orders of magnitude while rounding differences
    keep the size set by the larger quantities of the collision)."""
    a, b, b0 = _np(a), _np(b), _np(b0)
    out = 0.0
    for q in range(b.shape[0]):
        scale = max(np.abs(b[q]).max(), frac * np.abs(b0[q]).max())
        out = max(out, float(np.abs(a[q] - b[q]).max() / (scale if scale > 0 else 1.0)))
    return out


def plane_scales(b):
    """Largest |value| of every population plane (diagnostics)."""
    b = _np(b)
    return [float(np.abs(b[q]).max()) for q in range(b.shape[0])]


def absdiff(a, b):
    a, b = _np(a), _np(b)
    return float(np.abs(a - b).max())


def random_walls(cfg, seed, amp=0.1):
    """Per-node temperatures for every fixed-temperature face."""
    rng = np.random.default_rng(seed)
    over = {}
    for face, shp in enumerate(W.face_shapes(cfg)):
        if cfg["face_bc"][face] == W.DIRICHLET:
            over[face] = cfg["face_T"][face] + amp * rng.uniform(-1, 1, size=shp)
    return over


def make_cavity(cfg, T0=None, walls=None):
    from paper_1703_02652_amd import Cavity
    cav = Cavity(cfg, T0=T0, device="cuda")
    for face, field in (walls or {}).items():
        cav.set_wall_T(face, field)
    return cav
