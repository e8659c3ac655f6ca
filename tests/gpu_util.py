"""Helpers shared by the GPU tests (test side only)."""
from __future__ import annotations

import numpy as np

import workloads as W

# D3Q19 rest weights, used only to scale random test states
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def rel(a, b):
    """max |a - b| / max |b| (relative to the field's scale)."""
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    b = b.detach().cpu().numpy() if hasattr(b, "detach") else np.asarray(b)
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def absdiff(a, b):
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    b = b.detach().cpu().numpy() if hasattr(b, "detach") else np.asarray(b)
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
