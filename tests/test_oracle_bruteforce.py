"""The oracle against the independent tiny brute-force step (no GPU)."""
import numpy as np
import pytest

import bruteforce
import oracle
import workloads as W


def _face_lookup(cfg, tw):
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    sizes = [ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny]
    offs = np.concatenate([[0], np.cumsum(sizes)])

    def lookup(face, c):
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        d = face // 2
        node = (y + ny * z) if d == 0 else ((x + nx * z) if d == 1 else (x + nx * y))
        return tw[offs[face] + node]
    return lookup


CASES = [
    dict(model=W.MRT, bc=[W.DIRICHLET, W.DIRICHLET, W.ADIABATIC, W.ADIABATIC, W.ADIABATIC,
                          W.ADIABATIC], flow=1),
    dict(model=W.SRT, bc=[W.DIRICHLET, W.ADIABATIC, W.PERIODIC, W.PERIODIC, W.DIRICHLET,
                          W.ADIABATIC], flow=1),
    dict(model=W.MRT, bc=[W.PERIODIC] * 4 + [W.DIRICHLET, W.DIRICHLET], flow=0),
    dict(model=W.MRT, bc=[W.ADIABATIC, W.DIRICHLET, W.DIRICHLET, W.ADIABATIC, W.PERIODIC,
                          W.PERIODIC], flow=1, props=True),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_oracle_matches_bruteforce(case):
    c = CASES[case]
    kw = {}
    if c.get("props"):
        kw = dict(cp_s=1.0, cp_l=1.6, lambda_s=0.12, lambda_l=0.05, T_m=0.2)
    cfg = W.base_config(4, 3, 5, flow=c["flow"], enth_model=c["model"], face_bc=c["bc"],
                        face_T=[1.0, -0.5, 0.3, 0.7, 0.9, -0.2], g_beta=5e-3, latent=1.5,
                        **{"lambda_s": 0.09, "lambda_l": 0.09, **kw})
    rng = np.random.default_rng(case)
    tw = W.wall_fields(cfg) + 0.05 * rng.uniform(-1, 1, W.wall_fields(cfg).size)
    T0 = W.random_temperature(cfg, seed=10 + case, lo=-0.6, hi=2.5)
    f, g = oracle.init_state(cfg, T0)
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    bf = (f.reshape(19, n).copy() if f is not None else None, g.reshape(7, n).copy())
    st = (f, g)
    look = _face_lookup(cfg, tw)
    for _ in range(10):
        bf = bruteforce.step(cfg, bf[0], bf[1], look)
        st = oracle.run(cfg, st, 1, tw=tw)
    assert np.allclose(st[1].reshape(7, n), bf[1], rtol=0, atol=1e-13)
    if c["flow"]:
        assert np.allclose(st[0].reshape(19, n), bf[0], rtol=0, atol=1e-14)
