"""Tiny pure-numpy implementation of one time step, written independently of the
oracle: the whole lattice is one long vector, streaming is a global index
permutation (plus the affine wall term), and the collision is assembled per cell
from the polynomial moment bases.  Only usable for a few hundred cells."""
from __future__ import annotations

import itertools

import numpy as np

E7 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
E19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]])


def _opp(E):
    return np.array([next(j for j in range(len(E)) if (E[j] == -E[i]).all()) for i in range(len(E))])


def basis7(E):
    ex, ey, ez = E.T
    e2 = (E**2).sum(1)
    return np.stack([np.ones(len(E)), ex, ey, ez, 6 - 7 * e2, 3 * ex**2 - e2, ey**2 - ez**2]).astype(float)


def basis19(E):
    ex, ey, ez = E.T
    e2 = (E**2).sum(1)
    q, p = 5 * e2 - 9, 3 * e2 - 5
    return np.stack([np.ones(19), 19 * e2 - 30, (21 * e2**2 - 53 * e2 + 24) / 2, ex, q * ex, ey,
                     q * ey, ez, q * ez, 3 * ex**2 - e2, p * (3 * ex**2 - e2), ey**2 - ez**2,
                     p * (ey**2 - ez**2), ex * ey, ey * ez, ex * ez, ex * (ey**2 - ez**2),
                     ey * (ez**2 - ex**2), ez * (ex**2 - ey**2)]).astype(float)


def stream_maps(cfg, E):
    """For each (q, cell) of the post-streaming vector: source index into the
    post-collision vector, sign, and the face it came through (-1 if interior)."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    dims = (nx, ny, nz)
    opp = _opp(E)
    n = nx * ny * nz
    src = np.zeros((len(E), n), dtype=np.int64)
    face = -np.ones((len(E), n), dtype=np.int64)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        c = x + nx * (y + ny * z)
        for a, e in enumerate(E):
            p = [x - e[0], y - e[1], z - e[2]]
            fc = -1
            for d in range(3):
                if p[d] < 0 or p[d] >= dims[d]:
                    if cfg["face_bc"][2 * d] == 0:
                        p[d] %= dims[d]
                    else:
                        fc = 2 * d + (0 if p[d] < 0 else 1)
            if fc < 0:
                src[a, c] = a * n + p[0] + nx * (p[1] + ny * p[2])
            else:
                src[a, c] = opp[a] * n + c
                face[a, c] = fc
    return src, face


def step(cfg, f, g, tw_faces):
    """One step on SoA arrays f [19][n], g [7][n] (flattened cells).  tw_faces(face,
    cell) returns the wall temperature seen by that cell through that face."""
    n = g.shape[1]
    w = cfg["omega_T"]
    W7 = np.array([1 - 3 * w] + [w / 2] * 6)
    N = basis7(E7)
    M = basis19(E19)
    h = g.sum(0)
    hs = cfg["cp_s"] * cfg["T_m"]
    hl = cfg["cp_l"] * cfg["T_m"] + cfg["latent"]
    fl = np.clip((h - hs) / (hl - hs), 0.0, 1.0)
    T = np.where(h <= hs, h / cfg["cp_s"], np.where(h >= hl, (h - cfg["latent"]) / cfg["cp_l"],
                                                   cfg["T_m"]))
    cp = cfg["cp_s"] + fl * (cfg["cp_l"] - cfg["cp_s"])
    lam = cfg["lambda_s"] + fl * (cfg["lambda_l"] - cfg["lambda_s"])
    tau = lam / (cfg["rho0"] * cfg["cp_ref"] * w) + 0.5
    u = np.zeros((3, n))
    fs = None
    if cfg["flow"]:
        rho = f.sum(0)
        S = E19.T @ f
        Fb = np.zeros((3, n))
        Fb[2] = cfg["g_beta"] * cfg["rho0"] * (T - cfg["T_ref"])
        u = fl * (S + Fb / 2) / rho
        F = 2 * (rho * u - S)
        m = M @ f
        u2 = (u**2).sum(0)
        ux, uy, uz = u
        meq = np.stack([rho, rho * (-11 + 19 * u2), rho * (3 - 5.5 * u2), rho * ux, -2 / 3 * rho * ux,
                        rho * uy, -2 / 3 * rho * uy, rho * uz, -2 / 3 * rho * uz,
                        rho * (3 * ux**2 - u2), -0.5 * rho * (3 * ux**2 - u2),
                        rho * (uy**2 - uz**2), -0.5 * rho * (uy**2 - uz**2),
                        rho * ux * uy, rho * uy * uz, rho * ux * uz,
                        0 * rho, 0 * rho, 0 * rho])
        # forcing moments from the velocity-space Guo term projected with M
        W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
        eu = E19 @ u
        eF = E19 @ F
        uF = (u * F).sum(0)
        Fg = W19[:, None] * (3 * (eF - uF) + 9 * eu * eF)
        FF = M @ Fg
        s_nu = 1 / (3 * cfg["nu"] + 0.5)
        Ld = np.array([0, cfg["s_e"], cfg["s_eps"], 0, cfg["s_q"], 0, cfg["s_q"], 0, cfg["s_q"], s_nu,
                       cfg["s_pi"], s_nu, cfg["s_pi"], s_nu, s_nu, s_nu, cfg["s_t"], cfg["s_t"],
                       cfg["s_t"]])[:, None]
        fs = np.linalg.solve(M, m - Ld * (m - meq) + (1 - Ld / 2) * FF)
    eu7 = E7 @ u
    geq = W7[:, None] * cfg["cp_ref"] * T + eu7 / w * W7[:, None] * cp * T
    geq[0] = h - 3 * w * cfg["cp_ref"] * T
    if cfg["enth_model"] == 0:
        gs = g - (g - geq) / tau
    else:
        sig = 1 / tau
        sg = np.stack([sig] * 4 + [2 - sig] * 3)
        ov = np.asarray(cfg["sigma_override"], float)
        for k in range(7):
            if np.isfinite(ov[k]):
                sg[k] = ov[k]
        gs = g - np.linalg.solve(N, sg * (N @ g - N @ geq))
    # streaming as one permutation of the concatenated vector
    out_f = None
    if cfg["flow"]:
        src, _ = stream_maps(cfg, E19)
        out_f = fs.reshape(-1)[src.reshape(-1)].reshape(19, n)
    src, face = stream_maps(cfg, E7)
    out_g = gs.reshape(-1)[src.reshape(-1)].reshape(7, n)
    for a in range(7):
        for c in range(n):
            fc = face[a, c]
            if fc >= 0 and cfg["face_bc"][fc] == 1:
                out_g[a, c] = -out_g[a, c] + 2 * W7[a] * cfg["cp_ref"] * tw_faces(fc, c)
    return out_f, out_g
