"""Python face of the lbpc library: a batch of cavities on one HIP device.

PyTorch provides device memory (the workspace and the output tensors) and the
stream; all lattice Boltzmann work happens inside liblbpc.so.  A context is
bound to the torch stream that is current when it is created.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import FIELD_BITS, LbpcError, lib, make_configs


def _torch():
    import torch
    return torch


def _face_shape(cfg, face):
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    return [(nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)][face]


class Cavity:
    """A batch of one or more cavities advanced together.

    cfgs: one cavity dict or a list of them (keys of lbpc_config).
    T0:   None (T_m everywhere), or one array per cavity of shape (nz, ny, nx).
    """

    def __init__(self, cfgs, T0=None, device="cuda"):
        torch = _torch()
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = [dict(c) for c in cfgs]
        self.batch = len(self.cfgs)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("lbpc runs on a HIP device only")
        self._L = L = lib()
        self._arr = make_configs(self.cfgs)
        nbytes = L.lbpc_workspace_bytes(self._arr, self.batch)
        if nbytes == 0:
            raise LbpcError(-1, L.lbpc_last_error(None).decode())
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        t0 = None
        if T0 is not None:
            if self.batch == 1 and not isinstance(T0, (list, tuple)):
                T0 = [T0]
            parts = [torch.as_tensor(np.asarray(t, dtype=np.float64).reshape(-1)) for t in T0]
            t0 = torch.cat(parts).to(self.device)
            if t0.numel() != sum(c["nx"] * c["ny"] * c["nz"] for c in self.cfgs):
                raise ValueError("T0 does not match the cavity sizes")
        self._stream = torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        rc = L.lbpc_create(self._arr, self.batch, ctypes.c_void_p(self._ws_ptr), nbytes,
                           ctypes.c_void_p(t0.data_ptr() if t0 is not None else 0),
                           ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(self._ctx))
        if rc != 0:
            raise LbpcError(rc, L.lbpc_last_error(None).decode())
        self._adj_ws = None

    # ------------------------------------------------------------------ util
    def _check(self, rc):
        if rc != 0:
            raise LbpcError(rc, self._L.lbpc_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self._L.lbpc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ncell(self, cavity=0):
        c = self.cfgs[cavity]
        return c["nx"] * c["ny"] * c["nz"]

    def shape(self, cavity=0):
        c = self.cfgs[cavity]
        return (c["nz"], c["ny"], c["nx"])

    # ------------------------------------------------------------- stepping
    def step(self, n=1):
        self._check(self._L.lbpc_step(self._ctx, int(n)))

    def fields(self, cavity=0, names=("T", "fl")):
        torch = _torch()
        mask = 0
        for k in names:
            mask |= FIELD_BITS[k]
        order = [k for k in ("h", "T", "fl", "rho", "u") if mask & FIELD_BITS[k]]
        planes = sum(3 if k == "u" else 1 for k in order)
        out = torch.empty((planes,) + self.shape(cavity), dtype=torch.float64, device=self.device)
        self._check(self._L.lbpc_fields(self._ctx, cavity, mask, ctypes.c_void_p(out.data_ptr())))
        res, i = {}, 0
        for k in order:
            if k == "u":
                res["ux"], res["uy"], res["uz"] = out[i], out[i + 1], out[i + 2]
                i += 3
            else:
                res[k] = out[i]
                i += 1
        return res

    def state(self, cavity=0):
        torch = _torch()
        shp = self.shape(cavity)
        g = torch.empty((7,) + shp, dtype=torch.float64, device=self.device)
        f = None
        if self.cfgs[cavity]["flow"]:
            f = torch.empty((19,) + shp, dtype=torch.float64, device=self.device)
        self._check(self._L.lbpc_get_state(self._ctx, cavity,
                                           ctypes.c_void_p(f.data_ptr() if f is not None else 0),
                                           ctypes.c_void_p(g.data_ptr())))
        return f, g

    def set_state(self, f, g, cavity=0):
        torch = _torch()
        g = torch.as_tensor(g, dtype=torch.float64).to(self.device).contiguous()
        fp = 0
        if self.cfgs[cavity]["flow"]:
            f = torch.as_tensor(f, dtype=torch.float64).to(self.device).contiguous()
            fp = f.data_ptr()
        self._check(self._L.lbpc_set_state(self._ctx, cavity, ctypes.c_void_p(fp),
                                           ctypes.c_void_p(g.data_ptr())))
        self._stream.synchronize()

    def budgets(self):
        """(batch, 7): H, mass, sum f_l of the current state, wall inflow since
        creation, steps, inflow through the x- face in the next step, and the
        library's Nusselt number of the x- face (Eq. (65))."""
        out = np.zeros(7 * self.batch)
        self._check(self._L.lbpc_budgets(self._ctx, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.batch, 7)

    def nusselt(self, cavity=0, b=None):
        """Mean Nusselt number of the x- wall, Eq. (65), as lbpc_budgets
        returns it (b: an earlier budgets() result to read it from)."""
        b = self.budgets() if b is None else b
        return float(b[cavity, 6])

    def status(self):
        out = (ctypes.c_int32 * self.batch)()
        self._check(self._L.lbpc_status(self._ctx, out))
        return np.array(list(out), dtype=np.int32)

    def set_wall_T(self, face, Tw, cavity=0):
        torch = _torch()
        t = torch.as_tensor(Tw, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != _face_shape(self.cfgs[cavity], face) and t.numel() != int(
                np.prod(_face_shape(self.cfgs[cavity], face))):
            raise ValueError("wall field has the wrong shape")
        self._check(self._L.lbpc_set_wall_T(self._ctx, cavity, face, ctypes.c_void_p(t.data_ptr())))
        self._stream.synchronize()

    # --------------------------------------------------------- checkpoints
    def save(self) -> bytes:
        n = self._L.lbpc_state_bytes(self._ctx)
        buf = ctypes.create_string_buffer(n)
        self._check(self._L.lbpc_save(self._ctx, buf, n))
        return buf.raw

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self._L.lbpc_load(self._ctx, buf, len(blob)))

    # ------------------------------------------------------ launch shapes
    def set_launch(self, block=256, grid=0, graph_steps=16, xcd_run=4):
        """block: cells per tile (64..256); grid: 0 for one workgroup per tile,
        else a persistent grid; graph_steps: steps per HIP graph (<= 16, 0 none);
        xcd_run: tiles per XCD run of the queue (1 natural order), 0 for one
        y-block of every slab per XCD (see lbpc_set_launch)."""
        self._check(self._L.lbpc_set_launch(self._ctx, block, grid, graph_steps, xcd_run))

    def get_launch(self):
        """(block, grid, graph_steps, xcd_run)"""
        v = [ctypes.c_int32() for _ in range(4)]
        self._check(self._L.lbpc_get_launch(self._ctx, *[ctypes.byref(a) for a in v]))
        return tuple(a.value for a in v)

    def autotune(self, trial_steps=10):
        ms = ctypes.c_double()
        self._check(self._L.lbpc_autotune(self._ctx, trial_steps, ctypes.byref(ms)))
        return ms.value

    def time_step_kernel(self, nsteps):
        ms = ctypes.c_double()
        self._check(self._L.lbpc_time_step_kernel(self._ctx, nsteps, ctypes.byref(ms)))
        return ms.value

    # ------------------------------------------------------------ adjoint
    def adjoint_forward(self, nsteps, ckpt_every=100, loss=0):
        """Run nsteps with checkpoints; returns the loss (sum of f_l, or the
        front position sum f_l / (ny nz) for loss=1)."""
        torch = _torch()
        need = self._L.lbpc_adjoint_workspace_bytes(self._ctx, int(nsteps), int(ckpt_every))
        if need == 0:
            raise LbpcError(-1, "bad adjoint arguments")
        if self._adj_ws is None or self._adj_ws.numel() < need + 256:
            self._adj_ws = None
            self._adj_ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._adj_ws.data_ptr() + 255) // 256 * 256
        val = ctypes.c_double()
        self._check(self._L.lbpc_adjoint_forward(self._ctx, int(nsteps), int(ckpt_every),
                                                 int(loss), ctypes.c_void_p(ptr), need,
                                                 ctypes.byref(val)))
        return val.value

    def adjoint_backward(self, seed=1.0, want_T0=False):
        """Returns (dL/dT_w of every face, concatenated FP64 node fields; dL/dT0 or None)."""
        torch = _torch()
        c = self.cfgs[0]
        nw = 2 * (c["ny"] * c["nz"] + c["nx"] * c["nz"] + c["nx"] * c["ny"])
        dtw = torch.empty(nw, dtype=torch.float64, device=self.device)
        dt0 = torch.empty(self.shape(0), dtype=torch.float64, device=self.device) if want_T0 else None
        self._check(self._L.lbpc_adjoint_backward(
            self._ctx, float(seed), ctypes.c_void_p(dtw.data_ptr()),
            ctypes.c_void_p(dt0.data_ptr() if dt0 is not None else 0)))
        return dtw, dt0

    def adjoint(self, nsteps, ckpt_every=100, loss=0, want_T0=False):
        """Forward and reverse sweep in one library call (lbpc_adjoint).
        Returns (loss, dL/dT_w of every face concatenated, dL/dT0 or None)."""
        torch = _torch()
        need = self._L.lbpc_adjoint_workspace_bytes(self._ctx, int(nsteps), int(ckpt_every))
        if need == 0:
            raise LbpcError(-1, "bad adjoint arguments")
        if self._adj_ws is None or self._adj_ws.numel() < need + 256:
            self._adj_ws = None
            self._adj_ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._adj_ws.data_ptr() + 255) // 256 * 256
        c = self.cfgs[0]
        nw = 2 * (c["ny"] * c["nz"] + c["nx"] * c["nz"] + c["nx"] * c["ny"])
        dtw = torch.empty(nw, dtype=torch.float64, device=self.device)
        dt0 = torch.empty(self.shape(0), dtype=torch.float64, device=self.device) if want_T0 else None
        val = ctypes.c_double()
        self._check(self._L.lbpc_adjoint(
            self._ctx, int(nsteps), int(ckpt_every), int(loss), ctypes.c_void_p(ptr), need,
            ctypes.c_void_p(dtw.data_ptr()), ctypes.c_void_p(dt0.data_ptr() if dt0 is not None else 0),
            ctypes.byref(val)))
        return val.value, dtw, dt0

    def face_slice(self, flat, face, cavity=0):
        """View of one face inside a concatenated node-field vector."""
        c = self.cfgs[cavity]
        sizes = [int(np.prod(_face_shape(c, f))) for f in range(6)]
        o = sum(sizes[:face])
        return flat[o:o + sizes[face]].reshape(_face_shape(c, face))


def _loss_function():
    torch = _torch()

    class LbpcLoss(torch.autograd.Function):
        """L = final liquid fraction (or front position) after nsteps, as a
        differentiable function of the hot-wall (face x-) temperature field.

        Usage: loss = LbpcLoss.apply(Tw, cavity, nsteps, ckpt_every, loss_kind)
        The cavity advances by nsteps; backward runs the checkpointed adjoint."""

        @staticmethod
        def forward(ctx, Tw, cavity, nsteps, ckpt_every=100, loss_kind=0):
            cavity.set_wall_T(0, Tw.detach())
            val = cavity.adjoint_forward(nsteps, ckpt_every, loss_kind)
            ctx.cavity = cavity
            ctx.shape = Tw.shape
            return torch.tensor(val, dtype=torch.float64, device=Tw.device)

        @staticmethod
        def backward(ctx, grad):
            cav = ctx.cavity
            dtw, _ = cav.adjoint_backward(seed=float(grad))
            return cav.face_slice(dtw, 0).reshape(ctx.shape), None, None, None, None

    return LbpcLoss
