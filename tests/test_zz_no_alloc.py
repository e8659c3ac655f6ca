"""lbpc_budgets_noalloc (static device scratch, no allocation) against
lbpc_budgets, through the C ABI: two calls in a row, the second on a smaller
input, each equal bit for bit to the workspace variant on a twin context."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_util import make_cavity

pytestmark = pytest.mark.gpu


def _budgets(cav, name):
    from paper_1703_02652_amd import lib
    out = np.full(7 * cav.batch, -1.0)
    rc = getattr(lib(), name)(cav._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, lib().lbpc_last_error(cav._ctx)
    return out.reshape(cav.batch, 7)


def _batch():
    c1 = W.melting_cavity(40, 1e5, 0.02, 0.1, precision=W.FP64)
    c2 = W.melting_cavity(21, 1e4, 1.0, 0.2, precision=W.FP64)
    c2.update(ny=17, nz=13)
    c3 = W.melting_cavity(30, 1e5, 0.1, 0.1, precision=W.FP64)
    c3.update(face_bc=[W.ADIABATIC, W.DIRICHLET, W.ADIABATIC, W.ADIABATIC, W.ADIABATIC,
                       W.ADIABATIC])     # x- not fixed-temperature: Nu is NaN
    return [c1, c2, c3]


def test_budgets_noalloc_equals_budgets_on_two_calls_second_smaller():
    from paper_1703_02652_amd import Cavity
    cfgs = _batch()
    T0s = [W.random_temperature(c, seed=70 + i, lo=-0.2, hi=1.0) for i, c in enumerate(cfgs)]
    a = Cavity(cfgs, T0=T0s, device="cuda")
    b = Cavity(cfgs, T0=T0s, device="cuda")
    for cav in (a, b):
        cav.step(16)
        for _ in range(5):      # partials pending in the ring: the call reduces them first
            cav.step(1)
    got, ref = _budgets(a, "lbpc_budgets_noalloc"), _budgets(b, "lbpc_budgets")
    assert np.array_equal(got, ref, equal_nan=True)
    assert np.isnan(got[2, 6]) and np.isfinite(got[:2]).all() and got[0, 4] == 21
    # second call, smaller input: one cavity of 12 x 9 x 7 cells (the scratch
    # still holds the larger batch's records past this one's end)
    small = W.melting_cavity(12, 1e5, 0.02, 0.1, precision=W.FP64)
    small.update(ny=9, nz=7)
    c = make_cavity(small, walls={0: W.hot_wall_field(9, 7)})
    d = make_cavity(small, walls={0: W.hot_wall_field(9, 7)})
    for cav in (c, d):
        cav.step(9)
    got, ref = _budgets(c, "lbpc_budgets_noalloc"), _budgets(d, "lbpc_budgets")
    assert np.array_equal(got, ref, equal_nan=True)
    assert got[0, 4] == 9 and got[0, 3] > 0
    # and the first context again, after more steps
    for cav in (a, b):
        cav.step(3)
    assert np.array_equal(_budgets(a, "lbpc_budgets_noalloc"), _budgets(b, "lbpc_budgets"),
                          equal_nan=True)


def test_budgets_noalloc_refuses_a_batch_beyond_its_scratch():
    from paper_1703_02652_amd import LbpcError, lib
    cfg = W.precision_cavity(320, 0.02, precision=W.FP16S)
    cav = make_cavity(cfg)
    out = np.zeros(7)
    rc = lib().lbpc_budgets_noalloc(cav._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == -3
    assert b"scratch" in lib().lbpc_last_error(cav._ctx)
    with pytest.raises(LbpcError):
        cav._check(rc)
    assert cav.budgets()[0, 1] == pytest.approx(320**3, rel=1e-6)   # the workspace variant works
