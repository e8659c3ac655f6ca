"""GPU tests of the systems around the step: launch shapes and graphs,
checkpoint/resume, failure flags, 16-bit storage, batching at full size and
full-size sampled parity (through the C ABI)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import absdiff, make_cavity, rel

pytestmark = pytest.mark.gpu


def _state_bytes(cav):
    f, g = cav.state()
    out = [g.cpu().numpy()]
    if f is not None:
        out.append(f.cpu().numpy())
    return out


def test_launch_shapes_and_graphs_are_bitwise_identical():
    """Block sizes 64/128/256, persistent grids and graph vs eager stepping give
    the same state bit for bit (each cell's update is independent of the launch
    shape)."""
    cfg = W.melting_cavity(20, 1e5, 0.02, 0.1, precision=W.FP32)
    cfg.update(ny=13, nz=11)
    walls = {0: W.hot_wall_field(13, 11)}
    ref = None
    for launch in [(256, 0, 16, 8), (64, 0, 0, 1), (128, 37, 4, 8), (256, 512, 0, 1),
                   (192, 0, 2, 3), (64, 24, 16, 8), (256, 0, 16, 0), (64, 40, 4, 0)]:
        cav = make_cavity(cfg, walls=walls)
        cav.set_launch(*launch)
        cav.step(53)
        s = _state_bytes(cav)
        if ref is None:
            ref = s
        else:
            for a, b in zip(s, ref):
                assert np.array_equal(a, b), launch
        cav.close()


def test_queue_order_and_grid_do_not_change_state_or_budgets():
    """A batch of three cavities whose tiles interleave in the queue: XCD runs
    of 1, 3, 16 tiles, one run per XCD and y-blocks per XCD, with and without a
    persistent grid,
    give the same state and the same budgets bit for bit (the budget partials
    are indexed by the natural tile order)."""
    from paper_1703_02652_amd import Cavity
    c1 = W.melting_cavity(20, 1e5, 0.02, 0.1, precision=W.FP32)
    c2 = W.melting_cavity(13, 1e4, 1.0, 0.2, precision=W.FP32)
    c2.update(ny=11, nz=9)
    c3 = W.melting_cavity(16, 1e5, 0.1, 0.1, precision=W.FP32)
    cfgs = [c1, c2, c3]
    T0s = [W.random_temperature(c, seed=40 + i, lo=-0.2, hi=1.0) for i, c in enumerate(cfgs)]
    ref = None
    for launch in [(128, 0, 16, 1), (128, 0, 16, 3), (128, 40, 8, 16), (128, 0, 4, 1 << 20),
                   (128, 16, 0, 4), (128, 0, 16, 0), (128, 24, 2, 0)]:
        cav = Cavity(cfgs, T0=T0s, device="cuda")
        cav.set_launch(*launch)
        assert cav.get_launch() == launch
        cav.step(45)
        got = ([s for i in range(3) for s in _state_bytes_i(cav, i)], cav.budgets())
        if ref is None:
            ref = got
            assert (got[1][:, 3] > 0).all()
        else:
            for a, b in zip(got[0], ref[0]):
                assert np.array_equal(a, b), launch
            assert np.array_equal(got[1], ref[1]), launch
        cav.close()


def _state_bytes_i(cav, i):
    f, g = cav.state(i)
    return [g.cpu().numpy(), f.cpu().numpy()]


def test_graph_replays_match_eager_steps_every_replay():
    """The captured 16-step graph (with its in-graph reduction) replayed five
    times, with an eager budget pass and a host synchronisation between the
    replays, against the same steps launched one by one: state and budgets
    agree bit for bit after every replay."""
    cfg = W.melting_cavity(24, 1e5, 0.02, 0.1, precision=W.FP32)
    cfg.update(ny=19, nz=13)
    walls = {0: W.hot_wall_field(19, 13)}
    g = make_cavity(cfg, walls=walls)
    e = make_cavity(cfg, walls=walls)
    g.set_launch(128, 0, 16, 4)
    e.set_launch(128, 0, 0, 4)
    for replay in range(5):
        g.step(16)
        e.step(16)
        bg, be = g.budgets(), e.budgets()
        for x, y in zip(_state_bytes(g), _state_bytes(e)):
            assert np.array_equal(x, y), replay
        assert np.array_equal(bg, be), replay
        assert bg[0, 4] == 16 * (replay + 1)


def test_graph_remainders_and_pending_partials_match_eager_steps():
    """Graphs of every length against eager steps: five 1-step graphs, then 20
    steps as a 16-step and a 4-step graph, then 13 more as one 13-step graph
    (each graph closed by its reduction, walking the queue forward from its
    first step); and with graphs of at most 5 steps (an odd length), the same
    25 + 13 steps as graphs of 5, 5, 5, 5, 5 and 5, 5, 3.  State and budgets
    equal the same steps launched one by one, with the partials of up to 16
    reduced together, bit for bit."""
    cfg = W.melting_cavity(24, 1e5, 0.02, 0.1, precision=W.FP32)
    cfg.update(ny=17, nz=11)
    walls = {0: W.hot_wall_field(17, 11)}
    g = make_cavity(cfg, walls=walls)
    o = make_cavity(cfg, walls=walls)
    e = make_cavity(cfg, walls=walls)
    g.set_launch(256, 0, 16, 4)
    o.set_launch(256, 0, 5, 4)
    e.set_launch(256, 0, 0, 4)
    for _ in range(5):
        g.step(1)
    g.step(20)
    o.step(25)
    e.step(25)
    for more in (0, 13):
        g.step(more)
        o.step(more)
        e.step(more)
        be = e.budgets()
        for c in (g, o):
            for x, y in zip(_state_bytes(c), _state_bytes(e)):
                assert np.array_equal(x, y), more
            assert np.array_equal(c.budgets(), be), more
    assert be[0, 4] == 38


@pytest.mark.parametrize("n", [32, 128])
def test_block192_budgets_and_state_equal_block256(n):
    """Tiles of 192 cells leave an empty wavefront at the end of the last tile
    whenever the tile count is not a multiple of 4 (32^3, 128^3): the partial
    arrays hold it, and state and budgets equal those of 256-cell tiles bit
    for bit (a wave's partials do not depend on the tile size; at 32^3 one
    reduction chunk holds every wave in both)."""
    cfg = W.melting_cavity(n, 1e5, 0.02, 0.1, precision=W.FP32)
    walls = {0: W.hot_wall_field(n, n)}
    out = []
    for block in (256, 192):
        cav = make_cavity(cfg, walls=walls)
        cav.set_launch(block, 0, 16, 1)
        cav.step(37)
        out.append((_state_bytes(cav), cav.budgets()))
        cav.close()
    (s256, b256), (s192, b192) = out
    for x, y in zip(s256, s192):
        assert np.array_equal(x, y)
    if n == 32:
        assert np.array_equal(b256, b192)
    else:
        assert np.allclose(b256, b192, rtol=1e-13, atol=0)
    assert b192[0, 3] > 0 and b192[0, 1] == pytest.approx(n**3, rel=1e-6)


def test_autotune_does_not_advance_state():
    cfg = W.melting_cavity(16, 1e5, 0.02, 0.1, precision=W.FP32)
    a = make_cavity(cfg)
    a.step(10)
    b = make_cavity(cfg)
    b.step(10)
    b.autotune(3)
    a.step(7)
    b.step(7)
    for x, y in zip(_state_bytes(a), _state_bytes(b)):
        assert np.array_equal(x, y)


def test_save_load_resume_bitwise():
    """Checkpoint at step 40, run to 100; reload, run again: identical state and
    budgets (resume is bit-exact)."""
    cfg = W.melting_cavity(18, 1e5, 0.02, 0.1, precision=W.FP32)
    cav = make_cavity(cfg, walls={0: W.hot_wall_field(18, 18)})
    cav.step(40)
    blob = cav.save()
    cav.step(60)
    s1, b1 = _state_bytes(cav), cav.budgets()
    cav.load(blob)
    assert cav.budgets()[0, 4] == 40
    cav.step(60)
    s2, b2 = _state_bytes(cav), cav.budgets()
    for x, y in zip(s1, s2):
        assert np.array_equal(x, y)
    assert np.array_equal(b1, b2)


def test_unstable_cavity_is_flagged_and_frozen():
    """A NaN initial temperature in one cavity of a batch sets its status bit;
    the other cavity keeps stepping and further lbpc_step calls report it."""
    from paper_1703_02652_amd import Cavity, LbpcError
    c1 = W.melting_cavity(12, 1e4, 1.0, 0.1, precision=W.FP32)
    c2 = dict(c1)
    T_bad = np.zeros((12, 12, 12))
    T_bad[3, 4, 5] = np.nan
    cav = Cavity([c1, c2], T0=[np.zeros((12, 12, 12)), T_bad], device="cuda")
    cav.step(20)
    st = cav.status()
    assert st.tolist() == [0, 1]
    with pytest.raises(LbpcError) as e:
        cav.step(1)
    assert e.value.code == -4
    fl = cav.fields(0, names=("fl",))["fl"]
    assert float(fl.sum()) > 0


def test_invalid_arguments_raise():
    from paper_1703_02652_amd import Cavity, LbpcError
    cfg = W.melting_cavity(8, 1e4, 1.0, 0.1, precision=W.FP32)
    cav = Cavity(cfg, device="cuda")
    with pytest.raises(LbpcError):
        cav.set_launch(100, 0, 16)
    with pytest.raises(LbpcError):
        cav.set_launch(256, 0, 17)     # graphs of at most 16 steps (the budget ring)
    with pytest.raises(LbpcError):
        cav.set_launch(256, 0, -1)
    with pytest.raises(LbpcError):
        cav.set_launch(256, 0, 16, -1)
    with pytest.raises(LbpcError):
        cav.set_wall_T(2, np.zeros((8, 8)))   # adiabatic face
    import ctypes
    with pytest.raises(LbpcError):      # cavity index checked by the library
        cav._check(cav._L.lbpc_fields(cav._ctx, 5, 4, ctypes.c_void_p(0)))
    c16 = dict(cfg, precision=W.FP16S)
    c16cav = Cavity(c16, device="cuda")
    with pytest.raises(LbpcError):
        c16cav.adjoint_forward(10, 5)
    # checkpoints: a truncated buffer, and one from a context of another layout
    blob = cav.save()
    with pytest.raises(LbpcError):
        cav.load(blob[:-1])
    with pytest.raises(LbpcError):
        c16cav.load(blob[:len(c16cav.save())])
    other = Cavity(dict(cfg, nx=9), device="cuda")
    with pytest.raises(LbpcError):
        other.load(blob + bytes(len(other.save())))
    cav.load(blob)                      # the matching context takes it back


@pytest.mark.parametrize("prec", [W.FP16S, W.BF16S])
def test_sixteen_bit_storage_error_against_fp64_oracle(prec):
    """Shifted 16-bit populations with FP32 collision, 32^3 cavity, 400 steps.
    The error against the FP64 oracle is reported; bounds are loose sanity
    limits (FP16: 10 mantissa bits, BF16: 7)."""
    cfg64 = W.melting_cavity(32, 1e5, 0.02, 0.1, precision=W.FP64)
    cav = make_cavity(dict(cfg64, precision=prec))
    cav.step(400)
    ref = oracle.run(cfg64, oracle.init_state(cfg64), 400)
    fl = cav.fields(names=("T", "fl", "u"))
    rf = oracle.fields(cfg64, ref)
    eT, efl = absdiff(fl["T"], rf["T"]), absdiff(fl["fl"], rf["fl"])
    eu = absdiff(fl["uz"], rf["uz"]) / max(np.abs(rf["uz"]).max(), 1e-30)
    dmean = abs(float(fl["fl"].sum()) - rf["fl"].sum()) / rf["fl"].size
    print(f"prec {prec}: max|dT| {eT:.2e} max|dfl| {efl:.2e} rel|duz| {eu:.2e} "
          f"d(mean fl) {dmean:.2e}")
    lim = 5e-3 if prec == W.FP16S else 5e-2
    assert eT < lim and dmean < lim


def test_batch_of_64_cavities_first_steps_match_oracle_samples():
    """The 64-cavity batch (sizes 32..96, random Ra, Pr, Ste) in one launch:
    every cavity is stepped, and three of them match the FP64 oracle run alone
    after 20 FP32 steps (liquid fraction within 1e-5)."""
    from paper_1703_02652_amd import Cavity
    cfgs, draws = W.batch_cavities()
    cav = Cavity(cfgs, device="cuda")
    cav.autotune(3)
    cav.step(20)
    b = cav.budgets()
    assert (b[:, 3] > 0).all()     # heat entered every cavity
    for i in (0, 17, 63):
        c64 = dict(cfgs[i], precision=W.FP64)
        ref = oracle.run(c64, oracle.init_state(c64), 20)
        fl = cav.fields(i, names=("fl",))["fl"]
        assert absdiff(fl, oracle.fields(c64, ref)["fl"]) < 1e-5, i


def test_cavity128_full_size_one_step_against_oracle():
    """Full-size 128^3 FP32 workload in the launch shape the benchmark tunes:
    after 300 steps, the oracle's FP64 step from the GPU state (decoded) agrees
    with the GPU's next state to FP32 rounding, and mass is conserved."""
    cfg = W.cavity_128(precision=W.FP32)
    cav = make_cavity(cfg)
    cav.autotune(3)
    cav.step(300)
    f, g = cav.state()
    st = (f.cpu().numpy(), g.cpu().numpy())
    cav.step(1)
    f1, g1 = cav.state()
    ref = oracle.run(dict(cfg, precision=W.FP64), st, 1)
    ef, eg = absdiff(f1, ref[0]), absdiff(g1, ref[1])
    print(f"128^3 one step: max|df| {ef:.2e}, max|dg| {eg:.2e}")
    assert ef < 2e-6 and eg < 2e-5
    b = cav.budgets()[0]
    assert abs(b[1] / 128**3 - 1.0) < 1e-6


@pytest.mark.parametrize("Pr", [0.02, 6.2])
def test_sixteen_bit_errors_at_64_against_fp64_oracle(Pr):
    """Precision workload shape (Ra 1e6) at 64^3, 2000 steps: FP32, FP16 and
    BF16 storage against the FP64 oracle.  Errors of T, f_l and |u| are
    reported (printed: max and RMS) and bounded loosely for the 16-bit
    formats; FP32 keeps every cell's liquid fraction within 1e-5."""
    steps = 2000
    cfg64 = W.precision_cavity(64, Pr, precision=W.FP64)
    ref = oracle.run(cfg64, oracle.init_state(cfg64), steps)
    rf = oracle.fields(cfg64, ref)
    umag_ref = np.sqrt(rf["ux"] ** 2 + rf["uy"] ** 2 + rf["uz"] ** 2)
    for prec, lim in ((W.FP32, 1e-5), (W.FP16S, 1e-2), (W.BF16S, 1e-1)):
        cav = make_cavity(dict(cfg64, precision=prec))
        cav.step(steps)
        fl = cav.fields(names=("T", "fl", "u"))
        umag = np.sqrt(sum(fl[k].cpu().numpy() ** 2 for k in ("ux", "uy", "uz")))
        dT = np.abs(fl["T"].cpu().numpy() - rf["T"])
        dfl = np.abs(fl["fl"].cpu().numpy() - rf["fl"])
        du = np.abs(umag - umag_ref)
        print(f"Pr {Pr} prec {prec} {steps} steps: |dT| max {dT.max():.2e} rms "
              f"{np.sqrt((dT ** 2).mean()):.2e}; |dfl| max {dfl.max():.2e} rms "
              f"{np.sqrt((dfl ** 2).mean()):.2e}; |d|u|| max {du.max():.2e} "
              f"(max|u| {umag_ref.max():.2e}); d mean fl {abs(dfl.mean()):.2e}")
        assert dfl.max() < lim and dT.max() < lim
        cav.close()


def test_cavity128_y_mirror_commutes_with_the_step():
    """Full-size 128^3 FP32 workload (hot and cold x walls, adiabatic y and z
    walls, gravity along -z) from a random mixed-phase start: mirroring the
    state in y and stepping equals stepping and mirroring, to FP32 rounding.
    A wrong shift, wall rule or sign for any y-crossing link breaks this at
    any size."""
    import torch
    from paper_1703_02652_amd import Cavity
    cfg = W.cavity_128(precision=W.FP32)
    T0 = W.random_temperature(cfg, seed=128, lo=-0.3, hi=1.2)
    tab = oracle.tables()
    key19 = {tuple(v): i for i, v in enumerate(tab["e19"].astype(int))}
    key7 = {tuple(v): i for i, v in enumerate(tab["e7"].astype(int))}
    p19 = [key19[(int(v[0]), -int(v[1]), int(v[2]))] for v in tab["e19"]]
    p7 = [key7[(int(v[0]), -int(v[1]), int(v[2]))] for v in tab["e7"]]

    def mirror(f, g):   # [q][z][y][x]: cell y -> ny - 1 - y, e_y -> -e_y
        return f[p19].flip(2), g[p7].flip(2)

    a = Cavity(cfg, T0=T0, device="cuda")
    a.step(100)
    f, g = a.state()
    b = Cavity(cfg, device="cuda")
    b.set_state(*mirror(f, g))
    del f, g
    a.step(6)
    b.step(6)
    fa, ga = mirror(*a.state())
    fb, gb = b.state()
    u = a.fields(names=("u",))
    assert float(u["uy"].abs().max()) > 1e-4          # flow crosses the mirror plane
    ef = float((fa - fb).abs().max()) / float(fb.abs().max())
    eg = float((ga - gb).abs().max()) / float(gb.abs().max())
    print(f"128^3 y mirror after 6 steps: rel f {ef:.2e}, rel g {eg:.2e}")
    assert ef < 1e-5 and eg < 1e-5
    a.close()
    b.close()
    torch.cuda.empty_cache()


def test_every_field_mask_returns_the_planes_of_the_full_mask():
    """lbpc_fields with each of the 31 masks writes exactly the planes of the
    full mask that the mask names, in bit order (h, T, f_l, rho, u), bit for
    bit."""
    import itertools
    cfg = W.melting_cavity(12, 1e5, 0.02, 0.1, precision=W.FP32)
    cfg.update(ny=9, nz=7)
    cav = make_cavity(cfg, T0=W.random_temperature(cfg, seed=21, lo=-0.2, hi=1.0))
    cav.step(30)
    names = ("h", "T", "fl", "rho", "u")
    full = cav.fields(names=names)
    full = {k: v.cpu().numpy() for k, v in full.items()}
    for r in range(1, 6):
        for sub in itertools.combinations(names, r):
            got = cav.fields(names=sub)
            want = [k for k in ("h", "T", "fl", "rho") if k in sub] + (
                ["ux", "uy", "uz"] if "u" in sub else [])
            assert sorted(got) == sorted(want), sub
            for k in want:
                assert np.array_equal(got[k].cpu().numpy(), full[k]), (sub, k)
