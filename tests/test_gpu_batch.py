"""Batched stepping (lbm_ch_batch_*): many lattices of uneven sizes in one persistent
launch per step, optionally captured in one hipGraph.  Every lattice must come out
bitwise equal to stepping it on its own (the batch runs the same per-tile code), and
the plain path is itself held to the FP64 oracle; a few batch members are also
compared with the oracle directly."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import paper_1805_00007_amd as lbm
    lbm.lib()
    return lbm


def _solvers(lbm, ws, **kw):
    return [lbm.solver_for(w, **kw) for w in ws]


def _phis(solvers):
    out = [s.phi() for s in solvers]
    torch.cuda.synchronize()
    return [p.cpu().numpy() for p in out]


def _close(objs):
    for o in objs:
        o.close()


def _small_case(n_inst=12, seed=9):
    return workloads.batch_case(n_inst, seed=seed, sides=(64, 128, 192, 256), steps=200)


@pytest.mark.parametrize("tiles,graph,persistent", [
    ((0, 16), False, 0), ((0, 16), True, 1), ((64, 4), True, 0), ((64, 4), True, 1),
    ((256, 32), False, 1), ((128, 1), True, 0)])
def test_batch_bitwise_equals_single(lbm, tiles, graph, persistent):
    ws = _small_case()
    ref = _solvers(lbm, ws)
    for s in ref:
        s.step(37)
    want = _phis(ref)
    _close(ref)
    sol = _solvers(lbm, ws)
    b = lbm.Batch(sol).set_tiles(*tiles).set_schedule(persistent)
    assert b.persistent == bool(persistent)
    b.step(20, graph=graph)
    b.step(17, graph=graph)
    got = _phis(sol)
    assert all(s.step_count == 37 for s in sol)
    b.close()
    _close(sol)
    for w, g, r in zip(ws, got, want):
        assert np.array_equal(g, r), w.name


def test_batch_graph_replay_and_outside_steps(lbm):
    """The cached graph is replayed several times with eager work in between, and one
    member stepped on its own forces a table rebuild; results stay bitwise."""
    ws = _small_case(8, seed=10)
    ref = _solvers(lbm, ws)
    for s in ref:
        s.step(30)
    ref[3].step(5)
    for s in ref:
        s.step(30)
    want = _phis(ref)
    _close(ref)
    sol = _solvers(lbm, ws)
    b = lbm.Batch(sol)
    for _ in range(3):
        b.step(10, graph=True)
        torch.cuda.synchronize()
        _ = sol[0].diagnostics()
    sol[3].step(5)
    for _ in range(3):
        b.step(10, graph=True)
    got = _phis(sol)
    b.close()
    _close(sol)
    for w, g, r in zip(ws, got, want):
        assert np.array_equal(g, r), w.name


def test_batch_mixed_variants(lbm):
    """Model-I and Model-II, separable and field velocities, odd sizes: several kernel
    groups in one batch step."""
    ws = _small_case(4, seed=11)
    extra = [workloads.translation(96, steps=100, model=1),
             workloads.translation(100, steps=100, model=2)]
    for w in extra:
        w.velocity = dict(w.velocity, tf=None)
    ws2 = ws + extra
    ref = _solvers(lbm, ws2)
    for s in ref:
        s.step(40)
    want = _phis(ref)
    _close(ref)
    sol = _solvers(lbm, ws2)
    b = lbm.Batch(sol)
    b.step(40, graph=True)
    got = _phis(sol)
    b.close()
    _close(sol)
    for w, g, r in zip(ws2, got, want):
        assert np.array_equal(g, r), w.name


def test_full_batch_against_single_and_oracle(lbm):
    """The 64-lattice workload (sides 64-512): 200 batched steps in one graph against
    single stepping for every lattice, and against the FP64 oracle for one lattice of
    each of three sizes."""
    ws = workloads.batch_case(steps=200)
    sol = _solvers(lbm, ws)
    b = lbm.Batch(sol)
    print("batch of %d, %d nodes" % (len(ws), sum(w.nx * w.ny for w in ws)), flush=True)
    b.step(200, graph=True)
    got = _phis(sol)
    b.close()
    _close(sol)
    for i, w in enumerate(ws):
        s = lbm.solver_for(w)
        s.step(200)
        ph = s.phi().cpu().numpy()
        s.close()
        assert np.array_equal(got[i], ph), w.name
    seen = set()
    for i, w in enumerate(ws):
        if w.nx in seen or w.nx not in (64, 192, 512):
            continue
        seen.add(w.nx)
        p = oracle.Params(nx=w.nx, ny=w.ny, **w.phys)
        o = oracle.State(p, w.phi0, *w.field).run(200)
        err = oracle.rel_l2(got[i].astype(np.float64), o.phi)
        print(w.name, "rel L2 vs oracle %.3e" % err)
        assert err <= 1e-4


def test_full_batch_full_length(lbm):
    """The 64-lattice workload at its full length: 5000 batched steps in one graph
    launch, bitwise equal to single stepping for every lattice, and against the FP64
    oracle for one lattice of side 64 and one of side 128 (the larger ones take the
    oracle minutes at this length)."""
    steps = 5000
    ws = workloads.batch_case(steps=steps)
    sol = _solvers(lbm, ws)
    b = lbm.Batch(sol)
    b.step(steps, graph=True)
    got = _phis(sol)
    b.close()
    _close(sol)
    for i, w in enumerate(ws):
        s = lbm.solver_for(w)
        s.step(steps)
        ph = s.phi().cpu().numpy()
        s.close()
        assert np.array_equal(got[i], ph), w.name
    seen = set()
    for i, w in enumerate(ws):
        if w.nx in seen or w.nx not in (64, 128):
            continue
        seen.add(w.nx)
        p = oracle.Params(nx=w.nx, ny=w.ny, **w.phys)
        o = oracle.State(p, w.phi0, *w.field).run(steps)
        err = oracle.rel_l2(got[i].astype(np.float64), o.phi)
        drift = abs(got[i].astype(np.float64).sum() - w.phi0.sum()) / np.abs(w.phi0).sum()
        print(w.name, "after %d steps: rel L2 vs oracle %.3e, drift %.2e" % (steps, err, drift))
        assert err <= 1e-4
        assert drift <= 1e-6


def test_closed_member_is_refused(lbm):
    """Closing a member Solver before its batch is refused from Python (the library
    keeps the contexts' addresses) instead of reaching a destroyed context."""
    ws = _small_case(3, seed=13)
    sol = _solvers(lbm, ws)
    b = lbm.Batch(sol)
    b.step(2)
    sol[1].close()
    with pytest.raises(lbm.LbmChError):
        b.step(1)
    b.close()
    _close(sol)


def test_batch_autotune_restores_state(lbm):
    ws = _small_case(6, seed=12)
    sol = _solvers(lbm, ws)
    for s in sol:
        s.step(3)
    b = lbm.Batch(sol)
    tiles, us = b.autotune(trial_steps=3)
    print("batch autotune ->", tiles, "persistent" if b.persistent else "tile per workgroup",
          "%.1f us/step" % us)
    assert all(s.step_count == 3 for s in sol)
    assert tiles[0] in (0, 64, 128, 256) and tiles[1] in (4, 8, 16, 32) and us > 0
    b.step(10, graph=True)
    got = _phis(sol)
    b.close()
    _close(sol)
    ref = _solvers(lbm, ws)
    for s in ref:
        s.step(13)
    want = _phis(ref)
    _close(ref)
    for w, g, r in zip(ws, got, want):
        assert np.array_equal(g, r), w.name


def test_batch_rejects_unsupported(lbm):
    L = lbm.lib()
    w = workloads.translation(64, steps=10)
    w.velocity = dict(w.velocity, tf=None)  # steady: batchable
    ws = torch.empty(lbm.lib().lbm_ch_batch_workspace_bytes(2), dtype=torch.uint8,
                     device="cuda")
    ok = lbm.solver_for(w)
    for kw in (dict(walls=1), dict(storage=lbm.STORE_BF16)):
        s = lbm.solver_for(w, **kw)
        arr = (ctypes.c_void_p * 2)(ok.ctx.value, s.ctx.value)
        b = ctypes.c_void_p()
        assert L.lbm_ch_batch_create(ctypes.byref(b), arr, 2, ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel()) == lbm.EUNSUPPORTED, kw
        s.close()
    s = lbm.solver_for(workloads.vortex(64, period=100, steps=10))  # time-factor table
    arr = (ctypes.c_void_p * 2)(ok.ctx.value, s.ctx.value)
    b = ctypes.c_void_p()
    assert L.lbm_ch_batch_create(ctypes.byref(b), arr, 2, ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel()) == lbm.EUNSUPPORTED
    s.close()
    arr = (ctypes.c_void_p * 2)(ok.ctx.value, ok.ctx.value)
    assert L.lbm_ch_batch_create(ctypes.byref(b), arr, 2, ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel()) == lbm.EINVAL
    s = lbm.solver_for(w)
    arr = (ctypes.c_void_p * 2)(ok.ctx.value, s.ctx.value)
    assert L.lbm_ch_batch_create(ctypes.byref(b), arr, 2, ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel() - 1) == lbm.EINVAL
    assert L.lbm_ch_batch_create(ctypes.byref(b), arr, 2, ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel()) == lbm.OK
    assert L.lbm_ch_batch_destroy(b) == lbm.OK
    s.close()
    ok.close()
