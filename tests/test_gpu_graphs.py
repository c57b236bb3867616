"""Graph replay (lbm_ch_set_graphs): step, record and adjoint calls replayed from captured
hipGraphs give the same results as plain launches, bitwise, over repeated replays with
eager work in between, for both buffer parities, after a tile change, and in the modes
that fall back to plain launches."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import paper_1805_00007_amd as lbm
    lbm.lib()
    return lbm


def _case(mode):
    """(nx, ny, phi0, solver keywords) for one mode; 200 x 136 is ragged in both axes."""
    nx, ny = 200, 136
    phi0 = workloads.random_blobs(nx, seed=3, width=4.0)[:ny]
    phys = dict(workloads.PRESCRIBED, model=2)
    if mode == "rt":
        w = workloads.rayleigh_taylor_case(64, 128, steps=400)
        kw = dict(w.phys, walls=1)
        kw["ns"] = True
        return w.nx, w.ny, w.phi0, kw
    if mode in ("separable", "separable-tf"):
        tabs = workloads.single_vortex(nx, 0.05, 400, 400)
        tabs = dict(tabs, ay=tabs["ay"][:ny], by=tabs["by"][:ny])
        if mode == "separable":
            tabs["tf"] = None
        return nx, ny, phi0, dict(phys, velocity=tabs)
    U, V = workloads.random_stream_function(nx, 4, seed=4, umax=0.05)
    kw = dict(phys, field=(U[:ny], V[:ny]))
    if mode == "walls-half":
        kw.update(walls=1, storage=1)
    if mode == "model3":
        kw.update(model=3, tau_g=0.8)
    return nx, ny, phi0, kw


@pytest.mark.parametrize("mode", ["field", "separable", "separable-tf", "walls-half", "model3", "rt"])
def test_graph_steps_equal_plain_steps(lbm, mode):
    nx, ny, phi0, kw = _case(mode)
    dev = torch.device("cuda:0")
    a = lbm.Solver(nx, ny, phi0, device=dev, **kw)
    b = lbm.Solver(nx, ny, phi0, device=dev, **kw).set_graphs(True)
    # odd and even chunk lengths (both buffer parities), repeats (replays), a tile change
    for i, k in enumerate([5, 5, 4, 5, 4, 5, 7, 7]):
        if i == 5:
            a.set_tiles(64, 3)
            b.set_tiles(64, 3)
        a.step(k)
        b.step(k)
        pa, pb = a.phi().cpu().numpy(), b.phi().cpu().numpy()  # eager work between replays
        assert a.step_count == b.step_count
        assert np.array_equal(pa, pb), (mode, i, k)
    a.close()
    b.close()


def test_graph_record_and_adjoint_equal_plain(lbm):
    """Segments of a checkpointed backward pass: record then reverse steps with the same
    buffers, five times over (the first call of each kind captures, the rest replay)."""
    n, seg = 96, 9
    case = workloads.adjoint_case(n, 5 * seg)
    U, V = case.field()
    dev = torch.device("cuda:0")
    out = []
    for graphs in (False, True):
        s = lbm.Solver(n, n, case.phi0, field=(U, V), device=dev, **case.phys).set_graphs(graphs)
        traj = torch.empty((seg, n, n), dtype=torch.float32, device=dev)
        lam = torch.tensor(case.phi0, dtype=torch.float32, device=dev)
        gu, gv = torch.zeros_like(lam), torch.zeros_like(lam)
        scratch = torch.empty(s.adjoint_scratch_bytes(), dtype=torch.uint8, device=dev)
        snaps = []
        for r in range(5):
            buf, n0 = s.save_state()
            s.record(seg, traj)
            s.adjoint(n0 + seg, seg, traj, lam, gu, gv, scratch)
            torch.cuda.synchronize()
            snaps.append((traj.cpu().numpy().copy(), lam.cpu().numpy().copy(),
                          gu.cpu().numpy().copy(), s.phi().cpu().numpy()))
        s.close()
        out.append(snaps)
    for r, (x, y) in enumerate(zip(*out)):
        for u, v in zip(x, y):
            assert np.array_equal(u, v), r


def test_evolve_gradients_equal_with_and_without_graphs(lbm):
    from paper_1805_00007_amd.adjoint import evolve
    n, steps = 48, 40
    case = workloads.adjoint_case(n, steps)
    dev = torch.device("cuda:0")
    basis = torch.tensor(case.basis, dtype=torch.float32, device=dev)
    target = torch.zeros((n, n), dtype=torch.float32, device=dev)
    grads = []
    for graphs in (False, True):
        phi0 = torch.tensor(case.phi0, dtype=torch.float32, device=dev, requires_grad=True)
        theta = torch.tensor(case.theta, dtype=torch.float32, device=dev, requires_grad=True)
        uv = case.scale * torch.tensordot(theta, basis, dims=1)
        phi = evolve(phi0, uv[0], uv[1], steps, graphs=graphs, **case.phys)
        loss = ((phi - target) ** 2).sum()
        loss.backward()
        grads.append((phi0.grad.cpu().numpy(), theta.grad.cpu().numpy(), float(loss.detach())))
    assert np.array_equal(grads[0][0], grads[1][0])
    assert np.array_equal(grads[0][1], grads[1][1])
    assert grads[0][2] == grads[1][2]
