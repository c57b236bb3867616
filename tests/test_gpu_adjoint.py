"""GPU discrete adjoint at tau_g = 1 (lbm_ch_record / lbm_ch_adjoint and the
torch.autograd.Function on top) against FP64 central finite differences of the oracle.

The loss is L = ||phi(N) - phi_target||^2 (or a seeded linear functional of phi(N)); the
finite differences perturb the oracle's inputs by +-h with h = 1e-6 and take
sum (phi+ - phi-)(phi+ + phi- - 2 phi_target) / (2h).  In FP64 their truncation error is
O(h^2) and their rounding error about 1e-16 |L| / h, both far below the FP32 error of the
GPU gradient, which is evaluated along the FP32 trajectory and accumulates ~1e-7
relative rounding per step.  Gate: relative L2 of the sampled gradient vector <= 2e-4 at
small sizes, <= 2e-3 at 256^2 after 2000 steps.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = 1e-6
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "adjoint256_oracle_2000.npz")


@pytest.fixture(scope="module")
def lbm():
    import paper_1805_00007_amd as lbm
    lbm.lib()
    return lbm


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _oracle_phi(case, p, phi0, theta, scale, steps):
    U, V = case.field(theta, scale)
    return oracle.State(p, phi0, U, V).run(steps).phi


def _fd(f, x0, dirs, target):
    out = []
    for d in dirs:
        plus, minus = f(x0 + H * d), f(x0 - H * d)
        out.append(float(((plus - minus) * (plus + minus - 2.0 * target)).sum() / (2 * H)))
    return np.array(out)


def _gpu_grads(lbm, case, target, steps, segment=None, model=None, **kw):
    from paper_1805_00007_amd.adjoint import evolve
    dev = torch.device("cuda:0")
    phys = dict(case.phys)
    if model is not None:
        phys["model"] = model
    phi0 = torch.tensor(case.phi0, dtype=torch.float32, device=dev, requires_grad=True)
    theta = torch.tensor(case.theta, dtype=torch.float32, device=dev, requires_grad=True)
    basis = torch.tensor(case.basis, dtype=torch.float32, device=dev)
    uv = case.scale * torch.tensordot(theta, basis, dims=1)
    phi = evolve(phi0, uv[0], uv[1], steps, segment=segment, **kw, **phys)
    loss = ((phi - torch.tensor(target, dtype=torch.float32, device=dev)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (float(loss.detach()), theta.grad.double().cpu().numpy(),
            phi0.grad.double().cpu().numpy())


@pytest.mark.parametrize("model", [2, 1])
def test_adjoint_matches_oracle_fd_small(lbm, model):
    n, steps = 48, 40
    case = workloads.adjoint_case(n, steps, model=model)
    p = oracle.Params(nx=n, ny=n, **case.phys)
    target = _oracle_phi(case, p, case.phi0, case.theta_target, case.scale_target, steps)
    print("case adjoint%d model %d steps %d" % (n, model, steps), flush=True)
    loss, g_theta, g_phi0 = _gpu_grads(lbm, case, target, steps)
    base = _oracle_phi(case, p, case.phi0, case.theta, case.scale, steps)
    assert abs(loss - ((base - target) ** 2).sum()) <= 1e-4 * ((base - target) ** 2).sum()
    fd_theta = _fd(lambda th: _oracle_phi(case, p, case.phi0, th, case.scale, steps),
                   case.theta, np.eye(len(case.theta)), target)
    rng = np.random.default_rng(7)
    near = np.flatnonzero(np.abs(case.phi0.ravel()) < 0.9)
    idx = np.sort(np.concatenate([rng.choice(near, 6, replace=False), [n * n // 2 + n // 2]]))
    dirs = np.zeros((len(idx), n, n))
    for j, i in enumerate(idx):
        dirs[j].ravel()[i] = 1.0
    fd_phi = _fd(lambda ph: _oracle_phi(case, p, ph, case.theta, case.scale, steps),
                 case.phi0, dirs, target)
    e_theta, e_phi = _rel(g_theta, fd_theta), _rel(g_phi0.ravel()[idx], fd_phi)
    print("model %d rel err grad theta %.3e grad phi0 %.3e" % (model, e_theta, e_phi))
    assert e_theta <= 2e-4
    assert e_phi <= 2e-4


def test_adjoint_one_step_dot_product(lbm):
    """<lam', J delta> from the FP64 map against <J^T lam', delta> from one GPU reverse
    step, for a random lam', a random direction and a random velocity field."""
    n = 40
    rng = np.random.default_rng(11)
    phi = workloads.random_blobs(n, seed=3, width=4.0)
    U, V = workloads.random_stream_function(n, 4, seed=4, umax=0.05)
    phys = dict(workloads.PRESCRIBED, model=2)
    p = oracle.Params(nx=n, ny=n, **phys)
    lam1 = rng.standard_normal((n, n))
    delta = rng.standard_normal((n, n))

    def step(ph):
        return oracle.State(p, ph, U, V).run(1).phi

    jd = (step(phi + H * delta) - step(phi - H * delta)) / (2 * H)
    lhs = float((lam1 * jd).sum())
    dev = torch.device("cuda:0")
    s = lbm.Solver(n, n, phi, field=(U, V), device=dev, **phys)
    traj = torch.empty((1, n, n), dtype=torch.float32, device=dev)
    s.record(1, traj)
    lam = torch.tensor(lam1, dtype=torch.float32, device=dev)
    s.adjoint(1, 1, traj, lam)
    torch.cuda.synchronize()
    rhs = float((lam.double().cpu().numpy() * delta).sum())
    s.close()
    print("dot product %.9e vs %.9e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-5 * np.sqrt((lam1 ** 2).sum() * (delta ** 2).sum())


def test_adjoint_separable_time_dependent_velocity(lbm):
    """Separable single-vortex tables with tf[n] = cos(pi n / T): dL/dax[x] from the
    base-field gradient contracted with ay, against FD of the oracle."""
    n, steps, period = 40, 30, 40
    tabs = workloads.single_vortex(n, 0.05, period, steps)
    phi0 = workloads.circle(n, n, n / 2, 0.6 * n, 0.2 * n, 4.0)
    phys = dict(workloads.PRESCRIBED, model=2)
    p = oracle.Params(nx=n, ny=n, **phys)
    rng = np.random.default_rng(12)
    r = rng.standard_normal((n, n))

    def run(ax):
        t = dict(tabs, ax=ax)
        U, V = workloads.separable_field(t)
        return oracle.State(p, phi0, U, V, tabs["tf"]).run(steps).phi

    xs = [3, 11, 20, 33]
    fd = []
    for x in xs:
        e = np.zeros(n)
        e[x] = H
        fd.append(float((r * (run(tabs["ax"] + e) - run(tabs["ax"] - e))).sum() / (2 * H)))
    dev = torch.device("cuda:0")
    s = lbm.Solver(n, n, phi0, velocity=tabs, device=dev, **phys)
    traj = torch.empty((steps, n, n), dtype=torch.float32, device=dev)
    s.record(steps, traj)
    lam = torch.tensor(r, dtype=torch.float32, device=dev)
    gu, gv = torch.zeros_like(lam), torch.zeros_like(lam)
    s.adjoint(steps, steps, traj, lam, gu, gv)
    torch.cuda.synchronize()
    gax = (gu.double().cpu().numpy() * np.asarray(tabs["ay"])[:, None]).sum(0)
    s.close()
    err = _rel(gax[xs], fd)
    print("separable rel err %.3e" % err, gax[xs], fd)
    assert err <= 2e-4


def test_checkpoint_segments_agree(lbm):
    """sqrt(N) checkpointing recomputes the same trajectory: gradients with segment
    lengths 1, 7, 17, 25 (three and two segments), sqrt(N) and N, with the segments
    re-run on two solvers beside the reverse steps (the default) or all in order on one
    stream, with graph replay, with the whole trajectory stored instead of checkpoints,
    and with other or autotuned tile shapes, agree bitwise."""
    n, steps = 32, 50
    case = workloads.adjoint_case(n, steps)
    target = np.zeros((n, n))
    ref = None
    for seg, kw in ((None, {}), (1, {}), (7, {}), (17, {}), (25, {}), (steps, {}),
                    (None, dict(overlap=False)),
                    (1, dict(overlap=False)), (7, dict(graphs=True)),
                    (None, dict(store_trajectory=True)),
                    (None, dict(tiles=(64, 4))), (None, dict(autotune=2))):
        _, gt, gp = _gpu_grads(lbm, case, target, steps, segment=seg, **kw)
        if ref is None:
            ref = (gt, gp)
        else:
            assert np.array_equal(gt, ref[0]) and np.array_equal(gp, ref[1]), (seg, kw)


def test_adjoint_zero_steps_is_identity(lbm):
    n = 24
    case = workloads.adjoint_case(n, 0)
    _, gt, gp = _gpu_grads(lbm, case, np.zeros((n, n)), 0)
    _, gt2, gp2 = _gpu_grads(lbm, case, np.zeros((n, n)), 0, store_trajectory=True)
    assert np.array_equal(gt, gt2) and np.array_equal(gp, gp2)
    assert np.all(gt == 0)
    assert np.allclose(gp, 2 * case.phi0.astype(np.float32), rtol=0, atol=1e-6)


def test_adjoint_rejects_unsupported(lbm):
    n = 32
    phi0 = workloads.circle(n, n, 16, 16, 8, 4.0)
    dev = torch.device("cuda:0")
    traj = torch.empty((1, n, n), dtype=torch.float32, device=dev)
    lam = torch.zeros((n, n), dtype=torch.float32, device=dev)
    scratch = torch.empty(n * n * 4, dtype=torch.uint8, device=dev)
    L = lbm.lib()
    P = ctypes.c_void_p
    for kw in (dict(tau_g=0.8), dict(walls=1), dict(ns=True, tau_f=0.8, gravity=1e-5)):
        s = lbm.Solver(n, n, phi0, device=dev, **kw)
        st = L.lbm_ch_adjoint(s.ctx, 1, 1, P(traj.data_ptr()), P(lam.data_ptr()), None, None,
                              P(scratch.data_ptr()), scratch.numel(), s._s())
        assert st == lbm.EUNSUPPORTED, kw
        s.close()
    s = lbm.Solver(n, n, phi0, device=dev)
    st = L.lbm_ch_adjoint(s.ctx, 1, 1, P(traj.data_ptr()), P(lam.data_ptr()), None, None,
                          P(scratch.data_ptr()), scratch.numel() - 4, s._s())
    assert st == lbm.EINVAL
    st = L.lbm_ch_adjoint(s.ctx, 0, 1, P(traj.data_ptr()), P(lam.data_ptr()), None, None,
                          P(scratch.data_ptr()), scratch.numel(), s._s())
    assert st == lbm.EINVAL
    st = L.lbm_ch_adjoint(s.ctx, 1, 1, P(traj.data_ptr()), P(lam.data_ptr()),
                          P(lam.data_ptr()), None, P(scratch.data_ptr()), scratch.numel(),
                          s._s())
    assert st == lbm.EINVAL
    s.close()


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored oracle gradients not generated")
def test_adjoint_full_size_against_stored_fd(lbm):
    """256^2, 2000 steps, 16 coefficients: the loss and its gradients against the stored
    FP64 central differences (tests/golden/make_golden.py adjoint256)."""
    g = np.load(GOLDEN)
    steps = int(g["steps"])
    case = workloads.adjoint_case(256, steps)
    target = g["phi_target"].astype(np.float64)
    print("case adjoint256 steps %d" % steps, flush=True)
    loss, gt, gp = _gpu_grads(lbm, case, target, steps)
    e_loss = abs(loss - float(g["loss"])) / float(g["loss"])
    e_theta = _rel(gt, g["grad_theta"])
    e_phi = _rel(gp.ravel()[g["phi0_index"]], g["grad_phi0"])
    print("adjoint256 loss rel %.3e grad theta %.3e grad phi0 %.3e" % (e_loss, e_theta, e_phi))
    assert e_loss <= 1e-4
    assert e_theta <= 2e-3
    assert e_phi <= 2e-3


@pytest.mark.parametrize("mode", ["field-model2", "separable-model1", "walls", "half"])
def test_record_matches_plain_steps(lbm, mode):
    """lbm_ch_record writes phi^n before every step n (fused into the step kernel for
    periodic float32 lattices with a prescribed velocity and model 1 or 2, a separate
    phi launch otherwise): the trajectory equals phi() taken before each plain step,
    and the state afterwards equals the plain run's, bitwise.  Ragged 200 x 136 lattice
    (the last strip and row chunk are partial)."""
    nx, ny, steps = 200, 136, 7
    dev = torch.device("cuda:0")
    phi0 = workloads.random_blobs(nx, seed=3, width=4.0)[:ny]
    phys = dict(workloads.PRESCRIBED, model=2)
    kw = {}
    if mode == "separable-model1":
        tabs = workloads.single_vortex(nx, 0.05, 400, steps)
        tabs = dict(tabs, ay=tabs["ay"][:ny], by=tabs["by"][:ny])
        kw["velocity"] = tabs
        phys["model"] = 1
    else:
        U, V = workloads.random_stream_function(nx, 4, seed=4, umax=0.05)
        kw["field"] = (U[:ny], V[:ny])
    if mode == "walls":
        phys["walls"] = 1
    if mode == "half":
        phys["storage"] = 1

    def solver():
        return lbm.Solver(nx, ny, phi0, device=dev, **kw, **phys)

    a = solver()
    ref = []
    for _ in range(steps):
        ref.append(a.phi().cpu().numpy())
        a.step(1)
    ref_end = a.phi().cpu().numpy()
    b = solver()
    traj = torch.empty((steps, ny, nx), dtype=torch.float32, device=dev)
    b.record(steps, traj)
    got = traj.cpu().numpy()
    got_end = b.phi().cpu().numpy()
    assert b.step_count == steps
    a.close()
    b.close()
    for n in range(steps):
        assert np.array_equal(got[n], ref[n]), (mode, n)
    assert np.array_equal(got_end, ref_end), mode
