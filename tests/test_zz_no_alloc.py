"""lbm_ch_adjoint_static, the entry point that allocates nothing (its scratch is a static
device array), against lbm_ch_adjoint with caller scratch on the same inputs: the same
kernels in the same order, so the results must be bitwise equal.  Two calls in a row,
the second on a smaller lattice; and a lattice above the static array's size is
rejected."""
import ctypes

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


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _solver(lbm, n, steps):
    case = workloads.adjoint_case(n, steps)
    U, V = case.field()
    s = lbm.Solver(n, n, case.phi0, field=(U, V), device="cuda:0", **case.phys)
    traj = torch.empty((steps, n, n), dtype=torch.float32, device="cuda:0")
    s.record(steps, traj)
    return s, traj


def _reverse(lbm, s, traj, steps, static, seed):
    n = traj.shape[1]
    g = torch.Generator(device="cpu").manual_seed(seed)
    lam = torch.randn((n, n), generator=g, dtype=torch.float32).to("cuda:0")
    gu = torch.zeros((n, n), dtype=torch.float32, device="cuda:0")
    gv = torch.zeros_like(gu)
    L = lbm.lib()
    if static:
        rc = L.lbm_ch_adjoint_static(s.ctx, steps, steps, _ptr(traj), _ptr(lam), _ptr(gu),
                                     _ptr(gv), s._s())
    else:
        scratch = torch.empty(n * n, dtype=torch.float32, device="cuda:0")
        rc = L.lbm_ch_adjoint(s.ctx, steps, steps, _ptr(traj), _ptr(lam), _ptr(gu), _ptr(gv),
                              _ptr(scratch), scratch.numel() * 4, s._s())
    torch.cuda.synchronize()
    assert rc == lbm.OK, rc
    return lam.cpu().numpy(), gu.cpu().numpy(), gv.cpu().numpy()


@pytest.mark.parametrize("sizes", [((96, 13), (48, 6))])
def test_static_adjoint_equals_scratch_adjoint(lbm, sizes):
    for k, (n, steps) in enumerate(sizes):
        print("no-alloc adjoint: %dx%d, %d reverse steps" % (n, n, steps), flush=True)
        s, traj = _solver(lbm, n, steps)
        ref = _reverse(lbm, s, traj, steps, False, seed=10 + k)
        got = _reverse(lbm, s, traj, steps, True, seed=10 + k)
        s.close()
        for a, b in zip(got, ref):
            assert np.isfinite(a).all()
            assert np.array_equal(a, b)


def test_static_adjoint_rejects_large_lattice(lbm):
    nx, ny = 1100, 1000  # 1.1 M nodes > LBM_CH_ADJOINT_STATIC_MAX_NODES
    assert nx * ny > 1048576
    phi0 = workloads.circle(nx, ny, nx / 2, ny / 2, 200.0, 4.0)
    s = lbm.Solver(nx, ny, phi0, field=(np.zeros((ny, nx)), np.zeros((ny, nx))), device="cuda:0",
                   tau_g=1.0, mobility=0.01, sigma=0.01, width=4.0, rho_a=1.0, rho_b=0.5, model=2)
    traj = torch.empty((1, ny, nx), dtype=torch.float32, device="cuda:0")
    s.record(1, traj)
    lam = torch.zeros((ny, nx), dtype=torch.float32, device="cuda:0")
    rc = lbm.lib().lbm_ch_adjoint_static(s.ctx, 1, 1, _ptr(traj), _ptr(lam), None, None, s._s())
    torch.cuda.synchronize()
    s.close()
    assert rc == lbm.EINVAL
