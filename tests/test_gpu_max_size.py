"""The largest lattice the library accepts (nx ny x 36 B of float32 populations just
under 2^31 bytes, the range of one buffer resource): 7680 x 7760 = 59.6 M nodes.

The oracle cannot step this size in seconds, so the check uses a property that holds
at any size: a lattice tiled from a P x P periodic pattern (phi0 and a stream-function
velocity of period P) evolves exactly like the P x P lattice, node by node, because
every node's update reads only its neighbours' identical inputs.  The tiled lattice
is therefore compared bitwise with the P x P one, which is itself compared with the
oracle.  This exercises the 32-bit byte offsets near their limit, the block grid of
the full size and the ragged-free tiling at P = 80 (the largest common divisor of the
two sides)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NX, NY, P = 7680, 7760, 80


@pytest.fixture(scope="module")
def lbm():
    import paper_1805_00007_amd as lbm
    lbm.lib()
    return lbm


@pytest.mark.parametrize("storage", [0, 1])
def test_max_size_equals_tiled_pattern(lbm, storage):
    assert NX * NY * 36 < 2 ** 31 and NX % P == 0 and NY % P == 0
    steps = 40
    dev = torch.device("cuda:0")
    phi0 = workloads.random_blobs(P, seed=9, width=4.0).astype(np.float32)
    U, V = workloads.random_stream_function(P, 4, seed=10, umax=0.05)
    U, V = U.astype(np.float32), V.astype(np.float32)
    phys = dict(workloads.PRESCRIBED, model=2, storage=storage)

    small = lbm.Solver(P, P, phi0, field=(U, V), device=dev, **phys)
    small.step(steps)
    ref = small.phi()
    small.close()
    if storage == 0:
        st = oracle.State(oracle.Params(nx=P, ny=P, **{k: v for k, v in phys.items()
                                                        if k != "storage"}),
                          phi0.astype(np.float64), U.astype(np.float64), V.astype(np.float64))
        want = st.run(steps).phi
        got = ref.double().cpu().numpy()
        rel = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        print("80x80 against the oracle after %d steps: rel L2 %.2e" % (steps, rel), flush=True)
        assert rel <= 1e-4

    reps = (NY // P, NX // P)
    print("tiling %dx%d (%.1f M nodes), storage %d" % (NX, NY, NX * NY / 1e6, storage), flush=True)
    big = lbm.Solver(NX, NY, np.tile(phi0, reps), field=(np.tile(U, reps), np.tile(V, reps)),
                     device=dev, **phys)
    big.step(steps)
    phi = big.phi()
    diag = big.diagnostics()
    big.close()
    same = bool((phi.view(reps[0], P, reps[1], P) == ref.view(1, P, 1, P)).all())
    tiles = reps[0] * reps[1]
    mass0 = tiles * float(phi0.astype(np.float64).sum())
    drift = abs(diag["mass"] - mass0) / (tiles * float(np.abs(phi0.astype(np.float64)).sum()))
    print("tiled lattice bitwise equal to the pattern: %s; mass drift %.2e; nonfinite %d"
          % (same, drift, int(diag["nonfinite"])), flush=True)
    assert same
    assert diag["nonfinite"] == 0
    assert drift <= 1e-6
