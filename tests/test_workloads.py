"""Input generators (seeded, synthetic; no method arithmetic): shapes, seeds, scales."""
import math

import numpy as np

import workloads


def test_mobility_for_pe_inverts_the_definition():
    m = workloads.mobility_for_pe(200.0, 0.02, 2.0, 0.01)
    beta = 12 * 0.01 / (2.0 * 16)
    assert math.isclose(0.02 * 2.0 / (m * beta * 4), 200.0, rel_tol=1e-12)


def test_slotted_disk_area_and_symmetry():
    phi = workloads.slotted_disk(200, 100, 100, 80, 16, 20, 2.0)
    area = (phi > 0).sum()
    slot = 16 * (20 + math.sqrt(80 ** 2 - 8 ** 2))
    assert abs(area - (math.pi * 80 ** 2 - slot)) < 0.02 * area
    assert np.allclose(phi[:, 1:], phi[:, 1:][:, ::-1])  # mirror about x = 100
    assert phi[100, 100] < 0 < phi[100, 60]               # slot centre empty, disk full


def test_batch_case_is_seeded_and_spans_the_sizes():
    a = workloads.batch_case(16, seed=3, steps=10)
    b = workloads.batch_case(16, seed=3, steps=10)
    assert [w.nx for w in a] == [w.nx for w in b]
    assert all(np.array_equal(x.phi0, y.phi0) for x, y in zip(a, b))
    for w in a:
        U, V = w.field
        assert w.nx in (64, 128, 192, 256, 384, 512) and w.phi0.shape == (w.ny, w.nx)
        assert math.isclose(max(np.abs(U).max(), np.abs(V).max()), 0.05, rel_tol=1e-12)


def test_adjoint_case_velocity_is_linear_and_divergence_free():
    c = workloads.adjoint_case(64, 10)
    U, V = c.field()
    assert math.isclose(max(np.abs(U).max(), np.abs(V).max()), 0.05, rel_tol=1e-12)
    U2, V2 = c.field(2 * c.theta)
    assert np.allclose(U2, 2 * U) and np.allclose(V2, 2 * V)
    # spectral divergence of the analytic field vanishes
    k = 2 * np.pi * np.fft.fftfreq(64)
    div = np.fft.ifft2(1j * k[None, :] * np.fft.fft2(U) + 1j * k[:, None] * np.fft.fft2(V))
    assert np.abs(div).max() < 1e-12


def test_paper_setups_periods():
    assert workloads.translation_paper(1).steps == 10000
    assert workloads.zalesak(2).steps == 40000
    w = workloads.shear_paper()
    assert w.steps == 16000 and w.velocity["tf"][7999] == 1 and w.velocity["tf"][8000] == -1
