"""Pins of the oracle's parameters and single-node building blocks.

Each check is fixed by the paper or by mathematics, not by re-running the oracle's
own formula: the moment conditions of Eq. feqmoment and Eq. conservation, the
special relaxation times of Remarks I-II, the planar equilibrium of Eq. analytical
(which fixes the beta/kappa relation of Eq. betakappa) and its excess free energy,
which must equal sigma.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import CX, CY, W

CS2 = 1.0 / 3.0
C = np.stack([CX, CY], axis=1).astype(float)


def _coeffs(**kw):
    return oracle.coeffs(oracle.Params(nx=8, ny=8, **kw))


def test_special_relaxation_times():
    # Remark II: tau = 1 gives K = -1/3 and 2 tau - 1 + 3K = 0.
    c = _coeffs(tau_g=1.0)
    assert c["K"] == pytest.approx(-1.0 / 3.0, abs=1e-15)
    assert 2 * 1.0 - 1 + 3 * c["K"] == pytest.approx(0.0, abs=1e-15)
    # Remark I / Eq. phit3inserting: tau = 1/2 + sqrt(3)/6 is a root of tau - 1/6 - tau^2.
    c = _coeffs(tau_g=0.5 + math.sqrt(3) / 6)
    assert c["K"] == pytest.approx(0.0, abs=1e-14)


def test_mobility_relation_and_density_map():
    c = _coeffs(tau_g=0.8, mobility=0.02, rho_a=3.0, rho_b=1.0)
    # M = cs^2 eta (tau - 1/2)
    assert CS2 * c["eta"] * (0.8 - 0.5) == pytest.approx(0.02, rel=1e-14)
    # Eq. rho: rho(phi_A) = rho_A, rho(phi_B) = rho_B
    assert c["a"] * 1.0 + c["b"] == pytest.approx(3.0)
    assert c["a"] * -1.0 + c["b"] == pytest.approx(1.0)


def test_invalid_relaxation_time_rejected():
    with pytest.raises(ValueError):
        _coeffs(tau_g=0.5)


def test_tanh_is_continuous_equilibrium():
    """mu of Eq. mu vanishes on the planar profile of Eq. analytical only if kappa and
    beta satisfy Eq. betakappa.  Evaluate mu analytically from the oracle's beta,
    kappa: mu = 4 beta (phi^3 - phi) - kappa phi''."""
    for sigma, width in [(0.01, 4.0), (0.003, 7.0)]:
        c = _coeffs(sigma=sigma, width=width)
        z = np.linspace(-3 * width, 3 * width, 101)
        phi = np.tanh(2 * z / width)
        d2 = -8.0 / width ** 2 * phi * (1 - phi ** 2)
        mu = 4 * c["beta"] * (phi ** 3 - phi) - c["kappa"] * d2
        assert np.abs(mu).max() < 1e-15


def test_band_free_energy_equals_surface_tension():
    """Excess free energy per unit length of a planar interface is sigma; a band has two
    interfaces.  Discretisation error O((dx/W)^2)."""
    errs = []
    for width in (8.0, 16.0):
        n = 512
        p = oracle.Params(nx=4, ny=n, sigma=0.01, width=width)
        from workloads import band
        d = oracle.diag(p, band(4, n, width))
        per_length = d["energy"] / 4
        errs.append(abs(per_length - 2 * 0.01) / (2 * 0.01))
    assert errs[0] < 0.02 and errs[1] < errs[0] / 3.0


def test_equilibrium_moments():
    """Eq. feqmoment at random states."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        phi, mu, ux, uy, eta = rng.uniform(-1, 1), rng.uniform(-1e-2, 1e-2), *rng.uniform(
            -0.1, 0.1, 2), rng.uniform(0.01, 2)
        g = oracle.equilibrium_g(phi, mu, ux, uy, eta)
        u = np.array([ux, uy])
        assert g.sum() == pytest.approx(phi, abs=1e-15)
        np.testing.assert_allclose(C.T @ g, phi * u, atol=1e-15)
        second = np.einsum("ia,ib,i->ab", C, C, g)
        np.testing.assert_allclose(second, CS2 * eta * mu * np.eye(2) + phi * np.outer(u, u),
                                   atol=1e-15)


def test_source_moments():
    """Eq. conservation, Eq. liangFi, and the vanishing second moment used under Eq. F2-F."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        F = rng.standard_normal(2)
        s = oracle.source_g(*F)
        assert abs(s.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ s, F, atol=1e-15)
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", C, C, s), 0, atol=1e-15)


def test_ns_equilibrium_moments():
    """Pressure-based NS equilibrium: sum f = 0, sum c f = rho u, sum cc f = p I + rho uu."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        p, rho, ux, uy = rng.uniform(-1e-3, 1e-3), rng.uniform(0.3, 1.0), *rng.uniform(-0.1, 0.1, 2)
        f = oracle.equilibrium_f(p, rho, ux, uy)
        u = np.array([ux, uy])
        assert abs(f.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ f, rho * u, atol=1e-15)
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", C, C, f),
                                   p * np.eye(2) + rho * np.outer(u, u), atol=1e-15)


def test_ns_source_moments():
    """NS forcing: sum G = u.grad rho (so that div u = 0), sum c G = F, and
    sum cc G = uF + Fu + cs^2 (u.grad rho I + u grad rho + grad rho u)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        F, u, dr = rng.standard_normal(2), rng.uniform(-0.1, 0.1, 2), rng.standard_normal(2)
        s = oracle.source_f(*F, *u, *dr)
        assert s.sum() == pytest.approx(u @ dr, abs=1e-14)
        np.testing.assert_allclose(C.T @ s, F, atol=1e-14)
        want = (np.outer(u, F) + np.outer(F, u)
                + CS2 * ((u @ dr) * np.eye(2) + np.outer(u, dr) + np.outer(dr, u)))
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", C, C, s), want, atol=1e-14)


def test_lattice_is_d2q9_of_the_paper():
    # c_1 = -c_3 = (1,0), c_2 = -c_4 = (0,1), c_5 = -c_7 = (1,1), c_6 = -c_8 = (-1,1)
    assert (CX[1], CY[1]) == (1, 0) and (CX[3], CY[3]) == (-1, 0)
    assert (CX[2], CY[2]) == (0, 1) and (CX[4], CY[4]) == (0, -1)
    assert (CX[5], CY[5]) == (1, 1) and (CX[7], CY[7]) == (-1, -1)
    assert (CX[6], CY[6]) == (-1, 1) and (CX[8], CY[8]) == (1, -1)
    assert W.sum() == pytest.approx(1.0)
    # isotropy: sum w c_a c_b = cs^2 delta_ab
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", W, C, C), CS2 * np.eye(2), atol=1e-16)
