"""Pins of the oracle's isotropic gradient and Laplacian (the central schemes named in
Sec. III) and of its wall ghost rule.

The checks: exactness on polynomials (gradient up to degree 2, Laplacian up to
degree 3), the Fourier symbols written out from the neighbour formulas, isotropy of
the leading error term, and equality of a wall-bounded field with the periodic field
on the mirrored, doubled domain.
"""
import math

import numpy as np

import oracle


def _poly_field(nx, ny, coeffs):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    return sum(c * x ** i * y ** j for (i, j), c in coeffs.items()), x, y


def test_gradient_exact_on_quadratics_interior():
    nx, ny = 24, 20
    co = {(0, 0): 0.3, (1, 0): -1.1, (0, 1): 0.7, (2, 0): 0.05, (1, 1): -0.08, (0, 2): 0.02}
    psi, x, y = _poly_field(nx, ny, co)
    gx, gy = oracle.grad(oracle.Params(nx=nx, ny=ny), psi)
    ex = -1.1 + 2 * 0.05 * x - 0.08 * y
    ey = 0.7 - 0.08 * x + 2 * 0.02 * y
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    np.testing.assert_allclose(gx[inner], ex[inner], atol=1e-12)
    np.testing.assert_allclose(gy[inner], ey[inner], atol=1e-12)


def test_laplacian_exact_on_cubics_interior():
    nx, ny = 24, 20
    co = {(3, 0): 0.001, (2, 1): -0.002, (1, 2): 0.003, (0, 3): 0.0015, (2, 0): 0.1,
          (0, 2): -0.3, (1, 1): 0.2, (1, 0): 1.0}
    psi, x, y = _poly_field(nx, ny, co)
    lap = oracle.lap(oracle.Params(nx=nx, ny=ny), psi)
    # d2/dx2 + d2/dy2 of the cubic
    ex = (6 * 0.001 * x + 2 * -0.002 * y + 2 * 0.003 * x + 6 * 0.0015 * y
          + 2 * 0.1 + 2 * -0.3)
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    np.testing.assert_allclose(lap[inner], ex[inner], atol=1e-11)


def _symbols(kx, ky):
    """Symbols of the neighbour formulas
    d_x = (E - W)/3 + (NE + SE - NW - SW)/12,  lap = [4(E+W+N+S) + diagonals - 20 C]/6."""
    gx = 2 * math.sin(kx) / 3 + (math.sin(kx + ky) + math.sin(kx - ky)) / 6
    gy = 2 * math.sin(ky) / 3 + (math.sin(kx + ky) - math.sin(kx - ky)) / 6
    lam = -(8 * (math.cos(kx) + math.cos(ky)) + 2 * math.cos(kx + ky)
            + 2 * math.cos(kx - ky) - 20) / 6
    return gx, gy, lam


def test_fourier_symbols():
    nx, ny = 32, 24
    p = oracle.Params(nx=nx, ny=ny)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    for m, l in [(1, 0), (0, 1), (3, 2), (-5, 7), (16, 12)]:
        kx, ky = 2 * math.pi * m / nx, 2 * math.pi * l / ny
        th = kx * x + ky * y
        gx_s, gy_s, lam = _symbols(kx, ky)
        # cos(th) -> grad = -G sin(th), lap = -Lambda cos(th)
        gx, gy = oracle.grad(p, np.cos(th))
        np.testing.assert_allclose(gx, -gx_s * np.sin(th), atol=1e-13)
        np.testing.assert_allclose(gy, -gy_s * np.sin(th), atol=1e-13)
        np.testing.assert_allclose(oracle.lap(p, np.cos(th)), -lam * np.cos(th), atol=1e-13)


def test_isotropic_leading_error():
    """Lambda(k) = |k|^2 - |k|^4/12 + O(k^6) in every direction, and G = k + O(k^3)."""
    for ang in (0.0, math.pi / 8, math.pi / 4, 1.0):
        vals = []
        for k in (0.02, 0.04):
            kx, ky = k * math.cos(ang), k * math.sin(ang)
            gx, gy, lam = _symbols(kx, ky)
            vals.append((lam - k * k) / k ** 4)
            assert abs(gx - kx) < k ** 3 and abs(gy - ky) < k ** 3
        assert abs(vals[1] + 1 / 12) < 1e-3


def test_wall_ghost_rule_matches_mirrored_periodic_domain():
    """With walls at y = -1/2 and ny - 1/2, an even field (parity +1) or odd field
    (parity -1) gives the same gradient and Laplacian as the periodic field on the
    domain doubled by reflection."""
    nx, ny = 12, 10
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((ny, nx))
    pw = oracle.Params(nx=nx, ny=ny, walls=1)
    pp = oracle.Params(nx=nx, ny=2 * ny)
    for parity in (1, -1):
        doubled = np.concatenate([psi, parity * psi[::-1]], axis=0)
        gx, gy = oracle.grad(pw, psi, parity)
        gxp, gyp = oracle.grad(pp, doubled)
        np.testing.assert_allclose(gx, gxp[:ny], atol=1e-14)
        np.testing.assert_allclose(gy, gyp[:ny], atol=1e-14)
        np.testing.assert_allclose(oracle.lap(pw, psi, parity), oracle.lap(pp, doubled)[:ny],
                                   atol=1e-13)


def test_second_order_convergence_of_chemical_potential():
    """mu of a smooth periodic field converges to the continuous mu at second order."""
    errs = []
    for n in (32, 64):
        p = oracle.Params(nx=n, ny=n, sigma=0.01, width=4.0)
        c = oracle.coeffs(p)
        y, x = np.mgrid[0:n, 0:n].astype(float)
        k = 2 * math.pi / n
        phi = 0.5 * np.sin(k * x) * np.cos(2 * k * y)
        exact = 4 * c["beta"] * (phi ** 3 - phi) + c["kappa"] * 5 * k * k * phi
        mu = oracle.chemical_potential(p, phi)
        errs.append(np.abs(mu - exact).max() / (c["kappa"] * 5 * k * k * 0.5))
    assert errs[1] < errs[0] / 3.5
