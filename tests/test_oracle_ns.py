"""Pins of the oracle's coupled Navier-Stokes step (the Rayleigh-Taylor path, Sec. III.E).

The paper names the NS LBE standard and does not print it; the oracle uses a
pressure-based incompressible D2Q9 BGK model with the forcing whose moments
test_oracle_nodes checks.  Its dynamics are pinned here by textbook flows:
* Poiseuille flow between half-way bounce-back walls is exactly parabolic at
  tau_f = 1/2 + sqrt(3/16) and slips at other tau_f;
* a Taylor-Green vortex decays as exp(-2 nu k^2 t) with nu = cs^2 (tau_f - 1/2);
* phi mass is conserved exactly with walls and coupling;
* a planar, x-uniform two-phase state between walls equals the periodic run of the
  mirrored doubled domain.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def test_poiseuille_exact_at_magic_tau():
    ny, nx, a = 12, 4, 1e-6
    errs = {}
    for tau in (0.5 + math.sqrt(3.0 / 16.0), 0.7):
        nu = (tau - 0.5) / 3.0
        p = oracle.Params(nx=nx, ny=ny, walls=1, ns=1, tau_f=tau, rho_a=1.0, rho_b=1.0,
                          sigma=0.0, accel_x=a)
        s = oracle.State(p, np.ones((ny, nx))).run(12000)
        u = s.fields()[2]
        y = np.arange(ny) + 0.5
        exact = a / (2 * nu) * y * (ny - y)
        errs[tau] = np.abs(u - exact[:, None]).max() / exact.max()
    assert errs[0.5 + math.sqrt(3.0 / 16.0)] < 1e-7
    assert errs[0.7] > 1e-4


def test_taylor_green_decay():
    n, tau, U0 = 48, 0.8, 0.01
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / n
    y, x = np.mgrid[0:n, 0:n].astype(float)
    ux = -U0 * np.cos(k * x) * np.sin(k * y)
    uy = U0 * np.sin(k * x) * np.cos(k * y)
    p = oracle.Params(nx=n, ny=n, ns=1, tau_f=tau, rho_a=1.0, rho_b=1.0, sigma=0.0)
    steps = 600
    s = oracle.State(p, np.ones((n, n)), ux, uy).run(steps)
    _, _, u, v, _ = s.fields()
    amp = ((u * ux).sum() + (v * uy).sum()) / ((ux * ux).sum() + (uy * uy).sum())
    assert amp == pytest.approx(math.exp(-2 * nu * k * k * steps), rel=3e-3)


def test_rayleigh_taylor_mass_and_finiteness():
    w = workloads.rayleigh_taylor_case(nx=32, ny=128, steps=300, reynolds=200.0)
    p = oracle.Params(nx=32, ny=128, walls=1, ns=1, **w.phys)
    s = oracle.State(p, w.phi0)
    m0 = s.phi.sum()
    s.run(300)
    phi, mu, u, v, pr = s.fields()
    assert np.isfinite(phi).all() and np.isfinite(u).all()
    assert abs(phi.sum() - m0) / np.abs(w.phi0).sum() < 1e-13
    # the light phase rises where the interface is highest (x = 0, a bubble) and the
    # heavy phase falls where it is lowest (x = nx/2, a spike)
    ny = 128
    band = slice(ny // 2 - 8, ny // 2 + 8)
    assert v[band, 16].mean() < 0 < v[band, 0].mean()


def test_ns_walls_equal_mirrored_periodic_domain():
    nx, ny = 6, 40
    phi_col = np.tanh((np.arange(ny) - 14.2) / 2.0)
    phi0 = np.repeat(phi_col[:, None], nx, axis=1)
    kw = dict(ns=1, tau_f=0.7, tau_g=1.0, sigma=0.01, width=4.0, rho_a=1.0, rho_b=0.4,
              mobility=0.05)
    pw = oracle.Params(nx=nx, ny=ny, walls=1, **kw)
    pp = oracle.Params(nx=nx, ny=2 * ny, walls=0, **kw)
    a = oracle.State(pw, phi0).run(80)
    b = oracle.State(pp, np.concatenate([phi0, phi0[::-1]], axis=0)).run(80)
    fa, fb = a.fields(), b.fields()
    np.testing.assert_allclose(fa[0], fb[0][:ny], atol=1e-14)      # phi
    np.testing.assert_allclose(fa[3], fb[3][:ny], atol=1e-15)      # v
    np.testing.assert_allclose(fa[4], fb[4][:ny], atol=1e-14)      # p


def test_translating_density_interface_converges():
    """Variable-density terms of the NS step (the u.grad rho parts of the forcing and of
    the pressure): two layers of density ratio 3 moving with a uniform velocity are an
    exact solution (u = u0, div u = 0, constant p).  The lattice keeps it up to a
    discretisation error that falls with the interface width W: div u at second order
    (the interface gradients are resolved over W nodes), u - u0 at least at first order.
    A wrong sign or factor in those terms leaves an O(u0) error that does not shrink."""
    errs = []
    for W in (4.0, 8.0, 16.0):
        n = int(16 * W)
        x = np.arange(n)[None, :] * np.ones((8, 1))
        d = np.minimum(x - n / 4, 3 * n / 4 - x)
        phi0 = np.tanh(2 * d / W)
        p = oracle.Params(nx=n, ny=8, ns=1, tau_g=1.0, mobility=0.01, sigma=1e-4, width=W,
                          rho_a=1.0, rho_b=1 / 3, tau_f=0.8, gravity=0.0, model=2)
        s = oracle.State(p, phi0, np.full((8, n), 0.02), np.zeros((8, n))).run(int(20 * W))
        _, _, u, v, _ = s.fields()
        div = (np.roll(u, -1, 1) - np.roll(u, 1, 1)) / 2 + (np.roll(v, -1, 0) - np.roll(v, 1, 0)) / 2
        errs.append((np.abs(u - 0.02).max(), np.abs(div).max()))
    (u4, d4), (u8, d8), (u16, d16) = errs
    assert d4 / d8 > 3.5 and d8 / d16 > 3.5
    assert u4 / u16 > 3.0 and u16 < 0.025 * 0.02


def _rt_run(w, steps, chunk):
    """Run a Rayleigh-Taylor workload in the oracle; returns (steps reached while finite,
    extrema of phi seen, largest |u| seen)."""
    p = oracle.Params(nx=w.nx, ny=w.ny, walls=1, ns=1, **w.phys)
    s = oracle.State(p, w.phi0)
    done, ext, umax = 0, 1.0, 0.0
    while done < steps:
        s.run(chunk)
        phi, mu, u, v, pr = s.fields()
        if not (np.isfinite(phi).all() and np.isfinite(u).all()):
            return done, ext, umax
        done += chunk
        ext = max(ext, float(np.abs(phi).max()))
        umax = max(umax, float(np.hypot(u, v).max()))
    return done, ext, umax


@pytest.fixture
def two_threads():
    """Small lattices: a step is too short to share among many threads."""
    n = oracle.num_threads()
    oracle.set_num_threads(min(n, 2))
    yield
    oracle.set_num_threads(n)


def test_rayleigh_taylor_at05_re3000_diverges_paper_case_does_not(two_threads):
    """The At = 0.5, Re = 3000 Rayleigh-Taylor case is not reachable with the BGK
    Navier-Stokes model (reading R11) for 40000 steps: at full size (256x1024) the FP64
    oracle goes non-finite near 1.4 T.  The same dimensionless case at 64x256 (sqrt(gL) =
    0.04, W = 4, Pe = 1000, 0.1 L perturbation; T = 2263 steps) goes non-finite before
    2 T, after its largest velocity has passed 0.08 (lattice Mach number 0.14).  The
    paper's own case (Sec. III.E: At = 0.25, Re = 400, 0.05 d perturbation) at the same
    size stays finite through 3.125 T, the length of its 40000-step full-size run."""
    cfg = workloads.rayleigh_taylor_case(64, 256, steps=4600)
    T = 2263
    reached, ext, umax = _rt_run(cfg, 2 * T, 250)
    print("At 0.5 Re 3000 at 64x256: finite through %d steps (%.2f T), max |phi| %.3f, "
          "max |u| %.3f" % (reached, reached / T, ext, umax))
    assert reached < 2 * T
    assert umax > 0.08
    paper = workloads.rayleigh_taylor_paper(0.25, nx=64, ny=256, steps=10000)
    reached, ext, umax = _rt_run(paper, 10000, 1000)
    print("At 0.25 Re 400 at 64x256: finite through %d steps, max |phi| %.3f, max |u| %.3f"
          % (reached, ext, umax))
    assert reached == 10000
    assert ext < 1.5 and umax < 0.06
