"""Seeded synthetic inputs for the lattice Boltzmann Cahn-Hilliard workloads.

This module only describes workloads: initial order-parameter fields, prescribed
velocity fields and the physical parameters of each run.  It holds none of the
method's arithmetic (no chemical potential, equilibrium, source or collision), so
the GPU path and the oracle can both take their inputs from it.

Conventions
-----------
* Lattice units: dx = dt = 1.  Node (i, j) of a periodic grid sits at (x, y) = (i, j);
  with walls in y (walls at y = -1/2 and y = ny - 1/2) node j sits at y = j + 1/2.
* A field is a float64 array of shape (ny, nx).
* A separable velocity is a dict of 1-D float64 tables with
  ``u(x, y, t_n) = tf[n] * ax[x] * ay[y]`` and ``v(x, y, t_n) = tf[n] * bx[x] * by[y]``.
  Every prescribed flow of Sec. III of the paper has this form.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


# --------------------------------------------------------------------------- fields

def tanh_profile(dist, width, phi_a=1.0, phi_b=-1.0):
    """Planar equilibrium profile of Eq. analytical evaluated at signed distance ``dist``
    (positive inside phase A)."""
    return 0.5 * (phi_a + phi_b) + 0.5 * (phi_a - phi_b) * np.tanh(2.0 * dist / width)


def circle(nx, ny, cx, cy, radius, width, phi_a=1.0, phi_b=-1.0):
    """Circular drop of phase A (phi = phi_a inside) centred at (cx, cy) in node units."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return tanh_profile(radius - r, width, phi_a, phi_b)


def band(nx, ny, width, phi_a=1.0, phi_b=-1.0):
    """Horizontal band of phase A between y = ny/4 and y = 3 ny/4 (two planar interfaces)."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    d = np.minimum(y - ny / 4.0, 3.0 * ny / 4.0 - y)
    return tanh_profile(d, width, phi_a, phi_b)


def rayleigh_taylor(nx, ny, width, amp_frac=0.1):
    """Heavy phase (phi = +1) above a cosine-perturbed interface at mid-height:
    phi = tanh(2 (y - h(x)) / W), h = ny/2 + amp_frac * nx * cos(2 pi x / nx), with
    cell-centred coordinates (walls at y = 0 and y = ny in these units)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    x += 0.5
    y += 0.5
    h = ny / 2.0 + amp_frac * nx * np.cos(2.0 * math.pi * x / nx)
    return np.tanh(2.0 * (y - h) / width)


def random_blobs(n, seed, width):
    """1-3 circles or ellipses of phase A with radii 0.1-0.3 of the side, union by max."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    phi = -np.ones((n, n))
    for _ in range(int(rng.integers(1, 4))):
        cx, cy = rng.uniform(0.25, 0.75, size=2) * n
        a, b = rng.uniform(0.1, 0.3, size=2) * n
        th = rng.uniform(0, math.pi)
        xr = (x - cx) * math.cos(th) + (y - cy) * math.sin(th)
        yr = -(x - cx) * math.sin(th) + (y - cy) * math.cos(th)
        r_ell = np.sqrt((xr / a) ** 2 + (yr / b) ** 2)
        phi = np.maximum(phi, np.tanh(2.0 * min(a, b) * (1.0 - r_ell) / width))
    return phi


def perturbed_uniform(nx, ny, mean, amp, seed):
    """Uniform state plus seeded uniform noise (used by small parity cases)."""
    rng = np.random.default_rng(seed)
    return mean + amp * rng.uniform(-1.0, 1.0, size=(ny, nx))


# ----------------------------------------------------------------------- velocities

def uniform_velocity(nx, ny, u0, v0, nsteps):
    """Constant translation velocity (Sec. III.A)."""
    return dict(ax=np.full(nx, float(u0)), ay=np.ones(ny), bx=np.full(nx, float(v0)),
                by=np.ones(ny), tf=np.ones(nsteps + 1))


def single_vortex(n, umax, period, nsteps):
    """Time-reversing single vortex: psi = A sin^2(pi x/L) sin^2(pi y/L) cos(pi t/T),
    u = d psi/dy, v = -d psi/dx, with A = umax L / pi so that max |u| = umax."""
    L = float(n)
    A = umax * L / math.pi
    x = np.arange(n, dtype=np.float64)
    k = math.pi / L
    return dict(ax=A * k * np.sin(k * x) ** 2, ay=np.sin(2 * k * x),
                bx=-A * k * np.sin(2 * k * x), by=np.sin(k * x) ** 2,
                tf=np.cos(math.pi * np.arange(nsteps + 1) / period))


def rigid_rotation(n, u0, nsteps):
    """Zalesak rotation field of Sec. III.B: u = -U0 pi (y/L - 1/2), v = U0 pi (x/L - 1/2)."""
    x = np.arange(n, dtype=np.float64)
    return dict(ax=np.full(n, -u0 * math.pi), ay=x / n - 0.5, bx=u0 * math.pi * (x / n - 0.5),
                by=np.ones(n), tf=np.ones(nsteps + 1))


def shear_reversal(n, u0, period, nsteps):
    """Shear flow of Sec. III.C, reversed at t = T."""
    x = np.arange(n, dtype=np.float64)
    s = math.pi * (x / n - 0.5)
    t = np.arange(nsteps + 1)
    return dict(ax=-u0 * math.pi * np.cos(s), ay=np.sin(s), bx=u0 * math.pi * np.sin(s),
                by=np.cos(s), tf=np.where(t < period, 1.0, -1.0))


def deformation(n, u0, nvort, period, nsteps):
    """Deformation field of Sec. III.D with n vortices and reversal time T0."""
    x = np.arange(n, dtype=np.float64)
    s = nvort * math.pi * (x / n + 0.5)
    return dict(ax=-u0 * np.sin(s), ay=np.sin(s), bx=-u0 * np.cos(s), by=np.cos(s),
                tf=np.cos(math.pi * np.arange(nsteps + 1) / period))


def separable_field(tables):
    """Full (U, V) base fields (ny, nx) of a separable velocity at factor 1."""
    U = np.outer(tables["ay"], tables["ax"])
    V = np.outer(tables["by"], tables["bx"])
    return U, V


def random_stream_function(n, modes, seed, umax):
    """Divergence-free field from psi = sum a_kl sin(2 pi k x/n) sin(2 pi l y/n),
    k, l = 1..modes, a_kl ~ N(0,1)/(k^2+l^2) from the seed, scaled to max |u| = umax
    (the scale is computed once from the sampled field and then fixed)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((modes, modes)) / (
        np.arange(1, modes + 1)[:, None] ** 2 + np.arange(1, modes + 1)[None, :] ** 2)
    return stream_function_field(n, a, umax)


def stream_function_field(n, coeffs, umax=None):
    """u = d psi/dy, v = -d psi/dx of psi = sum_kl c_kl sin(2 pi k x/n) sin(2 pi l y/n)."""
    modes = coeffs.shape[0]
    x = np.arange(n, dtype=np.float64)
    kk = 2 * math.pi * np.arange(1, modes + 1) / n
    sx, cx = np.sin(np.outer(kk, x)), np.cos(np.outer(kk, x))  # (modes, n)
    # u = sum c_kl sin(k x) l cos(l y),  v = -sum c_kl k cos(k x) sin(l y)
    U = np.einsum("kl,lj,ki->ji", coeffs * kk[None, :], cx, sx)
    V = -np.einsum("kl,lj,ki->ji", coeffs * kk[:, None], sx, cx)
    if umax is not None:
        s = umax / max(np.abs(U).max(), np.abs(V).max())
        U, V = U * s, V * s
    return U, V


# -------------------------------------------------------------------------- configs

@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    steps: int
    phys: dict           # keyword arguments of the solver parameters
    phi0: np.ndarray
    velocity: dict | None = None     # separable tables, or None
    field: tuple | None = None       # stored (U, V) base fields, or None


# Prescribed-flow defaults of Sec. III: tau_g = 1, sigma = 0.01, rho_A = 1, rho_B = 0.5.
PRESCRIBED = dict(tau_g=1.0, mobility=0.01, sigma=0.01, width=4.0, phi_a=1.0, phi_b=-1.0,
                  rho_a=1.0, rho_b=0.5, model=2)


def translation(n=128, steps=3200, model=2):
    """Diagonal translation of a circle (radius 25 at n = 128) at u = (0.04, 0.04):
    one period is n / 0.04 = 3200 steps at n = 128."""
    phys = dict(PRESCRIBED, model=model)
    return Workload("translation%d" % n, n, n, steps, phys,
                    circle(n, n, n / 2, n / 2, 25.0 * n / 128, 4.0),
                    uniform_velocity(n, n, 0.04, 0.04, steps))


def vortex(n=512, period=20000, steps=None, radius_frac=77.0 / 512, model=2):
    """Circle (radius 77 at n = 512, centre (n/2, 3n/4)) in the time-reversing single vortex
    with max |u| = 0.05; the field returns at t = period."""
    steps = period if steps is None else steps
    phys = dict(PRESCRIBED, model=model)
    return Workload("vortex%d" % n, n, n, steps, phys,
                    circle(n, n, n / 2, 3 * n / 4, radius_frac * n, 4.0),
                    single_vortex(n, 0.05, period, max(steps, period)))


def metric2048(steps=1000):
    """The throughput workload: 2048^2 periodic, Model-II, tau_g = 1, circle of radius
    0.15 L at (L/2, 3L/4) in the single vortex (max |u| = 0.05, T = 80000)."""
    n = 2048
    return Workload("vortex2048", n, n, steps, dict(PRESCRIBED),
                    circle(n, n, n / 2, 3 * n / 4, 0.15 * n, 4.0),
                    single_vortex(n, 0.05, 80000, max(steps, 1)))


def rt_params(nx=256, atwood=0.5, reynolds=3000.0, sqrt_gl=0.04, sigma=5e-5, width=4.0,
              peclet=1000.0):
    """Rayleigh-Taylor parameters (Sec. III.E) from the dimensionless groups.
    rho_h = 1, rho_l = rho_h (1 - At)/(1 + At); g = sqrt_gl^2 / L;
    nu = L sqrt(At g L / (1 + At)) / Re, tau_f = 1/2 + 3 nu;
    Pe = U* W / (M beta (phi_A - phi_B)^2) with U* = sqrt(g L), so with
    beta = 12 sigma / (16 W) this gives M = U* W / (Pe * 12 sigma / (16 W) * 4)."""
    L = float(nx)
    g = sqrt_gl ** 2 / L
    nu = L * math.sqrt(atwood * g * L / (1.0 + atwood)) / reynolds
    rho_h = 1.0
    rho_l = rho_h * (1.0 - atwood) / (1.0 + atwood)
    beta_lit = 12.0 * sigma / (width * 16.0)   # Pe's beta for phi_A - phi_B = 2
    mob = sqrt_gl * width / (peclet * beta_lit * 4.0)
    return dict(tau_g=1.0, mobility=mob, sigma=sigma, width=width, phi_a=1.0, phi_b=-1.0,
                rho_a=rho_h, rho_b=rho_l, model=2, tau_f=0.5 + 3.0 * nu, gravity=g)


def rayleigh_taylor_case(nx=256, ny=1024, steps=40000, amp_frac=0.1, **kw):
    phys = rt_params(nx=nx, **kw)
    return Workload("rayleigh_taylor%dx%d" % (nx, ny), nx, ny, steps, phys,
                    rayleigh_taylor(nx, ny, phys["width"], amp_frac))


def rayleigh_taylor_paper(atwood, nx=256, ny=1024, steps=40000):
    """Sec. III.E's own case: Re = 400, rho_h = 1, D = W = 4, Pe = 1000, sqrt(g lambda) =
    0.04, d = lambda = nx, interface perturbed by 0.05 d cos(2 pi x / lambda)."""
    return rayleigh_taylor_case(nx, ny, steps, amp_frac=0.05, reynolds=400.0, atwood=atwood)


def stream_basis(n, modes):
    """Velocity of each unit stream-function mode: (modes*modes, 2, n, n) with entry
    [k*modes + l] = (u, v) of psi = sin(2 pi (k+1) x/n) sin(2 pi (l+1) y/n)."""
    out = np.zeros((modes * modes, 2, n, n))
    for k in range(modes):
        for l in range(modes):
            c = np.zeros((modes, modes))
            c[k, l] = 1.0
            out[k * modes + l] = stream_function_field(n, c)
    return out


def stream_coefficients(modes, seed):
    """a_kl ~ N(0, 1) / (k^2 + l^2), k, l = 1..modes, flattened row-major."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, modes + 1)
    return (rng.standard_normal((modes, modes)) / (k[:, None] ** 2 + k[None, :] ** 2)).ravel()


@dataclasses.dataclass
class AdjointCase:
    """Interface-matching problem: phi0 advected for `steps` steps by
    u = scale * sum_k theta_k B_k (B = stream_basis), loss ||phi(N) - phi_target||^2 with
    phi_target produced from held-out coefficients.  `scale` is fixed from the initial
    coefficients (max |u| = umax) and is not a parameter of the loss."""
    name: str
    n: int
    steps: int
    phys: dict
    phi0: np.ndarray
    basis: np.ndarray
    theta: np.ndarray
    scale: float
    theta_target: np.ndarray
    scale_target: float

    def field(self, theta=None, scale=None):
        th = self.theta if theta is None else theta
        sc = self.scale if scale is None else scale
        uv = sc * np.tensordot(th, self.basis, axes=1)
        return uv[0], uv[1]


def adjoint_case(n=256, steps=2000, modes=4, seed=5, target_seed=6, umax=0.05,
                 radius_frac=0.25, model=2):
    """Differentiation workload: 256^2, 2000 steps, 16 seeded Fourier coefficients of the
    stream function (k, l = 1..4), a circle of radius n/4 at the centre, Model-II at
    tau_g = 1 with the prescribed-flow parameters of Sec. III."""
    basis = stream_basis(n, modes)

    def scaled(seed_):
        th = stream_coefficients(modes, seed_)
        uv = np.tensordot(th, basis, axes=1)
        return th, umax / np.abs(uv).max()

    theta, scale = scaled(seed)
    theta_t, scale_t = scaled(target_seed)
    phys = dict(PRESCRIBED, model=model)
    phi0 = circle(n, n, n / 2.0, n / 2.0, radius_frac * n, phys["width"])
    return AdjointCase("adjoint%d" % n, n, steps, phys, phi0, basis, theta, scale, theta_t,
                       scale_t)


def batch_case(n_inst=64, seed=4, sides=(64, 128, 192, 256, 384, 512), modes=8, umax=0.05,
               steps=5000, model=2):
    """Many independent lattices of uneven sizes: side lengths drawn from `sides` by the
    seed, each with 1-3 random circles or ellipses (radii 0.1-0.3 of the side) and a
    steady divergence-free velocity from its own random stream function (modes x modes
    Fourier modes, scaled to max |u| = umax).  Prescribed-flow parameters of Sec. III."""
    rng = np.random.default_rng(seed)
    picks = rng.choice(np.asarray(sides), size=n_inst)
    phys = dict(PRESCRIBED, model=model)
    out = []
    for i, n in enumerate(picks.tolist()):
        phi0 = random_blobs(n, seed=seed * 1000 + i, width=phys["width"])
        U, V = random_stream_function(n, modes, seed * 1000 + 500 + i, umax)
        out.append(Workload("batch%d_%d" % (i, n), n, n, steps, phys, phi0, field=(U, V)))
    return out


# ------------------------------------------------------------- the paper's setups

def mobility_for_pe(pe, u_star, width, sigma, phi_a=1.0, phi_b=-1.0):
    """M from Pe = U* W / (M beta (phi_A - phi_B)^2), beta of Eq. betakappa."""
    d = abs(phi_a - phi_b)
    beta = 12.0 * sigma / (width * d ** 4)
    return u_star * width / (pe * beta * d * d)


def slotted_disk(n, cx, cy, radius, slot_width, slot_top, width, phi_a=1.0, phi_b=-1.0):
    """Zalesak's disk: a disk of phase A with a vertical slot of the given width cut
    from its bottom up to y = cy + slot_top.  The signed distance is the minimum of the
    disk's and the slot complement's (exact away from the slot corners)."""
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    d_disk = radius - np.hypot(x - cx, y - cy)
    # signed distance to the slot rectangle (positive inside it); the rectangle extends
    # below the disk so only its top and sides bound the shape
    hx = slot_width / 2.0
    ybot = cy - 2.0 * radius
    qx = np.abs(x - cx) - hx
    qy = np.maximum(y - (cy + slot_top), ybot - y)
    outside = np.hypot(np.maximum(qx, 0.0), np.maximum(qy, 0.0))
    inside = np.minimum(np.maximum(qx, qy), 0.0)
    d_slot = -(outside + inside)
    return tanh_profile(np.minimum(d_disk, -d_slot), width, phi_a, phi_b)


def paper_params(pe, u_star, width=2.0, sigma=0.01, tau_g=1.0, rho_a=1.0, rho_b=0.5, model=2):
    return dict(tau_g=tau_g, mobility=mobility_for_pe(pe, u_star, width, sigma), sigma=sigma,
                width=width, phi_a=1.0, phi_b=-1.0, rho_a=rho_a, rho_b=rho_b, model=model)


def translation_paper(periods=1, tau_g=1.0, rho_b=0.5, model=2, n=200, u0=0.02, pe=200.0):
    """Diagonal translation of Sec. III.A: L0 = 200, R = L0/5, U0 = 0.02 along (1, 1),
    W = 2, sigma = 0.01, Pe = 200; one period is L0/U0 steps."""
    steps = int(round(periods * n / u0))
    phys = paper_params(pe, u0, tau_g=tau_g, rho_b=rho_b, model=model)
    return Workload("translation_paper%d" % n, n, n, steps, phys,
                    circle(n, n, n / 2, n / 2, n / 5.0, phys["width"]),
                    uniform_velocity(n, n, u0, u0, steps))


def zalesak(periods=2, model=2, n=200, radius=80.0, slot=16.0, u0=0.02, pe=200.0):
    """Zalesak's disk of Sec. III.B: L0 = 200, R = 80, slot 16 wide reaching R/4 above the
    centre, rigid rotation with U0 = 0.02 (period 2 L0 / U0), W = 2, sigma = 0.01,
    Pe = 200, rho_A = 1, rho_B = 0.5."""
    steps = int(round(periods * 2 * n / u0))
    phys = paper_params(pe, u0, model=model)
    return Workload("zalesak%d" % n, n, n, steps, phys,
                    slotted_disk(n, n / 2, n / 2, radius, slot, radius / 4, phys["width"]),
                    rigid_rotation(n, u0, steps))


def shear_paper(model=2, n=200, u0=0.025, pe=1000.0):
    """Circle in the reversing shear flow of Sec. III.C: L0 = 200, R = L0/5 at (100, 60),
    U0 = 0.025, W = 2, Pe = 1000, reversed at T = L0 / U0, back at 2T."""
    period = int(round(n / u0))
    steps = 2 * period
    phys = paper_params(pe, u0, model=model)
    return Workload("shear_paper%d" % n, n, n, steps, phys,
                    circle(n, n, 100.0 * n / 200, 60.0 * n / 200, n / 5.0, phys["width"]),
                    shear_reversal(n, u0, period, steps))
