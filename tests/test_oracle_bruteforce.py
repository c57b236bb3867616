"""Brute-force pin of the oracle: two whole steps on an 8x8 periodic lattice computed
here in 50-digit arithmetic, node by node, against the FP64 oracle.

The computation below is written from the equations of the paper in forms that differ
from the oracle's: the isotropic derivatives as weighted sums over the lattice
directions, (1/cs^2) sum_i w_i c_i psi(x + c_i) and (2/cs^2) sum_i w_i (psi(x + c_i) -
psi(x)), instead of explicit neighbour formulas; streaming as a push of every
post-collision population to x + c_i instead of a pull; the lattice vectors and
weights generated from their definition (|c_i|^2 = 0, 1, 2 with w = 4/9, 1/9, 1/36)
instead of a table.  With 50 digits its own rounding is ~1e-50, so any difference
above the oracle's FP64 rounding (~1e-15 on O(1) populations) is a slip in one of the
two: a dropped term, a wrong sign, index or direction.
"""
import itertools

import numpy as np
import pytest

import oracle

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp


def _lattice():
    """D2Q9: c in {-1,0,1}^2; w = 4/9, 1/9, 1/36 for |c|^2 = 0, 1, 2 (Sec. II)."""
    cs = [(0, 0)] + [c for c in itertools.product((-1, 0, 1), repeat=2) if c != (0, 0)]
    w = {0: mp.mpf(4) / 9, 1: mp.mpf(1) / 9, 2: mp.mpf(1) / 36}
    return cs, [w[cx * cx + cy * cy] for cx, cy in cs]


def _step_mp(g, ux, uy, par, n, first):
    """One step of Eqs. LB, geq, liangFi, mu, t0-phiu, mark3 on the periodic lattice;
    g maps (c, x, y) -> population.  Returns the new populations.  With first, g is
    ignored and the equilibrium start of the scheme is returned instead."""
    cs, w = _lattice()
    cs2 = mp.mpf(1) / 3
    tau = par["tau"]
    pa, pb = par["phi_a"], par["phi_b"]
    beta = 12 * par["sigma"] / (par["width"] * (pa - pb) ** 4)
    kappa = 3 * par["sigma"] * par["width"] / (2 * (pa - pb) ** 2)
    eta = par["mobility"] / (cs2 * (tau - mp.mpf(1) / 2))
    K = (tau - mp.mpf(1) / 6 - tau * tau) / (tau - mp.mpf(1) / 2)
    a = (par["rho_a"] - par["rho_b"]) / (pa - pb)
    b = (par["rho_b"] * pa - pb * par["rho_a"]) / (pa - pb)
    nodes = [(x, y) for y in range(n) for x in range(n)]

    def shift(x, y, c):
        return ((x + c[0]) % n, (y + c[1]) % n)

    def grad(psi):
        return {p: (sum(wi * c[0] * psi[shift(*p, c)] for c, wi in zip(cs, w)) / cs2,
                    sum(wi * c[1] * psi[shift(*p, c)] for c, wi in zip(cs, w)) / cs2)
                for p in nodes}

    def lap(psi):
        return {p: 2 * sum(wi * (psi[shift(*p, c)] - psi[p]) for c, wi in zip(cs, w)) / cs2
                for p in nodes}

    r32 = (lambda d: {k: mp.mpf(float(np.float32(float(v)))) for k, v in d.items()}) \
        if par.get("round32") and not first else (lambda d: d)
    if first:
        phi = par["phi0"]
    else:
        phi = r32({p: sum(g[(c, *p)] for c in cs) for p in nodes})
    lp = lap(phi)
    mu = r32({p: 2 * beta * (phi[p] - pa) * (phi[p] - pb) * (2 * phi[p] - pa - pb) - kappa * lp[p]
              for p in nodes})

    def geq(p, c, wi):
        u, v = ux[p], uy[p]
        cu = c[0] * u + c[1] * v
        s = cu / cs2 + cu * cu / (2 * cs2 * cs2) - (u * u + v * v) / (2 * cs2)
        if c == (0, 0):
            return phi[p] - (1 - wi) * eta * mu[p] + wi * phi[p] * s
        return wi * (eta * mu[p] + phi[p] * s)

    if first:  # equilibrium start, no source term
        return {(c, *p): geq(p, c, wi) for p in nodes for c, wi in zip(cs, w)}
    gm = grad(mu)
    force = {}
    if par.get("f1_form", 0) == 1:
        # the material acceleration of a steady prescribed u: F1 = phi (u.grad) u
        gu, gv = grad(ux), grad(uy)
        for p in nodes:
            force[p] = [phi[p] * (ux[p] * gu[p][0] + uy[p] * gu[p][1]),
                        phi[p] * (ux[p] * gv[p][0] + uy[p] * gv[p][1])]
    else:
        for p in nodes:
            rho = a * phi[p] + b
            force[p] = [phi[p] / rho * (-phi[p] * gm[p][0]),
                        phi[p] / rho * (-phi[p] * gm[p][1])]
    if par["model"] == 2:
        qx = r32({p: phi[p] * ux[p] for p in nodes})
        qy = r32({p: phi[p] * uy[p] for p in nodes})
        gqx, gqy = grad(qx), grad(qy)
        div = r32({p: gqx[p][0] + gqy[p][1] for p in nodes})
        gd = grad(div)
        for p in nodes:
            force[p][0] += 3 * cs2 * K * gd[p][0]
            force[p][1] += 3 * cs2 * K * gd[p][1]
    out = {}
    for p in nodes:
        for c, wi in zip(cs, w):
            src = wi * (c[0] * force[p][0] + c[1] * force[p][1]) / cs2
            post = g[(c, *p)] - (g[(c, *p)] - geq(p, c, wi)) / tau + (1 - 1 / (2 * tau)) * src
            out[(c, *shift(*p, c))] = post  # push
    return r32(out)


@pytest.mark.parametrize("tau,model,f1_form", [(1.0, 2, 0), (0.8, 2, 0), (0.8, 1, 0),
                                               (1.3, 2, 0), (0.8, 1, 1), (1.3, 2, 1)])
def test_two_steps_match_50_digit_brute_force(tau, model, f1_form):
    """f1_form 1 is the alternative reading of F1 with a prescribed velocity (the
    material acceleration of u, here steady) that the oracle keeps for comparison."""
    mp.dps = 50
    n = 8
    rng = np.random.default_rng(21)
    phi0 = np.clip(rng.normal(0.0, 0.6, (n, n)), -1.2, 1.2)
    ux = rng.uniform(-0.05, 0.05, (n, n))
    uy = rng.uniform(-0.05, 0.05, (n, n))
    phys = dict(tau_g=tau, mobility=0.02, sigma=0.01, width=3.0, phi_a=1.0, phi_b=-1.0,
                rho_a=1.0, rho_b=0.4)
    p = oracle.Params(nx=n, ny=n, model=model, f1_form=f1_form, **phys)
    st = oracle.State(p, phi0, ux, uy)
    orc = [st.g.copy()]
    for _ in range(2):
        st.run(1)
        orc.append(st.g.copy())

    par = {"tau": mp.mpf(tau), "model": model, "f1_form": f1_form, "phi0": {}}
    for k in ("mobility", "sigma", "width", "phi_a", "phi_b", "rho_a", "rho_b"):
        par[k] = mp.mpf(phys[k])
    U, V = {}, {}
    for y in range(n):
        for x in range(n):
            par["phi0"][(x, y)] = mp.mpf(phi0[y, x])
            U[(x, y)] = mp.mpf(ux[y, x])
            V[(x, y)] = mp.mpf(uy[y, x])
    g = _step_mp(None, U, V, par, n, first=True)
    states = [g]
    for _ in range(2):
        g = _step_mp(g, U, V, par, n, first=False)
        states.append(g)

    # oracle population index i has c = (CX[i], CY[i]) in the standard D2Q9 order
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    for k, (gm, go) in enumerate(zip(states, orc)):
        err = 0.0
        for i in range(9):
            for y in range(n):
                for x in range(n):
                    err = max(err, abs(float(gm[((cx[i], cy[i]), x, y)]) - go[i, y, x]))
        print("tau %.2f model %d after %d steps: max |g_oracle - g_brute| = %.2e" % (tau, model, k, err))
        assert err <= 1e-14, (k, err)


def test_round_f32_rounds_where_the_gpu_holds_float32():
    """round_f32 (the sensitivity runs that derive long-run tolerances) rounds phi, mu,
    q = phi u and div q to float32 where they are formed, and the populations after each
    step; the 50-digit step with the same rounding points agrees to FP64 accuracy, and
    the rounding does change the result."""
    mp.dps = 50
    n = 8
    rng = np.random.default_rng(9)
    phi0 = np.clip(rng.normal(0.0, 0.6, (n, n)), -1.2, 1.2)
    ux = rng.uniform(-0.05, 0.05, (n, n))
    uy = rng.uniform(-0.05, 0.05, (n, n))
    phys = dict(tau_g=0.8, mobility=0.02, sigma=0.01, width=3.0, phi_a=1.0, phi_b=-1.0,
                rho_a=1.0, rho_b=0.4)
    st = oracle.State(oracle.Params(nx=n, ny=n, model=2, round_f32=1, **phys), phi0, ux, uy)
    plain = oracle.State(oracle.Params(nx=n, ny=n, model=2, **phys), phi0, ux, uy)
    st.run(2)
    plain.run(2)
    par = {"tau": mp.mpf(0.8), "model": 2, "round32": True, "phi0": {}}
    for k in ("mobility", "sigma", "width", "phi_a", "phi_b", "rho_a", "rho_b"):
        par[k] = mp.mpf(phys[k])
    U, V = {}, {}
    for y in range(n):
        for x in range(n):
            par["phi0"][(x, y)] = mp.mpf(phi0[y, x])
            U[(x, y)] = mp.mpf(ux[y, x])
            V[(x, y)] = mp.mpf(uy[y, x])
    g = _step_mp(None, U, V, par, n, first=True)
    for _ in range(2):
        g = _step_mp(g, U, V, par, n, first=False)
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    ref = np.array([[[float(g[((cx[i], cy[i]), x, y)]) for x in range(n)] for y in range(n)]
                    for i in range(9)])
    assert np.array_equal(st.g, st.g.astype(np.float32).astype(np.float64))
    assert np.abs(st.g - ref).max() <= 1e-14
    assert np.abs(st.g - plain.g).max() > 1e-10


def test_float32_build_is_the_same_method():
    """The float32 build of the oracle (sensitivity runs only) is the same code in another
    precision: a few steps agree with the FP64 oracle to float32 rounding, prescribed
    flow (Model-II, tau = 0.8) and coupled Navier-Stokes with walls, and they do differ."""
    n = 16
    rng = np.random.default_rng(11)
    phi0 = np.clip(rng.normal(0.0, 0.6, (n, n)), -1.2, 1.2)
    ux = rng.uniform(-0.05, 0.05, (n, n))
    uy = rng.uniform(-0.05, 0.05, (n, n))
    p = oracle.Params(nx=n, ny=n, model=2, tau_g=0.8, mobility=0.02, sigma=0.01, width=3.0,
                      rho_b=0.4)
    a = oracle.State(p, phi0, ux, uy).run(3)
    b = oracle.State32(p, phi0, ux, uy).run(3)
    d = np.abs(a.g - b.g).max()
    assert 0 < d <= 2e-6 and b.g.dtype == np.float32
    import workloads
    w = workloads.rayleigh_taylor_case(16, 48, steps=20, reynolds=100.0)
    q = oracle.Params(nx=16, ny=48, walls=1, ns=1, **w.phys)
    a = oracle.State(q, w.phi0).run(20)
    b = oracle.State32(q, w.phi0).run(20)
    assert 0 < np.abs(a.phi - b.phi).max() <= 1e-5
    assert 0 < np.abs(a.f - b.f).max() <= 1e-7
