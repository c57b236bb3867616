"""The paper's own test problems (Sec. III.A-C) on the GPU path: parity with the FP64
oracle on short runs, then the claims the paper makes in words, at full length:

* Sec. III.A, diagonal translation (L0 = 200, R = 40, U0 = 0.02, W = 2, Pe = 200,
  rho_A/rho_B = 2): over the tau sweep Model-I's error after one period is smallest at
  tau = 1/2 + sqrt(3)/6, and Model-II (the F2 of Eq. mark3, and Eq. F2-1 with time
  derivatives) has a smaller error than Model-I at every other tau;
* Sec. III.A, the same at tau = 1/2 + sqrt(3)/6 with rho_A = rho_B after 4T: the
  extrema of phi stay within a few percent of phi_A, phi_B (the printed values are a
  soft check, reported but not gated);
* Sec. III.B, Zalesak's disk after 2T: Model-II's error is below Model-I's;
* Sec. III.C, reversing shear flow: the interface comes back at 2T (error far below
  the error at T) and Model-II's error is below Model-I's.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAU_K0 = 0.5 + math.sqrt(3) / 6


@pytest.fixture(scope="module")
def lbm():
    import paper_1805_00007_amd as lbm
    lbm.lib()
    return lbm


def _error(lbm, w, steps, **over):
    s = lbm.solver_for(w, **over)
    s.step(steps)
    d = s.diagnostics(w.phi0)
    s.close()
    assert d["nonfinite"] == 0
    return math.sqrt(d["err2"] / d["ref2"]), d["max"], d["min"]


@pytest.mark.parametrize("make,over", [
    (lambda: workloads.zalesak(2, model=2), {}),
    (lambda: workloads.shear_paper(model=2), {}),
    (lambda: workloads.translation_paper(1, tau_g=TAU_K0, model=3), {})])
def test_paper_setups_match_oracle(lbm, make, over):
    w = make()
    steps = 400
    s = lbm.solver_for(w, **over)
    s.step(steps)
    phi = s.phi().double().cpu().numpy()
    s.close()
    U, V = workloads.separable_field(w.velocity)
    o = oracle.State(oracle.Params(nx=w.nx, ny=w.ny, **w.phys), w.phi0, U, V,
                     w.velocity["tf"]).run(steps)
    err = oracle.rel_l2(phi, o.phi)
    print("%s %d steps rel_l2 vs oracle %.3e" % (w.name, steps, err))
    assert err <= 1e-4


def test_translation_tau_sweep(lbm):
    taus = (0.6, 0.7, TAU_K0, 0.9, 1.0, 1.2, 1.5)
    err = {}
    for model in (1, 2, 3):
        for tau in taus:
            w = workloads.translation_paper(1, tau_g=tau, model=model)
            err[model, tau] = _error(lbm, w, w.steps)[0]
            print("translation tau %.4f model %d E_phi %.4e" % (tau, model, err[model, tau]))
    assert min(taus, key=lambda t: err[1, t]) == TAU_K0
    for tau in taus:
        if tau != TAU_K0:
            assert err[2, tau] < 0.7 * err[1, tau], tau
            assert err[3, tau] < 0.7 * err[1, tau], tau
    # at K = 0 Eq. mark3 adds nothing (K is zero up to rounding), so Model-II with it
    # equals Model-I
    assert abs(err[2, TAU_K0] - err[1, TAU_K0]) <= 1e-6 * err[1, TAU_K0]


def test_translation_extrema_soft(lbm):
    printed = (1.0487, -1.0361)
    for model in (2, 3):
        w = workloads.translation_paper(4, tau_g=TAU_K0, rho_b=1.0, model=model)
        e, mx, mn = _error(lbm, w, w.steps)
        print("4T, tau = 1/2 + sqrt(3)/6, rho_A = rho_B, model %d: max %.4f min %.4f "
              "(printed %.4f %.4f), E_phi %.3e" % (model, mx, mn, *printed, e))
        assert 1.0 < mx < 1.06 and -1.05 < mn < -1.0


def test_zalesak_model2_beats_model1(lbm):
    e = {}
    for model in (1, 2):
        w = workloads.zalesak(2, model=model)
        e[model] = _error(lbm, w, w.steps)[0]
    print("Zalesak 2T E_phi: Model-I %.4e, Model-II %.4e" % (e[1], e[2]))
    assert e[2] < 0.8 * e[1]


def test_shear_returns_and_model2_beats_model1(lbm):
    e = {}
    for model in (1, 2):
        w = workloads.shear_paper(model=model)
        half = _error(lbm, w, w.steps // 2)[0]
        e[model] = _error(lbm, w, w.steps)[0]
        print("shear model %d: E_phi at T %.4e, at 2T %.4e" % (model, half, e[model]))
        assert e[model] < 0.2 * half
    assert e[2] < e[1]
