"""Coupled Rayleigh-Taylor instability (Sec. III.E) at its full size, 256x1024 with walls,
At = 0.5, Re = 3000, W = 4, Pe = 1000, sqrt(gL) = 0.04 (time unit T = sqrt(L/(At g))
= 9051 steps):

* phi at stored FP64 oracle samples after 1000 and 4000 steps and at T (mass drift <=
  1e-6; the relative L2 gate is derived below, and is the 1e-4 of the other parity
  tests until the instability has grown);
* through t = T the run stays finite with the same mass bound, extrema within those of
  the oracle at T, and the heavy fluid's spike and the light fluid's bubble move down
  and up.  The oracle itself diverges past 1.3 T in this configuration (the lattice
  Mach number of the falling spike passes ~0.1 with tau_f = 0.506); the paper's own
  parameters are the full-length case;
* the paper's own parameters (Re = 400, At = 0.1 and 0.25) for the full 40000 steps,
  At = 0.25 also against stored FP64 oracle samples after those 40000 steps;
* 16-bit population storage (the f populations stay float32) against the float32 run.

Long-run gates come from the stored oracle runs themselves: next to each FP64 run the
golden file holds the same run with the oracle's own code compiled in float32
arithmetic, and the sampled distance between the two (sens32_rel_l2) is how far the
instability carries float32 rounding by that time.  The GPU computes in float32 too
(with FP64 sums for phi), so its distance from the FP64 oracle is gated at twice that
distance (and never below 1e-4); extrema likewise with sens32_max_abs.  (A rerun that
only rounds the values the float32 path stores, sens_rel_l2, stays 4-90 times lower
and understates the drift: two independently written float32 GPU kernels of the step
agree with each other to that level, while both drift from FP64 as the float32 build
of the oracle does.)
"""
import math
import os

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lbm():
    import paper_1805_00007_amd as lbm
    lbm.lib()
    return lbm


def _fronts(phi):
    """Lowest row holding heavy fluid (spike tip) and highest row holding light fluid
    (bubble tip), from the column extremes of the phi = 0 level."""
    heavy = phi > 0
    rows = np.arange(phi.shape[0])[:, None] * np.ones((1, phi.shape[1]))
    spike = rows[heavy].min() if heavy.any() else np.nan
    bubble = rows[~heavy].max() if (~heavy).any() else np.nan
    return float(spike), float(bubble)


def _gate(g, key="rel_l2"):
    """Gate of a stored run: 1e-4, or twice the distance of the float32 build of the
    oracle from the FP64 run (sens32_rel_l2 / sens32_max_abs) where that is larger."""
    return max(1e-4, 2.0 * float(g["sens32_" + key]))


@pytest.mark.parametrize("steps", [1000, 4000, 9051])
def test_rayleigh_taylor_full_size_against_stored_oracle(lbm, steps):
    path = os.path.join(HERE, "golden", "rt256_oracle_%d.npz" % steps)
    if not os.path.exists(path):
        pytest.skip("stored oracle samples missing: run tests/golden/make_golden.py")
    g = np.load(path)
    w = workloads.rayleigh_taylor_case(256, 1024, steps=steps)
    s = lbm.solver_for(w, walls=1)
    s.step(steps)
    d = s.diagnostics()
    phi = s.phi().double().cpu().numpy().ravel()
    s.close()
    idx, ref = g["index"], g["phi"]
    rel = float(np.sqrt(((phi[idx] - ref) ** 2).sum() / (ref ** 2).sum()))
    drift = abs(d["mass"] - float(g["mass0"])) / float(g["abs_mass0"])
    tol = _gate(g)
    print("rt256 %d steps: sampled rel_l2 %.3e (gate %.1e) max %.3e drift %.3e extrema "
          "%.4f/%.4f (oracle %.4f/%.4f)" % (steps, rel, tol, np.abs(phi[idx] - ref).max(),
                                            drift, d["max"], d["min"], float(g["max"]),
                                            float(g["min"])))
    assert rel <= tol
    assert drift <= 1e-6
    ext = _gate(g, "max_abs")
    assert d["max"] == pytest.approx(float(g["max"]), abs=ext)
    assert d["min"] == pytest.approx(float(g["min"]), abs=ext)


def _run(lbm, w, storage, checkpoints):
    s = lbm.solver_for(w, walls=1, storage=storage)
    m0 = s.diagnostics()["mass"]
    done, out = 0, {}
    for c in checkpoints:
        s.step(c - done)
        done = c
        d = s.diagnostics()
        out[c] = (d, s.phi().cpu().numpy())
    s.close()
    return m0, out


def test_rayleigh_taylor_first_period(lbm):
    """At = 0.5, Re = 3000 through t = T: finite, mass conserved, extrema within those the
    oracle reaches at T (which bound the earlier ones: the overshoots grow), the spike
    and bubble moving."""
    g = np.load(os.path.join(HERE, "golden", "rt256_oracle_9051.npz"))
    bound = max(float(g["max"]), -float(g["min"])) + 1e-3
    w = workloads.rayleigh_taylor_case(256, 1024, steps=40000)
    T = math.sqrt(256 / (0.5 * w.phys["gravity"]))
    checks = [int(round(f * T)) for f in (0.25, 0.5, 0.75, 1.0)]
    m0, out = _run(lbm, w, lbm.STORE_F32, checks)
    abs0 = np.abs(w.phi0).sum()
    spike0, bubble0 = _fronts(w.phi0)
    for c in checks:
        d, phi = out[c]
        spike, bubble = _fronts(phi)
        print("At 0.5, Re 3000, t = %.2f T: drift %.2e max %.4f min %.4f spike %.0f bubble %.0f"
              % (c / T, abs(d["mass"] - m0) / abs0, d["max"], d["min"], spike, bubble))
        assert d["nonfinite"] == 0
        assert abs(d["mass"] - m0) / abs0 <= 1e-6
        assert d["max"] < bound and d["min"] > -bound
    assert spike < spike0 and bubble > bubble0


@pytest.mark.parametrize("atwood", [0.1, 0.25])
def test_rayleigh_taylor_paper_parameters_full_length(lbm, atwood):
    """The paper's own Sec. III.E parameters (Re = 400, At = 0.1 and 0.25, sqrt(g L) =
    0.04, Pe = 1000, W = 4), 40000 steps: finite, mass conserved, fronts moving, extrema
    within those the FP64 oracle reaches at 40000 steps with At = 0.25 (the overshoots
    grow with time and with At)."""
    g = np.load(os.path.join(HERE, "golden", "rtpaper25_oracle_40000.npz"))
    bound = max(float(g["max"]), -float(g["min"])) + 1e-3
    w = workloads.rayleigh_taylor_paper(atwood, steps=40000)
    T = math.sqrt(256 / (atwood * w.phys["gravity"]))
    checks = [10000, 20000, 30000, 40000]
    m0, out = _run(lbm, w, lbm.STORE_F32, checks)
    abs0 = np.abs(w.phi0).sum()
    spike0, bubble0 = _fronts(w.phi0)
    for c in checks:
        d, phi = out[c]
        spike, bubble = _fronts(phi)
        print("At %.2f, Re 400, t = %.2f T: drift %.2e max %.4f min %.4f spike %.0f bubble %.0f"
              % (atwood, c / T, abs(d["mass"] - m0) / abs0, d["max"], d["min"], spike, bubble))
        assert d["nonfinite"] == 0
        assert abs(d["mass"] - m0) / abs0 <= 1e-6
        assert d["max"] < bound and d["min"] > -bound
    assert spike < spike0 - 50 and bubble > bubble0 + 20


def test_rayleigh_taylor_paper_parameters_against_stored_oracle(lbm):
    """At = 0.25, Re = 400 for the full 40000 steps (3.1 time units, the spike and bubble
    well developed) against stored FP64 oracle samples: the FP32-vs-FP64 error at the
    case's full length.  Rounding differences of ~1e-7 per step are carried by the
    instability as it grows: the gate is derived from the stored float32 build of the
    oracle (see the module docstring); mass is held to the same 1e-6."""
    path = os.path.join(HERE, "golden", "rtpaper25_oracle_40000.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle samples missing: run tests/golden/make_golden.py")
    g = np.load(path)
    steps = int(g["steps"])
    w = workloads.rayleigh_taylor_paper(0.25, steps=steps)
    s = lbm.solver_for(w, walls=1)
    s.step(steps)
    d = s.diagnostics()
    phi = s.phi().double().cpu().numpy().ravel()
    s.close()
    idx, ref = g["index"], g["phi"]
    rel = float(np.sqrt(((phi[idx] - ref) ** 2).sum() / (ref ** 2).sum()))
    drift = abs(d["mass"] - float(g["mass0"])) / float(g["abs_mass0"])
    print("At 0.25, Re 400, %d steps: sampled rel_l2 %.3e max %.3e drift %.3e extrema "
          "%.4f/%.4f (oracle %.4f/%.4f)" % (steps, rel, np.abs(phi[idx] - ref).max(), drift,
                                            d["max"], d["min"], float(g["max"]), float(g["min"])))
    tol = _gate(g)
    print("  gate %.3e (float32 build of the oracle: %.3e)" % (tol, float(g["sens32_rel_l2"])))
    assert rel <= tol
    assert drift <= 1e-6
    ext = _gate(g, "max_abs")
    assert abs(d["max"] - float(g["max"])) <= ext
    assert abs(d["min"] - float(g["min"])) <= ext


@pytest.mark.parametrize("storage,tol", [(1, 2.5e-4), (2, 2.5e-3)])
def test_rayleigh_taylor_16bit_storage(lbm, storage, tol):
    """Half and bfloat16 codes of g_i / w_i for the phase field (the f populations stay
    float32), paper parameters At = 0.25, Re = 400: relative L2 distance from the float32
    run at 0.5 T and 1 T within one rounding unit of the code (2^-12 for half's 11 bits,
    2^-9 for bfloat16's 8, rounded up), as at 2048^2; mass conservation."""
    w = workloads.rayleigh_taylor_paper(0.25, steps=20000)
    T = math.sqrt(256 / (0.25 * w.phys["gravity"]))
    checks = [int(round(0.5 * T)), int(round(T))]
    _, ref = _run(lbm, w, lbm.STORE_F32, checks)
    m0, out = _run(lbm, w, storage, checks)
    abs0 = np.abs(w.phi0).sum()
    for c in checks:
        d, phi = out[c]
        r = ref[c][1]
        dist = float(np.sqrt(((phi - r) ** 2).sum() / (r ** 2).sum()))
        print("storage %d, t = %.1f T: rel L2 to float32 %.3e, drift %.2e" % (
            storage, c / T, dist, abs(d["mass"] - m0) / abs0))
        assert d["nonfinite"] == 0
        assert abs(d["mass"] - m0) / abs0 <= 1e-6
        assert dist <= tol
