"""Write stored FP64 oracle samples for workloads too large to run in a test.

Calls only ``oracle`` and ``workloads``.  For each case it runs the oracle for the
stated number of steps and stores phi at seeded sample nodes, the full-field relative
L2 of phi against the initial field (Eq. err), the initial mass sums and the final
extrema.  The samples are stratified so that the interface, where the method does its
work, is well represented: about half of them where |phi| < 0.95 at the end of the
run, a uniform draw over the lattice, and one whole lattice row crossing the
interface (the row holding most interface nodes).

For the Rayleigh-Taylor cases the run is repeated twice in float32: with the values the
float32 path holds rounded to float32 where they are formed (round_f32; sens_rel_l2),
and with the oracle's own code compiled in float32 arithmetic (State32; sens32_rel_l2).
The sampled relative L2 distance of each from the FP64 run measures how far the
growing instability carries float32 rounding; the long-run GPU tolerance is derived
from the float32 build's (``--sens-only`` recomputes just these runs of an existing
file).

    python tests/golden/make_golden.py vortex2048     # 2048^2, 1000 steps
    python tests/golden/make_golden.py vortex512      # 512^2, one period T = 20000
    python tests/golden/make_golden.py rt256          # 256x1024 Rayleigh-Taylor, 1000 steps
    python tests/golden/make_golden.py rt256_4000     # the same after 4000 steps (0.44 T)
    python tests/golden/make_golden.py rt256_T        # the same through T = 9051 steps
    python tests/golden/make_golden.py rtpaper25_40000  # At 0.25, Re 400 (Sec. III.E), 40000 steps
    python tests/golden/make_golden.py adjoint256     # 256^2, 2000 steps: target + FD gradients

The adjoint case stores the target field phi_target (the oracle run with the held-out
coefficients) and FP64 central finite differences (h = 1e-6) of the loss
||phi(N) - phi_target||^2 with respect to all 16 stream-function coefficients and phi0
at 8 seeded nodes.
"""
import dataclasses
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

CASES = {
    "vortex2048": (lambda: workloads.metric2048(steps=1000), 1000, 0),
    "vortex512": (lambda: workloads.vortex(512, period=20000), 20000, 0),
    "rt256": (lambda: workloads.rayleigh_taylor_case(256, 1024, steps=1000), 1000, 1),
    "rt256_4000": (lambda: workloads.rayleigh_taylor_case(256, 1024, steps=4000), 4000, 1),
    # T = sqrt(L / (At g)) = 9051 steps for L = 256, At = 0.5, sqrt(g L) = 0.04
    "rt256_T": (lambda: workloads.rayleigh_taylor_case(256, 1024, steps=9051), 9051, 1),
    "rtpaper25_40000": (lambda: workloads.rayleigh_taylor_paper(0.25, steps=40000), 40000, 1),
}


def sample_index(phi, seed=20240601, n_band=2560, n_uniform=1536):
    """Stratified sample nodes of a final (ny, nx) field: n_band nodes where |phi| < 0.95,
    n_uniform nodes over the whole lattice, and the whole row with most band nodes."""
    ny, nx = phi.shape
    rng = np.random.default_rng(seed)
    flat = phi.ravel()
    band = np.flatnonzero(np.abs(flat) < 0.95)
    pick = [rng.choice(band, size=min(n_band, len(band)), replace=False)] if len(band) else []
    pick.append(rng.choice(nx * ny, size=n_uniform, replace=False))
    row = int(np.argmax((np.abs(phi) < 0.95).sum(axis=1)))
    pick.append(row * nx + np.arange(nx))
    return np.unique(np.concatenate(pick)), row


def _state(w, p):
    if w.velocity is not None:
        U, V = workloads.separable_field(w.velocity)
        return oracle.State(p, w.phi0, U, V, w.velocity["tf"])
    return oracle.State(p, w.phi0)


def sensitivity(w, p, steps, idx, ref, have=None):
    """Sampled distances of two float32 runs from the FP64 run at `idx` (values `ref`):
    the oracle with its float32 values rounded where the float32 path holds them
    (round_f32), and the oracle's own code compiled with float32 arithmetic (State32).
    The round_f32 run is skipped when `have` already holds its results."""
    rel = lambda x: float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))
    out = {}
    if have and "sens_rel_l2" in have:
        out = dict(sens_rel_l2=float(have["sens_rel_l2"]), sens_max_abs=float(have["sens_max_abs"]))
    else:
        r = _state(w, dataclasses.replace(p, round_f32=1)).run(steps).phi.ravel()[idx]
        out = dict(sens_rel_l2=rel(r), sens_max_abs=float(np.abs(r - ref).max()))
    if w.velocity is not None:
        U, V = workloads.separable_field(w.velocity)
        s32 = oracle.State32(p, w.phi0, U, V, w.velocity["tf"])
    else:
        s32 = oracle.State32(p, w.phi0)
    q = s32.run(steps).phi.ravel()[idx]
    out.update(sens32_rel_l2=rel(q), sens32_max_abs=float(np.abs(q - ref).max()))
    print("float32-rounded rerun: sampled rel L2 %.3e; float32 build: %.3e" % (
        out["sens_rel_l2"], out["sens32_rel_l2"]), flush=True)
    return out


def make(name, sens_only=False):
    """Run case `name` and write its file; with sens_only, keep the FP64 results of the
    existing file and recompute only its sensitivity runs."""
    build, steps, walls = CASES[name]
    w = build()
    p = oracle.Params(nx=w.nx, ny=w.ny, walls=walls, ns=1 if "tau_f" in w.phys else 0,
                      **w.phys)
    out = os.path.join(HERE, "%s_oracle_%d.npz" % (name.split("_")[0], steps))
    t0 = time.time()
    if sens_only:
        old = dict(np.load(out))
        old.update(sensitivity(w, p, steps, old["index"], old["phi"], have=old))
        np.savez_compressed(out, **old)
        print(out, "sensitivity %.0fs" % (time.time() - t0))
        return
    s = _state(w, p)
    d0 = oracle.diag(p, s.phi)
    s.run(steps)
    phi = s.phi
    d = oracle.diag(p, phi, w.phi0)
    idx, row = sample_index(phi)
    extra = sensitivity(w, p, steps, idx, phi.ravel()[idx]) if p.ns else {}
    np.savez_compressed(out, steps=steps, index=idx, phi=phi.ravel()[idx], row=row,
                        mass0=d0["mass"], abs_mass0=d0["abs_mass"], mass=d["mass"],
                        e_phi=np.sqrt(d["err2"] / d["ref2"]), max=d["max"], min=d["min"],
                        threads=oracle.num_threads(), seconds=time.time() - t0, **extra)
    print(out, "samples=%d E_phi=%.4e max=%.4f min=%.4f %.0fs" % (
        len(idx), np.sqrt(d["err2"] / d["ref2"]), d["max"], d["min"], time.time() - t0))


def adjoint_run(case, p, phi0, theta, scale):
    U, V = case.field(theta, scale)
    return oracle.State(p, phi0, U, V).run(case.steps).phi


def adjoint_fd(case, h=1e-6, nodes=8, seed=20240602):
    """Central differences of L = sum (phi(N) - phi_target)^2, each as
    sum (phi+ - phi-)(phi+ + phi- - 2 phi_target) / (2 h) to avoid cancelling L."""
    p = oracle.Params(nx=case.n, ny=case.n, **case.phys)
    target = adjoint_run(case, p, case.phi0, case.theta_target, case.scale_target)
    base = adjoint_run(case, p, case.phi0, case.theta, case.scale)

    def fd(plus, minus):
        return float(((plus - minus) * (plus + minus - 2.0 * target)).sum() / (2.0 * h))

    g_theta = np.zeros(len(case.theta))
    for k in range(len(case.theta)):
        e = np.zeros_like(case.theta)
        e[k] = h
        g_theta[k] = fd(adjoint_run(case, p, case.phi0, case.theta + e, case.scale),
                        adjoint_run(case, p, case.phi0, case.theta - e, case.scale))
        print("theta", k, g_theta[k], flush=True)
    rng = np.random.default_rng(seed)
    near = np.flatnonzero(np.abs(case.phi0.ravel()) < 0.9)
    idx = np.sort(np.concatenate([rng.choice(near, nodes - 1, replace=False),
                                  [case.n // 2 * case.n + case.n // 2]]))
    g_phi = np.zeros(len(idx))
    for j, i in enumerate(idx):
        d = np.zeros(case.n * case.n)
        d[i] = h
        d = d.reshape(case.n, case.n)
        g_phi[j] = fd(adjoint_run(case, p, case.phi0 + d, case.theta, case.scale),
                      adjoint_run(case, p, case.phi0 - d, case.theta, case.scale))
        print("phi0", i, g_phi[j], flush=True)
    return target, base, g_theta, idx, g_phi


def make_adjoint(n=256, steps=2000):
    case = workloads.adjoint_case(n, steps)
    t0 = time.time()
    target, base, g_theta, idx, g_phi = adjoint_fd(case)
    out = os.path.join(HERE, "adjoint%d_oracle_%d.npz" % (n, steps))
    np.savez_compressed(out, steps=steps, h=1e-6, phi_target=target.astype(np.float32),
                        loss=float(((base - target) ** 2).sum()), grad_theta=g_theta,
                        phi0_index=idx, grad_phi0=g_phi, threads=oracle.num_threads(),
                        seconds=time.time() - t0)
    print(out, "loss=%.6e %.0fs" % (((base - target) ** 2).sum(), time.time() - t0))


if __name__ == "__main__":
    args = sys.argv[1:]
    sens_only = "--sens-only" in args
    for n in [a for a in args if a != "--sens-only"] or ["vortex2048"]:
        if n == "adjoint256":
            make_adjoint()
        else:
            make(n, sens_only)
