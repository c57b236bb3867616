"""Write stored FP64 oracle samples for workloads too large to run in a test.

Calls only ``oracle`` and ``workloads``.  For each case it runs the oracle for the
stated number of steps and stores phi at 4096 seeded sample nodes, the full-field
relative L2 of phi against the initial field (Eq. err), the initial mass sums and
the final extrema.

    python tests/golden/make_golden.py vortex2048     # 2048^2, 1000 steps
    python tests/golden/make_golden.py vortex512      # 512^2, one period T = 20000
    python tests/golden/make_golden.py rt256          # 256x1024 Rayleigh-Taylor, 1000 steps
"""
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
}


def make(name):
    build, steps, walls = CASES[name]
    w = build()
    p = oracle.Params(nx=w.nx, ny=w.ny, walls=walls, ns=1 if "tau_f" in w.phys else 0,
                      **w.phys)
    if w.velocity is not None:
        U, V = workloads.separable_field(w.velocity)
        s = oracle.State(p, w.phi0, U, V, w.velocity["tf"])
    else:
        s = oracle.State(p, w.phi0)
    d0 = oracle.diag(p, s.phi)
    t0 = time.time()
    s.run(steps)
    phi = s.phi
    d = oracle.diag(p, phi, w.phi0)
    rng = np.random.default_rng(20240601)
    idx = np.sort(rng.choice(w.nx * w.ny, size=4096, replace=False))
    out = os.path.join(HERE, "%s_oracle_%d.npz" % (name, steps))
    np.savez_compressed(out, steps=steps, index=idx, phi=phi.ravel()[idx],
                        mass0=d0["mass"], abs_mass0=d0["abs_mass"], mass=d["mass"],
                        e_phi=np.sqrt(d["err2"] / d["ref2"]), max=d["max"], min=d["min"],
                        threads=oracle.num_threads(), seconds=time.time() - t0)
    print(out, "E_phi=%.4e max=%.4f min=%.4f %.0fs" % (
        np.sqrt(d["err2"] / d["ref2"]), d["max"], d["min"], time.time() - t0))


if __name__ == "__main__":
    for n in sys.argv[1:] or ["vortex2048"]:
        make(n)
