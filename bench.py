#!/usr/bin/env python3
"""Throughput of the fused FP32 phase-field step on one MI355X.

Workload: 2048^2 periodic lattice, Model-II, tau_g = 1, M = 0.01, sigma = 0.01, W = 4,
a circle of radius 0.15 L at (L/2, 3L/4) in the time-reversing single vortex
(max |u| = 0.05, T = 80000 steps), velocity from separable 1-D tables (seeded
synthetic inputs shaped like the paper's deformation tests).

A step is one launch of the fused kernel (pull, phi, mu, F1 + F2, collision,
store) over the whole lattice.  Prints one JSON line:
  value        MLUPS = nx*ny*steps / time of the timed steps (inputs resident in HBM)
  roofline     algorithmic bytes (72 B per node update: 9 float32 populations read and
               9 written) / average kernel duration from HIP events, against the
               8 TB/s HBM peak; traffic = measured HBM bytes per launch from the committed
               rocprofv3 counter summary (null when the kernel source changed since)
  cpu_baseline the FP64 oracle on the host cores on a bounded number of steps
  accuracy     relative L2 of phi after 1000 steps against stored FP64 oracle samples
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS and % HBM peak (FP32 fused step, 2048^2) vs FP64 oracle accuracy; "
          "adjoint ms")
HBM_PEAK_GBS = 8000.0
BYTES_PER_LU = 72.0
# sources of the fused step kernel: a counter summary is used only while they are unchanged
KERNEL_SRC = (os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_step.hip"),
              os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_device.h"),
              os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_stencil.h"))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phi_step_vortex2048_traffic.txt")
# the same for the coupled Rayleigh-Taylor step kernel
RT_KERNEL_SRC = (os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_ns.hip"),
                 os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_device.h"),
                 os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_stencil.h"))
RT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rt_step_rt256x1024_traffic.txt")
GOLDEN = os.path.join(ROOT, "tests", "golden", "vortex2048_oracle_1000.npz")
ADJ_GOLDEN = os.path.join(ROOT, "tests", "golden", "adjoint256_oracle_2000.npz")


def kernel_sha(sources=KERNEL_SRC):
    h = hashlib.sha256()
    for path in sources:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, sources=KERNEL_SRC, key="hbm_bytes_per_launch"):
    """Bytes per launch from a committed counter summary, if the kernel is unchanged."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_sha(sources):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """CPU model name of the host (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_mlups(w, steps, threads=None):
    import numpy as np
    import oracle
    import workloads
    oracle.build(force=False)
    if threads is not None:
        oracle.set_num_threads(threads)
    p = oracle.Params(nx=w.nx, ny=w.ny, **w.phys)
    U, V = workloads.separable_field(w.velocity)
    s = oracle.State(p, w.phi0, U, V, w.velocity["tf"])
    t0 = time.perf_counter()
    s.run(steps)
    dt = time.perf_counter() - t0
    assert np.isfinite(s.g).all()
    return w.nx * w.ny * steps / dt / 1e6, dt, oracle.num_threads()


def cpu_baseline(steps):
    """The FP64 oracle on the host cores: the 2048^2 workload on a bounded number of steps
    with every thread (the reported value), the same with one thread, the 128^2
    translation (3200 steps, one period) in full, and the 512^2 vortex on a sample of
    its 20000 steps (time extrapolated to the full run)."""
    import oracle
    import workloads
    oracle.build(force=False)
    nthreads = oracle.num_threads()
    v, dt, cores = _oracle_mlups(workloads.metric2048(steps=steps), steps)
    out = {"value": round(v, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": "%d steps of the 2048x2048 workload (FP64, OpenMP over rows), %.1f s"
                     % (steps, dt),
           "cpu_model": cpu_model(), "host_threads": os.cpu_count()}
    one_steps = max(2, steps // 40)
    v1, dt1, _ = _oracle_mlups(workloads.metric2048(steps=one_steps), one_steps, threads=1)
    out["one_thread"] = {"value": round(v1, 3), "unit": "MLUPS",
                         "sample": "%d steps of the 2048x2048 workload, %.1f s" % (one_steps, dt1)}
    oracle.set_num_threads(nthreads)
    w1 = workloads.translation(128, steps=3200)
    v1, dt1, _ = _oracle_mlups(w1, 3200)
    out["translation128_full"] = {"value": round(v1, 3), "unit": "MLUPS", "steps": 3200,
                                  "seconds": round(dt1, 2)}
    n2 = 2000
    w2 = workloads.vortex(512, period=20000, steps=n2)
    v2, dt2, _ = _oracle_mlups(w2, n2)
    out["vortex512_sample"] = {"value": round(v2, 3), "unit": "MLUPS", "steps": n2,
                               "seconds": round(dt2, 2),
                               "full_run_20000_steps_s_extrapolated": round(dt2 * 20000 / n2, 1)}
    return out


def accuracy(lbm, w, torch):
    """phi after 1000 steps at stored oracle sample points (tests/golden)."""
    import numpy as np
    if not os.path.exists(GOLDEN):
        return None
    g = np.load(GOLDEN)
    s = lbm.solver_for(w)
    s.step(int(g["steps"]))
    d = s.diagnostics()
    phi = s.phi().double().cpu().numpy().ravel()
    idx = g["index"]
    ref = g["phi"]
    rel = float(np.sqrt(((phi[idx] - ref) ** 2).sum() / (ref ** 2).sum()))
    drift = abs(d["mass"] - float(g["mass0"])) / float(g["abs_mass0"])
    s.close()
    return {"steps": int(g["steps"]), "rel_l2_phi_sampled": rel, "samples": int(len(idx)),
            "max_abs_err": float(np.abs(phi[idx] - ref).max()), "mass_drift": drift}


def roofline(bytes_per_lu, nodes, us, kernel, profile, traffic=None):
    """Roofline sub-object of a leg: algorithmic bytes of one launch over its duration,
    against the 8 TB/s HBM peak; traffic = measured HBM bytes per launch, where a
    committed counter summary of the unchanged kernel holds them."""
    achieved = bytes_per_lu * nodes / (us * 1e-6) / 1e9
    return {"bound": "hbm", "bytes_per_lu": bytes_per_lu, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": kernel, "kernel_avg_us": round(us, 2),
            "profile": profile}


def storage_variant(lbm, torch, storage, steps):
    """Same workload with 16-bit population storage (20 B per node update instead of 36
    read and 36 written): throughput over at least 500 steps, and phi at the stored
    1000-step oracle samples."""
    import numpy as np
    import workloads
    steps = max(steps, 500)
    w = workloads.metric2048(steps=steps + 1100)
    s = lbm.solver_for(w, storage=storage)
    s.step(50)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tiles = s.tiles
    s.close()
    kernel = ("k_phi_pass (16-bit storage, single-pass tiles of 64 x %d)" % tiles[1]
              if tiles[0] == 0 else "k_phi_step (16-bit storage, %d x %d tiles)" % tiles)
    out = {"MLUPS": round(w.nx * w.ny / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
           "timed_steps": steps, "bytes_per_lu": 40, "tiles": list(tiles),
           "effective_GBps": round(w.nx * w.ny * 40 / (ms * 1e-3) / 1e9, 1),
           "roofline": roofline(40, w.nx * w.ny, ms * 1e3, kernel,
                                "profiles/phi_step_vortex2048_16bit_kernel_trace.md")}
    if os.path.exists(GOLDEN):
        g = np.load(GOLDEN)
        s = lbm.solver_for(workloads.metric2048(steps=1000), storage=storage)
        s.step(int(g["steps"]))
        d = s.diagnostics()
        phi = s.phi().double().cpu().numpy().ravel()
        s.close()
        ref = g["phi"]
        out["rel_l2_phi_sampled_1000"] = float(np.sqrt(((phi[g["index"]] - ref) ** 2).sum()
                                                       / (ref ** 2).sum()))
        out["mass_drift_1000"] = abs(d["mass"] - float(g["mass0"])) / float(g["abs_mass0"])
    return out


def adjoint_leg(lbm, torch, reps=3):
    """One forward plus backward pass of the 256^2, 2000-step interface-matching problem
    (16 stream-function coefficients, sqrt(N) checkpointing; each segment's recomputation
    beside the reverse steps of the next on a second stream, and for comparison one after
    the other, and with the whole trajectory stored), against the plain forward
    run of the same workload (one call of N plain launches; also its segments replayed
    from captured hipGraphs), and its gradients against stored FP64 central differences.
    Both run on the tile shape the autotuner picks for this lattice (tuned once, not
    timed)."""
    import numpy as np
    import workloads
    from paper_1805_00007_amd.adjoint import evolve
    if not os.path.exists(ADJ_GOLDEN):
        return None
    g = np.load(ADJ_GOLDEN)
    steps = int(g["steps"])
    case = workloads.adjoint_case(256, steps)
    dev = torch.device("cuda:0")
    target = torch.tensor(g["phi_target"], dtype=torch.float32, device=dev)
    basis = torch.tensor(case.basis, dtype=torch.float32, device=dev)
    U, V = case.field()

    probe = lbm.Solver(case.n, case.n, case.phi0, field=(U, V), device=dev, **case.phys)
    tiles, _ = probe.autotune(5)
    probe.close()

    seg = int(np.ceil(np.sqrt(steps)))

    def plain(graphs=False):
        # graphs: the forward pass's own launch pattern (segments of ceil(sqrt(N)) steps
        # replayed from captured hipGraphs, the captures included in the time)
        s = lbm.Solver(case.n, case.n, case.phi0, field=(U, V), device=dev, **case.phys)
        s.set_tiles(*tiles)
        s.set_graphs(graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if graphs:
            n = 0
            while n < steps:
                s.step(min(seg, steps - n))
                n += seg
        else:
            s.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        return dt

    def fwd_bwd(store=False, overlap=True):
        phi0 = torch.tensor(case.phi0, dtype=torch.float32, device=dev, requires_grad=True)
        theta = torch.tensor(case.theta, dtype=torch.float32, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uv = case.scale * torch.tensordot(theta, basis, dims=1)
        phi = evolve(phi0, uv[0], uv[1], steps, tiles=tiles, store_trajectory=store,
                     overlap=overlap, **case.phys)
        loss = ((phi - target) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, float(loss.detach()), theta.grad.double().cpu().numpy(), \
            phi0.grad.double().cpu().numpy()

    plain()
    plain(True)
    fwd_bwd()
    t_plain = min(plain() for _ in range(reps))
    t_plain_g = min(plain(True) for _ in range(reps))
    runs = [fwd_bwd() for _ in range(reps)]
    t_adj = min(r[0] for r in runs)
    fwd_bwd(True)
    stored = [fwd_bwd(True) for _ in range(reps)]
    t_store = min(r[0] for r in stored)
    same = bool(np.array_equal(stored[0][2], runs[0][2]) and np.array_equal(stored[0][3], runs[0][3]))
    fwd_bwd(overlap=False)
    serial = [fwd_bwd(overlap=False) for _ in range(reps)]
    t_serial = min(r[0] for r in serial)
    same_serial = bool(np.array_equal(serial[0][2], runs[0][2])
                       and np.array_equal(serial[0][3], runs[0][3]))
    # the reverse-step kernel alone: lbm_ch_adjoint over a stored trajectory of `nrev`
    # steps (one launch of k_adjoint per step), timed with events on its stream
    nrev = 200
    s = lbm.Solver(case.n, case.n, case.phi0, field=(U, V), device=dev, **case.phys)
    s.set_tiles(*tiles)
    traj = torch.empty((nrev, case.n, case.n), dtype=torch.float32, device=dev)
    s.record(nrev, traj)
    lam = torch.ones((case.n, case.n), dtype=torch.float32, device=dev)
    gu, gv = torch.zeros_like(lam), torch.zeros_like(lam)
    scratch = torch.empty(case.n * case.n, dtype=torch.float32, device=dev)
    s.adjoint(nrev, nrev, traj, lam, gu, gv, scratch)  # untimed
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.adjoint(nrev, nrev, traj, lam, gu, gv, scratch)
    e1.record(s.stream)
    torch.cuda.synchronize()
    rev_us = e0.elapsed_time(e1) * 1e3 / nrev
    s.close()
    _, loss, gt, gp = runs[0]
    ref_t, ref_p = g["grad_theta"], g["grad_phi0"]
    return {"workload": "adjoint256: 256^2, %d steps, 16 stream-function coefficients" % steps,
            "adjoint_ms": round(t_adj * 1e3, 2),
            "forward_ms_plain": round(t_plain * 1e3, 2),
            "ratio_to_plain_forward": round(t_adj / t_plain, 2),
            "forward_ms_plain_graphs": round(t_plain_g * 1e3, 2),
            "ratio_to_plain_forward_graphs": round(t_adj / t_plain_g, 2),
            "adjoint_ms_serial_backward": round(t_serial * 1e3, 2),
            "serial_backward_grads_bitwise_equal": same_serial,
            "adjoint_ms_stored_trajectory": round(t_store * 1e3, 2),
            "stored_trajectory_MiB": round(steps * case.n * case.n * 4 / 2 ** 20, 1),
            "stored_trajectory_grads_bitwise_equal": same,

            "checkpoints": -(-steps // (int(np.ceil(np.sqrt(steps))))),
            "tiles": {"tx": tiles[0], "ty": tiles[1]},
            "loss_rel_err": abs(loss - float(g["loss"])) / float(g["loss"]),
            "grad_theta_rel_err": float(np.linalg.norm(gt - ref_t) / np.linalg.norm(ref_t)),
            "grad_phi0_rel_err": float(np.linalg.norm(gp.ravel()[g["phi0_index"]] - ref_p)
                                       / np.linalg.norm(ref_p)),
            "reference": "FP64 oracle central differences, h = %g" % float(g["h"]),
            # one reverse step per launch: phi^n and lam^{n+1} read, lam^n written, the two
            # velocity gradients read and written: 28 B per node
            "reverse_step_us": round(rev_us, 2),
            "roofline": roofline(28, case.n * case.n, rev_us, "k_adjoint (one reverse step)",
                                 "profiles/adjoint_adjoint256_kernel_trace.md")}


def rt_leg(lbm, torch, steps=500, warm=50):
    """The coupled Rayleigh-Taylor step at its full 256x1024 size (walls in y, Atwood
    0.5, Re 3000): one launch of k_rt_step per step (f and g together).  Algorithmic
    bytes per node update: g 36 + 36 and f 36 + 36 = 144 B in float32; 16-bit g storage
    makes g 20 + 20, 112 B."""
    import workloads
    w = workloads.rayleigh_taylor_case(256, 1024, steps=steps + warm)
    out = {"workload": "rayleigh_taylor 256x1024 (coupled NS + phase field, walls)"}
    for name, st, bytes_lu in (("f32", 0, 144), ("f16", 1, 112)):
        s = lbm.solver_for(w, walls=1, storage=st)
        s.step(warm)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        d = s.diagnostics()
        tiles = s.tiles
        s.close()
        lu = w.nx * w.ny / (ms * 1e-3)
        out[name] = {"MLUPS": round(lu / 1e6, 1), "us_per_step": round(ms * 1e3, 2),
                     "bytes_per_lu": bytes_lu, "tile_rows": tiles[1],
                     "effective_GBps": round(lu * bytes_lu / 1e9, 1),
                     "nonfinite": int(d["nonfinite"]),
                     "roofline": roofline(bytes_lu, w.nx * w.ny, ms * 1e3,
                                          "k_rt_step (one launch per step)",
                                          "profiles/rt_step_rt256x1024_kernel_trace.md",
                                          measured_traffic(RT_TRAFFIC_FILE, RT_KERNEL_SRC,
                                                           "hbm_bytes_per_launch_" + name))}
    return out


def batch_leg(lbm, torch, steps=5000, plain_steps=200, check_steps=100):
    """64 lattices of uneven sizes (sides 64-512, seeded): the batched kernel with the
    autotuned schedule (persistent grid or one workgroup per tile) and tiles, `steps`
    steps captured in one hipGraph and launched once,
    against the plain form (one lbm_ch_step launch per lattice per step) on the same GPU;
    both give bitwise the same fields."""
    import numpy as np
    import workloads
    ws = workloads.batch_case(steps=steps)
    nodes = sum(w.nx * w.ny for w in ws)
    sol = [lbm.solver_for(w) for w in ws]
    ref = [lbm.solver_for(w) for w in ws]
    b = lbm.Batch(sol)
    tiles, tuned_us = b.autotune(5)
    persistent = b.persistent
    b.step(check_steps, graph=True)
    for s in ref:
        s.step(check_steps)
    same = all(np.array_equal(x.phi().cpu().numpy(), y.phi().cpu().numpy())
               for x, y in zip(sol, ref))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(plain_steps):
        for s in ref:
            s.step(1)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / plain_steps
    for s in ref:
        s.close()
    b.step(steps, graph=True)  # captures and instantiates the graph (untimed)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    t0 = time.perf_counter()
    b.step(steps, graph=True)
    e1.record(b.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_batch = e0.elapsed_time(e1) * 1e-3 / steps
    nonfinite = sum(s.diagnostics()["nonfinite"] for s in sol)
    b.close()
    for s in sol:
        s.close()
    return {"workload": "batch64: 64 lattices, sides %s, %d nodes, steady random stream "
                        "functions, Model-II, FP32" % (sorted({w.nx for w in ws}), nodes),
            "steps_in_one_graph_launch": steps,
            "batched_MLUPS": round(nodes / t_batch / 1e6, 1),
            "batched_us_per_step": round(t_batch * 1e6, 2),
            "graph_launch_wall_s": round(wall, 4),
            "plain_MLUPS": round(nodes / t_plain / 1e6, 1),
            "plain_us_per_step": round(t_plain * 1e6, 2),
            "speedup_vs_plain": round(t_plain / t_batch, 2),
            "autotuned_tiles": {"tx": tiles[0], "ty": tiles[1], "trial_us": round(tuned_us, 2),
                                "schedule": "persistent" if persistent else "tile per workgroup"},
            "bitwise_equal_to_plain_after_%d" % check_steps: bool(same),
            "nonfinite": int(nonfinite),
            "bytes_per_lu": 80,
            "roofline": roofline(80, nodes, t_batch * 1e6, "k_phi_batch (all 64 lattices)",
                                 "profiles/phi_batch_batch64_kernel_trace.md")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=160,
                    help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB x 10 (counter calibration)")
    ap.add_argument("--rt-only", action="store_true",
                    help="only run the Rayleigh-Taylor leg (--steps timed, --warmup untimed)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_probe_bytes_read_per_launch": src.numel() * 4,
                          "launches": 11, "copy_GBps_read_plus_write":
                          round(2 * src.numel() * 4 / (ms * 1e-3) / 1e9, 1)}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; the multi-GPU domain "
              "decomposition is a design, not a runnable path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_1805_00007_amd as lbm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.rt_only:
        print(json.dumps({"rayleigh_taylor": rt_leg(lbm, torch, steps=args.steps,
                                                    warm=args.warmup)}), flush=True)
        return
    w = workloads.metric2048(steps=args.steps + args.warmup)
    s = lbm.solver_for(w)
    stream = s.stream
    s.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: exactly `steps` steps, bracketed by synchronisation
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    s.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_ms = ev0.elapsed_time(ev1)

    # average duration of one launch of the fused kernel over the timed region: every
    # step of this workload is exactly one launch of k_phi_step on `stream`, so the
    # events around the region give the average launch duration (gaps between the
    # back-to-back launches included)
    k_ms = t_ms / args.steps
    # for reference: isolated launches, each bracketed by its own events
    nprobe = min(200, max(20, args.steps // 5))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nprobe)]
    for a, b in evs:
        a.record(stream)
        s.step(1)
        b.record(stream)
    torch.cuda.synchronize()
    iso_ms = sum(a.elapsed_time(b) for a, b in evs) / nprobe
    d = s.diagnostics()
    assert d["nonfinite"] == 0, "non-finite phi in the benchmark run"
    s.close()

    nodes = w.nx * w.ny
    mlups = nodes * args.steps / (t_ms * 1e-3) / 1e6
    algo = BYTES_PER_LU * nodes
    achieved = algo / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "model": "II", "tau_g": 1.0,
                   "velocity": "single vortex, separable tables", "boundary": "periodic",
                   "storage": "f32"},
        "effective_GBps": round(mlups * BYTES_PER_LU / 1e3, 1),
        "hbm_frac_effective": round(mlups * BYTES_PER_LU / 1e3 / HBM_PEAK_GBS, 4),
        "wall_s_timed": round(wall, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_phi_step",
                     "kernel_avg_us": round(k_ms * 1e3, 2),
                     "isolated_launch_us": round(iso_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": algo},
    }
    if not args.no_accuracy:
        out["accuracy"] = accuracy(lbm, workloads.metric2048(steps=1000), torch)
        out["storage_variants"] = {name: storage_variant(lbm, torch, st, args.steps)
                                   for name, st in (("f16", 1), ("bf16", 2))}
        out["adjoint"] = adjoint_leg(lbm, torch)
        out["rayleigh_taylor"] = rt_leg(lbm, torch)
        out["batched"] = batch_leg(lbm, torch)
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
