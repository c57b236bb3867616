"""bench.py's command-line contract on the CPU: more than one GPU is refused with a
message and a non-zero status before any GPU work starts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_committed_traffic_summaries_match_the_kernel_sources():
    """The HBM traffic that bench.py reports comes from committed counter summaries; each
    is tied to the kernel sources it was measured on, is current, and states traffic
    close to the algorithmic bytes it names."""
    sys.path.insert(0, ROOT)
    import bench
    main = bench.measured_traffic()
    assert main is not None, "profiles/phi_step_vortex2048_traffic.txt is stale"
    assert 1.0 <= main / (72 * 2048 * 2048) < 1.1
    for name, bytes_lu in (("f32", 144), ("f16", 112)):
        t = bench.measured_traffic(bench.RT_TRAFFIC_FILE, bench.RT_KERNEL_SRC,
                                   "hbm_bytes_per_launch_" + name)
        assert t is not None, "profiles/rt_step_rt256x1024_traffic.txt is stale"
        assert 1.0 <= t / (bytes_lu * 256 * 1024) < 1.1
