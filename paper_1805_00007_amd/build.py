"""Build the gfx950 shared library liblbm_ch.so in this package directory (hipcc)."""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm_ch.so")
SOURCES = [os.path.join(HERE, "csrc", "lbm_ch_step.hip"),
           os.path.join(HERE, "csrc", "lbm_ch_step16.hip"),
           os.path.join(HERE, "csrc", "lbm_ch_ns.hip"),
           os.path.join(HERE, "csrc", "lbm_ch_aux.hip"),
           os.path.join(HERE, "csrc", "lbm_ch_api.cpp")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         # no packed-FP32 instructions in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
# per-source code-generation options: the 16-bit step kernels fit their register budget
# only without machine-level loop-invariant code motion (see lbm_ch_step16.hip)
EXTRA = {"lbm_ch_step16.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link liblbm_ch.so (always recompiles)."""
    with tempfile.TemporaryDirectory() as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            extra = EXTRA.get(os.path.basename(src), [])
            procs.append(subprocess.Popen(["hipcc", *FLAGS, *extra, "-c", src, "-o", obj],
                                          stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                          text=True))
        errs = []
        for src, p in zip(SOURCES, procs):
            _, err = p.communicate()
            if p.returncode != 0:
                errs.append("%s:\n%s" % (src, err))
            elif verbose and err:
                print(err)
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
        tmp = LIB + ".tmp"
        r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
                            "-o", tmp], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
