"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (no GPU).

* The FP64 oracle (``oracle/lbm_ch_oracle.c``, with OpenMP) is built with gcc's ASan and
  UBSan and driven through every function and mode on small odd-sized lattices
  (``tests/sanitize/oracle_driver.c``).
* The host side of the C ABI (``lbm_ch_api.cpp``: validation, layout, size queries,
  context handling up to HIP's "no device" error) is built with clang's ASan and UBSan
  and linked before the built library, so the driver's calls reach the sanitized copy
  (``tests/sanitize/abi_driver.c``); the kernel launchers come from the library.
* A planted out-of-bounds read shows that the flags really catch a fault.
Every sanitizer report aborts (-fno-sanitize-recover=all); leaks are reported too.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "lbm_ch_oracle.c"),
          "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    print(r.stdout)
    assert "0 failed checks" in r.stdout
    assert "Sanitizer" not in r.stderr


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_host_abi_under_asan_ubsan(tmp_path):
    import paper_1805_00007_amd as lbm
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("liblbm_ch.so is not built")
    inc = ["-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1805_00007_amd", "csrc"),
           "-I", os.path.join(ROCM, "include")]
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "abi_san")
    _run([CLANG + "++", "-std=c++17", *SAN, *inc, "-c",
          os.path.join(ROOT, "paper_1805_00007_amd", "csrc", "lbm_ch_api.cpp"), "-o", api])
    _run([CLANG, "-std=c11", *SAN, *inc, "-c", os.path.join(HERE, "abi_driver.c"), "-o", drv])
    _run([CLANG + "++", *SAN, drv, api, lbm.LIB_PATH, "-L", os.path.join(ROCM, "lib"),
          "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe])
    r = _run([exe], env=ENV)
    print(r.stdout)
    assert "abi driver: 0 failed checks" in r.stdout
    assert "Sanitizer" not in r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_planted_overflow_is_caught(tmp_path):
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "int main(int argc, char** argv) {\n"
                   "  double* a = malloc(8 * sizeof(double));\n"
                   "  double s = a[argc + 7];\n"  # one past the end
                   "  free(a);\n"
                   "  return s > 0;\n"
                   "}\n")
    exe = str(tmp_path / "planted")
    _run(["gcc", *SAN, str(src), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60, env=ENV)
    assert r.returncode != 0
    # whichever of the two sees it first reports it (UBSan's object-size check or ASan)
    assert "AddressSanitizer: heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr
