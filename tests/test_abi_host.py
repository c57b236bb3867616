"""Host-side checks of the C ABI (no GPU): the library loads, exports every function
include/lbm_ch.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1805_00007_amd as lbm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "lbm_ch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_ch_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 13
    L = ctypes.CDLL(lbm.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbm.EXPORTS)


def _params(**kw):
    return lbm.make_params(64, 48, **kw)


@pytest.mark.parametrize("bad", [dict(tau_g=0.5), dict(tau_g=0.2), dict(model=4), dict(model=0),
                                 dict(rho_a=0.0), dict(rho_b=-1.0), dict(phi_a=-1.0),
                                 dict(width=0.0), dict(walls=2), dict(velocity_mode=7),
                                 dict(ns=True, tau_f=0.5), dict(sigma=float("nan"))])
def test_invalid_params_rejected(bad):
    p = _params(**bad)
    assert lbm.lib().lbm_ch_workspace_bytes(ctypes.byref(p)) == 0
    ctx = ctypes.c_void_p()
    st = lbm.lib().lbm_ch_init(ctypes.byref(ctx), ctypes.byref(p), None,
                               ctypes.c_void_p(1 << 20), 1 << 40, ctypes.c_void_p(1 << 20), None)
    assert st == lbm.EINVAL and not ctx.value


def test_largest_lattice_accepted():
    # float32 populations of one buffer must stay below 2^31 bytes (9 x 4 B per node)
    assert lbm.lib().lbm_ch_workspace_bytes(ctypes.byref(lbm.make_params(7680, 7760))) > 0
    assert lbm.lib().lbm_ch_workspace_bytes(ctypes.byref(lbm.make_params(7680, 7776))) == 0


def test_sizes_rejected():
    for nx, ny in [(3, 64), (64, 3), (40000, 40000)]:
        p = lbm.make_params(nx, ny)
        assert lbm.lib().lbm_ch_workspace_bytes(ctypes.byref(p)) == 0


def test_workspace_and_alignment_checks():
    L = lbm.lib()
    p = _params()
    need = L.lbm_ch_workspace_bytes(ctypes.byref(p))
    assert need >= 2 * 9 * 64 * 48 * 4
    pns = _params(ns=True, tau_f=0.8)
    assert L.lbm_ch_workspace_bytes(ctypes.byref(pns)) >= 2 * need - 4 * 64 * 48 * 8
    ctx = ctypes.c_void_p()
    vel = lbm.Velocity()
    args = lambda ws, nb, phi: L.lbm_ch_init(ctypes.byref(ctx), ctypes.byref(p),
                                             ctypes.byref(vel), ctypes.c_void_p(ws), nb,
                                             ctypes.c_void_p(phi), None)
    assert args(0, need, 4096) == lbm.EINVAL                 # no workspace
    assert args(4096 + 64, need, 4096) == lbm.EINVAL         # workspace not 256-aligned
    assert args(4096, need - 1, 4096) == lbm.EINVAL          # workspace too small
    assert args(4096, need, 0) == lbm.EINVAL                 # no phi0
    assert args(4096, need, 4098) == lbm.EINVAL              # phi0 not 4-aligned
    # separable mode without tables
    p.velocity_mode = lbm.VEL_SEPARABLE
    assert args(4096, need, 4096) == lbm.EINVAL
    # a storage mode outside LBM_CH_STORE_*
    p.velocity_mode = lbm.VEL_NONE
    p.storage = 9
    assert L.lbm_ch_workspace_bytes(ctypes.byref(p)) == 0
    assert args(4096, need, 4096) == lbm.EINVAL


def test_storage_modes_shrink_the_workspace():
    L = lbm.lib()
    sizes = {}
    for st in (lbm.STORE_F32, lbm.STORE_F16, lbm.STORE_BF16):
        p = lbm.make_params(256, 256, storage=st)
        sizes[st] = L.lbm_ch_workspace_bytes(ctypes.byref(p))
    # two population buffers: 36 B per node in float32, 20 B per node in 16-bit modes
    assert sizes[lbm.STORE_F32] - sizes[lbm.STORE_F16] == 2 * 16 * 256 * 256
    assert sizes[lbm.STORE_F16] == sizes[lbm.STORE_BF16]


def test_context_calls_reject_null_and_strerror():
    L = lbm.lib()
    assert L.lbm_ch_step(None, 1, None) == lbm.ESTATE
    assert L.lbm_ch_moments(None, None, None, None, None, None, None) == lbm.ESTATE
    assert L.lbm_ch_diagnostics(None, None, None, None) == lbm.ESTATE
    assert L.lbm_ch_step_count(None) == -1
    assert L.lbm_ch_record(None, 1, None, None) == lbm.ESTATE
    assert L.lbm_ch_set_graphs(None, 1) == lbm.ESTATE
    assert L.lbm_ch_adjoint(None, 1, 1, None, None, None, None, None, 0, None) == lbm.ESTATE
    assert L.lbm_ch_destroy(None) == lbm.OK
    assert L.lbm_ch_batch_step(None, 1, 0, None) == lbm.ESTATE
    assert L.lbm_ch_batch_autotune(None, None, 0, 1, None, None) == lbm.ESTATE
    assert L.lbm_ch_batch_state_bytes(None) == 0
    assert L.lbm_ch_batch_set_schedule(None, 1) == lbm.ESTATE
    assert L.lbm_ch_batch_get_schedule(None) == lbm.ESTATE
    assert L.lbm_ch_batch_destroy(None) == lbm.OK
    b = ctypes.c_void_p()
    assert L.lbm_ch_batch_create(ctypes.byref(b), None, 0, None, 0) == lbm.EINVAL
    assert L.lbm_ch_batch_workspace_bytes(0) == 0
    assert L.lbm_ch_batch_workspace_bytes(64) > 0
    for st in (lbm.OK, lbm.EINVAL, lbm.EUNSUPPORTED, lbm.EHIP, lbm.ENONFINITE, lbm.ESTATE):
        assert L.lbm_ch_strerror(st)
    assert L.lbm_ch_strerror(12345) == b"unknown status"


def test_adjoint_scratch_size():
    L = lbm.lib()
    p = lbm.make_params(96, 40)
    assert L.lbm_ch_adjoint_scratch_bytes(ctypes.byref(p)) == 96 * 40 * 4
    p.tau_g = 0.4
    assert L.lbm_ch_adjoint_scratch_bytes(ctypes.byref(p)) == 0


def test_model3_workspace_holds_the_history():
    L = lbm.lib()
    a = L.lbm_ch_workspace_bytes(ctypes.byref(lbm.make_params(256, 256, model=2)))
    b = L.lbm_ch_workspace_bytes(ctypes.byref(lbm.make_params(256, 256, model=3)))
    assert b - a == 2 * 4 * 256 * 256


def test_missing_library_fails_loudly(tmp_path):
    """With no built library every call into the package raises: there is no fallback.
    The package is copied without its built library into a temporary directory."""
    import shutil
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    shutil.copytree(os.path.join(root, "paper_1805_00007_amd"),
                    str(tmp_path / "paper_1805_00007_amd"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    code = ("import paper_1805_00007_amd as lbm\n"
            "try:\n"
            "    lbm.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "raised: liblbm_ch.so is not built" in r.stdout


@pytest.mark.parametrize("n,storage,expect", [
    (2048, 0, (512, 8)), (2048, 1, (0, 16)), (2048, 2, (0, 16)), (3072, 0, (512, 8)),
    (4096, 0, (512, 16)), (4096, 1, (0, 16)), (7680, 0, (512, 16)),
    (128, 0, (0, 4)), (256, 0, (0, 4)), (512, 0, (0, 16)), (1536, 0, (0, 16)), (8, 0, (0, 4)),
    (256, 1, (0, 4)), (512, 1, (0, 8)), (1024, 2, (0, 8))])
def test_default_tiles_rule(n, storage, expect):
    """The default tile rule (include/lbm_ch.h) on the host, without a device: the
    shapes the size sweeps picked for square lattices (periodic, tau_g = 1, separable
    velocity, Model-II: single-pass tiles below 2048^2 with float32 storage, at every
    size with 16-bit storage)."""
    assert lbm.default_tiles(lbm.make_params(n, n, storage=storage)) == expect


@pytest.mark.parametrize("n,expect", [
    (128, (128, 1)), (200, (64, 1)), (256, (256, 1)), (512, (512, 2)), (768, (256, 4)),
    (1024, (512, 8)), (1280, (256, 8)), (1536, (256, 16))])
def test_default_marching_tiles_rule(n, expect):
    """Where single-pass tiles do not serve (here tau_g != 1) the marching tiles' rule."""
    assert lbm.default_tiles(lbm.make_params(n, n, tau_g=0.8)) == expect


@pytest.mark.parametrize("n,storage,expect", [(2048, 1, (512, 16)), (4096, 1, (512, 8)),
                                              (3072, 2, (512, 8))])
def test_default_marching_tiles_rule_16bit(n, storage, expect):
    """16-bit storage where single-pass tiles do not serve (walls): the marching rule."""
    assert lbm.default_tiles(lbm.make_params(n, n, storage=storage, walls=1)) == expect


def test_default_tiles_invariants():
    """Over many lattice shapes: a valid shape, ty within the lattice, no strip wider
    than needed, and the coupled step's 64 x 16 (clipped to ny)."""
    sizes = [4, 7, 33, 64, 65, 100, 130, 200, 257, 384, 600, 1000, 1500, 2047, 2048, 2500,
             4100, 7680]
    for nx in sizes:
        for ny in sizes:
            if lbm.workspace_bytes(lbm.make_params(nx, ny)) == 0:
                continue
            for storage in (0, 1, 2):
                for walls in (0, 1):
                    tx, ty = lbm.default_tiles(lbm.make_params(nx, ny, storage=storage,
                                                               walls=walls))
                    if tx == 0:  # single pass: periodic; float32 below 2048^2
                        assert walls == 0 and (storage != 0 or nx * ny < 4 << 20)
                        assert ty in (4, 8, 16), (nx, ny, ty)
                        continue
                    assert tx in (64, 128, 256, 512) and 1 <= ty <= min(ny, 32), (nx, ny, tx, ty)
                    assert tx == 64 or tx <= nx, (nx, ny, tx)
            tx, ty = lbm.default_tiles(lbm.make_params(nx, ny, walls=1, ns=True,
                                                       gravity=1e-6))
            assert (tx, ty) == (64, min(16, ny)), (nx, ny, tx, ty)


def test_default_tiles_rejects_invalid():
    L = lbm.lib()
    tx, ty = ctypes.c_int32(), ctypes.c_int32()
    bad = lbm.make_params(64, 48, tau_g=0.5)
    assert L.lbm_ch_default_tiles(ctypes.byref(bad), ctypes.byref(tx), ctypes.byref(ty)) \
        == lbm.EINVAL
    good = lbm.make_params(64, 48)
    assert L.lbm_ch_default_tiles(ctypes.byref(good), None, ctypes.byref(ty)) == lbm.EINVAL
