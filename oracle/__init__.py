"""FP64 CPU oracle for the lattice Boltzmann Cahn-Hilliard model of arXiv:1805.00007.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg
of ``bench.py`` import this package.  It wraps ``lbm_ch_oracle.c`` (plain C, double
precision, Sec. II of the paper step by step) through ctypes and shares no code
with the GPU library in ``paper_1805_00007_amd``.

Arrays are numpy float64, C-contiguous.  A field is ``(ny, nx)``; a population
array is ``(9, ny, nx)`` with direction order (0,0) (1,0) (0,1) (-1,0) (0,-1)
(1,1) (-1,1) (-1,-1) (1,-1).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_ch_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_ch_oracle.so")
# the same source in float32 arithmetic (sensitivity runs only, see State32)
_LIB32 = os.path.join(_HERE, "liblbm_ch_oracle_f32.so")

# Lattice of Sec. II.B, for the tests that reason about the method in k-space.
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over rows), and its float32 build.  Returns the
    path of the FP64 library."""
    for lib, extra in ((_LIB, []), (_LIB32, ["-DORC_REAL=float", "-fsingle-precision-constant"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
                   *extra, "-o", lib + ".tmp", _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(lib + ".tmp", lib)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("walls", ctypes.c_int),
                ("model", ctypes.c_int), ("ns", ctypes.c_int),
                ("tau_g", ctypes.c_double), ("mobility", ctypes.c_double),
                ("sigma", ctypes.c_double), ("width", ctypes.c_double),
                ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
                ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double),
                ("tau_f", ctypes.c_double), ("gravity", ctypes.c_double),
                ("accel_x", ctypes.c_double), ("f1_form", ctypes.c_int),
                ("round_f32", ctypes.c_int)]


class _Coeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("beta", "kappa", "eta", "K", "a", "b")]


@dataclasses.dataclass
class Params:
    """Physical and lattice parameters (lattice units, dx = dt = c = 1)."""
    nx: int
    ny: int
    walls: int = 0
    model: int = 2
    ns: int = 0
    tau_g: float = 1.0
    mobility: float = 0.01
    sigma: float = 0.01
    width: float = 4.0
    phi_a: float = 1.0
    phi_b: float = -1.0
    rho_a: float = 1.0
    rho_b: float = 0.5
    tau_f: float = 1.0
    gravity: float = 0.0
    accel_x: float = 0.0
    f1_form: int = 0  # 0: F1 = (phi/rho) F_s (grad p = 0); 1: F1 = phi Du/Dt of the prescribed u
    round_f32: int = 0  # 1: round what the GPU path holds in float32 (sensitivity runs)

    def c(self) -> _Params:
        return _Params(*[getattr(self, f.name) for f in dataclasses.fields(self)])


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        lib.orc_coeffs_from.argtypes = [P, ctypes.POINTER(_Coeffs)]
        lib.orc_equilibrium_g.argtypes = [ctypes.c_double] * 5 + [_D]
        lib.orc_source_g.argtypes = [ctypes.c_double] * 2 + [_D]
        lib.orc_equilibrium_f.argtypes = [ctypes.c_double] * 4 + [_D]
        lib.orc_source_f.argtypes = [ctypes.c_double] * 6 + [_D]
        lib.orc_grad.argtypes = [P, _D, ctypes.c_int, _D, _D]
        lib.orc_lap.argtypes = [P, _D, ctypes.c_int, _D]
        lib.orc_chemical_potential.argtypes = [P, _D, _D]
        lib.orc_init.argtypes = [P, _D, _D, _D, _D, _D]
        lib.orc_run.argtypes = [P, _D, _D, _D, _D, _D, ctypes.c_long, _D,
                                ctypes.POINTER(ctypes.c_int)]
        lib.orc_fields.argtypes = [P, _D, _D, _D, _D, ctypes.c_double] + [_D] * 5
        lib.orc_diag.argtypes = [P, _D, _D, _D]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def coeffs(p: Params) -> dict:
    c = _Coeffs()
    if _load().orc_coeffs_from(ctypes.byref(p.c()), ctypes.byref(c)) != 0:
        raise ValueError("invalid parameters (tau_g <= 1/2 or phi_a == phi_b)")
    return {n: getattr(c, n) for n, _ in _Coeffs._fields_}


def equilibrium_g(phi, mu, ux, uy, eta):
    out = np.zeros(9)
    _load().orc_equilibrium_g(phi, mu, ux, uy, eta, _ptr(out))
    return out


def source_g(fx, fy):
    out = np.zeros(9)
    _load().orc_source_g(fx, fy, _ptr(out))
    return out


def equilibrium_f(p, rho, ux, uy):
    out = np.zeros(9)
    _load().orc_equilibrium_f(p, rho, ux, uy, _ptr(out))
    return out


def source_f(fx, fy, ux, uy, drx, dry):
    out = np.zeros(9)
    _load().orc_source_f(fx, fy, ux, uy, drx, dry, _ptr(out))
    return out


def grad(p: Params, psi, parity=1):
    psi = _f64(psi)
    gx, gy = np.zeros_like(psi), np.zeros_like(psi)
    _load().orc_grad(ctypes.byref(p.c()), _ptr(psi), parity, _ptr(gx), _ptr(gy))
    return gx, gy


def lap(p: Params, psi, parity=1):
    psi = _f64(psi)
    out = np.zeros_like(psi)
    _load().orc_lap(ctypes.byref(p.c()), _ptr(psi), parity, _ptr(out))
    return out


def chemical_potential(p: Params, phi):
    phi = _f64(phi)
    out = np.zeros_like(phi)
    _load().orc_chemical_potential(ctypes.byref(p.c()), _ptr(phi), _ptr(out))
    return out


class State:
    """Populations g (and f for the coupled Navier-Stokes case) plus the step count."""

    def __init__(self, p: Params, phi0, ux=None, uy=None, tf=None):
        """Initialise to equilibrium.  ``ux``/``uy`` are the base velocity field, ``tf``
        an optional per-step factor (velocity at step n is ``tf[n] * (ux, uy)``)."""
        self.p = p
        self.ux, self.uy = _f64(ux), _f64(uy)
        self.tf = _f64(tf)
        self.n = 0
        phi0 = _f64(phi0)
        assert phi0.shape == (p.ny, p.nx)
        self.g = np.zeros((9, p.ny, p.nx))
        self.f = np.zeros((9, p.ny, p.nx)) if p.ns else None
        f0 = 1.0 if self.tf is None else float(self.tf[0])
        u0 = None if self.ux is None else f0 * self.ux
        v0 = None if self.uy is None else f0 * self.uy
        _load().orc_init(ctypes.byref(p.c()), _ptr(phi0), _ptr(u0), _ptr(v0), _ptr(self.g),
                         _ptr(self.f))
        # model 3: F1 and grad mu of the previous step (Eq. F2-1 time derivatives)
        self.hist = np.zeros((4, p.ny, p.nx))
        self.hist_valid = ctypes.c_int(0)

    def run(self, nsteps: int) -> "State":
        tf = None
        if self.tf is not None:
            assert self.n + nsteps <= len(self.tf), "time-factor table too short"
            tf = np.ascontiguousarray(self.tf[self.n:self.n + nsteps])
        _load().orc_run(ctypes.byref(self.p.c()), _ptr(self.g), _ptr(self.f), _ptr(self.ux),
                        _ptr(self.uy), _ptr(tf), int(nsteps), _ptr(self.hist),
                        ctypes.byref(self.hist_valid))
        self.n += nsteps
        return self

    def fields(self):
        """(phi, mu, u, v, p) at the current step."""
        p = self.p
        outs = [np.zeros((p.ny, p.nx)) for _ in range(5)]
        tfac = 1.0
        if self.tf is not None:
            tfac = float(self.tf[self.n]) if self.n < len(self.tf) else float(self.tf[-1])
        _load().orc_fields(ctypes.byref(p.c()), _ptr(self.g), _ptr(self.f), _ptr(self.ux),
                           _ptr(self.uy), tfac, *[_ptr(o) for o in outs])
        return tuple(outs)

    @property
    def phi(self):
        return self.g.sum(axis=0)


def diag(p: Params, phi, phi_ref=None):
    """FP64 diagnostics: dict of mass, abs_mass, energy, err2, ref2, max, min, nonfinite."""
    phi = _f64(phi)
    ref = _f64(phi_ref)
    out = np.zeros(8)
    _load().orc_diag(ctypes.byref(p.c()), _ptr(phi), _ptr(ref), _ptr(out))
    keys = ("mass", "abs_mass", "energy", "err2", "ref2", "max", "min", "nonfinite")
    return dict(zip(keys, out.tolist()))


def rel_l2(phi, phi_ref):
    """Relative L2 error of Eq. err."""
    phi, phi_ref = np.asarray(phi, np.float64), np.asarray(phi_ref, np.float64)
    return float(np.sqrt(((phi - phi_ref) ** 2).sum() / (phi_ref ** 2).sum()))


# --- the float32 build (sensitivity runs) ----------------------------------------------

class _Params32(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float if t is ctypes.c_double else t) for n, t in _Params._fields_]


_lib32 = None
_F = ctypes.POINTER(ctypes.c_float)


def _load32():
    global _lib32
    if _lib32 is None:
        if not os.path.exists(_LIB32):
            build(force=False)
        lib = ctypes.CDLL(_LIB32)
        P = ctypes.POINTER(_Params32)
        lib.orc_init.argtypes = [P, _F, _F, _F, _F, _F]
        lib.orc_run.argtypes = [P, _F, _F, _F, _F, _F, ctypes.c_long, _F, ctypes.POINTER(ctypes.c_int)]
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib32 = lib
    return _lib32


def _p32(a):
    if a is None:
        return None
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(_F)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


class State32:
    """The oracle's code compiled with float32 arithmetic (``orc_real = float``): the same
    method, steps and order as ``State``, every operation rounded to float32.  Not a
    reference: its distance from the FP64 ``State`` measures how far float32 evaluation
    of the method drifts over a run, which sets the tolerance of long unstable runs.
    Populations ``g`` (and ``f``) are float32 arrays; ``phi`` sums them in FP64."""

    def __init__(self, p: Params, phi0, ux=None, uy=None, tf=None):
        assert p.model != 3, "model 3 history is not wrapped for the float32 build"
        self.p = p
        self.c32 = _Params32(*[getattr(p, f.name) for f in dataclasses.fields(p)])
        self.ux, self.uy, self.tf = _f32(ux), _f32(uy), _f32(tf)
        self.n = 0
        phi0 = _f32(phi0)
        self.g = np.zeros((9, p.ny, p.nx), dtype=np.float32)
        self.f = np.zeros((9, p.ny, p.nx), dtype=np.float32) if p.ns else None
        f0 = 1.0 if self.tf is None else float(self.tf[0])
        u0 = None if self.ux is None else _f32(f0 * self.ux)
        v0 = None if self.uy is None else _f32(f0 * self.uy)
        _load32().orc_init(ctypes.byref(self.c32), _p32(phi0), _p32(u0), _p32(v0),
                           _p32(self.g), _p32(self.f))

    def run(self, nsteps: int) -> "State32":
        tf = None
        if self.tf is not None:
            assert self.n + nsteps <= len(self.tf), "time-factor table too short"
            tf = np.ascontiguousarray(self.tf[self.n:self.n + nsteps])
        _load32().orc_run(ctypes.byref(self.c32), _p32(self.g), _p32(self.f), _p32(self.ux),
                          _p32(self.uy), _p32(tf), int(nsteps), None, None)
        self.n += nsteps
        return self

    @property
    def phi(self):
        return self.g.astype(np.float64).sum(axis=0)
