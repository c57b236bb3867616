"""MI355X (gfx950) lattice Boltzmann solver for the Cahn-Hilliard equation of
Zhang, Guo & Liang, arXiv:1805.00007.

A thin ctypes binding of the C ABI in ``include/lbm_ch.h`` (same call names).  Every
step of the method runs in the HIP kernels of ``liblbm_ch.so``; this module only
marshals arguments.  PyTorch provides device memory (the workspace and the caller's
arrays are CUDA tensors) and the stream (the current torch stream).  Importing the
module does not need a GPU; calls that reach the library raise if the built library
is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_ch.so")

# Status codes and modes (include/lbm_ch.h).
OK, EINVAL, EUNSUPPORTED, EHIP, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5
VEL_NONE, VEL_SEPARABLE, VEL_FIELD, VEL_NS = 0, 1, 2, 3
STORE_F32, STORE_F16, STORE_BF16 = 0, 1, 2

# Every symbol include/lbm_ch.h declares.
EXPORTS = ("lbm_ch_workspace_bytes", "lbm_ch_init", "lbm_ch_step", "lbm_ch_moments",
           "lbm_ch_diagnostics", "lbm_ch_check_finite", "lbm_ch_step_count",
           "lbm_ch_state_bytes", "lbm_ch_save_state", "lbm_ch_load_state",
           "lbm_ch_set_tiles", "lbm_ch_get_tiles", "lbm_ch_default_tiles", "lbm_ch_set_graphs",
           "lbm_ch_autotune",
           "lbm_ch_adjoint_scratch_bytes", "lbm_ch_record", "lbm_ch_adjoint",
           "lbm_ch_adjoint_static",
           "lbm_ch_batch_workspace_bytes", "lbm_ch_batch_create", "lbm_ch_batch_set_tiles",
           "lbm_ch_batch_get_tiles", "lbm_ch_batch_set_schedule", "lbm_ch_batch_get_schedule",
           "lbm_ch_batch_step", "lbm_ch_batch_state_bytes",
           "lbm_ch_batch_autotune", "lbm_ch_batch_destroy", "lbm_ch_destroy",
           "lbm_ch_strerror", "lbm_ch_last_hip_error")


class LbmChError(RuntimeError):
    def __init__(self, status, call):
        self.status = status
        msg = lib().lbm_ch_strerror(status).decode()
        if status == EHIP:
            msg += " (hipError %d)" % lib().lbm_ch_last_hip_error()
        super().__init__("%s: %s (%d)" % (call, msg, status))


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls", ctypes.c_int32),
                ("model", ctypes.c_int32), ("velocity_mode", ctypes.c_int32),
                ("storage", ctypes.c_int32),
                ("tau_g", ctypes.c_double), ("mobility", ctypes.c_double),
                ("sigma", ctypes.c_double), ("width", ctypes.c_double),
                ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
                ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double),
                ("tau_f", ctypes.c_double), ("gravity", ctypes.c_double),
                ("accel_x", ctypes.c_double)]


class Velocity(ctypes.Structure):
    _fields_ = [("ax", ctypes.c_void_p), ("ay", ctypes.c_void_p), ("bx", ctypes.c_void_p),
                ("by", ctypes.c_void_p), ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p),
                ("time_factor", ctypes.POINTER(ctypes.c_double)),
                ("n_time_factor", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm_ch.so is not built: run paper_1805_00007_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        PP = ctypes.POINTER(Params)
        L.lbm_ch_workspace_bytes.argtypes = [PP]
        L.lbm_ch_workspace_bytes.restype = ctypes.c_size_t
        L.lbm_ch_default_tiles.argtypes = [PP, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]
        L.lbm_ch_init.argtypes = [ctypes.POINTER(vp), PP, ctypes.POINTER(Velocity), vp,
                                  ctypes.c_size_t, vp, vp]
        L.lbm_ch_step.argtypes = [vp, i64, vp]
        L.lbm_ch_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.lbm_ch_diagnostics.argtypes = [vp, vp, vp, vp]
        L.lbm_ch_check_finite.argtypes = [vp, vp]
        L.lbm_ch_step_count.argtypes = [vp]
        L.lbm_ch_step_count.restype = i64
        L.lbm_ch_state_bytes.argtypes = [vp]
        L.lbm_ch_state_bytes.restype = ctypes.c_size_t
        L.lbm_ch_save_state.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.lbm_ch_load_state.argtypes = [vp, vp, ctypes.c_size_t, i64, vp]
        L.lbm_ch_set_tiles.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.lbm_ch_set_graphs.argtypes = [vp, ctypes.c_int32]
        L.lbm_ch_get_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
        L.lbm_ch_autotune.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp,
                                      ctypes.POINTER(ctypes.c_float)]
        L.lbm_ch_adjoint_scratch_bytes.argtypes = [PP]
        L.lbm_ch_adjoint_scratch_bytes.restype = ctypes.c_size_t
        L.lbm_ch_record.argtypes = [vp, i64, vp, vp]
        L.lbm_ch_adjoint.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.lbm_ch_adjoint_static.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp]
        L.lbm_ch_batch_workspace_bytes.argtypes = [ctypes.c_int32]
        L.lbm_ch_batch_workspace_bytes.restype = ctypes.c_size_t
        L.lbm_ch_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32,
                                          vp, ctypes.c_size_t]
        L.lbm_ch_batch_set_tiles.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.lbm_ch_batch_get_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32)]
        L.lbm_ch_batch_set_schedule.argtypes = [vp, ctypes.c_int32]
        L.lbm_ch_batch_get_schedule.argtypes = [vp]
        L.lbm_ch_batch_step.argtypes = [vp, i64, ctypes.c_int32, vp]
        L.lbm_ch_batch_state_bytes.argtypes = [vp]
        L.lbm_ch_batch_state_bytes.restype = ctypes.c_size_t
        L.lbm_ch_batch_autotune.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp,
                                            ctypes.POINTER(ctypes.c_float)]
        L.lbm_ch_batch_destroy.argtypes = [vp]
        L.lbm_ch_destroy.argtypes = [vp]
        L.lbm_ch_strerror.argtypes = [i32]
        L.lbm_ch_strerror.restype = ctypes.c_char_p
        L.lbm_ch_last_hip_error.restype = i32
        for name in EXPORTS:
            assert hasattr(L, name), name
        _lib = L
    return _lib


def _check(status, call):
    if status != OK:
        raise LbmChError(status, call)


def make_params(nx, ny, *, walls=0, model=2, velocity_mode=VEL_SEPARABLE, storage=STORE_F32,
                tau_g=1.0, mobility=0.01, sigma=0.01, width=4.0, phi_a=1.0, phi_b=-1.0,
                rho_a=1.0, rho_b=0.5, tau_f=1.0, gravity=0.0, accel_x=0.0, ns=None):
    if ns:
        velocity_mode = VEL_NS
    return Params(nx, ny, walls, model, velocity_mode, storage, tau_g, mobility, sigma, width,
                  phi_a, phi_b, rho_a, rho_b, tau_f, gravity, accel_x)


def workspace_bytes(params: Params) -> int:
    return lib().lbm_ch_workspace_bytes(ctypes.byref(params))


def default_tiles(params: Params):
    """The tile shape (tx, ty) lbm_ch_init would choose for these parameters."""
    tx, ty = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbm_ch_default_tiles(ctypes.byref(params), ctypes.byref(tx), ctypes.byref(ty)),
           "lbm_ch_default_tiles")
    return tx.value, ty.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _device_f32(torch, a, device):
    """A contiguous float32 copy (or view) of an array or tensor on the device."""
    if isinstance(a, torch.Tensor):
        return a.detach().to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.asarray(a), dtype=torch.float32, device=device).contiguous()


class Solver:
    """One lattice: ``Solver(nx, ny, phi0, velocity=..., **params)``.

    ``phi0``: (ny, nx) array or tensor.  ``velocity``: a dict of separable tables
    ``ax, ay, bx, by`` (and ``tf``), or ``field=(U, V)`` (with optional ``tf``), or
    ``ns=True`` for the coupled Navier-Stokes velocity (optional ``u0=(U, V)``).
    Keyword parameters are those of ``lbm_ch_params``.
    """

    def __init__(self, nx, ny, phi0, velocity=None, field=None, tf=None, u0=None,
                 device="cuda", stream=None, **kw):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        L = lib()
        if field is not None:
            mode = VEL_FIELD
        elif kw.get("ns"):
            mode = VEL_NS
        elif velocity is not None:
            mode = VEL_SEPARABLE
        else:
            mode = VEL_NONE
        kw.pop("ns", None)
        self.params = make_params(nx, ny, velocity_mode=mode, **kw)
        nbytes = L.lbm_ch_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise LbmChError(EINVAL, "lbm_ch_workspace_bytes")
        f32 = dict(dtype=torch.float32, device=self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.nx, self.ny = nx, ny
        self._keep = []
        vel = Velocity()
        if mode == VEL_SEPARABLE:
            tabs = [torch.as_tensor(np.asarray(velocity[k]), **f32).contiguous()
                    for k in ("ax", "ay", "bx", "by")]
            self._keep += tabs
            vel.ax, vel.ay, vel.bx, vel.by = [t.data_ptr() for t in tabs]
            if tf is None:
                tf = velocity.get("tf")
        elif mode == VEL_FIELD:
            U, V = [_device_f32(torch, a, self.device) for a in field]
            self._keep += [U, V]
            vel.ux, vel.uy = U.data_ptr(), V.data_ptr()
        elif mode == VEL_NS and u0 is not None:
            U, V = [_device_f32(torch, a, self.device) for a in u0]
            self._keep += [U, V]
            vel.ux, vel.uy = U.data_ptr(), V.data_ptr()
        tfa = None
        if tf is not None:
            tfa = np.ascontiguousarray(tf, dtype=np.float64)
            vel.time_factor = tfa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            vel.n_time_factor = len(tfa)
        phi0 = _device_f32(torch, phi0, self.device)
        assert phi0.shape == (ny, nx)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _check(L.lbm_ch_init(ctypes.byref(ctx), ctypes.byref(self.params), ctypes.byref(vel),
                             ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                             ctypes.c_void_p(phi0.data_ptr()), self._s()), "lbm_ch_init")
        self._phi0 = phi0  # read by the enqueued init; kept until the stream passes it
        self.ctx = ctx

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def step(self, n=1):
        _check(lib().lbm_ch_step(self.ctx, int(n), self._s()), "lbm_ch_step")
        return self

    @property
    def step_count(self):
        return lib().lbm_ch_step_count(self.ctx)

    def moments(self, which=("phi", "mu", "u", "v", "p")):
        t = self.torch
        out = {k: t.empty((self.ny, self.nx), dtype=t.float32, device=self.device)
               for k in which}
        _check(lib().lbm_ch_moments(self.ctx, _ptr(out.get("phi")), _ptr(out.get("mu")),
                                    _ptr(out.get("u")), _ptr(out.get("v")), _ptr(out.get("p")),
                                    self._s()), "lbm_ch_moments")
        return out

    def phi(self):
        return self.moments(("phi",))["phi"]

    def diagnostics(self, phi_ref=None):
        t = self.torch
        out = t.empty(8, dtype=t.float64, device=self.device)
        ref = None
        if phi_ref is not None:
            ref = t.as_tensor(phi_ref, dtype=t.float32, device=self.device).contiguous()
        _check(lib().lbm_ch_diagnostics(self.ctx, _ptr(ref), _ptr(out), self._s()),
               "lbm_ch_diagnostics")
        self.stream.synchronize()
        v = out.cpu().numpy()
        keys = ("mass", "abs_mass", "energy", "err2", "ref2", "max", "min", "nonfinite")
        return dict(zip(keys, v.tolist()))

    def check_finite(self):
        return lib().lbm_ch_check_finite(self.ctx, self._s())

    def save_state(self):
        t = self.torch
        n = lib().lbm_ch_state_bytes(self.ctx)
        buf = t.empty(n, dtype=t.uint8, device=self.device)
        _check(lib().lbm_ch_save_state(self.ctx, _ptr(buf), n, self._s()), "lbm_ch_save_state")
        return buf, self.step_count

    def load_state(self, buf, step):
        _check(lib().lbm_ch_load_state(self.ctx, _ptr(buf), buf.numel(), int(step), self._s()),
               "lbm_ch_load_state")
        return self

    @property
    def tiles(self):
        tx, ty = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_ch_get_tiles(self.ctx, ctypes.byref(tx), ctypes.byref(ty)),
               "lbm_ch_get_tiles")
        return tx.value, ty.value

    def set_tiles(self, tx, ty):
        _check(lib().lbm_ch_set_tiles(self.ctx, int(tx), int(ty)), "lbm_ch_set_tiles")
        return self

    def set_graphs(self, enable=True):
        """Replay repeated step / record / adjoint calls as captured hipGraphs."""
        _check(lib().lbm_ch_set_graphs(self.ctx, int(bool(enable))), "lbm_ch_set_graphs")
        return self

    def autotune(self, trial_steps=20):
        """Pick the fastest tile shape by timing trial steps; the state is restored.
        Returns ((tx, ty), microseconds per step)."""
        t = self.torch
        n = lib().lbm_ch_state_bytes(self.ctx)
        backup = t.empty(n, dtype=t.uint8, device=self.device)
        us = ctypes.c_float()
        _check(lib().lbm_ch_autotune(self.ctx, _ptr(backup), n, int(trial_steps), self._s(),
                                     ctypes.byref(us)), "lbm_ch_autotune")
        return self.tiles, us.value

    def adjoint_scratch_bytes(self):
        return lib().lbm_ch_adjoint_scratch_bytes(ctypes.byref(self.params))

    def record(self, nsteps, phi_traj):
        """Advance ``nsteps`` steps, writing phi^n before each step into
        ``phi_traj[n - n0]`` (a (nsteps, ny, nx) float32 device tensor)."""
        assert phi_traj.is_contiguous() and phi_traj.dtype == self.torch.float32
        assert phi_traj.numel() >= nsteps * self.nx * self.ny
        _check(lib().lbm_ch_record(self.ctx, int(nsteps), _ptr(phi_traj), self._s()),
               "lbm_ch_record")
        return self

    def adjoint(self, n_end, nsteps, phi_traj, lam, grad_u=None, grad_v=None, scratch=None,
                stream=None):
        """Reverse steps n_end-1 .. n_end-nsteps of the tau_g = 1 map: ``lam`` holds
        dL/dphi^{n_end} and becomes dL/dphi^{n_end-nsteps}; ``grad_u``/``grad_v``
        accumulate the derivative with respect to the base velocity field.  ``stream``
        (default: the solver's) may differ from the solver's stream: the reverse steps
        read none of the state that steps and records advance."""
        t = self.torch
        for a in (phi_traj, lam, grad_u, grad_v):
            assert a is None or (a.is_contiguous() and a.dtype == t.float32)
        assert phi_traj.numel() >= nsteps * self.nx * self.ny
        nbytes = self.adjoint_scratch_bytes()
        if scratch is None:
            scratch = t.empty(nbytes, dtype=t.uint8, device=self.device)
        _check(lib().lbm_ch_adjoint(self.ctx, int(n_end), int(nsteps), _ptr(phi_traj), _ptr(lam),
                                    _ptr(grad_u), _ptr(grad_v), _ptr(scratch),
                                    scratch.numel() * scratch.element_size(),
                                    self._s() if stream is None
                                    else ctypes.c_void_p(stream.cuda_stream)),
               "lbm_ch_adjoint")
        return lam

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lib().lbm_ch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many solvers stepped together: ``Batch([solver, ...])``.  The solvers keep
    working on their own (moments, diagnostics, save/load); ``step`` advances all of
    them with the batched kernel, optionally through one captured hipGraph."""

    def __init__(self, solvers, stream=None):
        import torch
        self.torch = torch
        self.solvers = list(solvers)
        n = len(self.solvers)
        self.device = self.solvers[0].device
        self.stream = stream if stream is not None else self.solvers[0].stream
        nbytes = lib().lbm_ch_batch_workspace_bytes(n)
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        arr = (ctypes.c_void_p * n)(*[s.ctx.value for s in self.solvers])
        b = ctypes.c_void_p()
        _check(lib().lbm_ch_batch_create(ctypes.byref(b), arr, n,
                                         ctypes.c_void_p(self.workspace.data_ptr()), nbytes),
               "lbm_ch_batch_create")
        self.b = b

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _members_open(self):
        # the library keeps the contexts' addresses: a closed member must not be reached
        if any(getattr(s, "ctx", None) is None for s in self.solvers):
            raise LbmChError(ESTATE, "Batch: a member Solver was closed before the batch")

    def step(self, n=1, graph=False):
        self._members_open()
        _check(lib().lbm_ch_batch_step(self.b, int(n), 1 if graph else 0, self._s()),
               "lbm_ch_batch_step")
        return self

    @property
    def tiles(self):
        tx, ty = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_ch_batch_get_tiles(self.b, ctypes.byref(tx), ctypes.byref(ty)),
               "lbm_ch_batch_get_tiles")
        return tx.value, ty.value

    def set_tiles(self, tx, ty):
        _check(lib().lbm_ch_batch_set_tiles(self.b, int(tx), int(ty)), "lbm_ch_batch_set_tiles")
        return self

    @property
    def persistent(self):
        return bool(lib().lbm_ch_batch_get_schedule(self.b))

    def set_schedule(self, persistent):
        _check(lib().lbm_ch_batch_set_schedule(self.b, 1 if persistent else 0),
               "lbm_ch_batch_set_schedule")
        return self

    def autotune(self, trial_steps=5):
        """Time every schedule and tile policy; returns ((tx, ty), us per step) and leaves
        the fastest set (see ``persistent``)."""
        self._members_open()
        t = self.torch
        n = lib().lbm_ch_batch_state_bytes(self.b)
        backup = t.empty(n, dtype=t.uint8, device=self.device)
        us = ctypes.c_float()
        _check(lib().lbm_ch_batch_autotune(self.b, _ptr(backup), n, int(trial_steps),
                                           self._s(), ctypes.byref(us)),
               "lbm_ch_batch_autotune")
        return self.tiles, us.value

    def close(self):
        if getattr(self, "b", None):
            self.stream.synchronize()
            lib().lbm_ch_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solver_for(workload, device="cuda", **over):
    """Solver for a workloads.Workload (separable velocity, field or NS)."""
    kw = dict(workload.phys)
    kw.update(over)
    if kw.get("tau_f") is not None and kw.get("gravity") is not None and "ns" not in kw \
            and workload.velocity is None and workload.field is None:
        kw["ns"] = True
    if workload.field is not None:
        return Solver(workload.nx, workload.ny, workload.phi0, field=workload.field,
                      device=device, **kw)
    return Solver(workload.nx, workload.ny, workload.phi0, velocity=workload.velocity,
                  device=device, **kw)
