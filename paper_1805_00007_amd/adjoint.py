"""Reverse-mode derivatives of a phase-field run at tau_g = 1, as a torch.autograd.Function.

``evolve(phi0, U, V, steps, **params)`` returns phi^N of the solver started from phi0 in
the prescribed velocity field u^n = tf[n] (U, V), and is differentiable with respect to
phi0 and (U, V).  A parameterised velocity (for instance stream-function coefficients
times fixed mode fields) reaches its parameters through ordinary torch operations on U
and V before the call.

Forward: the solver runs N steps on the GPU and keeps its state every S = ceil(sqrt(N))
steps (``lbm_ch_save_state``); with ``graphs=True`` the repeated segment launches are
replayed as captured hipGraphs.  Backward: for each segment from the last, the state is
reloaded, the segment re-run with ``lbm_ch_record`` (phi^n of every step), and
``lbm_ch_adjoint`` carries dL/dphi back over it while accumulating dL/d(U, V).  The
reverse steps read none of the solver state, and the re-runs of different segments are
independent, so by default two solvers (the forward one and a second one with the same
parameters, each on its own stream) re-run alternate segments while a third stream runs
the reverse steps, which then form the critical path; three trajectory buffers are
taken in turn, and events order each buffer's writer after its previous reader and each
segment's reverse steps after its re-run.  Memory: ceil(N/S) states, 3 S phi fields and
the second solver's state.  All derivative arithmetic runs in the library's kernels;
this module only orders the calls.
"""
from __future__ import annotations

import math

import torch

from . import Solver


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, U, V, steps, segment, tf, params, tune, graphs, store, overlap):
        ny, nx = phi0.shape
        s = Solver(nx, ny, phi0.detach(), field=(U.detach(), V.detach()), tf=tf,
                   device=phi0.device, **params)
        s.stream.wait_stream(torch.cuda.current_stream(phi0.device))
        s.set_graphs(graphs)
        if isinstance(tune, tuple):
            s.set_tiles(*tune)
        elif tune:
            s.autotune(trial_steps=tune)
        ctx.traj = None
        if store:
            # the whole trajectory phi^0 .. phi^{N-1} (N nx ny floats) instead of
            # checkpoints: the backward pass then needs no recomputation
            traj = torch.empty((steps, s.ny, s.nx), dtype=torch.float32, device=s.device)
            if steps:
                s.record(steps, traj)
            phi = s.phi()
            torch.cuda.current_stream(phi0.device).wait_stream(s.stream)
            ctx.solver, ctx.ckpts, ctx.seg, ctx.traj = s, [], steps, traj
            ctx.overlap = False
            return phi
        seg = int(segment) if segment else max(1, math.isqrt(max(steps - 1, 0)) + 1)
        ckpts = []
        n = 0
        while n < steps:
            k = min(seg, steps - n)
            buf, _ = s.save_state()
            ckpts.append((n, k, buf))
            s.step(k)
            n += k
        phi = s.phi()
        torch.cuda.current_stream(phi0.device).wait_stream(s.stream)
        ctx.solver, ctx.ckpts, ctx.seg, ctx.overlap = s, ckpts, seg, overlap
        ctx.remake = (tf, params, graphs)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        s = ctx.solver
        dev = s.device
        s.stream.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s.stream):
            lam = gphi.detach().to(torch.float32).contiguous().clone()
            want_u = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
            gu = torch.zeros_like(lam) if want_u else None
            gv = torch.zeros_like(lam) if want_u else None
            scratch = torch.empty(s.adjoint_scratch_bytes(), dtype=torch.uint8, device=dev)
            if ctx.traj is not None:
                if ctx.seg:
                    s.adjoint(ctx.seg, ctx.seg, ctx.traj, lam, gu, gv, scratch)
            elif not ctx.overlap:
                traj = torch.empty((ctx.seg, s.ny, s.nx), dtype=torch.float32, device=dev)
                for n0, k, buf in reversed(ctx.ckpts):
                    s.load_state(buf, n0)
                    s.record(k, traj)
                    s.adjoint(n0 + k, k, traj, lam, gu, gv, scratch)
            else:
                # three streams of their own (consecutive pool streams), none of them the
                # stream the caller works on
                home = s.stream
                sa, sb, rs = (torch.cuda.Stream(device=dev) for _ in range(3))
                for st in (sa, sb, rs):
                    st.wait_stream(home)  # lam, gu, gv and the scratch are initialised
                s.stream = sa
                solvers = [s]
                if len(ctx.ckpts) > 1:
                    tf, params, graphs = ctx.remake
                    with torch.cuda.stream(sb):  # its memory belongs to its own stream
                        z = torch.zeros((s.ny, s.nx), dtype=torch.float32, device=dev)
                        s2 = Solver(s.nx, s.ny, z, field=tuple(s._keep[:2]), tf=tf,
                                    device=dev, stream=sb, **params)
                    s2.set_graphs(graphs).set_tiles(*s.tiles)
                    solvers.append(s2)
                nb = len(solvers) + 1
                trajs = [torch.empty((ctx.seg, s.ny, s.nx), dtype=torch.float32, device=dev)
                         for _ in range(nb)]
                read = [None] * nb  # event after the last reverse steps that read buffer b
                try:
                    for i, (n0, k, buf) in enumerate(reversed(ctx.ckpts)):
                        b = i % nb
                        sv = solvers[i % len(solvers)]
                        if read[b] is not None:
                            sv.stream.wait_event(read[b])
                        sv.load_state(buf, n0)
                        sv.record(k, trajs[b])
                        written = torch.cuda.Event()
                        written.record(sv.stream)
                        rs.wait_event(written)
                        s.adjoint(n0 + k, k, trajs[b], lam, gu, gv, scratch, stream=rs)
                        read[b] = torch.cuda.Event()
                        read[b].record(rs)
                finally:
                    for st in (sa, sb, rs):
                        home.wait_stream(st)
                    s.stream = home
                    for sv in solvers[1:]:
                        sv.close()
        torch.cuda.current_stream(dev).wait_stream(s.stream)
        return lam, gu, gv, None, None, None, None, None, None, None, None


def evolve(phi0, U, V, steps, *, tf=None, segment=None, autotune=0, tiles=None, graphs=False,
           store_trajectory=False, overlap=True, **params):
    """phi after ``steps`` steps from ``phi0`` (ny, nx) in the velocity field tf[n] (U, V),
    differentiable in phi0, U and V.  ``params`` are those of ``lbm_ch_params``; the
    derivative needs tau_g = 1, periodic boundaries and a prescribed velocity.
    ``tiles=(tx, ty)`` fixes the step kernels' tile shape; otherwise ``autotune`` > 0
    times that many trial steps per tile shape first (the state is restored; the
    forward run and its recomputation then use the fastest shape).  ``graphs``: replay
    the repeated segment launches as captured hipGraphs (``lbm_ch_set_graphs``; same
    results; at 256^2 the captures a pass needs cost about what the replays save).
    ``store_trajectory``: keep phi of every step (steps * nx * ny floats of device memory)
    instead of sqrt(N) checkpoints, so the backward pass recomputes nothing (same
    gradients).  ``overlap``: with checkpoints, re-run the segments on two solvers beside
    the reverse steps on a third stream (same gradients, bitwise; a second solver's
    state and two more segments of phi fields); ``False`` runs them one after the other
    on the forward solver's stream."""
    if float(params.get("tau_g", 1.0)) != 1.0 or params.get("walls", 0):
        raise ValueError("the discrete adjoint covers tau_g = 1 on a periodic lattice")
    tune = tuple(int(t) for t in tiles) if tiles is not None else int(autotune)
    return _Evolve.apply(phi0, U, V, int(steps), segment, tf, dict(params), tune, bool(graphs),
                         bool(store_trajectory), bool(overlap))
