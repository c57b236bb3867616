/*
 * lbm_ch -- C ABI of the MI355X (gfx950) lattice Boltzmann solver for the
 * Cahn-Hilliard equation of Zhang, Guo & Liang, "A high-order lattice Boltzmann
 * model for the Cahn-Hilliard equation" (arXiv:1805.00007).
 *
 * What one time step computes (Sec. II of the paper, in this order):
 *   phi = sum_i g_i                                            Eq. macroscopicg
 *   mu  = df/dphi - kappa lap(phi), f of Eq. bulk,
 *         beta and kappa from sigma and W                      Eqs. bulk, mu, betakappa
 *   F1  = (phi/rho)(F_s + F_b - grad p), F_s = -phi grad mu,
 *         rho = a phi + b                                      Eqs. NS, rho, t0-phiu
 *   F2  = 3 cs^2 K grad(div(phi u))   (Model-II only)          Eq. mark3, K below Eq. F2-1
 *         model 3, any tau_g: F2 = (2 tau_g - 1 + 3K) dF1/dt + 3 cs^2 eta K d(grad mu)/dt
 *         + 3 cs^2 K grad(div(phi u)) (Eq. F2-1; the time derivatives on the whole time
 *         scale as Remarks I and II allow, as differences over the last step, zero on
 *         the first step; the state then holds X = (2 tau_g - 1 + 3K) F1
 *         + 3 cs^2 eta K grad mu of the previous step)
 *   g_i^eq, S_i = w_i c_i.F/cs^2                               Eqs. geq, liangFi
 *   g_i(x + c_i, t + 1) = g_i - (g_i - g_i^eq)/tau_g
 *                         + (1 - 1/(2 tau_g)) S_i              Eq. LB
 * on the D2Q9 lattice of Sec. II.B (c_0..c_8 = (0,0) (1,0) (0,1) (-1,0) (0,-1)
 * (1,1) (-1,1) (-1,-1) (1,-1)).  The gradient and Laplacian are the isotropic
 * central schemes named in Sec. III:
 *   d_a psi = (1/cs^2) sum_i w_i c_ia psi(x + c_i),
 *   lap psi = (2/cs^2) sum_i w_i [psi(x + c_i) - psi(x)].
 * The velocity u is prescribed (the tests of Sec. III.A-D; then grad p = 0 and
 * F_b = 0) or comes from a coupled Navier-Stokes D2Q9 step (the Rayleigh-Taylor
 * test of Sec. III.E).  The paper calls that NS LBE standard without printing it;
 * the one used is a pressure-based incompressible BGK model:
 *   f_0^eq = (w_0 - 1) p/cs^2 + rho w_0 s_0(u),  f_i^eq = w_i p/cs^2 + rho w_i s_i(u),
 *   s_i(u) = 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u^2,
 *   G_i = w_i [ 3 (c_i - u).F + 9 (c_i.u)(c_i.F) + 3 (c_i.u)(c_i.grad rho) ],
 *   f_i(x + c_i, t + 1) = f_i - (f_i - f_i^eq)/tau_f + (1 - 1/(2 tau_f)) G_i,
 *   F = F_s + F_b + u a M lap(mu),  F_b = (rho accel_x, -(rho - (rho_A + rho_B)/2) g),
 *   rho u = sum_i c_i f_i + F/2,
 *   p = cs^2/(1 - w_0) [sum_{i>0} f_i + u.grad rho/2 + rho w_0 s_0(u)],
 * with kinematic viscosity nu = cs^2 (tau_f - 1/2).
 *
 * Boundaries: x is periodic.  y is periodic, or bounded by no-slip walls half a
 * node below row 0 and above row ny-1: populations leaving through a wall come back
 * in the opposite direction at the same node (half-way bounce-back), and the
 * stencils see mirror images across the walls (phi, mu, p even; u, v odd).
 *
 * Memory and ownership
 * --------------------
 * The library never allocates device memory for data: the caller supplies one device
 * workspace of lbm_ch_workspace_bytes() bytes (256-byte aligned) and keeps it,
 * and every device array it passes to lbm_ch_init, alive until lbm_ch_destroy.
 * Device arrays are float32, row-major (index y*nx + x), unless stated.  Host
 * arrays are copied during the call.  The context itself is host memory owned by
 * the library, with 4 bytes of pinned host memory for its non-finite flag (see
 * lbm_ch_step).  A batch (lbm_ch_batch_create) and a context's first graph capture
 * (lbm_ch_set_graphs) create a capture stream, and graph replay instantiates graphs;
 * the HIP runtime holds these until the batch or context is destroyed (or, for a
 * context, its graphs are dropped).
 *
 * The calls
 * ---------
 * The core is lbm_ch_init, lbm_ch_step and lbm_ch_moments.  The FP64 reductions have
 * a call of their own, lbm_ch_diagnostics, so that reading the fields never forces a
 * reduction and a reduction needs no field buffers; the velocity inputs of lbm_ch_init
 * travel in one struct (lbm_ch_velocity) because which of them are needed depends on
 * the velocity mode.  The rest (state copies, tiles, graphs, autotuning, the adjoint
 * and the batch) is optional.
 *
 * Streams and errors
 * ------------------
 * Calls that take a stream enqueue their device work on it and return without
 * waiting for it, except lbm_ch_check_finite, which synchronises that stream.
 * Every call returns an lbm_ch_status; no exception crosses the ABI.  On an
 * invalid argument nothing is enqueued and the context is unchanged.  A HIP
 * runtime error is returned as LBM_CH_EHIP (lbm_ch_last_hip_error() gives the
 * code).  Calls on one context must not overlap in time from several host threads.
 */
#ifndef LBM_CH_H
#define LBM_CH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ch_ctx lbm_ch_ctx; /* opaque, host-side */

typedef enum {
  LBM_CH_OK = 0,
  LBM_CH_EINVAL = -1,       /* invalid parameter, size, pointer or alignment        */
  LBM_CH_EUNSUPPORTED = -2, /* valid but not implemented combination                */
  LBM_CH_EHIP = -3,         /* HIP runtime error                                    */
  LBM_CH_ENONFINITE = -4,   /* the order parameter holds NaN or Inf                 */
  LBM_CH_ESTATE = -5        /* call out of order (e.g. NULL or destroyed context)   */
} lbm_ch_status;

enum {
  LBM_CH_VEL_NONE = 0,      /* u = 0                                                */
  LBM_CH_VEL_SEPARABLE = 1, /* u = tf[n] ax[x] ay[y], v = tf[n] bx[x] by[y]         */
  LBM_CH_VEL_FIELD = 2,     /* u = tf[n] ux[y*nx+x], v = tf[n] uy[y*nx+x]           */
  LBM_CH_VEL_NS = 3         /* u and p from the coupled Navier-Stokes step          */
};

enum {
  LBM_CH_STORE_F32 = 0,     /* g stored as nine float32 planes (36 B per node)       */
  LBM_CH_STORE_F16 = 1,     /* g_0 float32; g_1..g_8 as IEEE half codes of g_i / w_i */
  LBM_CH_STORE_BF16 = 2     /* g_0 float32; g_1..g_8 as bfloat16 codes of g_i / w_i  */
};
/* In the 16-bit modes (20 B per node) all arithmetic stays float32; only the stored
 * moving populations are rounded.  g_0 is written as phi minus the decoded others, so
 * phi mass is conserved to float32 rounding whatever the 16-bit rounding.  The f
 * populations of the Navier-Stokes coupling are always float32. */

typedef struct {
  int32_t nx, ny;         /* lattice nodes; 4 <= nx, ny and 36*nx*ny < 2^31 (one
                             buffer of nine float32 planes stays under 2 GiB)     */
  int32_t walls;          /* 0: periodic in y; 1: no-slip walls (see above)         */
  int32_t model;          /* 1: F = F1 (Model-I); 2: F = F1 + F2 of Eq. mark3 (Model-II);
                             3: F = F1 + F2 of Eq. F2-1 (see below; LBM_CH_STORE_F32) */
  int32_t velocity_mode;  /* LBM_CH_VEL_*                                           */
  int32_t storage;        /* LBM_CH_STORE_* (population storage of g)                */
  double tau_g;           /* relaxation time of g, > 1/2 (Eq. LB)                   */
  double mobility;        /* M = cs^2 eta (tau_g - 1/2)                             */
  double sigma, width;    /* surface tension and interface width W (Eq. betakappa)  */
  double phi_a, phi_b;    /* bulk values of the two phases (Eq. bulk), phi_a != phi_b */
  double rho_a, rho_b;    /* densities of the two phases (Eq. rho), > 0             */
  double tau_f;           /* NS relaxation time, > 1/2 (LBM_CH_VEL_NS only)        */
  double gravity;         /* NS: g along -y, as the force -(rho - rho_mean) g      */
  double accel_x;         /* NS: uniform acceleration along +x, force rho accel_x  */
} lbm_ch_params;

typedef struct {
  /* LBM_CH_VEL_SEPARABLE: device tables ax[nx], ay[ny], bx[nx], by[ny].            */
  const float *ax, *ay, *bx, *by;
  /* LBM_CH_VEL_FIELD: device fields ux[nx*ny], uy[nx*ny].
   * LBM_CH_VEL_NS: optional initial velocity fields (NULL: fluid at rest).       */
  const float *ux, *uy;
  /* Host array of per-step factors tf[n], n = 0.. (copied).  NULL: tf = 1.  Steps
   * beyond the table reuse its last entry.  Not used by LBM_CH_VEL_NS.           */
  const double* time_factor;
  int64_t n_time_factor;
} lbm_ch_velocity;

/* Bytes of device workspace lbm_ch_init needs for these parameters, or 0 if the
 * parameters are invalid. */
size_t lbm_ch_workspace_bytes(const lbm_ch_params* p);

/* Validate the parameters, bind the workspace and velocity inputs, and enqueue the
 * initial state on `stream`: g_i = g_i^eq(phi0, mu[phi0], u(t_0)) with no source
 * term (and f_i = f_i^eq(p = 0, rho(phi0), u0) with NS).  phi0 is a device array of
 * nx*ny floats; it is read during the call's device work only.  *out receives the
 * context.  Errors: LBM_CH_EINVAL for tau_g <= 1/2, tau_f <= 1/2 (NS), sizes out of
 * range, phi_a == phi_b, rho_a or rho_b <= 0, model not 1, 2 or 3, a NULL or unaligned
 * (4-byte) array the mode needs, a workspace smaller than lbm_ch_workspace_bytes or
 * not 256-byte aligned, or a storage mode outside LBM_CH_STORE_*; LBM_CH_EUNSUPPORTED
 * for model 3 with 16-bit storage. */
int lbm_ch_init(lbm_ch_ctx** out, const lbm_ch_params* p, const lbm_ch_velocity* vel,
                void* workspace, size_t workspace_bytes, const float* phi0,
                hipStream_t stream);

/* Enqueue nsteps >= 0 time steps (Eq. LB plus streaming; with NS also the coupled
 * NS step) on `stream`.  The step counter n advances by nsteps.  With NS and model 1 or
 * 2 a step is one launch that advances f and g together (velocity and pressure are
 * formed inside it and not stored; lbm_ch_moments recomputes them); model 3 runs the NS
 * step and then the phase-field step.  Non-finite values:
 * every step kernel raises a flag of the context when a phi it sums from the
 * populations is NaN or Inf; the flag lives in 4 bytes of pinned host memory mapped
 * into the device (allocated by lbm_ch_init, freed by lbm_ch_destroy), so it lands on
 * the host without any copy or synchronisation.  Once it has landed, this call (and
 * lbm_ch_record, lbm_ch_batch_step for a batch holding the context) returns
 * LBM_CH_ENONFINITE and enqueues nothing; lbm_ch_load_state clears it.  A flag raised
 * by steps still in flight is reported by a later call (lbm_ch_check_finite waits). */
int lbm_ch_step(lbm_ch_ctx* ctx, int64_t nsteps, hipStream_t stream);

/* Enqueue the macroscopic fields of the current state into caller device arrays of
 * nx*ny floats (any may be NULL): phi (Eq. macroscopicg), mu (Eq. mu), the velocity
 * u, v at the current time and the pressure p (0 for a prescribed velocity). */
int lbm_ch_moments(lbm_ch_ctx* ctx, float* phi, float* mu, float* ux, float* uy, float* p,
                   hipStream_t stream);

/* Enqueue FP64 reductions of the current order parameter into the caller device
 * array out[8]: sum phi, sum |phi|, free energy (Eq. freeEnergy with the isotropic
 * gradient), sum (phi - phi_ref)^2, sum phi_ref^2, max phi, min phi, number of
 * non-finite values (finite values only enter the other entries).  phi_ref may be
 * NULL (entries 3 and 4 are then 0).  The reduction order is fixed, so results are
 * bitwise reproducible. */
int lbm_ch_diagnostics(lbm_ch_ctx* ctx, const float* phi_ref, double* out, hipStream_t stream);

/* Synchronise `stream`, count non-finite phi values and return LBM_CH_ENONFINITE if
 * there are any, LBM_CH_OK otherwise. */
int lbm_ch_check_finite(lbm_ch_ctx* ctx, hipStream_t stream);

/* Current step counter n. */
int64_t lbm_ch_step_count(const lbm_ch_ctx* ctx);

/* Bytes of the solver state: the g populations in their storage layout, followed by
 * the float32 f populations with NS, then for model 3 the two float32 planes of X. */
size_t lbm_ch_state_bytes(const lbm_ch_ctx* ctx);

/* Enqueue a device-to-device copy of the state into dst (checkpoint), or from src
 * (resume; the step counter is set to `step`).  Sizes must equal
 * lbm_ch_state_bytes. */
int lbm_ch_save_state(lbm_ch_ctx* ctx, void* dst, size_t bytes, hipStream_t stream);
int lbm_ch_load_state(lbm_ch_ctx* ctx, const void* src, size_t bytes, int64_t step,
                      hipStream_t stream);

/* Tile shape of the step kernels: tx columns (one lane each; 64, 128, 256 or 512) by
 * ty >= 1 rows per thread block (ty is clipped to ny), marching down the rows; or tx = 0:
 * single-pass tiles of 64 columns x ty rows (ty 4, 8 or 16) that pull their rows and a
 * margin of 2 at once, for periodic float32 lattices with a prescribed velocity at
 * tau_g = 1, models 1 and 2 (LBM_CH_EINVAL elsewhere).  The default is chosen at init
 * from the lattice size and storage; it changes speed only, never results.
 *   Where single-pass tiles serve: with float32 storage below 2048^2 nodes, tx = 0 with
 *   ty = 4 up to 65536 nodes, else 16; with 16-bit storage at every size, ty = 4 up to
 *   65536 nodes, 8 below 2048^2, else 16.
 *   Otherwise from 2048^2 nodes up: the widest, then tallest, shape with ty from 32 down to 1 that
 *   gives at least 512 blocks with float32 storage, 1024 with 16-bit; tx = 512 needs
 *   1024 blocks of ty = 8 with float32 storage (and takes ty = 16 once that gives 2048
 *   blocks), and 512 blocks of ty = 16 with 16-bit storage (ty = 16 below 1024 such
 *   blocks, else ty = 8); 64 x 1 if none does.
 *   Other lattices below: the tallest ty (at most 16 with float32 storage, 4 with
 *   16-bit) with nx ny / (64 ty) >= 2048, then the widest tx whose strips span at most
 *   9/8 nx columns (tx = 512 only with ty <= 8 and 256 blocks or more; else 64).
 * The single-launch coupled step (NS, models 1 and 2) has output tiles of 64 columns
 * whatever tx, and 16, 8, 4 or 2 rows: the largest of these not above ty (2 below); its
 * default is 64 x 16.  lbm_ch_set_tiles: LBM_CH_EINVAL for other shapes. */
int lbm_ch_set_tiles(lbm_ch_ctx* ctx, int32_t tx, int32_t ty);
int lbm_ch_get_tiles(const lbm_ch_ctx* ctx, int32_t* tx, int32_t* ty);
/* The default tile shape lbm_ch_init would choose for these parameters (above), without
 * a device or a context.  Errors: LBM_CH_EINVAL for invalid parameters (as
 * lbm_ch_workspace_bytes rejects them) or null outputs. */
int lbm_ch_default_tiles(const lbm_ch_params* params, int32_t* tx, int32_t* ty);

/* Graph replay (enable = 1; 0, the default, turns it off and frees the cached graphs).
 * With it on, lbm_ch_step, lbm_ch_record and lbm_ch_adjoint capture the launches of a
 * call once into a hipGraph, on a capture stream the context owns, and replay it with
 * one graph launch whenever a later call repeats the same arguments (step count,
 * current buffer, caller pointers): on small lattices, where each launch is short, this
 * removes most of the gap between dependent launches.  Results are identical to the
 * plain launches.  Runs whose launch arguments change from step to step (a per-step
 * time-factor table) keep the plain launches; model 3's first step is launched plainly.
 * Up to 16 graphs are cached per context (least recently used dropped first); a change
 * of tile shape drops them all.  The caller buffers named in a cached graph must stay
 * allocated while it may be replayed; calls on one context must not overlap.  Errors:
 * LBM_CH_EINVAL for other values of enable. */
int lbm_ch_set_graphs(lbm_ch_ctx* ctx, int32_t enable);

/* Autotuner: time trial_steps >= 1 steps (after one untimed step) for each tile shape
 * tx in {64, 128, 256, 512} (skipping widths with more than half the lanes idle) and ty in
 * {1, 2, 4, 8, 16, 32}, keep the fastest, and restore the state and step counter from
 * `backup`, a caller device buffer of exactly lbm_ch_state_bytes(ctx) bytes.
 * Synchronises `stream`.  *best_us (may be NULL) receives the chosen shape's time per
 * step in microseconds. */
int lbm_ch_autotune(lbm_ch_ctx* ctx, void* backup, size_t backup_bytes, int32_t trial_steps,
                    hipStream_t stream, float* best_us);

/* Discrete adjoint of the step at tau_g = 1
 * -----------------------------------------
 * With tau_g = 1 the collision of Eq. LB keeps nothing of the incoming populations
 * (g* = g^eq + S/2 with Eqs. geq and liangFi), so one step is a map of the order
 * parameter alone:
 *   phi^{n+1} = phi^n + M lap(mu^n) + sum_i w_i T_{-c_i}[phi^n s_i(u^n)] - div(F^n)/2,
 * where (T_c psi)(x) = psi(x + c), s_i as above and F = F1 (+ F2 for Model-II) with
 * grad p = 0.  The calls below propagate a derivative dL/dphi^{n+1} back through this
 * map, using that lap is symmetric, grad and div are antisymmetric and T_c^T = T_{-c}
 * on the periodic lattice.  With 16-bit storage the forward map differs from this one
 * by the storage rounding. */

/* Bytes of device scratch lbm_ch_adjoint needs (nx*ny floats), 0 if p is invalid. */
size_t lbm_ch_adjoint_scratch_bytes(const lbm_ch_params* p);

/* Enqueue nsteps steps exactly as lbm_ch_step does, and before each step n write the
 * order parameter phi^n into phi_traj + (n - n0) nx ny (n0: the step counter at the
 * call; phi_traj holds nsteps * nx * ny floats): the forward trajectory that
 * lbm_ch_adjoint reads.  Any mode; for periodic float32 lattices with a prescribed
 * velocity and model 1 or 2 the step kernel writes phi^n itself (the phi it sums from
 * the pulled populations), otherwise a separate launch does before each step; the
 * populations are those of lbm_ch_step either way.  Errors: LBM_CH_EINVAL for
 * nsteps < 0 or a NULL or unaligned phi_traj when nsteps > 0. */
int lbm_ch_record(lbm_ch_ctx* ctx, int64_t nsteps, float* phi_traj, hipStream_t stream);

/* Enqueue the reverse steps n = n_end - 1 down to n_end - nsteps.  phi_traj holds
 * phi^n for n = n_end - nsteps .. n_end - 1 in that order (as lbm_ch_record writes it).
 * lam (nx*ny floats) holds dL/dphi^{n_end} on entry and dL/dphi^{n_end - nsteps} when
 * the work has run (updated in place).  grad_u and grad_v are both NULL or both device
 * arrays of nx*ny floats; they accumulate (+=) sum_n tf[n] dL/du^n and
 * sum_n tf[n] dL/dv^n, the derivative with respect to the base velocity field (ux, uy
 * with LBM_CH_VEL_FIELD; the products ax[x] ay[y] and bx[x] by[y] with
 * LBM_CH_VEL_SEPARABLE).  scratch: at least lbm_ch_adjoint_scratch_bytes device bytes,
 * 4-byte aligned, contents undefined afterwards.  The context's state and step counter
 * are not changed, and its device work reads no population state, only the velocity
 * inputs bound at lbm_ch_init: it may run on another stream at the same time as steps,
 * records or state loads of the same context (the calls themselves still come from one
 * host thread).  Errors: LBM_CH_EUNSUPPORTED unless tau_g == 1, walls == 0, model
 * is 1 or 2 and the velocity is prescribed; LBM_CH_EINVAL for nsteps < 0, n_end < nsteps, NULL or
 * unaligned arrays, or too little scratch. */
int lbm_ch_adjoint(lbm_ch_ctx* ctx, int64_t n_end, int64_t nsteps, const float* phi_traj,
                   float* lam, float* grad_u, float* grad_v, void* scratch,
                   size_t scratch_bytes, hipStream_t stream);

/* lbm_ch_adjoint without caller scratch, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid allocation):
 * the field the reverse steps alternate with lam lives in a static device array of
 * LBM_CH_ADJOINT_STATIC_MAX_NODES floats (4 MiB) that every GPU the library runs on holds
 * until the process ends; its address on the context's device is looked up by
 * lbm_ch_init.  Arguments, results, ordering and errors are those of lbm_ch_adjoint (the
 * same kernels; results bitwise equal), except: LBM_CH_EINVAL if nx*ny exceeds
 * LBM_CH_ADJOINT_STATIC_MAX_NODES; plain launches only (graph replay is not used); no
 * device or host allocation of any kind.  The array is shared by every call on one GPU
 * and keeps the last call's contents (each call overwrites what it reads, so nothing
 * needs clearing): calls that overlap on one GPU, from any context or stream, race. */
#define LBM_CH_ADJOINT_STATIC_MAX_NODES 1048576
int lbm_ch_adjoint_static(lbm_ch_ctx* ctx, int64_t n_end, int64_t nsteps,
                          const float* phi_traj, float* lam, float* grad_u, float* grad_v,
                          hipStream_t stream);

/* Batched stepping
 * ----------------
 * A batch advances many independent lattices (contexts created by lbm_ch_init) in one
 * launch per step: the tiles of every lattice form one work list, each XCD taking a
 * contiguous range of it, walked either by a persistent grid sized to the resident
 * capacity or by one workgroup per tile (lbm_ch_batch_set_schedule).  Results are
 * bitwise those of lbm_ch_step on each context.  Lattices with different tile widths
 * or kernel variants (velocity mode, Model-I/II) form groups of one launch each.
 * Supported: periodic lattices, LBM_CH_STORE_F32, model 1 or 2, prescribed velocity
 * without a time-factor table.  The contexts must outlive the batch; stepping a context on its
 * own between batch steps is allowed. */
typedef struct lbm_ch_batch lbm_ch_batch; /* opaque, host-side */

/* Device bytes of the batch's instance tables for n lattices (0 if n < 1). */
size_t lbm_ch_batch_workspace_bytes(int32_t n);

/* Create a batch over ctxs[0..n) (distinct, live).  workspace: caller device memory of
 * lbm_ch_batch_workspace_bytes(n) bytes, 256-byte aligned, kept until destroy.  No
 * device work is enqueued.  Errors: LBM_CH_EINVAL (sizes, NULL, duplicates),
 * LBM_CH_ESTATE (a dead context), LBM_CH_EUNSUPPORTED (walls, 16-bit storage, model 3,
 * NS velocity or a time-factor table). */
int lbm_ch_batch_create(lbm_ch_batch** out, lbm_ch_ctx* const* ctxs, int32_t n,
                        void* workspace, size_t workspace_bytes);

/* Tile shape of the batch: tx in {64, 128, 256} for every lattice, or 0 to give each
 * lattice the widest of those that leaves the fewest idle lanes; ty >= 1 rows (clipped
 * to each ny).  Default (64, 16). */
int lbm_ch_batch_set_tiles(lbm_ch_batch* b, int32_t tx, int32_t ty);
int lbm_ch_batch_get_tiles(const lbm_ch_batch* b, int32_t* tx, int32_t* ty);

/* Schedule of the batched launch: 1 = persistent (a grid of as many workgroups as the
 * GPU holds at once strides over the tiles), 0 = one workgroup per tile (default; the
 * kernel then has the register budget of the single-lattice step).  get returns the
 * schedule, or LBM_CH_ESTATE for a dead batch. */
int lbm_ch_batch_set_schedule(lbm_ch_batch* b, int32_t persistent);
int lbm_ch_batch_get_schedule(const lbm_ch_batch* b);

/* Enqueue nsteps steps of every lattice on `stream`.  use_graph != 0: the nsteps
 * launches are captured once into a hipGraph (cached for this nsteps) and the graph is
 * launched once.  When the instance tables must be (re)uploaded (first call, new tiles,
 * a context stepped on its own) the call first synchronises `stream`. */
int lbm_ch_batch_step(lbm_ch_batch* b, int64_t nsteps, int32_t use_graph, hipStream_t stream);

/* Bytes of a backup of every lattice's state (each rounded to 256 bytes). */
size_t lbm_ch_batch_state_bytes(const lbm_ch_batch* b);

/* Autotuner: time trial_steps >= 1 batch steps (after one untimed step) for both
 * schedules, every tile policy tx in {0, 64, 128, 256} and ty in {4, 8, 16, 32}, keep the
 * fastest, and
 * restore every lattice's state and step counter from `backup` (device memory of
 * exactly lbm_ch_batch_state_bytes bytes, 256-byte aligned).  Synchronises `stream`.
 * *best_us (may be NULL): the chosen shape's time per batch step in microseconds. */
int lbm_ch_batch_autotune(lbm_ch_batch* b, void* backup, size_t backup_bytes,
                          int32_t trial_steps, hipStream_t stream, float* best_us);

/* Release the batch (its cached graphs and capture stream); the contexts stay. */
int lbm_ch_batch_destroy(lbm_ch_batch* b);

/* Release the context (host memory only).  NULL is accepted. */
int lbm_ch_destroy(lbm_ch_ctx* ctx);

/* Static description of a status code; thread-safe. */
const char* lbm_ch_strerror(int status);

/* hipError_t of the last LBM_CH_EHIP returned on this thread. */
int lbm_ch_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_CH_H */
