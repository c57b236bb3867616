// Internal interface between the host ABI (lbm_ch_api.cpp) and the gfx950 kernels
// (lbm_ch_step.hip, lbm_ch_ns.hip, lbm_ch_aux.hip).  Not installed; the public interface is
// include/lbm_ch.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmch {

// Per-run constants in the form the kernels use (all float32).
struct Coef {
  float beta2;      // 2 beta, with mu_bulk = 2 beta (phi - phi_a)(phi - phi_b)(2 phi - phi_a - phi_b)
  float kappa;      // Eq. betakappa
  float phia, phib;
  float eta;        // M / (cs^2 (tau_g - 1/2))
  float k2;         // 3 cs^2 K = K, the factor of F2 (Eq. mark3); 0 for Model-I
  float a, b;       // rho = a phi + b (Eq. rho)
  float omega;      // 1 / tau_g
  float srcg;       // 3 (1 - 1/(2 tau_g)): S_i (1 - 1/(2 tau)) = srcg w_i c_i.F
  // coupled Navier-Stokes
  float omega_f;    // 1 / tau_f
  float srcf;       // 1 - 1/(2 tau_f)
  float gravity, accel_x, rho_mean;
  float aM;         // a * M, the factor of u lap(mu) in the NS force
  // model 3 (Eq. F2-1): X = x_f1 F1 + x_mu grad mu, F2 = X(t_n) - X(t_{n-1}) + k2 grad D
  float x_f1;       // 2 tau_g - 1 + 3K
  float x_mu;       // 3 cs^2 eta K
};

// Arguments of the fused phase-field step.
struct StepArgs {
  const void* src;    // populations at t_n (layout of the storage mode)
  void* dst;          // populations at t_{n+1}
  uint32_t pitch;     // values per population row (>= nx), see the layout in lbm_ch_device.h
  int nx, ny;
  int ty;             // rows per block
  int nstrips;        // ceil(nx / TX)
  int xcd_remap;      // 1: the grid is a multiple of 8 blocks, map each XCD to a band
  Coef c;
  // prescribed separable velocity (u = tf ax[x] ay[y], v = tf bx[x] by[y])
  const float *ax, *ay, *bx, *by;
  // velocity field (u = tf ux, v = tf uy), and pressure field for the NS coupling
  const float *ux, *uy, *pf;
  float tf;
  float* xh;          // model 3: X of the previous step (2 planes of nx*ny), rewritten
  int xfirst;         // model 3: 1 on the first step (no earlier X: zero difference)
  float* phi_rec;     // launch_phi_record only: phi of the source state (nx*ny), written
  int* nonfinite;     // set to 1 when a phi summed in stage 1 is NaN or Inf (may be null)
};

// Arguments of the batched step: one StepArgs per instance (src/dst as at parity 0),
// start[i] = first tile of instance i (start[n] = total), periodic float32 lattices.
struct BatchArgs {
  const StepArgs* args;
  const int* start;
  int n;
  int total;
  int parity;         // 1: swap src and dst of every instance
};

// Arguments of the coupled Navier-Stokes step.
struct NsArgs {
  const void* gsrc;   // phase-field populations at t_n (storage mode of g)
  const float* fsrc;  // NS populations at t_n
  float* fdst;        // NS populations at t_{n+1} (may be null: moments only)
  float *u, *v, *p;   // velocity and pressure at t_n (written)
  uint32_t pitch;     // values per population row (g and f)
  int nx, ny;
  int ty, nstrips, xcd_remap;
  Coef c;
};

enum VelMode { VEL_SEP = 0, VEL_FIELD = 1, VEL_NSFIELD = 2 };

// Population storage (LBM_CH_STORE_*): 0 float32; 1 half, 2 bfloat16 (g_0 float32, g_1..8
// as 16-bit codes of g_i / w_i).  Bytes of one population buffer of ny rows of `pitch`
// values per population (row-interleaved, see lbm_ch_device.h).
uint32_t population_bytes(int storage, uint32_t pitch, uint32_t ny);

// Launchers (return hipGetLastError() of the launch).
// t1: tau_g = 1 (omega = 1), which selects the reduced tile for models 1 and 2 with a
// prescribed velocity (other cases ignore it).
hipError_t launch_phi_step(int tx, bool walls, int vmode, int model, int storage, bool t1,
                           const StepArgs& a, int nblocks, hipStream_t s);
// The single-pass tau_g = 1 tile (64 columns x rows, rows 4, 8 or 16; nblocks =
// ceil(nx / 64) ceil(ny / rows); a.nstrips = ceil(nx / 64)): periodic lattices with a
// prescribed velocity, models 1 and 2, any storage (phi_pass_ok); with float32 storage
// it writes phi of the source state to a.phi_rec when that is set (16-bit: a.phi_rec
// must be null).  The 16-bit instances are in lbm_ch_step16.hip (launch_phi_pass16).
bool phi_pass_ok(bool walls, int vmode, int model, int storage, bool t1);
hipError_t launch_phi_pass(int rows, int vmode, int model, int storage, const StepArgs& a,
                           int nblocks, hipStream_t s);
hipError_t launch_phi_pass16(int rows, int vmode, int model, int storage, const StepArgs& a,
                             int nblocks, hipStream_t s);
// The 16-bit storage cases of launch_phi_step (storage ST_F16 / ST_BF16), defined in
// lbm_ch_step16.hip.
hipError_t launch_phi_step16(int tx, bool walls, int vmode, int model, int storage, bool t1,
                             const StepArgs& a, int nblocks, hipStream_t s);
// The same step that also writes phi of the source state to a.phi_rec (the sums stage 1
// forms anyway).  Periodic float32 lattices with a prescribed velocity (VEL_SEP or
// VEL_FIELD) and model 1 or 2 only; hipErrorInvalidValue otherwise.
bool phi_record_fused(bool walls, int vmode, int model, int storage);
hipError_t launch_phi_record(int tx, int vmode, int model, bool t1, const StepArgs& a,
                             int nblocks, hipStream_t s);
// grid: a multiple of 8 workgroups.  persistent: the grid strides over the tiles (size
// it with phi_batch_blocks_per_cu); otherwise one tile per workgroup (grid >= tiles).
int phi_batch_blocks_per_cu(int tx, int vmode, bool model2, bool t1);
hipError_t launch_phi_batch(int tx, int vmode, bool model2, bool t1, bool persistent,
                            const BatchArgs& b, int grid, hipStream_t s);
hipError_t launch_ns_step(int tx, bool walls, int storage, const NsArgs& a, int nblocks,
                          hipStream_t s);
// Single-launch coupled step (models 1 and 2): f and g of one time step, output tiles
// of 64 columns x rows (2, 4, 8 or 16; rt_step_rows maps a tile height onto them) in
// ceil(nx / 64) * ceil(ny / rows) workgroups; a.src/a.dst are the g buffers, a.nstrips =
// ceil(nx / 64).  hipErrorInvalidValue for other models.
int rt_step_rows(int ty);
hipError_t launch_rt_step(int rows, bool walls, int model, int storage, const StepArgs& a,
                          const float* fsrc, float* fdst, int nblocks, hipStream_t s);

hipError_t launch_init(bool walls, int vmode, int storage, const Coef& c, int nx, int ny,
                       uint32_t pitch, const float* phi0, const float* ax, const float* ay,
                       const float* bx, const float* by, const float* ux, const float* uy,
                       float tf, void* g, float* f, hipStream_t s);
hipError_t launch_phi_field(bool walls, int storage, const void* g, uint32_t pitch, int nx,
                            int ny, float* phi, hipStream_t s);
hipError_t launch_mu_field(bool walls, const Coef& c, const float* phi, int nx, int ny,
                           float* mu, hipStream_t s);
// One reverse step of the tau_g = 1 phi map (periodic); lam0 must not alias lam1.
hipError_t launch_adjoint_step(const Coef& c, float mobility, int nx, int ny, int vmode,
                                const float* ax, const float* ay, const float* bx,
                                const float* by, const float* ux, const float* uy, float tf,
                                const float* phi, const float* lam1, float* lam0, float* gu,
                                float* gv, hipStream_t s);
hipError_t launch_velocity_field(int vmode, int nx, int ny, const float* ax, const float* ay,
                                 const float* bx, const float* by, const float* ux,
                                 const float* uy, float tf, float* u, float* v,
                                 hipStream_t s);
hipError_t launch_fill(float* dst, float value, int64_t n, hipStream_t s);
// Static device scratch of lbm_ch_adjoint_static (nodes <= ADJ_STATIC_MAX_NODES floats per
// device).  static_scratch_setup(device) must run with `device` current (lbm_ch_init does
// it); static_scratch(device) is then that device's address, or null before the setup.
constexpr size_t ADJ_STATIC_MAX_NODES = size_t(1) << 20;
hipError_t static_scratch_setup(int device);
float* static_scratch(int device);
// FP64 reductions of a phi field; partial needs diag_partial_blocks()*8 doubles.
int diag_partial_blocks();
hipError_t launch_diag(bool walls, const Coef& c, const float* phi, const float* ref, int nx,
                       int ny, double* partial, double* out, hipStream_t s);

}  // namespace lbmch
