// Host implementation of the C ABI declared in include/lbm_ch.h: parameter checks and
// derivation (Eqs. betakappa, rho, the mobility relation below Eq. phit3, and K below
// Eq. F2-1), the workspace layout, the tile choice and the launch sequence.
#include "lbm_ch.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lbm_ch_internal.h"

using namespace lbmch;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return LBM_CH_EHIP;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  uint32_t pitch;  // values per population row: nx rounded up to 32 (rows start 128-B aligned)
  size_t g_state;  // bytes of the g populations (storage mode)
  size_t f_state;  // bytes of the f populations (nine float32 populations per node)
  size_t g_bytes;  // one g population buffer, 256-byte aligned
  size_t f_bytes;  // one f population buffer, 256-byte aligned
  size_t off_ga, off_gb, off_fa, off_fb, off_u, off_v, off_p, off_phi, off_ztab, off_part,
      off_diag, off_xh, total;
};

uint32_t pitch_of(int nx) { return (uint32_t)((nx + 31) / 32 * 32); }

bool valid_params(const lbm_ch_params* p) {
  if (!p) return false;
  if (p->nx < 4 || p->ny < 4) return false;
  if ((double)pitch_of(p->nx) * (double)p->ny * 9.0 * 4.0 >= 2147483648.0) return false;
  if (p->walls != 0 && p->walls != 1) return false;
  if (p->model < 1 || p->model > 3) return false;
  if (p->velocity_mode < LBM_CH_VEL_NONE || p->velocity_mode > LBM_CH_VEL_NS) return false;
  if (p->storage < LBM_CH_STORE_F32 || p->storage > LBM_CH_STORE_BF16) return false;
  if (!(p->tau_g > 0.5) || !isfinite(p->tau_g)) return false;
  if (!(p->phi_a != p->phi_b)) return false;
  if (!(p->rho_a > 0.0) || !(p->rho_b > 0.0)) return false;
  if (!isfinite(p->mobility) || !isfinite(p->sigma) || !(p->width > 0.0)) return false;
  if (p->sigma < 0.0 || p->mobility < 0.0) return false;
  if (p->velocity_mode == LBM_CH_VEL_NS) {
    if (!(p->tau_f > 0.5) || !isfinite(p->tau_f)) return false;
    if (!isfinite(p->gravity) || !isfinite(p->accel_x)) return false;
  }
  return true;
}

Layout layout_of(const lbm_ch_params* p) {
  Layout L{};
  const size_t nodes = (size_t)p->nx * p->ny;
  L.pitch = pitch_of(p->nx);
  L.g_state = population_bytes(p->storage, L.pitch, (uint32_t)p->ny);
  L.f_state = population_bytes(0, L.pitch, (uint32_t)p->ny);
  L.g_bytes = align_up(L.g_state);
  L.f_bytes = align_up(L.f_state);
  const bool ns = p->velocity_mode == LBM_CH_VEL_NS;
  const size_t field = align_up(nodes * sizeof(float));
  size_t o = 0;
  L.off_ga = o; o += L.g_bytes;
  L.off_gb = o; o += L.g_bytes;
  L.off_fa = o; if (ns) o += L.f_bytes;
  L.off_fb = o; if (ns) o += L.f_bytes;
  L.off_u = o; o += field;
  L.off_v = o; o += field;
  L.off_p = o; o += field;
  L.off_phi = o; o += field;
  L.off_ztab = o; o += align_up((size_t)2 * (p->nx + p->ny) * sizeof(float));
  L.off_part = o; o += align_up((size_t)diag_partial_blocks() * 8 * sizeof(double));
  L.off_diag = o; o += align_up(8 * sizeof(double));
  L.off_xh = o; if (p->model == 3) o += align_up(2 * nodes * sizeof(float));
  L.total = o;
  return L;
}

bool aligned4(const void* q) { return ((uintptr_t)q & 3u) == 0; }

}  // namespace

struct lbm_ch_ctx {
  int device;  // HIP device current at lbm_ch_init
  // non-finite flag: pinned host memory mapped into the device, set by the step kernels
  // when a phi they sum is NaN or Inf, read by the next lbm_ch_step / lbm_ch_record
  int* nf_host;
  int* nf_dev;
  lbm_ch_params p;
  Coef c;
  Layout L;
  char* ws;
  void* g[2];
  float *f[2], *u, *v, *pr, *phi, *ztab, *xh;
  double *part, *diag;
  int cur;  // index of the buffer holding the current state
  int64_t step;
  int vmode;  // internal VelMode of the prescribed velocity
  const float *ax, *ay, *bx, *by, *ux, *uy;
  std::vector<double> tf;
  int tx, ty, nstrips, nblocks, xcd_remap;
  int graphs;                     // lbm_ch_set_graphs: replay captured launch sequences
  hipStream_t cap;                // capture stream, created at the first capture
  std::vector<struct CtxExec> execs;  // cached executable graphs, most recently used last
  uint32_t magic;
};

// One cached launch sequence: kind 0 = steps, 1 = recorded steps, 2 = reverse steps;
// n steps starting from buffer `cur` (kinds 0, 1); p = the caller pointers it uses.
struct CtxExec {
  hipGraphExec_t exec;
  int kind;
  int64_t n;
  int cur;
  const void* p[5];
};

static void drop_graphs(lbm_ch_ctx* c) {
  for (CtxExec& x : c->execs) (void)hipGraphExecDestroy(x.exec);
  c->execs.clear();
}

static constexpr uint32_t CTX_MAGIC = 0x4c424d43u;

static bool live(const lbm_ch_ctx* c) { return c && c->magic == CTX_MAGIC; }

// tau_g = 1 exactly: the collision keeps none of the pulled populations (omega = 1).
static bool tau_one(const lbm_ch_ctx* c) { return c->p.tau_g == 1.0; }

// The single-pass tile (tx = 0 in lbm_ch_set_tiles) serves periodic lattices with a
// prescribed velocity at tau_g = 1, models 1 and 2.
static bool pass_eligible(const lbm_ch_params& p) {
  const int vmode = p.velocity_mode == LBM_CH_VEL_FIELD ? VEL_FIELD
                    : p.velocity_mode == LBM_CH_VEL_SEPARABLE ? VEL_SEP : -1;
  return vmode >= 0 && phi_pass_ok(p.walls != 0, vmode, p.model, p.storage, p.tau_g == 1.0);
}

static float time_factor(const lbm_ch_ctx* c, int64_t n) {
  if (c->tf.empty()) return 1.0f;
  if (n < (int64_t)c->tf.size()) return (float)c->tf[(size_t)n];
  return (float)c->tf.back();
}

// Tile shape: TX columns per block (one lane per column), TY rows per block.
static bool valid_tile(int tx, int ty) {
  return (tx == 64 || tx == 128 || tx == 256 || tx == 512) && ty >= 1;
}

static void apply_tiles(lbm_ch_ctx* c, int tx, int ty) {
  drop_graphs(c);  // the launch shape is part of every captured sequence
  const int nx = c->p.nx, ny = c->p.ny;
  if (tx == 0) {  // single-pass tiles of 64 columns x ty rows (ty is a kernel constant)
    c->tx = 0;
    c->ty = ty;
    c->nstrips = (nx + 63) / 64;
    c->nblocks = c->nstrips * ((ny + ty - 1) / ty);
    c->xcd_remap = (c->nblocks % 8 == 0) ? 1 : 0;
    return;
  }
  if (ty > ny) ty = ny;
  c->tx = tx;
  c->ty = ty;
  c->nstrips = (nx + tx - 1) / tx;
  const int nchunks = (ny + ty - 1) / ty;
  c->nblocks = c->nstrips * nchunks;
  c->xcd_remap = (c->nblocks % 8 == 0) ? 1 : 0;
}

// Default tile.  Lattices of 2048^2 nodes and more: the widest tile (fewest halo
// columns), then the tallest (fewest halo rows per row; heights 32 down to 1), that still
// gives at least 2 workgroups per CU on 256 CUs (float32), or 4 with 16-bit storage,
// whose extra decode work per byte needs more waves in flight to cover memory latency;
// the 512-column tile (8 waves per workgroup; half the halo columns of the 256-column
// one) by the measured rules below.  Smaller lattices: the single-pass tile where it
// serves, else the marching rule below; both from sweeps of every shape.
// lbm_ch_set_tiles overrides; lbm_ch_autotune measures.
static void default_tiles(const lbm_ch_params& p, int& tx_out, int& ty_out) {
  const int nx = p.nx, ny = p.ny;
  if (p.velocity_mode == LBM_CH_VEL_NS && (p.model == 1 || p.model == 2)) {
    // the single-launch coupled step: output tiles of 64 columns x 16 rows (256 x 1024
    // Rayleigh-Taylor: 11.0 us per step, against 11.6 us with 8 rows and 13.8 with 4)
    tx_out = 64;
    ty_out = 16;
    return;
  }
  const bool f32 = p.storage == LBM_CH_STORE_F32;
  const long nodes = (long)nx * ny;
  if (pass_eligible(p) && (!f32 || nodes < (4L << 20))) {
    // single-pass tiles where they serve: below 2048^2 with float32 storage (us per step,
    // marching default / single pass: 256^2 6.78 / 4.77 (4 rows); 512^2 9.27 / 5.93,
    // 768^2 16.1 / 12.8, 1536^2 44.0 / 39.7 (16 rows); 1024^2 20.6 / 21.0; from 2048^2
    // up the march is faster: 61.5 / 66.4), at every size with 16-bit storage (256^2
    // 7.07 / 4.75 (4 rows); 768^2 17.5 / 9.7, 1536^2 42.6 / 26.8 (8 rows); 2048^2
    // 52.4 / 42.9, 4096^2 243 / 199 (16 rows))
    tx_out = 0;
    ty_out = nodes <= 65536 ? 4 : (f32 || nodes >= (4L << 20)) ? 16 : 8;
    return;
  }
  if (nodes < (4L << 20)) {
    // Below 2048^2 a step is a short, latency-bound march.  Tallest chunk (at most 16
    // rows with float32 storage, 4 with 16-bit) that still gives 2048 waves of columns,
    // then the widest strip whose strips span at most 9/8 nx columns; 512-column strips
    // only with chunks of at most 8 rows and 256 blocks or more.  Sweeps of every shape
    // (square lattices, float32): 256^2 256 x 1, 512^2 512 x 2, 768^2 256 x 4, 1024^2
    // 512 x 8, 1280^2 256 x 8, 1536^2 256 x 16, each within 3 % of the fastest shape
    // (1792^2: 256 x 16, 9 %).
    const int ycap = f32 ? 16 : 4;
    int ty = 1;
    for (int yy : {16, 8, 4, 2, 1}) {
      if (yy <= ycap && nodes / (64L * yy) >= 2048) {
        ty = yy;
        break;
      }
    }
    int tx = 64;
    for (int xx : {512, 256, 128}) {
      if (xx > nx) continue;
      const long strips = (nx + xx - 1) / xx;
      if (strips * xx * 8 > 9L * nx) continue;
      if (xx == 512 && (ty > 8 || strips * ((ny + ty - 1) / ty) < 256)) continue;
      tx = xx;
      break;
    }
    tx_out = tx;
    ty_out = ty;
    return;
  }
  const long min_blocks = f32 ? 512 : 1024;
  int tx = 64, ty = 1;
  bool found = false;
  for (int xx : {512, 256, 128, 64}) {
    if (xx > nx && xx > 64) continue;
    // 512 columns: at least 1024 blocks with float32 storage, at least 512 blocks of 16
    // rows with 16-bit storage (2048^2: 512 x 16, 58.2 us against 63.5 us at 256 x 16)
    const long need = xx == 512 ? (f32 ? 2 * min_blocks : min_blocks / 2) : min_blocks;
    if (xx == 512 && f32) {
      // float32, 512 columns: 16-row chunks once they give 2048 blocks, else 8 rows
      // (2048^2: 61.5 us against 62.2 us at 512 x 16; 3072^2: 137 us against 143 us;
      // 4096^2: 215 us against 225 us at 512 x 8 and 219 us at 512 x 32; 7680^2: 796 us
      // against 825 us at 512 x 32)
      const long strips = (nx + xx - 1) / xx;
      const long n16 = strips * ((ny + 15) / 16), n8 = strips * ((ny + 7) / 8);
      if (n8 >= need) {
        tx = xx;
        ty = n16 >= 2048 ? 16 : 8;
        found = true;
        break;
      }
      continue;
    }
    if (xx == 512 && !f32) {
      // 16-bit, 512 columns: 16-row chunks while they give fewer than 1024 blocks
      // (2048^2), 8-row chunks from there up (3072^2: 147 us against 158 us at 512 x 16
      // and 180 us at 512 x 32; 4096^2: 242 us, as at 512 x 16; 259 us at 512 x 32)
      const long n16 = (long)((nx + xx - 1) / xx) * ((ny + 15) / 16);
      if (n16 >= need) {
        tx = xx;
        ty = n16 < 1024 ? 16 : 8;
        found = true;
        break;
      }
      continue;
    }
    for (int yy : {32, 16, 8, 4, 2, 1}) {
      const long nb = (long)((nx + xx - 1) / xx) * ((ny + yy - 1) / yy);
      if (nb >= need) {
        tx = xx;
        ty = yy;
        found = true;
        break;
      }
    }
    if (found) break;
  }
  tx_out = tx;
  ty_out = ty;
}

static void choose_tiles(lbm_ch_ctx* c) {
  int tx, ty;
  default_tiles(c->p, tx, ty);
  apply_tiles(c, tx, ty);
}

extern "C" {

size_t lbm_ch_workspace_bytes(const lbm_ch_params* p) {
  if (!valid_params(p)) return 0;
  return layout_of(p).total;
}

int lbm_ch_init(lbm_ch_ctx** out, const lbm_ch_params* p, const lbm_ch_velocity* vel,
                void* workspace, size_t workspace_bytes, const float* phi0,
                hipStream_t stream) {
  if (!out) return LBM_CH_EINVAL;
  *out = nullptr;
  if (!valid_params(p)) return LBM_CH_EINVAL;
  if (p->model == 3 && p->storage != LBM_CH_STORE_F32) return LBM_CH_EUNSUPPORTED;
  const Layout L = layout_of(p);
  if (!workspace || ((uintptr_t)workspace % ALIGN) != 0 || workspace_bytes < L.total)
    return LBM_CH_EINVAL;
  if (!phi0 || !aligned4(phi0)) return LBM_CH_EINVAL;
  const int vm = p->velocity_mode;
  if (vm == LBM_CH_VEL_SEPARABLE) {
    if (!vel || !vel->ax || !vel->ay || !vel->bx || !vel->by) return LBM_CH_EINVAL;
    if (!aligned4(vel->ax) || !aligned4(vel->ay) || !aligned4(vel->bx) || !aligned4(vel->by))
      return LBM_CH_EINVAL;
  }
  if (vm == LBM_CH_VEL_FIELD) {
    if (!vel || !vel->ux || !vel->uy || !aligned4(vel->ux) || !aligned4(vel->uy))
      return LBM_CH_EINVAL;
  }
  if (vm == LBM_CH_VEL_NS && vel && ((vel->ux != nullptr) != (vel->uy != nullptr)))
    return LBM_CH_EINVAL;
  if (vel && vel->time_factor && vel->n_time_factor < 0) return LBM_CH_EINVAL;

  int device = 0;
  hipError_t de = hipGetDevice(&device);
  // the device's copy of the static scratch of lbm_ch_adjoint_static, looked up once per
  // device while that device is current
  if (de == hipSuccess) de = static_scratch_setup(device);
  if (de != hipSuccess) return hip_fail(de);
  int* nf_host = nullptr;
  int* nf_dev = nullptr;
  de = hipHostMalloc((void**)&nf_host, sizeof(int), hipHostMallocMapped);
  if (de == hipSuccess) de = hipHostGetDevicePointer((void**)&nf_dev, nf_host, 0);
  if (de != hipSuccess) {
    if (nf_host) (void)hipHostFree(nf_host);
    return hip_fail(de);
  }
  *nf_host = 0;
  lbm_ch_ctx* c = new (std::nothrow) lbm_ch_ctx();
  if (!c) {
    (void)hipHostFree(nf_host);
    return LBM_CH_EINVAL;
  }
  c->device = device;
  c->nf_host = nf_host;
  c->nf_dev = nf_dev;
  c->p = *p;
  c->L = L;
  c->ws = (char*)workspace;
  c->g[0] = c->ws + L.off_ga;
  c->g[1] = c->ws + L.off_gb;
  const bool ns = vm == LBM_CH_VEL_NS;
  c->f[0] = ns ? (float*)(c->ws + L.off_fa) : nullptr;
  c->f[1] = ns ? (float*)(c->ws + L.off_fb) : nullptr;
  c->u = (float*)(c->ws + L.off_u);
  c->v = (float*)(c->ws + L.off_v);
  c->pr = (float*)(c->ws + L.off_p);
  c->phi = (float*)(c->ws + L.off_phi);
  c->ztab = (float*)(c->ws + L.off_ztab);
  c->part = (double*)(c->ws + L.off_part);
  c->diag = (double*)(c->ws + L.off_diag);
  c->xh = p->model == 3 ? (float*)(c->ws + L.off_xh) : nullptr;
  c->cur = 0;
  c->step = 0;

  // Coefficients.
  const double dphi = fabs(p->phi_a - p->phi_b);
  const double beta = 12.0 * p->sigma / (p->width * dphi * dphi * dphi * dphi);  // Eq. betakappa
  const double kappa = 3.0 * p->sigma * p->width / (2.0 * dphi * dphi);           // Eq. betakappa
  const double cs2 = 1.0 / 3.0;
  const double eta = p->mobility / (cs2 * (p->tau_g - 0.5));  // M = cs^2 eta (tau - 1/2)
  const double K = (p->tau_g - 1.0 / 6.0 - p->tau_g * p->tau_g) / (p->tau_g - 0.5);
  const double a = (p->rho_a - p->rho_b) / (p->phi_a - p->phi_b);                  // Eq. rho
  const double b = (p->rho_b * p->phi_a - p->phi_b * p->rho_a) / (p->phi_a - p->phi_b);
  Coef& k = c->c;
  k.beta2 = (float)(2.0 * beta);
  k.kappa = (float)kappa;
  k.phia = (float)p->phi_a;
  k.phib = (float)p->phi_b;
  k.eta = (float)eta;
  k.k2 = p->model >= 2 ? (float)(3.0 * cs2 * K) : 0.0f;
  k.a = (float)a;
  k.b = (float)b;
  k.omega = (float)(1.0 / p->tau_g);
  k.srcg = (float)(3.0 * (1.0 - 0.5 / p->tau_g));
  k.omega_f = ns ? (float)(1.0 / p->tau_f) : 0.0f;
  k.srcf = ns ? (float)(1.0 - 0.5 / p->tau_f) : 0.0f;
  k.gravity = ns ? (float)p->gravity : 0.0f;
  k.accel_x = ns ? (float)p->accel_x : 0.0f;
  k.rho_mean = (float)(0.5 * (p->rho_a + p->rho_b));
  k.aM = (float)(a * p->mobility);
  k.x_f1 = (float)(2.0 * p->tau_g - 1.0 + 3.0 * K);
  k.x_mu = (float)(3.0 * cs2 * eta * K);

  // Velocity inputs.  u = 0 is served by zero separable tables in the workspace.
  float* z = c->ztab;
  switch (vm) {
    case LBM_CH_VEL_SEPARABLE:
      c->vmode = VEL_SEP;
      c->ax = vel->ax; c->ay = vel->ay; c->bx = vel->bx; c->by = vel->by;
      break;
    case LBM_CH_VEL_FIELD:
      c->vmode = VEL_FIELD;
      c->ux = vel->ux; c->uy = vel->uy;
      break;
    case LBM_CH_VEL_NS:
      c->vmode = VEL_FIELD;  // for the initial state only
      c->ux = vel ? vel->ux : nullptr;
      c->uy = vel ? vel->uy : nullptr;
      break;
    default:
      c->vmode = VEL_SEP;
      c->ax = z; c->ay = z + p->nx; c->bx = z; c->by = z + p->nx;
      break;
  }
  if (vm != LBM_CH_VEL_NS && vel && vel->time_factor && vel->n_time_factor > 0)
    c->tf.assign(vel->time_factor, vel->time_factor + vel->n_time_factor);
  choose_tiles(c);
  c->magic = CTX_MAGIC;

  hipError_t e = launch_fill(z, 0.0f, 2 * (int64_t)(p->nx + p->ny), stream);
  if (e == hipSuccess)
    e = launch_init(p->walls != 0, c->vmode, p->storage, c->c, p->nx, p->ny, L.pitch, phi0,
                    c->ax, c->ay, c->bx, c->by, c->ux, c->uy, time_factor(c, 0), c->g[0],
                    c->f[0], stream);
  if (e != hipSuccess) {
    c->magic = 0;
    (void)hipHostFree(c->nf_host);
    delete c;
    return hip_fail(e);
  }
  if (ns) {
    c->ux = nullptr;
    c->uy = nullptr;
  }
  *out = c;
  return LBM_CH_OK;
}

// nsteps steps; with phi_out, phi^n of step n is also written to phi_out + (n - n0) nx ny.
static int run_steps(lbm_ch_ctx* c, int64_t nsteps, float* phi_out, hipStream_t stream) {
  const bool ns = c->p.velocity_mode == LBM_CH_VEL_NS;
  const bool walls = c->p.walls != 0;
  StepArgs a{};
  a.pitch = c->L.pitch;
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.ty = c->ty;
  a.nstrips = c->nstrips;
  a.xcd_remap = c->xcd_remap;
  a.c = c->c;
  a.ax = c->ax; a.ay = c->ay; a.bx = c->bx; a.by = c->by;
  a.ux = c->ux; a.uy = c->uy;
  a.nonfinite = c->nf_dev;
  NsArgs n{};
  if (ns) {
    n.pitch = c->L.pitch;
    n.nx = c->p.nx;
    n.ny = c->p.ny;
    n.ty = c->ty;
    n.nstrips = c->nstrips;
    n.xcd_remap = c->xcd_remap;
    n.c = c->c;
    n.u = c->u; n.v = c->v; n.p = c->pr;
    a.ux = c->u; a.uy = c->v; a.pf = c->pr;
  }
  const int vmode = ns ? VEL_NSFIELD : c->vmode;
  // Coupled steps of models 1 and 2 run as one launch (f and g together) on output tiles
  // of 64 columns x rows; model 3 keeps the two launches (NS step, then phase field).
  const bool fused = ns && (c->p.model == 1 || c->p.model == 2);
  StepArgs r = a;
  int rt_rows = 0, rt_blocks = 0;
  if (fused) {
    rt_rows = rt_step_rows(c->ty);
    r.nstrips = (c->p.nx + 63) / 64;
    rt_blocks = r.nstrips * ((c->p.ny + rt_rows - 1) / rt_rows);
    r.xcd_remap = rt_blocks % 8 == 0 ? 1 : 0;
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    const int src = c->cur, dst = 1 - c->cur;
    if (fused) {
      float* rec = phi_out ? phi_out + (size_t)s * c->p.nx * c->p.ny : nullptr;
      hipError_t e = hipSuccess;
      if (rec)
        e = launch_phi_field(walls, c->p.storage, c->g[src], c->L.pitch, c->p.nx, c->p.ny,
                             rec, stream);
      if (e == hipSuccess) {
        r.src = c->g[src];
        r.dst = c->g[dst];
        e = launch_rt_step(rt_rows, walls, c->p.model, c->p.storage, r, c->f[src], c->f[dst],
                           rt_blocks, stream);
      }
      if (e != hipSuccess) return hip_fail(e);
      c->cur = dst;
      c->step += 1;
      continue;
    }
    hipError_t e;
    if (ns) {
      n.gsrc = c->g[src];
      n.fsrc = c->f[src];
      n.fdst = c->f[dst];
      e = launch_ns_step(c->tx, walls, c->p.storage, n, c->nblocks, stream);
      if (e != hipSuccess) return hip_fail(e);
      a.tf = 1.0f;
    } else {
      a.tf = time_factor(c, c->step);
    }
    a.src = c->g[src];
    a.dst = c->g[dst];
    a.xh = c->xh;
    a.xfirst = c->step == 0 ? 1 : 0;
    float* rec = phi_out ? phi_out + (size_t)s * c->p.nx * c->p.ny : nullptr;
    if (c->tx == 0) {  // single-pass tiles (record phi themselves with float32 storage)
      e = hipSuccess;
      if (rec && c->p.storage != LBM_CH_STORE_F32)
        e = launch_phi_field(walls, c->p.storage, c->g[src], c->L.pitch, c->p.nx, c->p.ny,
                             rec, stream);
      else
        a.phi_rec = rec;
      if (e == hipSuccess)
        e = launch_phi_pass(c->ty, vmode, c->p.model, c->p.storage, a, c->nblocks, stream);
      a.phi_rec = nullptr;
    } else if (rec && phi_record_fused(walls, vmode, c->p.model, c->p.storage)) {
      // the step writes phi of its source state itself
      a.phi_rec = rec;
      e = launch_phi_record(c->tx, vmode, c->p.model, tau_one(c), a, c->nblocks, stream);
      a.phi_rec = nullptr;
    } else {
      if (rec) {
        e = launch_phi_field(walls, c->p.storage, c->g[src], c->L.pitch, c->p.nx, c->p.ny,
                             rec, stream);
        if (e != hipSuccess) return hip_fail(e);
      }
      e = launch_phi_step(c->tx, walls, vmode, c->p.model, c->p.storage, tau_one(c), a, c->nblocks,
                          stream);
    }
    if (e != hipSuccess) return hip_fail(e);
    c->cur = dst;
    c->step += 1;
  }
  return LBM_CH_OK;
}

extern "C++" {
// Replay of captured launch sequences (lbm_ch_set_graphs).  A sequence is captured once
// per key on the context's own stream and replayed with one graph launch; the key holds
// everything the captured kernel arguments depend on besides the context's fixed
// buffers and launch shape (apply_tiles drops the cache).
static bool same_key(const CtxExec& a, const CtxExec& b) {
  if (a.kind != b.kind || a.n != b.n || a.cur != b.cur) return false;
  for (int i = 0; i < 5; ++i)
    if (a.p[i] != b.p[i]) return false;
  return true;
}

// Launch the cached graph for `key`, or capture `enqueue(stream)` into one and launch it.
// Returns 1 if a cached graph was launched (the caller then applies the host-side effects
// of the sequence itself), 0 if it was captured now (enqueue has applied them), or a
// negative status.
template <class F>
static int graph_run(lbm_ch_ctx* c, CtxExec key, hipStream_t stream, F&& enqueue) {
  for (size_t i = 0; i < c->execs.size(); ++i) {
    if (!same_key(c->execs[i], key)) continue;
    const CtxExec hit = c->execs[i];
    c->execs.erase(c->execs.begin() + (long)i);
    c->execs.push_back(hit);
    const hipError_t e = hipGraphLaunch(hit.exec, stream);
    return e == hipSuccess ? 1 : hip_fail(e);
  }
  hipError_t e = hipSuccess;
  if (!c->cap) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e);
  const int r = enqueue(c->cap);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(c->cap, &graph);
  hipGraphExec_t exec = nullptr;
  if (r == LBM_CH_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (r != LBM_CH_OK) return r;
  if (e != hipSuccess) return hip_fail(e);
  if (c->execs.size() >= 16) {
    (void)hipGraphExecDestroy(c->execs.front().exec);
    c->execs.erase(c->execs.begin());
  }
  key.exec = exec;
  c->execs.push_back(key);
  e = hipGraphLaunch(exec, stream);
  return e == hipSuccess ? 0 : hip_fail(e);
}

// Steps (phi_out: recorded steps) through a graph where the launch arguments do not
// change from step to step: no per-step time-factor table, and past model 3's first step
// (the only one without an earlier history).
static int graph_steps(lbm_ch_ctx* c, int64_t nsteps, float* phi_out, hipStream_t stream) {
  if (!c->graphs || !c->tf.empty() || nsteps == 0) return run_steps(c, nsteps, phi_out, stream);
  if (c->p.model == 3 && c->step == 0) {
    const int r = run_steps(c, 1, phi_out, stream);
    if (r != LBM_CH_OK || nsteps == 1) return r;
    nsteps -= 1;
    if (phi_out) phi_out += (size_t)c->p.nx * c->p.ny;
  }
  CtxExec key{};
  key.kind = phi_out ? 1 : 0;
  key.n = nsteps;
  key.cur = c->cur;
  key.p[0] = phi_out;
  const int cur0 = c->cur;
  const int64_t step0 = c->step;
  const int r = graph_run(c, key, stream, [&](hipStream_t s) { return run_steps(c, nsteps, phi_out, s); });
  if (r == 1) {
    c->cur = cur0 ^ (int)(nsteps & 1);
    c->step = step0 + nsteps;
    return LBM_CH_OK;
  }
  if (r < 0) {  // nothing ran: the captured host-side updates are undone
    c->cur = cur0;
    c->step = step0;
  }
  return r;
}
}  // extern "C++"

// The non-finite flag as the host sees it now (it lands some time after the kernel that
// set it; nothing here waits for the device).
static bool nonfinite_seen(const lbm_ch_ctx* c) {
  return __atomic_load_n(c->nf_host, __ATOMIC_ACQUIRE) != 0;
}

int lbm_ch_step(lbm_ch_ctx* c, int64_t nsteps, hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (nsteps < 0) return LBM_CH_EINVAL;
  if (nonfinite_seen(c)) return LBM_CH_ENONFINITE;
  return graph_steps(c, nsteps, nullptr, stream);
}

int lbm_ch_set_graphs(lbm_ch_ctx* c, int32_t enable) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (enable != 0 && enable != 1) return LBM_CH_EINVAL;
  c->graphs = enable;
  if (!enable) drop_graphs(c);
  return LBM_CH_OK;
}

int lbm_ch_moments(lbm_ch_ctx* c, float* phi, float* mu, float* ux, float* uy, float* p,
                   hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  float* outs[5] = {phi, mu, ux, uy, p};
  for (float* o : outs)
    if (o && !aligned4(o)) return LBM_CH_EINVAL;
  const bool walls = c->p.walls != 0;
  const int nx = c->p.nx, ny = c->p.ny;
  const size_t fb = (size_t)nx * ny * sizeof(float);
  const bool ns = c->p.velocity_mode == LBM_CH_VEL_NS;
  float* ph = phi ? phi : c->phi;
  hipError_t e = hipSuccess;
  if (phi || mu || ns)
    e = launch_phi_field(walls, c->p.storage, c->g[c->cur], c->L.pitch, nx, ny, ph, stream);
  if (e == hipSuccess && mu) e = launch_mu_field(walls, c->c, ph, nx, ny, mu, stream);
  if (e != hipSuccess) return hip_fail(e);
  if (ns) {
    if (ux || uy || p) {
      NsArgs n{};
      n.gsrc = c->g[c->cur];
      n.fsrc = c->f[c->cur];
      n.fdst = nullptr;
      n.u = c->u; n.v = c->v; n.p = c->pr;
      n.pitch = c->L.pitch;
      n.nx = nx; n.ny = ny;
      n.ty = c->ty; n.nstrips = c->nstrips; n.xcd_remap = c->xcd_remap;
      n.c = c->c;
      e = launch_ns_step(c->tx, walls, c->p.storage, n, c->nblocks, stream);
      if (e == hipSuccess && ux) e = hipMemcpyAsync(ux, c->u, fb, hipMemcpyDeviceToDevice, stream);
      if (e == hipSuccess && uy) e = hipMemcpyAsync(uy, c->v, fb, hipMemcpyDeviceToDevice, stream);
      if (e == hipSuccess && p) e = hipMemcpyAsync(p, c->pr, fb, hipMemcpyDeviceToDevice, stream);
    }
  } else {
    if (ux || uy)
      e = launch_velocity_field(c->vmode, nx, ny, c->ax, c->ay, c->bx, c->by, c->ux, c->uy,
                                time_factor(c, c->step), ux, uy, stream);
    if (e == hipSuccess && p) e = launch_fill(p, 0.0f, (int64_t)nx * ny, stream);
  }
  return e == hipSuccess ? LBM_CH_OK : hip_fail(e);
}

int lbm_ch_diagnostics(lbm_ch_ctx* c, const float* phi_ref, double* out, hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (!out || ((uintptr_t)out & 7u) != 0) return LBM_CH_EINVAL;
  if (phi_ref && !aligned4(phi_ref)) return LBM_CH_EINVAL;
  const bool walls = c->p.walls != 0;
  hipError_t e = launch_phi_field(walls, c->p.storage, c->g[c->cur], c->L.pitch, c->p.nx,
                                  c->p.ny, c->phi, stream);
  if (e == hipSuccess)
    e = launch_diag(walls, c->c, c->phi, phi_ref, c->p.nx, c->p.ny, c->part, out, stream);
  return e == hipSuccess ? LBM_CH_OK : hip_fail(e);
}

int lbm_ch_check_finite(lbm_ch_ctx* c, hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  int r = lbm_ch_diagnostics(c, nullptr, c->diag, stream);
  if (r != LBM_CH_OK) return r;
  double h[8];
  hipError_t e = hipMemcpyAsync(h, c->diag, sizeof(h), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e);
  return h[7] > 0 ? LBM_CH_ENONFINITE : LBM_CH_OK;
}

int64_t lbm_ch_step_count(const lbm_ch_ctx* c) { return live(c) ? c->step : -1; }

size_t lbm_ch_state_bytes(const lbm_ch_ctx* c) {
  if (!live(c)) return 0;
  const size_t f = c->L.f_state;
  const size_t x = (size_t)2 * c->p.nx * c->p.ny * sizeof(float);
  return c->L.g_state + (c->p.velocity_mode == LBM_CH_VEL_NS ? f : 0) + (c->xh ? x : 0);
}

int lbm_ch_save_state(lbm_ch_ctx* c, void* dst, size_t bytes, hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (!dst || bytes != lbm_ch_state_bytes(c)) return LBM_CH_EINVAL;
  const size_t g = c->L.g_state, f = c->L.f_state;
  const size_t fo = c->f[0] ? f : 0, x = (size_t)2 * c->p.nx * c->p.ny * sizeof(float);
  hipError_t e = hipMemcpyAsync(dst, c->g[c->cur], g, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && c->f[0])
    e = hipMemcpyAsync((char*)dst + g, c->f[c->cur], f, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && c->xh)
    e = hipMemcpyAsync((char*)dst + g + fo, c->xh, x, hipMemcpyDeviceToDevice, stream);
  return e == hipSuccess ? LBM_CH_OK : hip_fail(e);
}

int lbm_ch_load_state(lbm_ch_ctx* c, const void* src, size_t bytes, int64_t step,
                      hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (!src || bytes != lbm_ch_state_bytes(c) || step < 0) return LBM_CH_EINVAL;
  __atomic_store_n(c->nf_host, 0, __ATOMIC_RELEASE);  // a new state: forget earlier NaNs
  const size_t g = c->L.g_state, f = c->L.f_state;
  const size_t fo = c->f[0] ? f : 0, x = (size_t)2 * c->p.nx * c->p.ny * sizeof(float);
  hipError_t e = hipMemcpyAsync(c->g[c->cur], src, g, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && c->f[0])
    e = hipMemcpyAsync(c->f[c->cur], (const char*)src + g, f, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && c->xh)
    e = hipMemcpyAsync(c->xh, (const char*)src + g + fo, x, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(e);
  c->step = step;
  return LBM_CH_OK;
}

int lbm_ch_set_tiles(lbm_ch_ctx* c, int32_t tx, int32_t ty) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (tx == 0) {
    if (!pass_eligible(c->p) || (ty != 4 && ty != 8 && ty != 16)) return LBM_CH_EINVAL;
  } else if (!valid_tile(tx, ty)) {
    return LBM_CH_EINVAL;
  }
  apply_tiles(c, tx, ty);
  return LBM_CH_OK;
}

int lbm_ch_default_tiles(const lbm_ch_params* p, int32_t* tx, int32_t* ty) {
  if (!tx || !ty || !valid_params(p)) return LBM_CH_EINVAL;
  int x, y;
  default_tiles(*p, x, y);
  *tx = x;
  *ty = (x != 0 && y > p->ny) ? p->ny : y;  // single-pass rows are a kernel constant
  return LBM_CH_OK;
}

int lbm_ch_get_tiles(const lbm_ch_ctx* c, int32_t* tx, int32_t* ty) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (!tx || !ty) return LBM_CH_EINVAL;
  *tx = c->tx;
  *ty = c->ty;
  return LBM_CH_OK;
}

int lbm_ch_autotune(lbm_ch_ctx* c, void* backup, size_t backup_bytes, int32_t trial_steps,
                    hipStream_t stream, float* best_us) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (!backup || backup_bytes != lbm_ch_state_bytes(c) || trial_steps < 1)
    return LBM_CH_EINVAL;
  const int64_t step0 = c->step;
  const int tx0 = c->tx, ty0 = c->ty;
  int r = lbm_ch_save_state(c, backup, backup_bytes, stream);
  if (r != LBM_CH_OK) return r;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = -1.0f;
  int btx = tx0, bty = ty0;
  const int nx = c->p.nx, ny = c->p.ny;
  const bool pass = pass_eligible(c->p);
  for (int xx : {0, 64, 128, 256, 512}) {
    if (e != hipSuccess) break;
    if (xx == 0 && !pass) continue;
    if (xx > 64 && xx / 2 >= nx) continue;  // more than half the lanes idle
    for (int yy : {1, 2, 4, 8, 16, 32}) {
      if (xx == 0 && yy != 4 && yy != 8 && yy != 16) continue;
      if (yy > ny && yy > 2) continue;
      apply_tiles(c, xx, yy);
      r = run_steps(c, 1, nullptr, stream);  // untimed: first launch of this kernel shape
      if (r == LBM_CH_OK) {
        e = hipEventRecord(e0, stream);
        if (e == hipSuccess) r = run_steps(c, trial_steps, nullptr, stream);
        if (e == hipSuccess && r == LBM_CH_OK) e = hipEventRecord(e1, stream);
        if (e == hipSuccess && r == LBM_CH_OK) e = hipEventSynchronize(e1);
      }
      float ms = 0.0f;
      if (e == hipSuccess && r == LBM_CH_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess || r != LBM_CH_OK) break;
      if (best < 0.0f || ms < best) {
        best = ms;
        btx = xx;
        bty = yy;
      }
    }
    if (r != LBM_CH_OK) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // restore the state and the step counter whatever happened above
  apply_tiles(c, (e == hipSuccess && r == LBM_CH_OK) ? btx : tx0,
              (e == hipSuccess && r == LBM_CH_OK) ? bty : ty0);
  const int r2 = lbm_ch_load_state(c, backup, backup_bytes, step0, stream);
  if (e != hipSuccess) return hip_fail(e);
  if (r != LBM_CH_OK) return r;
  if (best_us) *best_us = best * 1000.0f / (float)trial_steps;
  return r2;
}

size_t lbm_ch_adjoint_scratch_bytes(const lbm_ch_params* p) {
  if (!valid_params(p)) return 0;
  return (size_t)p->nx * p->ny * sizeof(float);
}

int lbm_ch_record(lbm_ch_ctx* c, int64_t nsteps, float* phi_traj, hipStream_t stream) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (nsteps < 0) return LBM_CH_EINVAL;
  if (nonfinite_seen(c)) return LBM_CH_ENONFINITE;
  if (nsteps == 0) return LBM_CH_OK;
  if (!phi_traj || !aligned4(phi_traj)) return LBM_CH_EINVAL;
  return graph_steps(c, nsteps, phi_traj, stream);
}

// Checks shared by lbm_ch_adjoint and lbm_ch_adjoint_static (scratch aside).
static int adjoint_check(const lbm_ch_ctx* c, int64_t n_end, int64_t nsteps,
                         const float* phi_traj, const float* lam, const float* grad_u,
                         const float* grad_v) {
  if (!live(c)) return LBM_CH_ESTATE;
  if (c->p.tau_g != 1.0 || c->p.walls != 0 || c->p.velocity_mode == LBM_CH_VEL_NS ||
      c->p.model == 3)
    return LBM_CH_EUNSUPPORTED;
  if (nsteps < 0 || n_end < nsteps) return LBM_CH_EINVAL;
  if (nsteps == 0) return LBM_CH_OK;
  if (!phi_traj || !lam || !aligned4(phi_traj) || !aligned4(lam)) return LBM_CH_EINVAL;
  if ((grad_u == nullptr) != (grad_v == nullptr)) return LBM_CH_EINVAL;
  if (grad_u && (!aligned4(grad_u) || !aligned4(grad_v))) return LBM_CH_EINVAL;
  return LBM_CH_OK;
}

// The reverse steps n_end - 1 .. n_end - nsteps, lam and `scratch` (nx*ny floats)
// alternating as source and destination; lam holds the result.
static int adjoint_enqueue(lbm_ch_ctx* c, int64_t n_end, int64_t nsteps, const float* phi_traj,
                           float* lam, float* grad_u, float* grad_v, float* scratch,
                           hipStream_t s) {
  const size_t nodes = (size_t)c->p.nx * c->p.ny;
  float* buf[2] = {lam, scratch};
  int cur = 0;
  for (int64_t k = nsteps - 1; k >= 0; --k) {
    const int64_t n = n_end - nsteps + k;
    hipError_t e = launch_adjoint_step(
        c->c, (float)c->p.mobility, c->p.nx, c->p.ny, c->vmode, c->ax, c->ay, c->bx, c->by,
        c->ux, c->uy, time_factor(c, n), phi_traj + (size_t)k * nodes, buf[cur],
        buf[cur ^ 1], grad_u, grad_v, s);
    if (e != hipSuccess) return hip_fail(e);
    cur ^= 1;
  }
  if (cur != 0) {
    hipError_t e = hipMemcpyAsync(lam, scratch, nodes * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  return LBM_CH_OK;
}

int lbm_ch_adjoint(lbm_ch_ctx* c, int64_t n_end, int64_t nsteps, const float* phi_traj,
                   float* lam, float* grad_u, float* grad_v, void* scratch,
                   size_t scratch_bytes, hipStream_t stream) {
  int r = adjoint_check(c, n_end, nsteps, phi_traj, lam, grad_u, grad_v);
  if (r != LBM_CH_OK || nsteps == 0) return r;
  if (!scratch || !aligned4(scratch) || scratch_bytes < lbm_ch_adjoint_scratch_bytes(&c->p))
    return LBM_CH_EINVAL;
  auto enqueue = [&](hipStream_t s) -> int {
    return adjoint_enqueue(c, n_end, nsteps, phi_traj, lam, grad_u, grad_v, (float*)scratch, s);
  };
  // the reverse steps of a steady velocity depend on n_end only through the trajectory
  if (!c->graphs || !c->tf.empty()) return enqueue(stream);
  CtxExec key{};
  key.kind = 2;
  key.n = nsteps;
  key.p[0] = phi_traj;
  key.p[1] = lam;
  key.p[2] = grad_u;
  key.p[3] = grad_v;
  key.p[4] = scratch;
  r = graph_run(c, key, stream, enqueue);
  return r > 0 ? LBM_CH_OK : r;
}

int lbm_ch_adjoint_static(lbm_ch_ctx* c, int64_t n_end, int64_t nsteps, const float* phi_traj,
                          float* lam, float* grad_u, float* grad_v, hipStream_t stream) {
  int r = adjoint_check(c, n_end, nsteps, phi_traj, lam, grad_u, grad_v);
  if (r != LBM_CH_OK || nsteps == 0) return r;
  static_assert(ADJ_STATIC_MAX_NODES == LBM_CH_ADJOINT_STATIC_MAX_NODES, "header limit");
  if ((size_t)c->p.nx * c->p.ny > ADJ_STATIC_MAX_NODES) return LBM_CH_EINVAL;
  float* ptr = static_scratch(c->device);  // set up by lbm_ch_init on this device
  if (!ptr) return LBM_CH_ESTATE;
  // plain launches only: no graph capture, which creates streams and graphs
  return adjoint_enqueue(c, n_end, nsteps, phi_traj, lam, grad_u, grad_v, ptr, stream);
}

int lbm_ch_destroy(lbm_ch_ctx* c) {
  if (!c) return LBM_CH_OK;
  if (!live(c)) return LBM_CH_ESTATE;
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  (void)hipHostFree(c->nf_host);
  c->magic = 0;
  delete c;
  return LBM_CH_OK;
}

const char* lbm_ch_strerror(int status) {
  switch (status) {
    case LBM_CH_OK: return "ok";
    case LBM_CH_EINVAL: return "invalid argument";
    case LBM_CH_EUNSUPPORTED: return "unsupported combination";
    case LBM_CH_EHIP: return "HIP runtime error";
    case LBM_CH_ENONFINITE: return "non-finite order parameter";
    case LBM_CH_ESTATE: return "invalid or destroyed context";
    default: return "unknown status";
  }
}

int lbm_ch_last_hip_error(void) { return g_last_hip; }

}  // extern "C"

// ---------------------------------------------------------------------------------
// Batched stepping of many lattices.
namespace {

struct BatchGroup {
  int tx, vmode;
  bool model2;
  bool t1;           // tau_g = 1 tile
  int first, count;  // range in the instance order
  int start_off;     // offset of this group's start[] in the device start array
  int total, grid;
};

struct BatchExec {
  hipGraphExec_t exec;
  int64_t steps;
  int phase;
};

constexpr uint32_t BATCH_MAGIC = 0x4c424d42u;

}  // namespace

struct lbm_ch_batch {
  std::vector<lbm_ch_ctx*> ctx;
  StepArgs* dargs;
  int* dstart;
  std::vector<StepArgs> hargs;
  std::vector<int> hstart;
  std::vector<int> built_cur;  // ctx->cur of each instance when the tables were built
  std::vector<BatchGroup> groups;
  int tx_policy;  // 0: per-instance width, else one width for all
  int ty;
  int persistent; // 1: a resident-size grid strides over the tiles; 0: a tile per workgroup
  int phase;      // steps taken since the tables were built, mod 2
  bool built;
  int cus;
  hipStream_t cap;
  std::vector<BatchExec> execs;
  uint32_t magic;
};

static bool batch_live(const lbm_ch_batch* b) { return b && b->magic == BATCH_MAGIC; }

static size_t batch_table_bytes(int32_t n) {
  return align_up((size_t)n * sizeof(StepArgs)) + align_up((size_t)(2 * n + 1) * sizeof(int));
}

// Width of instance tiles: the policy's width, or (policy 0) the widest of 256, 128, 64
// that leaves the fewest idle lanes in the last strip.
static int batch_tx(int policy, int nx) {
  if (policy) return policy;
  int best = 64, idle = 1 << 30;
  for (int tx : {256, 128, 64}) {
    const int w = (nx + tx - 1) / tx * tx - nx;
    if (w < idle) {
      idle = w;
      best = tx;
    }
  }
  return best;
}

static void batch_drop_graphs(lbm_ch_batch* b) {
  for (auto& x : b->execs) (void)hipGraphExecDestroy(x.exec);
  b->execs.clear();
}

// Rebuild the instance tables (grouped by kernel variant) and upload them on `stream`.
static int batch_build(lbm_ch_batch* b, hipStream_t stream) {
  const int n = (int)b->ctx.size();
  // the host tables may still be read by an earlier upload
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e);
  batch_drop_graphs(b);
  std::vector<int> order(n), txs(n);
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    txs[i] = batch_tx(b->tx_policy, b->ctx[i]->p.nx);
  }
  auto key = [&](int i) {
    const lbm_ch_ctx* c = b->ctx[i];
    return txs[i] * 32 + c->vmode * 4 + (c->p.model == 2 ? 2 : 0) + (tau_one(c) ? 1 : 0);
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
  b->hargs.assign(n, StepArgs{});
  b->hstart.clear();
  b->groups.clear();
  b->built_cur.assign(n, 0);
  for (int k = 0; k < n; ++k) {
    const int i = order[k];
    lbm_ch_ctx* c = b->ctx[i];
    if (b->groups.empty() || key(order[b->groups.back().first]) != key(i)) {
      if (!b->groups.empty()) b->hstart.push_back(b->groups.back().total);
      BatchGroup g{};
      g.tx = txs[i];
      g.vmode = c->vmode;
      g.model2 = c->p.model == 2;
      g.t1 = tau_one(c);
      g.first = k;
      g.start_off = (int)b->hstart.size();
      b->groups.push_back(g);
    }
    BatchGroup& g = b->groups.back();
    const int ty = b->ty < c->p.ny ? b->ty : c->p.ny;
    StepArgs& a = b->hargs[k];
    a.src = c->g[c->cur];
    a.dst = c->g[1 - c->cur];
    a.pitch = c->L.pitch;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.ty = ty;
    a.nstrips = (c->p.nx + g.tx - 1) / g.tx;
    a.xcd_remap = 0;
    a.c = c->c;
    a.ax = c->ax; a.ay = c->ay; a.bx = c->bx; a.by = c->by;
    a.ux = c->ux; a.uy = c->uy;
    a.tf = time_factor(c, c->step);
    a.nonfinite = c->nf_dev;
    b->built_cur[i] = c->cur;
    b->hstart.push_back(g.total);
    g.total += a.nstrips * ((c->p.ny + ty - 1) / ty);
    g.count += 1;
  }
  b->hstart.push_back(b->groups.back().total);
  for (BatchGroup& g : b->groups) {
    const int want = (g.total + 7) / 8 * 8;
    if (b->persistent) {
      const int per_cu = phi_batch_blocks_per_cu(g.tx, g.vmode, g.model2, g.t1);
      const int resident = b->cus * per_cu / 8 * 8;
      g.grid = want < resident ? want : (resident > 8 ? resident : 8);
    } else {
      g.grid = want;
    }
  }
  e = hipMemcpyAsync(b->dargs, b->hargs.data(), n * sizeof(StepArgs), hipMemcpyHostToDevice,
                     stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->dstart, b->hstart.data(), b->hstart.size() * sizeof(int),
                       hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e);
  b->phase = 0;
  b->built = true;
  return LBM_CH_OK;
}

static int batch_prepare(lbm_ch_batch* b, hipStream_t stream) {
  bool stale = !b->built;
  for (size_t i = 0; i < b->ctx.size() && !stale; ++i) {
    if (!live(b->ctx[i])) return LBM_CH_ESTATE;
    stale = b->ctx[i]->cur != (b->built_cur[i] ^ b->phase);
  }
  for (lbm_ch_ctx* c : b->ctx)
    if (!live(c)) return LBM_CH_ESTATE;
  return stale ? batch_build(b, stream) : LBM_CH_OK;
}

static hipError_t batch_enqueue(lbm_ch_batch* b, int64_t nsteps, int phase, hipStream_t s) {
  for (int64_t k = 0; k < nsteps; ++k) {
    for (const BatchGroup& g : b->groups) {
      BatchArgs a{};
      a.args = b->dargs + g.first;
      a.start = b->dstart + g.start_off;
      a.n = g.count;
      a.total = g.total;
      a.parity = (int)((phase + k) & 1);
      hipError_t e = launch_phi_batch(g.tx, g.vmode, g.model2, g.t1, b->persistent != 0, a, g.grid, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

static void batch_advance(lbm_ch_batch* b, int64_t nsteps) {
  for (lbm_ch_ctx* c : b->ctx) {
    if (nsteps & 1) c->cur = 1 - c->cur;
    c->step += nsteps;
  }
  b->phase = (int)((b->phase + nsteps) & 1);
}

extern "C" {

size_t lbm_ch_batch_workspace_bytes(int32_t n) {
  return n >= 1 ? batch_table_bytes(n) : 0;
}

int lbm_ch_batch_create(lbm_ch_batch** out, lbm_ch_ctx* const* ctxs, int32_t n,
                        void* workspace, size_t workspace_bytes) {
  if (!out) return LBM_CH_EINVAL;
  *out = nullptr;
  if (!ctxs || n < 1) return LBM_CH_EINVAL;
  if (!workspace || ((uintptr_t)workspace % ALIGN) != 0 ||
      workspace_bytes < batch_table_bytes(n))
    return LBM_CH_EINVAL;
  for (int32_t i = 0; i < n; ++i) {
    const lbm_ch_ctx* c = ctxs[i];
    if (!live(c)) return LBM_CH_ESTATE;
    for (int32_t j = 0; j < i; ++j)
      if (ctxs[j] == c) return LBM_CH_EINVAL;
    if (c->p.walls != 0 || c->p.storage != LBM_CH_STORE_F32 || c->p.model == 3 ||
        c->p.velocity_mode == LBM_CH_VEL_NS || !c->tf.empty())
      return LBM_CH_EUNSUPPORTED;
  }
  int cus = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e);
  lbm_ch_batch* b = new (std::nothrow) lbm_ch_batch();
  if (!b) return LBM_CH_EINVAL;
  b->ctx.assign(ctxs, ctxs + n);
  b->dargs = (StepArgs*)workspace;
  b->dstart = (int*)((char*)workspace + align_up((size_t)n * sizeof(StepArgs)));
  b->tx_policy = 64;
  b->ty = 16;
  b->persistent = 0;
  b->phase = 0;
  b->built = false;
  b->cus = cus > 0 ? cus : 1;
  e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e);
  }
  b->magic = BATCH_MAGIC;
  *out = b;
  return LBM_CH_OK;
}

int lbm_ch_batch_set_tiles(lbm_ch_batch* b, int32_t tx, int32_t ty) {
  if (!batch_live(b)) return LBM_CH_ESTATE;
  if (!(tx == 0 || (valid_tile(tx, 1) && tx <= 256)) || ty < 1) return LBM_CH_EINVAL;
  b->tx_policy = tx;
  b->ty = ty;
  b->built = false;
  return LBM_CH_OK;
}

int lbm_ch_batch_set_schedule(lbm_ch_batch* b, int32_t persistent) {
  if (!batch_live(b)) return LBM_CH_ESTATE;
  if (persistent != 0 && persistent != 1) return LBM_CH_EINVAL;
  b->persistent = persistent;
  b->built = false;
  return LBM_CH_OK;
}

int lbm_ch_batch_get_schedule(const lbm_ch_batch* b) {
  return batch_live(b) ? b->persistent : LBM_CH_ESTATE;
}

int lbm_ch_batch_get_tiles(const lbm_ch_batch* b, int32_t* tx, int32_t* ty) {
  if (!batch_live(b)) return LBM_CH_ESTATE;
  if (!tx || !ty) return LBM_CH_EINVAL;
  *tx = b->tx_policy;
  *ty = b->ty;
  return LBM_CH_OK;
}

int lbm_ch_batch_step(lbm_ch_batch* b, int64_t nsteps, int32_t use_graph, hipStream_t stream) {
  if (!batch_live(b)) return LBM_CH_ESTATE;
  if (nsteps < 0) return LBM_CH_EINVAL;
  for (const lbm_ch_ctx* m : b->ctx)
    if (live(m) && nonfinite_seen(m)) return LBM_CH_ENONFINITE;
  int r = batch_prepare(b, stream);
  if (r != LBM_CH_OK || nsteps == 0) return r;
  if (!use_graph) {
    hipError_t e = batch_enqueue(b, nsteps, b->phase, stream);
    if (e != hipSuccess) return hip_fail(e);
    batch_advance(b, nsteps);
    return LBM_CH_OK;
  }
  hipGraphExec_t exec = nullptr;
  for (const BatchExec& x : b->execs)
    if (x.steps == nsteps && x.phase == b->phase) exec = x.exec;
  if (!exec) {
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e);
    hipError_t el = batch_enqueue(b, nsteps, b->phase, b->cap);
    e = hipStreamEndCapture(b->cap, &graph);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e);
    if (b->execs.size() >= 4) {
      (void)hipGraphExecDestroy(b->execs.front().exec);
      b->execs.erase(b->execs.begin());
    }
    b->execs.push_back(BatchExec{exec, nsteps, b->phase});
  }
  hipError_t e = hipGraphLaunch(exec, stream);
  if (e != hipSuccess) return hip_fail(e);
  batch_advance(b, nsteps);
  return LBM_CH_OK;
}

size_t lbm_ch_batch_state_bytes(const lbm_ch_batch* b) {
  if (!batch_live(b)) return 0;
  size_t total = 0;
  for (const lbm_ch_ctx* c : b->ctx) total += align_up(lbm_ch_state_bytes(c));
  return total;
}

int lbm_ch_batch_autotune(lbm_ch_batch* b, void* backup, size_t backup_bytes,
                          int32_t trial_steps, hipStream_t stream, float* best_us) {
  if (!batch_live(b)) return LBM_CH_ESTATE;
  for (lbm_ch_ctx* c : b->ctx)
    if (!live(c)) return LBM_CH_ESTATE;
  if (!backup || ((uintptr_t)backup % ALIGN) != 0 ||
      backup_bytes != lbm_ch_batch_state_bytes(b) || trial_steps < 1)
    return LBM_CH_EINVAL;
  std::vector<int64_t> step0;
  size_t off = 0;
  for (lbm_ch_ctx* c : b->ctx) {
    step0.push_back(c->step);
    const int r = lbm_ch_save_state(c, (char*)backup + off, lbm_ch_state_bytes(c), stream);
    if (r != LBM_CH_OK) return r;
    off += align_up(lbm_ch_state_bytes(c));
  }
  const int tx0 = b->tx_policy, ty0 = b->ty, pe0 = b->persistent;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int r = LBM_CH_OK;
  float best = -1.0f;
  int btx = tx0, bty = ty0, bpe = pe0;
  for (int pe : {0, 1})
  for (int xx : {0, 64, 128, 256}) {
    for (int yy : {4, 8, 16, 32}) {
      if (e != hipSuccess || r != LBM_CH_OK) break;
      b->persistent = pe;
      b->tx_policy = xx;
      b->ty = yy;
      b->built = false;
      r = lbm_ch_batch_step(b, 1, 0, stream);  // rebuilds the tables; untimed
      if (r != LBM_CH_OK) break;
      e = hipEventRecord(e0, stream);
      if (e == hipSuccess) r = lbm_ch_batch_step(b, trial_steps, 0, stream);
      if (e == hipSuccess && r == LBM_CH_OK) e = hipEventRecord(e1, stream);
      if (e == hipSuccess && r == LBM_CH_OK) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess && r == LBM_CH_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && r == LBM_CH_OK && (best < 0.0f || ms < best)) {
        best = ms;
        btx = xx;
        bty = yy;
        bpe = pe;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const bool ok = e == hipSuccess && r == LBM_CH_OK;
  b->tx_policy = ok ? btx : tx0;
  b->ty = ok ? bty : ty0;
  b->persistent = ok ? bpe : pe0;
  b->built = false;
  off = 0;
  int r2 = LBM_CH_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    lbm_ch_ctx* c = b->ctx[i];
    const int ri = lbm_ch_load_state(c, (char*)backup + off, lbm_ch_state_bytes(c), step0[i],
                                     stream);
    if (ri != LBM_CH_OK) r2 = ri;
    off += align_up(lbm_ch_state_bytes(c));
  }
  if (e != hipSuccess) return hip_fail(e);
  if (r != LBM_CH_OK) return r;
  if (best_us && ok) *best_us = best * 1000.0f / (float)trial_steps;
  return r2;
}

int lbm_ch_batch_destroy(lbm_ch_batch* b) {
  if (!b) return LBM_CH_OK;
  if (!batch_live(b)) return LBM_CH_ESTATE;
  batch_drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->magic = 0;
  delete b;
  return LBM_CH_OK;
}

}  // extern "C"
