// gfx950 kernels of the lattice Boltzmann Cahn-Hilliard solver outside the time
// step: the initial state, macroscopic fields, FP64 diagnostics and the discrete
// adjoint of the tau_g = 1 step.  The fused step kernels are in lbm_ch_step.hip.
#include "lbm_ch_device.h"

#include <mutex>

namespace lbmch {
namespace {

// ---------------------------------------------------------------------------------
// Initial state: g = g^eq(phi0, mu[phi0], u(t0)); with NS f = f^eq(0, rho(phi0), u0).
template <bool WALLS>
__device__ __forceinline__ float field_at(const float* f, int nx, int ny, int x, int y) {
  x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
  float sg;
  y = row_of<WALLS>(y, ny, sg);
  return f[(uint32_t)y * nx + x];
}

template <bool WALLS>
__device__ __forceinline__ void stencil_at(const float* f, int nx, int ny, int x, int y,
                                           float& gx, float& gy, float& lap) {
  float v[3][3];
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) v[dy + 1][dx + 1] = field_at<WALLS>(f, nx, ny, x + dx, y + dy);
  gx = ddx(v[0], v[1], v[2], 1);
  gy = ddy(v[0], v[1], v[2], 1);
  lap = lap9(v[0], v[1], v[2], 1);
}

// The stored buffer holds post-collision populations, which the next step pulls:
// g_i(y) = stored_i(y - c_i), or stored_opp(i)(y) when y - c_i lies beyond a wall.
// The initial state is written in that form, so that the first pull returns
// g_i = g_i^eq(phi0, mu[phi0], u(t0)) (and f_i = f_i^eq(0, rho(phi0), u0)) at every node.
template <bool WALLS>
__device__ __forceinline__ void push_target(int nx, int ny, int x, int y, int i, int& pop_i,
                                            uint32_t& col, uint32_t& row) {
  int ty = y - CY[i];
  if (WALLS && (ty < 0 || ty >= ny)) {
    constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    pop_i = OPP[i];
    col = (uint32_t)x;
    row = (uint32_t)y;
    return;
  }
  int tx = x - CX[i];
  tx = tx < 0 ? tx + nx : (tx >= nx ? tx - nx : tx);
  ty = ty < 0 ? ty + ny : (ty >= ny ? ty - ny : ty);
  pop_i = i;
  col = (uint32_t)tx;
  row = (uint32_t)ty;
}

template <bool WALLS, int VMODE, int ST>
__global__ void __launch_bounds__(256) k_init(const Coef c, int nx, int ny, uint32_t pitch,
                                              const float* __restrict__ phi0, const float* ax,
                                              const float* ay, const float* bx, const float* by,
                                              const float* ux, const float* uy, float tf,
                                              char* __restrict__ g, float* __restrict__ f) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= nx) return;
  const uint32_t k = (uint32_t)y * nx + x;
  float gx, gy, lap;
  stencil_at<WALLS>(phi0, nx, ny, x, y, gx, gy, lap);
  const float phi = phi0[k];
  const float mu = mu_bulk(c, phi) - c.kappa * lap;
  float u = 0.f, v = 0.f;
  if (VMODE == VEL_SEP) {
    u = tf * ax[x] * ay[y];
    v = tf * bx[x] * by[y];
  } else if (ux) {
    u = tf * ux[k];
    v = tf * uy[k];
  }
  // g^eq of Eq. geq (no source term); g_0 through sum_i g_i^eq = phi as in the step
  const float em = c.eta * mu, usq15 = 1.5f * (u * u + v * v), A = em - phi * usq15;
  float geq[9];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float cu = CX[i] * u + CY[i] * v;
    geq[i] = WT[i] * (A + phi * cu * (3.0f + 4.5f * cu));
  }
  uint32_t h[9];
  if (ST == ST_F32) {
    close_mass((double)phi, geq);
  } else {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      h[i] = enc16<ST>(geq[i] * INV_W[i]);
      geq[i] = WT[i] * dec16<ST>(h[i]);
    }
    geq[0] = (float)((double)phi - sum8_hi(geq));
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int pi;
    uint32_t col, row;
    push_target<WALLS>(nx, ny, x, y, i, pi, col, row);
    if (ST == ST_F32 || pi == 0)
      *reinterpret_cast<float*>(g + pop_off<ST>(pi, pitch, row) + 4u * col) = geq[i];
    else
      *reinterpret_cast<unsigned short*>(g + pop_off<ST>(pi, pitch, row) + 2u * col) =
          (unsigned short)h[i];
  }
  if (f) {
    const float rho = c.a * phi + c.b;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cu = CX[i] * u + CY[i] * v;
      int pi;
      uint32_t col, row;
      push_target<WALLS>(nx, ny, x, y, i, pi, col, row);
      f[pop_off<ST_F32>(pi, pitch, row) / 4u + col] = WT[i] * rho * (cu * (3.0f + 4.5f * cu) - usq15);
    }
  }
}

template <bool WALLS, int ST>
__global__ void __launch_bounds__(256) k_phi_field(const void* __restrict__ g, uint32_t pitch,
                                                   int nx, int ny, float* __restrict__ phi) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= nx) return;
  float p[9];
  pull9<WALLS, ST>(make_rsrc(g, pop_bytes(ST, pitch, ny)), pitch, ny, y, x,
                   x == 0 ? nx - 1 : x - 1, x == nx - 1 ? 0 : x + 1, p);
  phi[(uint32_t)y * nx + x] = sum9(p);
}

template <bool WALLS>
__global__ void __launch_bounds__(256) k_mu_field(const Coef c, const float* __restrict__ phi,
                                                  int nx, int ny, float* __restrict__ mu) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= nx) return;
  float gx, gy, lap;
  stencil_at<WALLS>(phi, nx, ny, x, y, gx, gy, lap);
  mu[(uint32_t)y * nx + x] = mu_bulk(c, phi[(uint32_t)y * nx + x]) - c.kappa * lap;
}

__global__ void __launch_bounds__(256) k_velocity(int vmode, int nx, int ny, const float* ax,
                                                  const float* ay, const float* bx,
                                                  const float* by, const float* ux,
                                                  const float* uy, float tf, float* u,
                                                  float* v) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= nx || y >= ny) return;
  const uint32_t k = (uint32_t)y * nx + x;
  if (vmode == VEL_SEP) {
    if (u) u[k] = tf * ax[x] * ay[y];
    if (v) v[k] = tf * bx[x] * by[y];
  } else {
    if (u) u[k] = ux ? tf * ux[k] : 0.0f;
    if (v) v[k] = uy ? tf * uy[k] : 0.0f;
  }
}

__global__ void __launch_bounds__(256) k_fill(float* d, float value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = value;
}

// ---------------------------------------------------------------------------------
// FP64 diagnostics: a fixed grid of blocks, each thread a fixed strided set of nodes;
// each wavefront reduces its 64 lanes with cross-lane DPP moves (xor 1, xor 2 within
// quads, then the mirrors of 8 and 16 lanes, which leave every lane of a row of 16 with
// the row's value) and combines its four rows through readlane; the four wavefronts
// of a block meet in LDS, and one final block reduces the block partials the same way.
// Every combination happens in a fixed order: bitwise reproducible.
constexpr int DIAG_BLOCKS = 512;
constexpr int DIAG_THREADS = 256;
constexpr int DIAG_WAVES = DIAG_THREADS / 64;
constexpr int NDIAG = 8;

// Reduction operator of diagnostic q: sums, except the maximum (q = 5) and minimum (6).
__device__ __forceinline__ double diag_op(int q, double a, double b) {
  return q == 5 ? fmax(a, b) : (q == 6 ? fmin(a, b) : a + b);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// Value of diagnostic q over the 64 lanes of the calling wavefront (all lanes active).
__device__ __forceinline__ double wave_reduce(int q, double v) {
  v = diag_op(q, v, dpp_d<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = diag_op(q, v, dpp_d<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = diag_op(q, v, dpp_d<0x141>(v));  // row_half_mirror
  v = diag_op(q, v, dpp_d<0x140>(v));  // row_mirror
  return diag_op(q, diag_op(q, readlane_d(v, 0), readlane_d(v, 16)),
                 diag_op(q, readlane_d(v, 32), readlane_d(v, 48)));
}
// Block reduction of acc[NDIAG] (every thread of a DIAG_THREADS block calls it): the
// result is in threads 0 .. NDIAG-1 (thread q holds diagnostic q).
__device__ __forceinline__ double block_reduce(double acc[NDIAG], double (*sh)[DIAG_WAVES]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NDIAG; ++q) {
    const double w = wave_reduce(q, acc[q]);
    if (lane == 0) sh[q][wave] = w;
  }
  __syncthreads();
  double r = 0.0;
  if ((int)threadIdx.x < NDIAG) {
    const int q = threadIdx.x;
    r = sh[q][0];
#pragma unroll
    for (int w = 1; w < DIAG_WAVES; ++w) r = diag_op(q, r, sh[q][w]);
  }
  return r;
}

template <bool WALLS>
__global__ void __launch_bounds__(DIAG_THREADS) k_diag_partial(const Coef c,
                                                               const float* __restrict__ phi,
                                                               const float* __restrict__ ref,
                                                               int nx, int ny,
                                                               double* __restrict__ part) {
  __shared__ double sh[NDIAG][DIAG_WAVES];
  double acc[NDIAG] = {0, 0, 0, 0, 0, -INFINITY, INFINITY, 0};
  const int64_t n = (int64_t)nx * ny;
  for (int64_t k = (int64_t)blockIdx.x * DIAG_THREADS + threadIdx.x; k < n;
       k += (int64_t)DIAG_BLOCKS * DIAG_THREADS) {
    const float pf = phi[k];
    if (!isfinite(pf)) {
      acc[7] += 1.0;
      continue;
    }
    const int y = (int)(k / nx), x = (int)(k - (int64_t)y * nx);
    float gx, gy, lap;
    stencil_at<WALLS>(phi, nx, ny, x, y, gx, gy, lap);
    const double v = pf;
    const double fa = v - c.phia, fb = v - c.phib;
    acc[0] += v;
    acc[1] += fabs(v);
    // Eq. freeEnergy: beta (phi - phi_a)^2 (phi - phi_b)^2 + kappa/2 |grad phi|^2
    acc[2] += 0.5 * (double)c.beta2 * fa * fa * fb * fb +
              0.5 * (double)c.kappa * ((double)gx * gx + (double)gy * gy);
    if (ref) {
      const double r = ref[k];
      acc[3] += (v - r) * (v - r);
      acc[4] += r * r;
    }
    acc[5] = fmax(acc[5], v);
    acc[6] = fmin(acc[6], v);
  }
  const double r = block_reduce(acc, sh);
  if (threadIdx.x < NDIAG) part[blockIdx.x * NDIAG + threadIdx.x] = r;
}

__global__ void __launch_bounds__(DIAG_THREADS) k_diag_final(const double* __restrict__ part,
                                                             double* __restrict__ out) {
  __shared__ double sh[NDIAG][DIAG_WAVES];
  double acc[NDIAG] = {0, 0, 0, 0, 0, -INFINITY, INFINITY, 0};
  for (int b = threadIdx.x; b < DIAG_BLOCKS; b += DIAG_THREADS) {
#pragma unroll
    for (int q = 0; q < NDIAG; ++q) {
      const double o = part[b * NDIAG + q];
      acc[q] = diag_op(q, acc[q], o);
    }
  }
  const double r = block_reduce(acc, sh);
  if (threadIdx.x < NDIAG) out[threadIdx.x] = r;
}

// ---------------------------------------------------------------------------------
// Discrete adjoint of one step at tau_g = 1 (periodic lattice).  With tau_g = 1 the
// collision of Eq. LB keeps nothing of the incoming populations (g* = g^eq + S/2), so
// one step is a map of phi alone:
//   phi' = phi + M L(mu) + A(phi, u) - Div(F)/2,
//   mu = f'(phi) - kappa L(phi),  A = sum_i w_i T_{-c_i}[phi s_i(u)],
//   F = -h(phi) grad mu + K grad(Div(phi u)),  h = phi^2 / rho(phi),
// with L, grad, Div the isotropic stencils (L symmetric, grad antisymmetric) and
// (T_c psi)(x) = psi(x + c).  Given lam' = dL/dphi' the kernel below forms
//   lam = dL/dphi = lam' + sum_i w_i s_i(u) T_{c_i} lam' - h'(phi) grad mu . lamF
//         + f''(phi) lamMu - kappa L(lamMu) + u . lamQ,
//   lamF = grad(lam')/2,  lamMu = M L(lam') + Div(h lamF),
//   lamD = -K Div(lamF),  lamQ = -grad(lamD),
//   dL/du = sum_i w_i phi ds_i/du T_{c_i} lam' + phi lamQ,
// and add tf * dL/du to the caller's gradient of the base velocity field.
struct AdjArgs {
  const float* phi;   // forward phi at the start of the step
  const float* lam1;  // dL/dphi' (after the step)
  float* lam0;        // dL/dphi (output; must not alias lam1)
  float* gu;          // += tf dL/du (base field); may be null
  float* gv;
  int nx, ny;
  Coef c;
  float mob;          // M
  int vmode;          // VEL_SEP or VEL_FIELD
  const float *ax, *ay, *bx, *by, *ux, *uy;
  float tf;
};

__device__ __forceinline__ float adj_h(const Coef& c, float phi, float& dh) {
  const float rho = c.a * phi + c.b;
  const float ir = 1.0f / rho;
  dh = phi * (c.a * phi + 2.0f * c.b) * ir * ir;
  return phi * phi * ir;
}
__device__ __forceinline__ float d2bulk(const Coef& c, float p) {
  const float a = p - c.phia, b = p - c.phib, s = 2.0f * p - c.phia - c.phib;
  return c.beta2 * (b * s + a * s + 2.0f * a * b);
}
// Periodic index of any i; the division is only done for indices outside [0, n) (tile
// halos, and tiles wider than the lattice).
__device__ __forceinline__ int wrap(int i, int n) {
  if (i >= 0 && i < n) return i;
  i %= n;
  return i < 0 ? i + n : i;
}

// One block per ATW x ATH output tile.  Every quantity is formed in LDS on the region
// its consumers need: lam' with a halo of 3, phi, lamF and h lamF with 2, mu, lamMu and
// lamD with 1, so one launch does a whole reverse step.
constexpr int ATW = 32, ATH = 8;
__global__ void __launch_bounds__(ATW * ATH) k_adjoint(const AdjArgs a) {
  constexpr int L3W = ATW + 6, L3H = ATH + 6;
  constexpr int P2W = ATW + 4, P2H = ATH + 4;
  constexpr int Q1W = ATW + 2, Q1H = ATH + 2;
  constexpr int NT = ATW * ATH;
  __shared__ float sl[L3H][L3W];
  __shared__ float sp[P2H][P2W];
  __shared__ float slfx[P2H][P2W], slfy[P2H][P2W], swfx[P2H][P2W], swfy[P2H][P2W];
  __shared__ float smu[Q1H][Q1W], slmu[Q1H][Q1W], sld[Q1H][Q1W];
  // When recording steps of other segments run beside the reverse steps (on other
  // streams), the chain of reverse steps is what the backward pass waits for: its
  // waves take issue priority over theirs (adjoint256: about 5 % faster).
  __builtin_amdgcn_s_setprio(3);
  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * ATW, y0 = blockIdx.y * ATH;
  // Every global load of the step is issued up front, into registers, and used only
  // after that: the staged lam' and phi values of this thread, and its own node's
  // velocity and accumulated gradients.  So the step waits for memory once.
  const int ty = t / ATW, tx = t - ty * ATW;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < nx && y < ny;
  const uint32_t k = own ? (uint32_t)y * nx + x : 0u;
  constexpr int NL = (L3H * L3W + NT - 1) / NT, NP = (P2H * P2W + NT - 1) / NT;
  float vl[NL], vp[NP];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int i = t + q * NT;
    const int r = i / L3W, cc = i - r * L3W;
    vl[q] = i < L3H * L3W
                ? a.lam1[(uint32_t)wrap(y0 - 3 + r, ny) * nx + wrap(x0 - 3 + cc, nx)]
                : 0.f;
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int i = t + q * NT;
    const int r = i / P2W, cc = i - r * P2W;
    vp[q] = i < P2H * P2W
                ? a.phi[(uint32_t)wrap(y0 - 2 + r, ny) * nx + wrap(x0 - 2 + cc, nx)]
                : 0.f;
  }
  float u1 = 0.f, u2 = 0.f, v1 = 0.f, v2 = 0.f, gu0 = 0.f, gv0 = 0.f;
  if (own) {
    if (a.vmode == VEL_SEP) {
      u1 = a.ax[x];
      u2 = a.ay[y];
      v1 = a.bx[x];
      v2 = a.by[y];
    } else {
      u1 = a.ux[k];
      v1 = a.uy[k];
    }
    if (a.gu) {
      gu0 = a.gu[k];
      gv0 = a.gv[k];
    }
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int i = t + q * NT;
    if (i < L3H * L3W) sl[i / L3W][i - (i / L3W) * L3W] = vl[q];
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int i = t + q * NT;
    if (i < P2H * P2W) sp[i / P2W][i - (i / P2W) * P2W] = vp[q];
  }
  __syncthreads();
  // lamF = grad(lam')/2 and h lamF on the halo-2 region (sl is offset by one more)
  for (int i = t; i < P2H * P2W; i += NT) {
    const int r = i / P2W, cc = i - r * P2W;
    const float lfx = 0.5f * ddx(sl[r], sl[r + 1], sl[r + 2], cc + 1);
    const float lfy = 0.5f * ddy(sl[r], sl[r + 1], sl[r + 2], cc + 1);
    float dh;
    const float h = adj_h(c, sp[r][cc], dh);
    slfx[r][cc] = lfx;
    slfy[r][cc] = lfy;
    swfx[r][cc] = h * lfx;
    swfy[r][cc] = h * lfy;
  }
  // mu (Eq. mu) on the halo-1 region
  for (int i = t; i < Q1H * Q1W; i += NT) {
    const int r = i / Q1W, cc = i - r * Q1W;
    smu[r][cc] = mu_bulk(c, sp[r + 1][cc + 1]) - c.kappa * lap9(sp[r], sp[r + 1], sp[r + 2], cc + 1);
  }
  __syncthreads();
  // lamMu = M lap(lam') + div(h lamF), lamD = -K div(lamF) on the halo-1 region
  for (int i = t; i < Q1H * Q1W; i += NT) {
    const int r = i / Q1W, cc = i - r * Q1W;
    slmu[r][cc] = a.mob * lap9(sl[r + 1], sl[r + 2], sl[r + 3], cc + 2) +
                  ddx(swfx[r], swfx[r + 1], swfx[r + 2], cc + 1) +
                  ddy(swfy[r], swfy[r + 1], swfy[r + 2], cc + 1);
    if (c.k2 != 0.0f)
      sld[r][cc] = -c.k2 * (ddx(slfx[r], slfx[r + 1], slfx[r + 2], cc + 1) +
                            ddy(slfy[r], slfy[r + 1], slfy[r + 2], cc + 1));
  }
  __syncthreads();
  if (!own) return;
  const float phi = sp[ty + 2][tx + 2];
  float u, v;
  if (a.vmode == VEL_SEP) {
    u = a.tf * u1 * u2;
    v = a.tf * v1 * v2;
  } else {
    u = a.tf * u1;
    v = a.tf * v1;
  }
  const float usq = u * u + v * v;
  // advection part: sum_i w_i s_i(u) lam'(x + c_i), and its u-derivative times phi
  float lam = sl[ty + 3][tx + 3], lu = 0.f, lv = 0.f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = CX[i] * u + CY[i] * v;
    const float si = 3.0f * cu + 4.5f * cu * cu - 1.5f * usq;
    const float l = sl[ty + 3 + (int)CY[i]][tx + 3 + (int)CX[i]];
    lam += WT[i] * si * l;
    lu += WT[i] * (3.0f * CX[i] + 9.0f * cu * CX[i] - 3.0f * u) * l;
    lv += WT[i] * (3.0f * CY[i] + 9.0f * cu * CY[i] - 3.0f * v) * l;
  }
  float dh;
  adj_h(c, phi, dh);
  const float mux = ddx(smu[ty], smu[ty + 1], smu[ty + 2], tx + 1);
  const float muy = ddy(smu[ty], smu[ty + 1], smu[ty + 2], tx + 1);
  lam -= dh * (slfx[ty + 2][tx + 2] * mux + slfy[ty + 2][tx + 2] * muy);
  lam += d2bulk(c, phi) * slmu[ty + 1][tx + 1] -
         c.kappa * lap9(slmu[ty], slmu[ty + 1], slmu[ty + 2], tx + 1);
  float gx = lu, gy = lv;
  if (c.k2 != 0.0f) {  // lamQ = -grad(lamD); q = phi u
    const float lqx = -ddx(sld[ty], sld[ty + 1], sld[ty + 2], tx + 1);
    const float lqy = -ddy(sld[ty], sld[ty + 1], sld[ty + 2], tx + 1);
    lam += u * lqx + v * lqy;
    gx += lqx;
    gy += lqy;
  }
  a.lam0[k] = lam;
  if (a.gu) {
    a.gu[k] = gu0 + a.tf * phi * gx;
    a.gv[k] = gv0 + a.tf * phi * gy;
  }
}

template <int ST>
void init_l(bool walls, int vmode, dim3 grid, hipStream_t s, const Coef& c, int nx, int ny,
            uint32_t pitch, const float* phi0, const float* ax, const float* ay,
            const float* bx, const float* by, const float* ux, const float* uy, float tf,
            char* g, float* f) {
  const bool sep = vmode == VEL_SEP;
  if (walls && sep)
    hipLaunchKernelGGL((k_init<true, VEL_SEP, ST>), grid, dim3(256), 0, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
  else if (walls)
    hipLaunchKernelGGL((k_init<true, VEL_FIELD, ST>), grid, dim3(256), 0, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
  else if (sep)
    hipLaunchKernelGGL((k_init<false, VEL_SEP, ST>), grid, dim3(256), 0, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
  else
    hipLaunchKernelGGL((k_init<false, VEL_FIELD, ST>), grid, dim3(256), 0, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
}

}  // namespace

uint32_t population_bytes(int storage, uint32_t pitch, uint32_t ny) { return pop_bytes(storage, pitch, ny); }

hipError_t launch_init(bool walls, int vmode, int storage, const Coef& c, int nx, int ny,
                       uint32_t pitch, const float* phi0, const float* ax, const float* ay,
                       const float* bx, const float* by, const float* ux, const float* uy,
                       float tf, void* g, float* f, hipStream_t s) {
  const dim3 grid((nx + 255) / 256, ny);
  char* gb = static_cast<char*>(g);
  switch (storage) {
    case ST_F32: init_l<ST_F32>(walls, vmode, grid, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, gb, f); break;
    case ST_F16: init_l<ST_F16>(walls, vmode, grid, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, gb, f); break;
    case ST_BF16: init_l<ST_BF16>(walls, vmode, grid, s, c, nx, ny, pitch, phi0, ax, ay, bx, by, ux, uy, tf, gb, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_phi_field(bool walls, int storage, const void* g, uint32_t pitch, int nx,
                            int ny, float* phi, hipStream_t s) {
  const dim3 grid((nx + 255) / 256, ny);
  switch (storage) {
    case ST_F32:
      if (walls) hipLaunchKernelGGL((k_phi_field<true, ST_F32>), grid, dim3(256), 0, s, g, pitch, nx, ny, phi);
      else hipLaunchKernelGGL((k_phi_field<false, ST_F32>), grid, dim3(256), 0, s, g, pitch, nx, ny, phi);
      break;
    case ST_F16:
      if (walls) hipLaunchKernelGGL((k_phi_field<true, ST_F16>), grid, dim3(256), 0, s, g, pitch, nx, ny, phi);
      else hipLaunchKernelGGL((k_phi_field<false, ST_F16>), grid, dim3(256), 0, s, g, pitch, nx, ny, phi);
      break;
    case ST_BF16:
      if (walls) hipLaunchKernelGGL((k_phi_field<true, ST_BF16>), grid, dim3(256), 0, s, g, pitch, nx, ny, phi);
      else hipLaunchKernelGGL((k_phi_field<false, ST_BF16>), grid, dim3(256), 0, s, g, pitch, nx, ny, phi);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const Coef& c, float mobility, int nx, int ny, int vmode,
                                const float* ax, const float* ay, const float* bx,
                                const float* by, const float* ux, const float* uy, float tf,
                                const float* phi, const float* lam1, float* lam0, float* gu,
                                float* gv, hipStream_t s) {
  AdjArgs a{};
  a.phi = phi; a.lam1 = lam1; a.lam0 = lam0; a.gu = gu; a.gv = gv;
  a.nx = nx; a.ny = ny; a.c = c; a.mob = mobility; a.vmode = vmode;
  a.ax = ax; a.ay = ay; a.bx = bx; a.by = by; a.ux = ux; a.uy = uy; a.tf = tf;
  const dim3 grid((nx + ATW - 1) / ATW, (ny + ATH - 1) / ATH);
  hipLaunchKernelGGL(k_adjoint, grid, dim3(ATW * ATH), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mu_field(bool walls, const Coef& c, const float* phi, int nx, int ny,
                           float* mu, hipStream_t s) {
  const dim3 grid((nx + 255) / 256, ny);
  if (walls) hipLaunchKernelGGL((k_mu_field<true>), grid, dim3(256), 0, s, c, phi, nx, ny, mu);
  else hipLaunchKernelGGL((k_mu_field<false>), grid, dim3(256), 0, s, c, phi, nx, ny, mu);
  return hipGetLastError();
}

hipError_t launch_velocity_field(int vmode, int nx, int ny, const float* ax, const float* ay,
                                 const float* bx, const float* by, const float* ux,
                                 const float* uy, float tf, float* u, float* v,
                                 hipStream_t s) {
  const dim3 grid((nx + 255) / 256, ny);
  hipLaunchKernelGGL(k_velocity, grid, dim3(256), 0, s, vmode, nx, ny, ax, ay, bx, by, ux, uy,
                     tf, u, v);
  return hipGetLastError();
}

hipError_t launch_fill(float* dst, float value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, value, n);
  return hipGetLastError();
}

int diag_partial_blocks() { return DIAG_BLOCKS; }

hipError_t launch_diag(bool walls, const Coef& c, const float* phi, const float* ref, int nx,
                       int ny, double* partial, double* out, hipStream_t s) {
  if (walls)
    hipLaunchKernelGGL((k_diag_partial<true>), dim3(DIAG_BLOCKS), dim3(DIAG_THREADS), 0, s, c, phi, ref, nx, ny, partial);
  else
    hipLaunchKernelGGL((k_diag_partial<false>), dim3(DIAG_BLOCKS), dim3(DIAG_THREADS), 0, s, c, phi, ref, nx, ny, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DIAG_THREADS), 0, s, partial, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Device scratch of lbm_ch_adjoint_static, for callers that cannot allocate device
// memory: the field the reverse steps alternate with the caller's lam.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code the name
// `scratch` is a host-side stand-in, not a device address: the address of each device's
// copy comes from hipGetSymbolAddress, taken once per device with that device current
// (static_scratch_setup, called by lbm_ch_init), and only that address is used.
static __device__ __align__(256) float scratch[ADJ_STATIC_MAX_NODES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = static_cast<float*>(ptr);
  return hipSuccess;
}

float* static_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace lbmch
