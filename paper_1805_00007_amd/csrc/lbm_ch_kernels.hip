// gfx950 kernels of the lattice Boltzmann Cahn-Hilliard solver
// (Zhang, Guo & Liang, arXiv:1805.00007).  The public contract, the method and the
// boundary rules are stated in include/lbm_ch.h; this file holds the device code.
//
// The hot kernel, k_phi_step, is one fused pull-scheme update of all nine
// phase-field populations.  A block owns a strip of TX columns and marches down TY
// rows of it.  Per row it keeps three rolling rings in LDS:
//   stage 1, row y+2: pull g_i(x) = g_i*(x - c_i), phi = sum g_i, q = phi u   (Eq. macroscopicg)
//   stage 2, row y+1: mu = f'(phi) - kappa lap(phi), D = div q                 (Eqs. mu, mark3)
//   stage 3, row y  : grad mu, grad D (and grad p), F = F1 + F2, g^eq, S, BGK,
//                     store g*                                                 (Eqs. t0-phiu, mark3, geq, liangFi, LB)
// so every value is computed once per node and the only HBM traffic is the nine
// populations in and out (72 bytes per node update in float32).  The pops of a row
// are pulled two iterations before they are collided and stay in registers; the
// pull for the next row is issued before the barriers so that its latency overlaps
// the stencil work.  Four lanes of the block also compute phi (and mu, D) of the
// two halo columns on each side.  A row strip of the domain is handed to blocks in
// an order that keeps a band of neighbouring strips on one XCD (one L2), so the
// halo rows a block re-reads are L2 hits.
#include "lbm_ch_internal.h"

#include <math.h>

namespace lbmch {
namespace {

// D2Q9 lattice of Sec. II.B and its weights (below Eq. geq).
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr float WT[9] = {4.0f / 9, 1.0f / 9, 1.0f / 9, 1.0f / 9, 1.0f / 9,
                         1.0f / 36, 1.0f / 36, 1.0f / 36, 1.0f / 36};

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Logical row r (may lie one or two rows outside the lattice) -> stored row and the
// parity of the velocity there: periodic wrap, or mirror across the walls at
// y = -1/2 and y = ny - 1/2 (velocity odd).
template <bool WALLS>
__device__ __forceinline__ int row_of(int r, int ny, float& vsign) {
  if (WALLS) {
    if (r < 0) { vsign = -1.0f; return -1 - r; }
    if (r >= ny) { vsign = -1.0f; return 2 * ny - 1 - r; }
    vsign = 1.0f;
    return r;
  }
  vsign = 1.0f;
  r = r % ny;
  return r < 0 ? r + ny : r;
}

// Range-checked buffer access (gfx9 raw buffer, stride 0): an offset at or beyond
// the descriptor's byte count reads 0 and drops the store, so no index can reach
// memory outside the array it belongs to.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ float ldb(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void stb(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// Population storage.  ST_F32: nine float32 planes.  ST_F16 / ST_BF16: the rest
// population g_0 as a float32 plane, then eight 16-bit planes holding g_i / w_i
// (i = 1..8) in IEEE half or bfloat16.  The moving populations of Eq. geq are
// w_i (eta mu + phi s_i(u)), of order w_i |u|, so their scaled values are small and a
// 16-bit code keeps them to ~1e-4 of that size; g_0 ~ phi stays in float32 and, through
// the mass closure below, absorbs the rounding of the others.
enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };
constexpr float INV_W[9] = {9.0f / 4, 9.0f, 9.0f, 9.0f, 9.0f, 36.0f, 36.0f, 36.0f, 36.0f};

__host__ __device__ constexpr uint32_t pop_bytes(int st, uint32_t plane) {
  return st == ST_F32 ? 36u * plane : 20u * plane;
}
template <int ST>
__device__ __forceinline__ float dec16(uint32_t h) {
  if (ST == ST_F16) return (float)__builtin_bit_cast(_Float16, (unsigned short)h);
  return __builtin_bit_cast(float, h << 16);
}
template <int ST>
__device__ __forceinline__ uint32_t enc16(float f) {
  if (ST == ST_F16) return __builtin_bit_cast(unsigned short, (_Float16)f);
  const uint32_t u = __builtin_bit_cast(uint32_t, f);  // round to nearest even
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// Population i at (column col, row) of a buffer in storage ST.
template <int ST>
__device__ __forceinline__ float ldpop(rsrc_t s, int i, uint32_t plane, uint32_t nx,
                                       uint32_t col, uint32_t row) {
  if (ST == ST_F32 || i == 0) return ldb(s, col * 4u, ((uint32_t)i * plane + row * nx) * 4u);
  const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(
      s, col * 2u, plane * 4u + ((uint32_t)(i - 1) * plane + row * nx) * 2u, 0);
  return WT[i] * dec16<ST>(h);
}

// Pull of the nine populations arriving at (x, y): g_i(x, y) = g_i*(x - c_i, y - c_i).
// With walls, a population whose source lies beyond a wall is the opposite one that
// left (x, y) (half-way bounce-back).  y is a lattice row (block-uniform); cc, cm, cp
// are the columns x, x-1, x+1 (wrapped).  Plane and row offsets travel in the
// instruction's scalar offset, so a load costs no vector ALU work beyond its column.
template <bool WALLS, int ST>
__device__ __forceinline__ void pull9(rsrc_t s, uint32_t plane, uint32_t nx, int ny, int y,
                                      uint32_t cc, uint32_t cm, uint32_t cp, float g[9]) {
  const uint32_t ym = y == 0 ? ny - 1 : y - 1;
  const uint32_t yp = y == ny - 1 ? 0 : y + 1;
  const uint32_t yc = y;
  g[0] = ldpop<ST>(s, 0, plane, nx, cc, yc);
  g[1] = ldpop<ST>(s, 1, plane, nx, cm, yc);
  g[3] = ldpop<ST>(s, 3, plane, nx, cp, yc);
  if (WALLS && y == 0) {
    g[2] = ldpop<ST>(s, 4, plane, nx, cc, yc);
    g[5] = ldpop<ST>(s, 7, plane, nx, cc, yc);
    g[6] = ldpop<ST>(s, 8, plane, nx, cc, yc);
  } else {
    g[2] = ldpop<ST>(s, 2, plane, nx, cc, ym);
    g[5] = ldpop<ST>(s, 5, plane, nx, cm, ym);
    g[6] = ldpop<ST>(s, 6, plane, nx, cp, ym);
  }
  if (WALLS && y == ny - 1) {
    g[4] = ldpop<ST>(s, 2, plane, nx, cc, yc);
    g[7] = ldpop<ST>(s, 5, plane, nx, cc, yc);
    g[8] = ldpop<ST>(s, 6, plane, nx, cc, yc);
  } else {
    g[4] = ldpop<ST>(s, 4, plane, nx, cc, yp);
    g[7] = ldpop<ST>(s, 7, plane, nx, cp, yp);
    g[8] = ldpop<ST>(s, 8, plane, nx, cm, yp);
  }
}

// Order parameter of Eq. macroscopicg and mass bookkeeping.  The nine float32
// populations are summed in FP64, which is exact for their range of magnitudes, and
// the collision writes g_0* = (phi - sum_{i>0} g_i*) through the same FP64 sums, so
// the exact sum of the stored floats moves only by the rounding of g_0* -- no bias
// builds up in uniform regions, where every node would round identically.  In exact
// arithmetic this equals the direct form of Eq. LB, because the collision conserves
// sum_i g_i (Eqs. feqmoment, conservation).  phi itself (for the stencils) is the
// float32 rounding of the FP64 sum; lo keeps the remainder.
__device__ __forceinline__ double sum8_hi(const float g[9]) {
  return (((double)g[1] + (double)g[2]) + ((double)g[3] + (double)g[4])) +
         (((double)g[5] + (double)g[6]) + ((double)g[7] + (double)g[8]));
}
// Sets g[0] so that the exact sum of the nine floats equals m up to the rounding
// of g[8]: g[0] takes the float part of m - sum_{i>0} g_i, and the remainder (exact
// in FP64) goes into g[8].  g[8] is small (of order w_8 (eta mu + phi s_8(u))), so
// its rounding is ~100x finer than that of g[0] ~ phi.
__device__ __forceinline__ void close_mass(double m, float g[9]) {
  const double e0 = m - sum8_hi(g);
  g[0] = (float)e0;
  g[8] = (float)((double)g[8] + (e0 - (double)g[0]));
}
// Writes the nine post-collision populations of node (col, row) in storage ST such that
// the exact sum of the stored values is m (float32: up to the rounding of g_8; 16-bit:
// up to the float32 rounding of g_0, which takes m minus the decoded others).  Returns
// the stored values in g.
template <int ST>
__device__ __forceinline__ void finish_store(rsrc_t d, uint32_t plane, uint32_t nx,
                                             uint32_t col, uint32_t row, double m, float g[9]) {
  if (ST == ST_F32) {
    close_mass(m, g);
#pragma unroll
    for (int i = 0; i < 9; ++i) stb(d, g[i], col * 4u, ((uint32_t)i * plane + row * nx) * 4u);
    return;
  }
  uint32_t h[9];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    h[i] = enc16<ST>(g[i] * INV_W[i]);
    g[i] = WT[i] * dec16<ST>(h[i]);
  }
  g[0] = (float)(m - sum8_hi(g));
  stb(d, g[0], col * 4u, row * nx * 4u);
#pragma unroll
  for (int i = 1; i < 9; ++i)
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)h[i], d, col * 2u,
                                          plane * 4u + ((uint32_t)(i - 1) * plane + row * nx) * 2u, 0);
}

__device__ __forceinline__ float sum9(const float g[9], float& lo) {
  const double s = sum8_hi(g) + (double)g[0];
  const float f = (float)s;
  lo = (float)(s - (double)f);
  return f;
}
__device__ __forceinline__ float sum9(const float g[9]) {
  float lo;
  return sum9(g, lo);
}

// Bulk part of Eq. mu for the double well of Eq. bulk.
__device__ __forceinline__ float mu_bulk(const Coef& c, float phi) {
  return c.beta2 * (phi - c.phia) * (phi - c.phib) * (2.0f * phi - c.phia - c.phib);
}

// Isotropic stencils on three LDS rows (rm: y-1, r0: y, rp: y+1) around column j:
//   d_x = [4 (E - W) + (NE + SE - NW - SW)] / 12
//   d_y = [4 (N - S) + (NE + NW - SE - SW)] / 12
//   lap = [4 (E + W + N + S) + (NE + NW + SE + SW) - 20 C] / 6
__device__ __forceinline__ float ddx(const float* rm, const float* r0, const float* rp, int j) {
  return (4.0f * (r0[j + 1] - r0[j - 1]) + (rp[j + 1] + rm[j + 1] - rp[j - 1] - rm[j - 1])) *
         (1.0f / 12.0f);
}
__device__ __forceinline__ float ddy(const float* rm, const float* r0, const float* rp, int j) {
  return (4.0f * (rp[j] - rm[j]) + (rp[j + 1] + rp[j - 1] - rm[j + 1] - rm[j - 1])) *
         (1.0f / 12.0f);
}
__device__ __forceinline__ float lap9(const float* rm, const float* r0, const float* rp, int j) {
  return (4.0f * (r0[j + 1] + r0[j - 1] + rp[j] + rm[j]) +
          (rp[j + 1] + rp[j - 1] + rm[j + 1] + rm[j - 1]) - 20.0f * r0[j]) *
         (1.0f / 6.0f);
}

// Collision of Eq. LB with g^eq of Eq. geq and S_i = 3 w_i c_i.F (Eq. liangFi):
//   g_i* = (1 - omega) g_i + omega g_i^eq + srcg w_i c_i.F
__device__ __forceinline__ void collide_g(const Coef& c, float phi, float phi_lo, float mu,
                                          float u, float v, float fx, float fy, float g[9]) {
  const float em = c.eta * mu;
  const float usq15 = 1.5f * (u * u + v * v);
  const float A = em - phi * usq15;  // w_i (eta mu - 1.5 phi u^2) common to all i
  const float om1 = 1.0f - c.omega;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float cu = CX[i] * u + CY[i] * v;
    const float cf = CX[i] * fx + CY[i] * fy;
    const float eq = A + phi * cu * (3.0f + 4.5f * cu);
    g[i] = om1 * g[i] + WT[i] * (c.omega * eq + c.srcg * cf);
  }
  // g_0* = (1 - omega) g_0 + omega g_0^eq is written by finish_store through mass
  // conservation: sum_i g_i* = phi + phi_lo.
  (void)phi_lo;
}

// ---------------------------------------------------------------------------------
// Fused phase-field step.
//   VMODE VEL_SEP: u = tf ax[x] ay[y]; VEL_FIELD: u = tf ux[y][x];
//   VEL_NSFIELD: u, p from the NS step, F1 = (phi/rho)(F_s + F_b - grad p).
// One row record of the register pipeline: the pulled populations (plus velocity and
// pressure in the field modes) and the order parameter and velocity of the row.
struct RowRec {
  float g[9];
  float lu, lv, lp;       // loaded velocity / pressure (field modes)
  float phi, lo, u, v;    // stage-1 results (u, v in the field modes)
  float fy_u, fy_v;       // separable mode: ay[y], by[y] as loaded, then times tf
  float xpx, xpy;         // model 3: X of the previous step at this node
};

#ifndef WPE_PHI
#define WPE_PHI 4
#endif
// One tile of the step: strip (L % nstrips) of TX columns, row chunk L / nstrips.
// MODEL 1: F = F1; 2: F = F1 + K grad(div(phi u)) (Eq. mark3); 3: Eq. F2-1 with the
// time derivatives as one-step differences of X = cA F1 + cB grad mu, stored per node.
template <int TX, bool WALLS, int VMODE, int MODEL, int ST>
__device__ __forceinline__ void phi_tile(const StepArgs& a, const int L) {
  constexpr bool MODEL2 = MODEL >= 2;
  constexpr bool HIST = MODEL == 3;
  constexpr bool NSC = VMODE == VEL_NSFIELD;
  constexpr bool VFIELD = VMODE != VEL_SEP;
  constexpr int LW = TX + 4;
  constexpr int QR = MODEL2 ? 4 : 1;
  constexpr int PR = NSC ? 8 : 1;
  __shared__ float s_phi[4][LW];
  __shared__ float s_mu[4][LW];
  __shared__ float s_qx[QR][LW];
  __shared__ float s_qy[QR][LW];
  __shared__ float s_d[QR][LW];
  __shared__ float s_p[PR][LW];

  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const uint32_t nodes = (uint32_t)nx * ny;
  const uint32_t plane = a.plane;
  const uint32_t rb = (uint32_t)nx * 4u;
  const rsrc_t rsrc = make_rsrc(a.src, pop_bytes(ST, plane));
  const rsrc_t rdst = make_rsrc(a.dst, pop_bytes(ST, plane));
  rsrc_t ru, rv, rp;
  if (VFIELD) {
    ru = make_rsrc(a.ux, nodes * 4u);
    rv = make_rsrc(a.uy, nodes * 4u);
  }
  if (NSC) rp = make_rsrc(a.pf, nodes * 4u);
  rsrc_t rxh;
  if (HIST) rxh = make_rsrc(a.xh, 2u * nodes * 4u);

  const int t = threadIdx.x;
  const int x0 = (L % a.nstrips) * TX;
  const int chunk = L / a.nstrips;
  const int rows = min(a.ty, ny - chunk * a.ty);
  // Vertically adjacent chunks march in opposite directions, so the two blocks that
  // share a chunk boundary pass it at the same moment (both at their start or both
  // at their end) and the halo rows one re-reads are still in L2.
  const int dir = (chunk & 1) ? -1 : 1;
  const int y0 = dir > 0 ? chunk * a.ty : chunk * a.ty + rows - 1;  // first row marched

  // Own column (wrapped) and its neighbours.
  const int xl = x0 + t;
  const bool active = xl < nx;
  const int xc = xl % nx;
  const uint32_t vc = xc;
  const uint32_t vm = xc == 0 ? nx - 1 : xc - 1;
  const uint32_t vp = xc == nx - 1 ? 0 : xc + 1;
  // Halo lanes t < 4: logical columns x0-2, x0-1, x0+TX, x0+TX+1 -> LDS 0, 1, TX+2, TX+3.
  const bool hl = t < 4;
  const int hlog = t < 2 ? x0 - 2 + t : x0 + TX - 2 + t;
  const int hc = ((hlog % nx) + nx) % nx;
  // Every lane issues the halo pull, so that the wait-count bookkeeping does not depend
  // on a branch; lanes other than the four halo lanes use an offset beyond the buffer,
  // for which a raw buffer load returns 0 without accessing memory.
  constexpr uint32_t OOB = 0x3FFFFFC0u;  // column index whose byte offset exceeds any buffer
  const uint32_t hvc = hl ? hc : OOB;
  const uint32_t hvm = hl ? (hc == 0 ? nx - 1 : hc - 1) : OOB;
  const uint32_t hvp = hl ? (hc == nx - 1 ? 0 : hc + 1) : OOB;
  const int hj = t < 2 ? t : TX + t;
  const int j = t + 2;
  const int j2 = t == 0 ? 1 : TX + 2;  // stage-2 halo column of lanes 0 and 1

  float axc = 0.f, bxc = 0.f, axh = 0.f, bxh = 0.f;
  if (VMODE == VEL_SEP) {
    axc = a.ax[xc];
    bxc = a.bx[xc];
    if (hl) {
      axh = a.ax[hc];
      bxh = a.bx[hc];
    }
  }

  // Issue the pull of logical row r at one column (plus velocity and pressure in the
  // field modes) so that one wait covers all of it.
  auto issue = [&](int r, uint32_t cc, uint32_t cm, uint32_t cp, RowRec& R, bool own = true) {
    float sg;
    const int sr = row_of<WALLS>(r, ny, sg);
    pull9<WALLS, ST>(rsrc, plane, nx, ny, sr, cc, cm, cp, R.g);
    if (HIST && own) {
      R.xpx = ldb(rxh, cc * 4u, (uint32_t)sr * rb);
      R.xpy = ldb(rxh, cc * 4u, nodes * 4u + (uint32_t)sr * rb);
    }
    if (VMODE == VEL_SEP) {
      // row factors of the separable velocity, fetched with the pull so that one wait
      // covers both (a later load would make the wait cover the whole prefetch)
      R.fy_u = a.ay[sr];
      R.fy_v = a.by[sr];
    }
    if (VFIELD) {
      R.lu = ldb(ru, cc * 4u, (uint32_t)sr * rb);
      R.lv = ldb(rv, cc * 4u, (uint32_t)sr * rb);
      if (NSC) R.lp = ldb(rp, cc * 4u, (uint32_t)sr * rb);
    }
  };
  // Stage 1 for logical row r: phi (and q = phi u, p) into the rings at column jj.
  auto stage1 = [&](int r, RowRec& R, int jj, float axv, float bxv, bool wr = true) {
    float sg;
    row_of<WALLS>(r, ny, sg);
    R.phi = sum9(R.g, R.lo);
    float u, v;
    if (VMODE == VEL_SEP) {
      R.fy_u *= a.tf * sg;
      R.fy_v *= a.tf * sg;
      u = axv * R.fy_u;
      v = bxv * R.fy_v;
    } else {
      u = R.u = a.tf * R.lu * sg;
      v = R.v = a.tf * R.lv * sg;
    }
    if (!wr) return;
    s_phi[r & 3][jj] = R.phi;
    if (MODEL2) {
      s_qx[r & 3][jj] = R.phi * u;
      s_qy[r & 3][jj] = R.phi * v;
    }
    if (NSC) s_p[r & 7][jj] = R.lp;
  };
  // Stage 2 for logical row r at LDS column jj: mu (Eq. mu) and D = div(phi u).
  auto stage2 = [&](int r, int jj) {
    const float* pm = s_phi[(r - 1) & 3];
    const float* p0 = s_phi[r & 3];
    const float* pp = s_phi[(r + 1) & 3];
    s_mu[r & 3][jj] = mu_bulk(c, p0[jj]) - c.kappa * lap9(pm, p0, pp, jj);
    if (MODEL2) {
      s_d[r & 3][jj] = ddx(s_qx[(r - 1) & 3], s_qx[r & 3], s_qx[(r + 1) & 3], jj) +
                       ddy(s_qy[(r - 1) & 3], s_qy[r & 3], s_qy[(r + 1) & 3], jj);
    }
  };
  // Stage 3 for lattice row y: F = F1 (+ F2), collision, store.
  auto stage3 = [&](int y, RowRec& R) {
    if (!active) return;
    const float* mm = s_mu[(y - 1) & 3];
    const float* m0 = s_mu[y & 3];
    const float* mp = s_mu[(y + 1) & 3];
    const float mux = ddx(mm, m0, mp, j), muy = ddy(mm, m0, mp, j);
    const float rho = c.a * R.phi + c.b;
    float tx = -R.phi * mux, ty = -R.phi * muy;
    if (NSC) {
      const float* qm = s_p[(y - 1) & 7];
      const float* q0 = s_p[y & 7];
      const float* qp = s_p[(y + 1) & 7];
      tx += rho * c.accel_x - ddx(qm, q0, qp, j);
      ty += -(rho - c.rho_mean) * c.gravity - ddy(qm, q0, qp, j);
    }
    const float s1 = R.phi * rcp(rho);
    float fx = s1 * tx, fy = s1 * ty;
    if (HIST) {  // (2 tau - 1 + 3K) dF1/dt + 3 cs^2 eta K d(grad mu)/dt of Eq. F2-1
      const float xx = c.x_f1 * fx + c.x_mu * mux, xy = c.x_f1 * fy + c.x_mu * muy;
      stb(rxh, xx, vc * 4u, (uint32_t)y * rb);
      stb(rxh, xy, vc * 4u, nodes * 4u + (uint32_t)y * rb);
      if (!a.xfirst) {
        fx += xx - R.xpx;
        fy += xy - R.xpy;
      }
    }
    if (MODEL2) {
      const float* dm = s_d[(y - 1) & 3];
      const float* d0 = s_d[y & 3];
      const float* dp = s_d[(y + 1) & 3];
      fx += c.k2 * ddx(dm, d0, dp, j);
      fy += c.k2 * ddy(dm, d0, dp, j);
    }
    const float u = VMODE == VEL_SEP ? axc * R.fy_u : R.u;
    const float v = VMODE == VEL_SEP ? bxc * R.fy_v : R.v;
    collide_g(c, R.phi, R.lo, m0[j], u, v, fx, fy, R.g);
    finish_store<ST>(rdst, plane, nx, vc, (uint32_t)y, (double)R.phi + (double)R.lo, R.g);
  };

  // Prologue: rows y0-2d .. y0+d through stage 1, rows y0-d and y0 through stage 2,
  // and the pull of row y0+2d in flight (d = dir).
  //
  // Register pipeline.  A holds row y (collided in stage 3), B row y+d; the pull of
  // the next row lands in one of two slots, X0 or X1, which alternate, so registers
  // with a load in flight are never copied (copying them would make the wave wait for
  // every outstanding memory operation).  Completed rows move down A <- B <- X by copy.
  const int d = dir;
  RowRec A, B, X0, X1, H0;
  {
    RowRec T0, T1;
    issue(y0 - 2 * d, vc, vm, vp, T0);
    issue(y0 - d, vc, vm, vp, T1);
    issue(y0, vc, vm, vp, A);
    issue(y0 + d, vc, vm, vp, B);
    stage1(y0 - 2 * d, T0, j, axc, bxc);
    stage1(y0 - d, T1, j, axc, bxc);
    if (hl) {
      issue(y0 - 2 * d, hvc, hvm, hvp, T0, false);
      issue(y0 - d, hvc, hvm, hvp, T1, false);
    }
    stage1(y0, A, j, axc, bxc);
    stage1(y0 + d, B, j, axc, bxc);
    if (hl) {
      stage1(y0 - 2 * d, T0, hj, axh, bxh);
      stage1(y0 - d, T1, hj, axh, bxh);
      issue(y0, hvc, hvm, hvp, T0, false);
      issue(y0 + d, hvc, hvm, hvp, T1, false);
      stage1(y0, T0, hj, axh, bxh);
      stage1(y0 + d, T1, hj, axh, bxh);
    }
  }
  issue(y0 + 2 * d, hvc, hvm, hvp, H0, false);
  __builtin_amdgcn_sched_barrier(0);
  issue(y0 + 2 * d, vc, vm, vp, X0);
  __builtin_amdgcn_sched_barrier(0);
  __syncthreads();
  stage2(y0 - d, j);
  stage2(y0, j);
  if (t < 2) {
    stage2(y0 - d, j2);
    stage2(y0, j2);
  }
  __syncthreads();

  // One marching row: issue row y+3d into slot N, stage 1 of row y+2d from slot C
  // (pulled one row earlier), stage 2 of row y+d, stage 3 of row y.  On a block's last
  // row the pull of y+3d is not needed; it is clamped to the last row the block does
  // need (already in cache), so the pipeline has no branch and fetches nothing extra.
  const int last_needed = y0 + (rows + 1) * d;
  auto row = [&](int k, RowRec& C, RowRec& N) {
    const int y = y0 + k * d;
    const int ynext = k + 1 < rows ? y + 3 * d : last_needed;
    // Halo first: its pull was issued before C's, so waiting for it leaves C in flight.
    // The scheduling barriers keep the compiler from interleaving the two pulls, which
    // would make each wait cover the other pull as well.
    __builtin_amdgcn_sched_barrier(0);
    stage1(y + 2 * d, H0, hj, axh, bxh, hl);
    issue(ynext, hvc, hvm, hvp, H0, false);
    __builtin_amdgcn_sched_barrier(0);
    issue(ynext, vc, vm, vp, N);
    __builtin_amdgcn_sched_barrier(0);
    stage1(y + 2 * d, C, j, axc, bxc);
    __syncthreads();
    stage2(y + d, j);
    if (t < 2) stage2(y + d, j2);
    __syncthreads();
    stage3(y, A);
    A = B;
    B = C;
  };
  int k = 0;
#pragma unroll 1
  for (; k + 2 <= rows; k += 2) {
    row(k, X0, X1);
    row(k + 1, X1, X0);
  }
  if (k < rows) row(k, X0, X1);
}

// Model 3 carries two more values per row record; it gets the register budget of
// three waves per SIMD so that nothing spills.
template <int TX, bool WALLS, int VMODE, int MODEL, int ST>
__global__ void __launch_bounds__(TX)
__attribute__((amdgpu_waves_per_eu(MODEL == 3 ? 3 : WPE_PHI, 8)))
k_phi_step(const StepArgs a) {
  int L = blockIdx.x;
  if (a.xcd_remap) {  // workgroup w runs on XCD w % 8: give each XCD a band of chunks
    const int per = gridDim.x >> 3;
    L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  phi_tile<TX, WALLS, VMODE, MODEL, ST>(a, L);
}

// Batched step: the tiles of many lattices (one instance table entry each) in one
// persistent launch.  The tiles are numbered instance by instance; XCD x (workgroups
// w with w % 8 == x) owns the contiguous range [x per, (x + 1) per) and its workgroups
// stride through it, so vertically adjacent tiles of one lattice share that XCD's L2.
// Every workgroup leaves the loop after at most ceil(per / slots) tiles.
#ifndef WPE_BATCH
#define WPE_BATCH 3
#endif
template <int TX, int VMODE, bool MODEL2>
__global__ void __launch_bounds__(TX) __attribute__((amdgpu_waves_per_eu(WPE_BATCH, 8)))
k_phi_batch(const BatchArgs b) {
  const int slots = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per = (b.total + 7) >> 3;
  const int lo = xcd * per, hi = min(b.total, lo + per);
  int v = lo + slot;
  if (v >= hi) return;
  int lo_i = 0, hi_i = b.n;  // instance of tile v: start[inst] <= v < start[inst + 1]
  while (hi_i - lo_i > 1) {
    const int mid = (lo_i + hi_i) >> 1;
    if (b.start[mid] <= v) lo_i = mid; else hi_i = mid;
  }
  int inst = lo_i;
#pragma unroll 1
  for (; v < hi; v += slots) {
    while (b.start[inst + 1] <= v) ++inst;
    StepArgs a = b.args[inst];
    if (b.parity) {
      const void* t = a.src;
      a.src = a.dst;
      a.dst = const_cast<void*>(t);
    }
    phi_tile<TX, false, VMODE, MODEL2 ? 2 : 1, ST_F32>(a, v - b.start[inst]);
    __syncthreads();  // the LDS rings are reused by the next tile
  }
}

// ---------------------------------------------------------------------------------
// Coupled Navier-Stokes step (pressure-based incompressible D2Q9 BGK, see lbm_ch.h).
// Same marching layout: stage 1 pulls g for phi, stage 2 computes mu, stage 3 pulls
// f, forms the force, velocity and pressure, writes u, v, p and (if fdst) collides
// and stores f.
template <int TX, bool WALLS, int ST>
__global__ void __launch_bounds__(TX) k_ns_step(const NsArgs a) {
  constexpr int LW = TX + 4;
  __shared__ float s_phi[8][LW];
  __shared__ float s_mu[4][LW];
  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const uint32_t nodes = (uint32_t)nx * ny;
  const uint32_t pb = a.plane * 4u;
  const rsrc_t rg = make_rsrc(a.gsrc, pop_bytes(ST, a.plane));
  const rsrc_t rf = make_rsrc(a.fsrc, 9u * pb);
  const rsrc_t rfd = make_rsrc(a.fdst, a.fdst ? 9u * pb : 0u);
  const rsrc_t ru = make_rsrc(a.u, nodes * 4u);
  const rsrc_t rv = make_rsrc(a.v, nodes * 4u);
  const rsrc_t rpr = make_rsrc(a.p, nodes * 4u);
  const int t = threadIdx.x;
  int L = blockIdx.x;
  if (a.xcd_remap) {
    const int per = gridDim.x >> 3;
    L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int x0 = (L % a.nstrips) * TX;
  const int y0 = (L / a.nstrips) * a.ty;
  const int rows = min(a.ty, ny - y0);
  const int xl = x0 + t;
  const bool active = xl < nx;
  const int xc = xl % nx;
  const int xm = xc == 0 ? nx - 1 : xc - 1;
  const int xp = xc == nx - 1 ? 0 : xc + 1;
  const bool hl = t < 4;
  const int hlog = t < 2 ? x0 - 2 + t : x0 + TX - 2 + t;
  const int hc = ((hlog % nx) + nx) % nx;
  const int hm = hc == 0 ? nx - 1 : hc - 1;
  const int hp = hc == nx - 1 ? 0 : hc + 1;
  const int hj = t < 2 ? t : TX + t;
  const int j = t + 2;
  const int j2 = t == 0 ? 1 : TX + 2;

  const uint32_t rb = (uint32_t)nx * 4u;
  auto phi_at = [&](int r, int col, int cm, int cq) {
    float sg, g[9];
    const int sr = row_of<WALLS>(r, ny, sg);
    pull9<WALLS, ST>(rg, a.plane, nx, ny, sr, col, cm, cq, g);
    return sum9(g);
  };
  auto stage2 = [&](int r, int jj) {
    const float* pm = s_phi[(r - 1) & 7];
    const float* p0 = s_phi[r & 7];
    const float* pp = s_phi[(r + 1) & 7];
    s_mu[r & 3][jj] = mu_bulk(c, p0[jj]) - c.kappa * lap9(pm, p0, pp, jj);
  };

#pragma unroll 1
  for (int r = y0 - 2; r <= y0 + 1; ++r) {
    s_phi[r & 7][j] = phi_at(r, xc, xm, xp);
    if (hl) s_phi[r & 7][hj] = phi_at(r, hc, hm, hp);
  }
  __syncthreads();
  stage2(y0 - 1, j);
  stage2(y0, j);
  if (t < 2) {
    stage2(y0 - 1, j2);
    stage2(y0, j2);
  }
  float fpop[9];
  pull9<WALLS, ST_F32>(rf, a.plane, nx, ny, y0, xc, xm, xp, fpop);
  __syncthreads();

#pragma unroll 1
  for (int k = 0; k < rows; ++k) {
    const int y = y0 + k;
    float fnext[9];
    if (k + 1 < rows) pull9<WALLS, ST_F32>(rf, a.plane, nx, ny, y + 1, xc, xm, xp, fnext);
    s_phi[(y + 2) & 7][j] = phi_at(y + 2, xc, xm, xp);
    if (hl) s_phi[(y + 2) & 7][hj] = phi_at(y + 2, hc, hm, hp);
    __syncthreads();
    stage2(y + 1, j);
    if (t < 2) stage2(y + 1, j2);
    __syncthreads();
    if (active) {
      const float* pm = s_phi[(y - 1) & 7];
      const float* p0 = s_phi[y & 7];
      const float* pp = s_phi[(y + 1) & 7];
      const float* mm = s_mu[(y - 1) & 3];
      const float* m0 = s_mu[y & 3];
      const float* mp = s_mu[(y + 1) & 3];
      const float phi = p0[j];
      const float rho = c.a * phi + c.b;
      const float fsx = -phi * ddx(mm, m0, mp, j), fsy = -phi * ddy(mm, m0, mp, j);
      const float fbx = rho * c.accel_x, fby = -(rho - c.rho_mean) * c.gravity;
      const float corr = c.aM * lap9(mm, m0, mp, j);
      float mx = 0.f, my = 0.f, s = 0.f;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        mx += CX[i] * fpop[i];
        my += CY[i] * fpop[i];
        if (i > 0) s += fpop[i];
      }
      const float inv = rcp(rho - 0.5f * corr);
      const float u = (mx + 0.5f * (fsx + fbx)) * inv;
      const float v = (my + 0.5f * (fsy + fby)) * inv;
      const float Fx = fsx + fbx + u * corr, Fy = fsy + fby + v * corr;
      const float drx = c.a * ddx(pm, p0, pp, j), dry = c.a * ddy(pm, p0, pp, j);
      const float usq15 = 1.5f * (u * u + v * v);
      // p = cs^2/(1 - w0) [sum_{i>0} f_i + u.grad rho / 2 + rho w0 s_0(u)], cs^2/(1-w0) = 3/5
      const float pr = 0.6f * (s + 0.5f * (u * drx + v * dry) - WT[0] * rho * usq15);
      const uint32_t off = xc * 4u, ro = (uint32_t)y * rb;
      stb(ru, u, off, ro);
      stb(rv, v, off, ro);
      stb(rpr, pr, off, ro);
      if (a.fdst) {
        const float om = c.omega_f, om1 = 1.0f - om;
        const float p3 = 3.0f * pr;  // p / cs^2
        const float uF = u * Fx + v * Fy;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const float cu = CX[i] * u + CY[i] * v;
          const float cF = CX[i] * Fx + CY[i] * Fy;
          const float cr = CX[i] * drx + CY[i] * dry;
          const float su = cu * (3.0f + 4.5f * cu) - usq15;
          const float feq = WT[i] * (p3 + rho * su) - (i == 0 ? p3 : 0.0f);
          const float G = WT[i] * (3.0f * (cF - uF) + 9.0f * cu * cF + 3.0f * cu * cr);
          stb(rfd, om1 * fpop[i] + om * feq + c.srcf * G, off, i * pb + ro);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) fpop[i] = fnext[i];
  }
}

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
__device__ __forceinline__ void push_target(int nx, int ny, int x, int y, int i, int& plane_i,
                                            uint32_t& node) {
  int ty = y - CY[i];
  if (WALLS && (ty < 0 || ty >= ny)) {
    constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    plane_i = OPP[i];
    node = (uint32_t)y * nx + x;
    return;
  }
  int tx = x - CX[i];
  tx = tx < 0 ? tx + nx : (tx >= nx ? tx - nx : tx);
  ty = ty < 0 ? ty + ny : (ty >= ny ? ty - ny : ty);
  plane_i = i;
  node = (uint32_t)ty * nx + tx;
}

template <bool WALLS, int VMODE, int ST>
__global__ void __launch_bounds__(256) k_init(const Coef c, int nx, int ny, uint32_t plane,
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
    uint32_t node;
    push_target<WALLS>(nx, ny, x, y, i, pi, node);
    if (ST == ST_F32 || pi == 0)
      reinterpret_cast<float*>(g)[(uint32_t)pi * plane + node] = geq[i];
    else
      reinterpret_cast<unsigned short*>(g + 4u * plane)[(uint32_t)(pi - 1) * plane + node] =
          (unsigned short)h[i];
  }
  if (f) {
    const float rho = c.a * phi + c.b;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cu = CX[i] * u + CY[i] * v;
      int pi;
      uint32_t node;
      push_target<WALLS>(nx, ny, x, y, i, pi, node);
      f[(uint32_t)pi * plane + node] = WT[i] * rho * (cu * (3.0f + 4.5f * cu) - usq15);
    }
  }
}

template <bool WALLS, int ST>
__global__ void __launch_bounds__(256) k_phi_field(const void* __restrict__ g, uint32_t plane,
                                                   int nx, int ny, float* __restrict__ phi) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= nx) return;
  float p[9];
  pull9<WALLS, ST>(make_rsrc(g, pop_bytes(ST, plane)), plane, nx, ny, y, x,
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
  if (x >= nx) return;
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
// FP64 diagnostics: a fixed grid of blocks, each thread a fixed strided set of nodes,
// then a fixed-order tree in LDS and one final block: bitwise reproducible.
constexpr int DIAG_BLOCKS = 512;
constexpr int DIAG_THREADS = 256;
constexpr int NDIAG = 8;

template <bool WALLS>
__global__ void __launch_bounds__(DIAG_THREADS) k_diag_partial(const Coef c,
                                                               const float* __restrict__ phi,
                                                               const float* __restrict__ ref,
                                                               int nx, int ny,
                                                               double* __restrict__ part) {
  __shared__ double sh[NDIAG][DIAG_THREADS];
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
#pragma unroll
  for (int q = 0; q < NDIAG; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < NDIAG; ++q) {
        const double o = sh[q][threadIdx.x + s];
        double& m = sh[q][threadIdx.x];
        m = q == 5 ? fmax(m, o) : (q == 6 ? fmin(m, o) : m + o);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NDIAG) part[blockIdx.x * NDIAG + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(DIAG_THREADS) k_diag_final(const double* __restrict__ part,
                                                             double* __restrict__ out) {
  __shared__ double sh[NDIAG][DIAG_THREADS];
  double acc[NDIAG] = {0, 0, 0, 0, 0, -INFINITY, INFINITY, 0};
  for (int b = threadIdx.x; b < DIAG_BLOCKS; b += DIAG_THREADS) {
#pragma unroll
    for (int q = 0; q < NDIAG; ++q) {
      const double o = part[b * NDIAG + q];
      acc[q] = q == 5 ? fmax(acc[q], o) : (q == 6 ? fmin(acc[q], o) : acc[q] + o);
    }
  }
#pragma unroll
  for (int q = 0; q < NDIAG; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < NDIAG; ++q) {
        const double o = sh[q][threadIdx.x + s];
        double& m = sh[q][threadIdx.x];
        m = q == 5 ? fmax(m, o) : (q == 6 ? fmin(m, o) : m + o);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NDIAG) out[threadIdx.x] = sh[threadIdx.x][0];
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
__device__ __forceinline__ int wrap(int i, int n) {
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
  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * ATW, y0 = blockIdx.y * ATH;
  for (int i = t; i < L3H * L3W; i += NT) {
    const int r = i / L3W, cc = i - r * L3W;
    sl[r][cc] = a.lam1[(uint32_t)wrap(y0 - 3 + r, ny) * nx + wrap(x0 - 3 + cc, nx)];
  }
  for (int i = t; i < P2H * P2W; i += NT) {
    const int r = i / P2W, cc = i - r * P2W;
    sp[r][cc] = a.phi[(uint32_t)wrap(y0 - 2 + r, ny) * nx + wrap(x0 - 2 + cc, nx)];
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
  const int ty = t / ATW, tx = t - ty * ATW;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= nx || y >= ny) return;
  const uint32_t k = (uint32_t)y * nx + x;
  const float phi = sp[ty + 2][tx + 2];
  float u, v;
  if (a.vmode == VEL_SEP) {
    u = a.tf * a.ax[x] * a.ay[y];
    v = a.tf * a.bx[x] * a.by[y];
  } else {
    u = a.tf * a.ux[k];
    v = a.tf * a.uy[k];
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
    a.gu[k] += a.tf * phi * gx;
    a.gv[k] += a.tf * phi * gy;
  }
}

template <int TX, bool WALLS, int VMODE, int ST>
hipError_t phi_step_m(int model, const StepArgs& a, int nb, hipStream_t s) {
  if (model == 2)
    hipLaunchKernelGGL((k_phi_step<TX, WALLS, VMODE, 2, ST>), dim3(nb), dim3(TX), 0, s, a);
  else if (model == 1)
    hipLaunchKernelGGL((k_phi_step<TX, WALLS, VMODE, 1, ST>), dim3(nb), dim3(TX), 0, s, a);
  else if constexpr (ST == ST_F32)
    hipLaunchKernelGGL((k_phi_step<TX, WALLS, VMODE, 3, ST>), dim3(nb), dim3(TX), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int TX>
hipError_t phi_batch_t(int vmode, bool model2, const BatchArgs& b, int grid, hipStream_t s) {
  if (vmode == VEL_SEP) {
    if (model2) hipLaunchKernelGGL((k_phi_batch<TX, VEL_SEP, true>), dim3(grid), dim3(TX), 0, s, b);
    else hipLaunchKernelGGL((k_phi_batch<TX, VEL_SEP, false>), dim3(grid), dim3(TX), 0, s, b);
  } else {
    if (model2) hipLaunchKernelGGL((k_phi_batch<TX, VEL_FIELD, true>), dim3(grid), dim3(TX), 0, s, b);
    else hipLaunchKernelGGL((k_phi_batch<TX, VEL_FIELD, false>), dim3(grid), dim3(TX), 0, s, b);
  }
  return hipGetLastError();
}

template <int TX, bool WALLS, int ST>
hipError_t phi_step_v(int vmode, int model, const StepArgs& a, int nb, hipStream_t s) {
  switch (vmode) {
    case VEL_SEP: return phi_step_m<TX, WALLS, VEL_SEP, ST>(model, a, nb, s);
    case VEL_FIELD: return phi_step_m<TX, WALLS, VEL_FIELD, ST>(model, a, nb, s);
    default: return phi_step_m<TX, WALLS, VEL_NSFIELD, ST>(model, a, nb, s);
  }
}

template <int ST>
hipError_t phi_step_t(int tx, bool walls, int vmode, int model, const StepArgs& a, int nb,
                      hipStream_t s) {
  switch (tx) {
    case 64:
      return walls ? phi_step_v<64, true, ST>(vmode, model, a, nb, s)
                   : phi_step_v<64, false, ST>(vmode, model, a, nb, s);
    case 128:
      return walls ? phi_step_v<128, true, ST>(vmode, model, a, nb, s)
                   : phi_step_v<128, false, ST>(vmode, model, a, nb, s);
    case 256:
      return walls ? phi_step_v<256, true, ST>(vmode, model, a, nb, s)
                   : phi_step_v<256, false, ST>(vmode, model, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

template <int TX, int ST>
void ns_step_l(bool walls, const NsArgs& a, int nb, hipStream_t s) {
  if (walls) hipLaunchKernelGGL((k_ns_step<TX, true, ST>), dim3(nb), dim3(TX), 0, s, a);
  else hipLaunchKernelGGL((k_ns_step<TX, false, ST>), dim3(nb), dim3(TX), 0, s, a);
}

template <int ST>
hipError_t ns_step_t(int tx, bool walls, const NsArgs& a, int nb, hipStream_t s) {
  switch (tx) {
    case 64: ns_step_l<64, ST>(walls, a, nb, s); break;
    case 128: ns_step_l<128, ST>(walls, a, nb, s); break;
    case 256: ns_step_l<256, ST>(walls, a, nb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ST>
void init_l(bool walls, int vmode, dim3 grid, hipStream_t s, const Coef& c, int nx, int ny,
            uint32_t plane, const float* phi0, const float* ax, const float* ay,
            const float* bx, const float* by, const float* ux, const float* uy, float tf,
            char* g, float* f) {
  const bool sep = vmode == VEL_SEP;
  if (walls && sep)
    hipLaunchKernelGGL((k_init<true, VEL_SEP, ST>), grid, dim3(256), 0, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
  else if (walls)
    hipLaunchKernelGGL((k_init<true, VEL_FIELD, ST>), grid, dim3(256), 0, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
  else if (sep)
    hipLaunchKernelGGL((k_init<false, VEL_SEP, ST>), grid, dim3(256), 0, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
  else
    hipLaunchKernelGGL((k_init<false, VEL_FIELD, ST>), grid, dim3(256), 0, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, g, f);
}

}  // namespace

uint32_t population_bytes(int storage, uint32_t plane) { return pop_bytes(storage, plane); }

hipError_t launch_phi_step(int tx, bool walls, int vmode, int model, int storage,
                           const StepArgs& a, int nblocks, hipStream_t s) {
  switch (storage) {
    case ST_F32: return phi_step_t<ST_F32>(tx, walls, vmode, model, a, nblocks, s);
    case ST_F16: return phi_step_t<ST_F16>(tx, walls, vmode, model, a, nblocks, s);
    case ST_BF16: return phi_step_t<ST_BF16>(tx, walls, vmode, model, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

int phi_batch_blocks_per_cu(int tx, int vmode, bool model2) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  const bool sep = vmode == VEL_SEP;
#define LBM_OCC(T)                                                                          \
  e = sep ? (model2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch<T, VEL_SEP, true>, T, 0)    \
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch<T, VEL_SEP, false>, T, 0))   \
          : (model2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch<T, VEL_FIELD, true>, T, 0)  \
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch<T, VEL_FIELD, false>, T, 0))
  switch (tx) {
    case 64: LBM_OCC(64); break;
    case 128: LBM_OCC(128); break;
    case 256: LBM_OCC(256); break;
    default: break;
  }
#undef LBM_OCC
  return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_phi_batch(int tx, int vmode, bool model2, const BatchArgs& b, int grid,
                            hipStream_t s) {
  if (grid <= 0 || (grid & 7) != 0 || b.n <= 0) return hipErrorInvalidValue;
  switch (tx) {
    case 64: return phi_batch_t<64>(vmode, model2, b, grid, s);
    case 128: return phi_batch_t<128>(vmode, model2, b, grid, s);
    case 256: return phi_batch_t<256>(vmode, model2, b, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ns_step(int tx, bool walls, int storage, const NsArgs& a, int nblocks,
                          hipStream_t s) {
  switch (storage) {
    case ST_F32: return ns_step_t<ST_F32>(tx, walls, a, nblocks, s);
    case ST_F16: return ns_step_t<ST_F16>(tx, walls, a, nblocks, s);
    case ST_BF16: return ns_step_t<ST_BF16>(tx, walls, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init(bool walls, int vmode, int storage, const Coef& c, int nx, int ny,
                       uint32_t plane, const float* phi0, const float* ax, const float* ay,
                       const float* bx, const float* by, const float* ux, const float* uy,
                       float tf, void* g, float* f, hipStream_t s) {
  const dim3 grid((nx + 255) / 256, ny);
  char* gb = static_cast<char*>(g);
  switch (storage) {
    case ST_F32: init_l<ST_F32>(walls, vmode, grid, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, gb, f); break;
    case ST_F16: init_l<ST_F16>(walls, vmode, grid, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, gb, f); break;
    case ST_BF16: init_l<ST_BF16>(walls, vmode, grid, s, c, nx, ny, plane, phi0, ax, ay, bx, by, ux, uy, tf, gb, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_phi_field(bool walls, int storage, const void* g, uint32_t plane, int nx,
                            int ny, float* phi, hipStream_t s) {
  const dim3 grid((nx + 255) / 256, ny);
  switch (storage) {
    case ST_F32:
      if (walls) hipLaunchKernelGGL((k_phi_field<true, ST_F32>), grid, dim3(256), 0, s, g, plane, nx, ny, phi);
      else hipLaunchKernelGGL((k_phi_field<false, ST_F32>), grid, dim3(256), 0, s, g, plane, nx, ny, phi);
      break;
    case ST_F16:
      if (walls) hipLaunchKernelGGL((k_phi_field<true, ST_F16>), grid, dim3(256), 0, s, g, plane, nx, ny, phi);
      else hipLaunchKernelGGL((k_phi_field<false, ST_F16>), grid, dim3(256), 0, s, g, plane, nx, ny, phi);
      break;
    case ST_BF16:
      if (walls) hipLaunchKernelGGL((k_phi_field<true, ST_BF16>), grid, dim3(256), 0, s, g, plane, nx, ny, phi);
      else hipLaunchKernelGGL((k_phi_field<false, ST_BF16>), grid, dim3(256), 0, s, g, plane, nx, ny, phi);
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

}  // namespace lbmch
