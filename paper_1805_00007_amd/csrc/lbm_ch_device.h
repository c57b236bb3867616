// Device helpers shared by the gfx950 kernels of the lattice Boltzmann
// Cahn-Hilliard solver (Zhang, Guo & Liang, arXiv:1805.00007): the D2Q9 lattice,
// range-checked buffer access, the population storage modes, the mass-conserving
// store, and the isotropic stencils.  Included by the kernel sources only.
#pragma once

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

// A value that every lane of the wave holds identically (loaded from one address),
// moved into scalar registers word by word.  The compiler cannot prove such a value
// uniform when it is loaded after a store, and would then run every buffer access that
// takes it as a scalar operand once per lane value.
template <class T>
__device__ __forceinline__ T wave_uniform(const T& x) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T y;
  __builtin_memcpy(&y, w, sizeof(T));
  return y;
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
// Cache-policy bit "nt" (non-temporal) of a buffer access on gfx950: the populations a
// step writes are read again only by the next step, not by this one, so their stores
// stream past the caches and leave L2 to the rows that neighbouring tiles re-read.
// Measured on MI355X (2048^2): 2-5 % faster for float32 stores; the 2-byte stores of
// the 16-bit storage modes become ~10 % slower with it, so they keep the default.
constexpr int CP_NT = 2;
__device__ __forceinline__ void stb_nt(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, CP_NT);
}

// Population storage.  ST_F32: nine float32 populations.  ST_F16 / ST_BF16: the rest
// population g_0 in float32, then the eight moving populations as 16-bit codes of
// g_i / w_i (i = 1..8) in IEEE half or bfloat16.  The moving populations of Eq. geq are
// w_i (eta mu + phi s_i(u)), of order w_i |u|, so their scaled values are small and a
// 16-bit code keeps them to ~1e-4 of that size; g_0 ~ phi stays in float32 and, through
// the mass closure below, absorbs the rounding of the others.
//
// Layout in memory: row-interleaved.  Lattice row r holds its nine populations next to
// each other, each as a run of `pitch` values (x fastest, pitch >= nx), so that one
// row of the whole state is one contiguous range of memory:
//   float32: population i of row r starts at float (9 r + i) pitch;
//   16-bit:  row r starts at byte 20 r pitch, with g_0 as pitch float32 values followed
//            by g_1..g_8 as pitch 16-bit codes each.
// A step reads three consecutive rows of the source and writes one row of the
// destination per marched row, so the memory system sees a few compact streams rather
// than eighteen planes far apart.
enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };
constexpr float INV_W[9] = {9.0f / 4, 9.0f, 9.0f, 9.0f, 9.0f, 36.0f, 36.0f, 36.0f, 36.0f};

__host__ __device__ constexpr uint32_t pop_row_bytes(int st, uint32_t pitch) {
  return st == ST_F32 ? 36u * pitch : 20u * pitch;
}
__host__ __device__ constexpr uint32_t pop_bytes(int st, uint32_t pitch, uint32_t ny) {
  return pop_row_bytes(st, pitch) * ny;
}
// Byte offset of the first value of population i in lattice row `row`.
template <int ST>
__host__ __device__ constexpr uint32_t pop_off(int i, uint32_t pitch, uint32_t row) {
  return ST == ST_F32 ? ((row * 9u + (uint32_t)i) * pitch) * 4u
                      : row * 20u * pitch + (i == 0 ? 0u : 4u * pitch + (uint32_t)(i - 1) * 2u * pitch);
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
__device__ __forceinline__ float ldpop(rsrc_t s, int i, uint32_t pitch, uint32_t col,
                                       uint32_t row) {
  if (ST == ST_F32 || i == 0) return ldb(s, col * 4u, pop_off<ST>(i, pitch, row));
  const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(s, col * 2u, pop_off<ST>(i, pitch, row), 0);
  return WT[i] * dec16<ST>(h);
}

// Pull of the nine populations arriving at (x, y): g_i(x, y) = g_i*(x - c_i, y - c_i).
// With walls, a population whose source lies beyond a wall is the opposite one that
// left (x, y) (half-way bounce-back).  y is a lattice row (block-uniform); cc, cm, cp
// are the columns x, x-1, x+1 (wrapped).  Plane and row offsets travel in the
// instruction's scalar offset, so a load costs no vector ALU work beyond its column.
template <bool WALLS, int ST>
__device__ __forceinline__ void pull9(rsrc_t s, uint32_t pitch, int ny, int y, uint32_t cc,
                                      uint32_t cm, uint32_t cp, float g[9]) {
  const uint32_t ym = y == 0 ? ny - 1 : y - 1;
  const uint32_t yp = y == ny - 1 ? 0 : y + 1;
  const uint32_t yc = y;
  g[0] = ldpop<ST>(s, 0, pitch, cc, yc);
  g[1] = ldpop<ST>(s, 1, pitch, cm, yc);
  g[3] = ldpop<ST>(s, 3, pitch, cp, yc);
  if (WALLS && y == 0) {
    g[2] = ldpop<ST>(s, 4, pitch, cc, yc);
    g[5] = ldpop<ST>(s, 7, pitch, cc, yc);
    g[6] = ldpop<ST>(s, 8, pitch, cc, yc);
  } else {
    g[2] = ldpop<ST>(s, 2, pitch, cc, ym);
    g[5] = ldpop<ST>(s, 5, pitch, cm, ym);
    g[6] = ldpop<ST>(s, 6, pitch, cp, ym);
  }
  if (WALLS && y == ny - 1) {
    g[4] = ldpop<ST>(s, 2, pitch, cc, yc);
    g[7] = ldpop<ST>(s, 5, pitch, cc, yc);
    g[8] = ldpop<ST>(s, 6, pitch, cc, yc);
  } else {
    g[4] = ldpop<ST>(s, 4, pitch, cc, yp);
    g[7] = ldpop<ST>(s, 7, pitch, cp, yp);
    g[8] = ldpop<ST>(s, 8, pitch, cm, yp);
  }
}

// Population I at byte offset `off` (plane and row) and column col, everything in the
// lane's own offset: for loads whose row differs between the lanes of a wave.  (A scalar
// offset that differs between lanes makes the compiler issue the load once per distinct
// value.)  I fixes the element size and the weight of a 16-bit code.
template <int ST, int I>
__device__ __forceinline__ float ldpop_lane(rsrc_t s, uint32_t col, uint32_t off) {
  if (ST == ST_F32 || I == 0) return ldb(s, col * 4u + off, 0);
  const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(s, col * 2u + off, 0, 0);
  return WT[I] * dec16<ST>(h);
}

// pull9 for a row that differs between the lanes of a wave (the margins of a
// two-dimensional tile): same values, but all offsets travel in the lanes' own offsets
// and the wall cases are chosen per lane, so a wave issues nine loads whatever rows its
// lanes hold.  A bounced-back population has the weight of the one it replaces.
template <bool WALLS, int ST>
__device__ __forceinline__ void pull9_lanes(rsrc_t s, uint32_t pitch, int ny, int y,
                                            uint32_t cc, uint32_t cm, uint32_t cp,
                                            float g[9]) {
  const uint32_t ym = y == 0 ? ny - 1 : y - 1;
  const uint32_t yp = y == ny - 1 ? 0 : y + 1;
  const uint32_t yc = y;
  const bool w0 = WALLS && y == 0, w1 = WALLS && y == ny - 1;
  g[0] = ldpop_lane<ST, 0>(s, cc, pop_off<ST>(0, pitch, yc));
  g[1] = ldpop_lane<ST, 1>(s, cm, pop_off<ST>(1, pitch, yc));
  g[3] = ldpop_lane<ST, 3>(s, cp, pop_off<ST>(3, pitch, yc));
  g[2] = ldpop_lane<ST, 2>(s, cc, w0 ? pop_off<ST>(4, pitch, yc) : pop_off<ST>(2, pitch, ym));
  g[5] = ldpop_lane<ST, 5>(s, w0 ? cc : cm,
                           w0 ? pop_off<ST>(7, pitch, yc) : pop_off<ST>(5, pitch, ym));
  g[6] = ldpop_lane<ST, 6>(s, w0 ? cc : cp,
                           w0 ? pop_off<ST>(8, pitch, yc) : pop_off<ST>(6, pitch, ym));
  g[4] = ldpop_lane<ST, 4>(s, cc, w1 ? pop_off<ST>(2, pitch, yc) : pop_off<ST>(4, pitch, yp));
  g[7] = ldpop_lane<ST, 7>(s, w1 ? cc : cp,
                           w1 ? pop_off<ST>(5, pitch, yc) : pop_off<ST>(7, pitch, yp));
  g[8] = ldpop_lane<ST, 8>(s, w1 ? cc : cm,
                           w1 ? pop_off<ST>(6, pitch, yc) : pop_off<ST>(8, pitch, yp));
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
__device__ __forceinline__ void finish_store(rsrc_t d, uint32_t pitch, uint32_t col,
                                             uint32_t row, double m, float g[9]) {
  if (ST == ST_F32) {
    close_mass(m, g);
#pragma unroll
    for (int i = 0; i < 9; ++i) stb_nt(d, g[i], col * 4u, pop_off<ST>(i, pitch, row));
    return;
  }
  uint32_t h[9];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    h[i] = enc16<ST>(g[i] * INV_W[i]);
    g[i] = WT[i] * dec16<ST>(h[i]);
  }
  g[0] = (float)(m - sum8_hi(g));
  stb(d, g[0], col * 4u, pop_off<ST>(0, pitch, row));
#pragma unroll
  for (int i = 1; i < 9; ++i)
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)h[i], d, col * 2u,
                                          pop_off<ST>(i, pitch, row), 0);
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

}  // namespace
}  // namespace lbmch
