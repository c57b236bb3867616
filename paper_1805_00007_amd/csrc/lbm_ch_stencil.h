// Stencils, chemical potential and tau_g = 1 collision of the lattice Boltzmann
// Cahn-Hilliard solver (Zhang, Guo & Liang, arXiv:1805.00007) in a form that rounds the
// same wherever it is inlined: compiled without implicit multiply-add contraction, with
// every fused multiply-add written out.  Kernels that compute one value at several
// places (unrolled copies of a march, halo and own nodes of a tile) use these, so that
// their results do not depend on the tile shape.  Used by the tau_g = 1 tile
// (lbm_ch_step.hip) and the single-launch coupled step (lbm_ch_ns.hip); included by the
// kernel sources only.
#pragma once

#include "lbm_ch_device.h"

namespace lbmch {
namespace {

#pragma clang fp contract(off)
// The isotropic stencils of Sec. III on LDS rows in lattice order (rm: y-1, r0: y,
// rp: y+1), as the weighted neighbour sums
//   d_x = [4 (E - W) + (NE + SE) - (NW + SW)] / 12,  d_y = [4 (N - S) + (NE + NW) - (SE + SW)] / 12,
//   lap = [4 (E + W + N + S) + (NE + NW + SE + SW) - 20 C] / 6.
__device__ __forceinline__ float t1_dx(const float* rm, const float* r0, const float* rp, int j) {
  const float diag = (rp[j + 1] + rm[j + 1]) - (rp[j - 1] + rm[j - 1]);
  return fmaf(4.0f, r0[j + 1] - r0[j - 1], diag) * (1.0f / 12.0f);
}
__device__ __forceinline__ float t1_dy(const float* rm, const float* r0, const float* rp, int j) {
  const float diag = (rp[j + 1] + rp[j - 1]) - (rm[j + 1] + rm[j - 1]);
  return fmaf(4.0f, rp[j] - rm[j], diag) * (1.0f / 12.0f);
}
__device__ __forceinline__ float t1_lap(const float* rm, const float* r0, const float* rp, int j) {
  const float axis = (r0[j + 1] + r0[j - 1]) + (rp[j] + rm[j]);
  const float diag = (rp[j + 1] + rp[j - 1]) + (rm[j + 1] + rm[j - 1]);
  return fmaf(4.0f, axis, fmaf(-20.0f, r0[j], diag)) * (1.0f / 6.0f);
}
// mu of Eq. mu with the double well of Eq. bulk: 2 beta (phi - phi_A)(phi - phi_B)
// (2 phi - phi_A - phi_B) - kappa lap(phi).
__device__ __forceinline__ float t1_mu(const Coef& c, float phi, float lap) {
  const float bulk = c.beta2 * ((phi - c.phia) * (phi - c.phib)) * ((phi + phi) - (c.phia + c.phib));
  return fmaf(-c.kappa, lap, bulk);
}

// Collision at tau_g = 1: g_i* = w_i (eta mu + phi s_i(u)) + (3/2) w_i c_i.F (Eqs. geq,
// liangFi, LB), written pairwise for opposite directions c_i = -c_j:
//   g_i,j* = w_i (P +- Q),  P = eta mu - 1.5 phi u^2 + 4.5 phi (c_i.u)^2,
//                           Q = 3 phi c_i.u + 1.5 c_i.F.
// g_0* is left to the mass-conserving store.
__device__ __forceinline__ void collide_t1(const Coef& c, float phi, float mu, float u, float v,
                                           float fx, float fy, float g[9]) {
  const float A = fmaf(-1.5f * phi, fmaf(u, u, v * v), c.eta * mu);
  const float p3 = 3.0f * phi, p45 = 4.5f * phi;
  const float hx = 1.5f * fx, hy = 1.5f * fy;
  auto pair = [&](float e, float h, float w, float& gp, float& gm) {
    const float P = fmaf(p45 * e, e, A);
    const float Q = fmaf(p3, e, h);
    gp = w * (P + Q);
    gm = w * (P - Q);
  };
  pair(u, hx, WT[1], g[1], g[3]);
  pair(v, hy, WT[2], g[2], g[4]);
  pair(u + v, hx + hy, WT[5], g[5], g[7]);
  pair(v - u, hy - hx, WT[6], g[6], g[8]);
}

// Collision of Eq. LB at any tau_g (g^eq of Eq. geq, S_i = 3 w_i c_i.F of Eq. liangFi):
//   g_i* = (1 - omega) g_i + w_i (omega (eta mu + phi s_i(u)) + srcg c_i.F),  i = 1..8,
// with every multiply-add written out; g_0* is left to the mass-conserving store.
__device__ __forceinline__ void collide_strict(const Coef& c, float phi, float mu, float u,
                                               float v, float fx, float fy, float g[9]) {
  const float A = fmaf(-1.5f * phi, fmaf(u, u, v * v), c.eta * mu);
  const float om1 = 1.0f - c.omega;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float cu = CX[i] * u + CY[i] * v;
    const float cf = CX[i] * fx + CY[i] * fy;
    const float eq = fmaf(phi * cu, fmaf(4.5f, cu, 3.0f), A);
    g[i] = fmaf(om1, g[i], WT[i] * fmaf(c.omega, eq, c.srcg * cf));
  }
}
#pragma clang fp contract(fast)

}  // namespace
}  // namespace lbmch
