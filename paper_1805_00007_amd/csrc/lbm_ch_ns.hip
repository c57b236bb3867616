// gfx950 kernel of the coupled Navier-Stokes step of the lattice Boltzmann
// Cahn-Hilliard solver (Zhang, Guo & Liang, arXiv:1805.00007) for Rayleigh-Taylor
// flows: a pressure-based incompressible D2Q9 BGK model driven by the phase field's
// forces (the model and its moments are stated in include/lbm_ch.h).  The phase-field
// step then runs with the velocity and pressure this kernel writes.  The same file holds
// the single-launch coupled step, which does both in one kernel.
#include "lbm_ch_device.h"
#include "lbm_ch_stencil.h"

#include <type_traits>

namespace lbmch {
namespace {

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
  const uint32_t pitch = a.pitch;
  const rsrc_t rg = make_rsrc(a.gsrc, pop_bytes(ST, pitch, ny));
  const rsrc_t rf = make_rsrc(a.fsrc, pop_bytes(ST_F32, pitch, ny));
  const rsrc_t rfd = make_rsrc(a.fdst, a.fdst ? pop_bytes(ST_F32, pitch, ny) : 0u);
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
  auto stage2 = [&](int r, int jj) {
    const float* pm = s_phi[(r - 1) & 7];
    const float* p0 = s_phi[r & 7];
    const float* pp = s_phi[(r + 1) & 7];
    s_mu[r & 3][jj] = mu_bulk(c, p0[jj]) - c.kappa * lap9(pm, p0, pp, jj);
  };

  // Halo columns come from the four halo lanes of wave 0; the other lanes of that wave
  // issue the same pulls at an out-of-range offset (a raw buffer load returns 0 without
  // a memory access), and waves 1.. skip them (a scalar branch).
  constexpr uint32_t OOB = 0x3FFFFFC0u;
  const bool hwave = __builtin_amdgcn_readfirstlane(t) < 64;
  const uint32_t hvc = hl ? (uint32_t)hc : OOB, hvm = hl ? (uint32_t)hm : OOB,
                 hvp = hl ? (uint32_t)hp : OOB;
  auto pull_g = [&](int r, uint32_t cc, uint32_t cm, uint32_t cq, float g[9]) {
    float sg;
    const int sr = row_of<WALLS>(r, ny, sg);
    pull9<WALLS, ST>(rg, pitch, ny, sr, cc, cm, cq, g);
  };
  {
    // prologue: rows y0-2 .. y0+1 of g (own and halo columns), all pulled before any
    // is used, so the block waits for memory once
    float ga[4][9], gh[4][9];
#pragma unroll
    for (int q = 0; q < 4; ++q) pull_g(y0 - 2 + q, xc, xm, xp, ga[q]);
    if (hwave) {
#pragma unroll
      for (int q = 0; q < 4; ++q) pull_g(y0 - 2 + q, hvc, hvm, hvp, gh[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s_phi[(y0 - 2 + q) & 7][j] = sum9(ga[q]);
    if (hwave) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float ph = sum9(gh[q]);
        if (hl) s_phi[(y0 - 2 + q) & 7][hj] = ph;
      }
    }
  }
  __syncthreads();
  stage2(y0 - 1, j);
  stage2(y0, j);
  if (t < 2) {
    stage2(y0 - 1, j2);
    stage2(y0, j2);
  }
  __syncthreads();

#pragma unroll 1
  for (int k = 0; k < rows; ++k) {
    const int y = y0 + k;
    // g of row y+2 first (needed before the barrier), then f of row y (needed after
    // it): the wait for g leaves f in flight across the stage-2 work, and f is used in
    // the same row, so no load is outstanding when the loop branches back
    float gn[9], ghn[9], fpop[9];
    __builtin_amdgcn_sched_barrier(0);
    pull_g(y + 2, xc, xm, xp, gn);
    if (hwave) pull_g(y + 2, hvc, hvm, hvp, ghn);
    __builtin_amdgcn_sched_barrier(0);
    pull9<WALLS, ST_F32>(rf, pitch, ny, y, xc, xm, xp, fpop);
    __builtin_amdgcn_sched_barrier(0);
    s_phi[(y + 2) & 7][j] = sum9(gn);
    if (hwave) {
      const float ph = sum9(ghn);
      if (hl) s_phi[(y + 2) & 7][hj] = ph;
    }
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
          stb_nt(rfd, om1 * fpop[i] + om * feq + c.srcf * G, off, pop_off<ST_F32>(i, pitch, (uint32_t)y));
        }
      }
    }
  }
}


// ---------------------------------------------------------------------------------
// Single-launch coupled step: one time step of the Navier-Stokes populations f and the
// phase-field populations g in one kernel, without the velocity and pressure round
// trip through memory.
//
// A block owns an output tile of 64 columns x R rows and computes, from the source
// populations alone, every value its outputs depend on, each on the tile plus a margin:
//   phi  (pull g, Eq. macroscopicg)                    margin 4
//   mu   (Eq. mu)                                      margin 3
//   u, v, p and the NS force (pull f, model of lbm_ch.h) margin 2
//   D = div(phi u) (Eq. mark3)                         margin 1
//   F = F1 + F2 (Eqs. t0-phiu, mark3), the collisions of g and f, and the stores on the
//   tile itself.
// All pulls of a block are issued at once, so it waits for memory once; the margins
// are recomputed by every block that needs them (their pulls are L2 hits) instead of
// being marched through.  This suits lattices too small for a march to pay (the
// 256 x 1024 Rayleigh-Taylor case is latency-bound), and it moves only the state: 144
// bytes per node update in float32.  Every value is computed by code compiled without
// implicit multiply-add contraction, so a node computed as a margin of one block rounds
// exactly as in the block that owns it, and results do not depend on R.
//
// Walls: phi and mu of rows beyond a wall come from the mirrored rows (the pulls are
// taken there); u, v, p of such rows are copied from the mirrored rows after the NS
// stage, with u and v negated (lbm_ch.h).
#pragma clang fp contract(off)

constexpr int RT_C = 64;          // output columns per block
constexpr int RT_W = RT_C + 8;    // region row length (margin 4 on each side)

// Region node e of the band of width m around the output tile (e < band size):
// rows 4 - m .. 3 + R + m, columns 4 - m .. 67 + m, the tile's own nodes excluded.
template <int R>
__device__ __forceinline__ void band_node(int e, int m, int& rr, int& cc) {
  const int w = RT_C + 2 * m;
  if (e < m * w) {
    rr = 4 - m + e / w;
    cc = 4 - m + e % w;
    return;
  }
  e -= m * w;
  if (e < R * 2 * m) {
    rr = 4 + e / (2 * m);
    const int k = e % (2 * m);
    cc = k < m ? 4 - m + k : 4 + RT_C + k - m;
    return;
  }
  e -= R * 2 * m;
  rr = 4 + R + e / w;
  cc = 4 - m + e % w;
}

// The Navier-Stokes moments at one node from its pulled f and the phi / mu regions
// (index k, row stride RT_W): velocity, pressure and, with fo, the post-collision f.
__device__ __forceinline__ void ns_node(const Coef& c, const float* ph, const float* mu, int k,
                                        const float f[9], float& u, float& v, float& pr,
                                        float* fo) {
  const float phi = ph[k];
  const float rho = fmaf(c.a, phi, c.b);
  const float mux = t1_dx(mu + k - RT_W, mu + k, mu + k + RT_W, 0);
  const float muy = t1_dy(mu + k - RT_W, mu + k, mu + k + RT_W, 0);
  const float fsx = -phi * mux, fsy = -phi * muy;
  const float fbx = rho * c.accel_x, fby = -(rho - c.rho_mean) * c.gravity;
  const float corr = c.aM * t1_lap(mu + k - RT_W, mu + k, mu + k + RT_W, 0);
  const float mx = ((f[1] - f[3]) + (f[5] - f[6])) + (f[8] - f[7]);
  const float my = ((f[2] - f[4]) + (f[5] + f[6])) - (f[7] + f[8]);
  const float sm = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
  const float inv = rcp(rho - 0.5f * corr);
  u = (mx + 0.5f * (fsx + fbx)) * inv;
  v = (my + 0.5f * (fsy + fby)) * inv;
  const float drx = c.a * t1_dx(ph + k - RT_W, ph + k, ph + k + RT_W, 0);
  const float dry = c.a * t1_dy(ph + k - RT_W, ph + k, ph + k + RT_W, 0);
  const float usq15 = 1.5f * (u * u + v * v);
  // p = cs^2/(1 - w0) [sum_{i>0} f_i + u.grad rho / 2 + rho w0 s_0(u)], cs^2/(1-w0) = 3/5
  pr = 0.6f * ((sm + 0.5f * (u * drx + v * dry)) - WT[0] * rho * usq15);
  if (!fo) return;
  const float Fx = (fsx + fbx) + u * corr, Fy = (fsy + fby) + v * corr;
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
    const float G = WT[i] * ((3.0f * (cF - uF) + 9.0f * cu * cF) + 3.0f * cu * cr);
    fo[i] = (om1 * f[i] + om * feq) + c.srcf * G;
  }
}

template <int R, bool WALLS, bool MODEL2, int ST>
__global__ void __launch_bounds__(64 * R) k_rt_step(const StepArgs a, const float* fsrc, float* fdst) {
  constexpr int NT = 64 * R;
  constexpr int N = (R + 8) * RT_W;
  constexpr int NXG = N - R * RT_C;                       // phi margin nodes
  constexpr int NXF = (R + 4) * (RT_C + 4) - R * RT_C;    // NS margin nodes
  constexpr int EG = (NXG + NT - 1) / NT, EF = (NXF + NT - 1) / NT;
  __shared__ float s_ph[N], s_mu[N], s_qx[N], s_qy[N], s_p[N], s_d[MODEL2 ? N : 1];
  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const uint32_t pitch = a.pitch;
  const rsrc_t rg = make_rsrc(a.src, pop_bytes(ST, pitch, ny));
  const rsrc_t rgd = make_rsrc(a.dst, pop_bytes(ST, pitch, ny));
  const rsrc_t rf = make_rsrc(fsrc, pop_bytes(ST_F32, pitch, ny));
  const rsrc_t rfd = make_rsrc(fdst, pop_bytes(ST_F32, pitch, ny));
  int L = blockIdx.x;
  if (a.xcd_remap) {
    const int per = gridDim.x >> 3;
    L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int x0 = (L % a.nstrips) * RT_C;
  const int y0 = (L / a.nstrips) * R;
  const int t = threadIdx.x;

  // region node (rr, cc) <-> lattice row y0 - 4 + rr, column x0 - 4 + cc (wrapped).
  // x0 - 4 + cc lies in [-4, nx + 66] and y0 - 4 + rr in [-4, ny + R + 2], so one
  // conditional wrap suffices on lattices at least that wide (or tall); smaller ones
  // take the remainder.  Own rows are wave-uniform (one wave = one tile row) and keep
  // their row offsets in the scalar operand; margin rows differ between lanes.  In the
  // last, partly filled row chunk of a short walled lattice, margin rows far past the
  // wall mirror to negative rows: they feed only outputs outside the lattice (never
  // stored), and their offsets, in the range-checked lane operand, read as zero.
  auto pull = [&](rsrc_t r, auto st, auto lanes, int rr, int cc, float g[9]) {
    constexpr int S = decltype(st)::value;
    int sr = y0 - 4 + rr;
    if (WALLS || ny < R + 8) {
      float sg;
      sr = row_of<WALLS>(sr, ny, sg);
    } else {
      sr = sr < 0 ? sr + ny : (sr >= ny ? sr - ny : sr);
    }
    int x = x0 - 4 + cc;
    if (nx >= RT_W) x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    else x = (x % nx + nx) % nx;
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    if constexpr (decltype(lanes)::value)
      pull9_lanes<WALLS, S>(r, pitch, ny, sr, (uint32_t)x, xm, xp, g);
    else
      pull9<WALLS, S>(r, pitch, ny, sr, (uint32_t)x, xm, xp, g);
  };
  using GS = std::integral_constant<int, ST>;
  using FS = std::integral_constant<int, ST_F32>;
  using OWN = std::false_type;
  using MARGIN = std::true_type;
  // a row beyond a wall (its NS values are mirrored, not computed)
  auto beyond = [&](int rr) {
    const int y = y0 - 4 + rr;
    return WALLS && (y < 0 || y >= ny);
  };

  // own node: column x0 + (t % 64), row y0 + t / 64 (the same for a whole wave)
  static_assert(RT_C == 64, "one wave per tile row");
  const int tw = __builtin_amdgcn_readfirstlane(t / RT_C);
  const int ro = 4 + tw, co = 4 + t % RT_C, ko = ro * RT_W + co;
  const int xo = x0 + t % RT_C, yo = y0 + tw;
  const bool own = xo < nx && yo < ny;

  // --- all pulls at once: g of the own node and the phi margin, f of the own node and
  // the NS margin
  float go[9], fo[9], gx[EG][9], fx[EF][9];
  pull(rg, GS{}, OWN{}, ro, co, go);
  pull(rf, FS{}, OWN{}, ro, co, fo);
#pragma unroll
  for (int i = 0; i < EG; ++i) {
    const int e = t + i * NT;
    if (e < NXG) {
      int rr, cc;
      band_node<R>(e, 4, rr, cc);
      pull(rg, GS{}, MARGIN{}, rr, cc, gx[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < EF; ++i) {
    const int e = t + i * NT;
    if (e < NXF) {
      int rr, cc;
      band_node<R>(e, 2, rr, cc);
      pull(rf, FS{}, MARGIN{}, rr, cc, fx[i]);
    }
  }
  // --- phi (Eq. macroscopicg)
  float lo;
  const float phio = sum9(go, lo);
  if (__builtin_expect(!__builtin_isfinite(phio), 0) && own && a.nonfinite) *a.nonfinite = 1;
  s_ph[ko] = phio;
#pragma unroll
  for (int i = 0; i < EG; ++i) {
    const int e = t + i * NT;
    if (e < NXG) {
      int rr, cc;
      band_node<R>(e, 4, rr, cc);
      s_ph[rr * RT_W + cc] = sum9(gx[i]);
    }
  }
  __syncthreads();
  // --- mu on the tile plus 3 (Eq. mu)
  for (int e = t; e < (R + 6) * (RT_C + 6); e += NT) {
    const int k = (1 + e / (RT_C + 6)) * RT_W + 1 + e % (RT_C + 6);
    s_mu[k] = t1_mu(c, s_ph[k], t1_lap(s_ph + k - RT_W, s_ph + k, s_ph + k + RT_W, 0));
  }
  __syncthreads();
  // --- Navier-Stokes on the tile plus 2: q = phi u and p into LDS, f* of the own node
  float uo = 0.0f, vo = 0.0f, fn[9];
  if (!beyond(ro)) {
    float po;
    ns_node(c, s_ph, s_mu, ko, fo, uo, vo, po, fn);
    s_qx[ko] = phio * uo;
    s_qy[ko] = phio * vo;
    s_p[ko] = po;
  }
#pragma unroll
  for (int i = 0; i < EF; ++i) {
    const int e = t + i * NT;
    if (e < NXF) {
      int rr, cc;
      band_node<R>(e, 2, rr, cc);
      if (!beyond(rr)) {
        const int k = rr * RT_W + cc;
        float u, v, pr;
        ns_node(c, s_ph, s_mu, k, fx[i], u, v, pr, nullptr);
        s_qx[k] = s_ph[k] * u;
        s_qy[k] = s_ph[k] * v;
        s_p[k] = pr;
      }
    }
  }
  if (own && !beyond(ro)) {
#pragma unroll
    for (int i = 0; i < 9; ++i)
      stb_nt(rfd, fn[i], (uint32_t)xo * 4u, pop_off<ST_F32>(i, pitch, (uint32_t)yo));
  }
  if (WALLS && (y0 - 2 < 0 || y0 + R + 2 > ny)) {  // a block-uniform branch
    __syncthreads();
    // rows of the NS region beyond a wall: mirror images (q = phi u odd, p even)
    for (int e = t; e < (R + 4) * (RT_C + 4); e += NT) {
      const int rr = 2 + e / (RT_C + 4), cc = 2 + e % (RT_C + 4);
      if (!beyond(rr)) continue;
      const int y = y0 - 4 + rr;
      const int ym = y < 0 ? -1 - y : 2 * ny - 1 - y;
      const int rm = ym - (y0 - 4);
      const int k = rr * RT_W + cc, km = rm * RT_W + cc;
      const bool in = rm >= 2 && rm < R + 6 && !beyond(rm);
      s_qx[k] = in ? -s_qx[km] : 0.0f;
      s_qy[k] = in ? -s_qy[km] : 0.0f;
      s_p[k] = in ? s_p[km] : 0.0f;
    }
  }
  __syncthreads();
  // --- D = div(phi u) on the tile plus 1 (Eq. mark3)
  if (MODEL2) {
    for (int e = t; e < (R + 2) * (RT_C + 2); e += NT) {
      const int k = (3 + e / (RT_C + 2)) * RT_W + 3 + e % (RT_C + 2);
      s_d[k] = t1_dx(s_qx + k - RT_W, s_qx + k, s_qx + k + RT_W, 0) +
               t1_dy(s_qy + k - RT_W, s_qy + k, s_qy + k + RT_W, 0);
    }
    __syncthreads();
  }
  if (!own) return;
  // --- F = F1 + F2 with F1 = (phi/rho)(F_s + F_b - grad p), collision of g, store
  const float* m = s_mu + ko;
  const float mux = t1_dx(m - RT_W, m, m + RT_W, 0), muy = t1_dy(m - RT_W, m, m + RT_W, 0);
  const float* q = s_p + ko;
  const float pgx = t1_dx(q - RT_W, q, q + RT_W, 0), pgy = t1_dy(q - RT_W, q, q + RT_W, 0);
  const float rho = fmaf(c.a, phio, c.b);
  const float tx = (-phio * mux + rho * c.accel_x) - pgx;
  const float ty = (-phio * muy - (rho - c.rho_mean) * c.gravity) - pgy;
  const float s1 = phio * rcp(rho);
  float fxg = s1 * tx, fyg = s1 * ty;
  if (MODEL2) {
    const float* dd = s_d + ko;
    fxg = fmaf(c.k2, t1_dx(dd - RT_W, dd, dd + RT_W, 0), fxg);
    fyg = fmaf(c.k2, t1_dy(dd - RT_W, dd, dd + RT_W, 0), fyg);
  }
  collide_strict(c, phio, s_mu[ko], uo, vo, fxg, fyg, go);
  finish_store<ST>(rgd, pitch, (uint32_t)xo, (uint32_t)yo, (double)phio + (double)lo, go);
}
#pragma clang fp contract(fast)


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
    case 512: ns_step_l<512, ST>(walls, a, nb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R, int ST>
hipError_t rt_step_r(bool walls, bool model2, const StepArgs& a, const float* fs, float* fd,
                     int nb, hipStream_t s) {
#define LBM_RT(W, M) hipLaunchKernelGGL((k_rt_step<R, W, M, ST>), dim3(nb), dim3(64 * R), 0, s, a, fs, fd)
  if (walls) {
    if (model2) { LBM_RT(true, true); } else { LBM_RT(true, false); }
  } else {
    if (model2) { LBM_RT(false, true); } else { LBM_RT(false, false); }
  }
#undef LBM_RT
  return hipGetLastError();
}

template <int ST>
hipError_t rt_step_t(int rows, bool walls, bool model2, const StepArgs& a, const float* fs,
                     float* fd, int nb, hipStream_t s) {
  switch (rows) {
    case 2: return rt_step_r<2, ST>(walls, model2, a, fs, fd, nb, s);
    case 4: return rt_step_r<4, ST>(walls, model2, a, fs, fd, nb, s);
    case 8: return rt_step_r<8, ST>(walls, model2, a, fs, fd, nb, s);
    case 16: return rt_step_r<16, ST>(walls, model2, a, fs, fd, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_ns_step(int tx, bool walls, int storage, const NsArgs& a, int nblocks,
                          hipStream_t s) {
  switch (storage) {
    case ST_F32: return ns_step_t<ST_F32>(tx, walls, a, nblocks, s);
    case ST_F16: return ns_step_t<ST_F16>(tx, walls, a, nblocks, s);
    case ST_BF16: return ns_step_t<ST_BF16>(tx, walls, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

int rt_step_rows(int ty) { return ty >= 16 ? 16 : ty >= 8 ? 8 : ty >= 4 ? 4 : 2; }

hipError_t launch_rt_step(int rows, bool walls, int model, int storage, const StepArgs& a,
                          const float* fsrc, float* fdst, int nblocks, hipStream_t s) {
  if (model != 1 && model != 2) return hipErrorInvalidValue;
  switch (storage) {
    case ST_F32: return rt_step_t<ST_F32>(rows, walls, model == 2, a, fsrc, fdst, nblocks, s);
    case ST_F16: return rt_step_t<ST_F16>(rows, walls, model == 2, a, fsrc, fdst, nblocks, s);
    case ST_BF16: return rt_step_t<ST_BF16>(rows, walls, model == 2, a, fsrc, fdst, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbmch
