// gfx950 time-step kernels of the lattice Boltzmann Cahn-Hilliard solver
// (Zhang, Guo & Liang, arXiv:1805.00007).  The public contract, the method and the
// boundary rules are stated in include/lbm_ch.h; this file holds the fused phase-field
// step (single lattice and batched); the coupled Navier-Stokes step is in lbm_ch_ns.hip.
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
#include "lbm_ch_device.h"
#include "lbm_ch_stencil.h"

namespace lbmch {
namespace {

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
// REC: also store phi of every marched row (the source state's order parameter) to
// a.phi_rec.
template <int TX, bool WALLS, int VMODE, int MODEL, int ST, bool REC = false>
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
  const uint32_t pitch = a.pitch;
  const uint32_t rb = (uint32_t)nx * 4u;
  const rsrc_t rsrc = make_rsrc(a.src, pop_bytes(ST, pitch, ny));
  const rsrc_t rdst = make_rsrc(a.dst, pop_bytes(ST, pitch, ny));
  rsrc_t ru, rv, rp;
  if (VFIELD) {
    ru = make_rsrc(a.ux, nodes * 4u);
    rv = make_rsrc(a.uy, nodes * 4u);
  }
  if (NSC) rp = make_rsrc(a.pf, nodes * 4u);
  rsrc_t rxh;
  if (HIST) rxh = make_rsrc(a.xh, 2u * nodes * 4u);
  rsrc_t rrec;
  if (REC) rrec = make_rsrc(a.phi_rec, nodes * 4u);

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
  // They sit in wave 0; the other waves skip the halo pull (a scalar branch).
  const bool hl = t < 4;
  const bool hwave = __builtin_amdgcn_readfirstlane(t) < 64;
  const int hlog = t < 2 ? x0 - 2 + t : x0 + TX - 2 + t;
  const int hc = ((hlog % nx) + nx) % nx;
  // Every lane of wave 0 issues the halo pull (a wave-uniform branch, so the wait for
  // the halo row is the only wait inside it); lanes other than the four halo lanes use
  // an offset beyond the buffer, for which a raw buffer load returns 0 without
  // accessing memory.
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
    pull9<WALLS, ST>(rsrc, pitch, ny, sr, cc, cm, cp, R.g);
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
    if (__builtin_expect(!__builtin_isfinite(R.phi), 0) && a.nonfinite) *a.nonfinite = 1;
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
    // Lanes past the right edge of a ragged last strip wrap to columns another strip
    // owns and compute the very same values from the very same inputs, so their stores
    // duplicate identical data; they need no branch (which would make the wait for the
    // next row's pull also wait for this row's stores).  Model 3 keeps the branch: a
    // duplicate lane could read a history value its owner has already replaced.
    if (HIST && !active) return;
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
      stb_nt(rxh, xx, vc * 4u, (uint32_t)y * rb);
      stb_nt(rxh, xy, vc * 4u, nodes * 4u + (uint32_t)y * rb);
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
    if (REC) stb_nt(rrec, R.phi, vc * 4u, (uint32_t)y * rb);
    collide_g(c, R.phi, R.lo, m0[j], u, v, fx, fy, R.g);
    finish_store<ST>(rdst, pitch, vc, (uint32_t)y, (double)R.phi + (double)R.lo, R.g);
  };

  // Prologue: rows y0-2d .. y0+2d through stage 1, rows y0-d and y0 through stage 2.
  //
  // Register pipeline.  Iteration y issues the pull of row y+3d first, then runs stage
  // 2 of row y+d and stage 3 of row y while it is in flight, and consumes it (stage 1)
  // last, so no load is outstanding when the loop branches back (a record with a load
  // in flight is then never moved between registers, which would make the wave wait
  // for every outstanding load).  A, B, C hold rows y, y+d, y+2d; N receives y+3d.
  const int d = dir;
  RowRec A, B, C, N, H0;
  {
    // wave 0 pulls the first two halo rows with the own rows, so the prologue has two
    // dependent round trips to memory instead of three
    RowRec T0, T1, U0, U1;
    if (hwave) {
      issue(y0 - 2 * d, hvc, hvm, hvp, U0, false);
      issue(y0 - d, hvc, hvm, hvp, U1, false);
    }
    issue(y0 - 2 * d, vc, vm, vp, T0);
    issue(y0 - d, vc, vm, vp, T1);
    issue(y0, vc, vm, vp, A);
    issue(y0 + d, vc, vm, vp, B);
    if (hwave) {
      stage1(y0 - 2 * d, U0, hj, axh, bxh, hl);
      stage1(y0 - d, U1, hj, axh, bxh, hl);
      issue(y0, hvc, hvm, hvp, U0, false);
      issue(y0 + d, hvc, hvm, hvp, U1, false);
    }
    stage1(y0 - 2 * d, T0, j, axc, bxc);
    stage1(y0 - d, T1, j, axc, bxc);
    stage1(y0, A, j, axc, bxc);
    stage1(y0 + d, B, j, axc, bxc);
    if (hwave) {
      stage1(y0, U0, hj, axh, bxh, hl);
      stage1(y0 + d, U1, hj, axh, bxh, hl);
    }
  }
  if (hwave) issue(y0 + 2 * d, hvc, hvm, hvp, H0, false);
  issue(y0 + 2 * d, vc, vm, vp, C);
  __syncthreads();
  stage2(y0 - d, j);
  stage2(y0, j);
  if (t < 2) {
    stage2(y0 - d, j2);
    stage2(y0, j2);
  }
  __syncthreads();
  // row y0+2d shares its ring slot with y0-2d, which stage 2 no longer needs
  if (hwave) stage1(y0 + 2 * d, H0, hj, axh, bxh, hl);
  stage1(y0 + 2 * d, C, j, axc, bxc);

  // One marching row.  On a block's last row the pull of y+3d is not needed; it is
  // clamped to the last row the block does need (already in cache), so the pull has no
  // branch and fetches nothing extra, and its stage 1 is skipped (a scalar branch), so
  // the block does not wait for it.
  const int last_needed = y0 + (rows + 1) * d;
  // On tall tiles (bandwidth-bound marches) a wave raises its issue priority while it
  // puts its row's pull in flight, so waves about to load go before waves in their
  // compute stages (2048^2: 0.8 % faster with float32, ~6 % with 16-bit storage).  Short
  // tiles are latency-bound chains, where it costs a few per cent, and keep priority 0.
  const bool prio = a.ty >= 8;
#pragma unroll 1
  for (int k = 0; k < rows; ++k) {
    const int y = y0 + k * d;
    const int ynext = k + 1 < rows ? y + 3 * d : last_needed;
    __builtin_amdgcn_sched_barrier(0);
    if (prio) __builtin_amdgcn_s_setprio(2);
    if (hwave) issue(ynext, hvc, hvm, hvp, H0, false);
    __builtin_amdgcn_sched_barrier(0);
    issue(ynext, vc, vm, vp, N);
    __builtin_amdgcn_sched_barrier(0);
    if (prio) __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stage2(y + d, j);
    if (t < 2) stage2(y + d, j2);
    __syncthreads();
    stage3(y, A);
    __builtin_amdgcn_sched_barrier(0);
    // row y+3d takes the ring slot of row y-d, which no later stage reads
    if (k + 1 < rows) {
      if (hwave) stage1(y + 3 * d, H0, hj, axh, bxh, hl);
      stage1(y + 3 * d, N, j, axc, bxc);
    }
    A = B;
    B = C;
    C = N;
  }
}

// ---------------------------------------------------------------------------------
// Fused step at tau_g = 1 (models 1 and 2, prescribed velocity; any storage).
//
// With omega = 1 the collision of Eq. LB forgets the pulled populations: g_i* =
// g_i^eq + S_i / 2, so once a row has been pulled and summed its record keeps only
// phi (with the FP64 remainder of the sum) and the velocity of the row.  Four such
// small records rotate through a loop unrolled four times (once per marching
// direction), so every record and every LDS ring slot has a fixed register or
// address: no record is copied between registers at the back edge and no ring address
// is computed per row.  Stages, halo lanes, marching directions and the XCD band
// mapping are those of phi_tile.
//
// The unrolled copies of the stages must round identically, or results would depend
// on the tile shape: this section is compiled without implicit multiply-add
// contraction, and every fused multiply-add in it is written out.
#pragma clang fp contract(off)
// A row's pull in flight (populations plus the velocity inputs of the row), and a
// row's state after stage 1.
struct PullT1 {
  float g[9];
  float a, b;             // separable: ay[y], by[y]; field: u, v of the node (as loaded)
};
struct RowT1 {
  float phi, lo;          // phi and the FP64 remainder of the sum
  float a, b;             // separable: ay[y], by[y] times tf (and parity); field: u, v
};

template <int TX, bool WALLS, int VMODE, int MODEL, int ST, bool REC = false>
__device__ __forceinline__ void phi_tile_t1(const StepArgs& a, const int L) {
  static_assert(VMODE == VEL_SEP || VMODE == VEL_FIELD, "prescribed velocity only");
  static_assert(MODEL == 1 || MODEL == 2, "models 1 and 2");
  constexpr bool MODEL2 = MODEL == 2;
  constexpr bool VFIELD = VMODE == VEL_FIELD;
  constexpr int LW = TX + 4;
  constexpr int QR = MODEL2 ? 4 : 1;
  __shared__ float s_phi[4][LW];
  __shared__ float s_mu[4][LW];
  __shared__ float s_qx[QR][LW];
  __shared__ float s_qy[QR][LW];
  __shared__ float s_d[QR][LW];

  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const uint32_t nodes = (uint32_t)nx * ny;
  const uint32_t pitch = a.pitch;
  const uint32_t rb = (uint32_t)nx * 4u;
  const rsrc_t rsrc = make_rsrc(a.src, pop_bytes(ST, pitch, ny));
  const rsrc_t rdst = make_rsrc(a.dst, pop_bytes(ST, pitch, ny));
  rsrc_t ru, rv, rrec;
  if (VFIELD) {
    ru = make_rsrc(a.ux, nodes * 4u);
    rv = make_rsrc(a.uy, nodes * 4u);
  }
  if (REC) rrec = make_rsrc(a.phi_rec, nodes * 4u);

  const int t = threadIdx.x;
  const int x0 = (L % a.nstrips) * TX;
  const int chunk = L / a.nstrips;
  const int rows = min(a.ty, ny - chunk * a.ty);
  const int d = (chunk & 1) ? -1 : 1;  // vertically adjacent chunks march in opposite directions
  const int y0 = d > 0 ? chunk * a.ty : chunk * a.ty + rows - 1;

  const int xc = (x0 + t) % nx;
  const uint32_t vc = xc;
  const uint32_t vm = xc == 0 ? nx - 1 : xc - 1;
  const uint32_t vp = xc == nx - 1 ? 0 : xc + 1;
  const bool hl = t < 4;
  const bool hwave = __builtin_amdgcn_readfirstlane(t) < 64;
  const int hlog = t < 2 ? x0 - 2 + t : x0 + TX - 2 + t;
  const int hc = ((hlog % nx) + nx) % nx;
  constexpr uint32_t OOB = 0x3FFFFFC0u;  // column whose byte offset exceeds any buffer
  const uint32_t hvc = hl ? hc : OOB;
  const uint32_t hvm = hl ? (hc == 0 ? nx - 1 : hc - 1) : OOB;
  const uint32_t hvp = hl ? (hc == nx - 1 ? 0 : hc + 1) : OOB;
  const int hj = t < 2 ? t : TX + t;
  const int j = t + 2;
  const int j2 = t == 0 ? 1 : TX + 2;

  float axc = 0.f, bxc = 0.f, axh = 0.f, bxh = 0.f;
  if (VMODE == VEL_SEP) {
    axc = a.ax[xc];
    bxc = a.bx[xc];
    if (hl) {
      axh = a.ax[hc];
      bxh = a.bx[hc];
    }
  }

  // Row m of the march is lattice row y0 + m d (m = -2 .. rows + 1).  Its LDS slot is
  // (m + 2) & 3 and its state st[m & 3].
  auto issue = [&](int r, uint32_t cc, uint32_t cm, uint32_t cp, PullT1& P) {
    float sg;
    const int sr = row_of<WALLS>(r, ny, sg);
    pull9<WALLS, ST>(rsrc, pitch, ny, sr, cc, cm, cp, P.g);
    if (VMODE == VEL_SEP) {
      P.a = a.ay[sr];
      P.b = a.by[sr];
    } else {
      P.a = ldb(ru, cc * 4u, (uint32_t)sr * rb);
      P.b = ldb(rv, cc * 4u, (uint32_t)sr * rb);
    }
  };
  auto stage1 = [&](int r, const PullT1& P, RowT1& R, int jj, float axv, float bxv, int slot,
                    bool wr = true) {
    float sg;
    row_of<WALLS>(r, ny, sg);
    R.phi = sum9(P.g, R.lo);
    if (__builtin_expect(!__builtin_isfinite(R.phi), 0) && a.nonfinite) *a.nonfinite = 1;
    const float f = a.tf * sg;
    float u, v;
    if (VMODE == VEL_SEP) {
      R.a = P.a * f;
      R.b = P.b * f;
      u = axv * R.a;
      v = bxv * R.b;
    } else {
      u = R.a = f * P.a;
      v = R.b = f * P.b;
    }
    if (!wr) return;
    s_phi[slot][jj] = R.phi;
    if (MODEL2) {
      s_qx[slot][jj] = R.phi * u;
      s_qy[slot][jj] = R.phi * v;
    }
  };
  // Stencils take their three rows in lattice order (slots of lattice rows y - 1, y,
  // y + 1), whichever way the chunk marches, so that every value is computed by the same
  // expression in every tile.
  auto stage2 = [&](int jj, int sm, int s0, int sp) {
    const float* pm = s_phi[sm];
    const float* p0 = s_phi[s0];
    const float* pp = s_phi[sp];
    s_mu[s0][jj] = t1_mu(c, p0[jj], t1_lap(pm, p0, pp, jj));
    if (MODEL2)
      s_d[s0][jj] = t1_dx(s_qx[sm], s_qx[s0], s_qx[sp], jj) + t1_dy(s_qy[sm], s_qy[s0], s_qy[sp], jj);
  };
  auto stage3 = [&](int y, const RowT1& R, int sm, int s0, int sp) {
    const float mux = t1_dx(s_mu[sm], s_mu[s0], s_mu[sp], j);
    const float muy = t1_dy(s_mu[sm], s_mu[s0], s_mu[sp], j);
    // F1 = (phi/rho) F_s with F_s = -phi grad mu (Eq. t0-phiu, grad p = 0); F2 = K grad D
    const float rho = fmaf(c.a, R.phi, c.b);
    const float s1 = -(R.phi * R.phi) * rcp(rho);
    float fx = s1 * mux, fy = s1 * muy;
    if (MODEL2) {
      fx = fmaf(c.k2, t1_dx(s_d[sm], s_d[s0], s_d[sp], j), fx);
      fy = fmaf(c.k2, t1_dy(s_d[sm], s_d[s0], s_d[sp], j), fy);
    }
    const float u = VMODE == VEL_SEP ? axc * R.a : R.a;
    const float v = VMODE == VEL_SEP ? bxc * R.b : R.b;
    if (REC) stb_nt(rrec, R.phi, vc * 4u, (uint32_t)y * rb);
    float g[9];
    collide_t1(c, R.phi, s_mu[s0][j], u, v, fx, fy, g);
    finish_store<ST>(rdst, pitch, vc, (uint32_t)y, (double)R.phi + (double)R.lo, g);
  };

  // Rows the march needs: m = -2 .. rows + 1; a pull past the last one is clamped to it
  // (already in cache) so that every row issues the same loads.
  const int last_needed = y0 + (rows + 1) * d;
  RowT1 st[4];
  PullT1 pb, hb;
  {
    PullT1 T0, T1, P0, P1, U0, U1;
    RowT1 X;
    if (hwave) {
      issue(y0 - 2 * d, hvc, hvm, hvp, U0);
      issue(y0 - d, hvc, hvm, hvp, U1);
    }
    issue(y0 - 2 * d, vc, vm, vp, T0);
    issue(y0 - d, vc, vm, vp, T1);
    issue(y0, vc, vm, vp, P0);
    issue(y0 + d, vc, vm, vp, P1);
    // row m = 2 is pulled with the others (its stage 1 waits for the ring slot of row
    // m = -2, below), so a chunk start waits for memory once (twice in wave 0)
    issue(y0 + 2 * d, vc, vm, vp, pb);
    if (hwave) {
      stage1(y0 - 2 * d, U0, X, hj, axh, bxh, 0, hl);
      stage1(y0 - d, U1, X, hj, axh, bxh, 1, hl);
      issue(y0, hvc, hvm, hvp, U0);
      issue(y0 + d, hvc, hvm, hvp, U1);
      issue(y0 + 2 * d, hvc, hvm, hvp, hb);
    }
    stage1(y0 - 2 * d, T0, X, j, axc, bxc, 0);
    stage1(y0 - d, T1, X, j, axc, bxc, 1);
    stage1(y0, P0, st[0], j, axc, bxc, 2);
    stage1(y0 + d, P1, st[1], j, axc, bxc, 3);
    if (hwave) {
      stage1(y0, U0, X, hj, axh, bxh, 2, hl);
      stage1(y0 + d, U1, X, hj, axh, bxh, 3, hl);
    }
  }
  __syncthreads();
  {
    // rows m = -1 (slots 0, 1, 2 in march order) and m = 0 (slots 1, 2, 3)
    const int a0 = d > 0 ? 0 : 2, a2 = d > 0 ? 2 : 0, b1 = d > 0 ? 1 : 3, b3 = d > 0 ? 3 : 1;
    stage2(j, a0, 1, a2);
    stage2(j, b1, 2, b3);
    if (t < 2) {
      stage2(j2, a0, 1, a2);
      stage2(j2, b1, 2, b3);
    }
  }
  __syncthreads();
  {
    RowT1 X;
    if (hwave) stage1(y0 + 2 * d, hb, X, hj, axh, bxh, 0, hl);  // row m = 2, slot 0
  }
  stage1(y0 + 2 * d, pb, st[2], j, axc, bxc, 0);

  const bool prio = a.ty >= 8;
  // Row m = k + J (J = m & 3): pull row m + 3, stage 2 of row m + 1, stage 3 of row m
  // (st[J]), stage 1 of row m + 3 into st[(J + 3) & 3] once its pull has arrived.  Slots:
  // row m + q -> (J + q + 2) & 3; the stencils get the slots of rows m + q - D and
  // m + q + D (lattice order), so the loop exists once per marching direction D with
  // every slot and register a constant.  On the last row the pull is clamped to a row
  // already in cache and its stage 1 skipped.
#define LBM_T1_ROW(J, D)                                                                   \
  if (k + (J) < rows) {                                                                    \
    const int m = k + (J);                                                                 \
    const int y = y0 + m * (D);                                                            \
    const bool more = m + 1 < rows;                                                        \
    const int ynext = more ? y + 3 * (D) : last_needed;                                    \
    __builtin_amdgcn_sched_barrier(0);                                                     \
    if (prio) __builtin_amdgcn_s_setprio(2);                                               \
    if (hwave) issue(ynext, hvc, hvm, hvp, hb);                                            \
    __builtin_amdgcn_sched_barrier(0);                                                     \
    issue(ynext, vc, vm, vp, pb);                                                          \
    __builtin_amdgcn_sched_barrier(0);                                                     \
    if (prio) __builtin_amdgcn_s_setprio(0);                                               \
    __builtin_amdgcn_sched_barrier(0);                                                     \
    __syncthreads();                                                                       \
    {                                                                                      \
      constexpr int lo = (D) > 0 ? ((J) + 2) & 3 : (J) & 3;                                \
      constexpr int hi = (D) > 0 ? (J) & 3 : ((J) + 2) & 3;                                \
      stage2(j, lo, ((J) + 3) & 3, hi);                                                    \
      if (t < 2) stage2(j2, lo, ((J) + 3) & 3, hi);                                        \
    }                                                                                      \
    __syncthreads();                                                                       \
    {                                                                                      \
      constexpr int lo = (D) > 0 ? ((J) + 1) & 3 : ((J) + 3) & 3;                          \
      constexpr int hi = (D) > 0 ? ((J) + 3) & 3 : ((J) + 1) & 3;                          \
      stage3(y, st[(J) & 3], lo, ((J) + 2) & 3, hi);                                       \
    }                                                                                      \
    __builtin_amdgcn_sched_barrier(0);                                                     \
    if (more) {                                                                            \
      if (hwave) {                                                                         \
        RowT1 X;                                                                           \
        stage1(y + 3 * (D), hb, X, hj, axh, bxh, ((J) + 1) & 3, hl);                       \
      }                                                                                    \
      stage1(y + 3 * (D), pb, st[((J) + 3) & 3], j, axc, bxc, ((J) + 1) & 3);              \
    }                                                                                      \
  }
  if (d > 0) {
#pragma unroll 1
    for (int k = 0; k < rows; k += 4) {
      LBM_T1_ROW(0, 1)
      LBM_T1_ROW(1, 1)
      LBM_T1_ROW(2, 1)
      LBM_T1_ROW(3, 1)
    }
  } else {
#pragma unroll 1
    for (int k = 0; k < rows; k += 4) {
      LBM_T1_ROW(0, -1)
      LBM_T1_ROW(1, -1)
      LBM_T1_ROW(2, -1)
      LBM_T1_ROW(3, -1)
    }
  }
#undef LBM_T1_ROW
}
#pragma clang fp contract(fast)

// Model 3 carries two more values per row record; it gets the register budget of
// three waves per SIMD so that nothing spills.
// T1: the tau_g = 1 tile (models 1 and 2, prescribed velocity only).
template <int VMODE, int MODEL, int ST>
constexpr bool t1_ok() {
  return (MODEL == 1 || MODEL == 2) && (VMODE == VEL_SEP || VMODE == VEL_FIELD);
}
template <int TX, bool WALLS, int VMODE, int MODEL, int ST, bool REC, bool T1>
__device__ __forceinline__ void step_tile(const StepArgs& a, int L) {
  if constexpr (T1 && t1_ok<VMODE, MODEL, ST>())
    phi_tile_t1<TX, WALLS, VMODE, MODEL, ST, REC>(a, L);
  else
    phi_tile<TX, WALLS, VMODE, MODEL, ST, REC>(a, L);
}

// ---------------------------------------------------------------------------------
// Single-pass tile of the tau_g = 1 step (periodic lattice, float32 populations,
// prescribed velocity, models 1 and 2): for small lattices, where a march is a chain of
// dependent row loads.  A workgroup owns 64 columns x R rows (one wave per row) and
// issues every pull it needs at once: its own nodes and a margin of 2 (phi, and q =
// phi u for model 2); then mu and D on the tile plus 1, then stage 3 on the tile.  The
// margins are recomputed by each workgroup that needs them (L2 hits), so the workgroup
// waits for memory once.  Every value is formed by the same expressions as in
// phi_tile_t1, so results are bitwise those of the marching tiles.
#pragma clang fp contract(off)
constexpr int PS_C = 64;          // output columns per workgroup
constexpr int PS_W = PS_C + 4;    // region row length (margin 2 on each side)

template <int R, int VMODE, bool MODEL2, bool REC, int ST>
__global__ void __launch_bounds__(64 * R) k_phi_pass(const StepArgs a) {
  constexpr int NT = 64 * R;
  constexpr int N = (R + 4) * PS_W;
  constexpr int NX = N - R * PS_C;                 // margin nodes
  constexpr int EX = (NX + NT - 1) / NT;
  __shared__ float s_ph[N], s_mu[N], s_qx[MODEL2 ? N : 1], s_qy[MODEL2 ? N : 1],
      s_d[MODEL2 ? N : 1];
  const Coef& c = a.c;
  const int nx = a.nx, ny = a.ny;
  const uint32_t pitch = a.pitch;
  const rsrc_t rsrc = make_rsrc(a.src, pop_bytes(ST, pitch, ny));
  const rsrc_t rdst = make_rsrc(a.dst, pop_bytes(ST, pitch, ny));
  int L = blockIdx.x;
  if (a.xcd_remap) {
    const int per = gridDim.x >> 3;
    L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int x0 = (L % a.nstrips) * PS_C;
  const int y0 = (L / a.nstrips) * R;
  const int t = threadIdx.x;
  const uint32_t nodes = (uint32_t)nx * ny;
  const uint32_t rb = (uint32_t)nx * 4u;

  // region node (rr, cc) <-> lattice row y0 - 2 + rr, column x0 - 2 + cc (periodic);
  // x0 - 2 + cc lies in [-2, nx + 64] and y0 - 2 + rr in [-2, ny + R]
  auto col = [&](int cc) {
    int x = x0 - 2 + cc;
    if (nx >= PS_W) return x < 0 ? x + nx : (x >= nx ? x - nx : x);
    return (x % nx + nx) % nx;
  };
  auto row = [&](int rr) {
    int y = y0 - 2 + rr;
    if (ny >= R + 4) return y < 0 ? y + ny : (y >= ny ? y - ny : y);
    return (y % ny + ny) % ny;
  };
  // stage 1 at one region node: pull, phi (with its FP64 remainder), the velocity factors
  // as phi_tile_t1 keeps them (separable: ay[y] tf and bx[x] ... as a, b) and q = phi u
  struct Node {
    float phi, lo, a, b, u, v;
  };
  auto node = [&](auto lanes, int rr, int cc) {
    const int x = col(cc), y = row(rr);
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    float g[9];
    if constexpr (decltype(lanes)::value)
      pull9_lanes<false, ST>(rsrc, pitch, ny, y, (uint32_t)x, xm, xp, g);
    else
      pull9<false, ST>(rsrc, pitch, ny, y, (uint32_t)x, xm, xp, g);
    Node n;
    n.phi = sum9(g, n.lo);
    const float f = a.tf;  // periodic: the row parity factor is 1
    if (VMODE == VEL_SEP) {
      n.a = a.ay[y] * f;
      n.b = a.by[y] * f;
      n.u = a.ax[x] * n.a;
      n.v = a.bx[x] * n.b;
    } else {
      const uint32_t k = (uint32_t)y * nx + x;
      n.a = n.u = f * a.ux[k];
      n.b = n.v = f * a.uy[k];
    }
    return n;
  };
  using OWN = std::false_type;
  using MARGIN = std::true_type;

  // own node: column x0 + (t % 64), row y0 + t / 64 (the same for a whole wave)
  static_assert(PS_C == 64, "one wave per tile row");
  const int tw = __builtin_amdgcn_readfirstlane(t / PS_C);
  const int ro = 2 + tw, co = 2 + t % PS_C, ko = ro * PS_W + co;
  const int xo = x0 + t % PS_C, yo = y0 + tw;
  const bool own = xo < nx && yo < ny;

  const Node no = node(OWN{}, ro, co);
  if (__builtin_expect(!__builtin_isfinite(no.phi), 0) && own && a.nonfinite) *a.nonfinite = 1;
  s_ph[ko] = no.phi;
  if (MODEL2) {
    s_qx[ko] = no.phi * no.u;
    s_qy[ko] = no.phi * no.v;
  }
#pragma unroll
  for (int i = 0; i < EX; ++i) {
    const int e = t + i * NT;
    if (e < NX) {
      int rr, cc;  // the band of width 2 around the tile, row by row
      if (e < 2 * PS_W) {
        rr = e / PS_W;
        cc = e % PS_W;
      } else if (e < 2 * PS_W + 4 * R) {
        const int q = e - 2 * PS_W;
        rr = 2 + q / 4;
        const int k = q % 4;
        cc = k < 2 ? k : PS_C + k;
      } else {
        const int q = e - 2 * PS_W - 4 * R;
        rr = 2 + R + q / PS_W;
        cc = q % PS_W;
      }
      const Node m = node(MARGIN{}, rr, cc);
      const int k = rr * PS_W + cc;
      s_ph[k] = m.phi;
      if (MODEL2) {
        s_qx[k] = m.phi * m.u;
        s_qy[k] = m.phi * m.v;
      }
    }
  }
  __syncthreads();
  // stage 2: mu and D on the tile plus 1 (Eqs. mu, mark3)
  for (int e = t; e < (R + 2) * (PS_C + 2); e += NT) {
    const int k = (1 + e / (PS_C + 2)) * PS_W + 1 + e % (PS_C + 2);
    s_mu[k] = t1_mu(c, s_ph[k], t1_lap(s_ph + k - PS_W, s_ph + k, s_ph + k + PS_W, 0));
    if (MODEL2)
      s_d[k] = t1_dx(s_qx + k - PS_W, s_qx + k, s_qx + k + PS_W, 0) +
               t1_dy(s_qy + k - PS_W, s_qy + k, s_qy + k + PS_W, 0);
  }
  __syncthreads();
  if (!own) return;
  // stage 3 (as in phi_tile_t1)
  const float* m = s_mu + ko;
  const float mux = t1_dx(m - PS_W, m, m + PS_W, 0), muy = t1_dy(m - PS_W, m, m + PS_W, 0);
  const float rho = fmaf(c.a, no.phi, c.b);
  const float s1 = -(no.phi * no.phi) * rcp(rho);
  float fx = s1 * mux, fy = s1 * muy;
  if (MODEL2) {
    const float* dd = s_d + ko;
    fx = fmaf(c.k2, t1_dx(dd - PS_W, dd, dd + PS_W, 0), fx);
    fy = fmaf(c.k2, t1_dy(dd - PS_W, dd, dd + PS_W, 0), fy);
  }
  if (REC) {
    const rsrc_t rrec = make_rsrc(a.phi_rec, nodes * 4u);
    stb_nt(rrec, no.phi, (uint32_t)xo * 4u, (uint32_t)yo * rb);
  }
  float g[9];
  collide_t1(c, no.phi, s_mu[ko], no.u, no.v, fx, fy, g);
  finish_store<ST>(rdst, pitch, (uint32_t)xo, (uint32_t)yo, (double)no.phi + (double)no.lo, g);
}
#pragma clang fp contract(fast)

template <int TX, bool WALLS, int VMODE, int MODEL, int ST, bool REC = false, bool T1 = false>
__global__ void __launch_bounds__(TX)
__attribute__((amdgpu_waves_per_eu(MODEL == 3 ? 3 : WPE_PHI, 8)))
k_phi_step(const StepArgs a) {
  int L = blockIdx.x;
  if (a.xcd_remap) {  // workgroup w runs on XCD w % 8: give each XCD a band of chunks
    const int per = gridDim.x >> 3;
    L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  step_tile<TX, WALLS, VMODE, MODEL, ST, REC, T1>(a, L);
}

// Batched step, one tile per workgroup: the tiles of many lattices (one instance table
// entry each) in one launch.  The tiles are numbered instance by instance; when the grid
// is a multiple of 8, XCD x (workgroups w with w % 8 == x) gets the contiguous range
// [x per, (x + 1) per), so vertically adjacent tiles of one lattice share an L2.  Same
// register budget as the single-lattice kernel.
template <int TX, int VMODE, bool MODEL2, bool T1>
__global__ void __launch_bounds__(TX) __attribute__((amdgpu_waves_per_eu(WPE_PHI, 8)))
k_phi_batch(const BatchArgs b) {
  int v = blockIdx.x;
  if ((gridDim.x & 7) == 0) {
    const int per = gridDim.x >> 3;
    v = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  if (v >= b.total) return;
  int lo_i = 0, hi_i = b.n;  // instance of tile v: start[inst] <= v < start[inst + 1]
  while (hi_i - lo_i > 1) {
    const int mid = (lo_i + hi_i) >> 1;
    if (b.start[mid] <= v) lo_i = mid; else hi_i = mid;
  }
  StepArgs a = b.args[lo_i];
  if (b.parity) {
    const void* t = a.src;
    a.src = a.dst;
    a.dst = const_cast<void*>(t);
  }
  step_tile<TX, false, VMODE, MODEL2 ? 2 : 1, ST_F32, false, T1>(a, v - b.start[lo_i]);
}

// Batched step, persistent: the tiles of many lattices (one instance table entry each)
// in one launch of a grid sized to the resident capacity.  The tiles are numbered instance by instance; XCD x (workgroups
// w with w % 8 == x) owns the contiguous range [x per, (x + 1) per) and its workgroups
// stride through it, so vertically adjacent tiles of one lattice share that XCD's L2.
// Every workgroup leaves the loop after at most ceil(per / slots) tiles.
#ifndef WPE_BATCH
#define WPE_BATCH 3
#endif
template <int TX, int VMODE, bool MODEL2, bool T1>
__global__ void __launch_bounds__(TX) __attribute__((amdgpu_waves_per_eu(WPE_BATCH, 8)))
k_phi_batch_persistent(const BatchArgs b) {
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
  int inst = __builtin_amdgcn_readfirstlane(lo_i);
#pragma unroll 1
  for (; v < hi; v += slots) {
    // the table is read after the previous tile's stores: its values (the same in every
    // lane) are moved to scalar registers explicitly
    while (__builtin_amdgcn_readfirstlane(b.start[inst + 1]) <= v) ++inst;
    StepArgs a = wave_uniform(b.args[inst]);
    if (b.parity) {
      const void* t = a.src;
      a.src = a.dst;
      a.dst = const_cast<void*>(t);
    }
    step_tile<TX, false, VMODE, MODEL2 ? 2 : 1, ST_F32, false, T1>(
        a, v - __builtin_amdgcn_readfirstlane(b.start[inst]));
    __syncthreads();  // the LDS rings are reused by the next tile
  }
}

template <int TX, bool WALLS, int VMODE, int ST>
hipError_t phi_step_m(int model, bool t1, const StepArgs& a, int nb, hipStream_t s) {
  if constexpr (t1_ok<VMODE, 2, ST>()) {
    if (t1 && (model == 1 || model == 2)) {
      if (model == 2)
        hipLaunchKernelGGL((k_phi_step<TX, WALLS, VMODE, 2, ST, false, true>), dim3(nb), dim3(TX), 0, s, a);
      else
        hipLaunchKernelGGL((k_phi_step<TX, WALLS, VMODE, 1, ST, false, true>), dim3(nb), dim3(TX), 0, s, a);
      return hipGetLastError();
    }
  }
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

template <int TX, bool PERSIST, bool T1>
hipError_t phi_batch_t(int vmode, bool model2, const BatchArgs& b, int grid, hipStream_t s) {
#define LBM_BATCH_LAUNCH(V, M)                                                                 \
  if (PERSIST)                                                                                 \
    hipLaunchKernelGGL((k_phi_batch_persistent<TX, V, M, T1>), dim3(grid), dim3(TX), 0, s, b); \
  else                                                                                         \
    hipLaunchKernelGGL((k_phi_batch<TX, V, M, T1>), dim3(grid), dim3(TX), 0, s, b)
  if (vmode == VEL_SEP) {
    if (model2) { LBM_BATCH_LAUNCH(VEL_SEP, true); } else { LBM_BATCH_LAUNCH(VEL_SEP, false); }
  } else {
    if (model2) { LBM_BATCH_LAUNCH(VEL_FIELD, true); } else { LBM_BATCH_LAUNCH(VEL_FIELD, false); }
  }
#undef LBM_BATCH_LAUNCH
  return hipGetLastError();
}

template <int TX, bool WALLS, int ST>
hipError_t phi_step_v(int vmode, int model, bool t1, const StepArgs& a, int nb, hipStream_t s) {
  switch (vmode) {
    case VEL_SEP: return phi_step_m<TX, WALLS, VEL_SEP, ST>(model, t1, a, nb, s);
    case VEL_FIELD: return phi_step_m<TX, WALLS, VEL_FIELD, ST>(model, t1, a, nb, s);
    default: return phi_step_m<TX, WALLS, VEL_NSFIELD, ST>(model, t1, a, nb, s);
  }
}

template <int ST>
hipError_t phi_step_t(int tx, bool walls, int vmode, int model, bool t1, const StepArgs& a,
                      int nb, hipStream_t s) {
  switch (tx) {
    case 64:
      return walls ? phi_step_v<64, true, ST>(vmode, model, t1, a, nb, s)
                   : phi_step_v<64, false, ST>(vmode, model, t1, a, nb, s);
    case 128:
      return walls ? phi_step_v<128, true, ST>(vmode, model, t1, a, nb, s)
                   : phi_step_v<128, false, ST>(vmode, model, t1, a, nb, s);
    case 256:
      return walls ? phi_step_v<256, true, ST>(vmode, model, t1, a, nb, s)
                   : phi_step_v<256, false, ST>(vmode, model, t1, a, nb, s);
    case 512:
      return walls ? phi_step_v<512, true, ST>(vmode, model, t1, a, nb, s)
                   : phi_step_v<512, false, ST>(vmode, model, t1, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

template <int R, int ST>
hipError_t phi_pass_r(int vmode, bool model2, bool rec, const StepArgs& a, int nb, hipStream_t s) {
#define LBM_PASS(V, M, RC) hipLaunchKernelGGL((k_phi_pass<R, V, M, RC, ST>), dim3(nb), dim3(64 * R), 0, s, a)
  if (vmode == VEL_SEP) {
    if (model2) { if (rec) LBM_PASS(VEL_SEP, true, true); else LBM_PASS(VEL_SEP, true, false); }
    else { if (rec) LBM_PASS(VEL_SEP, false, true); else LBM_PASS(VEL_SEP, false, false); }
  } else {
    if (model2) { if (rec) LBM_PASS(VEL_FIELD, true, true); else LBM_PASS(VEL_FIELD, true, false); }
    else { if (rec) LBM_PASS(VEL_FIELD, false, true); else LBM_PASS(VEL_FIELD, false, false); }
  }
#undef LBM_PASS
  return hipGetLastError();
}

template <int ST>
hipError_t phi_pass_t(int rows, int vmode, int model, const StepArgs& a, int nb, hipStream_t s) {
  const bool rec = a.phi_rec != nullptr, m2 = model == 2;
  if (rec && ST != ST_F32) return hipErrorInvalidValue;  // 16-bit: phi recorded apart
  switch (rows) {
    case 4: return phi_pass_r<4, ST>(vmode, m2, rec, a, nb, s);
    case 8: return phi_pass_r<8, ST>(vmode, m2, rec, a, nb, s);
    case 16: return phi_pass_r<16, ST>(vmode, m2, rec, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

#ifdef LBM_STEP_16BIT_TU
// The 16-bit storage instances of the step, in their own translation unit
// (lbm_ch_step16.hip, built with other code-generation options).
hipError_t launch_phi_step16(int tx, bool walls, int vmode, int model, int storage, bool t1,
                             const StepArgs& a, int nblocks, hipStream_t s) {
  switch (storage) {
    case ST_F16: return phi_step_t<ST_F16>(tx, walls, vmode, model, t1, a, nblocks, s);
    case ST_BF16: return phi_step_t<ST_BF16>(tx, walls, vmode, model, t1, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_phi_pass16(int rows, int vmode, int model, int storage, const StepArgs& a,
                             int nblocks, hipStream_t s) {
  switch (storage) {
    case ST_F16: return phi_pass_t<ST_F16>(rows, vmode, model, a, nblocks, s);
    case ST_BF16: return phi_pass_t<ST_BF16>(rows, vmode, model, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}
#else
bool phi_record_fused(bool walls, int vmode, int model, int storage) {
  return !walls && storage == ST_F32 && (vmode == VEL_SEP || vmode == VEL_FIELD) &&
         (model == 1 || model == 2);
}

template <int TX, bool T1>
static hipError_t phi_record_t(int vmode, int model, const StepArgs& a, int nb, hipStream_t s) {
#define LBM_REC_LAUNCH(V, M) \
  hipLaunchKernelGGL((k_phi_step<TX, false, V, M, ST_F32, true, T1>), dim3(nb), dim3(TX), 0, s, a)
  if (vmode == VEL_SEP) {
    if (model == 2) { LBM_REC_LAUNCH(VEL_SEP, 2); } else { LBM_REC_LAUNCH(VEL_SEP, 1); }
  } else {
    if (model == 2) { LBM_REC_LAUNCH(VEL_FIELD, 2); } else { LBM_REC_LAUNCH(VEL_FIELD, 1); }
  }
#undef LBM_REC_LAUNCH
  return hipGetLastError();
}

hipError_t launch_phi_record(int tx, int vmode, int model, bool t1, const StepArgs& a,
                             int nblocks, hipStream_t s) {
  if (!phi_record_fused(false, vmode, model, ST_F32) || !a.phi_rec) return hipErrorInvalidValue;
  switch (tx) {
    case 64: return t1 ? phi_record_t<64, true>(vmode, model, a, nblocks, s)
                       : phi_record_t<64, false>(vmode, model, a, nblocks, s);
    case 128: return t1 ? phi_record_t<128, true>(vmode, model, a, nblocks, s)
                        : phi_record_t<128, false>(vmode, model, a, nblocks, s);
    case 256: return t1 ? phi_record_t<256, true>(vmode, model, a, nblocks, s)
                        : phi_record_t<256, false>(vmode, model, a, nblocks, s);
    case 512: return t1 ? phi_record_t<512, true>(vmode, model, a, nblocks, s)
                        : phi_record_t<512, false>(vmode, model, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

bool phi_pass_ok(bool walls, int vmode, int model, int storage, bool t1) {
  return !walls && t1 && (vmode == VEL_SEP || vmode == VEL_FIELD) && (model == 1 || model == 2) &&
         (storage == ST_F32 || storage == ST_F16 || storage == ST_BF16);
}

hipError_t launch_phi_pass(int rows, int vmode, int model, int storage, const StepArgs& a,
                           int nblocks, hipStream_t s) {
  if (!phi_pass_ok(false, vmode, model, storage, true)) return hipErrorInvalidValue;
  if (storage != ST_F32) return launch_phi_pass16(rows, vmode, model, storage, a, nblocks, s);
  return phi_pass_t<ST_F32>(rows, vmode, model, a, nblocks, s);
}

hipError_t launch_phi_step(int tx, bool walls, int vmode, int model, int storage, bool t1,
                           const StepArgs& a, int nblocks, hipStream_t s) {
  switch (storage) {
    case ST_F32: return phi_step_t<ST_F32>(tx, walls, vmode, model, t1, a, nblocks, s);
    case ST_F16:
    case ST_BF16: return launch_phi_step16(tx, walls, vmode, model, storage, t1, a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

int phi_batch_blocks_per_cu(int tx, int vmode, bool model2, bool t1) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  const bool sep = vmode == VEL_SEP;
#define LBM_OCC1(T, T1)                                                                                                          \
  e = sep ? (model2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch_persistent<T, VEL_SEP, true, T1>, T, 0)    \
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch_persistent<T, VEL_SEP, false, T1>, T, 0))   \
          : (model2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch_persistent<T, VEL_FIELD, true, T1>, T, 0)  \
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phi_batch_persistent<T, VEL_FIELD, false, T1>, T, 0))
#define LBM_OCC(T) if (t1) { LBM_OCC1(T, true); } else { LBM_OCC1(T, false); }
  switch (tx) {
    case 64: LBM_OCC(64); break;
    case 128: LBM_OCC(128); break;
    case 256: LBM_OCC(256); break;
    default: break;
  }
#undef LBM_OCC
#undef LBM_OCC1
  return e == hipSuccess && nb > 0 ? nb : 1;
}

template <bool PERSIST, bool T1>
static hipError_t phi_batch_tx(int tx, int vmode, bool model2, const BatchArgs& b, int grid,
                               hipStream_t s) {
  switch (tx) {
    case 64: return phi_batch_t<64, PERSIST, T1>(vmode, model2, b, grid, s);
    case 128: return phi_batch_t<128, PERSIST, T1>(vmode, model2, b, grid, s);
    case 256: return phi_batch_t<256, PERSIST, T1>(vmode, model2, b, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_phi_batch(int tx, int vmode, bool model2, bool t1, bool persistent,
                            const BatchArgs& b, int grid, hipStream_t s) {
  if (grid <= 0 || (grid & 7) != 0 || b.n <= 0) return hipErrorInvalidValue;
  if (persistent)
    return t1 ? phi_batch_tx<true, true>(tx, vmode, model2, b, grid, s)
              : phi_batch_tx<true, false>(tx, vmode, model2, b, grid, s);
  return t1 ? phi_batch_tx<false, true>(tx, vmode, model2, b, grid, s)
            : phi_batch_tx<false, false>(tx, vmode, model2, b, grid, s);
}
#endif  // LBM_STEP_16BIT_TU

}  // namespace lbmch
