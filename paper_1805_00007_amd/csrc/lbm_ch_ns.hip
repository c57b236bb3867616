// gfx950 kernel of the coupled Navier-Stokes step of the lattice Boltzmann
// Cahn-Hilliard solver (Zhang, Guo & Liang, arXiv:1805.00007) for Rayleigh-Taylor
// flows: a pressure-based incompressible D2Q9 BGK model driven by the phase field's
// forces (the model and its moments are stated in include/lbm_ch.h).  The phase-field
// step then runs with the velocity and pressure this kernel writes.
#include "lbm_ch_device.h"

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

}  // namespace lbmch
