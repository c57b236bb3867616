/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see lbm_ch_oracle.h).
 *
 * Zhang, Guo & Liang, "A high-order lattice Boltzmann model for the Cahn-Hilliard
 * equation", arXiv:1805.00007.  Plain full-grid loops, double precision, in the
 * order of Sec. II.  OpenMP splits the row loops only; every value is computed by
 * the same expression whatever the thread count, so results do not depend on it.
 */
#include "lbm_ch_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 lattice of Sec. II.B: c_0 = 0, c_1 = -c_3 = (1,0), c_2 = -c_4 = (0,1),
 * c_5 = -c_7 = (1,1), c_6 = -c_8 = (-1,1); weights below Eq. geq. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const orc_real W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const orc_real CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 with c = 1 */

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- parameters */

int orc_coeffs_from(const orc_params* p, orc_coeffs* c) {
  orc_real dphi = p->phi_a - p->phi_b;
  if (!(p->tau_g > 0.5) || dphi == 0.0) return -1;
  orc_real ad = fabs(dphi);
  /* Eq. betakappa */
  c->beta = 12.0 * p->sigma / (p->width * ad * ad * ad * ad);
  c->kappa = 3.0 * p->sigma * p->width / (2.0 * ad * ad);
  /* M = cs^2 eta (tau_g - 1/2), stated below Eq. phit3 */
  c->eta = p->mobility / (CS2 * (p->tau_g - 0.5));
  /* K below Eq. F2-1 */
  c->K = (p->tau_g - 1.0 / 6.0 - p->tau_g * p->tau_g) / (p->tau_g - 0.5);
  /* Eq. rho */
  c->a = (p->rho_a - p->rho_b) / dphi;
  c->b = (p->rho_b * p->phi_a - p->phi_b * p->rho_a) / dphi;
  return 0;
}

/* ---------------------------------------------------------- node primitives */

/* s_i(u) = c_i.u/cs^2 + (c_i.u)^2/(2 cs^4) - u^2/(2 cs^2), the bracket of Eq. geq. */
static orc_real s_poly(int i, orc_real ux, orc_real uy) {
  orc_real cu = CX[i] * ux + CY[i] * uy;
  orc_real u2 = ux * ux + uy * uy;
  return cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - u2 / (2.0 * CS2);
}

/* Eq. geq. */
void orc_equilibrium_g(orc_real phi, orc_real mu, orc_real ux, orc_real uy, orc_real eta, orc_real geq[9]) {
  orc_real u2 = ux * ux + uy * uy;
  geq[0] = phi + (W[0] - 1.0) * eta * mu - W[0] * phi * u2 / (2.0 * CS2);
  for (int i = 1; i < 9; ++i) geq[i] = W[i] * eta * mu + W[i] * phi * s_poly(i, ux, uy);
}

/* Eq. liangFi: S_i = w_i c_i . F / cs^2. */
void orc_source_g(orc_real fx, orc_real fy, orc_real s[9]) {
  for (int i = 0; i < 9; ++i) s[i] = W[i] * (CX[i] * fx + CY[i] * fy) / CS2;
}

/* Navier-Stokes equilibrium (pressure-based incompressible form):
 * f_0 = (w_0 - 1) p/cs^2 + rho w_0 s_0(u),  f_i = w_i p/cs^2 + rho w_i s_i(u),
 * so that sum f = 0, sum c f = rho u, sum c c f = p I + rho u u. */
void orc_equilibrium_f(orc_real p, orc_real rho, orc_real ux, orc_real uy, orc_real feq[9]) {
  feq[0] = (W[0] - 1.0) * p / CS2 + rho * W[0] * s_poly(0, ux, uy);
  for (int i = 1; i < 9; ++i) feq[i] = W[i] * p / CS2 + rho * W[i] * s_poly(i, ux, uy);
}

/* Navier-Stokes forcing with moments sum G = u.grad rho, sum c G = F,
 * sum c c G = u F + F u + cs^2 (u.grad rho I + u grad rho + grad rho u):
 * G_i = w_i [ (c_i - u).F/cs^2 + (c_i.u)(c_i.F)/cs^4 + (c_i.u)(c_i.grad rho)/cs^2 ]. */
void orc_source_f(orc_real fx, orc_real fy, orc_real ux, orc_real uy, orc_real drx, orc_real dry,
                  orc_real s[9]) {
  for (int i = 0; i < 9; ++i) {
    orc_real cu = CX[i] * ux + CY[i] * uy;
    orc_real cf = CX[i] * fx + CY[i] * fy;
    orc_real cr = CX[i] * drx + CY[i] * dry;
    orc_real cmuf = (CX[i] - ux) * fx + (CY[i] - uy) * fy;
    s[i] = W[i] * (cmuf / CS2 + cu * cf / (CS2 * CS2) + cu * cr / CS2);
  }
}

/* ------------------------------------------------------------ grid helpers */

static size_t nn(const orc_params* p) { return (size_t)p->nx * (size_t)p->ny; }

/* Value of a grid field at any (x, y): x periodic; y periodic, or mirrored across
 * the walls at y = -1/2 and y = ny - 1/2 with the given parity (+1 for phi, mu, p;
 * -1 for the velocity, whose no-slip value on the wall is zero). */
static orc_real at(const orc_params* p, const orc_real* a, int parity, int x, int y) {
  int nx = p->nx, ny = p->ny;
  x = ((x % nx) + nx) % nx;
  if (!p->walls) {
    y = ((y % ny) + ny) % ny;
    return a[(size_t)y * nx + x];
  }
  if (y < 0) return parity * a[(size_t)(-1 - y) * nx + x];
  if (y >= ny) return parity * a[(size_t)(2 * ny - 1 - y) * nx + x];
  return a[(size_t)y * nx + x];
}

/* Isotropic central schemes (Sec. III), built from the lattice weights:
 *   d_a psi(x) = (1/cs^2) sum_i w_i c_ia psi(x + c_i)
 *   lap psi(x) = (2/cs^2) sum_i w_i [psi(x + c_i) - psi(x)]
 * The gradient is exact for quadratics and the Laplacian for cubics. */
static void grad_at(const orc_params* p, const orc_real* a, int parity, int x, int y,
                    orc_real* gx, orc_real* gy) {
  orc_real sx = 0.0, sy = 0.0;
  for (int i = 1; i < 9; ++i) {
    orc_real v = at(p, a, parity, x + CX[i], y + CY[i]);
    sx += W[i] * CX[i] * v;
    sy += W[i] * CY[i] * v;
  }
  *gx = sx / CS2;
  *gy = sy / CS2;
}

static orc_real lap_at(const orc_params* p, const orc_real* a, int parity, int x, int y) {
  orc_real c = at(p, a, parity, x, y);
  orc_real s = 0.0;
  for (int i = 1; i < 9; ++i) s += W[i] * (at(p, a, parity, x + CX[i], y + CY[i]) - c);
  return 2.0 * s / CS2;
}

void orc_grad(const orc_params* p, const orc_real* psi, int parity, orc_real* gx, orc_real* gy) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      grad_at(p, psi, parity, x, y, &gx[k], &gy[k]);
    }
}

void orc_lap(const orc_params* p, const orc_real* psi, int parity, orc_real* out) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) out[(size_t)y * p->nx + x] = lap_at(p, psi, parity, x, y);
}

/* df/dphi of Eq. bulk: 2 beta (phi - phi_A)(phi - phi_B)(2 phi - phi_A - phi_B). */
static orc_real dbulk(const orc_params* p, const orc_coeffs* c, orc_real phi) {
  return 2.0 * c->beta * (phi - p->phi_a) * (phi - p->phi_b) * (2.0 * phi - p->phi_a - p->phi_b);
}

/* Eq. mu. */
void orc_chemical_potential(const orc_params* p, const orc_real* phi, orc_real* mu) {
  orc_coeffs c;
  orc_coeffs_from(p, &c);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      mu[k] = dbulk(p, &c, phi[k]) - c.kappa * lap_at(p, phi, +1, x, y);
    }
}

/* Eq. macroscopicg. */
static void order_parameter(const orc_params* p, const orc_real* g, orc_real* phi) {
  size_t n = nn(p);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      orc_real s = 0.0;
      for (int i = 0; i < 9; ++i) s += g[i * n + k];
      phi[k] = s;
    }
}

/* Streaming g_i(x + c_i, t + 1) = g_i*(x, t) in pull form; with walls a
 * population whose source lies beyond a wall is the one that left the same node in
 * the opposite direction (half-way bounce-back). */
static void stream(const orc_params* p, const orc_real* post, orc_real* out) {
  size_t n = nn(p);
  int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      for (int i = 0; i < 9; ++i) {
        int sx = ((x - CX[i]) % nx + nx) % nx;
        int sy = y - CY[i];
        size_t k = (size_t)y * nx + x;
        if (p->walls && (sy < 0 || sy >= ny))
          out[i * n + k] = post[OPP[i] * n + k];
        else
          out[i * n + k] = post[i * n + (size_t)((sy % ny + ny) % ny) * nx + sx];
      }
}

/* ------------------------------------------------------------------- method */

typedef struct {
  orc_real *phi, *mu, *mux, *muy, *lapmu, *phx, *phy; /* order parameter and derived   */
  orc_real *gux, *guy, *gvx, *gvy;                    /* gradient of a prescribed u   */
  const orc_real *ux0, *uy0;                          /* base field of a prescribed u */
  orc_real dtf;                                       /* d/dt of its time factor      */
  orc_real *u, *v, *pr, *px, *py;                     /* velocity and pressure         */
  orc_real *qx, *qy, *dext;                           /* phi u and its divergence      */
  orc_real *fx, *fy, *ftx, *fty;                      /* CH force F; NS total force    */
  orc_real* post;                                     /* post-collision populations    */
} orc_work;

static orc_real* zalloc(size_t n) { return (orc_real*)calloc(n, sizeof(orc_real)); }

static void work_alloc(const orc_params* p, orc_work* w) {
  size_t n = nn(p);
  w->phi = zalloc(n); w->mu = zalloc(n); w->mux = zalloc(n); w->muy = zalloc(n);
  w->lapmu = zalloc(n); w->phx = zalloc(n); w->phy = zalloc(n);
  w->u = zalloc(n); w->v = zalloc(n); w->pr = zalloc(n); w->px = zalloc(n); w->py = zalloc(n);
  w->qx = zalloc(n); w->qy = zalloc(n); w->dext = zalloc((size_t)p->nx * (p->ny + 2));
  w->fx = zalloc(n); w->fy = zalloc(n); w->ftx = zalloc(n); w->fty = zalloc(n);
  w->gux = zalloc(n); w->guy = zalloc(n); w->gvx = zalloc(n); w->gvy = zalloc(n);
  w->ux0 = NULL; w->uy0 = NULL; w->dtf = 0.0;
  w->post = zalloc(9 * n);
}

static void work_free(orc_work* w) {
  orc_real* all[] = {w->phi, w->mu, w->mux, w->muy, w->lapmu, w->phx, w->phy, w->u, w->v,
                   w->pr, w->px, w->py, w->qx, w->qy, w->dext, w->fx, w->fy, w->ftx,
                   w->fty, w->gux, w->guy, w->gvx, w->gvy, w->post};
  for (size_t i = 0; i < sizeof(all) / sizeof(all[0]); ++i) free(all[i]);
}

/* Navier-Stokes macroscopic step (the Rayleigh-Taylor coupling, Sec. III.E):
 * total force F = F_s + F_b + u (drho/dphi) M lap(mu), where F_s = -phi grad mu is
 * the surface-tension force of Eq. NS and the last term turns the conservative
 * momentum balance that the LBE recovers into the non-conservative Eq. NS(b);
 * rho u = sum_i c_i f_i + F/2 (solved for u); and
 * p = cs^2/(1 - w_0) [sum_{i>0} f_i + u.grad rho / 2 + rho w_0 s_0(u)]. */
static void ns_velocity_pressure(const orc_params* p, const orc_coeffs* c, const orc_real* f,
                                 orc_work* w) {
  size_t n = nn(p);
  orc_real rho_mean = 0.5 * (p->rho_a + p->rho_b);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      orc_real phi = w->phi[k];
      orc_real rho = c->a * phi + c->b;
      orc_real fsx = -phi * w->mux[k], fsy = -phi * w->muy[k];
      orc_real fbx = rho * p->accel_x, fby = -(rho - rho_mean) * p->gravity;
      orc_real mx = 0.0, my = 0.0;
      for (int i = 0; i < 9; ++i) {
        mx += CX[i] * f[i * n + k];
        my += CY[i] * f[i * n + k];
      }
      orc_real corr = c->a * p->mobility * w->lapmu[k];
      orc_real ux = (mx + 0.5 * (fsx + fbx)) / (rho - 0.5 * corr);
      orc_real uy = (my + 0.5 * (fsy + fby)) / (rho - 0.5 * corr);
      w->u[k] = ux;
      w->v[k] = uy;
      w->ftx[k] = fsx + fbx + ux * corr;
      w->fty[k] = fsy + fby + uy * corr;
      orc_real drx = c->a * w->phx[k], dry = c->a * w->phy[k];
      orc_real s = 0.0;
      for (int i = 1; i < 9; ++i) s += f[i * n + k];
      w->pr[k] = CS2 / (1.0 - W[0]) *
                 (s + 0.5 * (ux * drx + uy * dry) + rho * W[0] * s_poly(0, ux, uy));
    }
}

/* Order parameter, chemical potential and their gradients for the current g. */
/* Sensitivity runs (round_f32): round a field to float32, as the GPU path holds it. */
static void to_f32(const orc_params* p, orc_real* a, size_t n) {
  if (!p->round_f32) return;
  for (size_t k = 0; k < n; ++k) a[k] = (orc_real)(float)a[k];
}

static void phase_fields(const orc_params* p, const orc_coeffs* c, const orc_real* g, orc_work* w) {
  (void)c;
  order_parameter(p, g, w->phi);
  to_f32(p, w->phi, nn(p));
  orc_chemical_potential(p, w->phi, w->mu);
  to_f32(p, w->mu, nn(p));
  orc_grad(p, w->mu, +1, w->mux, w->muy);
  if (p->ns) {
    orc_lap(p, w->mu, +1, w->lapmu);
    orc_grad(p, w->phi, +1, w->phx, w->phy);
  }
}

/* Velocity at step n: prescribed (factor times base field) or from the NS populations. */
static void velocity_fields(const orc_params* p, const orc_coeffs* c, const orc_real* f,
                            const orc_real* ux, const orc_real* uy, orc_real tfac, orc_work* w) {
  size_t n = nn(p);
  if (p->ns) {
    ns_velocity_pressure(p, c, f, w);
    to_f32(p, w->u, n);
    to_f32(p, w->v, n);
    to_f32(p, w->pr, n);
    orc_grad(p, w->pr, +1, w->px, w->py);
    return;
  }
  for (size_t k = 0; k < n; ++k) {
    w->u[k] = ux ? tfac * ux[k] : 0.0;
    w->v[k] = uy ? tfac * uy[k] : 0.0;
    w->pr[k] = 0.0;
    w->px[k] = 0.0;
    w->py[k] = 0.0;
  }
}

/* F = F1 (+ F2): Eq. t0-phiu and Eq. mark3 (model 2) or Eq. F2-1 (model 3).  For
 * model 3, hist holds F1 and grad mu of the previous step (planes F1x, F1y, mux, muy)
 * and *hist_valid says whether there was one. */
static void ch_force(const orc_params* p, const orc_coeffs* c, orc_work* w, orc_real* hist,
                     int* hist_valid) {
  size_t n = nn(p);
  int nx = p->nx, ny = p->ny;
  orc_real rho_mean = 0.5 * (p->rho_a + p->rho_b);
  /* F1 = (phi/rho) (F_s + F_b - grad p), F_s = -phi grad mu.  With a prescribed
   * velocity there is no pressure field or body force: grad p = 0, F_b = 0. */
  if (p->f1_form == 1 && !p->ns) {
    /* F1 of Eq. cFi1 from the prescribed field: d_t(phi u) + div(phi u u)
     * = u (d_t phi + div(phi u)) + phi (d_t u + u.grad u) = phi (d_t u + u.grad u) on the
     * t1 scale, where d_t phi + div(phi u) = 0. */
    orc_grad(p, w->u, -1, w->gux, w->guy);
    orc_grad(p, w->v, -1, w->gvx, w->gvy);
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
      orc_real dtu = w->ux0 ? w->dtf * w->ux0[k] : 0.0, dtv = w->uy0 ? w->dtf * w->uy0[k] : 0.0;
      orc_real ax = dtu + w->u[k] * w->gux[k] + w->v[k] * w->guy[k];
      orc_real ay = dtv + w->u[k] * w->gvx[k] + w->v[k] * w->gvy[k];
      w->fx[k] = w->phi[k] * ax;
      w->fy[k] = w->phi[k] * ay;
    }
  } else {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = (size_t)y * nx + x;
      orc_real phi = w->phi[k];
      orc_real rho = c->a * phi + c->b;
      orc_real tx = -phi * w->mux[k] - w->px[k];
      orc_real ty = -phi * w->muy[k] - w->py[k];
      if (p->ns) {
        tx += rho * p->accel_x;
        ty += -(rho - rho_mean) * p->gravity;
      }
      w->fx[k] = phi / rho * tx;
      w->fy[k] = phi / rho * ty;
    }
  }
  if (p->model == 1) return;
  /* Eq. F2-1, model 3: the time derivatives of F1 and grad mu (taken on the whole time
   * scale, as Remarks I and II allow) as differences over the last step; zero on the
   * first step, which has no earlier state. */
  if (p->model == 3) {
    orc_real cA = 2.0 * p->tau_g - 1.0 + 3.0 * c->K;
    orc_real cB = 3.0 * CS2 * c->eta * c->K;
    int valid = hist_valid ? *hist_valid : 0;
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
      orc_real f1x = w->fx[k], f1y = w->fy[k];
      orc_real dF1x = valid ? f1x - hist[k] : 0.0;
      orc_real dF1y = valid ? f1y - hist[n + k] : 0.0;
      orc_real dmux = valid ? w->mux[k] - hist[2 * n + k] : 0.0;
      orc_real dmuy = valid ? w->muy[k] - hist[3 * n + k] : 0.0;
      hist[k] = f1x;
      hist[n + k] = f1y;
      hist[2 * n + k] = w->mux[k];
      hist[3 * n + k] = w->muy[k];
      w->fx[k] = f1x + cA * dF1x + cB * dmux;
      w->fy[k] = f1y + cA * dF1y + cB * dmuy;
    }
    if (hist_valid) *hist_valid = 1;
  }
  /* F2 (models 2 and 3) contains 3 cs^2 K grad(div(phi u)): two composed isotropic
   * gradients.  q = phi u takes the velocity's ghost parity (-1) across walls; div q
   * is evaluated on the rows -1..ny (stored with a one-row offset) so that its
   * gradient reaches every fluid row. */
  for (size_t k = 0; k < n; ++k) {
    w->qx[k] = w->phi[k] * w->u[k];
    w->qy[k] = w->phi[k] * w->v[k];
  }
  to_f32(p, w->qx, n);
  to_f32(p, w->qy, n);
  int ylo = p->walls ? -1 : 0, yhi = p->walls ? ny : ny - 1;
#pragma omp parallel for schedule(static)
  for (int y = ylo; y <= yhi; ++y)
    for (int x = 0; x < nx; ++x) {
      orc_real ax, ay, bx, by;
      grad_at(p, w->qx, -1, x, y, &ax, &ay);
      grad_at(p, w->qy, -1, x, y, &bx, &by);
      w->dext[(size_t)(y + 1) * nx + x] = ax + by;
    }
  to_f32(p, w->dext, (size_t)nx * (ny + 2));
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      orc_real sx = 0.0, sy = 0.0;
      for (int i = 1; i < 9; ++i) {
        int xx = ((x + CX[i]) % nx + nx) % nx;
        int yy = y + CY[i];
        if (!p->walls) yy = (yy % ny + ny) % ny;
        orc_real d = w->dext[(size_t)(yy + 1) * nx + xx];
        sx += W[i] * CX[i] * d;
        sy += W[i] * CY[i] * d;
      }
      size_t k = (size_t)y * nx + x;
      w->fx[k] += 3.0 * CS2 * c->K * (sx / CS2);
      w->fy[k] += 3.0 * CS2 * c->K * (sy / CS2);
    }
}

/* Eq. LB collision for g (and the NS collision for f), then streaming. */
static void collide_stream(const orc_params* p, const orc_coeffs* c, orc_real* g, orc_real* f,
                           orc_work* w) {
  size_t n = nn(p);
  orc_real tg = p->tau_g;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      orc_real geq[9], s[9];
      orc_equilibrium_g(w->phi[k], w->mu[k], w->u[k], w->v[k], c->eta, geq);
      orc_source_g(w->fx[k], w->fy[k], s);
      for (int i = 0; i < 9; ++i)
        w->post[i * n + k] = g[i * n + k] - (g[i * n + k] - geq[i]) / tg + (1.0 - 0.5 / tg) * s[i];
    }
  stream(p, w->post, g);
  if (!p->ns) return;
  orc_real tf = p->tau_f;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      orc_real feq[9], s[9];
      orc_real rho = c->a * w->phi[k] + c->b;
      orc_equilibrium_f(w->pr[k], rho, w->u[k], w->v[k], feq);
      orc_source_f(w->ftx[k], w->fty[k], w->u[k], w->v[k], c->a * w->phx[k], c->a * w->phy[k], s);
      for (int i = 0; i < 9; ++i)
        w->post[i * n + k] = f[i * n + k] - (f[i * n + k] - feq[i]) / tf + (1.0 - 0.5 / tf) * s[i];
    }
  stream(p, w->post, f);
}

void orc_init(const orc_params* p, const orc_real* phi0, const orc_real* ux0, const orc_real* uy0,
              orc_real* g, orc_real* f) {
  orc_coeffs c;
  orc_coeffs_from(p, &c);
  size_t n = nn(p);
  orc_real* mu = zalloc(n);
  orc_chemical_potential(p, phi0, mu);
  for (size_t k = 0; k < n; ++k) {
    orc_real geq[9];
    orc_equilibrium_g(phi0[k], mu[k], ux0 ? ux0[k] : 0.0, uy0 ? uy0[k] : 0.0, c.eta, geq);
    for (int i = 0; i < 9; ++i) g[i * n + k] = geq[i];
    if (p->ns && f) {
      orc_real feq[9];
      orc_equilibrium_f(0.0, c.a * phi0[k] + c.b, ux0 ? ux0[k] : 0.0, uy0 ? uy0[k] : 0.0, feq);
      for (int i = 0; i < 9; ++i) f[i * n + k] = feq[i];
    }
  }
  free(mu);
}

void orc_run(const orc_params* p, orc_real* g, orc_real* f, const orc_real* ux, const orc_real* uy,
             const orc_real* tf, long nsteps, orc_real* hist, int* hist_valid) {
  orc_coeffs c;
  if (orc_coeffs_from(p, &c) != 0) return;
  if (p->model == 3 && (!hist || !hist_valid)) return;
  orc_work w;
  work_alloc(p, &w);
  w.ux0 = ux;
  w.uy0 = uy;
  for (long s = 0; s < nsteps; ++s) {
    phase_fields(p, &c, g, &w);
    velocity_fields(p, &c, f, ux, uy, tf ? tf[s] : 1.0, &w);
    /* d/dt of the time factor at step s: backward difference, forward on the first step
     * of the call (the table given covers this call's steps) */
    w.dtf = 0.0;
    if (tf && s > 0) w.dtf = tf[s] - tf[s - 1];
    else if (tf && nsteps > 1) w.dtf = tf[1] - tf[0];
    ch_force(p, &c, &w, hist, hist_valid);
    collide_stream(p, &c, g, f, &w);
    to_f32(p, g, 9 * nn(p));
    if (p->ns && f) to_f32(p, f, 9 * nn(p));
  }
  work_free(&w);
}

void orc_fields(const orc_params* p, const orc_real* g, const orc_real* f, const orc_real* ux,
                const orc_real* uy, orc_real tfac, orc_real* phi, orc_real* mu, orc_real* u, orc_real* v,
                orc_real* pr) {
  orc_coeffs c;
  orc_coeffs_from(p, &c);
  orc_work w;
  work_alloc(p, &w);
  size_t n = nn(p);
  phase_fields(p, &c, g, &w);
  velocity_fields(p, &c, f, ux, uy, tfac, &w);
  if (phi) memcpy(phi, w.phi, n * sizeof(orc_real));
  if (mu) memcpy(mu, w.mu, n * sizeof(orc_real));
  if (u) memcpy(u, w.u, n * sizeof(orc_real));
  if (v) memcpy(v, w.v, n * sizeof(orc_real));
  if (pr) memcpy(pr, w.pr, n * sizeof(orc_real));
  work_free(&w);
}

void orc_diag(const orc_params* p, const orc_real* phi, const orc_real* phi_ref, orc_real out[8]) {
  orc_coeffs c;
  orc_coeffs_from(p, &c);
  orc_real s = 0, sa = 0, e = 0, d2 = 0, r2 = 0, mx = -INFINITY, mn = INFINITY, bad = 0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      orc_real v = phi[k];
      if (!isfinite(v)) { bad += 1; continue; }
      s += v;
      sa += fabs(v);
      /* Eq. freeEnergy with the bulk density of Eq. bulk */
      orc_real gx, gy;
      grad_at(p, phi, +1, x, y, &gx, &gy);
      orc_real fa = v - p->phi_a, fb = v - p->phi_b;
      e += c.beta * fa * fa * fb * fb + 0.5 * c.kappa * (gx * gx + gy * gy);
      if (phi_ref) {
        d2 += (v - phi_ref[k]) * (v - phi_ref[k]);
        r2 += phi_ref[k] * phi_ref[k];
      }
      if (v > mx) mx = v;
      if (v < mn) mn = v;
    }
  out[0] = s; out[1] = sa; out[2] = e; out[3] = d2; out[4] = r2; out[5] = mx; out[6] = mn;
  out[7] = bad;
}
