/* Drives every function of the FP64 oracle on small, odd-sized lattices in every mode
 * (walls, coupled NS, models 1-3, both F1 readings, float32 rounding, a time-factor
 * table) so that an AddressSanitizer / UndefinedBehaviorSanitizer build can check its
 * memory accesses and arithmetic.  Prints one checksum line; exits non-zero on a
 * failed consistency check (a sanitizer aborts by itself). */
#define _USE_MATH_DEFINES
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdio.h>
#include <stdlib.h>

#include "lbm_ch_oracle.h"

static double* zeros(size_t n) {
  double* a = calloc(n, sizeof(double));
  if (!a) exit(3);
  return a;
}

static int run_case(int nx, int ny, int walls, int model, int ns, int f1_form, int round_f32,
                    int with_u, int with_tf, double* checksum) {
  orc_params p = {0};
  p.nx = nx; p.ny = ny; p.walls = walls; p.model = model; p.ns = ns;
  p.tau_g = 0.8; p.mobility = 0.02; p.sigma = 0.01; p.width = 3.0;
  p.phi_a = 1.0; p.phi_b = -1.0; p.rho_a = 1.0; p.rho_b = 0.4;
  p.tau_f = 0.7; p.gravity = ns ? 1e-5 : 0.0; p.accel_x = ns ? 1e-6 : 0.0;
  p.f1_form = f1_form; p.round_f32 = round_f32;
  orc_coeffs c;
  if (orc_coeffs_from(&p, &c) != 0) return 1;
  size_t n = (size_t)nx * ny;
  double *phi0 = zeros(n), *ux = zeros(n), *uy = zeros(n), *g = zeros(9 * n);
  double *f = ns ? zeros(9 * n) : NULL, *hist = zeros(4 * n), tf[7];
  double *phi = zeros(n), *mu = zeros(n), *u = zeros(n), *v = zeros(n), *pr = zeros(n);
  double *gx = zeros(n), *gy = zeros(n), *lp = zeros(n), out[8];
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = (size_t)y * nx + x;
      phi0[k] = tanh((hypot(x - 0.4 * nx, y - 0.5 * ny) - 0.3 * ny) / 1.5);
      ux[k] = 0.03 * sin(2 * M_PI * y / ny);
      uy[k] = -0.02 * sin(2 * M_PI * x / nx);
    }
  for (int s = 0; s < 7; ++s) tf[s] = cos(M_PI * s / 12.0);
  const double* uu = with_u ? ux : NULL;
  const double* vv = with_u ? uy : NULL;
  int hist_valid = 0;
  orc_init(&p, phi0, uu, vv, g, f);
  /* a table shorter than the run: orc_run reads tf[s] only for s < nsteps */
  orc_run(&p, g, f, ns ? NULL : uu, ns ? NULL : vv, with_tf ? tf : NULL, 5, hist, &hist_valid);
  orc_fields(&p, g, f, uu, vv, with_tf ? tf[5] : 1.0, phi, mu, u, v, pr);
  orc_fields(&p, g, f, NULL, NULL, 1.0, phi, NULL, NULL, NULL, NULL);
  orc_grad(&p, phi, 1, gx, gy);
  orc_grad(&p, u, -1, gx, gy);
  orc_lap(&p, phi, 1, lp);
  orc_chemical_potential(&p, phi, mu);
  orc_diag(&p, phi, phi0, out);
  orc_diag(&p, phi, NULL, out);
  int bad = out[7] != 0.0;
  for (size_t k = 0; k < n; ++k) *checksum += phi[k] + 1e-3 * (mu[k] + gx[k] + lp[k]);
  free(phi0); free(ux); free(uy); free(g); free(f); free(hist);
  free(phi); free(mu); free(u); free(v); free(pr); free(gx); free(gy); free(lp);
  return bad;
}

int main(void) {
  double geq[9], s[9], feq[9], sf[9], sum = 0.0;
  orc_equilibrium_g(0.3, -0.01, 0.02, -0.03, 1.5, geq);
  orc_source_g(1e-4, -2e-4, s);
  orc_equilibrium_f(1e-3, 0.8, 0.02, 0.01, feq);
  orc_source_f(1e-4, 2e-4, 0.02, 0.01, 1e-3, -1e-3, sf);
  for (int i = 0; i < 9; ++i) sum += geq[i] - 0.3 / 9.0 + s[i] + feq[i] + sf[i];
  orc_params bad = {0};
  bad.nx = 8; bad.ny = 8; bad.tau_g = 0.5; bad.phi_a = 1.0; bad.phi_b = -1.0;
  orc_coeffs c;
  if (orc_coeffs_from(&bad, &c) != -1) return 2;
  orc_set_num_threads(orc_num_threads());
  int fails = 0;
  const int sizes[][2] = {{7, 5}, {9, 11}, {4, 4}};
  for (int z = 0; z < 3; ++z)
    for (int walls = 0; walls < 2; ++walls)
      for (int model = 1; model <= 3; ++model)
        for (int ns = 0; ns < 2; ++ns)
          for (int form = 0; form < 2; ++form) {
            if (ns && form) continue; /* the F1 reading is for prescribed velocities */
            fails += run_case(sizes[z][0], sizes[z][1], walls, model, ns, form,
                              (model + walls) % 2, 1, !ns, &sum);
            fails += run_case(sizes[z][0], sizes[z][1], walls, model, ns, form, 0, 0, 0, &sum);
          }
  printf("oracle driver: %d failed checks, checksum %.12e\n", fails, sum);
  return fails ? 1 : 0;
}
