/*
 * FP64 CPU oracle for the single-relaxation-time D2Q9 lattice Boltzmann model of
 * the Cahn-Hilliard equation (Zhang, Guo & Liang, arXiv:1805.00007).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the GPU path with a
 * plain, slow, obviously correct implementation.  The product path never links,
 * loads or calls it, and it shares no code, header, table or constant with the
 * GPU library.
 *
 * Everything is double precision, plain loops over full-grid arrays, in the order
 * the paper states the method (Sec. II):
 *   phi = sum_i g_i                               (Eq. macroscopicg)
 *   mu  = f'(phi) - kappa lap(phi)                (Eqs. bulk, mu, betakappa)
 *   F1  = (phi/rho) (F_s [+ body force] - grad p) (Eq. t0-phiu, F_s = -phi grad mu)
 *   F2  = 3 cs^2 K grad(div(phi u))               (Eq. mark3, Model-II only)
 *   g_i^eq, S_i = w_i c_i.F / cs^2                (Eqs. geq, liangFi)
 *   g_i* = g_i - (g_i - g_i^eq)/tau + (1 - 1/(2 tau)) S_i   (Eq. LB)
 *   stream g_i(x + c_i) <- g_i*(x)
 * The gradient and Laplacian are the isotropic central schemes named in Sec. III
 * (written out in the .c file).  The coupled Navier-Stokes populations f (used
 * for the Rayleigh-Taylor case, Sec. III.E) follow a pressure-based incompressible
 * D2Q9 BGK model; the paper calls that LBE standard and does not print it, so the
 * model used is the one written out in the .c file.
 *
 * Memory layout of every field: row-major, index y*nx + x, x periodic.  A
 * population array holds 9 such planes, plane i at offset i*nx*ny.
 * Velocity ordering c_0..c_8 = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 * (-1,-1) (1,-1), as listed with the D2Q9 lattice in Sec. II.B.
 *
 * Parity pins: every function here is checked by the CPU test-suite against
 * closed forms, identities and special cases fixed by the paper (see the tests);
 * none is "parity unpinned".
 */
#ifndef LBM_CH_ORACLE_H
#define LBM_CH_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* The arithmetic type: double.  Built with -DORC_REAL=float (and single-precision
 * constants) the same code runs in float32 arithmetic; that build is used only to
 * measure how far evaluating the method in float32 drifts from FP64 over a long
 * unstable run (the sensitivity that sets long-run tolerances), never as a reference. */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL orc_real;

typedef struct {
  int nx, ny;
  int walls;     /* 0: periodic in y; 1: no-slip walls below row 0 and above row ny-1 */
  int model;     /* 1: F = F1 (Model-I); 2: F = F1 + F2 of Eq. mark3 (Model-II);
                    3: F = F1 + F2 of Eq. F2-1 with the time derivatives as one-step
                    backward differences (Model-II at any tau_g)                       */
  int ns;        /* 0: prescribed velocity, grad p = 0; 1: coupled Navier-Stokes        */
  orc_real tau_g, mobility, sigma, width, phi_a, phi_b, rho_a, rho_b;
  orc_real tau_f;    /* NS relaxation time, nu = cs^2 (tau_f - 1/2)                      */
  orc_real gravity;  /* NS: acceleration g along -y, applied as -(rho - rho_mean) g        */
  orc_real accel_x;  /* NS: uniform acceleration along +x, applied as rho * accel_x        */
  int f1_form;     /* reading of F1 with a prescribed velocity (ns = 0):
                      0: Eq. t0-phiu with grad p = 0, F1 = (phi/rho) F_s = -(phi^2/rho) grad mu;
                      1: Eq. cFi1 evaluated from the prescribed field, F1 = d_t(phi u) +
                         div(phi u u) = phi (d_t u + u.grad u), using the t1-scale balance
                         d_t phi + div(phi u) = 0 (Eq. moments0order a); d_t u from a
                         one-step difference of the time factor                          */
  int round_f32;   /* 0 normally.  1: every value the GPU path holds in float32 between
                      its stages is rounded to float32 where it is formed: phi, mu, the
                      NS velocity and pressure, q = phi u and div q within a step, and the
                      populations after it.  Used to measure how much the dynamics
                      amplify perturbations of that size when deriving a long-run
                      tolerance; the method itself is unchanged                          */
} orc_params;

typedef struct {
  orc_real beta, kappa;  /* Eq. betakappa                    */
  orc_real eta;          /* M = cs^2 eta (tau_g - 1/2)        */
  orc_real K;            /* (tau - 1/6 - tau^2)/(tau - 1/2)   */
  orc_real a, b;         /* rho = a phi + b, Eq. rho          */
} orc_coeffs;

/* Derived coefficients.  Returns 0, or -1 if tau_g <= 1/2 or phi_a == phi_b. */
int orc_coeffs_from(const orc_params* p, orc_coeffs* c);

/* Single-node building blocks (exposed so that the tests can pin them). */
void orc_equilibrium_g(orc_real phi, orc_real mu, orc_real ux, orc_real uy, orc_real eta, orc_real geq[9]);
void orc_source_g(orc_real fx, orc_real fy, orc_real s[9]);
void orc_equilibrium_f(orc_real p, orc_real rho, orc_real ux, orc_real uy, orc_real feq[9]);
void orc_source_f(orc_real fx, orc_real fy, orc_real ux, orc_real uy, orc_real drx, orc_real dry,
                  orc_real s[9]);

/* Grid operators with the ghost rule of the boundary (periodic, or mirror with the
 * given parity +1/-1 across the walls).  Outputs are full nx*ny grids. */
void orc_grad(const orc_params* p, const orc_real* psi, int parity, orc_real* gx, orc_real* gy);
void orc_lap(const orc_params* p, const orc_real* psi, int parity, orc_real* out);

/* Chemical potential of a phi field, Eq. mu with the bulk energy of Eq. bulk. */
void orc_chemical_potential(const orc_params* p, const orc_real* phi, orc_real* mu);

/* Initial populations: g_i = g_i^eq(phi0, mu[phi0], u0), no source; f_i = f_i^eq
 * (p = 0, rho(phi0), u0) when ns = 1.  u0 may be NULL (zero). */
void orc_init(const orc_params* p, const orc_real* phi0, const orc_real* ux0, const orc_real* uy0,
              orc_real* g, orc_real* f);

/* Advance nsteps.  g (and f when ns = 1) hold the state on entry and exit.
 * Prescribed velocity at step n (from t_n to t_{n+1}) is tf[n]*ux, tf[n]*uy;
 * tf may be NULL (factor 1); ux/uy may be NULL (zero velocity).  Model 3 also needs
 * hist (4*nx*ny doubles: F1 and grad mu of the previous step, updated) and
 * *hist_valid (0 before the first step, set to 1); both may be NULL otherwise. */
void orc_run(const orc_params* p, orc_real* g, orc_real* f, const orc_real* ux, const orc_real* uy,
             const orc_real* tf, long nsteps, orc_real* hist, int* hist_valid);

/* Macroscopic fields of a state.  For ns = 0 the velocity written is tfac*ux, tfac*uy
 * and p = 0.  Any output pointer may be NULL. */
void orc_fields(const orc_params* p, const orc_real* g, const orc_real* f, const orc_real* ux,
                const orc_real* uy, orc_real tfac, orc_real* phi, orc_real* mu, orc_real* u,
                orc_real* v, orc_real* pr);

/* FP64 diagnostics of a phi field (phi_ref may be NULL):
 * out[0] sum phi, out[1] sum |phi|, out[2] free energy (Eq. freeEnergy),
 * out[3] sum (phi-phi_ref)^2, out[4] sum phi_ref^2, out[5] max phi, out[6] min phi,
 * out[7] number of non-finite values. */
void orc_diag(const orc_params* p, const orc_real* phi, const orc_real* phi_ref, orc_real out[8]);

/* Threads the OpenMP loops use (1 when built without OpenMP). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
