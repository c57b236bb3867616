/* Drives the host side of the C ABI with no GPU present: parameter validation, size
 * queries, NULL-context calls, status strings, and lbm_ch_init / lbm_ch_batch_create
 * up to the point where HIP reports that there is no device.  Built with
 * AddressSanitizer / UndefinedBehaviorSanitizer on the host code (device code is not
 * compiled); exits non-zero on an unexpected status. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lbm_ch.h"

static int fails = 0;
#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

static lbm_ch_params params(int nx, int ny) {
  lbm_ch_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx; p.ny = ny; p.model = 2; p.tau_g = 0.8; p.mobility = 0.01;
  p.sigma = 0.01; p.width = 4.0; p.phi_a = 1.0; p.phi_b = -1.0;
  p.rho_a = 1.0; p.rho_b = 1.0; p.tau_f = 0.8;
  return p;
}

int main(void) {
  /* sizes and workspace queries over every mode */
  for (int storage = 0; storage < 4; ++storage)
    for (int vm = 0; vm < 5; ++vm)
      for (int model = 0; model < 5; ++model)
        for (int walls = 0; walls < 3; ++walls) {
          lbm_ch_params p = params(67, 45);
          p.storage = storage; p.velocity_mode = vm; p.model = model; p.walls = walls;
          size_t b = lbm_ch_workspace_bytes(&p);
          int ok = storage < 3 && vm < 4 && model >= 1 && model <= 3 && walls < 2;
          EXPECT((b > 0) == ok);
          (void)lbm_ch_adjoint_scratch_bytes(&p);
        }
  lbm_ch_params p = params(7680, 7760);
  EXPECT(lbm_ch_workspace_bytes(&p) > 0);
  p.ny = 7776;
  EXPECT(lbm_ch_workspace_bytes(&p) == 0);
  p = params(3, 64);
  EXPECT(lbm_ch_workspace_bytes(&p) == 0);
  p = params(40000, 40000);
  EXPECT(lbm_ch_workspace_bytes(&p) == 0);
  EXPECT(lbm_ch_workspace_bytes(NULL) == 0);
  EXPECT(lbm_ch_adjoint_scratch_bytes(NULL) == 0);

  /* lbm_ch_init: every validation path, then a valid call that reaches HIP */
  p = params(64, 48);
  size_t need = lbm_ch_workspace_bytes(&p);
  lbm_ch_ctx* ctx = NULL;
  void* ws = (void*)(uintptr_t)4096;
  const float* phi0 = (const float*)(uintptr_t)8192;
  EXPECT(lbm_ch_init(NULL, &p, NULL, ws, need, phi0, NULL) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_init(&ctx, NULL, NULL, ws, need, phi0, NULL) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_init(&ctx, &p, NULL, NULL, need, phi0, NULL) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_init(&ctx, &p, NULL, (char*)ws + 64, need, phi0, NULL) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_init(&ctx, &p, NULL, ws, need - 1, phi0, NULL) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_init(&ctx, &p, NULL, ws, need, NULL, NULL) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_init(&ctx, &p, NULL, ws, need, (const float*)((char*)phi0 + 2), NULL) ==
         LBM_CH_EINVAL);
  lbm_ch_velocity vel;
  memset(&vel, 0, sizeof vel);
  p.velocity_mode = LBM_CH_VEL_SEPARABLE;
  EXPECT(lbm_ch_init(&ctx, &p, &vel, ws, need, phi0, NULL) == LBM_CH_EINVAL);
  p.velocity_mode = LBM_CH_VEL_FIELD;
  EXPECT(lbm_ch_init(&ctx, &p, &vel, ws, lbm_ch_workspace_bytes(&p), phi0, NULL) ==
         LBM_CH_EINVAL);
  p.velocity_mode = LBM_CH_VEL_NS;
  vel.ux = phi0;
  EXPECT(lbm_ch_init(&ctx, &p, &vel, ws, lbm_ch_workspace_bytes(&p), phi0, NULL) ==
         LBM_CH_EINVAL);
  vel.ux = NULL;
  p.velocity_mode = LBM_CH_VEL_NONE;
  vel.time_factor = (const double*)phi0;
  vel.n_time_factor = -1;
  EXPECT(lbm_ch_init(&ctx, &p, &vel, ws, need, phi0, NULL) == LBM_CH_EINVAL);
  p.model = 3;
  p.storage = LBM_CH_STORE_F16;
  EXPECT(lbm_ch_init(&ctx, &p, NULL, ws, lbm_ch_workspace_bytes(&p), phi0, NULL) ==
         LBM_CH_EUNSUPPORTED);
  p = params(64, 48);
  int st = lbm_ch_init(&ctx, &p, NULL, ws, need, phi0, NULL);
  EXPECT(st == LBM_CH_EHIP && ctx == NULL);  /* no device here */
  printf("init without a device: %s (hip error %d)\n", lbm_ch_strerror(st),
         lbm_ch_last_hip_error());

  /* NULL contexts and batches */
  EXPECT(lbm_ch_step(NULL, 1, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_moments(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_diagnostics(NULL, NULL, NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_check_finite(NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_step_count(NULL) == -1);
  EXPECT(lbm_ch_state_bytes(NULL) == 0);
  EXPECT(lbm_ch_save_state(NULL, NULL, 0, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_load_state(NULL, NULL, 0, 0, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_set_tiles(NULL, 64, 8) == LBM_CH_ESTATE);
  int32_t tx = 0, ty = 0;
  EXPECT(lbm_ch_get_tiles(NULL, &tx, &ty) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_set_graphs(NULL, 1) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_autotune(NULL, NULL, 0, 1, NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_record(NULL, 1, NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_adjoint(NULL, 1, 1, NULL, NULL, NULL, NULL, NULL, 0, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_adjoint_static(NULL, 1, 1, NULL, NULL, NULL, NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_destroy(NULL) == LBM_CH_OK);
  lbm_ch_batch* b = NULL;
  EXPECT(lbm_ch_batch_create(&b, NULL, 0, NULL, 0) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_batch_create(NULL, NULL, 1, NULL, 0) == LBM_CH_EINVAL);
  EXPECT(lbm_ch_batch_workspace_bytes(0) == 0);
  EXPECT(lbm_ch_batch_workspace_bytes(64) > 0);
  EXPECT(lbm_ch_batch_set_tiles(NULL, 64, 8) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_batch_get_tiles(NULL, &tx, &ty) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_batch_set_schedule(NULL, 1) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_batch_get_schedule(NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_batch_step(NULL, 1, 0, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_batch_state_bytes(NULL) == 0);
  EXPECT(lbm_ch_batch_autotune(NULL, NULL, 0, 1, NULL, NULL) == LBM_CH_ESTATE);
  EXPECT(lbm_ch_batch_destroy(NULL) == LBM_CH_OK);
  for (int s = -6; s <= 1; ++s) EXPECT(lbm_ch_strerror(s) != NULL);
  EXPECT(strcmp(lbm_ch_strerror(12345), "unknown status") == 0);
  printf("abi driver: %d failed checks\n", fails);
  return fails ? 1 : 0;
}
