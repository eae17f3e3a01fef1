/* Host-side checks of the C ABI without a GPU, built against a host-only,
 * AddressSanitizer + UndefinedBehaviorSanitizer build of the library
 * (tests/test_host_sanitizers.py): every entry point rejects missing
 * arguments before touching a device, psca_create fails cleanly where no
 * usable GPU exists, and the status strings and version are well formed. */
#include <stdio.h>
#include <string.h>

#include "psca.h"

static int failures = 0;

#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                 \
    }                                                             \
  } while (0)

int main(void) {
  EXPECT(psca_version() > 0);
  for (int code = 1; code >= -8; --code) {
    const char *s = psca_strerror(code);
    EXPECT(s != NULL && strlen(s) > 0);
  }

  psca_params prm;
  memset(&prm, 0, sizeof prm);
  prm.variant = PSCA_ML_UD;
  prm.iters = 10;
  prm.rho0 = 0.5f;
  prm.rho_decay = 0.5f;
  prm.sigma2 = 1.0f;
  prm.M = 8;
  psca_c32 dummy_c[4];
  float dummy_f[4];
  int32_t status = 0;

  /* no context */
  EXPECT(psca_create(NULL, 0) == PSCA_EINVAL);
  EXPECT(psca_destroy(NULL) == PSCA_OK);
  EXPECT(psca_sample_cov(NULL, dummy_c, 2, 2, dummy_c, NULL) == PSCA_EINVAL);
  EXPECT(psca_sample_cov_batch(NULL, 1, dummy_c, 4, 2, 2, dummy_c, 4, NULL) == PSCA_EINVAL);
  EXPECT(psca_detect(NULL, dummy_c, dummy_c, 2, 2, &prm, dummy_f, &status, NULL) == PSCA_EINVAL);
  EXPECT(psca_detect_y(NULL, dummy_c, dummy_c, 2, 2, &prm, dummy_f, &status, NULL) == PSCA_EINVAL);
  EXPECT(psca_detect_noalloc(NULL, dummy_c, dummy_c, 2, 2, &prm, dummy_f, &status, NULL) == PSCA_EINVAL);
  EXPECT(psca_iterate(NULL, dummy_c, dummy_c, 2, 2, &prm, 0.5f, dummy_f, dummy_f + 2, NULL, NULL, NULL, &status,
                      NULL) == PSCA_EINVAL);
  EXPECT(psca_net_forward(NULL, dummy_c, dummy_c, 2, 2, &prm, dummy_f, &status, NULL) == PSCA_EINVAL);
  EXPECT(psca_layer_backward(NULL, dummy_c, dummy_c, 2, 2, &prm, 0.5f, dummy_f, dummy_f, dummy_f, dummy_f, &status,
                             NULL) == PSCA_EINVAL);
  EXPECT(psca_layer_backward_batch(NULL, 1, NULL, 0.5f, NULL) == PSCA_EINVAL);
  EXPECT(psca_detect_batch(NULL, 1, NULL, NULL) == PSCA_EINVAL);
  int team = 0;
  EXPECT(psca_autotune_batch(NULL, 1, NULL, 2, &team, NULL) == PSCA_EINVAL);
  psca_plan *plan = NULL;
  EXPECT(psca_plan_create(NULL, 1, NULL, 0, &plan) == PSCA_EINVAL);
  EXPECT(plan == NULL);
  EXPECT(psca_plan_launch(NULL, NULL) == PSCA_EINVAL);
  EXPECT(psca_plan_team_size(NULL) == PSCA_EINVAL);
  EXPECT(psca_plan_destroy(NULL) == PSCA_OK);
  EXPECT(psca_threshold(NULL, 4, 0.5f, NULL, NULL) == PSCA_EINVAL);

  /* a context on a device that does not exist: a clean failure, nothing leaked */
  psca_ctx *ctx = (psca_ctx *)0x1;
  const int rc = psca_create(&ctx, 1 << 20);
  EXPECT(rc == PSCA_EINVAL || rc == PSCA_EHIP);
  EXPECT(ctx == NULL);
  EXPECT(psca_create(&ctx, -1) != PSCA_OK);
  EXPECT(ctx == NULL);

  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("host ABI checks passed\n");
  return 0;
}
