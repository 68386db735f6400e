/* Host-side checks of the C-ABI under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Exercises every entry point that runs on the host alone (no device is needed): config
 * validation and workspace sizing, the clustering workspace sizes, NULL-handle and
 * NULL-argument rejection, and the status and error strings.  Built against a copy of the
 * library whose host code is instrumented; the build and run commands are given where the
 * sanitizer runs are documented.  Exit status 0 when every check holds. */
#include <stdio.h>
#include <string.h>
#include "vp.h"

static int failures = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++failures; } } while (0)

static vp_config good(void) {
  vp_config c;
  memset(&c, 0, sizeof c);
  c.n = 4096; c.ng = 64; c.precision = VP_FP64; c.L = 12.566370614359172; c.dt = 0.1;
  c.hist_cap = 16; c.element_order = 1;
  return c;
}

int main(void) {
  size_t b = 0;
  CHECK(vp_abi_version() > 0);
  vp_config c = good();
  CHECK(vp_workspace_bytes(&c, &b) == VP_OK && b > 0);
  c.element_order = 2;
  size_t b2 = 0;
  CHECK(vp_workspace_bytes(&c, &b2) == VP_OK && b2 > b);
  /* invalid configurations: each must be refused with a message */
  vp_config bad[8];
  for (int i = 0; i < 8; ++i) bad[i] = good();
  bad[0].ng = 100; bad[1].n = 0; bad[2].L = -1.0; bad[3].dt = 0.0; bad[4].element_order = 3;
  bad[5].moment_order = 4; bad[6].ng = 4096; bad[7].hist_cap = 0;
  for (int i = 0; i < 8; ++i) {
    CHECK(vp_workspace_bytes(&bad[i], &b) != VP_OK);
    const char* m = vp_last_error();
    CHECK(m != NULL && strlen(m) > 0);
  }
  CHECK(vp_workspace_bytes(NULL, &b) != VP_OK);
  CHECK(vp_workspace_bytes(&c, NULL) != VP_OK);
  CHECK(vp_cluster_workspace_bytes(100000, 1000, &b) == VP_OK && b > 0);
  CHECK(vp_cluster_workspace_bytes(0, 10, &b) != VP_OK);
  CHECK(vp_cluster_minibatch_workspace_bytes(100000, 1000, 4096, &b) == VP_OK && b > 0);
  CHECK(vp_cluster_minibatch_workspace_bytes(100000, 1000, 0, &b) != VP_OK);
  /* NULL handles */
  vp_diag d;
  vp_tuning t;
  memset(&t, 0, sizeof t);
  CHECK(vp_step(NULL, 1) != VP_OK);
  CHECK(vp_deposit(NULL) != VP_OK);
  CHECK(vp_poisson(NULL) != VP_OK);
  CHECK(vp_gather_push(NULL, 0.5, 1.0) != VP_OK);
  CHECK(vp_sync_state(NULL) != VP_OK);
  CHECK(vp_diagnostics(NULL, 0, &d, NULL) != VP_OK);
  CHECK(vp_set_tuning(NULL, &t) != VP_OK);
  CHECK(vp_get_tuning(NULL, &t) != VP_OK);
  CHECK(vp_retire(NULL, 0) != VP_OK);
  CHECK(vp_tune_scratch_bytes(NULL, &b) != VP_OK);
  /* every status has a string, out-of-range ones too */
  for (int s = -2; s < 64; ++s) {
    const char* m = vp_status_string((vp_status)s);
    CHECK(m != NULL && strlen(m) > 0);
  }
  if (failures == 0) printf("host sanitizer checks: all passed\n");
  return failures == 0 ? 0 : 1;
}
