/* Compiles include/ramlt.h as C99 and calls the library's host-side entry points (no GPU
 * work): the ABI version, workspace sizes, and validation errors of every entry point. */
#include <stdio.h>
#include <string.h>

#include "ramlt.h"

int main(void) {
  ramlt_frame f;
  memset(&f, 0, sizeof f);
  printf("abi %d %d\n", (int)(ramlt_abi_version() >> 16), (int)sizeof(ramlt_frame));
  f.W = 64;
  f.H = 32;
  f.S = 4;
  printf("stats_null %d\n", stats_accumulate(NULL, NULL, 1, NULL, 0, NULL));
  printf("stats_noptr %d\n", stats_accumulate(&f, NULL, 1, NULL, 0, NULL));
  printf("last_error_set %d\n", ramlt_last_error()[0] != '\0');
  printf("adapt_ws %d\n", ramlt_adapt_workspace_size(1000, 400) > 0);
  printf("adapt_null %d\n", region_adapt(NULL, NULL, NULL, NULL, 0, NULL, 0, NULL));
  printf("qt_ws %d\n", ramlt_quadtree_workspace_size(1000) > 0);
  printf("qt_null %d\n", quadtree_lookup(NULL, NULL, NULL, NULL, NULL, 0, 1, NULL));
  printf("perturb_bad %d\n", perturb_directions(NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL, 0, NULL));
  printf("rrmse_bad %d\n", rrmse(NULL, NULL, 0, 0, 0.01, NULL, NULL, NULL, 0, NULL));
  printf("lens_bad %d\n", lens_chain_step(NULL, 64, 32, 0.5f, NULL, 4, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, 0, NULL));
  printf("lens_ws %d\n", ramlt_lens_workspace_size(20) > 0);
  printf("lens_sort_bad %d\n", lens_chain_sort(0, 32, 0.5f, NULL, NULL, 10, NULL, NULL, NULL, NULL, 0, NULL));
  printf("lens_sort_ws %d\n", ramlt_lens_sort_workspace_size(1 << 20) > 0);
  printf("rrmse_ws %d\n", ramlt_rrmse_workspace_size(1920, 1080) > 0);
  return 0;
}
