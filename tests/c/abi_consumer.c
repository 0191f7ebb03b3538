/* A plain C consumer of the library: compiled with a C compiler against include/did.h and
 * linked to libdid.so, it exercises the calls that need no GPU (options, validation, memory
 * accounting, error reporting) and prints one line per check.  Exit status 0 when all
 * checks hold. */
#include <stdio.h>
#include <string.h>

#include "did.h"

static int failures = 0;

static void check(int cond, const char* what) {
  printf("%s %s\n", cond ? "ok" : "FAIL", what);
  if (!cond) ++failures;
}

int main(void) {
  did_opts o;
  check(did_default_opts(&o) == DID_OK, "did_default_opts");
  check(o.x_dtype == DID_F32 && o.refresh_every == 1 && o.algorithm == DID_ALG_DID && o.row_blocks == 0 &&
            o.x_tiled == 0 && o.col_waves == 0 && o.stream == NULL,
        "default option values");
  check(did_default_opts(NULL) == DID_EINVAL, "NULL options rejected");

  int64_t borrowed = 0, copied = 0;
  o.borrow_x = 1;
  check(did_mem_estimate(5000, 1000000, 50, &o, 1, &borrowed) == DID_OK && borrowed > 0, "estimate, borrowed X");
  check(did_mem_estimate(5000, 1000000, 50, &o, 0, &copied) == DID_OK, "estimate, copied X");
  check(copied - borrowed == (int64_t)4 * 5000 * 1000000, "a copied float32 X adds 4MN bytes");

  int64_t b = 0;
  check(did_mem_estimate(100, 100, 65, &o, 1, &b) == DID_EINVAL, "K > 64 rejected");
  check(strlen(did_last_error()) > 0, "did_last_error explains the failure");
  o.col_waves = 6;
  check(did_mem_estimate(1000, 5000, 20, &o, 1, &b) == DID_EINVAL, "col_waves outside {0, 4, 8} rejected");
  o.col_waves = 0;
  o.refresh_every = 0;
  check(did_mem_estimate(1000, 5000, 20, &o, 1, &b) == DID_EINVAL, "refresh_every 0 rejected");

  int32_t rb = 0, cw = 0;
  check(did_autotune(5, 1000, 3, DID_F32, 0, &rb, &cw, NULL) == DID_EINVAL, "autotune refuses thin shapes");
  check(did_iterate(NULL, 1) == DID_EINVAL, "NULL handle rejected");
  check(did_free(NULL) == DID_OK, "did_free(NULL) is a no-op");
  return failures ? 1 : 0;
}
