/* Host-side exercise of the C ABI (include/mpofit.h) for the AddressSanitizer
   build of the library: workspace queries, validation errors and error
   strings, with placeholder device pointers that the host code never
   dereferences.  Exit status 0 when every call returns the expected status. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/mpofit.h"

static int failures = 0;
#define EXPECT(call, want)                                                          \
  do {                                                                              \
    int got_ = (int)(call);                                                         \
    if (got_ != (want)) {                                                           \
      fprintf(stderr, "%s:%d: %s -> %d, want %d (%s)\n", __FILE__, __LINE__, #call, \
              got_, (int)(want), mpo_last_error());                                 \
      ++failures;                                                                   \
    }                                                                               \
  } while (0)

enum { L = 6, D = 2 };
static int32_t dims_a[L + 1] = {1, 4, 8, 8, 8, 4, 1};
static int32_t dims_b[L + 1] = {1, 4, 6, 6, 6, 4, 1};
static int32_t dims_p[L + 1] = {1, 3, 3, 3, 3, 3, 1};
static const double* cores[L];

static mpo_tt tt(int32_t* dims) {
  mpo_tt t;
  t.L = L;
  t.d = D;
  t.chi = dims;
  t.cores = cores;
  return t;
}

int main(void) {
  for (int i = 0; i < L; ++i) cores[i] = (const double*)(uintptr_t)(0x100000 + 4096 * i);
  mpo_pair pair;
  pair.A = tt(dims_a);
  pair.B = tt(dims_b);
  pair.chi_max = 0;
  mpo_fit_opts o;
  memset(&o, 0, sizeof o);
  o.chi_max = 8;
  o.precision = MPO_FP32;
  o.schedule = MPO_SCHED_SERIAL;
  o.sketch_p = 4;
  size_t bytes = 0, bytes2 = 0;
  EXPECT(mpo_fit_workspace_bytes(&pair, 1, &o, &bytes), MPO_OK);
  o.schedule = MPO_SCHED_EVEN_ODD;
  EXPECT(mpo_fit_workspace_bytes(&pair, 1, &o, &bytes2), MPO_OK);
  if (!(bytes > 0 && bytes2 > 0)) { fprintf(stderr, "zero workspace\n"); ++failures; }
  o.chi_max = 0;
  EXPECT(mpo_fit_workspace_bytes(&pair, 1, &o, &bytes), MPO_ERR_INVALID_ARG);
  o.chi_max = 8;
  EXPECT(mpo_fit_workspace_bytes(NULL, 1, &o, &bytes), MPO_ERR_INVALID_ARG);
  mpo_pair bad = pair;
  bad.B.L = 5;
  EXPECT(mpo_fit_workspace_bytes(&bad, 1, &o, &bytes), MPO_ERR_SHAPE);
  /* an initial guess of the wrong length, then a valid one */
  mpo_tt guess = tt(dims_b);
  guess.L = 4;
  o.c_init = &guess;
  EXPECT(mpo_fit_workspace_bytes(&pair, 1, &o, &bytes), MPO_ERR_SHAPE);
  guess.L = L;
  EXPECT(mpo_fit_workspace_bytes(&pair, 1, &o, &bytes), MPO_OK);
  o.c_init = NULL;
  /* init with a workspace that is too small fails before any device call */
  mpo_fit_ctx* ctx = NULL;
  EXPECT(mpo_fit_init(&ctx, &pair, 1, &o, (void*)(uintptr_t)0x200000, 1024, NULL), MPO_ERR_WORKSPACE);
  EXPECT(mpo_fit_init(NULL, &pair, 1, &o, (void*)(uintptr_t)0x200000, 1024, NULL), MPO_ERR_INVALID_ARG);
  /* exact-check and bond-projection queries */
  mpo_tt c = tt(dims_p);
  EXPECT(mpo_contract_check_bytes(&pair, &c, &bytes), MPO_OK);
  EXPECT(mpo_bond_project_bytes(&pair.A, 3, &bytes), MPO_OK);
  EXPECT(mpo_bond_project_bytes(&pair.A, 0, &bytes), MPO_ERR_INVALID_ARG);
  mpo_tt wrong = tt(dims_a);
  EXPECT(mpo_bond_project(&pair.A, 3, 0, 0, MPO_PROJ_STREAM_A, &wrong, (void*)(uintptr_t)0x200000,
                          (size_t)1 << 40, NULL), MPO_ERR_SHAPE);
  EXPECT(mpo_bond_project(&pair.A, 3, 0, 0, MPO_PROJ_STREAM_A, &c, (void*)(uintptr_t)0x200001,
                          (size_t)1 << 40, NULL), MPO_ERR_WORKSPACE);
  if (strlen(mpo_last_error()) == 0) { fprintf(stderr, "empty error string\n"); ++failures; }
  mpo_fit_destroy(NULL);
  printf("abi driver: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
