/* A plain C program that runs the engine on the GPU through the ABI alone (no Python, no
 * HIP calls of its own): host X in, factors and objectives out.  Two instances of a planted
 * problem (X = B0 C0 from a fixed linear congruential sequence) run 20 iterations each,
 * one alone and one in a batch with a second, differently shaped member; the program prints
 * the objective history and the factor checksums of both, then checks that the objective
 * does not increase, that the factors are nonnegative and that the batched member equals
 * the instance run alone bit for bit.  Exit status 0 when every check holds. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "did.h"

static uint64_t lcg_state = 12345;
static float unif(void) {
  lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return (float)((lcg_state >> 40) & 0xFFFFFF) / 16777216.0f;
}

static float* planted(int64_t M, int64_t N, int K) {
  float* B0 = (float*)malloc(sizeof(float) * M * K);
  float* C0 = (float*)malloc(sizeof(float) * K * N);
  float* X = (float*)malloc(sizeof(float) * M * N);
  for (int64_t i = 0; i < M * K; ++i) B0[i] = unif();
  for (int64_t i = 0; i < K * N; ++i) C0[i] = unif();
  for (int64_t j = 0; j < N; ++j)
    for (int64_t m = 0; m < M; ++m) {
      double s = 0.0;
      for (int k = 0; k < K; ++k) s += (double)B0[k * M + m] * C0[j * K + k];
      X[j * M + m] = (float)s;
    }
  free(B0);
  free(C0);
  return X;
}

static int failures = 0;
#define CHECK(cond, what)                                   \
  do {                                                      \
    const int ok_ = (cond);                                 \
    printf("%s %s\n", ok_ ? "ok" : "FAIL", what);           \
    if (!ok_) {                                             \
      ++failures;                                           \
      printf("  last error: %s\n", did_last_error());       \
    }                                                       \
  } while (0)

int main(void) {
  const int64_t M = 300, N = 2000, M2 = 200, N2 = 1500;
  const int K = 12, K2 = 40, T = 20;
  float* X = planted(M, N, K);
  float* X2 = planted(M2, N2, K2);

  did_handle a = NULL, b = NULL, c = NULL;
  CHECK(did_init(X, M, N, K, 7, &a) == DID_OK, "did_init (host X)");
  CHECK(did_iterate(a, T) == DID_OK, "did_iterate alone");
  double fa[32];
  int64_t na = 0;
  CHECK(did_history(a, fa, 32, &na) == DID_OK && na == T, "history of the instance alone");
  int mono = 1;
  for (int64_t t = 1; t < na; ++t) mono = mono && fa[t] <= fa[t - 1];
  CHECK(mono, "objective does not increase");
  float* Ba = (float*)malloc(sizeof(float) * M * K);
  float* Ca = (float*)malloc(sizeof(float) * K * N);
  CHECK(did_factors(a, Ba, Ca) == DID_OK, "did_factors");
  int nonneg = 1;
  double sb = 0.0, scs = 0.0;
  for (int64_t i = 0; i < M * K; ++i) { nonneg = nonneg && Ba[i] >= 0.0f; sb += Ba[i]; }
  for (int64_t i = 0; i < K * N; ++i) { nonneg = nonneg && Ca[i] >= 0.0f; scs += Ca[i]; }
  CHECK(nonneg, "factors are nonnegative");

  /* the same instance again, advanced in a batch beside a second member */
  did_batch bt = NULL;
  CHECK(did_init(X, M, N, K, 7, &b) == DID_OK && did_init(X2, M2, N2, K2, 9, &c) == DID_OK, "two more instances");
  CHECK(did_batch_create(NULL, &bt) == DID_OK && did_batch_add(bt, b) == DID_OK && did_batch_add(bt, c) == DID_OK,
        "batch of two members");
  CHECK(did_batch_iterate(bt, T) == DID_OK && did_batch_sync(bt) == DID_OK, "batched iterations");
  CHECK(did_batch_remove(bt, b) == DID_OK && did_batch_remove(bt, c) == DID_OK, "members leave");
  double fb[32];
  int64_t nb = 0;
  CHECK(did_history(b, fb, 32, &nb) == DID_OK && nb == T, "history of the batched member");
  float* Bb = (float*)malloc(sizeof(float) * M * K);
  float* Cb = (float*)malloc(sizeof(float) * K * N);
  CHECK(did_factors(b, Bb, Cb) == DID_OK, "factors of the batched member");
  CHECK(memcmp(Ba, Bb, sizeof(float) * M * K) == 0 && memcmp(Ca, Cb, sizeof(float) * K * N) == 0 &&
            memcmp(fa, fb, sizeof(double) * T) == 0,
        "batched member equals the instance alone bit for bit");

  double f = 0.0;
  CHECK(did_objective(a, &f) == DID_OK && f <= fa[T - 1], "final objective");
  printf("objective f[0] %.17g f[%d] %.17g final %.17g\n", fa[0], T - 1, fa[T - 1], f);
  printf("history");
  for (int64_t t = 0; t < na; ++t) printf(" %.17g", fa[t]);
  printf("\n");
  printf("checksums B %.17g C %.17g\n", sb, scs);

  CHECK(did_batch_free(bt) == DID_OK, "did_batch_free");
  CHECK(did_free(a) == DID_OK && did_free(b) == DID_OK && did_free(c) == DID_OK, "did_free");
  free(Ba); free(Ca); free(Bb); free(Cb); free(X); free(X2);
  return failures ? 1 : 0;
}
