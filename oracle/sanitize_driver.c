/*
 * sanitize_driver.c -- runs the oracle and the cyclic Jacobi on a fixed set
 * of matrices (random, special and extreme-scale) so that the tests can
 * execute them under AddressSanitizer and UndefinedBehaviorSanitizer.
 * TEST INFRASTRUCTURE ONLY.  Exit status 0 when every result is finite for
 * finite input and NaN for non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_solve(const double a_in[6], double lam[3], double V[9], unsigned flags,
                  int info[4]);
int oracle_solve_batch(int64_t n, const double *A, double *lam, double *V,
                       unsigned flags, int *info, int nthreads);
int jacobi_cyclic_solve(const double a6[6], double lam[3], double V[9]);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double unif(void) { /* xorshift64*, uniform in [0,1) */
  state ^= state >> 12; state ^= state << 25; state ^= state >> 27;
  return (double)((state * 2685821657736338717ull) >> 11) * 0x1p-53;
}

int main(void) {
  enum { N = 20000 };
  double *A = malloc(sizeof(double) * 6 * N), *lam = malloc(sizeof(double) * 3 * N),
         *V = malloc(sizeof(double) * 9 * N);
  int *info = malloc(sizeof(int) * 4 * N);
  if (!A || !lam || !V || !info) return 2;
  for (int i = 0; i < N; ++i) {
    double s = ldexp(1.0, (int)(unif() * 1800.0) - 900);
    for (int k = 0; k < 6; ++k) A[6 * i + k] = (2.0 * unif() - 1.0) * s;
    switch (i % 10) {
      case 1: A[6 * i + 1] = A[6 * i + 2] = A[6 * i + 4] = 0.0; break; /* diagonal */
      case 2: A[6 * i + 1] = 0.0; A[6 * i + 2] = 0.0; break;            /* beta */
      case 3: A[6 * i + 1] = 0.0; A[6 * i + 3] = A[6 * i + 0]; break;   /* combo */
      case 4: A[6 * i + 2] *= 1e-15; A[6 * i + 1] = 0.0; break;         /* near */
      case 5: for (int k = 0; k < 6; ++k) A[6 * i + k] = 0.0; break;    /* zero */
      default: break;
    }
  }
  A[6 * 7 + 2] = NAN;
  A[6 * 17 + 4] = INFINITY;
  int bad = 0;
  for (unsigned flags = 0; flags < 8; ++flags) {
    oracle_solve_batch(N, A, lam, V, flags, info, 3);
    for (int i = 0; i < N; ++i) {
      int nonfinite_in = (i == 7 || i == 17);
      for (int k = 0; k < 3; ++k)
        if (nonfinite_in != (isnan(lam[3 * i + k]) != 0)) ++bad;
    }
  }
  for (int i = 0; i < 2000; ++i) {
    double l[3], W[9];
    if (i == 7 || i == 17) continue;
    jacobi_cyclic_solve(A + 6 * i, l, W);
    for (int k = 0; k < 3; ++k)
      if (!isfinite(l[k])) ++bad;
  }
  printf("sanitized oracle run: %d bad results\n", bad);
  free(A); free(lam); free(V); free(info);
  return bad ? 1 : 0;
}
