/*
 * jacobi_cyclic.c -- brute-force reference for the 3x3 symmetric
 * eigenproblem: the textbook cyclic-by-row Jacobi method (Golub & Van Loan,
 * "Matrix Computations", cyclic Jacobi), iterated until the off-diagonal
 * part is negligible.
 *
 * TEST INFRASTRUCTURE ONLY.  It is an independent check of the oracle in
 * syev3_oracle.c (a different algorithm, written separately), used on small
 * batches by the tests.  It is not the paper's method.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>

/* One symmetric Schur rotation on the full 3x3 M (row-major) in the (p,q)
 * plane; M <- J^T M J and W <- W J, where J is the identity except
 * J[p][p] = J[q][q] = c, J[p][q] = s, J[q][p] = -s. */
static void rotate(double M[9], double W[9], int p, int q) {
  double apq = M[3 * p + q];
  if (apq == 0.0) return;
  double tau = (M[3 * q + q] - M[3 * p + p]) / (2.0 * apq);
  double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                          : -1.0 / (-tau + sqrt(1.0 + tau * tau));
  if (!isfinite(tau)) t = 0.0; /* a_pq negligible against the diagonal gap */
  double c = 1.0 / sqrt(1.0 + t * t);
  double s = t * c;
  double Jm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  Jm[3 * p + p] = c;
  Jm[3 * q + q] = c;
  Jm[3 * p + q] = s;
  Jm[3 * q + p] = -s;
  double T[9], R[9];
  /* T = M J */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += M[3 * i + k] * Jm[3 * k + j];
      T[3 * i + j] = acc;
    }
  /* R = J^T T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Jm[3 * k + i] * T[3 * k + j];
      R[3 * i + j] = acc;
    }
  R[3 * p + q] = 0.0; /* annihilated by construction */
  R[3 * q + p] = 0.0;
  for (int i = 0; i < 9; ++i) M[i] = R[i];
  /* W <- W J */
  for (int i = 0; i < 3; ++i) {
    double wp = W[3 * i + p], wq = W[3 * i + q];
    W[3 * i + p] = c * wp - s * wq;
    W[3 * i + q] = s * wp + c * wq;
  }
}

/* a6 = (a11 a12 a13 a22 a23 a33).  lam ascending, V row-major with column c
 * the eigenvector of lam[c].  Returns the number of sweeps used. */
int jacobi_cyclic_solve(const double a6[6], double lam[3], double V[9]) {
  /* exact power-of-two scaling keeps the squares below in range */
  double m = 0.0;
  for (int i = 0; i < 6; ++i)
    if (fabs(a6[i]) > m) m = fabs(a6[i]);
  int k = (m > 0.0) ? ilogb(m) : 0;
  double M[9];
  M[0] = ldexp(a6[0], -k); M[1] = ldexp(a6[1], -k); M[2] = ldexp(a6[2], -k);
  M[3] = M[1];             M[4] = ldexp(a6[3], -k); M[5] = ldexp(a6[4], -k);
  M[6] = M[2];             M[7] = M[5];             M[8] = ldexp(a6[5], -k);
  double W[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double fro = 0.0;
  for (int i = 0; i < 9; ++i) fro += M[i] * M[i];
  fro = sqrt(fro);
  int sweep;
  for (sweep = 0; sweep < 100; ++sweep) {
    double off = 2.0 * (M[1] * M[1] + M[2] * M[2] + M[5] * M[5]);
    if (sqrt(off) <= 1e-3 * DBL_EPSILON * fro) break;
    rotate(M, W, 0, 1);
    rotate(M, W, 0, 2);
    rotate(M, W, 1, 2);
  }
  double l[3] = {M[0], M[4], M[8]};
  int ord[3] = {0, 1, 2};
  for (int i = 1; i < 3; ++i) {
    int key = ord[i], j = i - 1;
    while (j >= 0 && l[ord[j]] > l[key]) { ord[j + 1] = ord[j]; --j; }
    ord[j + 1] = key;
  }
  for (int c = 0; c < 3; ++c) {
    lam[c] = ldexp(l[ord[c]], k);
    for (int r = 0; r < 3; ++r) V[3 * r + c] = W[3 * r + ord[c]];
  }
  return sweep;
}

void jacobi_cyclic_batch(int64_t n, const double *A, double *lam, double *V,
                         int *sweeps) {
  for (int64_t i = 0; i < n; ++i) {
    int s = jacobi_cyclic_solve(A + 6 * i, lam + 3 * i, V + 9 * i);
    if (sweeps) sweeps[i] = s;
  }
}
