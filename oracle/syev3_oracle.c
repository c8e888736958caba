/*
 * syev3_oracle.c -- CPU oracle for the 3x3 real symmetric eigenproblem.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that
 * the GPU library is checked against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU path.
 *
 * It follows C. F. Borges, "Solving the 3x3 Real Symmetric Eigenproblem"
 * (arXiv:1806.06698), step by step, in IEEE double precision, one matrix at
 * a time:
 *   Sec. 1      Jacobi rotation in the (1,2)-plane to an ordered arrow
 *   Sec. 1.1    beta-, combo- and numerical deflation (Givens rotation G,
 *               the EISPACK-style test and its simplified variant)
 *   Sec. 1.2    the two shifted fully reduced arrows (mu and nu), the
 *               eigenvector formulas u1, u3, u2 and the trace identity
 *   Sec. 1.4.1  the Borges-Gragg zero finder (rational model, increment
 *               quadratic, start from +infinity, relative stop test)
 *   Sec. 1.4.2  Newton's method from the left (alternative zero finder)
 *
 * Readings where the paper is silent:
 *   - Input scaling by a power of two so that max|a_ij| lies in [1,2); the
 *     eigenvalues are scaled back at the end.  Exact, reversible.
 *   - The Jacobi rotation is the textbook symmetric Schur rotation (Golub &
 *     Van Loan); the paper's own rotation comes from a paper that is not
 *     available.  Ordering alpha1 >= alpha2 by swapping the two columns.
 *   - h is treated as zero when h <= eps*(|alpha1|+|alpha2|+|gamma|), the
 *     EISPACK criterion applied to the other off-diagonal of the same
 *     tridiagonal (Sec. 1.1).  Flag ORACLE_NO_H_GUARD gives the literal
 *     "h == 0 only" behaviour.
 *   - The constant C of both deflation tests is 1 and the comparison is
 *     "<=" as printed; the constant of the zero-finder stop test is 2.
 *   - The Borges-Gragg iteration also stops when rounding has carried it
 *     onto or past the root (f <= 0) or when it no longer decreases; the
 *     square-root argument of the increment is clamped at zero.
 *   - Output: eigenvalues ascending, eigenvector columns permuted with
 *     them (stable for ties); no sign normalisation.
 *   - Non-finite input gives NaN eigenvalues and eigenvectors.
 *
 * Parity unpinned: the iteration counts it reports (the paper prints none)
 * and the identity of each eigenvector, i.e. its sign and the basis chosen
 * inside a repeated eigenvalue's eigenspace (several results are correct).
 * What the tests pin: the arrow reduction (interlacing), the exact
 * deflations, the zero finder's root (the largest eigenvalue of the reduced
 * arrow), the eigenvalues, the two accuracy measures of Sec. 1.5 and the
 * Sec. 1.3 orthogonality bound, against closed forms, invariants, LAPACK
 * and cyclic Jacobi.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no contraction, so the
 * result does not depend on FMA formation).
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_SIMPLIFIED_DEFLATION 1u /* Sec. 1.1, simplified test */
#define ORACLE_NO_H_GUARD 2u           /* only h == 0 exits as diagonal */
#define ORACLE_NEWTON 4u               /* Sec. 1.4.2 zero finder */
#define ORACLE_NO_SCALE 8u             /* skip the power-of-two scaling */

/* branch codes reported per matrix */
#define BR_ZERO 0
#define BR_NONFINITE 1
#define BR_DIAGONAL 2
#define BR_DEFLATED 3
#define BR_REDUCED 4

static const double EPS = DBL_EPSILON; /* 2^-52 */
static const double C_DEFL = 1.0;      /* constant C of the deflation tests */
static const double C_STOP = 2.0;      /* constant C of the zero-finder stops */
#define MAX_ITER 64

/* ------------------------------------------------------------------------ */
/* 2x2 symmetric eigenproblem [[p, r], [r, q]] by one Jacobi rotation.       */
/* Returns l1 >= l2 and the rotation K (row-major 2x2) whose first column is */
/* the eigenvector of l1 and whose second column is that of l2.              */
/* Textbook symmetric Schur rotation: tau = (q-p)/(2r),                     */
/* t = sign(tau)/(|tau| + sqrt(1+tau^2)), c = 1/sqrt(1+t^2), s = t c; then   */
/* J = [[c, s], [-s, c]] gives J^T B J = diag(p - t r, q + t r).             */
/* ------------------------------------------------------------------------ */
static void jacobi2(double p, double r, double q, double *l1, double *l2,
                    double K[4]) {
  double c = 1.0, s = 0.0, t = 0.0;
  if (r != 0.0) {
    double tau = (q - p) / (2.0 * r);
    double sg = (tau >= 0.0) ? 1.0 : -1.0;
    t = sg / (fabs(tau) + hypot(1.0, tau));
    c = 1.0 / hypot(1.0, t);
    s = t * c;
  }
  double a1 = p - t * r;
  double a2 = q + t * r;
  if (a1 >= a2) {
    *l1 = a1; *l2 = a2;
    K[0] = c;  K[1] = s;
    K[2] = -s; K[3] = c;
  } else { /* swap the columns so that the larger eigenvalue comes first */
    *l1 = a2; *l2 = a1;
    K[0] = s; K[1] = c;
    K[2] = c; K[3] = -s;
  }
}

/* ------------------------------------------------------------------------ */
/* The spectral function of the fully reduced arrow                          */
/*   [[0, 0, b1], [0, -ab, b2], [b1, b2, gb]]   (Sec. 1.4)                   */
/* f(x) = x - gb - b1^2/x - b2^2/(x+ab),                                     */
/* f'(x) = 1 + b1^2/x^2 + b2^2/(x+ab)^2.                                     */
/* ------------------------------------------------------------------------ */
static double spec_f(double b1, double b2, double ab, double gb, double x) {
  return x - gb - b1 * b1 / x - b2 * b2 / (x + ab);
}
static double spec_fp(double b1, double b2, double ab, double x) {
  double p = x + ab;
  return 1.0 + b1 * b1 / (x * x) + b2 * b2 / (p * p);
}

/* ------------------------------------------------------------------------ */
/* Borges-Gragg zero finder for the unique positive zero of f (Sec. 1.4.1).  */
/* The local model phi(x) = w0 x - sigma - w1/x matches f, f', f'' at x_j.   */
/* The increment Delta = x_j - x_{j+1} solves a D^2 + b D - f = 0 with       */
/* a = -w0/x_j and b = f' + f/x_j, evaluated as                              */
/* (2f/b) / (1 + sqrt(1 + (2a/b)(2f/b))), or, when that step would remove   */
/* more than half of x_j, as the zero of phi_j itself.  x_0 is the zero of   */
/* the model taken from +infinity, x - gb - (b1^2+b2^2)/x.  Stop when        */
/* f/f' < C eps x.                                                           */
/* trace (if not NULL) receives x_0, x_1, ...; *iters the number of f        */
/* evaluations.                                                              */
/* ------------------------------------------------------------------------ */
double oracle_bg_root(double b1, double b2, double ab, double gb, int *iters,
                      double *trace, int trace_cap) {
  double H = b1 * b1 + b2 * b2;
  double g2 = gb / 2.0;
  double x;
  if (gb >= 0.0)
    x = g2 + sqrt(g2 * g2 + H);
  else /* multiply top and bottom by the conjugate (no cancellation) */
    x = H / (-g2 + sqrt(g2 * g2 + H));
  int j;
  for (j = 0; j < MAX_ITER; ++j) {
    if (trace && j < trace_cap) trace[j] = x;
    double f = spec_f(b1, b2, ab, gb, x);
    double fp = spec_fp(b1, b2, ab, x);
    if (f <= 0.0) break;                /* rounding reached the root */
    if (f / fp < C_STOP * EPS * x) break; /* |x_j - root| < f/f' */
    double p = x + ab;
    double w0 = 1.0 + b2 * b2 * ab / (p * p * p);
    double a = -w0 / x;
    double b = fp + f / x;
    double F = 2.0 * f / b;
    double D = 1.0 + (2.0 * a / b) * F;
    if (D < 0.0) D = 0.0;
    double delta = F / (1.0 + sqrt(D));
    double xn;
    if (delta <= 0.5 * x) {
      xn = x - delta;
    } else {
      /* The step removes more than half of x_j, so x_j - Delta would lose
       * the leading digits of a root much smaller than x_j (a root next to
       * the pole at 0).  x_{j+1} is by definition the zero of phi_j in
       * (0, inf): solve w0 x^2 - sigma x - w1 = 0 for it without
       * cancellation, with w1 and sigma as the paper defines them. */
      double r = x / p;
      double w1 = b1 * b1 + b2 * b2 * r * r * r;
      double sigma = w0 * x - w1 / x - f;
      double disc = sqrt(sigma * sigma + 4.0 * w0 * w1);
      xn = (sigma >= 0.0) ? (sigma + disc) / (2.0 * w0)
                          : 2.0 * w1 / (disc - sigma);
    }
    if (!(xn < x)) break; /* no further decrease in floating point */
    x = xn;
  }
  if (iters) *iters = (j < MAX_ITER) ? j + 1 : MAX_ITER;
  return x;
}

/* ------------------------------------------------------------------------ */
/* Newton's method for the same zero, from the left (Sec. 1.4.2).  x_0 is    */
/* where f meets -b2^2/(x+ab): x_0 = gb/2 + sqrt((gb/2)^2 + b1^2).  Stop     */
/* when |f| < C eps x.                                                       */
/* ------------------------------------------------------------------------ */
double oracle_newton_root(double b1, double b2, double ab, double gb,
                          int *iters, double *trace, int trace_cap) {
  double g2 = gb / 2.0;
  double x;
  if (gb >= 0.0)
    x = g2 + sqrt(g2 * g2 + b1 * b1);
  else
    x = b1 * b1 / (-g2 + sqrt(g2 * g2 + b1 * b1));
  int j;
  for (j = 0; j < MAX_ITER; ++j) {
    if (trace && j < trace_cap) trace[j] = x;
    double f = spec_f(b1, b2, ab, gb, x);
    if (f >= 0.0) break;                    /* rounding reached the root */
    if (fabs(f) < C_STOP * EPS * x) break;  /* |x_j - root| < |f| */
    double fp = spec_fp(b1, b2, ab, x);
    double xn = x - f / fp;
    if (!(xn > x)) break;
    x = xn;
  }
  if (iters) *iters = (j < MAX_ITER) ? j + 1 : MAX_ITER;
  return x;
}

/* Normalise a 3-vector: divide by its largest magnitude, then by the     */
/* 2-norm of the result (no overflow or underflow in the squares).          */
static void normalize3(double u[3]) {
  double m = fabs(u[0]);
  if (fabs(u[1]) > m) m = fabs(u[1]);
  if (fabs(u[2]) > m) m = fabs(u[2]);
  if (m == 0.0) return;
  double v0 = u[0] / m, v1 = u[1] / m, v2 = u[2] / m;
  double nrm = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
  u[0] = v0 / nrm; u[1] = v1 / nrm; u[2] = v2 / nrm;
}

/* Arrow reduction (Sec. 1): alpha1 >= alpha2, beta, gamma and the 2x2    */
/* rotation J (row-major) with J^T [[a11,a12],[a12,a22]] J diagonal.        */
void oracle_arrow(const double a[6], double arrow[5], double J[4]) {
  double l1, l2;
  jacobi2(a[0], a[1], a[3], &l1, &l2, J);
  /* [beta1; beta2] = J^T [a13; a23] */
  arrow[0] = l1;
  arrow[1] = l2;
  arrow[2] = J[0] * a[2] + J[2] * a[4];
  arrow[3] = J[1] * a[2] + J[3] * a[4];
  arrow[4] = a[5];
}

/* info[0] = branch, info[1] = iterations for mu, info[2] = for nu,         */
/* info[3] = scaling exponent k.                                            */
void oracle_solve(const double a_in[6], double lam[3], double V[9],
                  unsigned flags, int info[4]) {
  int br, it_mu = 0, it_nu = 0, k = 0;
  double a[6];
  int finite = 1;
  double m = 0.0;
  for (int i = 0; i < 6; ++i) {
    if (!isfinite(a_in[i])) finite = 0;
    if (fabs(a_in[i]) > m) m = fabs(a_in[i]);
  }
  if (!finite) {
    for (int i = 0; i < 3; ++i) lam[i] = NAN;
    for (int i = 0; i < 9; ++i) V[i] = NAN;
    if (info) { info[0] = BR_NONFINITE; info[1] = info[2] = info[3] = 0; }
    return;
  }
  if (m == 0.0) {
    for (int i = 0; i < 3; ++i) lam[i] = 0.0;
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    if (info) { info[0] = BR_ZERO; info[1] = info[2] = info[3] = 0; }
    return;
  }
  /* scale by 2^-k so that max|a_ij| lies in [1, 2) */
  if (!(flags & ORACLE_NO_SCALE)) k = ilogb(m);
  for (int i = 0; i < 6; ++i) a[i] = ldexp(a_in[i], -k);

  /* Sec. 1: ordered arrow */
  double arrow[5], J[4];
  oracle_arrow(a, arrow, J);
  double al1 = arrow[0], al2 = arrow[1], be1 = arrow[2], be2 = arrow[3],
         ga = arrow[4];

  double l[3];     /* eigenvalues (unordered) */
  double U[3][3];  /* U[c][r]: column c, row r, in arrow coordinates */

  /* Sec. 1.1: h = sqrt(beta1^2 + beta2^2) */
  double h = hypot(be1, be2);
  int diagonal = (h == 0.0);
  if (!diagonal && !(flags & ORACLE_NO_H_GUARD))
    diagonal = (h <= EPS * (fabs(al1) + fabs(al2) + fabs(ga)));

  if (diagonal) {
    br = BR_DIAGONAL;
    l[0] = al1; l[1] = al2; l[2] = ga;
    memset(U, 0, sizeof U);
    U[0][0] = U[1][1] = U[2][2] = 1.0;
  } else {
    int deflate = 0;
    double d1 = 0.0, d2 = 0.0, cg = 0.0, sg = 0.0;
    double al = al1 - al2;
    if (be1 == 0.0 || be2 == 0.0 || al == 0.0) {
      /* exact beta- or combo-deflation: e = 0 below */
      deflate = 1;
    } else {
      /* numerical deflation test on G A G^T */
      double lhs = fabs(al * be1 * be2);
      double rhs;
      if (flags & ORACLE_SIMPLIFIED_DEFLATION)
        rhs = C_DEFL * EPS * fabs(al1 + al2) * h * h;
      else
        rhs = C_DEFL * EPS *
              (fabs(al1 * be2 * be2 + al2 * be1 * be1) +
               fabs(al1 * be1 * be1 + al2 * be2 * be2));
      deflate = (lhs <= rhs);
    }
    if (deflate) {
      br = BR_DEFLATED;
      /* G = [[b2/h, -b1/h, 0], [b1/h, b2/h, 0], [0, 0, 1]] */
      cg = be2 / h;
      sg = be1 / h;
      if (be1 == 0.0) {        /* beta-deflation at position 1 */
        d1 = al1; d2 = al2;
      } else if (be2 == 0.0) { /* beta-deflation at position 2 */
        d1 = al2; d2 = al1;
      } else if (al == 0.0) {  /* combo-deflation */
        d1 = al1; d2 = al1;
      } else {                 /* numerical deflation, entries of G A G^T */
        d1 = (al1 * be2 * be2 + al2 * be1 * be1) / (h * h);
        d2 = (al1 * be1 * be1 + al2 * be2 * be2) / (h * h);
      }
      /* accept d1 with eigenvector G^T e1 = (cg, -sg, 0) */
      l[0] = d1;
      U[0][0] = cg; U[0][1] = -sg; U[0][2] = 0.0;
      /* the rest from the 2x2 [[d2, h], [h, gamma]] */
      double t1, t2, K[4];
      jacobi2(d2, h, ga, &t1, &t2, K);
      l[1] = t1;
      l[2] = t2;
      /* eigenvector G^T (0, p, q) = (sg p, cg p, q) */
      U[1][0] = sg * K[0]; U[1][1] = cg * K[0]; U[1][2] = K[2];
      U[2][0] = sg * K[1]; U[2][1] = cg * K[1]; U[2][2] = K[3];
    } else {
      br = BR_REDUCED;
      /* ordered and reduced: alpha1 > alpha2, beta1 beta2 != 0 */
      if (!(al > 0.0) || be1 == 0.0 || be2 == 0.0) abort();
      double ab = al;
      double mu, nu;
      /* mu = lambda1 - alpha1: rightmost eigenvalue of A - alpha1 I */
      /* nu = alpha2 - lambda3: of P(alpha2 I - A)P (betas swapped)  */
      if (flags & ORACLE_NEWTON) {
        mu = oracle_newton_root(be1, be2, ab, ga - al1, &it_mu, NULL, 0);
        nu = oracle_newton_root(be2, be1, ab, al2 - ga, &it_nu, NULL, 0);
      } else {
        mu = oracle_bg_root(be1, be2, ab, ga - al1, &it_mu, NULL, 0);
        nu = oracle_bg_root(be2, be1, ab, al2 - ga, &it_nu, NULL, 0);
      }
      l[0] = al1 + mu;       /* lambda1 */
      l[1] = nu - mu + ga;   /* lambda2, trace identity */
      l[2] = al2 - nu;       /* lambda3 */
      /* u1 */
      U[0][0] = be1 * (mu + ab); U[0][1] = be2 * mu; U[0][2] = mu * (mu + ab);
      /* u2 */
      U[1][0] = -be2 * mu * (nu + ab);
      U[1][1] = be1 * nu * (mu + ab);
      U[1][2] = be1 * be2 * ab;
      /* u3 */
      U[2][0] = be1 * nu; U[2][1] = be2 * (nu + ab); U[2][2] = -nu * (nu + ab);
      normalize3(U[0]);
      normalize3(U[1]);
      normalize3(U[2]);
    }
  }

  /* back to the coordinates of A: V = diag(J, 1) [u1 u2 u3] */
  double W[3][3]; /* W[c][r] */
  for (int c = 0; c < 3; ++c) {
    W[c][0] = J[0] * U[c][0] + J[1] * U[c][1];
    W[c][1] = J[2] * U[c][0] + J[3] * U[c][1];
    W[c][2] = U[c][2];
  }
  /* unscale the eigenvalues */
  for (int i = 0; i < 3; ++i) l[i] = ldexp(l[i], k);

  /* ascending order, stable insertion sort carrying the columns */
  int ord[3] = {0, 1, 2};
  for (int i = 1; i < 3; ++i) {
    int key = ord[i], j = i - 1;
    while (j >= 0 && l[ord[j]] > l[key]) { ord[j + 1] = ord[j]; --j; }
    ord[j + 1] = key;
  }
  for (int c = 0; c < 3; ++c) {
    lam[c] = l[ord[c]];
    for (int r = 0; r < 3; ++r) V[3 * r + c] = W[ord[c]][r];
  }
  if (info) { info[0] = br; info[1] = it_mu; info[2] = it_nu; info[3] = k; }
}

/* ------------------------------------------------------------------------ */
/* Batch driver: A is n x 6 (a11 a12 a13 a22 a23 a33), lam n x 3 ascending, */
/* V n x 9 row-major (column c is the eigenvector of lam[c]).  info, if not */
/* NULL, is n x 4.  Work is split over nthreads POSIX threads.              */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t lo, hi;
  const double *A;
  double *lam, *V;
  int *info;
  unsigned flags;
} job_t;

static void *run_job(void *p) {
  job_t *jb = (job_t *)p;
  double scratch_v[9];
  for (int64_t i = jb->lo; i < jb->hi; ++i) {
    double *v = jb->V ? jb->V + 9 * i : scratch_v;
    oracle_solve(jb->A + 6 * i, jb->lam + 3 * i, v, jb->flags,
                 jb->info ? jb->info + 4 * i : NULL);
  }
  return NULL;
}

int oracle_solve_batch(int64_t n, const double *A, double *lam, double *V,
                       unsigned flags, int *info, int nthreads) {
  if (n < 0 || !A || !lam) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((int64_t)nthreads > n) nthreads = (int)(n > 0 ? n : 1);
  pthread_t th[256];
  job_t jobs[256];
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].lo = t * chunk < n ? t * chunk : n;
    jobs[t].hi = (t + 1) * chunk < n ? (t + 1) * chunk : n;
    jobs[t].A = A; jobs[t].lam = lam; jobs[t].V = V;
    jobs[t].info = info; jobs[t].flags = flags;
  }
  if (nthreads == 1) {
    run_job(&jobs[0]);
    return 0;
  }
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    if (pthread_create(&th[t], NULL, run_job, &jobs[t]) != 0) break;
    ++started;
  }
  for (int t = started; t < nthreads; ++t) run_job(&jobs[t]);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  return 0;
}

/* Exposed for the zero-finder pins. */
double oracle_spec_f(double b1, double b2, double ab, double gb, double x) {
  return spec_f(b1, b2, ab, gb, x);
}
double oracle_spec_fp(double b1, double b2, double ab, double x) {
  return spec_fp(b1, b2, ab, x);
}
void oracle_jacobi2(double p, double r, double q, double out[2], double K[4]) {
  jacobi2(p, r, q, &out[0], &out[1], K);
}
