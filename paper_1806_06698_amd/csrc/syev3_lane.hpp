// syev3_lane.hpp -- per-lane solver for one 3x3 real symmetric eigenproblem.
//
// One GPU lane owns one matrix and keeps everything in registers: no LDS, no
// cross-lane traffic, no MFMA (the work is a short chain of scalar
// recurrences per matrix, not a contraction).  The method is Borges,
// "Solving the 3x3 Real Symmetric Eigenproblem":
//   Sec. 1    Jacobi rotation in the (1,2)-plane -> ordered arrow
//             (alpha1 >= alpha2, beta1, beta2, gamma)
//   Sec. 1.1  Givens rotation G taking beta1 to zero; h = ||beta||; exact
//             beta- and combo-deflations and the EISPACK-style numerical
//             deflation test on G A G^T (or its simplified form)
//   Sec. 1.2  for an ordered, reduced arrow: mu = lambda1 - alpha1 and
//             nu = alpha2 - lambda3 as rightmost zeros of two fully reduced
//             arrows, lambda2 from the trace identity, eigenvectors u1, u3, u2
//   Sec. 1.4  the zeros by the Borges-Gragg iteration (rational model
//             w0 x - sigma - w1/x, increment quadratic, start from +inf,
//             stop when f/f' < 2 eps x), or by Newton's method from the left.
//
// Choices made here (the paper leaves them open):
//   * every matrix is scaled by a power of two so that max |a_ij| is in
//     [1/2, 1); exact, undone on the eigenvalues at the end;
//   * the Jacobi rotation is the textbook symmetric Schur rotation written
//     with hypot(d, a12), d = (a22 - a11)/2, so it cannot overflow; entries
//     below 2^-500 of the scaled matrix count as zero in it;
//   * h counts as zero when h <= eps (|alpha1| + |alpha2| + |gamma|) (the
//     EISPACK criterion on the other off-diagonal of the tridiagonal
//     G A G^T) unless SYEV3_FLAG_NO_H_GUARD;
//   * the diagonal entries d1, d2 of G A G^T are formed as alpha1 - alpha s^2
//     etc., choosing the form with the smaller correction; algebraically the
//     paper's ratios, and bitwise exact for beta- and combo-deflations;
//   * a Borges-Gragg step that would remove more than half of x_j takes
//     x_{j+1} directly as the zero of the rational model (no cancellation
//     for roots next to the pole at 0);
//   * eigenvalues ascending, eigenvector columns carried along.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace syev3 {

constexpr double kEps64 = 0x1p-52;
constexpr float kEps32 = 0x1p-23f;
constexpr int kMaxIter = 32;     // zero-finder evaluations per root (FP64)
constexpr int kMaxIter32 = 24;   // FP32 zero-finder evaluations per root

constexpr uint32_t kFlagSimplified = 1u;
constexpr uint32_t kFlagNoHGuard = 2u;
constexpr uint32_t kFlagNewton = 4u;

enum Branch : int { kZero = 0, kNonFinite = 1, kDiagonal = 2, kDeflated = 3,
                    kReduced = 4 };

// ---------------------------------------------------------------------------
// Arithmetic primitives.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ double drcp(double x) { return 1.0 / x; }
__device__ __forceinline__ double drsqrt(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ __forceinline__ double ddiv(double a, double b) { return a / b; }

// ---------------------------------------------------------------------------
// 2x2 symmetric eigenproblem [[p, r], [r, q]] by one Jacobi rotation.
// l1 >= l2; (k11, k21) is the unit eigenvector of l1, (k12, k22) that of l2.
// t = sign(d) r / (|d| + hypot(d, r)), d = (q - p)/2, is the tangent of the
// textbook rotation; c = 1/sqrt(1 + t^2), s = t c; J = [[c, s], [-s, c]]
// gives J^T B J = diag(p - t r, q + t r).
// ---------------------------------------------------------------------------
struct Rot2 {
  double l1, l2, k11, k12, k21, k22;
};

__device__ __forceinline__ Rot2 rot2(double p, double r, double q) {
  const double d = 0.5 * (q - p);
  const double ad = dabs(d);
  double t = 0.0;
  if (__builtin_fmax(ad, dabs(r)) >= 0x1p-500) {
    const double rr = dsqrt(__builtin_fma(d, d, r * r));
    t = ddiv(d >= 0.0 ? r : -r, ad + rr);
  }
  const double c = drsqrt(__builtin_fma(t, t, 1.0));
  const double s = t * c;
  const double a1 = __builtin_fma(-t, r, p);
  const double a2 = __builtin_fma(t, r, q);
  Rot2 o;
  const bool keep = a1 >= a2;
  o.l1 = keep ? a1 : a2;
  o.l2 = keep ? a2 : a1;
  o.k11 = keep ? c : s;
  o.k12 = keep ? s : c;
  o.k21 = keep ? -s : c;
  o.k22 = keep ? c : -s;
  return o;
}

// ---------------------------------------------------------------------------
// Fully reduced arrow [[0, 0, b1], [0, -ab, b2], [b1, b2, gb]] (Sec. 1.4):
// spectral function f(x) = x - gb - b1^2/x - b2^2/(x + ab), rightmost zero.
// The arguments carry b1^2 and b2^2.
// ---------------------------------------------------------------------------
struct Arrow1 {
  double b1s, b2s, ab, gb;
};

// x0: positive zero of x - gb - (b1^2 + b2^2)/x (the model from +infinity),
// in the conjugate form when gb < 0.
__device__ __forceinline__ double bg_start(const Arrow1& P) {
  const double H = P.b1s + P.b2s;
  const double g2 = 0.5 * P.gb;
  const double disc = dsqrt(__builtin_fma(g2, g2, H));
  return P.gb >= 0.0 ? g2 + disc : ddiv(H, disc - g2);
}

// One Borges-Gragg step at x.  Sets stop (and returns x) when the stop test
// f/f' <= 2 eps x holds at x, when rounding has reached the root (f <= 0),
// or when the step no longer decreases x.
__device__ __forceinline__ double bg_step(const Arrow1& P, double x, bool& stop) {
  const double p = x + P.ab;
  const double rx = drcp(x);
  const double rp = drcp(p);
  const double q1 = P.b1s * rx;
  const double q2 = P.b2s * rp;
  const double f = ((x - P.gb) - q1) - q2;
  const double fp = __builtin_fma(q1, rx, __builtin_fma(q2, rp, 1.0));
  if (f <= 0.0 || f <= 2.0 * kEps64 * x * fp) {
    stop = true;
    return x;
  }
  // model: w0 = 1 + b2^2 ab / p^3; a = -w0/x; b = f' + f/x
  const double w0 = __builtin_fma(q2 * P.ab, rp * rp, 1.0);
  const double a = -w0 * rx;
  const double b = __builtin_fma(f, rx, fp);
  // increment: a D^2 + b D - f = 0, D = (2f/b) / (1 + sqrt(1 + (2a/b)(2f/b)))
  const double F = ddiv(2.0 * f, b);
  const double D = __builtin_fmax(0.0, __builtin_fma(ddiv(2.0 * a, b), F, 1.0));
  const double dl = ddiv(F, 1.0 + dsqrt(D));
  double xn;
  if (dl <= 0.5 * x) {
    xn = x - dl;
  } else {
    // zero of w0 x^2 - sigma x - w1 = 0 without cancellation
    const double r = x * rp;
    const double w1 = __builtin_fma(P.b2s * r, r * r, P.b1s);
    const double sigma = (w0 * x - w1 * rx) - f;
    const double disc = dsqrt(__builtin_fma(sigma, sigma, 4.0 * w0 * w1));
    xn = sigma >= 0.0 ? ddiv(sigma + disc, 2.0 * w0) : ddiv(2.0 * w1, disc - sigma);
  }
  if (!(xn < x)) {
    stop = true;
    return x;
  }
  return xn;
}

// Newton from the left (Sec. 1.4.2): x0 where f meets -b2^2/(x + ab),
// i.e. x0 = gb/2 + sqrt((gb/2)^2 + b1^2); stop when |f| < 2 eps x.
__device__ __forceinline__ double newton_start(const Arrow1& P) {
  const double g2 = 0.5 * P.gb;
  const double disc = dsqrt(__builtin_fma(g2, g2, P.b1s));
  return P.gb >= 0.0 ? g2 + disc : ddiv(P.b1s, disc - g2);
}

__device__ __forceinline__ double newton_step(const Arrow1& P, double x, bool& stop) {
  const double p = x + P.ab;
  const double rx = drcp(x);
  const double rp = drcp(p);
  const double q1 = P.b1s * rx;
  const double q2 = P.b2s * rp;
  const double f = ((x - P.gb) - q1) - q2;
  if (f >= 0.0 || -f < 2.0 * kEps64 * x) {
    stop = true;
    return x;
  }
  const double fp = __builtin_fma(q1, rx, __builtin_fma(q2, rp, 1.0));
  const double xn = x - ddiv(f, fp);
  if (!(xn > x)) {
    stop = true;
    return x;
  }
  return xn;
}

// Both zeros (mu and nu) in one loop: the two recurrences are independent,
// so their latencies overlap; the loop runs until both have stopped.
__device__ __forceinline__ void zeros_bg(const Arrow1& P1, const Arrow1& P2,
                                         double& x1, double& x2, int& it1, int& it2) {
  x1 = bg_start(P1);
  x2 = bg_start(P2);
  bool s1 = false, s2 = false;
  it1 = 0;
  it2 = 0;
  for (int k = 0; k < kMaxIter; ++k) {
    if (s1 && s2) break;
    if (!s1) { ++it1; x1 = bg_step(P1, x1, s1); }
    if (!s2) { ++it2; x2 = bg_step(P2, x2, s2); }
  }
}

__device__ __forceinline__ void zeros_newton(const Arrow1& P1, const Arrow1& P2,
                                             double& x1, double& x2, int& it1, int& it2) {
  x1 = newton_start(P1);
  x2 = newton_start(P2);
  bool s1 = false, s2 = false;
  it1 = 0;
  it2 = 0;
  for (int k = 0; k < 4 * kMaxIter; ++k) {
    if (s1 && s2) break;
    if (!s1) { ++it1; x1 = newton_step(P1, x1, s1); }
    if (!s2) { ++it2; x2 = newton_step(P2, x2, s2); }
  }
}

// ---------------------------------------------------------------------------
// FP32 Borges-Gragg for the FP32-storage form: the same iteration in single
// precision, stop when f/f' <= 2 eps32 x.
// ---------------------------------------------------------------------------
struct Arrow1f {
  float b1s, b2s, ab, gb;
};

__device__ __forceinline__ float bg_start32(const Arrow1f& P) {
  const float H = P.b1s + P.b2s;
  const float g2 = 0.5f * P.gb;
  const float disc = __builtin_sqrtf(__builtin_fmaf(g2, g2, H));
  return P.gb >= 0.0f ? g2 + disc : H / (disc - g2);
}

__device__ __forceinline__ float bg_step32(const Arrow1f& P, float x, bool& stop, bool& conv) {
  const float p = x + P.ab;
  const float rx = 1.0f / x;
  const float rp = 1.0f / p;
  const float q1 = P.b1s * rx;
  const float q2 = P.b2s * rp;
  const float f = ((x - P.gb) - q1) - q2;
  const float fp = __builtin_fmaf(q1, rx, __builtin_fmaf(q2, rp, 1.0f));
  if (f <= 0.0f || f <= 2.0f * kEps32 * x * fp) {
    stop = true;
    conv = true;
    return x;
  }
  const float w0 = __builtin_fmaf(q2 * P.ab, rp * rp, 1.0f);
  const float a = -w0 * rx;
  const float b = __builtin_fmaf(f, rx, fp);
  const float F = 2.0f * f / b;
  const float D = __builtin_fmaxf(0.0f, __builtin_fmaf(2.0f * a / b, F, 1.0f));
  const float dl = F / (1.0f + __builtin_sqrtf(D));
  float xn;
  if (dl <= 0.5f * x) {
    xn = x - dl;
  } else {
    const float r = x * rp;
    const float w1 = __builtin_fmaf(P.b2s * r, r * r, P.b1s);
    const float sigma = (w0 * x - w1 * rx) - f;
    const float disc = __builtin_sqrtf(__builtin_fmaf(sigma, sigma, 4.0f * w0 * w1));
    xn = sigma >= 0.0f ? (sigma + disc) / (2.0f * w0) : 2.0f * w1 / (disc - sigma);
  }
  if (!(xn < x)) {
    stop = true;
    conv = true;
    return x;
  }
  return xn;
}

// One FP64 Newton step on f from an FP32 zero (Sec. 1.4.2's iteration,
// applied once as a refinement).  Returns the refined zero; sets bad when
// the correction is not small (the FP32 zero was not close).
__device__ __forceinline__ double newton_refine(const Arrow1& P, double x, bool& bad) {
  const double p = x + P.ab;
  const double rx = drcp(x);
  const double rp = drcp(p);
  const double q1 = P.b1s * rx;
  const double q2 = P.b2s * rp;
  const double f = ((x - P.gb) - q1) - q2;
  const double fp = __builtin_fma(q1, rx, __builtin_fma(q2, rp, 1.0));
  const double dx = ddiv(f, fp);
  const double xn = x - dx;
  bad = !(dabs(dx) <= 0x1p-12 * x) || !(xn > 0.0);
  return xn;
}

// ---------------------------------------------------------------------------
// The whole solve.  Input: the 6 unique entries (any finite doubles, or
// not).  Output: lam ascending, V[3r + c] = row r of eigenvector c.
// MODE_F32R selects the FP32 zero finder with FP64 refinement and an FP64
// re-orthogonalisation of the eigenvectors.
// Returns branch | it_mu << 8 | it_nu << 16.
// ---------------------------------------------------------------------------
struct Vec3 {
  double x, y, z;
};

__device__ __forceinline__ Vec3 normalized(Vec3 u) {
  const double r = drsqrt(__builtin_fma(u.x, u.x, __builtin_fma(u.y, u.y, u.z * u.z)));
  return Vec3{u.x * r, u.y * r, u.z * r};
}

__device__ __forceinline__ double dot(const Vec3& a, const Vec3& b) {
  return __builtin_fma(a.x, b.x, __builtin_fma(a.y, b.y, a.z * b.z));
}

__device__ __forceinline__ Vec3 axpy(double s, const Vec3& a, const Vec3& b) {
  return Vec3{__builtin_fma(s, a.x, b.x), __builtin_fma(s, a.y, b.y),
              __builtin_fma(s, a.z, b.z)};
}

template <bool VECS, bool F32R>
__device__ __forceinline__ int solve3(const double (&ain)[6], uint32_t flags,
                                      double (&lam)[3], double (&V)[9]) {
  double a11 = ain[0], a12 = ain[1], a13 = ain[2], a22 = ain[3], a23 = ain[4],
         a33 = ain[5];
  const bool finite = __builtin_isfinite(a11) && __builtin_isfinite(a12) &&
                      __builtin_isfinite(a13) && __builtin_isfinite(a22) &&
                      __builtin_isfinite(a23) && __builtin_isfinite(a33);
  if (!finite) { a11 = a12 = a13 = a22 = a23 = a33 = 0.0; }
  const double m = __builtin_fmax(__builtin_fmax(__builtin_fmax(dabs(a11), dabs(a12)),
                                                 __builtin_fmax(dabs(a13), dabs(a22))),
                                  __builtin_fmax(dabs(a23), dabs(a33)));
  // scale by 2^-e so that max |a_ij| is in [1/2, 1); m == 0 keeps e = 0
  const int e = __builtin_amdgcn_frexp_exp(m);
  a11 = __builtin_amdgcn_ldexp(a11, -e);
  a12 = __builtin_amdgcn_ldexp(a12, -e);
  a13 = __builtin_amdgcn_ldexp(a13, -e);
  a22 = __builtin_amdgcn_ldexp(a22, -e);
  a23 = __builtin_amdgcn_ldexp(a23, -e);
  a33 = __builtin_amdgcn_ldexp(a33, -e);

  // Sec. 1: ordered arrow
  const Rot2 J = rot2(a11, a12, a22);
  const double al1 = J.l1, al2 = J.l2;
  const double be1 = __builtin_fma(J.k11, a13, J.k21 * a23);
  const double be2 = __builtin_fma(J.k12, a13, J.k22 * a23);
  const double ga = a33;

  // Sec. 1.1: h, Givens rotation, deflation test
  const double h = dsqrt(__builtin_fma(be1, be1, be2 * be2));
  const bool diag = (flags & kFlagNoHGuard)
                        ? (h == 0.0)
                        : (h <= kEps64 * (dabs(al1) + dabs(al2) + dabs(ga)));
  const double rh = drcp(h);
  const double cg = be2 * rh;  // G = [[cg, -sg, 0], [sg, cg, 0], [0, 0, 1]]
  const double sg = be1 * rh;
  const double al = al1 - al2;
  const bool small_s = dabs(sg) <= dabs(cg);
  const double s2 = sg * sg, c2 = cg * cg;
  const double d1 = small_s ? __builtin_fma(-al, s2, al1) : __builtin_fma(al, c2, al2);
  const double d2 = small_s ? __builtin_fma(al, s2, al2) : __builtin_fma(-al, c2, al1);
  const double ee = al * sg * cg;
  const double rhs = (flags & kFlagSimplified) ? dabs(al1 + al2) : dabs(d1) + dabs(d2);
  const bool defl = !diag && dabs(ee) <= kEps64 * rhs;

  // Three eigenpairs, two of them known to be ordered: (lx, ux) >= (ly, uy);
  // (lz, uz) anywhere.  Vectors in arrow coordinates.
  // Diagonal arrow: (alpha1, e1), (alpha2, e2), (gamma, e3).
  double lx = al1, ly = al2, lz = ga;
  Vec3 ux{1.0, 0.0, 0.0}, uy{0.0, 1.0, 0.0}, uz{0.0, 0.0, 1.0};
  int branch = diag ? kDiagonal : kDeflated;
  int it1 = 0, it2 = 0;
  if (defl) {
    // accept d1 with G^T e1 = (cg, -sg, 0); solve [[d2, h], [h, gamma]]
    const Rot2 T = rot2(d2, h, ga);
    lx = T.l1;
    ly = T.l2;
    lz = d1;
    if (VECS) {
      ux = Vec3{sg * T.k11, cg * T.k11, T.k21};  // G^T (0, p, q)
      uy = Vec3{sg * T.k12, cg * T.k12, T.k22};
      uz = Vec3{cg, -sg, 0.0};
    }
  } else if (!diag) {
    branch = kReduced;
    // mu: rightmost zero of A - alpha1 I; nu: of P(alpha2 I - A)P
    const double b1s = be1 * be1, b2s = be2 * be2;
    const Arrow1 P1{b1s, b2s, al, ga - al1};
    const Arrow1 P2{b2s, b1s, al, al2 - ga};
    double mu = 0.0, nu = 0.0;
    if (F32R) {
      const Arrow1f Q1{(float)P1.b1s, (float)P1.b2s, (float)P1.ab, (float)P1.gb};
      const Arrow1f Q2{(float)P2.b1s, (float)P2.b2s, (float)P2.ab, (float)P2.gb};
      // the FP32 problem must be representable away from the poles
      bool fb = !(Q1.b1s >= 0x1p-100f && Q1.b2s >= 0x1p-100f && Q1.ab >= 0x1p-60f);
      float y1 = bg_start32(Q1), y2 = bg_start32(Q2);
      bool s1 = false, s2 = false, c1 = false, c2 = false;
      for (int k = 0; k < kMaxIter32; ++k) {
        if (s1 && s2) break;
        if (!s1) { ++it1; y1 = bg_step32(Q1, y1, s1, c1); }
        if (!s2) { ++it2; y2 = bg_step32(Q2, y2, s2, c2); }
      }
      fb = fb || !c1 || !c2 || !(y1 > 0x1p-100f) || !(y2 > 0x1p-100f);
      bool bad1 = false, bad2 = false;
      if (!fb) {
        mu = newton_refine(P1, (double)y1, bad1);
        nu = newton_refine(P2, (double)y2, bad2);
      }
      if (fb || bad1 || bad2) {
        // near-degenerate root isolation falls back to the FP64 zero finder
        int j1, j2;
        zeros_bg(P1, P2, mu, nu, j1, j2);
        it1 += j1;
        it2 += j2;
      }
    } else if (flags & kFlagNewton) {
      zeros_newton(P1, P2, mu, nu, it1, it2);
    } else {
      zeros_bg(P1, P2, mu, nu, it1, it2);
    }
    lx = al1 + mu;                                   // lambda1
    ly = al2 - nu;                                   // lambda3
    lz = __builtin_fmin(__builtin_fmax((ga - mu) + nu, ly), lx);  // lambda2
    if (VECS) {
      const double mua = mu + al, nua = nu + al;
      Vec3 u1{be1 * mua, be2 * mu, mu * mua};
      Vec3 u3{be1 * nu, be2 * nua, -nu * nua};
      Vec3 u2{-be2 * mu * nua, be1 * nu * mua, be1 * be2 * al};
      u1 = normalized(u1);
      u3 = normalized(u3);
      u2 = normalized(u2);
      if (F32R) {
        // one modified Gram-Schmidt pass over (u1, u3, u2)
        u3 = normalized(axpy(-dot(u1, u3), u1, u3));
        u2 = axpy(-dot(u1, u2), u1, u2);
        u2 = normalized(axpy(-dot(u3, u2), u3, u2));
      }
      ux = u1;
      uy = u3;
      uz = u2;
    }
  }

  // Ascending order of (lx >= ly, lz), stable in the listing order x, y, z
  // for ties: when lx == ly the two trade places first, so that equal
  // eigenvalues keep their arrow order (lambda I and 0 give V = I).
  if (lx == ly) {
    const Vec3 tu = ux;
    ux = uy;
    uy = tu;
  }
  double l0, l1, l2;
  Vec3 v0, v1, v2;
  if (lz < ly) {
    l0 = lz; l1 = ly; l2 = lx; v0 = uz; v1 = uy; v2 = ux;
  } else if (lz < lx) {
    l0 = ly; l1 = lz; l2 = lx; v0 = uy; v1 = uz; v2 = ux;
  } else {
    l0 = ly; l1 = lx; l2 = lz; v0 = uy; v1 = ux; v2 = uz;
  }
  lam[0] = __builtin_amdgcn_ldexp(l0, e);
  lam[1] = __builtin_amdgcn_ldexp(l1, e);
  lam[2] = __builtin_amdgcn_ldexp(l2, e);
  if (VECS) {
    // back to A's coordinates: V = diag(J, 1) [v0 v1 v2]
    V[0] = __builtin_fma(J.k11, v0.x, J.k12 * v0.y);
    V[1] = __builtin_fma(J.k11, v1.x, J.k12 * v1.y);
    V[2] = __builtin_fma(J.k11, v2.x, J.k12 * v2.y);
    V[3] = __builtin_fma(J.k21, v0.x, J.k22 * v0.y);
    V[4] = __builtin_fma(J.k21, v1.x, J.k22 * v1.y);
    V[5] = __builtin_fma(J.k21, v2.x, J.k22 * v2.y);
    V[6] = v0.z;
    V[7] = v1.z;
    V[8] = v2.z;
  }
  if (!finite) {
    const double qnan = __builtin_nan("");
    lam[0] = lam[1] = lam[2] = qnan;
    if (VECS) {
#pragma unroll
      for (int k = 0; k < 9; ++k) V[k] = qnan;
    }
    branch = kNonFinite;
  } else if (m == 0.0) {
    branch = kZero;
  }
  return branch | (it1 << 8) | (it2 << 16);
}

}  // namespace syev3
