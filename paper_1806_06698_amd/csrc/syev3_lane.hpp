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
constexpr uint32_t kFlagPaperBG = 8u;
constexpr uint32_t kFlagRefineConverge = 16u;
constexpr uint32_t kFlagNoScale = 32u;

// Arithmetic forms of the solve, a template argument (equal to the dtype
// codes of the interface): FP64 throughout; FP32 storage with FP64
// refinement; FP32 storage with the FP32 zero finder's zeros used as they
// are and no re-orthogonalisation (an ablation of the refinement).  Each
// form is compiled on its own, so no form's kernel holds another's code.
constexpr int kFormF64 = 0;
constexpr int kFormF32R = 1;
constexpr int kFormF32 = 2;

enum Branch : int { kZero = 0, kNonFinite = 1, kDiagonal = 2, kDeflated = 3,
                    kReduced = 4 };

// ---------------------------------------------------------------------------
// Arithmetic primitives.  gfx950's v_rcp_f64, v_rsq_f64 and v_sqrt_f64 are
// accurate to about 2^-24 (measured); Newton-Raphson, Goldschmidt or
// third-order correction steps built from FMAs bring them to the rounding
// level at a fraction of the cost of the IEEE-exact division and square-root
// sequences.  Arguments must be
// normal positive numbers (or, for rcp, any normal non-zero number).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }

// 1/x to ~2^-48 (one Newton-Raphson step).
__device__ __forceinline__ double rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// a/b to about one ulp from a ~2^-47 reciprocal rb of b: quotient plus one
// residual correction.
__device__ __forceinline__ double div_r(double a, double b, double rb) {
  const double q = a * rb;
  return __builtin_fma(__builtin_fma(-b, q, a), rb, q);
}

__device__ __forceinline__ double ddiv(double a, double b) { return div_r(a, b, rcp1(b)); }

// 1/sqrt(x) to about one ulp: v_rsq_f64 and one third-order correction.
// With e = 1 - x y^2, 1/sqrt(x) = y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 +
// 5e^3/16 + ...); for |e| ~ 2^-23 the neglected terms are below 2^-66, and
// e itself is formed by one FMA from x y, so the result carries the
// roundings of the last FMA and of e's product, under one ulp together.
__device__ __forceinline__ double rsqrt2(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-(x * y), y, 1.0);
  return __builtin_fma(y, e * __builtin_fma(e, 0.375, 0.5), y);
}

// sqrt(x) to ~2^-47 for normal x > 0: one Goldschmidt step.
__device__ __forceinline__ double sqrt1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-g, h, 0.5);
  return __builtin_fma(g, r, g);
}

// sqrt(x) to about one ulp: one Goldschmidt step and a residual correction.
__device__ __forceinline__ double sqrt2(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  return __builtin_fma(__builtin_fma(-g, g, x), h, g);
}

// ---------------------------------------------------------------------------
// 2x2 symmetric eigenproblem [[p, r], [r, q]] by one Jacobi rotation, the
// textbook symmetric Schur rotation written so that it comes out ordered.
// With d = (q - p)/2 and u = r / (|d| + hypot(d, r)) (|u| <= 1, the
// rotation's tangent up to sign), the correction u r = r^2 / (|d| + hypot)
// is >= 0 and
//   l1 = max(p, q) + u r,  l2 = min(p, q) - u r  (l1 >= l2),
// with unit eigenvector (c, u c) of l1 when p >= q, else (u c, c),
// c = 1/sqrt(1 + u^2).  (From 2|d| D + r^2 = D^2, D = |d| + hypot(d, r).)
// The eigenvector of l2 is that of l1 turned by 90 degrees, (-k21, k11), so
// J = [[k11, k12], [k21, k22]] is a rotation with J^T B J = diag(l1, l2);
// choosing the order costs two selects, not six.  Ties p == q keep (c, uc).
// ---------------------------------------------------------------------------
struct Rot2 {
  double l1, l2, k11, k12, k21, k22;
};

__device__ __forceinline__ Rot2 rot2(double p, double r, double q) {
  const double d = 0.5 * (q - p);
  const double ad = dabs(d);
  // 2^-1000 under the root keeps it normal and the quotient's divisor at
  // least 2^-500 (d = r = 0 gives u = 0, and r = 0 gives u = 0 exactly), at
  // no cost in the FMA chain; it moves hypot(d, r) by under half an ulp
  // unless d^2 + r^2 < 2^-946, where the block is below 2^-470 of a matrix
  // scaled to max |a_ij| >= 1/2.
  const double rr = sqrt2(__builtin_fma(d, d, __builtin_fma(r, r, 0x1p-1000)));
  const double u = ddiv(r, ad + rr);
  const double c = rsqrt2(__builtin_fma(u, u, 1.0));
  const double s = u * c;
  const bool keep = p >= q;
  Rot2 o;
  o.l1 = __builtin_fma(u, r, __builtin_fmax(p, q));
  o.l2 = __builtin_fma(-u, r, __builtin_fmin(p, q));
  o.k11 = keep ? c : s;
  o.k21 = keep ? s : c;
  o.k12 = -o.k21;
  o.k22 = o.k11;
  return o;
}

// ---------------------------------------------------------------------------
// Fully reduced arrow [[0, 0, b1], [0, -ab, b2], [b1, b2, gb]] (Sec. 1.4):
// spectral function f(x) = x - gb - b1^2/x - b2^2/(x + ab), its rightmost
// zero.  The structure carries b1^2 and b2^2.
// ---------------------------------------------------------------------------
struct Arrow1 {
  double b1s, b2s, ab, gb;
};

// f and f' at x > 0, with b1^2/x and b2^2/(x + ab) to about one ulp from a
// single reciprocal of x (x + ab).
struct Spec {
  double f, fp, rx, rp, q2;
};

__device__ __forceinline__ Spec spec_eval(const Arrow1& P, double x) {
  const double p = x + P.ab;
  const double r = rcp1(x * p);
  const double rx = p * r, rp = x * r;
  const double q1 = div_r(P.b1s, x, rx);
  const double q2 = div_r(P.b2s, p, rp);
  Spec s;
  s.f = ((x - P.gb) - q1) - q2;
  s.fp = __builtin_fma(q1, rx, __builtin_fma(q2, rp, 1.0));
  s.rx = rx;
  s.rp = rp;
  s.q2 = q2;
  return s;
}

// Starting point: an upper bound of the zero, tightened twice.  Each
// bound is the positive zero of a function that lies below f on an interval
// holding the zero (f is increasing, so that zero is right of f's).
//  * U0 = x_inf, the zero of x - gb - (b1^2 + b2^2)/x: the first iterate
//    from +infinity (Sec. 1.4.1); below f because 1/(x + ab) < 1/x.
//  * U_{k+1}: the zero of x - gb - b1^2/x - b2^2 chord_k(x), where chord_k
//    is the chord of the convex 1/(x + ab) over [0, U_k], which lies above
//    it there, so the function lies below f on (0, U_k].  U_{k+1} is in
//    [zero, U_k].  Over a wide interval the chord is about 1/ab, which makes
//    U_1 tight next to the pole at 0, where x_inf can be off by orders of
//    magnitude; narrower intervals tighten it everywhere.
// In a CPU emulation of this arithmetic, two chords leave under 1% of zeros
// needing a third evaluation of f (x_inf alone: 10%); on the GPU two chords
// time best (one chord costs about what it saves in zero-finder trips from
// the third on).  rab = 1/ab.
// quad_zero(c, k, a): positive zero of a x^2 - c x - k (a, k > 0), in the
// form without cancellation.
__device__ __forceinline__ double quad_zero(double c, double k, double a) {
  const double c2 = 0.5 * c;
  const double s = dabs(c2) + sqrt1(__builtin_fma(c2, c2, a * k));
  const bool pos = c >= 0.0;
  return (pos ? s : k) * rcp1(pos ? a : s);
}

constexpr int kChords = 2;
// Chords of the FP32-storage form's start, before its one FP32 step.  In a
// CPU emulation, the Newton step's check then sends 6% of SPD wavefronts
// and 1% of N(0,1) ones to FP64 Borges-Gragg with three chords, 34% and 20%
// with two; iterating FP32 to its own stop test instead takes a second
// FP32 trip in 89% and 99% of wavefronts.
constexpr int kChordsRefine = 3;

__device__ __forceinline__ double bg_start(const Arrow1& P, double rab) {
  double U = quad_zero(P.gb, P.b1s + P.b2s, 1.0);
  const double b2r = P.b2s * rab;
  const double c = P.gb + b2r;
#pragma unroll
  for (int j = 0; j < kChords; ++j) {
    // chord of 1/(x + ab) over [0, U]: 1/ab - x / (ab (U + ab))
    const double k = b2r * rcp1(U + P.ab);
    U = __builtin_fmin(U, quad_zero(c, P.b1s, 1.0 + k));
  }
  return U;
}

// FP32 versions (v_rcp_f32 and v_sqrt_f32 are accurate to about one ulp),
// for the start of the FP64 iteration, for the FP32 start and step that the
// FP32-storage form's Newton step refines, and for the FP32 zero finder of
// the unrefined FP32 ablation.  The FP64 iteration's start only has to be
// close: it converges from either side (bg_step), and a start within about
// 1e-5 of the zero still needs a single evaluation of f in FP64.  FP32 is
// cheaper than the FP64 sequences, and the FP64 path is limited as much by
// the clock the chip sustains under FP64 load as by HBM.
// c0 = gb + b2^2/ab and rab = 1/ab, formed in FP64 and rounded, for the two
// FP32-storage forms' chords and steps (unused by start_point).
struct Arrow1f {
  float b1s, b2s, ab, gb;
  float c0 = 0.0f, rab = 0.0f;
};

__device__ __forceinline__ float quad_zero32(float c, float k, float a) {
  const float c2 = 0.5f * c;
  const float s = __builtin_fabsf(c2) + __builtin_amdgcn_sqrtf(__builtin_fmaf(c2, c2, a * k));
  const bool pos = c >= 0.0f;
  return (pos ? s : k) * __builtin_amdgcn_rcpf(pos ? a : s);
}

// The same for a = 1: positive zero of x^2 - c x - k.
__device__ __forceinline__ float quad_zero32_1(float c, float k) {
  const float c2 = 0.5f * c;
  const float s = __builtin_fabsf(c2) + __builtin_amdgcn_sqrtf(__builtin_fmaf(c2, c2, k));
  return c >= 0.0f ? s : k * __builtin_amdgcn_rcpf(s);
}

// The chord bounds of bg_start in FP32 (CHORDS chords); the chords'
// constant is c0, which FP32 could not form where its terms cancel.
template <int CHORDS>
__device__ __forceinline__ float bg_start32(const Arrow1f& P) {
  float U = quad_zero32(P.gb, P.b1s + P.b2s, 1.0f);
  const float b2r = P.b2s * P.rab;
  const float c = P.c0;
#pragma unroll
  for (int j = 0; j < CHORDS; ++j) {
    const float k = b2r * __builtin_amdgcn_rcpf(U + P.ab);
    U = __builtin_fminf(U, quad_zero32(c, P.b1s, 1.0f + k));
  }
  return U;
}

// Start of the FP64 iteration, in FP32 from the arrow rounded to FP32: a
// bracket [L, U] of the zero, narrowed twice, and its upper end.
//  * L0 = the paper's Newton start (Sec. 1.4.2), the zero of x - gb - b1^2/x
//    (the term b2^2/(x + ab) dropped), a lower bound; U0 = x_inf, an upper
//    bound (see bg_start).
//  * Chord of the convex 1/(x + ab) over [L, U]: it lies above the
//    function there, so x - gb - b1^2/x - b2^2 chord(x) lies below f on
//    [L, U] and its zero is a new upper bound U.
//  * Tangent of 1/(x + ab) at U: it lies below the function everywhere, so
//    the same construction gives a function above f and a new lower bound L.
//  * A second chord over the narrowed [L, U] gives the start (PAIRS such
//    tangent-and-chord pairs after the first chord).
// Each bound is the positive zero of (1 + w) x^2 - c x - b1^2, w the line's
// slope times -b2^2.  The constants c = gb + b2^2 * (the line's value at 0)
// are written as c0 + b2^2 ((value at 0) - 1/ab), with c0 = gb + b2^2/ab
// formed in FP64: for a zero small next to |gb| the terms of c0 nearly
// cancel, while the differences, -L U / ((L + ab)(U + ab) ab) for a chord
// and -t^2 / ((t + ab)^2 ab) for the tangent at t, are accurate in FP32.
// In a CPU emulation this start leaves no zero needing three evaluations of
// f on the SPD and normal workloads (the two chords over [0, U] of bg_start:
// about 1%), and the FP32 arithmetic costs less than the trips it saves.
// It is used when the arrow is well inside FP32's normal range (the squares
// b^2 and a zero b1^2/|gb| that a tiny b1 gives stay normal, b2^2/ab stays
// finite); otherwise the FP64 bounds of bg_start.  The start may fall on
// either side of the zero by FP32 rounding; the step handles both.
// rab = 1/ab.
template <int PAIRS>
__device__ __forceinline__ double start_point(const Arrow1& P, double rab) {
  const Arrow1f Q{(float)P.b1s, (float)P.b2s, (float)P.ab, (float)P.gb};
  const bool ok = Q.b1s >= 0x1p-120f && Q.b2s >= 0x1p-120f && Q.ab >= 0x1p-100f;
  const float c0 = (float)__builtin_fma(P.b2s, rab, P.gb);
  const float rabf = __builtin_amdgcn_rcpf(Q.ab);
  float L = quad_zero32_1(Q.gb, Q.b1s);
  float U = quad_zero32_1(Q.gb, Q.b1s + Q.b2s);
  float rl = __builtin_amdgcn_rcpf(L + Q.ab);
  float ru = __builtin_amdgcn_rcpf(U + Q.ab);
  float w = Q.b2s * rl * ru;
  U = __builtin_fminf(U, quad_zero32(c0 - w * (L * U) * rabf, Q.b1s, 1.0f + w));
#pragma unroll
  for (int j = 0; j < PAIRS; ++j) {
    ru = __builtin_amdgcn_rcpf(U + Q.ab);
    w = Q.b2s * ru * ru;
    L = __builtin_fmaxf(L, quad_zero32(c0 - w * (U * U) * rabf, Q.b1s, 1.0f + w));
    rl = __builtin_amdgcn_rcpf(L + Q.ab);
    w = Q.b2s * rl * ru;
    U = __builtin_fminf(U, quad_zero32(c0 - w * (L * U) * rabf, Q.b1s, 1.0f + w));
  }
  if (ok && U >= 0x1p-124f && U < 0x1p100f) return (double)U;
  return bg_start(P, rab);
}

// Tangent-and-chord pairs of the two starts (mu, nu).
constexpr int kStartPairsMu = 1;
constexpr int kStartPairsNu = 2;


// One Borges-Gragg step from x on either side of the zero (Sec. 1.4.1: the
// iteration converges monotonically from any start in (0, inf)).  Sets stop
// when the returned value is final.
//  * The model phi_j = w0 x - sigma - w1/x matches f, f', f'' at x_j, and
//    f - phi_j = -b2^2 ab (x - x_j)^3 / ((x_j + ab)^3 x (x + ab)) (exactly).
//    Since phi_j(x_new) = 0, f(x_new) = -(w0 - 1) D^3 / (x_new (x_new + ab))
//    with D = x_new - x_j: the iterate stays on the side it started from.
//  * Right of the zero (f > 0) the paper's increment D = 2f / (b + sqrt(b^2
//    + 4af)), a = -w0/x, b = f' + f/x > 0.  When it removes more than half
//    of x, x_new is the model zero itself, w0 x^2 - sigma x - w1 = 0, solved
//    without the cancellation of x - D next to the pole.
//  * Left of it (f < 0), a < 0 makes b^2 + 4af exceed b^2, so the increment
//    has no cancellation as 2f / (b + sqrt(b^2 + 4af)) for b >= 0 nor as
//    (sqrt(b^2 + 4af) - b) / (2a) for b < 0 (b is negative where
//    f/x < -f').
//  * Stop right of the zero: the paper's bound x - zero < f(x)/f'(x) at
//    x_new, with f(x_new) from the closed form and f'(x_new) > f'(x_j) (f'
//    decreases): x_new - zero < (w0 - 1)|D|^3 / (x_new (x_new + ab) f'(x_j)),
//    cubic in the step and checked without evaluating f at x_new.  Left of
//    it: zero - x_new < |f(x_new)| / f'(c) <= |f(x_new)| (f' >= 1, the bound
//    of Sec. 1.4.2).  Either is compared with 2 eps x_new.  A step that
//    rounding at the zero leaves in place, or moves by an ulp the wrong way,
//    passes it too.
// D is computed to about 2^-46: near the zero a cubic step's own error must
// stay below the rounding level.
__device__ __forceinline__ double bg_update(const Arrow1& P, double x, const Spec& s,
                                            bool& stop) {
  const bool left = s.f < 0.0;
  const double w0m1 = (s.q2 * P.ab) * (s.rp * s.rp);
  const double b = __builtin_fma(s.f, s.rx, s.fp);
  // 4 a f, with -4 w0 = -4 w0m1 - 4 in one FMA (bitwise the same product)
  const double a4f = (__builtin_fma(w0m1, -4.0, -4.0) * s.rx) * s.f;
  const double disc = __builtin_fmax(0x1p-1000, __builtin_fma(b, b, a4f));
  const double sq = sqrt1(disc);
  double dl = (2.0 * s.f) * rcp1(b + sq);
  if (b < 0.0) {
    // the conjugate form, only far left of the zero (f/x < -f'); in a
    // branch of its own (the empty asm keeps the compiler from evaluating
    // it on every lane and selecting), as no lane takes it after a start
    // close to the zero
    double bb = b, wm = w0m1;
    asm volatile("" : "+v"(bb), "+v"(wm));
    const double a = -(wm + 1.0) * s.rx;
    dl = (sq - bb) * rcp1(2.0 * a);
  }
  double xn;
  if (dl <= 0.5 * x) {
    xn = x - dl;
  } else {
    // right of the zero, a step of more than half of x: the model zero
    double wm = w0m1;
    asm volatile("" : "+v"(wm));
    const double w0 = wm + 1.0;
    const double r = x * s.rp;
    const double w1 = __builtin_fma(P.b2s * r, r * r, P.b1s);
    const double sigma = (w0 * x - w1 * s.rx) - s.f;
    const double sq2 = sqrt2(__builtin_fma(sigma, sigma, 4.0 * w0 * w1));
    xn = sigma >= 0.0 ? ddiv(sigma + sq2, 2.0 * w0) : ddiv(2.0 * w1, sq2 - sigma);
  }
  // Written as "not above", so that a NaN stops the iteration.  A step
  // that rounding at the zero sends the wrong way is below the rounding
  // level and passes the test.
  const double D = dabs(x - xn);
  if (!(w0m1 * (D * D) * D > 2.0 * kEps64 * (xn * xn) * (xn + P.ab) * (left ? 1.0 : s.fp)))
    stop = true;
  return xn;
}

__device__ __forceinline__ double bg_step(const Arrow1& P, double x, bool& stop) {
  return bg_update(P, x, spec_eval(P, x), stop);
}

// Borges-Gragg as the paper states it, for measuring what the start and the
// stop test above save (flag kFlagPaperBG): the start is x_inf, the first
// iterate from +infinity (Sec. 1.4.1); before each step the iteration stops
// when f/f' < 2 eps x (the paper's test with C = 2), when rounding has
// reached the zero (f <= 0), or when the step no longer decreases x.
// Taking f <= 0 as convergence, it needs a start and steps that do not land
// left of the zero by more than rounding, so its arithmetic is rounded to
// about one ulp (ddiv, sqrt2) in the order of the formulas of Sec. 1.4.1.
// The default finder's 2^-46 primitives would not do here (a start 2^-46
// left of the zero would be returned as it is); they do there, since that
// finder iterates from either side and bounds the new iterate.
// quad_zero_ulp: the positive zero of x^2 - c x - k, k > 0.
__device__ __forceinline__ double quad_zero_ulp(double c, double k) {
  const double c2 = 0.5 * c;
  const double s = dabs(c2) + sqrt2(__builtin_fma(c2, c2, k));
  return c >= 0.0 ? s : ddiv(k, s);
}
// One evaluation of the paper's iteration at x: stop (returning x) when f
// <= 0 or f/f' < 2 eps x, else the next iterate; a step that does not
// decrease x stops with x.
__device__ __forceinline__ double paper_step(const Arrow1& P, double x, bool& stop) {
  const double p = x + P.ab;
  const double q1 = ddiv(P.b1s, x), q2 = ddiv(P.b2s, p);
  const double f = ((x - P.gb) - q1) - q2;
  const double fp = (1.0 + ddiv(q1, x)) + ddiv(q2, p);
  if (!(f > 0.0) || ddiv(f, fp) < 2.0 * kEps64 * x) {
    stop = true;
    return x;
  }
  const double w0 = 1.0 + ddiv(ddiv(q2, p) * P.ab, p);
  const double a = -ddiv(w0, x);
  const double b = fp + ddiv(f, x);
  const double F = ddiv(2.0 * f, b);
  const double D = __builtin_fmax(0.0, 1.0 + ddiv(2.0 * a, b) * F);
  const double dl = ddiv(F, 1.0 + sqrt2(D));
  double xn;
  if (dl <= 0.5 * x) {
    xn = x - dl;
  } else {
    // the zero of the model itself (see bg_update)
    const double r = ddiv(x, p);
    const double w1 = P.b1s + P.b2s * r * r * r;
    const double sigma = (w0 * x - ddiv(w1, x)) - f;
    const double sq = sqrt2(sigma * sigma + 4.0 * w0 * w1);
    xn = sigma >= 0.0 ? ddiv(sigma + sq, 2.0 * w0) : ddiv(2.0 * w1, sq - sigma);
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
  const double disc = sqrt2(__builtin_fma(g2, g2, P.b1s));
  return P.gb >= 0.0 ? g2 + disc : ddiv(P.b1s, disc - g2);
}

__device__ __forceinline__ double newton_step(const Arrow1& P, double x, bool& stop) {
  const Spec s = spec_eval(P, x);
  if (s.f >= 0.0 || -s.f < 2.0 * kEps64 * x) {
    stop = true;
    return x;
  }
  const double xn = x - ddiv(s.f, s.fp);
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
  const double rab = rcp1(P1.ab);  // both problems share abar
  x1 = start_point<kStartPairsMu>(P1, rab);
  x2 = start_point<kStartPairsNu>(P2, rab);
  bool s1 = false, s2 = false;
  it1 = 0;
  it2 = 0;
  for (int k = 0; k < kMaxIter; ++k) {
    if (s1 && s2) break;
    if (!s1) { ++it1; x1 = bg_step(P1, x1, s1); }
    if (!s2) { ++it2; x2 = bg_step(P2, x2, s2); }
  }
}

__device__ __forceinline__ void zeros_bg_paper(const Arrow1& P1, const Arrow1& P2,
                                               double& x1, double& x2, int& it1, int& it2) {
  x1 = quad_zero_ulp(P1.gb, P1.b1s + P1.b2s);
  x2 = quad_zero_ulp(P2.gb, P2.b1s + P2.b2s);
  bool s1 = false, s2 = false;
  it1 = 0;
  it2 = 0;
  for (int k = 0; k < 2 * kMaxIter; ++k) {
    if (s1 && s2) break;
    if (!s1) { ++it1; x1 = paper_step(P1, x1, s1); }
    if (!s2) { ++it2; x2 = paper_step(P2, x2, s2); }
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
// FP32 Borges-Gragg for the unrefined FP32 form (an ablation): the same
// iteration in single precision (v_rcp_f32 and v_sqrt_f32 are accurate to
// about one ulp).
// conv reports a stop by the precision test or at the zero.
// ---------------------------------------------------------------------------
struct Move32 {
  float xn, f, fp, w0m1;
};

__device__ __forceinline__ Move32 bg_move32(const Arrow1f& P, float x) {
  const float p = x + P.ab;
  const float rx = __builtin_amdgcn_rcpf(x);
  const float rp = __builtin_amdgcn_rcpf(p);
  const float q1 = P.b1s * rx;
  const float q2 = P.b2s * rp;
  // For x < ab, f = x - c0 - b1^2/x + b2^2 x / (ab (x + ab)) exactly: with
  // c0 formed in FP64 this keeps a zero that is small next to |gb| (where
  // gb and b2^2/ab nearly cancel) resolvable in FP32.  For x >= ab the
  // usual form has no such cancellation.
  const float f = x < P.ab ? ((x - P.c0) - q1) + q2 * (x * P.rab) : ((x - P.gb) - q1) - q2;
  const float fp = __builtin_fmaf(q1, rx, __builtin_fmaf(q2, rp, 1.0f));
  const float w0m1 = (q2 * P.ab) * (rp * rp);
  const float w0 = w0m1 + 1.0f;
  const float a = -w0 * rx;
  const float b = __builtin_fmaf(f, rx, fp);
  const float disc = __builtin_fmaxf(0.0f, __builtin_fmaf(b, b, 4.0f * a * f));
  const float dl = (2.0f * f) * __builtin_amdgcn_rcpf(b + __builtin_amdgcn_sqrtf(disc));
  float xn;
  if (dl <= 0.5f * x) {
    xn = x - dl;
  } else {
    const float r = x * rp;
    const float w1 = __builtin_fmaf(P.b2s * r, r * r, P.b1s);
    const float sigma = (w0 * x - w1 * rx) - f;
    const float sq = __builtin_amdgcn_sqrtf(__builtin_fmaf(sigma, sigma, 4.0f * w0 * w1));
    xn = sigma >= 0.0f ? (sigma + sq) * __builtin_amdgcn_rcpf(2.0f * w0)
                       : (2.0f * w1) * __builtin_amdgcn_rcpf(sq - sigma);
  }
  return Move32{xn, f, fp, w0m1};
}

// One step of the iteration with its stop tests (the unrefined form).
__device__ __forceinline__ float bg_step32(const Arrow1f& P, float x, bool& stop, bool& conv) {
  const Move32 m = bg_move32(P, x);
  if (m.f <= 0.0f || !(m.xn < x)) {
    // at the zero, or rounding no longer moves x down
    stop = true;
    conv = true;
    return x;
  }
  const float D = x - m.xn;
  if (m.w0m1 * (D * D) * D <= 4.0f * kEps32 * (m.xn * m.xn) * (m.xn + P.ab) * m.fp) {
    stop = true;
    conv = true;
  }
  return m.xn;
}

// One step from an upper bound of the zero with no stop test, for the start
// of the FP32-storage form's Newton step (which checks what it is given); a
// step that does not give a positive iterate leaves x as it is.
__device__ __forceinline__ float bg_once32(const Arrow1f& P, float x) {
  const float xn = bg_move32(P, x).xn;
  return xn > 0.0f ? xn : x;
}

// One FP64 Newton step on f from an FP32 estimate x of the zero (the
// iteration of Sec. 1.4.2, as a refinement).  f is increasing and concave
// with t |f''(t)| <= 2 f'(t), so from a start delta away from the zero, on
// either side, the step lands left of it by at most about delta^2 / x.
//  * bad: a correction above 2^-14 x (or a non-positive iterate); the lane
//    then goes on with FP64 Borges-Gragg steps.  Below it the step leaves
//    at most about 2^-28 x: as the zero is at most 2 ||A||, an eigenvalue
//    off by at most eps32 ||A|| / 16 before rounding.
//  * again: a correction above 2^-22 x; one more step then leaves at most
//    about 2^-56 x.  An eigenvalue formed as a difference (alpha2 - nu, say)
//    can be far smaller than the zero, and its relative error is the
//    zero's error over it: on SPD matrices of condition 1e8, a CPU
//    emulation of this arithmetic puts the smallest eigenvalue's worst
//    relative error at 3e-3 after one step and 1e-6 with the second step
//    where the first moved more than 2^-22 x.
__device__ __forceinline__ double newton_refine(const Arrow1& P, double x, bool& bad,
                                                bool& again) {
  const Spec s = spec_eval(P, x);
  const double dx = ddiv(s.f, s.fp);
  const double xn = x - dx;
  bad = !(dabs(dx) <= 0x1p-14 * x) || !(xn > 0.0);
  again = !(dabs(dx) <= 0x1p-22 * x);
  return xn;
}

// ---------------------------------------------------------------------------
// The whole solve.  Input: the 6 unique entries (any doubles).  Output: lam
// ascending, V[3r + c] = row r of eigenvector c.  kFormF32R takes an FP32
// estimate of each zero, one FP64 Newton step and an FP64
// re-orthogonalisation; kFormF32 uses the zeros of an FP32 Borges-Gragg
// iteration as they are, with the paper's vector formulas (zeros the FP32
// finder cannot give still go to FP64 BG).
// Returns branch | it_mu << 8 | it_nu << 16.  bad is set for a matrix with
// a NaN or infinite entry: its outputs are then meaningless (the solve runs
// on the non-finite values, every loop bounded) and the caller stores NaN in
// their place, in a branch that costs nothing when no lane of the wavefront
// takes it.
// ---------------------------------------------------------------------------
struct Vec3 {
  double x, y, z;
};

__device__ __forceinline__ double dot(const Vec3& a, const Vec3& b) {
  return __builtin_fma(a.x, b.x, __builtin_fma(a.y, b.y, a.z * b.z));
}

__device__ __forceinline__ Vec3 normalized(Vec3 u) {
  const double r = rsqrt2(dot(u, u));
  return Vec3{u.x * r, u.y * r, u.z * r};
}

__device__ __forceinline__ Vec3 axpy(double s, const Vec3& a, const Vec3& b) {
  return Vec3{__builtin_fma(s, a.x, b.x), __builtin_fma(s, a.y, b.y),
              __builtin_fma(s, a.z, b.z)};
}

// max(|x|, |y|) and max(x, y) as one v_max_f64 each.  Written with
// __builtin_fmax, each input loaded from memory first gets a canonicalising
// v_max_f64 x, x of its own (fmax must quiet a signalling NaN), 11
// instructions for the six-entry maximum instead of 5.  The maximum only
// sets the scaling exponent; a NaN input is caught by the finiteness test.
__device__ __forceinline__ double vmax_abs(double x, double y) {
  double r;
  asm("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(x), "v"(y));
  return r;
}
__device__ __forceinline__ double vmax(double x, double y) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
  return r;
}

template <bool VECS, int FORM>
__device__ __forceinline__ int solve3(const double (&ain)[6], uint32_t flags,
                                      double (&lam)[3], double (&V)[9], bool& bad) {
  double a11 = ain[0], a12 = ain[1], a13 = ain[2], a22 = ain[3], a23 = ain[4],
         a33 = ain[5];
  const bool finite = __builtin_isfinite(a11) && __builtin_isfinite(a12) &&
                      __builtin_isfinite(a13) && __builtin_isfinite(a22) &&
                      __builtin_isfinite(a23) && __builtin_isfinite(a33);
  // Kept as a word from here on: left as a condition the compiler re-derives
  // it at the stores from the six inputs, holding them through the solve.
  uint32_t badw = finite ? 0u : 1u;
  asm volatile("" : "+v"(badw));
  bad = badw != 0u;
  const double m = vmax(vmax(vmax_abs(a11, a12), vmax_abs(a13, a22)), vmax_abs(a23, a33));
  // scale by 2^-e so that max |a_ij| is in [1/2, 1); m == 0 keeps e = 0
  // (kFlagNoScale, a uniform flag: e = 0, the unscaled matrix)
  // (The flags are the same for every lane: their alternatives are taken in
  // uniform branches, which the empty asm keeps the compiler from turning
  // into per-lane selects that every lane would pay for.)
  int e = __builtin_amdgcn_frexp_exp(m);
  if (flags & kFlagNoScale) {
    asm volatile("");
    e = 0;
  }
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

  // Sec. 1.1: h = ||beta||, the Givens rotation G and the deflation test.
  // h <= eps (|alpha1| + |alpha2| + |gamma|) is tested as h^2 <= (eps ...)^2.
  const double hh = __builtin_fma(be1, be1, be2 * be2);
  const double tol_h = kEps64 * (dabs(al1) + dabs(al2) + dabs(ga));
  bool diag;
  if (flags & kFlagNoHGuard) {
    asm volatile("");
    diag = hh == 0.0;
  } else {
    diag = !(hh > tol_h * tol_h);
  }
  const double al = al1 - al2;
  // The test |e| <= eps (|d1| + |d2|) on G A G^T, whose off-diagonal entry
  // is e = alpha sg cg and whose diagonal is d1 = alpha1 cg^2 + alpha2 sg^2,
  // d2 = alpha1 sg^2 + alpha2 cg^2 (sg = beta1/h, cg = beta2/h), taken
  // times h^2: |alpha beta1 beta2| <= eps (|alpha1 beta2^2 + alpha2 beta1^2|
  // + |alpha1 beta1^2 + alpha2 beta2^2|).  It needs no root or quotient, so
  // G itself is formed only on lanes that deflate.  The exact beta- and
  // combo-deflations (beta1, beta2 or alpha zero) make the left side zero.
  const double b1s = be1 * be1, b2s = be2 * be2;
  const double ee = al * be1 * be2;
  double rhs;
  if (flags & kFlagSimplified) {
    asm volatile("");
    rhs = dabs(al1 + al2) * hh;
  } else {
    rhs = dabs(__builtin_fma(al1, b2s, al2 * b1s)) + dabs(__builtin_fma(al1, b1s, al2 * b2s));
  }
  const bool defl = !diag && dabs(ee) <= kEps64 * rhs;

  double l0, l1, l2;  // ascending
  Vec3 v0, v1, v2;    // their eigenvectors, arrow coordinates
  int branch, it1 = 0, it2 = 0;
  if (diag || defl) {
    // Two pairs known ordered, (lx, ux) >= (ly, uy); (lz, uz) anywhere.
    double lx, ly, lz;
    Vec3 ux, uy, uz;
    if (defl) {
      // accept d1 with G^T e1 = (cg, -sg, 0); solve [[d2, h], [h, gamma]]
      branch = kDeflated;
      const double rh = rsqrt2(hh);
      const double h = hh * rh;
      const double cg = be2 * rh;  // G = [[cg, -sg, 0], [sg, cg, 0], [0, 0, 1]]
      const double sg = be1 * rh;
      // d1, d2 with the smaller correction: bitwise exact for the beta- and
      // combo-deflations (sg or cg zero, or alpha zero)
      const bool small_s = dabs(sg) <= dabs(cg);
      const double s2 = sg * sg, c2 = cg * cg;
      const double d1 = small_s ? __builtin_fma(-al, s2, al1) : __builtin_fma(al, c2, al2);
      const double d2 = small_s ? __builtin_fma(al, s2, al2) : __builtin_fma(-al, c2, al1);
      const Rot2 T = rot2(d2, h, ga);
      lx = T.l1;
      ly = T.l2;
      lz = d1;
      ux = Vec3{sg * T.k11, cg * T.k11, T.k21};  // G^T (0, p, q)
      uy = Vec3{sg * T.k12, cg * T.k12, T.k22};
      uz = Vec3{cg, -sg, 0.0};
    } else {
      // diagonal arrow: (alpha1, e1), (alpha2, e2), (gamma, e3)
      branch = kDiagonal;
      lx = al1;
      ly = al2;
      lz = ga;
      ux = Vec3{1.0, 0.0, 0.0};
      uy = Vec3{0.0, 1.0, 0.0};
      uz = Vec3{0.0, 0.0, 1.0};
    }
    // Ascending, stable in the listing order x, y, z for ties: when
    // lx == ly the two trade vectors first, so equal eigenvalues keep their
    // arrow order (lambda I and 0 give V = I).
    if (lx == ly) {
      const Vec3 tu = ux;
      ux = uy;
      uy = tu;
    }
    if (lz < ly) {
      l0 = lz; l1 = ly; l2 = lx; v0 = uz; v1 = uy; v2 = ux;
    } else if (lz < lx) {
      l0 = ly; l1 = lz; l2 = lx; v0 = uy; v1 = uz; v2 = ux;
    } else {
      l0 = ly; l1 = lx; l2 = lz; v0 = uy; v1 = ux; v2 = uz;
    }
  } else {
    branch = kReduced;
    // mu: rightmost zero of A - alpha1 I; nu: of P(alpha2 I - A)P
    const Arrow1 P1{b1s, b2s, al, ga - al1};
    const Arrow1 P2{b2s, b1s, al, al2 - ga};
    double mu = 0.0, nu = 0.0;
    if (FORM == kFormF32R) {
      // FP32 storage with FP64 refinement: in FP32, the three-chord upper
      // bound of the zero and one Borges-Gragg step from it; then an FP64
      // Newton step (Sec. 1.4.2), which squares the relative error, and a
      // second one where the first moved the zero by more than 2^-22.
      const double rab = rcp1(P1.ab);  // both problems share abar
      const Arrow1f Q1{(float)P1.b1s, (float)P1.b2s, (float)P1.ab, (float)P1.gb,
                       (float)__builtin_fma(P1.b2s, rab, P1.gb), (float)rab};
      const Arrow1f Q2{(float)P2.b1s, (float)P2.b2s, (float)P2.ab, (float)P2.gb,
                       (float)__builtin_fma(P2.b2s, rab, P2.gb), (float)rab};
      const float y1 = bg_once32(Q1, bg_start32<kChordsRefine>(Q1));
      const float y2 = bg_once32(Q2, bg_start32<kChordsRefine>(Q2));
      double x1 = (double)y1, x2 = (double)y2;
      // the FP32 problem must be representable away from the poles
      if (!(Q1.b1s >= 0x1p-100f && Q1.b2s >= 0x1p-100f && Q1.ab >= 0x1p-60f &&
            y1 > 0x1p-100f && y2 > 0x1p-100f)) {
        // no usable FP32 start: the FP64 bounds of bg_start, too far for
        // the Newton step, whose check then hands them to FP64 Borges-Gragg
        // (a branch of its own, which the empty asm keeps from being
        // evaluated on every lane)
        asm volatile("");
        x1 = bg_start(P1, rab);
        x2 = bg_start(P2, rab);
      }
      bool bad1, bad2, again1, again2, unused;
      mu = newton_refine(P1, x1, bad1, again1);
      nu = newton_refine(P2, x2, bad2, again2);
      it1 = it2 = 2;  // one FP32 and one FP64 evaluation of f per root
      if (flags & kFlagRefineConverge) bad1 = bad2 = true;
      // the second Newton step, per root, where the first moved the zero by
      // more than 2^-22 of it (and the lane is not going on to Borges-Gragg);
      // branches of their own (the empty asm keeps the compiler from
      // evaluating them on every lane), skipped by wavefronts none of whose
      // lanes need them
      if (again1 && !bad1) {
        asm volatile("");
        ++it1;
        mu = newton_refine(P1, mu, unused, unused);
      }
      if (again2 && !bad2) {
        asm volatile("");
        ++it2;
        nu = newton_refine(P2, nu, unused, unused);
      }
      if (bad1 || bad2) {
        // The start was too far for one Newton step (a zero FP32 does not
        // resolve, or an arrow outside FP32's range), or every root
        // converges (kFlagRefineConverge): continue with FP64 Borges-Gragg
        // steps.  f is concave, so the Newton iterate lies left of the zero
        // when the start is right of it; when it is not positive the start
        // is taken instead.
        if (bad1 && !(mu > 0.0)) mu = x1;
        if (bad2 && !(nu > 0.0)) nu = x2;
        bool s1 = !bad1, s2 = !bad2;
        for (int k = 0; k < kMaxIter; ++k) {
          if (s1 && s2) break;
          if (!s1) { ++it1; mu = bg_step(P1, mu, s1); }
          if (!s2) { ++it2; nu = bg_step(P2, nu, s2); }
        }
      }
    } else if (FORM == kFormF32) {
      // The unrefined FP32 ablation: Borges-Gragg in FP32 from the FP32
      // two-chord start, its zeros used as they are.
      const double rab = rcp1(P1.ab);  // both problems share abar
      const Arrow1f Q1{(float)P1.b1s, (float)P1.b2s, (float)P1.ab, (float)P1.gb,
                       (float)__builtin_fma(P1.b2s, rab, P1.gb), (float)rab};
      const Arrow1f Q2{(float)P2.b1s, (float)P2.b2s, (float)P2.ab, (float)P2.gb,
                       (float)__builtin_fma(P2.b2s, rab, P2.gb), (float)rab};
      // the FP32 problem must be representable away from the poles
      bool fb = !(Q1.b1s >= 0x1p-100f && Q1.b2s >= 0x1p-100f && Q1.ab >= 0x1p-60f);
      float y1 = bg_start32<kChords>(Q1), y2 = bg_start32<kChords>(Q2);
      bool s1 = false, s2 = false, c1 = false, c2 = false;
      for (int k = 0; k < kMaxIter32; ++k) {
        if (s1 && s2) break;
        if (!s1) { ++it1; y1 = bg_step32(Q1, y1, s1, c1); }
        if (!s2) { ++it2; y2 = bg_step32(Q2, y2, s2, c2); }
      }
      fb = fb || !c1 || !c2 || !(y1 > 0x1p-100f) || !(y2 > 0x1p-100f);
      if (fb) {
        // no usable FP32 zero: the FP64 zero finder from its own start
        int j1, j2;
        zeros_bg(P1, P2, mu, nu, j1, j2);
        it1 += j1;
        it2 += j2;
      } else {
        mu = (double)y1;
        nu = (double)y2;
      }
    } else if (flags & kFlagNewton) {
      zeros_newton(P1, P2, mu, nu, it1, it2);
    } else if (flags & kFlagPaperBG) {
      zeros_bg_paper(P1, P2, mu, nu, it1, it2);
    } else {
      zeros_bg(P1, P2, mu, nu, it1, it2);
    }
    // lambda3 <= lambda2 <= lambda1; lambda2 by the trace identity
    l2 = al1 + mu;
    l0 = al2 - nu;
    l1 = __builtin_fmin(__builtin_fmax((ga - mu) + nu, l0), l2);
    if (VECS) {
      const double mua = mu + al, nua = nu + al;
      const Vec3 u1{be1 * mua, be2 * mu, mu * mua};
      const Vec3 u3{be1 * nu, be2 * nua, -nu * nua};
      if (FORM == kFormF32R) {
        // one Gram-Schmidt re-orthogonalisation of u3 against the unit u1,
        // before u3 is normalised
        v2 = normalized(u1);
        v0 = normalized(axpy(-dot(v2, u3), v2, u3));
      } else {
        v2 = normalized(u1);
        v0 = normalized(u3);
      }
      if (FORM == kFormF32) {
        // the ablation keeps the paper's formula for u2
        const Vec3 u2{-be2 * mu * nua, be1 * nu * mua, be1 * be2 * al};
        v1 = normalized(u2);
      } else {
        // The paper's u2 is (mu + nu + abar) (u1 x u3), a positive multiple
        // of the cross product (expand u1 x u3 and factor), so the middle
        // vector is taken as the cross product of the two unit vectors:
        // orthogonal to both by construction, and 15 operations cheaper
        // than forming and normalising u2.
        v1 = Vec3{__builtin_fma(v2.y, v0.z, -v2.z * v0.y), __builtin_fma(v2.z, v0.x, -v2.x * v0.z),
                  __builtin_fma(v2.x, v0.y, -v2.y * v0.x)};
      }
    }
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
    branch = kNonFinite;
  } else if (m == 0.0) {
    branch = kZero;
  }
  return branch | (it1 << 8) | (it2 << 16);
}

}  // namespace syev3
