// Host-only check of the C API's argument validation (include/syev3.h),
// built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer by
// test_api_sanitizers.py.  The library's API source is compiled in with the
// two launchers replaced by stubs that record their arguments, so no GPU is
// touched and every pointer is a number that is never dereferenced.
//
// Randomized calls of every entry point must
//   * return SYEV3_OK exactly when the stub launched (n > 0) or n == 0;
//   * when accepted, hand the launcher the caller's arguments (ld resolved);
//   * agree with a model of the documented rules, for sizes far from the
//     library's limit (valid arguments accepted, invalid ones rejected with a
//     documented error code);
//   * raise no sanitizer report (the size and span arithmetic of the checks).
#include "syev3_api.cpp"

#include <cstdio>
#include <cstdlib>
#include <random>

namespace {
struct Launch {
  int count = 0;
  int64_t n, ld, ldl, ldv;
  int layout, dtype;
  const void* A;
  void* lam;
  void* V;
  uint32_t flags;
  int32_t* info;
} g_launch;
}  // namespace

namespace syev3 {
hipError_t launch_batched(int64_t n, const void* A, Strides ld, int layout, void* lambda,
                          void* V, int dtype, uint32_t flags, int32_t* info, hipStream_t) {
  g_launch = Launch{g_launch.count + 1, n, ld.a, ld.l, ld.v, layout, dtype, A, lambda, V,
                    flags, info};
  return hipSuccess;
}
hipError_t launch_stream_probe(int64_t n, const void* A, void* lambda, void* V, int dtype,
                               uint32_t, hipStream_t) {
  g_launch = Launch{g_launch.count + 1, n, n, n, n, 0, dtype, A, lambda, V, 0u, nullptr};
  return hipSuccess;
}
}  // namespace syev3

// The API clears any stale HIP error before it launches; there is no HIP
// runtime in this test.
extern "C" hipError_t hipGetLastError(void) { return hipSuccess; }

namespace {

typedef unsigned __int128 u128;

struct Span {
  u128 lo, hi;
};
bool hits(Span a, Span b) { return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi; }
Span span_of(uint64_t p, int64_t n, int64_t ld, int layout, int planes, int es) {
  if (!p || n == 0) return Span{p, p};
  const u128 elems = layout == 0 ? (u128)(planes - 1) * (u128)ld + (u128)n
                                 : (u128)planes * (u128)n;
  return Span{p, (u128)p + elems * (u128)es};
}

// The documented rules, for |n|, |ld| < 2^40 (far from the size limit).
bool model_valid(int64_t n, uint64_t A, int64_t ld, int64_t ldl, int64_t ldv, int layout,
                 uint64_t lam, uint64_t V, int dtype, uint32_t flags, uint64_t info,
                 bool allow_inplace) {
  if (dtype < 0 || dtype > 2) return false;
  if (flags & ~63u) return false;
  if ((flags & 12u) && dtype != 0) return false;  // Newton, paper BG: FP64 only
  if ((flags & 4u) && (flags & 8u)) return false;  // not both
  if ((flags & 16u) && dtype != 1) return false;  // converge: FP32 refined only
  if (layout < 0 || layout > 2) return false;
  if (n < 0) return false;
  if (layout == 0) {
    if (ld == 0) ld = n;
    if (ldl == 0) ldl = n;
    if (ldv == 0) ldv = n;
    if (ld < n || ldl < n || ldv < n) return false;
  } else if (ld != 0 || ldl != 0 || ldv != 0) {
    return false;
  }
  if (n == 0) return true;
  if (!A || !lam) return false;
  const int es = dtype == 0 ? 8 : 4;
  const Span a = span_of(A, n, ld, layout, layout == 2 ? 9 : 6, es);
  const Span l = span_of(lam, n, ldl, layout, 3, es);
  const Span v = span_of(V, n, ldv, layout, 9, es);
  const bool inplace = allow_inplace && layout == 2 && V == A;
  if (hits(a, l) || (!inplace && hits(a, v)) || hits(l, v)) return false;
  if (info) {
    const Span f{info, (u128)info + (u128)n * 4};
    if (hits(f, a) || hits(f, l) || hits(f, v)) return false;
  }
  return true;
}

int failures = 0;
long long n_launched = 0, n_rejected = 0, n_noop = 0, n_modelled = 0;
void fail(const char* what, long long i) {
  if (failures++ < 20) std::fprintf(stderr, "case %lld: %s\n", i, what);
}

}  // namespace

int main(int argc, char** argv) {
  const long long cases = argc > 1 ? std::atoll(argv[1]) : 200000;
  std::mt19937_64 rng(12345);
  auto pick = [&](std::initializer_list<int64_t> v) {
    return *(v.begin() + rng() % v.size());
  };
  const int64_t big = INT64_MAX;
  for (long long i = 0; i < cases; ++i) {
    const bool far = rng() % 4 != 0;  // sizes far from the limit (model applies)
    int64_t n = far ? pick({-3, 0, 1, 2, 255, 256, 257, 1000, 65536 + 7, 1 << 20})
                    : pick({big, big - 1, big / 2, big / 144, big / 143, (int64_t)1 << 40,
                            ((int64_t)1 << 32) * 256, INT64_MIN, -1});
    auto draw_ld = [&]() {
      int64_t ld = 0;
      switch (rng() % 5) {
        case 0: ld = 0; break;
        case 1: ld = n; break;
        case 2: ld = n > big - 5 ? n : n + (int64_t)(rng() % 5); break;
        case 3: ld = n == INT64_MIN ? n : n - 1; break;
        default: ld = far ? (int64_t)(rng() % 3000000) : pick({big, big / 8, INT64_MIN});
      }
      if (far && (ld > ((int64_t)1 << 40) || ld < -((int64_t)1 << 40))) ld = 0;
      return ld;
    };
    // one stride for every array, and two more for the strided entry point
    const int64_t ld = draw_ld(), ld_l = draw_ld(), ld_v = draw_ld();
    const int layout = (int)pick({0, 0, 1, 2, -1, 3});
    const int dtype = (int)pick({0, 0, 1, 2, -1, 3});
    const uint32_t flags = (uint32_t)pick({0, 0, 0, 1, 2, 4, 7, 8, 12, 15, 16, 17, 19, 31, 32, 33, 63, 64,
                                           0x7fffffff});
    // addresses: separate regions or overlapping ones, 0 for NULL
    const uint64_t base = (uint64_t)1 << 44;
    auto addr = [&](int slot) -> uint64_t {
      switch (rng() % 8) {
        case 0: return 0;
        case 1: return base + (uint64_t)(rng() % 4096) * 8;   // near the others
        default: return base + ((uint64_t)slot << 40) + (uint64_t)(rng() % 64) * 8;
      }
    };
    uint64_t A = addr(0), L = addr(1), V = addr(2), F = rng() % 3 == 0 ? addr(3) : 0;
    const int which = (int)(rng() % 6);
    if (which == 3 && rng() % 2) V = A;  // in place
    g_launch.count = 0;
    int rc;
    bool allow_inplace = true;
    uint64_t info = 0;
    int64_t exp_ld = ld, exp_ldl = ld, exp_ldv = ld;
    int exp_layout = layout;
    uint32_t exp_flags = flags;
    int64_t mn = n;
    int mlayout = layout;
    uint32_t mflags = flags;
    switch (which) {
      case 0:  // batched_syev3: SoA, ld = n, no flags
        rc = batched_syev3(n, (void*)A, (void*)L, (void*)V, dtype, nullptr);
        exp_ld = 0; exp_layout = 0; exp_flags = 0; mlayout = 0; mflags = 0;
        break;
      case 1:
        rc = batched_syev3_ex(n, (void*)A, ld, layout, (void*)L, (void*)V, dtype, flags, nullptr);
        break;
      case 2:
        info = F;
        rc = batched_syev3_info(n, (void*)A, ld, layout, (void*)L, (void*)V, dtype, flags,
                                (int32_t*)info, nullptr);
        break;
      case 3:  // in place: AoS9, V = A
        rc = batched_syev3_inplace(n, (void*)A, (void*)L, dtype, nullptr);
        V = A; exp_ld = 0; exp_layout = 2; exp_flags = 0; mlayout = 2; mflags = 0;
        break;
      case 5:  // SoA with a stride per array
        rc = batched_syev3_strided(n, (void*)A, ld, (void*)L, ld_l, (void*)V, ld_v, dtype, flags,
                                   nullptr);
        exp_ldl = ld_l; exp_ldv = ld_v; exp_layout = 0; mlayout = 0;
        allow_inplace = false;
        break;
      default:
        rc = syev3_stream_reference(n, (void*)A, (void*)L, (void*)V, dtype, nullptr);
        exp_ld = 0; exp_layout = 0; exp_flags = 0; mlayout = 0; mflags = 0;
        allow_inplace = false;
        break;
    }
    const bool strided_args = which == 1 || which == 2 || which == 5;
    if (which != 5) exp_ldl = exp_ldv = exp_ld;  // one stride for all arrays
    const int64_t mld = strided_args ? ld : 0;
    const int64_t mldl = which == 5 ? ld_l : mld, mldv = which == 5 ? ld_v : mld;
    // accepted <=> launched (n > 0) or a no-op (n == 0)
    const bool launched = g_launch.count == 1;
    n_launched += launched;
    n_rejected += rc != SYEV3_OK;
    n_noop += rc == SYEV3_OK && !launched;
    n_modelled += far;
    if (rc == SYEV3_OK && mn > 0 && !launched) fail("accepted without a launch", i);
    if (rc == SYEV3_OK && mn == 0 && launched) fail("n == 0 launched", i);
    if (rc != SYEV3_OK && launched) fail("rejected but launched", i);
    if (rc != SYEV3_OK && (rc > -1 || rc < -7 || rc == SYEV3_E_HIP)) fail("undocumented code", i);
    if (launched) {
      auto want = [&](int64_t s) { return exp_layout == 0 ? (s == 0 ? mn : s) : 0; };
      const int64_t want_ld = want(exp_ld);
      if (g_launch.n != mn || (uint64_t)g_launch.A != A || (uint64_t)g_launch.lam != L ||
          (uint64_t)g_launch.V != V || g_launch.dtype != dtype)
        fail("launcher got other pointers or sizes", i);
      if (which != 4 && (g_launch.ld != want_ld || g_launch.ldl != want(exp_ldl) ||
                         g_launch.ldv != want(exp_ldv) || g_launch.layout != exp_layout ||
                         (g_launch.flags & 63u) != exp_flags || (uint64_t)g_launch.info != info))
        fail("launcher got another layout, stride, flags or info", i);
    }
    if (far) {
      const bool ok = model_valid(mn, A, mld, mldl, mldv, mlayout, L, V, dtype, mflags, info,
                                  allow_inplace);
      if (ok != (rc == SYEV3_OK)) fail(ok ? "valid call rejected" : "invalid call accepted", i);
    }
  }
  std::printf("%lld cases (%lld launched, %lld rejected, %lld no-op; %lld against the model), "
              "%d failures\n", cases, n_launched, n_rejected, n_noop, n_modelled, failures);
  return failures ? 1 : 0;
}
