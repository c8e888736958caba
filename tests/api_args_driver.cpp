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
#include <vector>

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
// the no-allocation segment call: a copy of the table it would upload
int g_seg_launches = 0;
TickTable g_seg_seen;
hipError_t launch_segments_noalloc(const TickTable* t, hipStream_t) {
  ++g_seg_launches;
  g_seg_seen.nseg = t->nseg;
  g_seg_seen.total_tiles = t->total_tiles;
  for (int i = 0; i < t->nseg && i < kMaxSegmentsPerTick; ++i) g_seg_seen.seg[i] = t->seg[i];
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

// syev3_solve_segments_noalloc: random lists of segments (mostly short, so
// the model's all-pairs alias test stays cheap; now and then the longest
// accepted and one more).  Accepted exactly when every segment passes the
// batched rules (SoA, outputs at stride n, FP64 or FP32-refined only) and
// no output of any segment overlaps an input or output of another; then the
// launcher gets the non-empty segments in order with their tile ranges.
long long n_seg_launched = 0, n_seg_rejected = 0;
long long segment_cases(std::mt19937_64& rng, long long cases) {
  auto pick = [&](std::initializer_list<int64_t> v) { return *(v.begin() + rng() % v.size()); };
  const uint64_t base = (uint64_t)1 << 44;
  static syev3_segment segs[SYEV3_SEGMENTS_MAX + 1];
  for (long long i = 0; i < cases; ++i) {
    const int roll = (int)(rng() % 100);
    const int nseg = roll == 0 ? SYEV3_SEGMENTS_MAX : roll == 1 ? SYEV3_SEGMENTS_MAX + 1
                   : roll == 2 ? -1 : (int)(rng() % 9);
    const int made = nseg < 0 ? 0 : nseg;
    // the long lists, and half of the short ones: valid segments in separate
    // regions (accepted: their tables are checked)
    const bool big = nseg > 16 || rng() % 2 == 0;
    for (int k = 0; k < made; ++k) {
      syev3_segment& q = segs[k];
      q.n = nseg > 16 ? pick({0, 1, 300}) : big ? pick({0, 1, 255, 256, 257, 1000})
                                           : pick({-2, 0, 1, 255, 256, 257, 1000});
      q.lda = big ? 0 : pick({0, 0, q.n, q.n + 3, q.n - 1});
      q.dtype = big ? (int32_t)(rng() % 2) : (int32_t)pick({0, 0, 1, 1, 2, -1});
      q.flags = big ? 0u : (uint32_t)pick({0, 0, 0, 1, 4, 16, 32, 64});
      // each segment in its own region, or (short lists) near or inside
      // another segment's arrays; 0 for NULL now and then
      auto addr = [&](int slot) -> uint64_t {
        const uint64_t own = base + ((uint64_t)(4 * k + slot) << 32);
        if (big) return own;
        switch (rng() % 8) {
          case 0: return 0;
          case 1: return base + ((uint64_t)(rng() % 32) << 32) + (uint64_t)(rng() % 2048) * 8;
          case 2:
          case 3: {
            // into an array of an earlier segment
            if (k == 0) return own;
            const syev3_segment& e = segs[rng() % k];
            const uint64_t p = (uint64_t)(rng() % 3 == 0 ? e.A : rng() % 2 ? (const void*)e.lambda
                                                                            : (const void*)e.V);
            return p ? p + (uint64_t)(rng() % 64) * 8 : own;
          }
          default: return own + (uint64_t)(rng() % 16) * 8;
        }
      };
      q.A = (const void*)addr(0);
      q.lambda = (void*)addr(1);
      q.V = rng() % 5 == 0 ? nullptr : (void*)addr(2);
    }
    syev3::g_seg_launches = 0;
    const int rc = syev3_solve_segments_noalloc(nseg, nseg >= 0 ? segs : nullptr, nullptr);
    // the model
    bool ok = nseg >= 0 && nseg <= SYEV3_SEGMENTS_MAX;
    std::vector<Span> outs, ins;
    for (int k = 0; ok && k < nseg; ++k) {
      const syev3_segment& q = segs[k];
      if (q.dtype != 0 && q.dtype != 1) ok = false;
      else if (!model_valid(q.n, (uint64_t)q.A, q.lda, 0, 0, 0, (uint64_t)q.lambda,
                            (uint64_t)q.V, q.dtype, q.flags, 0, false)) ok = false;
      if (!ok || q.n <= 0) continue;
      const int es = q.dtype == 0 ? 8 : 4;
      ins.push_back(span_of((uint64_t)q.A, q.n, q.lda ? q.lda : q.n, 0, 6, es));
      outs.push_back(span_of((uint64_t)q.lambda, q.n, q.n, 0, 3, es));
      if (q.V) outs.push_back(span_of((uint64_t)q.V, q.n, q.n, 0, 9, es));
    }
    for (size_t a = 0; ok && a < outs.size(); ++a) {
      for (size_t b = a + 1; ok && b < outs.size(); ++b) ok = !hits(outs[a], outs[b]);
      for (size_t b = 0; ok && b < ins.size(); ++b) ok = !hits(outs[a], ins[b]);
    }
    n_seg_rejected += rc != SYEV3_OK;
    n_seg_launched += syev3::g_seg_launches;
    if (ok != (rc == SYEV3_OK)) fail(ok ? "valid segment call rejected" : "invalid segment call accepted", i);
    if (rc != SYEV3_OK && syev3::g_seg_launches) fail("segment call rejected but launched", i);
    if (rc != SYEV3_OK && (rc > -1 || rc < -13 || rc == SYEV3_E_HIP))
      fail("undocumented code from the segment call", i);
    if (rc == SYEV3_OK) {
      int want = 0;
      int64_t tiles = 0;
      bool same = true;
      for (int k = 0; k < nseg; ++k) {
        const syev3_segment& q = segs[k];
        if (q.n == 0) continue;
        const syev3::Segment& g = syev3::g_seg_seen.seg[want++];
        same = same && g.A == q.A && g.lambda == q.lambda && g.V == q.V && g.n == q.n &&
               g.lda == (q.lda ? q.lda : q.n) && g.tile_begin == tiles && g.dtype == q.dtype &&
               g.flags == q.flags;
        tiles += (q.n + 255) / 256;
      }
      if (syev3::g_seg_launches != (tiles > 0 ? 1 : 0)) fail("segment launch count", i);
      if (tiles > 0 && (!same || syev3::g_seg_seen.nseg != want ||
                        syev3::g_seg_seen.total_tiles != tiles))
        fail("segment table differs from the call", i);
    }
  }
  return cases;
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
  const int case_failures = failures;
  const long long seg_cases = segment_cases(rng, cases / 10);
  std::printf("%lld cases (%lld launched, %lld rejected, %lld no-op; %lld against the model), "
              "%d failures; %lld segment calls (%lld launched, %lld rejected), %d failures\n",
              cases, n_launched, n_rejected, n_noop, n_modelled, case_failures, seg_cases,
              n_seg_launched, n_seg_rejected, failures - case_failures);
  return failures ? 1 : 0;
}
