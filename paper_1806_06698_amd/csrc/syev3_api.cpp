// syev3_api.cpp -- C ABI of the batched solver: argument checks, then one
// kernel launch on the caller's stream.  See include/syev3.h.
#include "syev3.h"

#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "syev3_internal.hpp"

namespace {

struct Range {
  uintptr_t lo, hi;  // [lo, hi) in bytes; hi == lo for an absent array
};

bool overlap(const Range& a, const Range& b) {
  return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi;
}

// Bytes spanned by `planes` planes of n elements at stride ld (SoA) or by
// n*planes packed elements (AoS).
Range span(const void* p, int64_t n, int64_t ld, int layout, int planes,
           size_t esize) {
  Range r{(uintptr_t)p, (uintptr_t)p};
  if (!p || n == 0) return r;
  uint64_t elems = layout == SYEV3_SOA ? (uint64_t)(planes - 1) * (uint64_t)ld + (uint64_t)n
                                       : (uint64_t)planes * (uint64_t)n;
  r.hi = r.lo + elems * esize;
  return r;
}

// ld: the SoA plane strides of A, lambda and V (0 means n), resolved here;
// all 0 for AoS.
int check_args(int64_t n, const void* A, syev3::Strides& ld, int layout,
               const void* lambda, const void* V, int dtype, uint32_t flags) {
  if (dtype != SYEV3_F64 && dtype != SYEV3_F32_REFINE && dtype != SYEV3_F32)
    return SYEV3_E_DTYPE;
  if (flags & ~SYEV3_FLAGS_ALL) return SYEV3_E_FLAGS;
  if ((flags & (SYEV3_FLAG_NEWTON | SYEV3_FLAG_PAPER_BG)) && dtype != SYEV3_F64)
    return SYEV3_E_DTYPE;
  if ((flags & SYEV3_FLAG_NEWTON) && (flags & SYEV3_FLAG_PAPER_BG)) return SYEV3_E_FLAGS;
  if ((flags & SYEV3_FLAG_REFINE_CONVERGE) && dtype != SYEV3_F32_REFINE) return SYEV3_E_DTYPE;
  if (layout != SYEV3_SOA && layout != SYEV3_AOS && layout != SYEV3_AOS9)
    return SYEV3_E_LAYOUT;
  if (n < 0) return SYEV3_E_N;
  // every element index (at most 9 planes of ld) must fit in int64 bytes
  const int64_t max_elems = (int64_t)(INT64_MAX / 16 / 9);
  if (layout == SYEV3_SOA) {
    for (int64_t* s : {&ld.a, &ld.l, &ld.v}) {
      if (*s == 0) *s = n;
      if (*s < n || *s > max_elems) return SYEV3_E_LAYOUT;
    }
  } else {
    if (ld.a != 0 || ld.l != 0 || ld.v != 0) return SYEV3_E_LAYOUT;
    if (n > max_elems) return SYEV3_E_N;
  }
  // the grid has one workgroup per 256 matrices
  if ((n + syev3::kBlock - 1) / syev3::kBlock > (int64_t)UINT32_MAX) return SYEV3_E_N;
  if (n == 0) return SYEV3_OK;
  if (!A || !lambda) return SYEV3_E_NULL;
  const size_t es = dtype == SYEV3_F64 ? sizeof(double) : sizeof(float);
  const Range ra = span(A, n, ld.a, layout, layout == SYEV3_AOS9 ? 9 : 6, es);
  const Range rl = span(lambda, n, ld.l, layout, 3, es);
  const Range rv = span(V, n, ld.v, layout, 9, es);
  // in place: the full-matrix input may be overwritten by V exactly
  const bool inplace = layout == SYEV3_AOS9 && V == A;
  if (overlap(ra, rl) || (!inplace && overlap(ra, rv)) || overlap(rl, rv))
    return SYEV3_E_ALIAS;
  return SYEV3_OK;
}

// Every entry point of the solver: checks, then the launch.
int solve(int64_t n, const void* A, syev3::Strides ld, int layout, void* lambda, void* V,
          int dtype, uint32_t flags, int32_t* info, hipStream_t stream) {
  const int rc = check_args(n, A, ld, layout, lambda, V, dtype, flags);
  if (rc != SYEV3_OK || n == 0) return rc;
  if (info) {
    const Range ri{(uintptr_t)info, (uintptr_t)info + (uintptr_t)n * sizeof(int32_t)};
    const size_t es = dtype == SYEV3_F64 ? sizeof(double) : sizeof(float);
    if (overlap(ri, span(A, n, ld.a, layout, layout == SYEV3_AOS9 ? 9 : 6, es)) ||
        overlap(ri, span(lambda, n, ld.l, layout, 3, es)) ||
        overlap(ri, span(V, n, ld.v, layout, 9, es)))
      return SYEV3_E_ALIAS;
  }
  // The launchers read the launch status with hipGetLastError, which also
  // returns an error left by any earlier HIP call of this thread (a failed
  // allocation the caller recovered from, say): clear it first, so that the
  // status is this launch's own.
  (void)hipGetLastError();
  const hipError_t e = syev3::launch_batched(n, A, ld, layout, lambda, V, dtype,
                                             flags, info, stream);
  return e == hipSuccess ? SYEV3_OK : SYEV3_E_HIP;
}

// Host image of the no-allocation entry point's segment table and the
// output ranges its alias check sorts: static, so that the call allocates
// nothing; one call at a time fills them (the table copy completes before
// the call returns).
std::mutex g_seg_mu;
syev3::TickTable g_seg_table;
Range g_seg_out[2 * SYEV3_SEGMENTS_MAX];

int solve_segments(int32_t nseg, const syev3_segment* segs, hipStream_t stream) {
  if (nseg < 0 || nseg > SYEV3_SEGMENTS_MAX) return SYEV3_E_SEGMENTS;
  if (nseg > 0 && !segs) return SYEV3_E_NULL;
  std::lock_guard<std::mutex> lock(g_seg_mu);
  syev3::TickTable& t = g_seg_table;
  int k = 0, nout = 0;
  int64_t tiles = 0;
  for (int i = 0; i < nseg; ++i) {
    const syev3_segment& q = segs[i];
    // the segment kernel holds the FP64 and the refined FP32 form
    if (q.dtype != SYEV3_F64 && q.dtype != SYEV3_F32_REFINE) return SYEV3_E_DTYPE;
    syev3::Strides ld{q.lda, 0, 0};
    const int rc = check_args(q.n, q.A, ld, SYEV3_SOA, q.lambda, q.V, q.dtype, q.flags);
    if (rc != SYEV3_OK) return rc;
    if (q.n == 0) continue;
    const size_t es = q.dtype == SYEV3_F64 ? sizeof(double) : sizeof(float);
    g_seg_out[nout++] = span(q.lambda, q.n, q.n, SYEV3_SOA, 3, es);
    if (q.V) g_seg_out[nout++] = span(q.V, q.n, q.n, SYEV3_SOA, 9, es);
    syev3::Segment& g = t.seg[k++];
    g.A = q.A;
    g.lambda = q.lambda;
    g.V = q.V;
    g.n = q.n;
    g.lda = ld.a;
    g.tile_begin = tiles;
    g.dtype = q.dtype;
    g.flags = q.flags;
    tiles += (q.n + syev3::kBlock - 1) / syev3::kBlock;
  }
  // Across segments: the outputs pairwise disjoint (sorted by start, each
  // ends before the next begins), and no input overlapping an output (the
  // last output starting below the input's end is the only candidate).
  // Inputs may share memory: they are only read.
  std::sort(g_seg_out, g_seg_out + nout,
            [](const Range& x, const Range& y) { return x.lo < y.lo; });
  for (int i = 1; i < nout; ++i)
    if (overlap(g_seg_out[i - 1], g_seg_out[i])) return SYEV3_E_ALIAS;
  for (int i = 0; i < k; ++i) {
    const syev3::Segment& g = t.seg[i];
    const size_t es = g.dtype == SYEV3_F64 ? sizeof(double) : sizeof(float);
    const Range ra = span(g.A, g.n, g.lda, SYEV3_SOA, 6, es);
    const Range* o = std::upper_bound(g_seg_out, g_seg_out + nout, ra.hi,
                                      [](uintptr_t v, const Range& x) { return v <= x.lo; });
    if (o != g_seg_out && overlap(o[-1], ra)) return SYEV3_E_ALIAS;
  }
  t.nseg = k;
  t.reserved = 0;
  t.total_tiles = tiles;
  if (tiles == 0) return SYEV3_OK;
  (void)hipGetLastError();  // a stale error is not this call's
  return syev3::launch_segments_noalloc(&t, stream) == hipSuccess ? SYEV3_OK : SYEV3_E_HIP;
}

}  // namespace

extern "C" {

int syev3_solve_segments_noalloc(int32_t nseg, const syev3_segment* segs,
                                 hipStream_t stream) {
  return solve_segments(nseg, segs, stream);
}

int batched_syev3_info(int64_t n, const void* A, int64_t ld, int layout,
                       void* lambda, void* V, int dtype, uint32_t flags,
                       int32_t* info, hipStream_t stream) {
  return solve(n, A, syev3::Strides{ld, ld, ld}, layout, lambda, V, dtype, flags, info,
               stream);
}

int batched_syev3_strided(int64_t n, const void* A, int64_t lda, void* lambda, int64_t ldl,
                          void* V, int64_t ldv, int dtype, uint32_t flags,
                          hipStream_t stream) {
  return solve(n, A, syev3::Strides{lda, ldl, ldv}, SYEV3_SOA, lambda, V, dtype, flags,
               nullptr, stream);
}

int batched_syev3_ex(int64_t n, const void* A, int64_t ld, int layout,
                     void* lambda, void* V, int dtype, uint32_t flags,
                     hipStream_t stream) {
  return batched_syev3_info(n, A, ld, layout, lambda, V, dtype, flags, nullptr,
                            stream);
}

int batched_syev3(int64_t n, const void* A_upper6, void* lambda, void* V,
                  int dtype, hipStream_t stream) {
  return batched_syev3_info(n, A_upper6, 0, SYEV3_SOA, lambda, V, dtype, 0u,
                            nullptr, stream);
}

int batched_syev3_inplace(int64_t n, void* A, void* lambda, int dtype,
                          hipStream_t stream) {
  return batched_syev3_info(n, A, 0, SYEV3_AOS9, lambda, A, dtype, 0u, nullptr, stream);
}

int syev3_stream_probe(int64_t n, const void* A, void* lambda, void* V, int dtype,
                       uint32_t mode, hipStream_t stream) {
  if ((mode & ~(SYEV3_PROBE_READ | SYEV3_PROBE_WRITE | SYEV3_PROBE_XCD_ORDER)) ||
      !(mode & (SYEV3_PROBE_READ | SYEV3_PROBE_WRITE)))
    return SYEV3_E_FLAGS;
  syev3::Strides ld{0, 0, 0};
  const int rc = check_args(n, A, ld, SYEV3_SOA, lambda, V, dtype, 0u);
  if (rc != SYEV3_OK || n == 0) return rc;
  if (n > ((int64_t)1 << 31)) return SYEV3_E_N;  // one launch
  (void)hipGetLastError();  // a stale error is not this launch's
  const hipError_t e = syev3::launch_stream_probe(n, A, lambda, V, dtype, mode, stream);
  return e == hipSuccess ? SYEV3_OK : SYEV3_E_HIP;
}

int syev3_stream_reference(int64_t n, const void* A, void* lambda, void* V, int dtype,
                           hipStream_t stream) {
  return syev3_stream_probe(n, A, lambda, V, dtype, SYEV3_PROBE_READ | SYEV3_PROBE_WRITE,
                            stream);
}

const char* syev3_strerror(int code) {
  switch (code) {
    case SYEV3_OK: return "success";
    case SYEV3_E_N: return "invalid matrix count n";
    case SYEV3_E_NULL: return "null pointer for a required array";
    case SYEV3_E_DTYPE: return "unknown dtype, or a flag the dtype does not support";
    case SYEV3_E_LAYOUT: return "unknown layout or invalid leading dimension";
    case SYEV3_E_ALIAS: return "an output overlaps the input or another output";
    case SYEV3_E_HIP: return "HIP runtime error at kernel launch";
    case SYEV3_E_FLAGS: return "unknown flag bits";
    case SYEV3_E_BUDGET: return "request larger than the server's HBM budget";
    case SYEV3_E_AGAIN: return "server full; retry after a release";
    case SYEV3_E_STATE: return "invalid server handle or request state";
    case SYEV3_E_TIMEOUT: return "timed out waiting for the request";
    case SYEV3_E_NOMEM: return "server: out of host memory";
    case SYEV3_E_SEGMENTS: return "segment count outside 0 .. SYEV3_SEGMENTS_MAX";
    default: return "unknown error code";
  }
}

int syev3_version(void) { return 10000; }

}  // extern "C"
