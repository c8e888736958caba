// syev3_kernels.hip -- batched 3x3 symmetric eigensolver kernels (gfx950).
//
// One lane per matrix.  Each workgroup handles kBlock = 256 consecutive
// matrices.
//   * SoA: each of the 6 input planes and of the 3 + 9 output planes is read
//     or written by a wavefront as one contiguous 512-byte (FP64) or 256-byte
//     (FP32) run: fully coalesced, no LDS.
//   * AoS: the workgroup's 256 x 6 input block is contiguous in memory; it is
//     read with unit-stride lanes (16 bytes each) into LDS and each lane then
//     picks up its own 6 entries (the transpose).  Outputs go back through
//     LDS the same way, so global stores are unit-stride as well.
// Streams are read and written once, with non-temporal hints (no reuse).
#include <type_traits>

#include "syev3_internal.hpp"
#include "syev3_lane.hpp"

namespace syev3 {

// Workgroup order.  The dispatcher deals workgroups to the 8 XCDs in turn,
// so in launch order neighbouring tiles of the batch run on different XCDs.
// For large batches each XCD instead takes kXcdChunk consecutive tiles at a
// time (the blocks of a partial last round of 8 * kXcdChunk keep their own
// index; any bijection is correct).  Measured on FP64 SoA solves of N(0,1)
// matrices: launch order falls from 5.7 TB/s at 2^25 matrices to 5.1-5.3
// TB/s at 2^26-2^28, chunks of 256 tiles (64K matrices, 512 KB of each FP64
// plane) hold 5.4-5.8 TB/s there (+9% at 2^26); at 2^24 launch order is as
// good or better; 64-tile chunks are slower than launch order, 512-1024
// close to 256.  The pure streaming reference is fastest in launch order,
// so it keeps it.
constexpr uint32_t kXcds = 8;
constexpr int kWave = 64;  // gfx950 runs wave64
constexpr uint32_t kXcdChunk = 256;
constexpr uint32_t kChunkFromBlocks = 1u << 17;  // 2^25 matrices

__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t nb) {
  constexpr uint32_t G = kXcds * kXcdChunk;
  if (nb < kChunkFromBlocks || b >= nb / G * G) return b;
  const uint32_t x = b % kXcds, slot = b / kXcds;
  return slot / kXcdChunk * G + x * kXcdChunk + slot % kXcdChunk;
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}

// The element type a form stores: double for FP64, float for both FP32
// forms.
template <int FORM>
using Storage = typename std::conditional<FORM == kFormF64, double, float>::type;

template <typename T>
__device__ __forceinline__ T qnan() {
  return (T)__builtin_nan("");
}

// The 18 plane base addresses of an SoA solve, passed as kernel arguments
// (uniform, held in scalar registers): each array has a plane stride of its
// own, so they may lie anywhere.
template <typename T>
struct Planes {
  const T* a[6];
  T* l[3];
  T* v[9];
};

// T = double: FP64 path.  T = float: FP32 storage with FP64 refinement.
// 64-bit element offsets, for planes of more than 2^32 bytes.
template <int FORM, bool VECS, bool INFO>
__global__ __launch_bounds__(kBlock) void k_syev3_soa(int64_t n, Planes<Storage<FORM>> P,
                                                     uint32_t flags, int32_t* __restrict__ info) {
  using T = Storage<FORM>;
  const int64_t i = (int64_t)tile_of_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double a[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) a[k] = (double)ld_stream(P.a[k] + i);
  double l[3], v[9];
  bool bad;
  const int code = solve3<VECS, FORM>(a, flags, l, v, bad);
#pragma unroll
  for (int j = 0; j < 3; ++j) st_stream((T)l[j], P.l[j] + i);
  if (VECS) {
#pragma unroll
    for (int k = 0; k < 9; ++k) st_stream((T)v[k], P.v[k] + i);
  }
  if (bad) {  // a NaN or infinite entry: NaN in every output of the matrix
#pragma unroll
    for (int j = 0; j < 3; ++j) st_stream(qnan<T>(), P.l[j] + i);
    if (VECS) {
#pragma unroll
      for (int k = 0; k < 9; ++k) st_stream(qnan<T>(), P.v[k] + i);
    }
  }
  if (INFO) info[i] = code;
}

// The same with a 32-bit byte offset per lane, for n * sizeof(T) < 2^32:
// loads and stores take the scalar-base addressing form and need no 64-bit
// address arithmetic per lane.

template <int FORM, bool VECS, bool INFO>
__global__ __launch_bounds__(kBlock) void k_syev3_soa32(uint32_t n, Planes<Storage<FORM>> P,
                                                       uint32_t flags, int32_t* __restrict__ info) {
  using T = Storage<FORM>;
  const uint32_t i = tile_of_block(blockIdx.x, gridDim.x) * (uint32_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t off = i * (uint32_t)sizeof(T);  // byte offset within a plane
  double a[6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
    a[k] = (double)ld_stream((const T*)((const char*)P.a[k] + off));
  double l[3], v[9];
  bool bad;
  const int code = solve3<VECS, FORM>(a, flags, l, v, bad);
  // The offset is re-defined here (an empty asm emits nothing) so that the
  // stores, past the solve's branches, again see a 32-bit offset and take
  // the scalar-base form rather than a 64-bit address add per store: 12
  // fewer VALU per wavefront, 2.4% faster for the VALU-bound FP32 form.
  uint32_t soff = off;
  asm volatile("" : "+v"(soff));
#pragma unroll
  for (int j = 0; j < 3; ++j) st_stream((T)l[j], (T*)((char*)P.l[j] + soff));
  if (VECS) {
#pragma unroll
    for (int k = 0; k < 9; ++k) st_stream((T)v[k], (T*)((char*)P.v[k] + soff));
  }
  if (bad) {  // a NaN or infinite entry: NaN in every output of the matrix
#pragma unroll
    for (int j = 0; j < 3; ++j) st_stream(qnan<T>(), (T*)((char*)P.l[j] + soff));
    if (VECS) {
#pragma unroll
      for (int k = 0; k < 9; ++k) st_stream(qnan<T>(), (T*)((char*)P.v[k] + soff));
    }
  }
  if (INFO) info[i] = code;
}

// Block copies between global memory and the LDS buffer of the AoS kernel:
// 16 bytes per lane when the global address is 16-byte aligned (it is for
// every block when the caller's array is), else one element per lane.
// total elements; lanes t = 0 .. kBlock - 1.  Measured on 2^26 matrices:
// 4% faster in FP64 and 9% in FP32 than element-wide copies.
template <typename T>
__device__ __forceinline__ void copy_in(T* sm, const T* g, int total, int t) {
  constexpr int W = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(W)));
  int k0 = 0;
  if (((uintptr_t)g & 15u) == 0) {
    const int nv = total / W;
    for (int k = t; k < nv; k += kBlock) ((vec*)sm)[k] = ld_stream((const vec*)g + k);
    k0 = nv * W;
  }
  for (int k = k0 + t; k < total; k += kBlock) sm[k] = ld_stream(g + k);
}

// The same for a full tile, whose size is known at compile time: every lane
// issues all of its loads (or LDS reads) before the first write, so its
// memory requests are in flight together rather than one after another.
// g must be 16-byte aligned.  TOTAL = elements, a multiple of 16 / sizeof(T).
template <typename T, int TOTAL>
__device__ __forceinline__ void copy_in_full(T* sm, const T* g, int t) {
  constexpr int W = 16 / sizeof(T);
  constexpr int NV = TOTAL / W;
  constexpr int R = (NV + kBlock - 1) / kBlock;
  static_assert(TOTAL % W == 0, "whole 16-byte vectors");
  typedef T vec __attribute__((ext_vector_type(W)));
  vec x[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int k = t + j * kBlock;
    if (j + 1 < R || k < NV) x[j] = ld_stream((const vec*)g + k);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int k = t + j * kBlock;
    if (j + 1 < R || k < NV) ((vec*)sm)[k] = x[j];
  }
}

template <typename T, int TOTAL>
__device__ __forceinline__ void copy_out_full(T* g, const T* sm, int t) {
  constexpr int W = 16 / sizeof(T);
  constexpr int NV = TOTAL / W;
  constexpr int R = (NV + kBlock - 1) / kBlock;
  static_assert(TOTAL % W == 0, "whole 16-byte vectors");
  typedef T vec __attribute__((ext_vector_type(W)));
  vec x[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int k = t + j * kBlock;
    if (j + 1 < R || k < NV) x[j] = ((const vec*)sm)[k];
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int k = t + j * kBlock;
    if (j + 1 < R || k < NV) st_stream(x[j], (vec*)g + k);
  }
}

template <typename T>
__device__ __forceinline__ void copy_out(T* g, const T* sm, int total, int t) {
  constexpr int W = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(W)));
  int k0 = 0;
  if (((uintptr_t)g & 15u) == 0) {
    const int nv = total / W;
    for (int k = t; k < nv; k += kBlock) st_stream(((const vec*)sm)[k], (vec*)g + k);
    k0 = nv * W;
  }
  for (int k = k0 + t; k < total; k += kBlock) st_stream(sm[k], g + k);
}

// AoS: IN = 6 (unique entries) or 9 (full row-major matrix, upper triangle
// read).  The whole block is read into LDS before any global store, so the
// full-matrix input may be overwritten by V (in place).  A is therefore not
// __restrict__.  The outputs leave through the same LDS buffer in two
// rounds, lambda and then V, so the buffer holds 9 values per matrix rather
// than 12: 18 KB per workgroup in FP64, which lets 8 waves per SIMD fit in
// the 160 KB of LDS (24 KB allowed only 6).
template <int FORM, int IN, bool VECS, bool INFO>
__global__ __launch_bounds__(kBlock) void k_syev3_aos(
    int64_t n, const Storage<FORM>* A, Storage<FORM>* __restrict__ lam, Storage<FORM>* V,
    uint32_t flags, int32_t* __restrict__ info) {
  using T = Storage<FORM>;
  __shared__ __attribute__((aligned(16))) T sm[kBlock * 9];
  const int64_t base = (int64_t)tile_of_block(blockIdx.x, gridDim.x) * kBlock;
  const int cnt = (int)((n - base) < kBlock ? (n - base) : kBlock);
  const int t = threadIdx.x;
  const T* Ab = A + base * IN;
  // full tiles of a 16-byte-aligned array take the unrolled copies (every
  // tile but the last, when the caller's arrays are aligned)
  const bool full = cnt == kBlock && ((uintptr_t)A & 15u) == 0 &&
                    ((uintptr_t)lam & 15u) == 0 && (!VECS || ((uintptr_t)V & 15u) == 0);
  if (full) copy_in_full<T, kBlock * IN>(sm, Ab, t);
  else copy_in(sm, Ab, cnt * IN, t);
  __syncthreads();
  double a[6];
  if (t < cnt) {
    if (IN == 6) {
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] = (double)sm[6 * t + k];
    } else {
      const T* m = sm + IN * t;
      a[0] = (double)m[0]; a[1] = (double)m[1]; a[2] = (double)m[2];
      a[3] = (double)m[4]; a[4] = (double)m[5]; a[5] = (double)m[8];
    }
  }
  __syncthreads();
  double l[3], v[9];
  bool bad = false;
  if (t < cnt) {
    const int code = solve3<VECS, FORM>(a, flags, l, v, bad);
#pragma unroll
    for (int j = 0; j < 3; ++j) sm[3 * t + j] = (T)l[j];
    if (bad) {  // a NaN or infinite entry: NaN in every output of the matrix
#pragma unroll
      for (int j = 0; j < 3; ++j) sm[3 * t + j] = qnan<T>();
    }
    if (INFO) info[base + t] = code;
  }
  __syncthreads();
  if (full) copy_out_full<T, kBlock * 3>(lam + base * 3, sm, t);
  else copy_out(lam + base * 3, sm, cnt * 3, t);
  if (VECS) {
    __syncthreads();  // every lambda read from LDS before V overwrites it
    if (t < cnt) {
#pragma unroll
      for (int k = 0; k < 9; ++k) sm[9 * t + k] = (T)v[k];
      if (bad) {
#pragma unroll
        for (int k = 0; k < 9; ++k) sm[9 * t + k] = qnan<T>();
      }
    }
    __syncthreads();
    if (full) copy_out_full<T, kBlock * 9>(V + base * 9, sm, t);
    else copy_out(V + base * 9, sm, cnt * 9, t);
  }
}

template <int FORM, bool VECS, bool INFO>
static hipError_t launch_t(int64_t n, const void* A, Strides ld, int layout,
                           void* lambda, void* V, uint32_t flags, int32_t* info,
                           hipStream_t stream) {
  using T = Storage<FORM>;
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  const dim3 grid((unsigned)blocks), block(kBlock);
  if (layout == 0) {
    Planes<T> P;
    for (int k = 0; k < 6; ++k) P.a[k] = (const T*)A + k * ld.a;
    for (int j = 0; j < 3; ++j) P.l[j] = (T*)lambda + j * ld.l;
    for (int k = 0; k < 9; ++k) P.v[k] = VECS ? (T*)V + k * ld.v : nullptr;
    if ((uint64_t)n * sizeof(T) <= (uint64_t)UINT32_MAX)
      hipLaunchKernelGGL((k_syev3_soa32<FORM, VECS, INFO>), grid, block, 0, stream, (uint32_t)n,
                         P, flags, info);
    else
      hipLaunchKernelGGL((k_syev3_soa<FORM, VECS, INFO>), grid, block, 0, stream, n, P, flags,
                         info);
  } else if (layout == 1) {
    hipLaunchKernelGGL((k_syev3_aos<FORM, 6, VECS, INFO>), grid, block, 0, stream, n,
                       (const T*)A, (T*)lambda, (T*)V, flags, info);
  } else {
    hipLaunchKernelGGL((k_syev3_aos<FORM, 9, VECS, INFO>), grid, block, 0, stream, n,
                       (const T*)A, (T*)lambda, (T*)V, flags, info);
  }
  return hipGetLastError();
}

// A dispatch counts its grid in work-items with 32 bits per dimension, so one
// launch covers at most 2^31 matrices (2^23 workgroups); larger batches are
// solved by consecutive launches on the same stream.  Each matrix is solved
// by its own lane, so the split changes no result.
constexpr int64_t kMaxPerLaunch = (int64_t)1 << 31;

template <int FORM>
static hipError_t launch_dt(int64_t n, const void* A, Strides ld, int layout,
                            void* lambda, void* V, uint32_t flags, int32_t* info,
                            hipStream_t stream) {
  using T = Storage<FORM>;
  // elements per matrix between consecutive matrices: SoA planes are
  // offset as a whole (ld is unchanged), AoS rows are packed
  const int64_t w_in = layout == 0 ? 1 : (layout == 1 ? 6 : 9);
  const int64_t w_lam = layout == 0 ? 1 : 3, w_v = layout == 0 ? 1 : 9;
  for (int64_t s = 0; s < n; s += kMaxPerLaunch) {
    const int64_t m = n - s < kMaxPerLaunch ? n - s : kMaxPerLaunch;
    const T* As = (const T*)A + s * w_in;
    T* ls = (T*)lambda + s * w_lam;
    T* Vs = V ? (T*)V + s * w_v : nullptr;
    int32_t* is = info ? info + s : nullptr;
    hipError_t e;
    if (V) {
      e = info ? launch_t<FORM, true, true>(m, As, ld, layout, ls, Vs, flags, is, stream)
               : launch_t<FORM, true, false>(m, As, ld, layout, ls, Vs, flags, is, stream);
    } else {
      e = info ? launch_t<FORM, false, true>(m, As, ld, layout, ls, Vs, flags, is, stream)
               : launch_t<FORM, false, false>(m, As, ld, layout, ls, Vs, flags, is, stream);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batched(int64_t n, const void* A, Strides ld, int layout,
                          void* lambda, void* V, int dtype, uint32_t flags,
                          int32_t* info, hipStream_t stream) {
  if (dtype == kFormF64)
    return launch_dt<kFormF64>(n, A, ld, layout, lambda, V, flags, info, stream);
  if (dtype == kFormF32R)
    return launch_dt<kFormF32R>(n, A, ld, layout, lambda, V, flags, info, stream);
  return launch_dt<kFormF32>(n, A, ld, layout, lambda, V, flags, info, stream);
}

// ---------------------------------------------------------------------------
// Serving: one launch solves every request of a tick.  A tile is kBlock
// matrices of one segment, so each wavefront runs one dtype and one code
// path; the launch has one workgroup per tile unless its grid is capped, in
// which case workgroups stride over the tiles.  Per-matrix arithmetic is
// exactly the batched kernels' (eigenvalues do not depend on whether
// vectors are formed).
// ---------------------------------------------------------------------------
// One tile of segment s: matrices t0 .. t0 + kBlock - 1.  The tile's first
// matrix is folded into the plane bases (uniform, in scalar registers), so
// each lane adds only threadIdx.x elements as a 32-bit byte offset, whatever
// the request's size: every load and store of the solve is a global access
// of a scalar base and that offset, as in the batched SoA kernel (empty asm
// statements keep the bases scalar and the offset 32-bit; only the NaN path
// forms full addresses).  Every tile solves for vectors, and a request
// without them (V null, a uniform branch) skips only their stores: with one
// solve per form the kernel holds two inlined solves, not four, and fits in
// 62 VGPRs (8 waves per SIMD; four solves needed 84, 5 waves).
template <int FORM>
__device__ __forceinline__ void solve_segment_tile(const Segment& s, int64_t t0) {
  using T = Storage<FORM>;
  // the table's pointers are generic: cast to global memory, else every
  // access is a flat one with a 64-bit address per lane
  using GT = __attribute__((address_space(1))) T;
  using GC = __attribute__((address_space(1))) char;
  const int64_t pa = s.lda * (int64_t)sizeof(T), po = s.n * (int64_t)sizeof(T);
  const GC* A = (const GC*)s.A + t0 * (int64_t)sizeof(T);
  GC* L = (GC*)s.lambda + t0 * (int64_t)sizeof(T);
  GC* W = (GC*)s.V + t0 * (int64_t)sizeof(T);
  const bool vecs = s.V != nullptr;
  uint32_t off = threadIdx.x * (uint32_t)sizeof(T);
  asm volatile("" : "+v"(off));
  double a[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    // each plane's base pinned in scalar registers (else the compiler chains
    // the planes' addresses per lane in 64 bits)
    const GC* p = A + k * pa;
    asm volatile("" : "+s"(p));
    a[k] = (double)__builtin_nontemporal_load((const GT*)(p + off));
  }
  double l[3], v[9];
  bool bad;
  solve3<true, FORM>(a, s.flags, l, v, bad);
  uint32_t soff = off;
  asm volatile("" : "+v"(soff));
  GC* lp[3];
  GC* vp[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    lp[j] = L + j * po;
    asm volatile("" : "+s"(lp[j]));
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    vp[k] = W + k * po;
    asm volatile("" : "+s"(vp[k]));
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) __builtin_nontemporal_store((T)l[j], (GT*)(lp[j] + soff));
  if (vecs) {
    uint32_t voff = soff;
    asm volatile("" : "+v"(voff));
#pragma unroll
    for (int k = 0; k < 9; ++k) __builtin_nontemporal_store((T)v[k], (GT*)(vp[k] + voff));
  }
  if (bad) {  // a NaN or infinite entry: NaN in every output of the matrix
#pragma unroll
    for (int j = 0; j < 3; ++j) __builtin_nontemporal_store(qnan<T>(), (GT*)(lp[j] + soff));
    if (vecs) {
#pragma unroll
      for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(qnan<T>(), (GT*)(vp[k] + soff));
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_syev3_segments(const TickTable* __restrict__ t) {
  const int nseg = t->nseg;
  const int64_t total_tiles = t->total_tiles;
  // A tile's segment is the last whose tile_begin <= tile (uniform across
  // the workgroup).  The table is in ascending tile_begin order, so its index
  // is the count of segments starting at or before the tile, minus one: each
  // lane tests four segments and ballots count them, kRound per round, with
  // the four loads in flight together.  A round not all of whose segments
  // start at or before the tile is the last.  A workgroup's tiles ascend, so
  // its next search starts at the round that held this tile's segment.
  constexpr int kRound = 4 * kWave;
  int from = 0;  // a multiple of kRound; every segment before it qualifies
  for (int64_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    int cnt = from;
    for (int base = from; base < nseg; base += kRound) {
      int64_t tb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = base + u * kWave + (int)(threadIdx.x % kWave);
        tb[u] = j < nseg ? t->seg[j].tile_begin : INT64_MAX;
      }
      int c = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) c += __popcll(__ballot(tb[u] <= tile));
      cnt += c;
      if (c < kRound) break;
    }
    const int lo = cnt - 1;
    from = lo / kRound * kRound;
    const Segment s = t->seg[lo];
    const int64_t t0 = (tile - s.tile_begin) * kBlock;  // the tile's first matrix
    if (t0 + threadIdx.x < s.n) {
      // the server admits the FP64 and the refined FP32 form
      if (s.dtype == kFormF64) solve_segment_tile<kFormF64>(s, t0);
      else solve_segment_tile<kFormF32R>(s, t0);
    }
  }
}

hipError_t launch_segments(const TickTable* table, int32_t grid_blocks,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_syev3_segments, dim3((unsigned)grid_blocks), dim3(kBlock), 0,
                     stream, table);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming probes: the SoA kernel's loads (RD) and/or stores (WR), with a
// sum in place of the solve, in launch order or in the solver's XCD-chunked
// workgroup order.  A read-only probe's one store is taken only for a NaN
// sum, so its loads are kept and it writes nothing for finite input.  RD and
// WR together in launch order is the streaming reference.
// ---------------------------------------------------------------------------
template <typename T, bool VECS, bool RD, bool WR, bool XCD>
__global__ __launch_bounds__(kBlock) void k_stream_reference(int64_t n, const T* __restrict__ A,
                                                             T* __restrict__ lam,
                                                             T* __restrict__ V) {
  const uint32_t b = XCD ? tile_of_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t i = (int64_t)b * kBlock + threadIdx.x;
  if (i >= n) return;
  T s = RD ? (T)0 : (T)threadIdx.x;
  if (RD) {
#pragma unroll
    for (int k = 0; k < 6; ++k) s += ld_stream(A + k * n + i);
  }
  if (WR) {
#pragma unroll
    for (int j = 0; j < 3; ++j) st_stream(s * (T)(j + 1), lam + j * n + i);
    if (VECS) {
#pragma unroll
      for (int k = 0; k < 9; ++k) st_stream(s * (T)(k + 4), V + k * n + i);
    }
  } else if (__builtin_isnan(s)) {
    lam[i] = s;
  }
}

template <typename T, bool VECS>
static hipError_t launch_probe_t(int64_t n, const T* A, T* lambda, T* V, uint32_t mode,
                                 hipStream_t stream) {
  const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
  const bool rd = mode & 1u, wr = mode & 2u, xcd = mode & 4u;
#define SYEV3_PROBE_CASE(R, W, X)                                                         \
  if (rd == R && wr == W && xcd == X) {                                                   \
    hipLaunchKernelGGL((k_stream_reference<T, VECS, R, W, X>), grid, block, 0, stream, n, \
                       A, lambda, V);                                                     \
    return hipGetLastError();                                                             \
  }
  SYEV3_PROBE_CASE(true, true, false)
  SYEV3_PROBE_CASE(true, true, true)
  SYEV3_PROBE_CASE(true, false, false)
  SYEV3_PROBE_CASE(true, false, true)
  SYEV3_PROBE_CASE(false, true, false)
  SYEV3_PROBE_CASE(false, true, true)
#undef SYEV3_PROBE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_stream_probe(int64_t n, const void* A, void* lambda, void* V, int dtype,
                               uint32_t mode, hipStream_t stream) {
  // the kernel's planes are n apart, so a split batch is not expressible:
  // the probes are for batches one launch can hold
  if (n > kMaxPerLaunch) return hipErrorInvalidValue;
  if (dtype == 0) {
    return V ? launch_probe_t<double, true>(n, (const double*)A, (double*)lambda, (double*)V,
                                            mode, stream)
             : launch_probe_t<double, false>(n, (const double*)A, (double*)lambda, nullptr,
                                             mode, stream);
  }
  return V ? launch_probe_t<float, true>(n, (const float*)A, (float*)lambda, (float*)V, mode,
                                         stream)
           : launch_probe_t<float, false>(n, (const float*)A, (float*)lambda, nullptr, mode,
                                          stream);
}

}  // namespace syev3
