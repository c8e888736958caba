// syev3_internal.hpp -- declarations shared by the library's host sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "syev3.h"

namespace syev3 {

constexpr int kBlock = 256;  // lanes (matrices) per workgroup: 4 wavefronts

// Plane strides (elements) of the three SoA arrays; unused (0) for AoS.
struct Strides {
  int64_t a, l, v;
};

// Launch the batched solver; arguments already validated (SoA strides
// resolved: each >= n).  Returns the HIP status of the launch.
hipError_t launch_batched(int64_t n, const void* A, Strides ld, int layout,
                          void* lambda, void* V, int dtype, uint32_t flags,
                          int32_t* info, hipStream_t stream);

// One request of a serving tick, as the segment kernel reads it from device
// memory.  Matrices of segment s occupy tiles [tile_begin, tile_begin +
// ceil(n / kBlock)) of the tick's tile space, so no workgroup spans two
// segments.
struct Segment {
  const void* A;  // 6 planes of n, plane stride lda
  void* lambda;   // 3 planes of n, plane stride n
  void* V;        // 9 planes of n, plane stride n; NULL: eigenvalues only
  int64_t n;
  int64_t lda;    // >= n
  int64_t tile_begin;
  int32_t dtype;
  uint32_t flags;
};

// The solver's SoA loads and/or stores with trivial arithmetic (measurement
// aid); mode: SYEV3_PROBE_* bits, at least one of READ and WRITE.
hipError_t launch_stream_probe(int64_t n, const void* A, void* lambda, void* V, int dtype,
                               uint32_t mode, hipStream_t stream);

// A tick's table in device memory: header, then the segments in ascending
// tile_begin order.  Sized for kMaxSegmentsPerTick; only nseg are read.
constexpr int kMaxSegmentsPerTick = SYEV3_SERVER_MAX_SEGMENTS;
struct TickTable {
  int32_t nseg;
  int32_t reserved;
  int64_t total_tiles;
  Segment seg[kMaxSegmentsPerTick];
};
// Bytes of a table with room for `max_segments` segments.
inline size_t tick_table_bytes(int max_segments) {
  return offsetof(TickTable, seg) + sizeof(Segment) * (size_t)max_segments;
}

// Launch the segment kernel on a table in device memory: grid_blocks
// workgroups stride over the table's tiles.
hipError_t launch_segments(const TickTable* table, int32_t grid_blocks,
                           hipStream_t stream);

// The same on the library's fixed per-device table (no allocation): copies
// host_table (nseg segments, total_tiles > 0) into the table of the stream's
// device, then launches on it.  The copy is from pageable host memory, which
// HIP completes before returning.
hipError_t launch_segments_noalloc(const TickTable* host_table, hipStream_t stream);

}  // namespace syev3
