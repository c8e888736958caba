// syev3_noalloc.hip -- the segment table of syev3_solve_segments_noalloc: a
// fixed array in each GPU's memory instead of one allocated per call or per
// server, for callers that cannot allocate device memory.
//
// Every device holds its own copy of the array, at its own address, with
// room for the most segments one call accepts, until the process ends.  In
// host code the array's name stands for a host-side shadow, not a device
// address: the address comes from hipGetSymbolAddress, looked up once per
// device with that device current (here, at the entry point's first call on
// the device), and only that address is passed on, to the copy and to the
// segment kernel.
#include <algorithm>
#include <mutex>

#include "syev3_internal.hpp"

namespace syev3 {

static __device__ __align__(256) unsigned char scratch[sizeof(TickTable)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

hipError_t scratch_of_device(int dev, TickTable** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    g_scratch[dev] = ptr;
  }
  *out = (TickTable*)g_scratch[dev];
  return hipSuccess;
}

}  // namespace

hipError_t launch_segments_noalloc(const TickTable* host_table, hipStream_t stream) {
  int dev = 0;
  hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  TickTable* table = nullptr;
  if ((e = scratch_of_device(dev, &table)) != hipSuccess) return e;
  // In stream order: the kernel of an earlier call on this stream has read
  // the table before this copy overwrites it.
  e = hipMemcpyAsync(table, host_table, tick_table_bytes(host_table->nseg),
                     hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  // one workgroup per tile (as a server's ticks), up to 2^24
  const int64_t grid = std::min<int64_t>(host_table->total_tiles, (int64_t)1 << 24);
  (void)hipGetLastError();  // launch_segments reads it: drop any stale error
  return launch_segments(table, (int32_t)grid, stream);
}

}  // namespace syev3
