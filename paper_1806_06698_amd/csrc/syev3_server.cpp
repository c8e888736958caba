// syev3_server.cpp -- continuous-batching server for batched 3x3 solves.
//
// Clients acquire a request (admission: a free slot and room in the device
// pool, which is one hipMalloc of the HBM budget carved by a first-fit free
// list), fill its input on the device, and submit it.  A scheduler thread
// forms ticks from everything submitted so far: a table of the requests
// (segments) is written to pinned host memory and the tick is launched on
// one of `max_inflight_ticks` streams: the copy of the table to the device,
// then the segment kernel with one workgroup per tile of the tick, issued
// directly or (use_graphs) as a graph captured once per tick slot whose
// kernel node's grid is set before each replay.  While some ticks
// run, newly submitted requests go into the next free slot's tick, so work
// of different ticks overlaps on the device.  Completion is observed by
// polling each tick's event; results are then readable and the request can
// be released, freeing its memory for waiting requests.
//
// The per-matrix arithmetic of the segment kernel is that of the batched
// kernels, so each request's results are bitwise the same as a separate
// batched_syev3 call on the same input, whatever else shares its tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <system_error>
#include <random>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "syev3.h"
#include "syev3_internal.hpp"
#include "syev3_pool.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t) {
  return std::chrono::duration<double>(t - t0).count();
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum ReqState { kFree = 0, kAdmitted, kQueued, kRunning, kDone };

struct Request {
  int state = kFree;
  bool failed = false;  // its tick could not be launched
  uint32_t gen = 0;
  int64_t n = 0;
  int dtype = 0;
  bool vecs = true;
  size_t off = 0, bytes = 0;
  const void* A = nullptr;
  int64_t lda = 0;      // plane stride of A (n, or the caller's for a view)
  bool view = false;    // A is the caller's memory (syev3_server_acquire_view)
  void* lam = nullptr;
  void* V = nullptr;
  // What the tick waits for before reading A: the server's own event (own)
  // recorded behind the caller's, or an event the load generator keeps
  // alive itself.  NULL: A is complete already.
  hipEvent_t ready = nullptr;
  hipEvent_t own = nullptr;  // created on this slot's first submit with an event
  // host staging (NULL when the request's data lives on the device)
  const void* h_A = nullptr;
  void* h_lam = nullptr;
  void* h_V = nullptr;
  Clock::time_point t_submit, t_done;
};

struct TickSlot {
  // A tick runs in order on its own stream: the host-staged inputs' copies,
  // the table copy and the kernel, the copies of host-staged results, then
  // its completion event.  Ticks overlap one another (one tick's copies with
  // another's kernel) because each slot has its own stream.  Copy streams of
  // their own per slot had only multiplied the streams sharing the process's
  // few hardware queues: host-staged throughput at 4 slots was about half of
  // that at 2.
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  syev3::TickTable* h_table = nullptr;  // pinned host
  syev3::TickTable* d_table = nullptr;  // device
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the captured kernel node and its parameters: the grid is set per tick
  hipGraphNode_t knode = nullptr;
  hipKernelNodeParams kparams{};
  int32_t grid_set = 0;  // the grid the instantiated graph launches now
  std::vector<int> reqs;
  bool busy = false;
  // a profiler range from launch to observed completion
  // (rocprofv3 --marker-trace shows the ticks in flight)
  roctx_range_id_t range = 0;
};

}  // namespace

struct syev3_server {
  syev3_server_opts o{};
  int device = 0;
  char* pool = nullptr;
  // Submissions with a ready event: the server waits for the caller's event
  // here at submit and records its own per-request event behind it, so the
  // caller may destroy or re-record its event as soon as submit returns.
  hipStream_t ingress = nullptr;
  syev3::PoolAllocator* alloc = nullptr;
  std::vector<Request> req;
  std::vector<int> free_slots;
  std::deque<int> queue;
  std::vector<TickSlot> ticks;
  size_t table_bytes = 0;
  int64_t grid_cap = 0;  // most workgroups of one tick's launch

  // Workgroups for a tick of `tiles` tiles: one per tile up to grid_cap
  // (beyond it they stride over the tiles); at least one.
  int32_t tick_grid(int64_t tiles) const {
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(tiles, grid_cap));
  }

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  bool stop = false;
  std::thread thr;

  syev3_server_stats st{};
  // completion list for the built-in load generator (off otherwise)
  bool track_done = false;
  std::vector<int64_t> done_ids;
  int busy_ticks = 0;
  Clock::time_point busy_since;
  Clock::time_point t0 = Clock::now();

  int init(const syev3_server_opts& opts);
  void scheduler();
  int launch_tick(int slot);
  // after every push onto the queue (mu held)
  void note_queue() {
    st.queue_depth_peak = std::max<int64_t>(st.queue_depth_peak, (int64_t)queue.size());
  }
};

namespace {

// id = gen << 32 | slot, with gen kept to 31 bits so that ids stay positive
int64_t make_id(int slot, uint32_t gen) { return ((int64_t)gen << 32) | (int64_t)slot; }

Request* lookup(syev3_server* s, int64_t id, int* slot_out) {
  if (!s || id < 0) return nullptr;
  const int slot = (int)(id & 0xffffffff);
  const uint32_t gen = (uint32_t)(id >> 32);
  if (slot < 0 || slot >= (int)s->req.size()) return nullptr;
  Request* r = &s->req[slot];
  if (r->gen != gen || r->state == kFree) return nullptr;
  if (slot_out) *slot_out = slot;
  return r;
}

}  // namespace

int syev3_server::launch_tick(int slot) {
  TickSlot& tk = ticks[slot];
  syev3::TickTable* t = tk.h_table;
  int nseg = 0;
  int64_t tiles = 0;
  bool staged_out = false;
  hipError_t e = hipSuccess;
  hipEvent_t last_ready = nullptr;
  tk.reqs.clear();
  while (!queue.empty() && nseg < o.max_segments_per_tick) {
    const int ri = queue.front();
    queue.pop_front();
    Request& r = req[ri];
    syev3::Segment& sg = t->seg[nseg++];
    sg.A = r.A;
    sg.lambda = r.lam;
    sg.V = r.vecs ? r.V : nullptr;
    sg.n = r.n;
    sg.lda = r.lda;
    sg.tile_begin = tiles;
    sg.dtype = r.dtype;
    sg.flags = 0;
    tiles += (r.n + syev3::kBlock - 1) / syev3::kBlock;
    r.state = kRunning;
    tk.reqs.push_back(ri);
    // requests submitted together often share one ready event: wait once.
    // A wait that cannot be enqueued fails the tick: its input may not be
    // complete.
    if (r.ready && r.ready != last_ready && e == hipSuccess)
      e = hipStreamWaitEvent(tk.stream, r.ready, 0);
    last_ready = r.ready;
    if (r.h_A && e == hipSuccess) {
      const size_t es = r.dtype == SYEV3_F64 ? 8 : 4;
      e = hipMemcpyAsync(const_cast<void*>(r.A), r.h_A, 6 * (size_t)r.n * es,
                         hipMemcpyHostToDevice, tk.stream);
    }
    if (r.h_lam) staged_out = true;
  }
  t->nseg = nseg;
  t->total_tiles = tiles;
  if (e == hipSuccess) {
    const int32_t grid = tick_grid(tiles);
    if (tk.exec) {
      // the slot's previous tick has completed, so its graph may be changed
      if (grid != tk.grid_set) {
        tk.kparams.gridDim = dim3((unsigned)grid);
        e = hipGraphExecKernelNodeSetParams(tk.exec, tk.knode, &tk.kparams);
        if (e == hipSuccess) tk.grid_set = grid;
      }
      if (e == hipSuccess) e = hipGraphLaunch(tk.exec, tk.stream);
    } else {
      e = hipMemcpyAsync(tk.d_table, tk.h_table, table_bytes, hipMemcpyHostToDevice, tk.stream);
      // launch_segments reads hipGetLastError: clear any stale error first
      if (e == hipSuccess) (void)hipGetLastError();
      if (e == hipSuccess) e = syev3::launch_segments(tk.d_table, grid, tk.stream);
    }
  }
  if (staged_out && e == hipSuccess) {
    // results back to the host; the tick completes after them
    for (int ri : tk.reqs) {
      const Request& r = req[ri];
      if (!r.h_lam || e != hipSuccess) continue;
      const size_t es = r.dtype == SYEV3_F64 ? 8 : 4;
      e = hipMemcpyAsync(r.h_lam, r.lam, 3 * (size_t)r.n * es, hipMemcpyDeviceToHost,
                         tk.stream);
      if (e == hipSuccess && r.h_V && r.vecs)
        e = hipMemcpyAsync(r.h_V, r.V, 9 * (size_t)r.n * es, hipMemcpyDeviceToHost,
                           tk.stream);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(tk.done, tk.stream);
  if (e != hipSuccess) return SYEV3_E_HIP;
  tk.range = roctxRangeStartA("syev3 tick");
  tk.busy = true;
  if (busy_ticks++ == 0) busy_since = Clock::now();
  st.ticks++;
  st.inflight_ticks_peak = std::max(st.inflight_ticks_peak, busy_ticks);
  st.segments_per_tick_peak = std::max(st.segments_per_tick_peak, nseg);
  return SYEV3_OK;
}

void syev3_server::scheduler() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // completions
    bool any_done = false;
    for (auto& tk : ticks) {
      if (!tk.busy) continue;
      const hipError_t q = hipEventQuery(tk.done);
      if (q == hipErrorNotReady) continue;
      const auto now = Clock::now();
      for (int ri : tk.reqs) {
        Request& r = req[ri];
        r.state = kDone;
        r.failed = q != hipSuccess;
        r.t_done = now;
        if (r.failed) {
          st.failed++;
        } else {
          st.completed++;
          st.matrices_completed += r.n;
        }
        if (track_done) done_ids.push_back(make_id(ri, r.gen));
      }
      tk.reqs.clear();
      tk.busy = false;
      roctxRangeStop(tk.range);
      if (--busy_ticks == 0) st.busy_seconds += seconds_since(busy_since, now);
      any_done = true;
    }
    // launches: every free tick slot takes the queue's head
    for (int k = 0; k < (int)ticks.size() && !queue.empty(); ++k) {
      if (!ticks[k].busy) {
        if (launch_tick(k) != SYEV3_OK) {
          // The tick's requests complete as failed; the slot stays idle.
          // Copies enqueued before the failure may still write into their
          // buffers: let them finish before the buffers can be released.
          (void)hipStreamSynchronize(ticks[k].stream);
          const auto now = Clock::now();
          for (int ri : ticks[k].reqs) {
            req[ri].state = kDone;
            req[ri].failed = true;
            req[ri].t_done = now;
            st.failed++;
            if (track_done) done_ids.push_back(make_id(ri, req[ri].gen));
          }
          ticks[k].reqs.clear();
          any_done = true;
        }
      }
    }
    if (any_done) cv_done.notify_all();
    if (stop && busy_ticks == 0 && queue.empty()) break;
    if (busy_ticks > 0) {
      // poll completions while work is on the device (the scheduler keeps
      // one host core busy then; it sleeps when the device is idle)
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      cv_sched.wait(lk, [&] { return stop || !queue.empty(); });
    }
  }
}

// Allocates everything and starts the scheduler; on failure the caller
// frees what was made with syev3_server_destroy.  Every vector the scheduler
// thread appends to is reserved here, so that thread never allocates.
int syev3_server::init(const syev3_server_opts& opts) {
  o = opts;
  if (hipGetDevice(&device) != hipSuccess) return SYEV3_E_HIP;
  if (hipMalloc((void**)&pool, o.hbm_budget_bytes) != hipSuccess) {
    pool = nullptr;
    // reported as SYEV3_E_BUDGET: take the error off the thread's last-error
    // state, where the caller's next launch check would find it as its own
    (void)hipGetLastError();
    return SYEV3_E_BUDGET;
  }
  alloc = new syev3::PoolAllocator(o.hbm_budget_bytes);
  if (hipStreamCreateWithFlags(&ingress, hipStreamNonBlocking) != hipSuccess) {
    ingress = nullptr;
    return SYEV3_E_HIP;
  }
  req.resize(o.max_requests);
  free_slots.reserve(o.max_requests);
  for (int k = o.max_requests - 1; k >= 0; --k) free_slots.push_back(k);
  done_ids.reserve(o.max_requests);
  table_bytes = syev3::tick_table_bytes(o.max_segments_per_tick);
  // By default one workgroup per tile of each tick.  A workgroup that goes
  // on to a second tile likely waits, before that tile's loads complete, for
  // the first tile's stores as well (one counter tracks both), which one that
  // ends after its stores never does: on a tick of 202 stress-mix requests
  // (16.8 M matrices) the kernel took 0.49 ms with one workgroup per tile
  // against 0.59 ms with 32 per compute unit striding over the tiles, and
  // the serving load (input views, 256 requests in flight) served 35.9 G
  // matrices/s with a fixed 32768 workgroups against 33.0 with 8192 (32
  // per compute unit).  A fixed grid
  // far above the tiles costs latency instead (workgroups with no tile:
  // p50 at 2000 requests/s 0.07 ms with 131072, 0.15 ms with 524288), so
  // the grid is sized per tick.
  grid_cap = o.grid_blocks > 0 ? o.grid_blocks : (int64_t)1 << 24;
  ticks.resize(o.max_inflight_ticks);
  for (auto& tk : ticks) {
    tk.reqs.reserve(o.max_segments_per_tick);
    if (hipStreamCreateWithFlags(&tk.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&tk.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&tk.h_table, table_bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&tk.d_table, table_bytes) != hipSuccess)
      return SYEV3_E_HIP;
    std::memset(tk.h_table, 0, table_bytes);
    if (o.use_graphs) {
      // capture: table copy, then the segment kernel; replayed per tick
      bool ok = hipStreamBeginCapture(tk.stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        ok = hipMemcpyAsync(tk.d_table, tk.h_table, table_bytes, hipMemcpyHostToDevice,
                            tk.stream) == hipSuccess;
        (void)hipGetLastError();  // launch_segments reads it: drop any stale error
        ok = ok && syev3::launch_segments(tk.d_table, 1, tk.stream) == hipSuccess;
        const bool ended = hipStreamEndCapture(tk.stream, &tk.graph) == hipSuccess;
        ok = ok && ended;
      }
      // the kernel node, whose grid each tick sets
      size_t nn = 0;
      ok = ok && hipGraphGetNodes(tk.graph, nullptr, &nn) == hipSuccess && nn <= 8;
      hipGraphNode_t nodes[8];
      ok = ok && hipGraphGetNodes(tk.graph, nodes, &nn) == hipSuccess;
      for (size_t i = 0; ok && i < nn; ++i) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nodes[i], &ty) == hipSuccess && ty == hipGraphNodeTypeKernel)
          tk.knode = nodes[i];
      }
      ok = ok && tk.knode && hipGraphKernelNodeGetParams(tk.knode, &tk.kparams) == hipSuccess;
      tk.grid_set = 1;
      ok = ok && hipGraphInstantiate(&tk.exec, tk.graph, nullptr, nullptr, 0) == hipSuccess;
      if (!ok) return SYEV3_E_HIP;
    }
  }
  thr = std::thread([this] { scheduler(); });
  return SYEV3_OK;
}

namespace {

// Admission.  A == NULL: the request's input, eigenvalues and vectors all
// take pool memory (A has plane stride n).  A != NULL: the input is the
// caller's device memory with plane stride lda (a view; nothing copied) and
// only the outputs take pool memory.
int64_t admit(syev3_server* s, int64_t n, int dtype, int want_vectors, const void* A,
              int64_t lda, syev3_request_buffers* bufs) {
  if (!s || !bufs) return SYEV3_E_NULL;
  if (n < 1 || n > ((int64_t)1 << 40)) return SYEV3_E_N;
  if (dtype != SYEV3_F64 && dtype != SYEV3_F32_REFINE) return SYEV3_E_DTYPE;
  if (A && (lda < n || lda > ((int64_t)1 << 40))) return SYEV3_E_LAYOUT;
  const bool vecs = want_vectors != 0;
  const size_t es = dtype == SYEV3_F64 ? 8 : 4;
  const size_t in_bytes = A ? 0 : align_up(6 * (size_t)n * es);
  const size_t bytes = in_bytes + align_up(3 * (size_t)n * es) +
                       (vecs ? align_up(9 * (size_t)n * es) : 0);
  if (bytes > s->o.hbm_budget_bytes) return SYEV3_E_BUDGET;
  std::lock_guard<std::mutex> lk(s->mu);
  size_t off = 0;
  bool got = false;
  if (!s->free_slots.empty()) {
    try {
      got = s->alloc->alloc(bytes, &off);
    } catch (const std::bad_alloc&) {
      return SYEV3_E_NOMEM;  // the allocator is unchanged (strong guarantee)
    }
  }
  if (!got) {
    s->st.acquire_rejections++;
    return SYEV3_E_AGAIN;
  }
  const int slot = s->free_slots.back();
  s->free_slots.pop_back();
  Request& r = s->req[slot];
  r.state = kAdmitted;
  r.n = n;
  r.dtype = dtype;
  r.vecs = vecs;
  r.off = off;
  r.bytes = bytes;
  r.view = A != nullptr;
  r.A = A ? A : (const void*)(s->pool + off);
  r.lda = A ? lda : n;
  r.lam = s->pool + off + in_bytes;
  r.V = vecs ? s->pool + off + in_bytes + align_up(3 * (size_t)n * es) : nullptr;
  r.ready = nullptr;
  r.failed = false;
  r.h_A = nullptr;
  r.h_lam = nullptr;
  r.h_V = nullptr;
  s->st.pool_bytes_in_use = s->alloc->in_use();
  s->st.pool_bytes_peak = std::max<uint64_t>(s->st.pool_bytes_peak, s->alloc->in_use());
  bufs->A = const_cast<void*>(r.A);
  bufs->lambda = r.lam;
  bufs->V = r.V;
  bufs->n = n;
  bufs->dtype = dtype;
  return make_id(slot, r.gen);
}

}  // namespace

extern "C" {

void syev3_server_default_opts(syev3_server_opts* o) {
  if (!o) return;
  o->hbm_budget_bytes = 64ull << 30;
  o->max_requests = 4096;
  o->max_inflight_ticks = 4;
  o->max_segments_per_tick = 256;
  o->grid_blocks = 0;
  // ticks replay a graph captured once per slot (direct launches, the
  // option, complete 15-20 us sooner at low load, with the same throughput
  // at saturation)
  o->use_graphs = 1;
}

int syev3_server_create(const syev3_server_opts* opts, syev3_server** out) {
  if (!out) return SYEV3_E_NULL;
  *out = nullptr;
  syev3_server_opts o;
  syev3_server_default_opts(&o);
  if (opts) o = *opts;
  if (o.hbm_budget_bytes < kAlign || o.max_requests < 1 ||
      o.max_requests > SYEV3_SERVER_MAX_REQUESTS || o.max_inflight_ticks < 1 ||
      o.max_inflight_ticks > 64 || o.max_segments_per_tick < 1 ||
      o.max_segments_per_tick > syev3::kMaxSegmentsPerTick || o.grid_blocks < 0 ||
      o.grid_blocks > (1 << 24))
    return SYEV3_E_N;
  syev3_server* s = nullptr;
  int rc = SYEV3_OK;
  try {
    s = new syev3_server();
    rc = s->init(o);
  } catch (const std::bad_alloc&) {
    rc = SYEV3_E_NOMEM;
  } catch (const std::system_error&) {  // the scheduler thread could not start
    rc = SYEV3_E_NOMEM;
  }
  if (rc != SYEV3_OK) {
    if (s) syev3_server_destroy(s);
    return rc;
  }
  *out = s;
  return SYEV3_OK;
}

int syev3_server_destroy(syev3_server* s) {
  if (!s) return SYEV3_E_STATE;
  if (s->thr.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_sched.notify_all();
    s->thr.join();
  }
  for (auto& tk : s->ticks) {
    if (tk.stream) (void)hipStreamSynchronize(tk.stream);
    if (tk.exec) (void)hipGraphExecDestroy(tk.exec);
    if (tk.graph) (void)hipGraphDestroy(tk.graph);
    if (tk.d_table) (void)hipFree(tk.d_table);
    if (tk.h_table) (void)hipHostFree(tk.h_table);
    if (tk.done) (void)hipEventDestroy(tk.done);
    if (tk.stream) (void)hipStreamDestroy(tk.stream);
  }
  if (s->ingress) {
    (void)hipStreamSynchronize(s->ingress);
    (void)hipStreamDestroy(s->ingress);
  }
  for (auto& r : s->req)
    if (r.own) (void)hipEventDestroy(r.own);
  if (s->pool) (void)hipFree(s->pool);
  delete s->alloc;
  delete s;
  return SYEV3_OK;
}

int64_t syev3_server_acquire(syev3_server* s, int64_t n, int dtype, int want_vectors,
                             syev3_request_buffers* bufs) {
  return admit(s, n, dtype, want_vectors, nullptr, 0, bufs);
}

int64_t syev3_server_acquire_view(syev3_server* s, int64_t n, int dtype, int want_vectors,
                                  const void* A, int64_t lda, syev3_request_buffers* bufs) {
  if (!A) return SYEV3_E_NULL;
  return admit(s, n, dtype, want_vectors, A, lda, bufs);
}

int syev3_server_submit(syev3_server* s, int64_t id, hipEvent_t ready) {
  if (!s) return SYEV3_E_STATE;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    int slot;
    Request* r = lookup(s, id, &slot);
    if (!r || r->state != kAdmitted) return SYEV3_E_STATE;
    hipEvent_t own = nullptr;
    if (ready) {
      // Wait for the caller's event now, on the server's ingress stream,
      // and mark that point with the request's own event: the tick waits on
      // that one, so the caller's event is free for reuse once this returns.
      if (!r->own && hipEventCreateWithFlags(&r->own, hipEventDisableTiming) != hipSuccess) {
        r->own = nullptr;
        return SYEV3_E_HIP;  // still admitted
      }
      if (hipStreamWaitEvent(s->ingress, ready, 0) != hipSuccess ||
          hipEventRecord(r->own, s->ingress) != hipSuccess)
        return SYEV3_E_HIP;  // still admitted
      own = r->own;
    }
    try {
      s->queue.push_back(slot);
    } catch (const std::bad_alloc&) {
      return SYEV3_E_NOMEM;  // still admitted
    }
    r->state = kQueued;
    r->ready = own;
    r->t_submit = Clock::now();
    s->note_queue();
    s->st.submitted++;
  }
  s->cv_sched.notify_one();
  return SYEV3_OK;
}

int syev3_server_submit_host(syev3_server* s, int64_t id, const void* host_A,
                             void* host_lambda, void* host_V) {
  if (!s) return SYEV3_E_STATE;
  if (!host_A || !host_lambda) return SYEV3_E_NULL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    int slot;
    Request* r = lookup(s, id, &slot);
    // a view's input is the caller's device memory: there is nothing to stage
    if (!r || r->state != kAdmitted || r->view) return SYEV3_E_STATE;
    try {
      s->queue.push_back(slot);
    } catch (const std::bad_alloc&) {
      return SYEV3_E_NOMEM;  // still admitted
    }
    r->state = kQueued;
    r->ready = nullptr;
    r->h_A = host_A;
    r->h_lam = host_lambda;
    r->h_V = r->vecs ? host_V : nullptr;
    r->t_submit = Clock::now();
    s->note_queue();
    s->st.submitted++;
  }
  s->cv_sched.notify_one();
  return SYEV3_OK;
}

int syev3_server_poll(syev3_server* s, int64_t id, double* latency_s) {
  if (!s) return SYEV3_E_STATE;
  std::lock_guard<std::mutex> lk(s->mu);
  Request* r = lookup(s, id, nullptr);
  if (!r || r->state == kAdmitted) return SYEV3_E_STATE;
  if (r->state != kDone) return 0;
  if (r->failed) return SYEV3_E_HIP;
  if (latency_s) *latency_s = seconds_since(r->t_submit, r->t_done);
  return 1;
}

int syev3_server_wait(syev3_server* s, int64_t id, double timeout_s, double* latency_s) {
  if (!s) return SYEV3_E_STATE;
  if (std::isnan(timeout_s)) return SYEV3_E_N;
  // a limit beyond any real wait (and beyond what a clock duration holds)
  // is no limit
  const bool unlimited = timeout_s < 0 || timeout_s > 1e9;
  std::unique_lock<std::mutex> lk(s->mu);
  Request* r = lookup(s, id, nullptr);
  if (!r || r->state == kAdmitted) return SYEV3_E_STATE;
  // another thread may release the request while this one waits (and the
  // slot may be acquired again): that ends the wait with E_STATE
  const uint32_t gen = r->gen;
  auto done = [&] { return r->gen != gen || r->state == kDone; };
  if (unlimited) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return SYEV3_E_TIMEOUT;
  }
  if (r->gen != gen) return SYEV3_E_STATE;
  if (r->failed) return SYEV3_E_HIP;
  if (latency_s) *latency_s = seconds_since(r->t_submit, r->t_done);
  return 1;
}

int syev3_server_release(syev3_server* s, int64_t id) {
  if (!s) return SYEV3_E_STATE;
  std::lock_guard<std::mutex> lk(s->mu);
  int slot;
  Request* r = lookup(s, id, &slot);
  if (!r || (r->state != kDone && r->state != kAdmitted)) return SYEV3_E_STATE;
  try {
    s->alloc->release(r->off, r->bytes);
  } catch (const std::bad_alloc&) {
    return SYEV3_E_NOMEM;  // nothing changed: the request is still held
  }
  s->st.pool_bytes_in_use = s->alloc->in_use();
  r->state = kFree;
  s->cv_done.notify_all();  // a waiter on this id ends with E_STATE
  r->gen = (r->gen + 1) & 0x7fffffffu;
  s->free_slots.push_back(slot);
  return SYEV3_OK;
}

int syev3_server_get_stats(syev3_server* s, syev3_server_stats* out) {
  if (!s || !out) return SYEV3_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queue_depth = (int64_t)s->queue.size();
  if (s->busy_ticks > 0) out->busy_seconds += seconds_since(s->busy_since, Clock::now());
  return SYEV3_OK;
}

int syev3_server_loadgen(syev3_server* s, const syev3_loadgen_opts* o,
                         syev3_loadgen_result* out) {
  if (!s || !o || !out) return SYEV3_E_NULL;
  const bool closed = o->qps == 0.0;
  // The limits keep every quantity representable and the host-side queue of
  // arrivals bounded: at most 1e8 open-loop arrivals (1e8 per second) or
  // 2^20 closed-loop requests in flight, requests of at most 2^40 matrices.
  if (!(o->qps >= 0) || !(o->qps <= 1e8) || (closed && o->closed_concurrency < 1) ||
      (closed && o->closed_concurrency > (1 << 20)) || !(o->duration_s > 0) ||
      !(o->duration_s <= 1e6) || (!closed && !(o->qps * o->duration_s <= 1e8)) ||
      o->src_n < 1 || !o->src_f64 || !o->src_f32 || !(o->max_log2_n >= 0) ||
      !(o->max_log2_n <= 40) ||
      (o->host_staged && (!o->sink || std::exp2(o->max_log2_n) > (double)o->src_n)) ||
      (o->host_staged && o->input_views))
    return SYEV3_E_N;
  std::memset(out, 0, sizeof(*out));
  // the ready-event ring and the completion list are made before anything
  // needs undoing
  std::vector<hipEvent_t> ring;
  std::vector<int64_t> done;
  try {
    ring.assign((size_t)s->o.max_requests, nullptr);
    done.reserve((size_t)s->o.max_requests);
  } catch (const std::bad_alloc&) {
    return SYEV3_E_NOMEM;
  }
  hipStream_t prod = nullptr;
  if (hipStreamCreateWithFlags(&prod, hipStreamNonBlocking) != hipSuccess) return SYEV3_E_HIP;
  // Ready events of submitted groups.  A group's event is recorded again only
  // after ring.size() = max_requests later groups; those cannot all be
  // admitted while the group's own requests are still held, so an event is
  // never re-recorded while a queued request still refers to it.
  constexpr int kGroup = 64;
  size_t ring_next = 0;
  for (auto& e : ring) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto& f : ring)
        if (f) (void)hipEventDestroy(f);
      (void)hipStreamDestroy(prod);
      return SYEV3_E_HIP;
    }
  }
  std::mt19937_64 rng(o->seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::exponential_distribution<double> gap(closed ? 1.0 : o->qps);
  struct Arrival {
    double t;
    int64_t n;
    int64_t off;  // the request's window of the device source pool
    int dtype;
  };
  struct Live {
    double t_arrival;
    int64_t n;
  };
  std::map<int64_t, Live> live;
  std::vector<double> lat;
  double admit_wait_sum = 0.0;
  int64_t admitted = 0;
  syev3_server_stats st0{};
  syev3_server_get_stats(s, &st0);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->track_done = true;
    s->done_ids.clear();
  }
  const auto t0 = Clock::now();
  double next_t = closed ? 0.0 : gap(rng);
  double last_done = 0.0;
  int rc = SYEV3_OK;
  // Host allocations below (the arrival queue, the live map, the latency
  // list) can fail; that ends the run like any other error, and the drain
  // and cleanup after the loop allocate nothing.
  try {
  std::deque<Arrival> waiting;
  std::vector<int64_t> batch;
  auto draw = [&](double t) {
    Arrival a;
    a.t = t;
    const double nd = std::floor(std::exp2(U(rng) * o->max_log2_n));
    a.n = std::max<int64_t>(1, (int64_t)std::min((double)o->src_n, nd));
    a.dtype = U(rng) < o->frac_f32 ? SYEV3_F32_REFINE : SYEV3_F64;
    a.off = std::min<int64_t>(o->src_n - a.n,
                              (int64_t)(U(rng) * (double)(o->src_n - a.n + 1)));
    return a;
  };
  for (;;) {
    const double now = seconds_since(t0, Clock::now());
    if (closed) {
      if (now >= o->duration_s) next_t = o->duration_s;
      while (now < o->duration_s &&
             (int64_t)(live.size() + waiting.size()) < o->closed_concurrency)
        waiting.push_back(draw(now));
    } else {
      while (next_t <= now && next_t < o->duration_s) {
        waiting.push_back(draw(next_t));
        next_t += gap(rng);
      }
    }
    // Admit in arrival order.  The inputs of each group of up to kGroup
    // requests are copied on the producer stream, an event marks the end of
    // the copies, and the group is submitted with that event as its ready
    // point: the tick waits for the copies on the device while the host goes
    // on with the next group, so input copies overlap the solves of ticks
    // already launched.  With input views nothing is copied: a request reads
    // its window of the source pool, which is complete before the run, and
    // is submitted with no ready event.
    batch.clear();
    auto flush = [&]() {
      if (batch.empty() || rc != SYEV3_OK) return;
      hipEvent_t ev = nullptr;
      if (!o->input_views) {
        ev = ring[ring_next];
        ring_next = (ring_next + 1) % ring.size();
        if (hipEventRecord(ev, prod) != hipSuccess) {
          rc = SYEV3_E_HIP;
          return;
        }
      }
      {
        std::lock_guard<std::mutex> lk(s->mu);
        const auto ts = Clock::now();
        for (int64_t id : batch) {
          int slot;
          Request* r = lookup(s, id, &slot);
          if (!r || r->state != kAdmitted) { rc = SYEV3_E_STATE; break; }
          s->queue.push_back(slot);  // may throw: the request stays admitted
          r->state = kQueued;
          r->ready = ev;
          r->t_submit = ts;
          s->note_queue();
          s->st.submitted++;
        }
      }
      s->cv_sched.notify_one();
      batch.clear();
    };
    while (!waiting.empty()) {
      const Arrival a = waiting.front();
      syev3_request_buffers b;
      const size_t es = a.dtype == SYEV3_F64 ? 8 : 4;
      const char* src = (const char*)(a.dtype == SYEV3_F64 ? o->src_f64 : o->src_f32);
      const int64_t id =
          o->input_views
              ? syev3_server_acquire_view(s, a.n, a.dtype, o->want_vectors,
                                          src + (size_t)a.off * es, o->src_n, &b)
              : syev3_server_acquire(s, a.n, a.dtype, o->want_vectors, &b);
      if (id == SYEV3_E_AGAIN) break;
      if (id < 0) { rc = (int)id; break; }
      waiting.pop_front();
      // tracked from here on: on any error below the drain releases it
      try {
        live[id] = Live{a.t, a.n};
      } catch (const std::bad_alloc&) {
        (void)syev3_server_release(s, id);
        throw;
      }
      admit_wait_sum += seconds_since(t0, Clock::now()) - a.t;
      admitted++;
      if (o->host_staged) {
        // the request's input is the first 6 n values of the host source;
        // every request's results land in the same host sink
        char* sink = (char*)o->sink;
        rc = syev3_server_submit_host(s, id, src, sink,
                                      o->want_vectors ? sink + 3 * (size_t)a.n * es : nullptr);
        if (rc != SYEV3_OK) break;
      } else {
        // a random window of the source pool: read in place (a view), or
        // copied into the request's own input buffer
        if (!o->input_views &&
            hipMemcpy2DAsync(b.A, (size_t)a.n * es, src + (size_t)a.off * es,
                             (size_t)o->src_n * es, (size_t)a.n * es, 6,
                             hipMemcpyDeviceToDevice, prod) != hipSuccess) {
          rc = SYEV3_E_HIP;
          break;
        }
        batch.push_back(id);
        if ((int)batch.size() == kGroup) flush();
      }
    }
    flush();
    if (rc != SYEV3_OK) break;
    // completions
    {
      std::lock_guard<std::mutex> lk(s->mu);
      // copy, so that the server's list keeps the capacity reserved for it
      done.assign(s->done_ids.begin(), s->done_ids.end());
      s->done_ids.clear();
    }
    if (!done.empty()) {
      const double tnow = seconds_since(t0, Clock::now());
      for (int64_t id : done) {
        auto it = live.find(id);
        if (it == live.end()) continue;
        // a request whose tick failed ends the run with that error
        const int q = syev3_server_poll(s, id, nullptr);
        if (q != 1) {
          if (rc == SYEV3_OK) rc = q < 0 ? q : SYEV3_E_STATE;
          (void)syev3_server_release(s, id);
          live.erase(it);
          continue;
        }
        lat.push_back(tnow - it->second.t_arrival);
        last_done = tnow;
        out->matrices += it->second.n;
        out->requests++;
        const int p = syev3_server_release(s, id);
        if (p < 0 && rc == SYEV3_OK) rc = p;
        live.erase(it);
      }
      done.clear();
    }
    if (rc != SYEV3_OK) break;
    if (next_t >= o->duration_s && waiting.empty() && live.empty()) break;
    std::this_thread::yield();
  }
  } catch (const std::bad_alloc&) {
    rc = SYEV3_E_NOMEM;
  }
  // Drain whatever is still live after an error.  Input copies of requests
  // never submitted may still be running: finish them before any release.
  (void)hipStreamSynchronize(prod);
  for (auto& kv : live) {
    (void)syev3_server_wait(s, kv.first, 10.0, nullptr);
    (void)syev3_server_release(s, kv.first);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->track_done = false;
    s->done_ids.clear();
  }
  (void)hipStreamSynchronize(prod);
  (void)hipStreamDestroy(prod);
  for (auto& e : ring) (void)hipEventDestroy(e);
  if (rc != SYEV3_OK) return rc;
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    const size_t i =
        std::min(lat.size() - 1, (size_t)std::floor(q * (double)(lat.size() - 1) + 0.5));
    return lat[i];
  };
  double sum = 0.0;
  for (double x : lat) sum += x;
  syev3_server_stats st1{};
  syev3_server_get_stats(s, &st1);
  out->elapsed_s = last_done;
  out->matrices_per_s = last_done > 0 ? (double)out->matrices / last_done : 0.0;
  out->requests_per_s = last_done > 0 ? (double)out->requests / last_done : 0.0;
  out->lat_p50_s = pct(0.50);
  out->lat_p90_s = pct(0.90);
  out->lat_p99_s = pct(0.99);
  out->lat_p999_s = pct(0.999);
  out->lat_max_s = lat.empty() ? 0.0 : lat.back();
  out->lat_mean_s = lat.empty() ? 0.0 : sum / (double)lat.size();
  out->admit_wait_mean_s = admitted ? admit_wait_sum / (double)admitted : 0.0;
  out->ticks = st1.ticks - st0.ticks;
  out->mean_segments_per_tick =
      out->ticks ? (double)(st1.submitted - st0.submitted) / (double)out->ticks : 0.0;
  out->inflight_ticks_peak = st1.inflight_ticks_peak;
  out->pool_bytes_peak = st1.pool_bytes_peak;
  return SYEV3_OK;
}

}  // extern "C"
