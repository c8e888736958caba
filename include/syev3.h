/*
 * syev3.h -- batched solver for 3x3 real symmetric eigenproblems on AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * Method: C. F. Borges, "Solving the 3x3 Real Symmetric Eigenproblem"
 * (arXiv:1806.06698).  Each matrix is reduced by a Jacobi rotation in the
 * (1,2)-plane to an ordered arrow (Sec. 1), tested for beta-, combo- and
 * numerical deflation with a Givens rotation (Sec. 1.1), and otherwise
 * solved through the two shifted fully reduced arrows: the rightmost zero of
 * each spectral function by the Borges-Gragg zero finder (Sec. 1.4.1), the
 * middle eigenvalue by the trace identity and the eigenvectors by the
 * closed forms u1, u3 and u2 (Sec. 1.2).  The problem solved is the one the
 * paper's accuracy measures define (Sec. 1.5): for each symmetric A find the
 * diagonal Lambda and orthonormal V with A V = V Lambda.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * A matrix is given by its 6 unique entries in the order
 *     a11, a12, a13, a22, a23, a33.
 * Layouts:
 *   SYEV3_SOA  structure of arrays.  Entry k of matrix i is A[k*ld + i]
 *              (6 planes); eigenvalue j is lambda[j*ld + i] (3 planes);
 *              V[(3*r + c)*ld + i] is row r of eigenvector c (9 planes).
 *              ld >= n is the plane stride in elements (0 means n).
 *   SYEV3_AOS  array of structures, packed: A[6*i + k], lambda[3*i + j],
 *              V[9*i + 3*r + c] (row-major 3x3, column c is eigenvector c,
 *              as torch.linalg.eigh).  ld must be 0.
 *   SYEV3_AOS9 as SYEV3_AOS, but the input is the full matrix,
 *              A[9*i + 3*r + c]; entries below the diagonal are not read.
 *              V may be the same pointer as A (in place).
 * Eigenvalues are in ascending order; column c of V belongs to lambda c.
 * The sign of each eigenvector, and the basis inside an eigenspace of a
 * repeated eigenvalue, are whatever the method produces.
 * dtype SYEV3_F64: every array is double.  dtypes SYEV3_F32_REFINE and
 * SYEV3_F32: every array is float; the arithmetic is mixed (see below).
 * V may be NULL: eigenvalues only.
 *
 * Memory: every pointer is device memory owned by the caller, alive until
 * the work queued on `stream` has finished.  The library allocates nothing
 * on these paths.  Outputs must not overlap the input or each other.
 *
 * Execution: asynchronous on `stream` (a hipStream_t of the current device;
 * NULL is the null stream).  A return of 0 means the work was enqueued.  A
 * batch of more than 2^31 matrices is enqueued as consecutive launches of
 * at most 2^31 (a dispatch counts its grid in 32 bits); the results are the
 * same as in one launch.
 *
 * Errors: negative return values, listed below, with nothing enqueued
 * (except SYEV3_E_HIP on a later launch of a split batch, which leaves the
 * earlier launches enqueued).  Before it launches, a call clears any error
 * an earlier HIP call of the thread left pending (hipGetLastError), so that
 * SYEV3_E_HIP reports this launch only.
 * n == 0 is a no-op returning 0.  Numerical trouble in one matrix never fails
 * a call: a matrix with a NaN or infinite entry gets NaN eigenvalues and
 * eigenvectors.  No C++ exception crosses this interface.  Calls may be made
 * from several host threads at once; the library keeps no mutable global
 * state on these paths.
 */
#ifndef SYEV3_H
#define SYEV3_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dtypes */
#define SYEV3_F64 0          /* FP64 storage, FP64 arithmetic */
#define SYEV3_F32_REFINE 1   /* FP32 storage; FP64 reduction, deflation test
                                and eigenvectors.  Each root: an FP32 start
                                and one FP32 Borges-Gragg step, then an FP64
                                Newton step (Sec. 1.4.2), a second one where
                                the first moved it by more than 2^-22 of
                                itself, and FP64 Borges-Gragg steps where it
                                moved it by more than 2^-14.  Eigenvalues
                                within eps32 ||A|| / 16 of the exact ones
                                before rounding to FP32 */
#define SYEV3_F32 2          /* FP32 storage without the refinement: the
                                zeros of an FP32 Borges-Gragg iteration are
                                used as they are and the vectors come from
                                the formulas of Sec. 1 without
                                re-orthogonalisation.  For measuring what
                                the refinement buys (an ablation); the
                                server does not accept it */

/* layouts */
#define SYEV3_SOA 0
#define SYEV3_AOS 1
#define SYEV3_AOS9 2   /* input n x 9: full row-major 3x3 matrices (only the
                          upper triangle is read); outputs as SYEV3_AOS */

/* flags for batched_syev3_ex */
#define SYEV3_FLAG_SIMPLIFIED_DEFLATION 1u /* the simplified test of Sec. 1.1,
                                              |e| <= eps |alpha1 + alpha2|,
                                              instead of the EISPACK form */
#define SYEV3_FLAG_NO_H_GUARD 2u  /* treat only h == 0 as diagonal (Sec. 1.1
                                     literally); by default h <= eps (|alpha1|
                                     + |alpha2| + |gamma|) also is */
#define SYEV3_FLAG_NEWTON 4u      /* Newton's method from the left
                                     (Sec. 1.4.2) instead of Borges-Gragg;
                                     SYEV3_F64 only */
#define SYEV3_FLAG_PAPER_BG 8u    /* Borges-Gragg exactly as Sec. 1.4.1
                                     states it: start from the first iterate
                                     from +infinity, stop when f/f' < 2 eps x.
                                     For measuring what the default start
                                     and stop test save; SYEV3_F64 only, not
                                     with SYEV3_FLAG_NEWTON */
#define SYEV3_FLAG_REFINE_CONVERGE 16u /* FP32 storage: after the first FP64
                                     Newton step, continue every root with
                                     FP64 Borges-Gragg steps (Sec. 1.4.1)
                                     until their stop test, as is otherwise
                                     done only when the Newton correction
                                     exceeds 2^-14 of the root.  Eigenvalues as
                                     accurate as the FP64 zero finder makes
                                     them, for one or two more FP64
                                     evaluations per root; SYEV3_F32_REFINE
                                     only */
#define SYEV3_FLAG_NO_SCALE 32u   /* no power-of-two scaling of each matrix
                                     (the paper has none): for measuring
                                     what the scaling costs.  Matrices whose
                                     entries lie outside about 2^-500 ..
                                     2^+300 may then lose accuracy or
                                     overflow */
#define SYEV3_FLAGS_ALL 63u

/* error codes */
#define SYEV3_OK 0
#define SYEV3_E_N (-1)        /* n < 0, or n too large for the layout */
#define SYEV3_E_NULL (-2)     /* A or lambda is NULL (with n > 0) */
#define SYEV3_E_DTYPE (-3)    /* unknown dtype, or a flag the dtype lacks */
#define SYEV3_E_LAYOUT (-4)   /* unknown layout, or bad ld */
#define SYEV3_E_ALIAS (-5)    /* an output overlaps the input or another
                                 output */
#define SYEV3_E_HIP (-6)      /* the HIP runtime refused the launch */
#define SYEV3_E_FLAGS (-7)    /* unknown flag bits */
#define SYEV3_E_BUDGET (-8)   /* server: request larger than the HBM budget */
#define SYEV3_E_AGAIN (-9)    /* server: no room now; retry after a release */
#define SYEV3_E_STATE (-10)   /* server: bad handle or request state */
#define SYEV3_E_TIMEOUT (-11) /* server: wait timed out */
#define SYEV3_E_NOMEM (-12)   /* server: host memory could not be allocated */
#define SYEV3_E_SEGMENTS (-13) /* more segments than the fixed table holds */

/*
 * batched_syev3 -- eigenvalues (and eigenvectors if V != NULL) of n
 * symmetric 3x3 matrices in structure-of-arrays layout with ld = n.
 * Same as batched_syev3_ex(n, A, 0, SYEV3_SOA, lambda, V, dtype, 0, stream).
 */
int batched_syev3(int64_t n, const void* A_upper6, void* lambda, void* V,
                  int dtype, hipStream_t stream);

/*
 * batched_syev3_ex -- full form: any layout, plane stride ld (SoA), flags.
 */
int batched_syev3_ex(int64_t n, const void* A, int64_t ld, int layout,
                     void* lambda, void* V, int dtype, uint32_t flags,
                     hipStream_t stream);

/*
 * batched_syev3_strided -- structure-of-arrays with a plane stride of its own
 * for each array: entry k of matrix i is A[k*lda + i], eigenvalue j is
 * lambda[j*ldl + i], row r of eigenvector c is V[(3*r + c)*ldv + i].  Each
 * stride is >= n (0 means n).  The arithmetic is that of batched_syev3_ex,
 * so the results are bitwise the same for any strides.
 *
 * Separate strides let a caller solve planes that live in buffers of their
 * own (rows of wider arrays, outputs written into a larger result set)
 * without copies.  Performance note: the 18 planes are streamed together,
 * each wavefront touching all of them at the same element offset, so how
 * fast a very large batch runs depends on which HBM channels the planes'
 * physical pages share.  On an MI355X a 2^28-matrix FP64 solve took 6.2 to
 * 8.3 ms from one allocation to the next (the AoS layout, three streams,
 * 6.4 to 6.9 ms); within one allocation, strides 32.5 KiB longer than n
 * were as fast or up to 7% slower.
 * Arrays whose plane ranges interleave are refused (SYEV3_E_ALIAS) even
 * when their planes do not overlap.  Errors as batched_syev3_ex.
 */
int batched_syev3_strided(int64_t n, const void* A, int64_t lda, void* lambda,
                          int64_t ldl, void* V, int64_t ldv, int dtype,
                          uint32_t flags, hipStream_t stream);

/*
 * batched_syev3_inplace -- for callers that keep full 3x3 matrices (one per
 * finite element, say): A is n x 9 row-major (SYEV3_AOS9) and is overwritten
 * by the eigenvectors (column c of each 3x3 is eigenvector c); lambda is n x 3.
 * Same as batched_syev3_ex(n, A, 0, SYEV3_AOS9, lambda, A, dtype, 0, stream).
 */
int batched_syev3_inplace(int64_t n, void* A, void* lambda, int dtype,
                          hipStream_t stream);

/*
 * batched_syev3_info -- batched_syev3_ex that also writes, per matrix,
 * info[i] = branch | (iterations for mu) << 8 | (iterations for nu) << 16,
 * branch: 0 zero matrix, 1 non-finite input, 2 diagonal arrow (h negligible),
 * 3 deflated (Sec. 1.1), 4 ordered and reduced (Sec. 1.2); iterations are the
 * spectral-function evaluations of the zero finder (Sec. 1.4).  info is
 * device memory of n int32 values.  Used to measure iteration counts.
 */
int batched_syev3_info(int64_t n, const void* A, int64_t ld, int layout,
                       void* lambda, void* V, int dtype, uint32_t flags,
                       int32_t* info, hipStream_t stream);

/*
 * syev3_stream_reference -- measurement aid, not a solver: reads the 6
 * input planes and writes the 3 + 9 output planes (V may be NULL) exactly
 * as batched_syev3 does in SoA layout with ld = n, with trivial arithmetic
 * in between, its workgroups in launch order.  A yardstick for the solver's
 * memory traffic, not a bound: the solver orders its workgroups by XCD for
 * large batches and can run faster.  Same argument rules as batched_syev3,
 * and n at most 2^31 (one launch; SYEV3_E_N above).
 */
int syev3_stream_reference(int64_t n, const void* A_upper6, void* lambda, void* V,
                           int dtype, hipStream_t stream);

/*
 * syev3_stream_probe -- measurement aid, not a solver: the loads and/or the
 * stores of the SoA solve (ld = n) with trivial arithmetic, for measuring
 * what HBM sustains for each part of this traffic on the device.  mode is
 * a bitwise OR of SYEV3_PROBE_READ (read the 6 input planes),
 * SYEV3_PROBE_WRITE (write the 3 + 9 output planes; V may be NULL) and
 * SYEV3_PROBE_XCD_ORDER (run the workgroups in the solver's XCD-chunked
 * order; else launch order), with READ or WRITE or both.  A read-only probe
 * writes nothing for finite input (its one store is taken only for a NaN
 * sum).  syev3_stream_reference is mode READ | WRITE.  Same argument rules
 * as syev3_stream_reference; SYEV3_E_FLAGS for another mode.
 */
#define SYEV3_PROBE_READ 1u
#define SYEV3_PROBE_WRITE 2u
#define SYEV3_PROBE_XCD_ORDER 4u
int syev3_stream_probe(int64_t n, const void* A_upper6, void* lambda, void* V, int dtype,
                       uint32_t mode, hipStream_t stream);

/* Text for an error code (static storage). */
const char* syev3_strerror(int code);

/* Library version, major*10000 + minor*100 + patch. */
int syev3_version(void);

/*
 * ------------------------------------------------------------------------
 * Serving: continuous batching of independent requests.
 *
 * A server owns one device pool of `hbm_budget_bytes`.  A client asks for a
 * request of n matrices of a dtype (syev3_server_acquire); the server admits
 * it if its input and output buffers fit in the pool and a request slot is
 * free, and returns device pointers into the pool (SoA layout, ld = n).  The
 * client writes A (on any stream; it must be complete before submit) and
 * calls syev3_server_submit.  A scheduler thread gathers every submitted
 * request into the next tick: one launch of a kernel that reads a device
 * table of the tick's requests (mixed dtypes) and solves them with the
 * same per-matrix arithmetic as batched_syev3, so each result is bitwise the
 * same alone and in any mix.  Up to `max_inflight_ticks` ticks run at once on
 * separate streams, so requests that arrive while others are on the GPU start
 * without waiting for them.  Completion is detected by events; then
 * syev3_server_poll reports the request done and its outputs are readable.
 * syev3_server_release returns the request's memory to the pool, which admits
 * waiting requests.  A tick is the table's copy and the kernel, replayed
 * from a HIP graph captured once per tick slot (use_graphs, the default) or
 * launched directly.
 * ------------------------------------------------------------------------
 */
typedef struct syev3_server syev3_server;

/* Largest accepted syev3_server_opts.max_requests. */
#define SYEV3_SERVER_MAX_REQUESTS 65536
/* Largest accepted syev3_server_opts.max_segments_per_tick. */
#define SYEV3_SERVER_MAX_SEGMENTS 1024

typedef struct {
  uint64_t hbm_budget_bytes;   /* device pool size (request buffers), >= 256 */
  int32_t max_requests;        /* request slots (admitted, not released),
                                  1 .. SYEV3_SERVER_MAX_REQUESTS */
  int32_t max_inflight_ticks;  /* ticks on the GPU at once (streams), 1 .. 64 */
  int32_t max_segments_per_tick; /* requests per tick,
                                    1 .. SYEV3_SERVER_MAX_SEGMENTS */
  int32_t grid_blocks;         /* most workgroups of a tick's launch, at
                                  most 2^24 (beyond it they stride over the
                                  tick's tiles of 256 matrices); 0 = one per
                                  tile, up to 2^24 */
  int32_t use_graphs;          /* 1: launch ticks through captured graphs
                                  (each tick sets the kernel node's grid);
                                  0: launch the table copy and the kernel */
} syev3_server_opts;

typedef struct {
  void* A;        /* device, 6 planes of n (SoA, ld = n), dtype elements */
  void* lambda;   /* device, 3 planes of n */
  void* V;        /* device, 9 planes of n, or NULL if vals-only */
  int64_t n;
  int32_t dtype;
} syev3_request_buffers;

typedef struct {
  int64_t submitted;
  int64_t completed;           /* requests done with their results written */
  int64_t ticks;
  int64_t matrices_completed;  /* matrices of the completed requests */
  uint64_t pool_bytes_in_use, pool_bytes_peak;
  int64_t acquire_rejections;  /* acquire calls answered SYEV3_E_AGAIN */
  int32_t inflight_ticks_peak;
  int32_t segments_per_tick_peak;
  double busy_seconds;         /* wall time with at least one tick on the GPU */
  int64_t queue_depth;         /* requests submitted and not yet in a tick */
  int64_t queue_depth_peak;
  int64_t failed;              /* requests done without results (their tick
                                  could not be launched or did not finish) */
} syev3_server_stats;

/* Defaults: 64 GiB pool, 4096 slots, 4 ticks in flight, 256 segments/tick,
 * one workgroup per tile, graphs on (launched directly instead, the table
 * copy and the kernel complete 15-20 us sooner at low load, with the same
 * throughput at saturation). */
void syev3_server_default_opts(syev3_server_opts* opts);

/* Create a server on the current device.  Allocates the pool and starts the
 * scheduler thread.  *out receives the handle (NULL on failure).  Returns
 * SYEV3_E_N for an option outside its range, SYEV3_E_BUDGET if the pool
 * cannot be allocated on the device, SYEV3_E_NOMEM if host memory runs out,
 * SYEV3_E_HIP for another HIP failure (streams, events, graphs). */
int syev3_server_create(const syev3_server_opts* opts, syev3_server** out);

/* Stop the scheduler (after the queued and in-flight ticks finish) and free
 * everything.  No other call on this server may be in progress (a thread
 * blocked in syev3_server_wait, say) or follow. */
int syev3_server_destroy(syev3_server* s);

/* Admit a request of n matrices (vals+vecs if want_vectors) of dtype.
 * Returns a request id >= 0 and fills *bufs, or SYEV3_E_AGAIN if the pool or
 * the slots are full now, or SYEV3_E_BUDGET if it can never fit,
 * SYEV3_E_NOMEM if host memory for the pool's bookkeeping runs out (nothing
 * is admitted then). */
int64_t syev3_server_acquire(syev3_server* s, int64_t n, int dtype,
                             int want_vectors, syev3_request_buffers* bufs);

/* Admit a request whose input stays where the caller keeps it: A is device
 * memory holding 6 planes of n entries with plane stride lda >= n (SoA, the
 * request's dtype), read by the request's tick and not copied.  Only the
 * outputs take pool memory (bufs->lambda, bufs->V: planes of n); bufs->A is
 * A.  The caller keeps A valid and unchanged until the request is done.
 * Submit it with syev3_server_submit (not syev3_server_submit_host).
 * SYEV3_E_NULL for a NULL A, SYEV3_E_LAYOUT for lda < n; otherwise as
 * syev3_server_acquire. */
int64_t syev3_server_acquire_view(syev3_server* s, int64_t n, int dtype,
                                  int want_vectors, const void* A, int64_t lda,
                                  syev3_request_buffers* bufs);

/* Queue an admitted request for the next tick.  Its A must be complete
 * when `ready` (a hipEvent_t, or NULL) has completed: the tick waits for it
 * on the device, the host does not block.  The wait on `ready` is enqueued
 * here, on a stream of the server, behind which the server records an event
 * of its own that the tick waits on; so once this call returns the caller
 * may destroy `ready` or record it again.  NULL: A is complete now.
 * SYEV3_E_HIP if the wait could not be enqueued (the request stays admitted
 * and may be submitted again). */
int syev3_server_submit(syev3_server* s, int64_t request, hipEvent_t ready);

/* Host-staged submission (not for a request admitted as a view, which gives
 * SYEV3_E_STATE): the request's input is copied from host memory
 * host_A (6 planes of n, SoA, the request's dtype) to its device buffer
 * before its tick, and the outputs are copied back to host_lambda (3 x n)
 * and host_V (9 x n, or NULL) after it.  The copies run in order on the
 * tick's own stream, before and after its kernel; ticks run on separate
 * streams, so one tick's copies overlap other ticks' kernels.  The host memory must stay valid and untouched until
 * the request completes; it should be pinned (hipHostMalloc), otherwise the
 * copies do not overlap.  Completion (poll/wait) includes the copy back. */
int syev3_server_submit_host(syev3_server* s, int64_t request, const void* host_A,
                             void* host_lambda, void* host_V);

/* 1 if the request's results are complete, 0 if not yet, < 0 on error.
 * If done and latency_s is not NULL, it receives submit-to-completion time
 * in seconds. */
int syev3_server_poll(syev3_server* s, int64_t request, double* latency_s);

/* Block until the request completes or timeout_s passes (< 0, or above 1e9
 * seconds: no limit; NaN: SYEV3_E_N).
 * Returns 1 when complete, SYEV3_E_TIMEOUT, SYEV3_E_HIP if its tick failed,
 * or SYEV3_E_STATE if the id is stale, which includes a release of the
 * request by another thread during the wait. */
int syev3_server_wait(syev3_server* s, int64_t request, double timeout_s,
                      double* latency_s);

/* Return the request's buffers to the pool (after it completed).
 * SYEV3_E_NOMEM if host memory for the pool's bookkeeping runs out; the
 * request is then still held, and the call may be repeated. */
int syev3_server_release(syev3_server* s, int64_t request);

int syev3_server_get_stats(syev3_server* s, syev3_server_stats* out);

/* ------------------------------------------------------------------------
 * A tick without the server, allocating nothing
 * ------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Solves
 * nseg independent requests of different sizes and forms in one launch of
 * the kernel that runs a server's ticks, on buffers the caller owns.  That
 * kernel reads a table of the requests; a server allocates one per tick
 * slot in syev3_server_create, this call uses a fixed array of the library
 * in each GPU's memory instead (room for SYEV3_SEGMENTS_MAX segments, about
 * 56 KiB, held until the process ends) and makes no hipMalloc, hipFree or
 * other allocating call.  Results are bitwise those of the same requests
 * served by a server or solved by batched_syev3_strided.
 *
 * segs[i]: n >= 0 matrices of dtype SYEV3_F64 or SYEV3_F32_REFINE; A holds
 * 6 SoA planes at plane stride lda elements (0 means n, else >= n); lambda
 * 3 planes and V 9 planes (NULL: eigenvalues only) at plane stride n; flags
 * as for batched_syev3_ex.  All device memory of the stream's device.
 * Segments with n == 0 are skipped.  The table is built from segs on the
 * host and copied to the device from pageable host memory, which HIP does
 * synchronously with respect to the host: segs may be reused as soon as
 * the call returns.  The solve is enqueued on `stream`.
 *
 * Every call on one GPU uses that GPU's one table, which keeps the last
 * call's contents (each call writes all of the table it reads).  Calls in
 * one stream's order are safe; calls that overlap on one GPU (on streams
 * not ordered with each other) race, and a kernel may then read a table
 * that another call has overwritten.  The table's device address
 * is looked up at the first call on each GPU and kept: after a
 * hipDeviceReset of that GPU the call must not be used again in the
 * process.
 *
 * Returns SYEV3_OK (nothing is enqueued when every n is 0); SYEV3_E_SEGMENTS
 * for nseg < 0 or nseg > SYEV3_SEGMENTS_MAX; SYEV3_E_NULL for segs == NULL
 * with nseg > 0; per segment the errors of batched_syev3_strided, with
 * SYEV3_F32 answered SYEV3_E_DTYPE; SYEV3_E_ALIAS also when an output of
 * one segment overlaps an input or an output of another; SYEV3_E_HIP when
 * the copy or the launch fails.  Nothing is enqueued on an argument error.
 */
#define SYEV3_SEGMENTS_MAX SYEV3_SERVER_MAX_SEGMENTS

typedef struct {
  int64_t n;
  const void* A;   /* 6 planes, plane stride lda */
  int64_t lda;
  void* lambda;    /* 3 planes, plane stride n */
  void* V;         /* 9 planes, plane stride n, or NULL */
  int32_t dtype;
  uint32_t flags;
} syev3_segment;

int syev3_solve_segments_noalloc(int32_t nseg, const syev3_segment* segs,
                                 hipStream_t stream);

/*
 * Load generator for a server (benchmark support).  Open loop (qps > 0):
 * requests arrive as a Poisson process of rate qps for duration_s seconds.
 * Closed loop (qps == 0): closed_concurrency requests are kept in flight, a
 * new one arriving when one completes, for duration_s seconds.  Each has
 * n = floor(2^U(0, max_log2_n)) matrices (at most src_n) and is FP32-storage
 * with probability frac_f32, else FP64.  Its input is copied on the device
 * from a source pool (SoA, ld = src_n, one pool per dtype) at a random
 * offset, then submitted; a request that does not fit waits (FIFO) until
 * releases make room.  Completed requests are released at once.  Latency is
 * measured from arrival (so it includes waiting for admission) to the
 * scheduler's observation of the tick's completion event.
 */
typedef struct {
  double qps;            /* > 0 (at most 1e8): open loop (Poisson); 0: closed
                            loop */
  int32_t closed_concurrency; /* closed loop: requests kept in flight,
                                  1 to 2^20 */
  double duration_s;     /* > 0, at most 1e6; open loop: qps * duration_s at
                            most 1e8 arrivals */
  double max_log2_n;     /* 0 to 40 */
  double frac_f32;
  uint64_t seed;
  const void* src_f64;   /* 6 planes of src_n doubles (device, or pinned
                            host memory when host_staged) */
  const void* src_f32;   /* 6 planes of src_n floats (likewise) */
  int64_t src_n;
  int32_t want_vectors;
  int32_t host_staged;   /* 1: submit through syev3_server_submit_host; a
                            request's input is the first 6 n values of the
                            (host) source, its results go to the host sink,
                            which every request overwrites */
  void* sink;            /* host_staged: pinned host memory of at least
                            12 * 2^max_log2_n * 8 bytes for the results */
  int32_t input_views;   /* 1 (device sources only): each request reads its
                            window of the source pool in place
                            (syev3_server_acquire_view); nothing is copied
                            and only the outputs take pool memory */
} syev3_loadgen_opts;

typedef struct {
  int64_t requests, matrices;
  double elapsed_s;              /* first arrival to last completion */
  double matrices_per_s, requests_per_s;
  double lat_p50_s, lat_p90_s, lat_p99_s, lat_p999_s, lat_max_s, lat_mean_s;
  double admit_wait_mean_s;      /* arrival to admission */
  int64_t ticks;
  double mean_segments_per_tick;
  int32_t inflight_ticks_peak;
  uint64_t pool_bytes_peak;
} syev3_loadgen_result;

/* Runs the load on s (the caller's own requests may share it) and fills
 * *out.  Returns SYEV3_OK; SYEV3_E_N for options out of range; SYEV3_E_HIP if
 * a copy, an event or a tick failed (the run stops at the first error, and
 * every request it admitted is waited for and released before the return);
 * SYEV3_E_NOMEM if host memory runs out. */
int syev3_server_loadgen(syev3_server* s, const syev3_loadgen_opts* opts,
                         syev3_loadgen_result* out);

#ifdef __cplusplus
}
#endif

#endif /* SYEV3_H */
