"""Python handle on the library's continuous-batching server (C ABI
syev3_server_*).  The scheduling, pool, graphs and load generator are native;
this module only marshals arguments."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import RequestBuffers, ServerOpts, ServerStats


class LoadgenOpts(ctypes.Structure):
    _fields_ = [("qps", ctypes.c_double), ("closed_concurrency", ctypes.c_int32),
                ("duration_s", ctypes.c_double),
                ("max_log2_n", ctypes.c_double), ("frac_f32", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("src_f64", ctypes.c_void_p),
                ("src_f32", ctypes.c_void_p), ("src_n", ctypes.c_int64),
                ("want_vectors", ctypes.c_int32), ("host_staged", ctypes.c_int32),
                ("sink", ctypes.c_void_p), ("input_views", ctypes.c_int32)]


class LoadgenResult(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("matrices", ctypes.c_int64),
                ("elapsed_s", ctypes.c_double), ("matrices_per_s", ctypes.c_double),
                ("requests_per_s", ctypes.c_double),
                ("lat_p50_s", ctypes.c_double), ("lat_p90_s", ctypes.c_double),
                ("lat_p99_s", ctypes.c_double), ("lat_p999_s", ctypes.c_double),
                ("lat_max_s", ctypes.c_double), ("lat_mean_s", ctypes.c_double),
                ("admit_wait_mean_s", ctypes.c_double), ("ticks", ctypes.c_int64),
                ("mean_segments_per_tick", ctypes.c_double),
                ("inflight_ticks_peak", ctypes.c_int32),
                ("pool_bytes_peak", ctypes.c_uint64)]


def _bind(L):
    if getattr(L, "_serve_bound", False):
        return L
    L.syev3_server_loadgen.argtypes = [ctypes.c_void_p, ctypes.POINTER(LoadgenOpts),
                                       ctypes.POINTER(LoadgenResult)]
    L.syev3_server_loadgen.restype = ctypes.c_int
    L.syev3_server_submit_host.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]
    L.syev3_server_submit_host.restype = ctypes.c_int
    L.syev3_server_acquire_view.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.POINTER(RequestBuffers)]
    L.syev3_server_acquire_view.restype = ctypes.c_int64
    L._serve_bound = True
    return L


def check_host_buffers(n, dtype, host_A, host_lam, host_V=None):
    """The host buffers of a host-staged request of n matrices: contiguous
    CPU tensors of the request's dtype holding at least 6n, 3n and 9n
    values (the server copies exactly that many in and out)."""
    tdt = torch.float64 if dtype == _lib.F64 else torch.float32
    for name, t, k in (("host_A", host_A, 6), ("host_lam", host_lam, 3), ("host_V", host_V, 9)):
        if t is None:
            if name == "host_V":
                continue
            raise ValueError(f"{name} is required")
        if t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CPU tensor")
        if t.dtype != tdt:
            raise ValueError(f"{name} must be {tdt} for this request, got {t.dtype}")
        if t.numel() < k * n:
            raise ValueError(f"{name} holds {t.numel()} values; the request needs {k * n}")


def check_loadgen_sources(src_f64, src_f32, max_log2_n, sink):
    """Sources of the load generator: (6, src_n) float64 and float32 tensors
    with the same src_n, contiguous, both on the GPU (inputs copied on the
    device) or both in host memory with a host sink of at least
    12 * 2^max_log2_n doubles (host-staged).  The native generator reads
    them through raw pointers, so a short or mistyped source would be read
    out of bounds."""
    for name, t, dt in (("src_f64", src_f64, torch.float64), ("src_f32", src_f32, torch.float32)):
        if t.dim() != 2 or t.shape[0] != 6 or not t.is_contiguous() or t.dtype != dt:
            raise ValueError(f"{name} must be a contiguous (6, src_n) {dt} tensor")
    if src_f64.shape[1] != src_f32.shape[1] or src_f64.shape[1] < 1:
        raise ValueError("src_f64 and src_f32 must have the same src_n >= 1")
    if src_f64.is_cuda != src_f32.is_cuda:
        raise ValueError("both sources on the GPU, or both in host memory")
    if not src_f64.is_cuda:
        if sink is None or sink.is_cuda or not sink.is_contiguous():
            raise ValueError("host-staged load needs a contiguous pinned host sink")
        if 2.0 ** max_log2_n > src_f64.shape[1]:
            raise ValueError("host-staged requests take their input from the first 6n "
                             "source values: src_n must be >= 2^max_log2_n")
        need = 12 * int(2.0 ** max_log2_n) * 8
        if sink.numel() * sink.element_size() < need:
            raise ValueError(f"sink holds {sink.numel() * sink.element_size()} bytes; "
                             f"requests up to 2^max_log2_n matrices need {need}")


class Request:
    """An admitted request: device tensors over the server's pool (A is the
    caller's own tensor for a request admitted as a view)."""

    def __init__(self, server, rid, bufs: RequestBuffers, dtype, A=None):
        self.server, self.id, self.n = server, rid, bufs.n
        self.dtype = bufs.dtype
        tdt = torch.float64 if bufs.dtype == _lib.F64 else torch.float32
        es = 8 if tdt == torch.float64 else 4
        dev = server.device
        # a view's input: the caller's tensor, held until release
        self.A = A if A is not None else _tensor_at(bufs.A, (6, bufs.n), tdt, es, dev)
        self.lam = _tensor_at(bufs.lam, (3, bufs.n), tdt, es, dev)
        self.V = _tensor_at(bufs.V, (9, bufs.n), tdt, es, dev) if bufs.V else None
        self.host_buffers = None  # held from a host-staged submit to release


def _tensor_at(ptr, shape, dtype, esize, dev):
    """A torch view of memory owned by the server on device `dev` (no
    copy)."""
    numel = shape[0] * shape[1]
    class _Holder:
        __cuda_array_interface__ = {
            "shape": shape, "typestr": "<f8" if esize == 8 else "<f4",
            "data": (int(ptr), False), "version": 3, "strides": None}
    return torch.as_tensor(_Holder(), device=f"cuda:{dev}").view(shape) if numel else \
        torch.empty(shape, dtype=dtype, device=f"cuda:{dev}")


class Server:
    def __init__(self, hbm_budget_bytes=64 << 30, max_requests=4096,
                 max_inflight_ticks=4, max_segments_per_tick=256, grid_blocks=0,
                 use_graphs=True):
        self.L = _bind(_lib.lib())
        o = ServerOpts()
        self.L.syev3_server_default_opts(ctypes.byref(o))
        o.hbm_budget_bytes = hbm_budget_bytes
        o.max_requests = max_requests
        o.max_inflight_ticks = max_inflight_ticks
        o.max_segments_per_tick = max_segments_per_tick
        o.grid_blocks = grid_blocks
        o.use_graphs = 1 if use_graphs else 0
        h = ctypes.c_void_p()
        # the server lives on the device current now: its pool, streams and
        # requests' tensors
        self.device = torch.cuda.current_device()
        _lib.check(self.L.syev3_server_create(ctypes.byref(o), ctypes.byref(h)),
                   "syev3_server_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.check(self.L.syev3_server_destroy(self.h), "syev3_server_destroy")
            self.h = None

    def __del__(self):
        # a server dropped without close(): stop its scheduler thread while
        # the runtime is still up (best effort; close() is the way)
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def acquire(self, n, dtype=_lib.F64, vectors=True):
        """Request or None when the pool/slots are full now (E_AGAIN)."""
        b = RequestBuffers()
        rid = self.L.syev3_server_acquire(self.h, n, dtype, 1 if vectors else 0,
                                          ctypes.byref(b))
        if rid == _lib.E_AGAIN:
            return None
        _lib.check(rid, "syev3_server_acquire")
        return Request(self, rid, b, dtype)

    def acquire_view(self, A: torch.Tensor, vectors=True):
        """Admit a request whose input is the caller's tensor A, (6, n) with
        unit column stride and row stride >= n, on the server's device,
        float64 (FP64) or float32 (FP32 storage + refinement).  A is read in
        place by the tick (not copied); only the outputs take pool memory.
        The request holds A until release.  None when the pool or the slots
        are full now."""
        from . import _soa_geometry
        if not A.is_cuda or A.device != torch.device(f"cuda:{self.device}"):
            raise ValueError(f"A must be on cuda:{self.device}, the server's device")
        n, lda = _soa_geometry(A)
        if n == 0:
            raise ValueError("a request holds at least one matrix")
        dtype = {torch.float64: _lib.F64, torch.float32: _lib.F32_REFINE}.get(A.dtype)
        if dtype is None:
            raise TypeError(f"A must be float64 or float32, got {A.dtype}")
        b = RequestBuffers()
        rid = self.L.syev3_server_acquire_view(self.h, n, dtype, 1 if vectors else 0,
                                               A.data_ptr(), lda, ctypes.byref(b))
        if rid == _lib.E_AGAIN:
            return None
        _lib.check(rid, "syev3_server_acquire_view")
        return Request(self, rid, b, dtype, A=A)

    def submit(self, req: Request, ready_event=None):
        """Queue req; its tick waits on the device for ready_event (a
        torch.cuda.Event recorded after req.A was written).  The server takes
        its own mark of the event during this call, so the event may be
        dropped or recorded again as soon as submit returns."""
        ev = ctypes.c_void_p(ready_event.cuda_event if ready_event is not None else 0)
        _lib.check(self.L.syev3_server_submit(self.h, req.id, ev), "syev3_server_submit")

    def submit_host(self, req: Request, host_A, host_lam, host_V=None):
        """Host-staged submission: host_A (6, n), host_lam (3, n), host_V
        (9, n) are CPU tensors of the request's dtype, preferably pinned; the
        server copies A in before the tick and the results out after it."""
        check_host_buffers(req.n, req.dtype, host_A, host_lam, host_V)
        _lib.check(self.L.syev3_server_submit_host(
            self.h, req.id, host_A.data_ptr(), host_lam.data_ptr(),
            host_V.data_ptr() if host_V is not None else None), "syev3_server_submit_host")
        # the copies run when the tick does: keep the buffers alive till release
        req.host_buffers = (host_A, host_lam, host_V)

    def poll(self, req):
        lat = ctypes.c_double()
        rc = _lib.check(self.L.syev3_server_poll(self.h, req.id, ctypes.byref(lat)),
                        "syev3_server_poll")
        return lat.value if rc == 1 else None

    def wait(self, req, timeout_s=-1.0):
        lat = ctypes.c_double()
        _lib.check(self.L.syev3_server_wait(self.h, req.id, timeout_s, ctypes.byref(lat)),
                   "syev3_server_wait")
        return lat.value

    def release(self, req):
        _lib.check(self.L.syev3_server_release(self.h, req.id), "syev3_server_release")
        req.host_buffers = None

    def stats(self) -> dict:
        s = ServerStats()
        _lib.check(self.L.syev3_server_get_stats(self.h, ctypes.byref(s)), "stats")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def loadgen(self, src_f64, src_f32, qps, duration_s, max_log2_n=20.0,
                frac_f32=0.5, seed=0, vectors=True, concurrency=0, sink=None,
                input_views=False) -> dict:
        """qps > 0: open-loop Poisson arrivals; qps == 0: closed loop with
        `concurrency` requests in flight.  Sources on the device: inputs are
        copied on the device, or with input_views read in place (each request
        a view of its window of the source).  Sources in (pinned) host memory
        together with a host `sink`: host-staged requests."""
        check_loadgen_sources(src_f64, src_f32, max_log2_n, sink)
        staged = not src_f64.is_cuda
        if staged and input_views:
            raise ValueError("input views need device sources")
        o = LoadgenOpts(qps=qps, closed_concurrency=concurrency,
                        duration_s=duration_s, max_log2_n=max_log2_n,
                        frac_f32=frac_f32, seed=seed, src_f64=src_f64.data_ptr(),
                        src_f32=src_f32.data_ptr(), src_n=src_f64.shape[-1],
                        want_vectors=1 if vectors else 0, host_staged=1 if staged else 0,
                        sink=sink.data_ptr() if sink is not None else None,
                        input_views=1 if input_views else 0)
        r = LoadgenResult()
        _lib.check(self.L.syev3_server_loadgen(self.h, ctypes.byref(o), ctypes.byref(r)),
                   "syev3_server_loadgen")
        return {f: getattr(r, f) for f, _ in r._fields_}


def bench(duration_s=4.0, budget_bytes=64 << 30, seed=3):
    """Serving measurement: request sizes 2^U(0,20) from the stress mix, 50%
    FP64 / 50% FP32-storage, eigenvalues and vectors.  Requests read their
    input in place from a resident pool (input views): only their outputs
    take pool memory, so the client side costs little and the figures are
    the server's.
      * saturation: closed loop, 256 requests in flight;
      * open-loop Poisson arrivals at 50% and 80% of that rate;
      * a low fixed rate (2000 requests/s, about one request per tick): the
        latency floor of the path;
      * budget pressure: a closed loop deep enough (16384 requests) that the
        64 GiB pool fills and admissions are refused, with p50/p99 there;
      * for comparison, requests whose input is copied into the pool on the
        device (64 in flight) and host-staged requests (pinned host memory
        in and out, 64 in flight);
      * ticks launched directly instead of through their captured HIP
        graphs, at saturation and at 2000 requests/s."""
    from . import gen
    src_n = 1 << 20
    A, _ = gen.stress_mix(src_n, seed=seed, device="cuda")
    Af = A.float().contiguous()
    torch.cuda.synchronize()
    out = {"workload": "Poisson arrivals; n = floor(2^U(0,20)) stress-mix matrices per "
                       "request; 50% FP64 / 50% FP32-storage; vals+vecs; inputs read in place "
                       "from a resident pool (views) unless stated; HBM budget "
                       f"{budget_bytes / 2**30:.0f} GiB",
           "latency": "arrival to observed completion (includes waiting for admission)"}
    with Server(hbm_budget_bytes=budget_bytes) as srv:
        sat = srv.loadgen(A, Af, qps=0.0, concurrency=256, duration_s=min(2.0, duration_s),
                          seed=seed, input_views=True)
        out["closed_loop_256_in_flight"] = sat
        rate = sat["requests_per_s"]
        for rho in (0.5, 0.8):
            r = srv.loadgen(A, Af, qps=rho * rate, duration_s=duration_s, seed=seed + 1,
                            input_views=True)
            r["offered_qps"] = rho * rate
            out[f"open_loop_{int(rho * 100)}pct"] = r
        r = srv.loadgen(A, Af, qps=2000.0, duration_s=min(1.0, duration_s), seed=seed + 3,
                        input_views=True)
        r["offered_qps"] = 2000.0
        out["open_loop_2000qps"] = r
        r = srv.loadgen(A, Af, qps=0.0, concurrency=64, duration_s=min(1.0, duration_s),
                        seed=seed + 4)
        out["copied_inputs_closed_loop_64_in_flight"] = r
        # host-staged: inputs from pinned host memory, results back to it
        m = 1 << 20
        hA = A[:, :m].cpu().contiguous().pin_memory()
        hAf = Af[:, :m].cpu().contiguous().pin_memory()
        sink = torch.empty(12 * m, dtype=torch.float64).pin_memory()
        r = srv.loadgen(hA, hAf, qps=0.0, concurrency=64, duration_s=min(2.0, duration_s),
                        seed=seed + 2, sink=sink)
        out["host_staged_closed_loop_64_in_flight"] = r
        out["server_stats"] = srv.stats()
    # a server with room for enough requests to fill its pool
    with Server(hbm_budget_bytes=budget_bytes, max_requests=16384) as srv:
        r = srv.loadgen(A, Af, qps=0.0, concurrency=16384, duration_s=min(2.0, duration_s),
                        seed=seed + 5, input_views=True)
        st = srv.stats()
        r["acquire_rejections"] = st["acquire_rejections"]
        r["pool_bytes_peak_over_budget"] = st["pool_bytes_peak"] / budget_bytes
        out["budget_pressure_closed_loop_16384"] = r
    # the same ticks launched directly (the table copy and the kernel) instead
    # of through their captured graphs, at saturation and at the low rate
    with Server(hbm_budget_bytes=budget_bytes, use_graphs=False) as srv:
        r = srv.loadgen(A, Af, qps=0.0, concurrency=256, duration_s=min(2.0, duration_s),
                        seed=seed, input_views=True)
        out["direct_closed_loop_256_in_flight"] = r
        r = srv.loadgen(A, Af, qps=2000.0, duration_s=min(1.0, duration_s), seed=seed + 3,
                        input_views=True)
        r["offered_qps"] = 2000.0
        out["direct_open_loop_2000qps"] = r
    return out
