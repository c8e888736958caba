"""Serving: continuous batching through the library's server (C ABI
syev3_server_*).  Each request's result must be bitwise the one a separate
batched_syev3 call gives on the same input, whatever shares its tick;
admission must respect the HBM budget; graph-launched ticks must stay
correct over many replays with other GPU work in between."""
import numpy as np
import pytest
import torch

import paper_1806_06698_amd as s3
from gpu_common import check_vs_oracle, need_gpu
from paper_1806_06698_amd import gen, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def source():
    A, _ = gen.stress_mix(1 << 21, seed=7, device="cuda")
    return A, A.float().contiguous()


def _fill(req, src, off):
    """Copy n source matrices into the request's input (on the current
    stream); returns the event that marks them ready."""
    n = req.n
    req.A.copy_(src[:, off:off + n])
    ev = torch.cuda.Event()
    ev.record()
    return ev


def _reference(req):
    lam, V = s3.syev3(req.A.clone(), vectors=req.V is not None)
    return lam, V


def _check_bitwise(req):
    lam, V = _reference(req)
    torch.cuda.synchronize()
    assert torch.equal(lam, req.lam), f"lambda differs for n={req.n}"
    if V is not None:
        assert torch.equal(V, req.V), f"V differs for n={req.n}"


def _check_oracle(req, sample=20_000, label="served"):
    """The served results themselves against the CPU oracle (the segment
    kernel is code of its own, so equality with the batched kernel alone
    would not show it right)."""
    check_vs_oracle(req.A, req.lam, req.V, f32=req.dtype == s3.F32_REFINE,
                    sample=sample, seed=req.n, label=f"{label} dtype={req.dtype}")


@pytest.mark.parametrize("use_graphs", [True, False])
def test_each_result_same_alone_and_in_the_mix(source, use_graphs):
    A64, A32 = source
    rng = np.random.default_rng(1)
    sizes = [1, 63, 64, 255, 256, 257, 1000, 4097, 50_000, 123_457, 1 << 20]
    with serve.Server(hbm_budget_bytes=2 << 30, use_graphs=use_graphs,
                      max_inflight_ticks=3) as srv:
        reqs = []
        for k, n in enumerate(sizes):
            dt = s3.F32_REFINE if k % 2 else s3.F64
            vec = k % 5 != 4
            r = srv.acquire(n, dt, vectors=vec)
            assert r is not None
            off = int(rng.integers(0, (1 << 21) - n))
            ev = _fill(r, A32 if dt == s3.F32_REFINE else A64, off)
            srv.submit(r, ev)
            reqs.append(r)
        for r in reqs:
            lat = srv.wait(r, timeout_s=60.0)
            assert lat >= 0.0
        for r in reqs:
            _check_bitwise(r)
            _check_oracle(r)
            srv.release(r)
        st = srv.stats()
        assert st["completed"] == len(sizes)
        assert st["pool_bytes_in_use"] == 0
        assert st["queue_depth"] == 0 and 1 <= st["queue_depth_peak"] <= len(sizes)


@pytest.mark.parametrize("use_graphs", [True, False])
def test_many_ticks_with_eager_work_between_replays(source, use_graphs):
    """Forty ticks of varying grids (one workgroup per tile: with graphs,
    each replay first sets the captured kernel node's grid), with the
    program's own eager work and a synchronisation between them."""
    A64, A32 = source
    rng = np.random.default_rng(2)
    scratch = torch.zeros(1 << 20, device="cuda")
    with serve.Server(hbm_budget_bytes=1 << 30, max_inflight_ticks=2,
                      use_graphs=use_graphs) as srv:
        for it in range(40):
            reqs = []
            for _ in range(int(rng.integers(1, 5))):
                n = int(2 ** rng.uniform(0, 16))
                dt = s3.F64 if rng.random() < 0.5 else s3.F32_REFINE
                r = srv.acquire(n, dt)
                ev = _fill(r, A64 if dt == s3.F64 else A32, int(rng.integers(0, 1 << 20)))
                srv.submit(r, ev)
                reqs.append(r)
            # the program's own eager work and a synchronisation between ticks
            scratch.add_(1.0).mul_(0.5)
            torch.cuda.synchronize()
            for r in reqs:
                srv.wait(r, timeout_s=60.0)
                _check_bitwise(r)
                srv.release(r)
        assert srv.stats()["ticks"] >= 40


def test_admission_by_budget():
    budget = 64 << 20
    with serve.Server(hbm_budget_bytes=budget, max_requests=64) as srv:
        with pytest.raises(s3.Syev3Error) as ei:
            srv.acquire(1 << 20, s3.F64)          # 151 MB > 64 MiB: never fits
        assert ei.value.code == -8
        held = []
        while True:
            r = srv.acquire(100_000, s3.F64)      # 14.4 MB each
            if r is None:
                break
            held.append(r)
        assert len(held) == 4                     # 4 * 14.4 MB fit in 64 MiB
        assert srv.stats()["acquire_rejections"] >= 1
        srv.release(held.pop())
        r = srv.acquire(100_000, s3.F64)
        assert r is not None
        held.append(r)
        for r in held:
            srv.release(r)
        assert srv.stats()["pool_bytes_in_use"] == 0


def test_request_state_errors(source):
    A64, _ = source
    with serve.Server(hbm_budget_bytes=64 << 20) as srv:
        r = srv.acquire(1000, s3.F64)
        with pytest.raises(s3.Syev3Error):
            srv.poll(r)                           # not submitted yet
        srv.submit(r, _fill(r, A64, 0))
        with pytest.raises(s3.Syev3Error):
            srv.submit(r)                         # twice
        srv.wait(r, 60.0)
        srv.release(r)
        with pytest.raises(s3.Syev3Error):
            srv.release(r)                        # released id is stale


def test_loadgen_short_run(source):
    A64, A32 = source
    with serve.Server(hbm_budget_bytes=4 << 30) as srv:
        res = srv.loadgen(A64[:, :1 << 18].contiguous(), A32[:, :1 << 18].contiguous(),
                          qps=2000.0, duration_s=0.5, max_log2_n=14, seed=5)
    print(res, flush=True)
    assert res["requests"] > 100
    assert 0 < res["lat_p50_s"] <= res["lat_p99_s"] <= res["lat_max_s"]
    assert res["matrices"] > 0 and res["ticks"] > 0


def test_host_staged_requests_match_the_device_path(source):
    A64, A32 = source
    with serve.Server(hbm_budget_bytes=1 << 30, max_inflight_ticks=3) as srv:
        reqs = []
        for k, n in enumerate([1, 300, 4097, 70_000, 200_001]):
            dt = s3.F64 if k % 2 == 0 else s3.F32_REFINE
            src = (A64 if dt == s3.F64 else A32)[:, 1000:1000 + n]
            tdt = torch.float64 if dt == s3.F64 else torch.float32
            hA = src.cpu().contiguous().pin_memory()
            hl = torch.empty((3, n), dtype=tdt).pin_memory()
            hV = torch.empty((9, n), dtype=tdt).pin_memory()
            r = srv.acquire(n, dt)
            srv.submit_host(r, hA, hl, hV)
            reqs.append((r, src.contiguous(), hl, hV))
        for r, src, hl, hV in reqs:
            srv.wait(r, timeout_s=60.0)
            lam, V = s3.syev3(src)
            torch.cuda.synchronize()
            assert torch.equal(lam.cpu(), hl) and torch.equal(V.cpu(), hV)
            check_vs_oracle(src, hl, hV, f32=r.dtype == s3.F32_REFINE, sample=20_000,
                            seed=r.n, label="host-staged")
            srv.release(r)


def test_host_staged_loadgen(source):
    A64, A32 = source
    m = 1 << 16
    hA = A64[:, :m].cpu().contiguous().pin_memory()
    hAf = A32[:, :m].cpu().contiguous().pin_memory()
    sink = torch.empty(12 * m, dtype=torch.float64).pin_memory()
    with serve.Server(hbm_budget_bytes=1 << 30) as srv:
        res = srv.loadgen(hA, hAf, qps=0.0, concurrency=16, duration_s=0.5,
                          max_log2_n=16, seed=9, sink=sink)
    print(res, flush=True)
    assert res["requests"] > 10 and res["lat_p99_s"] > 0


def test_concurrent_clients(source):
    """Four host threads use one server at once, each on its own stream:
    acquire (retrying while the small pool is full), fill, submit, wait,
    check, release.  Every result equals a separate batched solve of the
    same input bitwise, and the pool ends empty."""
    import threading
    import time
    A64, A32 = source
    per_thread, errors = 25, []

    def client(k, srv):
        try:
            rng = np.random.default_rng(100 + k)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for it in range(per_thread):
                    n = int(rng.integers(1, 20_000))
                    dt = s3.F64 if (it + k) % 2 == 0 else s3.F32_REFINE
                    vec = (it + k) % 3 != 0
                    deadline = time.monotonic() + 30.0
                    r = srv.acquire(n, dt, vectors=vec)
                    while r is None:
                        assert time.monotonic() < deadline, "admission starved"
                        time.sleep(0.0005)
                        r = srv.acquire(n, dt, vectors=vec)
                    off = int(rng.integers(0, (1 << 21) - n))
                    srv.submit(r, _fill(r, A32 if dt == s3.F32_REFINE else A64, off))
                    srv.wait(r, timeout_s=30.0)
                    lam, V = _reference(r)
                    stream.synchronize()
                    assert torch.equal(lam, r.lam), f"thread {k}: lambda differs, n={n}"
                    if vec:
                        assert torch.equal(V, r.V), f"thread {k}: V differs, n={n}"
                    srv.release(r)
        except Exception as exc:  # reported by the main thread
            errors.append(exc)

    # 6 MB: room for two of the largest FP64 requests with vectors at once
    with serve.Server(hbm_budget_bytes=6 << 20, max_requests=8) as srv:
        threads = [threading.Thread(target=client, args=(k, srv)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=90.0)
        assert not any(t.is_alive() for t in threads), "a client did not finish"
        assert not errors, errors[0]
        st = srv.stats()
        assert st["completed"] == 4 * per_thread
        assert st["pool_bytes_in_use"] == 0 and st["queue_depth"] == 0
        print(f"concurrent clients: {st['completed']} requests, {st['ticks']} ticks, "
              f"{st['acquire_rejections']} rejected acquisitions", flush=True)


def test_create_failures_and_limits():
    """A pool larger than the device fails with SYEV3_E_BUDGET after freeing
    what creation had made, and leaves no HIP error behind for the caller's
    next launch (torch checks the last error after each); the largest
    allowed max_requests works."""
    total = torch.cuda.get_device_properties(0).total_memory
    with pytest.raises(s3.Syev3Error) as exc:
        serve.Server(hbm_budget_bytes=total + (64 << 30))
    assert exc.value.code == -8
    with serve.Server(hbm_budget_bytes=64 << 20, max_requests=65536) as srv:
        r = srv.acquire(1000, s3.F64)
        A = torch.randn(6, 1000, dtype=torch.float64, device="cuda")
        r.A.copy_(A)
        ev = torch.cuda.Event()
        ev.record()
        srv.submit(r, ev)
        srv.wait(r, timeout_s=30.0)
        _check_bitwise(r)
        srv.release(r)
        assert srv.stats()["pool_bytes_in_use"] == 0


def test_one_segment_per_tick(source):
    """The smallest configuration: one request per tick, one tick in flight.
    Every request still completes with the bits of a separate solve."""
    A64, A32 = source
    with serve.Server(hbm_budget_bytes=256 << 20, max_inflight_ticks=1,
                      max_segments_per_tick=1) as srv:
        reqs = []
        for k in range(12):
            dt = s3.F64 if k % 2 == 0 else s3.F32_REFINE
            r = srv.acquire(1000 + 37 * k, dt, vectors=k % 3 != 2)
            srv.submit(r, _fill(r, A64 if dt == s3.F64 else A32, 1000 * k))
            reqs.append(r)
        for r in reqs:
            srv.wait(r, timeout_s=30.0)
            _check_bitwise(r)
            srv.release(r)
        st = srv.stats()
        assert st["ticks"] == 12 and st["segments_per_tick_peak"] == 1
        assert st["inflight_ticks_peak"] == 1


@pytest.mark.parametrize("nreq,grid_blocks,use_graphs", [(200, 0, False), (600, 7, True),
                                                         (600, 0, False)])
def test_a_tick_of_many_segments(source, nreq, grid_blocks, use_graphs):
    """A tick of many requests: the kernel finds each tile's request by
    counting, 256 table entries per round, the requests that start at or
    before it.  The first request's ready event waits behind a short spin on
    the GPU (one tick slot), so the next nreq requests queue up and leave in
    one tick (600: three rounds of the count).  With the grid capped at 7
    workgroups each strides over hundreds of tiles, its search resuming at
    the round of its last tile.  Every result equals a separate solve
    bitwise, and a sample meets the oracle's bars."""
    A64, A32 = source
    rng = np.random.default_rng(11)
    with serve.Server(hbm_budget_bytes=1 << 30, max_inflight_ticks=1,
                      max_segments_per_tick=1024, grid_blocks=grid_blocks,
                      use_graphs=use_graphs) as srv:
        first = srv.acquire(4096, s3.F64)
        # about 50 ms per 200 requests at the GPU's clock, the time to queue them
        torch.cuda._sleep(100_000_000 * (nreq // 200 + 1))
        srv.submit(first, _fill(first, A64, 0))
        reqs, off = [], 4096
        for k in range(nreq):
            n = int(rng.integers(1, 3000))
            dt = s3.F64 if k % 2 == 0 else s3.F32_REFINE
            r = srv.acquire(n, dt, vectors=k % 5 != 4)
            srv.submit(r, _fill(r, A64 if dt == s3.F64 else A32, off))
            off += n
            reqs.append(r)
        for r in [first] + reqs:
            srv.wait(r, timeout_s=60.0)
            _check_bitwise(r)
        for r in reqs[::20]:
            _check_oracle(r, sample=3000, label="many-segment tick")
        for r in [first] + reqs:
            srv.release(r)
        st = srv.stats()
        print(f"  ticks {st['ticks']}, segments per tick at peak "
              f"{st['segments_per_tick_peak']}", flush=True)
        assert st["segments_per_tick_peak"] > (512 if nreq > 512 else 128)


def test_caller_may_drop_its_ready_event_right_after_submit(source):
    """The server waits for the caller's event during submit and keeps a
    mark of its own, so a caller that destroys its event (or records it
    again) as soon as submit returns still gets its input honoured: every
    result equals a separate solve of the same input, bitwise."""
    import gc
    A64, A32 = source
    rng = np.random.default_rng(11)
    with serve.Server(hbm_budget_bytes=1 << 30, max_inflight_ticks=2) as srv:
        reqs = []
        reuse = torch.cuda.Event()
        for k in range(24):
            n = int(rng.integers(1, 60_000))
            dt = s3.F64 if k % 2 == 0 else s3.F32_REFINE
            r = srv.acquire(n, dt)
            off = int(rng.integers(0, (1 << 21) - n))
            r.A.copy_((A64 if dt == s3.F64 else A32)[:, off:off + n])
            if k % 3 == 0:
                ev = torch.cuda.Event()        # dropped right after submit
                ev.record()
                srv.submit(r, ev)
                del ev
                gc.collect()
            else:
                reuse.record()                 # one event recorded again for the next
                srv.submit(r, reuse)
            reqs.append(r)
        for r in reqs:
            srv.wait(r, timeout_s=60.0)
            _check_bitwise(r)
            srv.release(r)
        assert srv.stats()["completed"] == 24


def test_requests_admitted_as_views_of_the_callers_input(source):
    """A request admitted as a view reads its input in place from the
    caller's tensor, with the caller's plane stride (a window of a larger
    pool), and only its outputs take pool memory.  Its results equal a
    separate solve bitwise and meet the oracle's bars."""
    A64, A32 = source
    ld = A64.shape[1]
    with serve.Server(hbm_budget_bytes=256 << 20, max_inflight_ticks=2) as srv:
        reqs = []
        for k, (n, off) in enumerate([(1, 5), (255, 1000), (70_001, 3), (300_000, 1_500_000)]):
            src = A64 if k % 2 == 0 else A32
            view = src[:, off:off + n]
            assert view.stride(0) == ld
            r = srv.acquire_view(view, vectors=k != 2)
            assert r is not None and r.A.data_ptr() == view.data_ptr()
            srv.submit(r)
            reqs.append(r)
        es = {s3.F64: 8, s3.F32_REFINE: 4}
        used = srv.stats()["pool_bytes_in_use"]
        want = sum(-(-3 * r.n * es[r.dtype] // 256) * 256
                   + (-(-9 * r.n * es[r.dtype] // 256) * 256 if r.V is not None else 0)
                   for r in reqs)
        assert used == want, (used, want)      # outputs only
        for r in reqs:
            srv.wait(r, timeout_s=60.0)
            lam, V = s3.syev3(r.A.contiguous(), vectors=r.V is not None)
            torch.cuda.synchronize()
            assert torch.equal(lam, r.lam) and (V is None or torch.equal(V, r.V))
            _check_oracle(r, label="view")
            srv.release(r)
        # a view has no input of its own to stage from the host
        r = srv.acquire_view(A64[:, :100])
        with pytest.raises(s3.Syev3Error) as ei:
            srv.submit_host(r, A64[:, :100].cpu().contiguous(),
                            torch.empty(3, 100, dtype=torch.float64))
        assert ei.value.code == -10
        srv.submit(r)
        srv.wait(r, timeout_s=30.0)
        srv.release(r)
        with pytest.raises(ValueError):
            srv.acquire_view(A64[:, :10].t().contiguous().t())  # column stride != 1
        assert srv.stats()["pool_bytes_in_use"] == 0


def test_loadgen_with_input_views(source):
    A64, A32 = source
    with serve.Server(hbm_budget_bytes=2 << 30) as srv:
        res = srv.loadgen(A64, A32, qps=0.0, concurrency=32, duration_s=0.5, max_log2_n=16,
                          seed=5, input_views=True)
    print(res, flush=True)
    assert res["requests"] > 32 and 0 < res["lat_p50_s"] <= res["lat_p99_s"]


@pytest.mark.parametrize("use_graphs", [True, False])
def test_non_finite_inputs_in_served_requests(source, use_graphs):
    """Requests whose inputs hold NaN and infinite entries in some matrices,
    in both forms, with and without vectors: exactly those matrices come out
    NaN (every eigenvalue and vector entry), and every output equals a
    separate batched solve bit for bit (the serving kernel's NaN stores
    included)."""
    A64, A32 = source
    specs = [(1000, s3.F64, True), (777, s3.F32_REFINE, True), (300, s3.F64, False),
             (2049, s3.F32_REFINE, False)]
    with serve.Server(hbm_budget_bytes=1 << 30, use_graphs=use_graphs) as srv:
        reqs = []
        for k, (n, dt, vec) in enumerate(specs):
            r = srv.acquire(n, dt, vectors=vec)
            src = (A64 if dt == s3.F64 else A32)[:, 5000 * k:5000 * k + n].clone()
            bad = (torch.arange(n, device="cuda") % 97) == 3
            cols = bad.nonzero().flatten()
            for i, c in enumerate(cols.tolist()):
                src[i % 6, c] = (float("nan"), float("inf"), float("-inf"))[i % 3]
            r.A.copy_(src)
            ev = torch.cuda.Event()
            ev.record()
            srv.submit(r, ev)
            reqs.append((r, bad))
        for r, bad in reqs:
            srv.wait(r, timeout_s=60.0)
            lam, V = s3.syev3(r.A.clone(), vectors=r.V is not None)
            torch.cuda.synchronize()
            ib = torch.int64 if lam.dtype == torch.float64 else torch.int32
            assert torch.equal(lam.view(ib), r.lam.view(ib)), f"lambda differs for n={r.n}"
            assert torch.isnan(r.lam[:, bad]).all() and torch.isfinite(r.lam[:, ~bad]).all()
            if V is not None:
                assert torch.equal(V.view(ib), r.V.view(ib)), f"V differs for n={r.n}"
                assert torch.isnan(r.V[:, bad]).all() and torch.isfinite(r.V[:, ~bad]).all()
            srv.release(r)
        assert srv.stats()["pool_bytes_in_use"] == 0
