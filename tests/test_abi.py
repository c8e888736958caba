"""The C ABI without a GPU: the library loads, exports every function that
include/syev3.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_1806_06698_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "syev3.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted({n for n in names if n.startswith(("batched_", "syev3_"))})


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("batched_syev3", "batched_syev3_ex", "batched_syev3_info",
                     "syev3_strerror", "syev3_server_create", "syev3_server_submit"):
        assert required in names


def test_library_exports_every_declared_function(L):
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, f"declared in syev3.h but not exported: {missing}"


def test_strerror_and_version(L):
    for code in range(0, -14, -1):
        s = L.syev3_strerror(code).decode()
        assert s and s != "unknown error code"
    assert L.syev3_version() >= 10000


# Fake, never-dereferenced device addresses: every call below must fail in
# argument checking, before any launch.
A = ctypes.c_void_p(0x100000)
LAM = ctypes.c_void_p(0x200000)
VV = ctypes.c_void_p(0x300000)
NUL = ctypes.c_void_p(0)
S = ctypes.c_void_p(0)


ARG_ERRORS = {-1, -2, -3, -4, -5, -7}   # argument checks; -6 means a launch was tried


def _rejecting(fn):
    """fn, required to fail in argument checking.  An accepted call would
    launch a kernel on the fake addresses above; without a GPU that launch
    fails with SYEV3_E_HIP, which this wrapper reports as a test failure, so
    a wrongly written check is caught here on the CPU."""
    def call(*a):
        rc = fn(*a)
        assert rc in ARG_ERRORS, f"rc={rc}: the call got past argument checking"
        return rc
    return call


@pytest.fixture
def no_device():
    """The fake-address tests run only where no GPU is visible: on a GPU
    machine an accepted call would be a real launch on unmapped memory."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("fake device addresses: run without a GPU")


def test_bad_arguments_are_rejected(L, no_device):
    ex = _rejecting(L.batched_syev3_ex)
    assert ex(-1, A, 0, 0, LAM, VV, 0, 0, S) == -1             # n < 0
    assert ex(10, NUL, 0, 0, LAM, VV, 0, 0, S) == -2           # A NULL
    assert ex(10, A, 0, 0, NUL, VV, 0, 0, S) == -2             # lambda NULL
    assert ex(10, A, 0, 0, LAM, VV, 7, 0, S) == -3             # dtype
    assert ex(10, A, 0, 0, LAM, VV, 1, 4, S) == -3             # Newton needs F64
    assert ex(10, A, 0, 0, LAM, VV, 2, 4, S) == -3
    assert ex(10, A, 0, 0, LAM, VV, 1, 8, S) == -3             # paper BG needs F64
    assert ex(10, A, 0, 0, LAM, VV, 0, 12, S) == -7            # Newton and paper BG
    assert ex(10, A, 0, 0, LAM, VV, 0, 16, S) == -3            # converge needs F32_REFINE
    assert ex(10, A, 0, 0, LAM, VV, 2, 16, S) == -3
    assert ex(10, A, 0, 0, LAM, VV, 0, 128, S) == -7           # unknown flag
    assert ex(10, A, 0, 0, LAM, VV, 3, 0, S) == -3
    # the unrefined FP32 dtype has FP32 spans: lambda 4 bytes past A's end is fine
    assert ex(10, A, 0, 1, ctypes.c_void_p(0x100000 + 4 * 59), NUL, 2, 0, S) == -5
    assert ex(10, A, 0, 3, LAM, VV, 0, 0, S) == -4             # layout
    assert ex(10, A, 5, 0, LAM, VV, 0, 0, S) == -4             # ld < n
    assert ex(10, A, 10, 1, LAM, VV, 0, 0, S) == -4            # AoS needs ld 0
    assert ex(10, A, 0, 0, LAM, VV, 0, 64, S) == -7            # unknown flag
    # aliasing: lambda inside A's 6 planes; V overlapping lambda
    assert ex(10, A, 0, 0, ctypes.c_void_p(0x100000 + 8 * 30), VV, 0, 0, S) == -5
    assert ex(10, A, 0, 0, LAM, ctypes.c_void_p(0x200000 + 8), 0, 0, S) == -5
    # AoS spans: A is 6n packed elements
    assert ex(10, A, 0, 1, ctypes.c_void_p(0x100000 + 8 * 59), NUL, 0, 0, S) == -5
    # (that adjacent arrays are accepted is a GPU test: an accepted call
    # launches, and these addresses are not device memory)
    # full-matrix AoS: V may be A exactly (in place), not partly
    assert ex(10, A, 0, 2, ctypes.c_void_p(0x100000 + 8 * 89), NUL, 0, 0, S) == -5
    assert ex(10, A, 0, 2, LAM, ctypes.c_void_p(0x100000 + 8), 0, 0, S) == -5
    inplace = _rejecting(L.batched_syev3_inplace)
    assert inplace(-1, A, LAM, 0, S) == -1
    assert inplace(10, A, ctypes.c_void_p(0x100000 + 8 * 10), 0, S) == -5
    # huge n for the grid
    assert ex(1 << 62, A, 0, 0, LAM, VV, 0, 0, S) in (-1, -4)


def test_segment_call_rejects_bad_arguments(L, no_device):
    """syev3_solve_segments_noalloc: the segment count against the fixed
    table, the per-segment rules of the batched calls (SYEV3_F32, which the
    segment kernel lacks, included) and aliasing across segments, all
    answered before any HIP call."""
    from paper_1806_06698_amd._lib import Segment, SEGMENTS_MAX
    call = L.syev3_solve_segments_noalloc

    def seg(n=10, a=0x100000, lda=0, lam=0x200000, v=0x300000, dtype=0, flags=0):
        return Segment(n, a, lda, lam, v, dtype, flags)

    def run(*segs, nseg=None):
        arr = (Segment * max(len(segs), 1))(*segs)
        rc = call(len(segs) if nseg is None else nseg, arr, S)
        assert rc in ARG_ERRORS | {-13}, f"rc={rc}: the call got past argument checking"
        return rc

    assert run(seg(), nseg=-1) == -13
    assert run(seg(), nseg=SEGMENTS_MAX + 1) == -13
    assert call(1, None, S) == -2
    assert run(seg(dtype=2)) == -3                    # the unrefined ablation
    assert run(seg(dtype=7)) == -3
    assert run(seg(flags=128)) == -7
    assert run(seg(lda=5)) == -4
    assert run(seg(n=-1)) == -1
    assert run(seg(a=0)) == -2
    assert run(seg(lam=0x100000 + 8 * 30)) == -5      # inside its own input
    # across segments: an output inside another segment's input, outputs
    # overlapping each other
    assert run(seg(), seg(a=0x400000, lam=0x100000 + 8, v=0)) == -5
    assert run(seg(), seg(a=0x400000, lam=0x500000, v=0x300000 + 8 * 80)) == -5
    assert run(seg(), seg(a=0x400000, lam=0x200000, v=0)) == -5
    # a bad segment after valid ones rejects the whole call
    assert run(seg(), seg(a=0x400000, lam=0x500000, v=0x600000, dtype=3)) == -3


def test_segment_call_with_nothing_to_solve_is_a_noop(L):
    """No segments, or only empty ones: accepted, nothing enqueued (no HIP
    call is made, so this holds without a GPU too)."""
    from paper_1806_06698_amd._lib import Segment
    empty = (Segment * 2)(Segment(0, 0, 0, 0, 0, 0, 0), Segment(0, 0, 0, 0, 0, 1, 0))
    assert L.syev3_solve_segments_noalloc(0, None, S) == 0
    assert L.syev3_solve_segments_noalloc(2, empty, S) == 0


def test_n_zero_is_a_noop(L):
    assert L.batched_syev3(0, NUL, NUL, NUL, 0, S) == 0
    assert L.batched_syev3_ex(0, NUL, 0, 1, NUL, NUL, 1, 0, S) == 0


def test_python_binding_refuses_cpu_tensors():
    import torch
    import paper_1806_06698_amd as s3
    with pytest.raises(ValueError):
        s3.syev3(torch.zeros(6, 4, dtype=torch.float64))


def test_loadgen_and_wait_options_are_range_checked(L, no_device):
    """Options out of range are refused (SYEV3_E_N) before the server is
    touched: a NaN or oversized rate, a duration or an arrival count too
    large to represent or queue, a request size exponent above 40, a
    closed-loop concurrency outside 1..2^20, and a NaN wait timeout.  Each
    case breaks one option of an otherwise valid set; the server handle is a
    fake address that the checks never reach."""
    from paper_1806_06698_amd import serve
    serve._bind(L)
    fake = ctypes.c_void_p(1 << 40)

    def opts(**kw):
        o = serve.LoadgenOpts(qps=1000.0, closed_concurrency=0, duration_s=1.0,
                              max_log2_n=10.0, frac_f32=0.5, seed=0, src_f64=1 << 41,
                              src_f32=1 << 42, src_n=1024, want_vectors=1, host_staged=0,
                              sink=None)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    bad = [dict(qps=2e8), dict(qps=float("nan")), dict(qps=1e6, duration_s=1000.0),
           dict(qps=1.0, duration_s=2e6), dict(duration_s=0.0), dict(max_log2_n=41.0),
           dict(max_log2_n=float("inf")), dict(qps=0.0, closed_concurrency=(1 << 20) + 1),
           dict(qps=0.0, closed_concurrency=0)]
    for kw in bad:
        r = serve.LoadgenResult()
        assert L.syev3_server_loadgen(fake, ctypes.byref(opts(**kw)), ctypes.byref(r)) == -1, kw
    lat = ctypes.c_double()
    assert L.syev3_server_wait(fake, 0, float("nan"), ctypes.byref(lat)) == -1


def test_server_rejects_bad_options_without_a_gpu(L):
    from paper_1806_06698_amd import _lib as lb
    o = lb.ServerOpts()
    L.syev3_server_default_opts(ctypes.byref(o))
    assert o.hbm_budget_bytes == 64 << 30 and o.max_inflight_ticks == 4
    h = ctypes.c_void_p()
    o.max_requests = 0
    assert L.syev3_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    L.syev3_server_default_opts(ctypes.byref(o))
    o.max_segments_per_tick = 100000
    assert L.syev3_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    L.syev3_server_default_opts(ctypes.byref(o))
    o.grid_blocks = (1 << 24) + 1
    assert L.syev3_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    o.grid_blocks = -1
    assert L.syev3_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    assert L.syev3_server_create(ctypes.byref(o), None) == -2
    b = lb.RequestBuffers()
    assert L.syev3_server_acquire(None, 10, 0, 1, ctypes.byref(b)) == -2
    assert L.syev3_server_submit(None, 0, None) == -10
    assert L.syev3_server_release(None, 0) == -10


def test_stream_probe_modes_are_checked(L, no_device):
    probe = _rejecting(L.syev3_stream_probe)
    assert probe(10, A, LAM, VV, 0, 0, S) == -7               # neither read nor write
    assert probe(10, A, LAM, VV, 0, 4, S) == -7               # order alone
    assert probe(10, A, LAM, VV, 0, 8, S) == -7               # unknown bit
    assert probe(10, A, LAM, VV, 5, 3, S) == -3               # dtype
    assert probe(-1, A, LAM, VV, 0, 3, S) == -1
    far = [ctypes.c_void_p(x << 40) for x in (1, 2, 3)]        # no overlap at this size
    assert probe((1 << 31) + 1, *far, 0, 3, S) == -1          # more than one launch


def test_server_options_are_range_checked(L):
    """syev3_server_create rejects options outside the documented ranges
    before it touches the device, and leaves *out NULL."""
    def opts(**kw):
        o = _lib.ServerOpts()
        L.syev3_server_default_opts(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o
    bad = [dict(max_requests=0), dict(max_requests=65537), dict(max_requests=-1),
           dict(max_inflight_ticks=0), dict(max_inflight_ticks=65),
           dict(max_segments_per_tick=0), dict(max_segments_per_tick=1025),
           dict(grid_blocks=-1), dict(hbm_budget_bytes=255)]
    for kw in bad:
        h = ctypes.c_void_p(0x1234)
        rc = L.syev3_server_create(ctypes.byref(opts(**kw)), ctypes.byref(h))
        assert rc == -1, (kw, rc)
        assert not h.value, kw
    assert L.syev3_server_create(ctypes.byref(opts()), None) == -2
