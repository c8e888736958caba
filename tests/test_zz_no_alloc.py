"""The entry point that allocates nothing, syev3_solve_segments_noalloc,
through the C ABI: several requests solved by one launch of the serving
kernel on the library's fixed per-GPU segment table.  Its results must
equal, bitwise, those the server gives for the same requests
(syev3_server_*, whose ticks run that kernel on tables the server
allocates), over two calls in a row on one stream, the second smaller: its
table overwrites the first's, which the stream's order keeps from racing the
first call's kernel.  A sample of each call also meets the CPU oracle."""
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
    A, _ = gen.stress_mix(1 << 21, seed=11, device="cuda")
    return A, A.float().contiguous()


def _requests(src, sizes, start):
    """Requests over windows of the (6, N) sources from column `start`:
    alternately FP64 and FP32 storage, every third input read in place at the
    source's plane stride (above n), every fourth without vectors; outputs
    filled with NaN, so that anything left unwritten shows."""
    src64, src32 = src
    reqs, off = [], start
    for i, n in enumerate(sizes):
        s = src32 if i % 2 else src64
        A = s[:, off:off + n]
        if i % 3:
            A = A.contiguous()
        off += n
        lam = torch.full((3, n), float("nan"), dtype=A.dtype, device="cuda")
        V = (torch.full((9, n), float("nan"), dtype=A.dtype, device="cuda")
             if i % 4 != 3 else None)
        reqs.append((A, lam, V))
    return reqs, off


def _served(reqs):
    """The same requests through a server (inputs read in place)."""
    out = []
    with serve.Server(hbm_budget_bytes=1 << 30, max_segments_per_tick=64) as srv:
        ev = torch.cuda.Event()
        ev.record()
        handles = [srv.acquire_view(A, vectors=V is not None) for A, _, V in reqs]
        assert all(h is not None for h in handles)
        for h in handles:
            srv.submit(h, ev)
        for h in handles:
            srv.wait(h)
            out.append((h.lam.clone(), None if h.V is None else h.V.clone()))
            srv.release(h)
    return out


def _check_equal(reqs, served, label):
    for i, ((A, lam, V), (sl, sV)) in enumerate(zip(reqs, served)):
        n = A.shape[1]
        assert torch.equal(lam, sl), f"{label} request {i} (n={n}, {A.dtype}): eigenvalues"
        if V is not None:
            assert torch.equal(V, sV), f"{label} request {i} (n={n}, {A.dtype}): vectors"


def test_two_calls_in_a_row_match_the_server(source):
    sizes1 = [1, 255, 256, 257, 1000, 4099, 65_553, 300_001, 3, 70_000, 12_345, 2, 511,
              100_000, 0, 31]
    sizes2 = [7, 300, 5_000, 1]  # the second call: fewer and smaller requests
    reqs1, off = _requests(source, sizes1, 0)
    reqs2, _ = _requests(source, sizes2, off)
    print(f"no-alloc: call 1 {len(sizes1)} requests ({sum(sizes1)} matrices), "
          f"call 2 {len(sizes2)} ({sum(sizes2)})", flush=True)
    s3.syev3_solve_segments_noalloc(reqs1)
    s3.syev3_solve_segments_noalloc(reqs2)  # same stream, no wait in between
    torch.cuda.synchronize()
    live1 = [r for r in reqs1 if r[0].shape[1] > 0]
    _check_equal(live1, _served(live1), "call 1")
    _check_equal(reqs2, _served(reqs2), "call 2")
    for label, reqs in (("call 1", reqs1), ("call 2", reqs2)):
        for A, lam, V in sorted(reqs, key=lambda r: -r[0].shape[1])[:2]:
            check_vs_oracle(A, lam, V, f32=A.dtype == torch.float32, sample=20_000,
                            seed=A.shape[1], label=f"no-alloc {label} n={A.shape[1]}")


def test_repeated_calls_on_one_stream(source):
    """Ten calls of varying length back to back on one stream (each table
    overwriting the last), then one synchronisation: each call's results
    equal the batched solver's on the same inputs."""
    g = torch.Generator().manual_seed(5)
    calls, off = [], 0
    for c in range(10):
        k = int(torch.randint(1, 40, (1,), generator=g))
        sizes = torch.randint(1, 20_000, (k,), generator=g).tolist()
        reqs, off = _requests(source, sizes, off % (1 << 20))
        calls.append(reqs)
    print(f"no-alloc: {len(calls)} calls of {[len(r) for r in calls]} requests", flush=True)
    for reqs in calls:
        s3.syev3_solve_segments_noalloc(reqs)
    torch.cuda.synchronize()
    for c, reqs in enumerate(calls):
        for i, (A, lam, V) in enumerate(reqs):
            rl, rV = s3.syev3(A, vectors=V is not None)
            assert torch.equal(lam, rl), f"call {c} request {i}: eigenvalues"
            if V is not None:
                assert torch.equal(V, rV), f"call {c} request {i}: vectors"
