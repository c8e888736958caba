"""Argument checks of the serving wrapper (no GPU): the native server and
load generator take raw pointers, so sizes and dtypes are checked before any
call."""
import pytest
import torch

from paper_1806_06698_amd import _lib, serve


def test_host_buffers_must_fit_the_request():
    n = 100
    A = torch.zeros(6 * n, dtype=torch.float64)
    lam = torch.zeros(3 * n, dtype=torch.float64)
    V = torch.zeros(9 * n, dtype=torch.float64)
    serve.check_host_buffers(n, _lib.F64, A, lam, V)
    serve.check_host_buffers(n, _lib.F64, A, lam, None)
    with pytest.raises(ValueError):
        serve.check_host_buffers(n, _lib.F64, A[:-1], lam, V)          # short input
    with pytest.raises(ValueError):
        serve.check_host_buffers(n, _lib.F64, A, lam, V[:-1])          # short V
    with pytest.raises(ValueError):
        serve.check_host_buffers(n, _lib.F32_REFINE, A, lam, V)        # dtype
    with pytest.raises(ValueError):
        serve.check_host_buffers(n, _lib.F64, A.view(6, n).t(), lam, V)  # not contiguous


def test_loadgen_sources_are_checked():
    m = 1 << 10
    a64 = torch.zeros(6, m, dtype=torch.float64)
    a32 = torch.zeros(6, m, dtype=torch.float32)
    sink = torch.zeros(12 * m, dtype=torch.float64)
    serve.check_loadgen_sources(a64, a32, 10, sink)
    with pytest.raises(ValueError):
        serve.check_loadgen_sources(a64, a32[:, : m // 2].contiguous(), 10, sink)  # src_n differ
    with pytest.raises(ValueError):
        serve.check_loadgen_sources(a64, a64, 10, sink)                 # f32 source of doubles
    with pytest.raises(ValueError):
        serve.check_loadgen_sources(a64, a32, 11, sink)                 # 2^11 > src_n
    with pytest.raises(ValueError):
        serve.check_loadgen_sources(a64, a32, 10, sink[:-1])            # sink too small
    with pytest.raises(ValueError):
        serve.check_loadgen_sources(a64, a32, 10, None)                 # no sink
    with pytest.raises(ValueError):
        serve.check_loadgen_sources(a64[:5].contiguous(), a32, 10, sink)  # not 6 rows
