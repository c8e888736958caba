"""Output-tensor checks of the Python binding (no GPU): the kernels write
through raw pointers, so an out= tensor must have exactly the shape, strides,
dtype and device they assume."""
import pytest
import torch

import paper_1806_06698_amd as s3


def test_out_tensors_are_checked():
    n = 10
    A = torch.zeros(6, n, dtype=torch.float64)
    ok_lam = torch.empty(3, n, dtype=torch.float64)
    s3._check_out(ok_lam, (3, n), (n, 1), A, "lam")
    wide = torch.empty(3, 2 * n, dtype=torch.float64)[:, :n]       # ld = 2n
    s3._check_out(wide, (3, n), (2 * n, 1), A, "lam")
    with pytest.raises(ValueError):
        s3._check_out(wide, (3, n), (n, 1), A, "lam")                # stride differs from A's
    with pytest.raises(ValueError):
        s3._check_out(torch.empty(3, n - 1, dtype=torch.float64), (3, n), (n, 1), A, "lam")
    with pytest.raises(ValueError):
        s3._check_out(torch.empty(3, n, dtype=torch.float32), (3, n), (n, 1), A, "lam")
    with pytest.raises(ValueError):
        s3._check_out(torch.empty(n, 3, dtype=torch.float64).t(), (3, n), (n, 1), A, "lam")
    with pytest.raises(ValueError):
        s3._check_out(None, (9, n), (n, 1), A, "V")
    aos = torch.empty(n, 3, 3, dtype=torch.float64)
    s3._check_out(aos, (n, 3, 3), (9, 3, 1), A, "V")
    with pytest.raises(ValueError):
        s3._check_out(aos.transpose(1, 2), (n, 3, 3), (9, 3, 1), A, "V")


def test_soa_input_planes_must_be_disjoint():
    n = 10
    ok = torch.zeros(6, n, dtype=torch.float64)
    assert s3._soa_geometry(ok) == (n, n)
    assert s3._soa_geometry(torch.zeros(6, 2 * n, dtype=torch.float64)[:, :n]) == (n, 2 * n)
    assert s3._soa_geometry(torch.zeros(6, 0, dtype=torch.float64)) == (0, 0)
    assert s3._soa_geometry(torch.zeros(6, 1, dtype=torch.float64)) == (1, 1)
    # a broadcast row: stride (0, 1), six planes on the same n elements
    with pytest.raises(ValueError, match="overlap"):
        s3._soa_geometry(torch.randn(n, dtype=torch.float64).expand(6, n))
    with pytest.raises(ValueError, match="overlap"):
        s3._soa_geometry(torch.randn(1, dtype=torch.float64).expand(6, 1))
    # overlapping planes: a (6, n) window with row stride n // 2
    buf = torch.zeros(6 * n, dtype=torch.float64)
    with pytest.raises(ValueError, match="overlap"):
        s3._soa_geometry(buf.as_strided((6, n), (n // 2, 1)))
    with pytest.raises(ValueError):
        s3._soa_geometry(torch.zeros(n, 6, dtype=torch.float64).t())   # column stride 6
    with pytest.raises(ValueError):
        s3._soa_geometry(torch.zeros(5, n, dtype=torch.float64))


def test_broadcast_out_tensors_are_refused():
    n = 10
    A = torch.zeros(6, n, dtype=torch.float64)
    with pytest.raises(ValueError):
        s3._check_out(torch.empty(n, dtype=torch.float64).expand(3, n), (3, n), (n, 1), A,
                      "lam")
    with pytest.raises(ValueError):
        s3._check_out(torch.empty(9, dtype=torch.float64).expand(n, 9).t(), (9, n), (n, 1), A,
                      "V")


def test_soa_out_tensors_and_the_output_stride():
    n = 10
    A = torch.zeros(6, n, dtype=torch.float64)
    s3._check_out_soa(torch.empty(3, n, dtype=torch.float64), 3, n, A, "lam")
    s3._check_out_soa(torch.empty(12, 2 * n, dtype=torch.float64)[3:, :n], 9, n, A, "V")
    with pytest.raises(ValueError):          # the info path needs the input's stride
        s3._check_out_soa(torch.empty(3, 2 * n, dtype=torch.float64)[:, :n], 3, n, A, "lam",
                          ld=n)
    with pytest.raises(ValueError):          # broadcast rows
        s3._check_out_soa(torch.empty(n, dtype=torch.float64).expand(3, n), 3, n, A, "lam")
    with pytest.raises(ValueError):          # column stride
        s3._check_out_soa(torch.empty(n, 3, dtype=torch.float64).t(), 3, n, A, "lam")
    with pytest.raises(ValueError):
        s3._check_out_soa(torch.empty(3, n, dtype=torch.float32), 3, n, A, "lam")


def test_segment_call_binding_checks_its_tensors():
    """syev3_solve_segments_noalloc's binding: no segments is a no-op, and
    host tensors are refused before anything reaches the library (the
    kernels have no CPU path)."""
    s3.syev3_solve_segments_noalloc([])
    n = 8
    A = torch.zeros(6, n, dtype=torch.float64)
    lam = torch.empty(3, n, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        s3.syev3_solve_segments_noalloc([(A, lam, None)])
