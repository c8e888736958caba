"""Batched 3x3 real symmetric eigensolver for AMD MI355X (gfx950).

The solver is libsyev3.so (hand-written HIP kernels behind a C ABI, see
include/syev3.h); this package is a thin binding that hands it torch device
tensors and the current HIP stream.  Method: Borges, "Solving the 3x3 Real
Symmetric Eigenproblem" (arXiv:1806.06698).

    import torch, paper_1806_06698_amd as s3
    A = torch.randn(6, n, dtype=torch.float64, device="cuda")   # a11 a12 a13 a22 a23 a33
    lam, V = s3.syev3(A)          # lam (3, n) ascending; V (9, n): V[3r+c] = row r of vector c
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (AOS, AOS9, F32, F32_REFINE, F64, FLAG_NEWTON, FLAG_NO_H_GUARD,
                   FLAG_NO_SCALE, FLAG_PAPER_BG, FLAG_REFINE_CONVERGE,
                   FLAG_SIMPLIFIED_DEFLATION, SOA,
                   Syev3Error)

__all__ = ["syev3", "syev3_inplace", "batched_syev3", "batched_syev3_ex", "batched_syev3_info",
           "batched_syev3_strided", "syev3_solve_segments_noalloc",
           "F64", "F32_REFINE", "F32", "SOA", "AOS", "AOS9", "FLAG_SIMPLIFIED_DEFLATION",
           "FLAG_NO_H_GUARD", "FLAG_NEWTON", "FLAG_PAPER_BG", "FLAG_REFINE_CONVERGE", "FLAG_NO_SCALE",
           "Syev3Error",
           "lib_path"]

lib_path = _lib.LIB_PATH


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream, device):
    """The stream to launch on: the given one, else the current stream of the
    device that holds the data (the launch runs on the stream's device)."""
    if stream is None:
        stream = torch.cuda.current_stream(device)
    elif stream.device != device:
        raise ValueError(f"stream is on {stream.device}, the tensors on {device}")
    return ctypes.c_void_p(stream.cuda_stream)


def batched_syev3(n, A_ptr, lam_ptr, V_ptr, dtype, stream_handle) -> int:
    """Raw C entry point with integer device pointers; returns the status."""
    return _lib.lib().batched_syev3(n, A_ptr, lam_ptr, V_ptr, dtype, stream_handle)


def batched_syev3_ex(n, A_ptr, ld, layout, lam_ptr, V_ptr, dtype, flags,
                     stream_handle) -> int:
    return _lib.lib().batched_syev3_ex(n, A_ptr, ld, layout, lam_ptr, V_ptr,
                                       dtype, flags, stream_handle)


def batched_syev3_info(n, A_ptr, ld, layout, lam_ptr, V_ptr, dtype, flags,
                       info_ptr, stream_handle) -> int:
    return _lib.lib().batched_syev3_info(n, A_ptr, ld, layout, lam_ptr, V_ptr,
                                         dtype, flags, info_ptr, stream_handle)


def batched_syev3_strided(n, A_ptr, lda, lam_ptr, ldl, V_ptr, ldv, dtype, flags,
                          stream_handle) -> int:
    return _lib.lib().batched_syev3_strided(n, A_ptr, lda, lam_ptr, ldl, V_ptr, ldv, dtype,
                                            flags, stream_handle)


def syev3_solve_segments_noalloc(segments, *, stream=None) -> None:
    """Solve several independent requests in one launch, allocating nothing
    (C ABI syev3_solve_segments_noalloc).  segments: (A, lam, V) or (A, lam,
    V, flags) per request, all on one GPU: A (6, n) float64 (FP64) or float32
    (FP32 storage + FP64 refinement) with unit column stride and row stride
    >= n; lam (3, n) and V (9, n) or None, contiguous, of A's dtype; they are
    written in place.  Asynchronous on the stream; calls on one GPU that are
    not ordered on one stream race (they share the library's segment
    table)."""
    segs = (_lib.Segment * max(len(segments), 1))()
    device = None
    for i, item in enumerate(segments):
        A, lam, V = item[:3]
        flags = item[3] if len(item) > 3 else 0
        if not A.is_cuda:
            raise ValueError("segment inputs must be GPU tensors")
        if device is None:
            device = A.device
        elif A.device != device:
            raise ValueError("all segments must be on one device")
        dt = _dtype_code(A)
        n, ld = _soa_geometry(A)
        for name, t, rows in (("lam", lam, 3), ("V", V, 9)):
            if t is None and name == "V":
                continue
            _check_out(t, (rows, n), (n, 1), A, f"segment {i} {name}")
        segs[i] = _lib.Segment(n, _ptr(A).value, ld, _ptr(lam).value, _ptr(V).value, dt, flags)
    if device is None:
        return
    rc = _lib.lib().syev3_solve_segments_noalloc(len(segments), segs,
                                                _stream_handle(stream, device))
    _lib.check(rc, "syev3_solve_segments_noalloc")


def _dtype_code(t: torch.Tensor, refine: bool = True) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32_REFINE if refine else F32
    raise TypeError(f"A must be float64 or float32, got {t.dtype}")


def _check_out(t, shape, strides, A, name):
    """An output tensor the kernels will write through its data pointer:
    exactly the shape, strides, dtype and device they assume (the
    library checks only pointers and aliasing)."""
    if t is None:
        raise ValueError(f"out: {name} is required")
    if (tuple(t.shape) != shape or t.dtype != A.dtype or t.device != A.device
            or (t.numel() > 1 and tuple(t.stride()) != strides)):
        raise ValueError(f"out: {name} must be a {A.dtype} tensor of shape {shape} with "
                         f"strides {strides} on {A.device}, got {tuple(t.shape)}, "
                         f"{tuple(t.stride())}, {t.dtype}, {t.device}")


def _check_out_soa(t, rows, n, A, name, ld=None):
    """An SoA output: (rows, n), unit column stride, row stride >= n (ld
    exactly, when the kernel takes the input's stride for every array)."""
    if t is None:
        raise ValueError(f"out: {name} is required")
    if (t.dim() != 2 or tuple(t.shape) != (rows, n) or t.dtype != A.dtype
            or t.device != A.device):
        raise ValueError(f"out: {name} must be a {A.dtype} tensor of shape {(rows, n)} on "
                         f"{A.device}, got {tuple(t.shape)}, {t.dtype}, {t.device}")
    if n > 1 and t.stride(1) != 1:
        raise ValueError(f"out: {name} must have unit column stride, got {tuple(t.stride())}")
    if n > 0 and (t.stride(0) < n or (ld is not None and t.stride(0) != ld)):
        want = f"row stride {ld}" if ld is not None else f"row stride >= n = {n}"
        raise ValueError(f"out: {name} needs {want} (disjoint rows), got {tuple(t.stride())}")


def _soa_geometry(A):
    """(n, ld) of an SoA input: shape (6, n), unit column stride and a plane
    stride ld >= n, so that the 6 planes are disjoint runs of n elements (a
    broadcast or overlapping view would make the kernels read and write
    past the storage the outputs are sized from)."""
    if A.dim() != 2 or A.shape[0] != 6 or (A.shape[1] > 1 and A.stride(1) != 1):
        raise ValueError("SoA input must have shape (6, n) with unit column stride")
    n = A.shape[1]
    if n == 0:
        return 0, 0
    ld = A.stride(0)
    if ld < n:
        raise ValueError(f"SoA input planes overlap: row stride {ld} is below n = {n} "
                         "(a broadcast or overlapping view); pass a (6, n) tensor whose "
                         "rows are disjoint, e.g. A.contiguous()")
    return n, ld


def syev3(A: torch.Tensor, *, vectors: bool = True, layout: str = "soa",
          flags: int = 0, info: bool = False, out=None, stream=None,
          refine: bool = True):
    """Eigen-decompose a batch of symmetric 3x3 matrices on the GPU.

    layout "soa": A has shape (6, n), rows a11 a12 a13 a22 a23 a33, row
    stride ld >= n (a slice of a (6, ld) buffer is fine).  Returns lam (3, n)
    and V (9, n) with V[3*r + c, i] = row r of eigenvector c of matrix i,
    rows of one contiguous (12, n) buffer (with info=True, of one (12, ld)
    buffer: the kernel then takes the input's stride for every array).
    layout "aos": A has shape (n, 6), contiguous.  Returns lam (n, 3) and
    V (n, 3, 3) with columns the eigenvectors (as torch.linalg.eigh).
    layout "aos9": A holds full matrices, (n, 3, 3) or (n, 9), contiguous
    (only the upper triangle is read); outputs as for "aos".
    float64 input runs the FP64 path; float32 input the FP32-storage path
    with FP64 refinement (refine=False: the unrefined FP32 ablation,
    dtype F32).  vectors=False skips V.  info=True also returns the
    per-matrix branch and iteration counts (int32).
    out: optional (lam, V) tensors to write into (same shapes as returned;
    for SoA any row stride >= n, or exactly the input's with info=True).
    """
    if not A.is_cuda:
        raise ValueError("A must be a GPU tensor (the solver has no CPU path)")
    dt = _dtype_code(A, refine)
    if layout == "soa":
        n, ld = _soa_geometry(A)
        if out is None:
            # one buffer of 3 (+ 9) planes; with info the kernel takes one
            # stride for every array, the input's
            ldo = ld if info else n
            buf = torch.empty((12 if vectors else 3, max(ldo, 1)), dtype=A.dtype,
                              device=A.device)
            lam, V = buf[:3, :n], (buf[3:12, :n] if vectors else None)
        else:
            lam, V = out
            _check_out_soa(lam, 3, n, A, "lam", ld if info else None)
            if vectors:
                _check_out_soa(V, 9, n, A, "V", ld if info else None)
            else:
                V = None
        if not info:
            rc = _lib.lib().batched_syev3_strided(
                n, _ptr(A), ld, _ptr(lam), lam.stride(0) if n else 0, _ptr(V),
                V.stride(0) if (V is not None and n) else 0, dt, flags,
                _stream_handle(stream, A.device))
            _lib.check(rc, "batched_syev3_strided")
            return lam, V
        lay = SOA
    elif layout in ("aos", "aos9"):
        width = 6 if layout == "aos" else 9
        if layout == "aos9" and A.dim() == 3 and A.shape[1:] == (3, 3):
            A = A.reshape(A.shape[0], 9)
        if A.dim() != 2 or A.shape[1] != width or not A.is_contiguous():
            raise ValueError(f"{layout} input must be a contiguous (n, {width}) tensor"
                             + (" or (n, 3, 3)" if width == 9 else ""))
        n = A.shape[0]
        ld = 0
        if out is None:
            lam = torch.empty((n, 3), dtype=A.dtype, device=A.device)
            V = torch.empty((n, 3, 3), dtype=A.dtype, device=A.device) if vectors else None
        else:
            lam, V = out
            _check_out(lam, (n, 3), (3, 1), A, "lam")
            if vectors:
                _check_out(V, (n, 3, 3), (9, 3, 1), A, "V")
            else:
                V = None
        lay = AOS if layout == "aos" else AOS9
    else:
        raise ValueError(f"unknown layout {layout!r}")
    inf = torch.empty(n, dtype=torch.int32, device=A.device) if info else None
    rc = _lib.lib().batched_syev3_info(
        n, _ptr(A), ld, lay, _ptr(lam), _ptr(V), dt, flags, _ptr(inf),
        _stream_handle(stream, A.device))
    _lib.check(rc, "batched_syev3_info")
    if info:
        return lam, V, inf
    return lam, V


def syev3_inplace(A: torch.Tensor, *, stream=None) -> torch.Tensor:
    """Full matrices A (n, 3, 3), contiguous, are overwritten by their
    eigenvectors (columns); returns the eigenvalues (n, 3), ascending."""
    if not A.is_cuda:
        raise ValueError("A must be a GPU tensor (the solver has no CPU path)")
    if A.dim() != 3 or A.shape[1:] != (3, 3) or not A.is_contiguous():
        raise ValueError("A must be a contiguous (n, 3, 3) tensor")
    lam = torch.empty((A.shape[0], 3), dtype=A.dtype, device=A.device)
    rc = _lib.lib().batched_syev3_inplace(A.shape[0], _ptr(A), _ptr(lam), _dtype_code(A),
                                          _stream_handle(stream, A.device))
    _lib.check(rc, "batched_syev3_inplace")
    return lam
