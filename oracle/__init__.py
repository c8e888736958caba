"""CPU oracle for the batched 3x3 real symmetric eigenproblem.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 reference
that the GPU library is checked against.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it;
the product path never does, and it shares no code with the GPU library.

* ``syev3_oracle.c`` -- the method of Borges, "Solving the 3x3 Real Symmetric
  Eigenproblem" (arXiv:1806.06698), Sec. 1 to 1.4, step by step in IEEE double.
* ``jacobi_cyclic.c`` -- textbook cyclic-by-row Jacobi, an independent
  brute-force check of the oracle on small batches.

Array conventions (numpy, float64, C order):
  A    (n, 6)    a11 a12 a13 a22 a23 a33
  lam  (n, 3)    eigenvalues ascending
  V    (n, 3, 3) V[i, :, c] is the unit eigenvector of lam[i, c]
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = ["syev3_oracle.c", "jacobi_cyclic.c"]

# flags (values are the oracle's own; the GPU library keeps its own table)
SIMPLIFIED_DEFLATION = 1
NO_H_GUARD = 2
NEWTON = 4
NO_SCALE = 8

# branch codes in info[:, 0]
BR_ZERO, BR_NONFINITE, BR_DIAGONAL, BR_DEFLATED, BR_REDUCED = range(5)

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-pthread"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_SO):
        srcs = [os.path.join(_HERE, s) for s in _SRCS]
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_solve_batch.argtypes = [ctypes.c_int64, dp, dp, dp,
                                           ctypes.c_uint, ip, ctypes.c_int]
        lib.oracle_solve_batch.restype = ctypes.c_int
        lib.oracle_solve.argtypes = [dp, dp, dp, ctypes.c_uint, ip]
        lib.oracle_solve.restype = None
        for name in ("oracle_bg_root", "oracle_newton_root"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_double] * 4 + [ip, dp, ctypes.c_int]
            fn.restype = ctypes.c_double
        lib.oracle_spec_f.argtypes = [ctypes.c_double] * 5
        lib.oracle_spec_f.restype = ctypes.c_double
        lib.oracle_spec_fp.argtypes = [ctypes.c_double] * 4
        lib.oracle_spec_fp.restype = ctypes.c_double
        lib.oracle_arrow.argtypes = [dp, dp, dp]
        lib.oracle_arrow.restype = None
        lib.oracle_jacobi2.argtypes = [ctypes.c_double] * 3 + [dp, dp]
        lib.oracle_jacobi2.restype = None
        lib.jacobi_cyclic_batch.argtypes = [ctypes.c_int64, dp, dp, dp, ip]
        lib.jacobi_cyclic_batch.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _as_aos(A) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    if A.ndim != 2 or A.shape[1] != 6:
        raise ValueError("A must be (n, 6) float64: a11 a12 a13 a22 a23 a33")
    return A


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1


def solve(A, flags: int = 0, nthreads: int | None = None, vecs: bool = True,
          return_info: bool = False):
    """Eigen-decompose n symmetric 3x3 matrices given as (n, 6) rows.

    Returns (lam (n,3), V (n,3,3)) and, with return_info, info (n,4):
    branch, BG/Newton iterations for mu, for nu, and the scaling exponent.
    """
    lib = _load()
    A = _as_aos(A)
    n = A.shape[0]
    lam = np.empty((n, 3), dtype=np.float64)
    V = np.empty((n, 3, 3), dtype=np.float64) if vecs else None
    info = np.empty((n, 4), dtype=np.int32) if return_info else None
    nt = nthreads if nthreads is not None else default_threads()
    if n:
        rc = lib.oracle_solve_batch(
            n, _dp(A), _dp(lam),
            _dp(V) if V is not None else ctypes.POINTER(ctypes.c_double)(),
            flags, _ip(info) if info is not None else ctypes.POINTER(ctypes.c_int)(),
            nt)
        if rc != 0:
            raise RuntimeError(f"oracle_solve_batch returned {rc}")
    out = (lam, V)
    if return_info:
        out = out + (info,)
    return out


def bg_root(b1, b2, ab, gb, trace_cap: int = 0):
    """Borges-Gragg zero of the fully reduced arrow; (root, iters, trace)."""
    lib = _load()
    it = np.zeros(1, dtype=np.int32)
    tr = np.full(max(trace_cap, 1), np.nan)
    x = lib.oracle_bg_root(b1, b2, ab, gb, _ip(it), _dp(tr), trace_cap)
    return x, int(it[0]), tr[: min(int(it[0]), trace_cap)]


def newton_root(b1, b2, ab, gb, trace_cap: int = 0):
    """Newton zero (from the left) of the fully reduced arrow."""
    lib = _load()
    it = np.zeros(1, dtype=np.int32)
    tr = np.full(max(trace_cap, 1), np.nan)
    x = lib.oracle_newton_root(b1, b2, ab, gb, _ip(it), _dp(tr), trace_cap)
    return x, int(it[0]), tr[: min(int(it[0]), trace_cap)]


def spec_f(b1, b2, ab, gb, x):
    return _load().oracle_spec_f(b1, b2, ab, gb, x)


def spec_fp(b1, b2, ab, x):
    return _load().oracle_spec_fp(b1, b2, ab, x)


def arrow(a6):
    """Ordered arrow of one matrix: (alpha1, alpha2, beta1, beta2, gamma), J."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(a6, dtype=np.float64).reshape(6))
    out = np.empty(5)
    J = np.empty(4)
    lib.oracle_arrow(_dp(a), _dp(out), _dp(J))
    return out, J.reshape(2, 2)


def jacobi2(p, r, q):
    """2x2 [[p, r], [r, q]]: ((l1, l2), K) with l1 >= l2, K columns vectors."""
    lib = _load()
    out = np.empty(2)
    K = np.empty(4)
    lib.oracle_jacobi2(p, r, q, _dp(out), _dp(K))
    return out, K.reshape(2, 2)


def jacobi_cyclic(A):
    """Brute-force cyclic Jacobi on (n, 6) rows: (lam, V, sweeps)."""
    lib = _load()
    A = _as_aos(A)
    n = A.shape[0]
    lam = np.empty((n, 3))
    V = np.empty((n, 3, 3))
    sw = np.empty(n, dtype=np.int32)
    if n:
        lib.jacobi_cyclic_batch(n, _dp(A), _dp(lam), _dp(V), _ip(sw))
    return lam, V, sw
