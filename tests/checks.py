"""Acceptance measures for 3x3 symmetric eigendecompositions (numpy, FP64).

Independent of both the GPU library and the oracle.  The two accuracy
measures are the paper's (Sec. 1.5): ||I - V^T V||_F and ||T V - V Lambda||_F.
Every matrix is first scaled by a power of two (exact) so that its largest
entry lies in [1, 2); the measures are then free of overflow and underflow for
inputs anywhere in the double range, and residuals and eigenvalue errors are
reported in units of eps * ||A||_F.
"""
from __future__ import annotations

import numpy as np

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23
IDX = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def full(A6: np.ndarray) -> np.ndarray:
    """(n, 6) unique entries -> (n, 3, 3) symmetric."""
    A6 = np.asarray(A6, dtype=np.float64)
    M = np.empty((A6.shape[0], 3, 3))
    for k, (i, j) in enumerate(IDX):
        M[:, i, j] = A6[:, k]
        M[:, j, i] = A6[:, k]
    return M


def scale_exponents(A6: np.ndarray) -> np.ndarray:
    m = np.abs(np.asarray(A6, dtype=np.float64)).max(axis=1)
    e = np.zeros(m.shape, dtype=np.int64)
    ok = (m > 0) & np.isfinite(m)
    e[ok] = np.floor(np.log2(m[ok])).astype(np.int64)
    return e


def _scaled(A6, lam):
    e = scale_exponents(A6)
    M = np.ldexp(full(A6), -e[:, None, None])
    L = np.ldexp(np.asarray(lam, dtype=np.float64), -e[:, None])
    fro = np.linalg.norm(M, axis=(1, 2))
    return M, L, fro


def residual(A6, lam, V) -> np.ndarray:
    """||A V - V Lambda||_F / (eps64 ||A||_F) per matrix (0 for A = 0)."""
    M, L, fro = _scaled(A6, lam)
    V = np.asarray(V, dtype=np.float64)
    R = M @ V - V * L[:, None, :]
    r = np.linalg.norm(R, axis=(1, 2))
    out = np.where(fro > 0, r / np.where(fro > 0, fro, 1.0), r)
    return out / EPS64


def orthogonality(V) -> np.ndarray:
    """||V^T V - I||_F / eps64 per matrix."""
    V = np.asarray(V, dtype=np.float64)
    G = np.einsum("nij,nik->njk", V, V) - np.eye(3)
    return np.linalg.norm(G, axis=(1, 2)) / EPS64


def eig_error(A6, lam, lam_ref) -> np.ndarray:
    """max_i |lam_i - lam_ref_i| / (eps64 ||A||_F), both ascending."""
    e = scale_exponents(A6)
    M = np.ldexp(full(A6), -e[:, None, None])
    fro = np.linalg.norm(M, axis=(1, 2))
    d = np.abs(np.ldexp(np.asarray(lam, dtype=np.float64), -e[:, None])
               - np.ldexp(np.asarray(lam_ref, dtype=np.float64), -e[:, None]))
    d = d.max(axis=1)
    return np.where(fro > 0, d / np.where(fro > 0, fro, 1.0), d) / EPS64


def lapack_eigvals(A6) -> np.ndarray:
    """Ascending eigenvalues from LAPACK (numpy.linalg.eigvalsh), computed on
    the power-of-two scaled matrices and scaled back."""
    e = scale_exponents(A6)
    M = np.ldexp(full(A6), -e[:, None, None])
    return np.ldexp(np.linalg.eigvalsh(M), e[:, None])


def invariants(A6, lam):
    """Errors of the characteristic-polynomial invariants, on the scaled
    problem: trace, sum of 2x2 principal minors, determinant, and
    max_i |det(A - lam_i I)|.  Returned divided by eps*||A||_F^k."""
    M, L, fro = _scaled(A6, lam)
    f = np.where(fro > 0, fro, 1.0)
    tr = np.trace(M, axis1=1, axis2=2)
    e_tr = np.abs(L.sum(1) - tr) / f
    minors = (M[:, 0, 0] * M[:, 1, 1] - M[:, 0, 1] ** 2
              + M[:, 0, 0] * M[:, 2, 2] - M[:, 0, 2] ** 2
              + M[:, 1, 1] * M[:, 2, 2] - M[:, 1, 2] ** 2)
    s2 = L[:, 0] * L[:, 1] + L[:, 0] * L[:, 2] + L[:, 1] * L[:, 2]
    e_m = np.abs(s2 - minors) / f ** 2
    det = np.linalg.det(M)
    e_det = np.abs(L.prod(1) - det) / f ** 3
    I = np.eye(3)
    cp = np.stack([np.abs(np.linalg.det(M - L[:, i, None, None] * I))
                   for i in range(3)], 1).max(1)
    e_cp = cp / f ** 3
    return e_tr / EPS64, e_m / EPS64, e_det / EPS64, e_cp / EPS64
