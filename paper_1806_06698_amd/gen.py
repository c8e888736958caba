"""Seeded synthetic inputs for batched 3x3 symmetric eigenproblems.

This module only draws matrices; it holds none of the solver's arithmetic and
is shared by the GPU path's tests and benchmark and by the CPU oracle's tests.
Every generator returns a structure-of-arrays float64 tensor of shape (6, n)
whose rows are the unique entries (a11, a12, a13, a22, a23, a33), on the
requested device, drawn from a torch generator seeded with ``seed``.  Results
for one seed differ between CPU and GPU generators: a test draws on one device
and copies to the other.

Workloads (the paper draws random symmetric matrices, Sec. 1.5; the larger
mixes add the numerically hard cases the method singles out in Sec. 1.1):

* ``normal``      entries iid N(0, 1).
* ``stress_mix``  70% iid N(0,1); 10% exactly diagonal; 10% Q diag(l, l(1+d), m)
                  Q^T with Haar Q, l, m ~ N(0,1), d = 10^U(-16,-4); 10% arrow-like
                  (a12 = 0) whose betas straddle the deflation threshold.
* ``spd_fe``      Q diag(e^x1, e^x2, e^x3) Q^T, x_i ~ U(0, ln 1e8): SPD blocks with
                  condition number up to 1e8, shaped like finite-element stiffness.
* ``wide_range``  N(0,1) entries times 10^U(-150,150) per matrix, plus 1% exact
                  multiples of the identity and 1% zero matrices.
* ``paper_dist``  entries iid U(0,1), N(0,1) or chi-square(1) (Sec. 1.5).
"""
from __future__ import annotations

import math

import torch

ENTRY_NAMES = ("a11", "a12", "a13", "a22", "a23", "a33")

# category labels returned by the mixed generators
CAT_NORMAL, CAT_DIAGONAL, CAT_NEAR_DEGENERATE, CAT_ARROW = 0, 1, 2, 3
CAT_WIDE, CAT_SCALAR_IDENTITY, CAT_ZERO = 4, 5, 6


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _randn(n, g, device):
    return torch.randn(n, generator=g, device=device, dtype=torch.float64)


def _rand(n, g, device):
    return torch.rand(n, generator=g, device=device, dtype=torch.float64)


def haar_rotation(n: int, g: torch.Generator, device) -> torch.Tensor:
    """(3, 3, n) rotations, Haar-distributed on SO(3).

    A unit quaternion with iid normal components is uniform on the 3-sphere,
    and its rotation matrix is then Haar on SO(3).  Q D Q^T is unchanged by
    Q -> -Q, so SO(3) covers the orthogonal group for these workloads.
    """
    q = torch.stack([_randn(n, g, device) for _ in range(4)])
    q = q / torch.linalg.vector_norm(q, dim=0, keepdim=True)
    w, x, y, z = q
    R = torch.empty((3, 3, n), dtype=torch.float64, device=device)
    R[0, 0] = 1 - 2 * (y * y + z * z)
    R[0, 1] = 2 * (x * y - w * z)
    R[0, 2] = 2 * (x * z + w * y)
    R[1, 0] = 2 * (x * y + w * z)
    R[1, 1] = 1 - 2 * (x * x + z * z)
    R[1, 2] = 2 * (y * z - w * x)
    R[2, 0] = 2 * (x * z - w * y)
    R[2, 1] = 2 * (y * z + w * x)
    R[2, 2] = 1 - 2 * (x * x + y * y)
    return R


def q_diag_qt(Q: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """Unique entries of Q diag(d) Q^T for Q (3,3,n) and d (3,n) -> (6,n)."""
    idx = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
    out = torch.empty((6, Q.shape[2]), dtype=torch.float64, device=Q.device)
    for e, (i, j) in enumerate(idx):
        out[e] = (Q[i, 0] * d[0] * Q[j, 0] + Q[i, 1] * d[1] * Q[j, 1]
                  + Q[i, 2] * d[2] * Q[j, 2])
    return out


def normal(n: int, seed: int = 0, device="cpu") -> torch.Tensor:
    """(6, n) with iid N(0,1) unique entries."""
    g = _gen(seed, device)
    return torch.randn((6, n), generator=g, device=device, dtype=torch.float64)


def stress_mix(n: int, seed: int = 1, device="cpu"):
    """(A (6,n), cat (n,) int8): the stress mix with categories interleaved
    at random per matrix (the worst case for divergence inside a wavefront).

    Arrow-like slice (a12 = 0): in half of it one randomly chosen beta entry is
    N(0,1) 10^U(-18,-8) and the other N(0,1), so the coupling of the Givens
    form straddles the deflation threshold; in the other half both betas are
    scaled independently.  1% of the slice has a11 == a22 (combo-deflation).
    """
    g = _gen(seed, device)
    A = torch.randn((6, n), generator=g, device=device, dtype=torch.float64)
    u = _rand(n, g, device)
    cat = torch.full((n,), CAT_NORMAL, dtype=torch.int8, device=device)
    diag = (u >= 0.70) & (u < 0.80)
    neardeg = (u >= 0.80) & (u < 0.90)
    arrow = u >= 0.90
    cat[diag] = CAT_DIAGONAL
    cat[neardeg] = CAT_NEAR_DEGENERATE
    cat[arrow] = CAT_ARROW

    # exactly diagonal
    for e in (1, 2, 4):
        A[e] = torch.where(diag, torch.zeros_like(A[e]), A[e])

    # near-degenerate pair: Q diag(l, l(1+d), m) Q^T
    Q = haar_rotation(n, g, device)
    lv = _randn(n, g, device)
    mv = _randn(n, g, device)
    dv = torch.pow(10.0, -16.0 + 12.0 * _rand(n, g, device))
    Aq = q_diag_qt(Q, torch.stack([lv, lv * (1 + dv), mv]))
    del Q
    A = torch.where(neardeg.unsqueeze(0), Aq, A)
    del Aq

    # arrow-like: a12 = 0, betas straddling the deflation threshold
    s13 = torch.pow(10.0, -18.0 + 10.0 * _rand(n, g, device))
    s23 = torch.pow(10.0, -18.0 + 10.0 * _rand(n, g, device))
    half = _rand(n, g, device) < 0.5           # one beta scaled
    which = _rand(n, g, device) < 0.5          # which one (a13 or a23)
    combo = _rand(n, g, device) < 0.01         # a11 == a22 exactly
    one = torch.ones_like(s13)
    f13 = torch.where(half, torch.where(which, s13, one), s13)
    f23 = torch.where(half, torch.where(which, one, s23), s23)
    A[1] = torch.where(arrow, torch.zeros_like(A[1]), A[1])
    A[2] = torch.where(arrow, A[2] * f13, A[2])
    A[4] = torch.where(arrow, A[4] * f23, A[4])
    A[3] = torch.where(arrow & combo, A[0], A[3])
    return A, cat


def spd_fe(n: int, seed: int = 2, device="cpu") -> torch.Tensor:
    """(6, n) SPD Q diag(e^x1, e^x2, e^x3) Q^T, x_i ~ U(0, ln 1e8)."""
    g = _gen(seed, device)
    Q = haar_rotation(n, g, device)
    lmax = math.log(1e8)
    d = torch.exp(lmax * torch.rand((3, n), generator=g, device=device,
                                    dtype=torch.float64))
    return q_diag_qt(Q, d)


def wide_range(n: int, seed: int = 4, device="cpu"):
    """(A (6,n), cat): N(0,1) * 10^U(-150,150) per matrix; 1% lambda*I exactly;
    1% exactly zero."""
    g = _gen(seed, device)
    A = torch.randn((6, n), generator=g, device=device, dtype=torch.float64)
    scale = torch.pow(10.0, -150.0 + 300.0 * _rand(n, g, device))
    A *= scale
    u = _rand(n, g, device)
    cat = torch.full((n,), CAT_WIDE, dtype=torch.int8, device=device)
    ident = u < 0.01
    zero = (u >= 0.01) & (u < 0.02)
    cat[ident] = CAT_SCALAR_IDENTITY
    cat[zero] = CAT_ZERO
    lam = A[0]
    for e in (1, 2, 4):
        A[e] = torch.where(ident, torch.zeros_like(A[e]), A[e])
    A[3] = torch.where(ident, lam, A[3])
    A[5] = torch.where(ident, lam, A[5])
    A = torch.where(zero.unsqueeze(0), torch.zeros_like(A), A)
    return A, cat


def paper_dist(n: int, dist: str, seed: int = 0, device="cpu") -> torch.Tensor:
    """(6, n) entries iid from 'uniform' U(0,1), 'normal' N(0,1) or
    'chi2' chi-square with one degree of freedom (Sec. 1.5)."""
    g = _gen(seed, device)
    shape = (6, n)
    if dist == "uniform":
        return torch.rand(shape, generator=g, device=device, dtype=torch.float64)
    z = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    if dist == "normal":
        return z
    if dist == "chi2":
        return z * z
    raise ValueError(f"unknown distribution {dist!r}")


def to_aos(A_soa: torch.Tensor) -> torch.Tensor:
    """(6, n) -> contiguous (n, 6)."""
    return A_soa.t().contiguous()


def to_full(A_soa: torch.Tensor) -> torch.Tensor:
    """(6, n) -> (n, 3, 3) full symmetric matrices."""
    a11, a12, a13, a22, a23, a33 = A_soa
    return torch.stack([torch.stack([a11, a12, a13], -1),
                        torch.stack([a12, a22, a23], -1),
                        torch.stack([a13, a23, a33], -1)], -2)


CONFIGS = {
    # name: (n, generator, seed)
    "normal_4k": (4096, "normal", 0),
    "stress_mix_16m": (1 << 24, "stress_mix", 1),
    "spd_fe_64m": (1 << 26, "spd_fe", 2),
    "wide_range_256m": (1 << 28, "wide_range", 4),
}


def make(kind: str, n: int, seed: int, device="cpu"):
    """(A (6,n), cat or None) for a generator name."""
    if kind == "normal":
        return normal(n, seed, device), None
    if kind == "stress_mix":
        return stress_mix(n, seed, device)
    if kind == "spd_fe":
        return spd_fe(n, seed, device), None
    if kind == "wide_range":
        return wide_range(n, seed, device)
    if kind in ("uniform", "chi2"):
        return paper_dist(n, kind, seed, device), None
    raise ValueError(kind)
