"""Helpers for the GPU tests: run the library through its C ABI binding and
evaluate the paper's measures on the device for batches too large to copy
back (power-of-two scaled, FP64, chunked)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1806_06698_amd as s3

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def soa_to_numpy(lam, V):
    """(3, n), (9, n) device tensors -> (n, 3), (n, 3, 3) float64 numpy."""
    l = lam.t().double().cpu().numpy()
    v = None if V is None else V.t().double().cpu().numpy().reshape(-1, 3, 3)
    return l, v


def solve_soa(A_soa_dev, **kw):
    out = s3.syev3(A_soa_dev, **kw)
    torch.cuda.synchronize()
    return out


def _bmm33(X, Y):
    """(n,3,3) @ (n,3,3) by broadcasting (no batched BLAS call)."""
    return (X[:, :, :, None] * Y[:, None, :, :]).sum(2)


def device_measures(A_soa, lam, V, chunk=1 << 22):
    """Per-matrix residual ||AV - V Lambda||_F / ||A||_F and orthogonality
    ||V^T V - I||_F, computed on the GPU in FP64 after exact power-of-two
    scaling.  Returns (res, orth) float64 device tensors."""
    n = A_soa.shape[1]
    res = torch.empty(n, dtype=torch.float64, device=A_soa.device)
    orth = torch.empty(n, dtype=torch.float64, device=A_soa.device)
    idx = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a = A_soa[:, s:e].double()
        m = a.abs().amax(0)
        _, ex = torch.frexp(torch.where(m > 0, m, torch.ones_like(m)))
        sc = torch.ldexp(torch.ones_like(m), -ex)
        M = torch.empty((e - s, 3, 3), dtype=torch.float64, device=a.device)
        for k, (i, j) in enumerate(idx):
            M[:, i, j] = a[k] * sc
            M[:, j, i] = a[k] * sc
        L = lam[:, s:e].double().t() * sc[:, None]
        W = V[:, s:e].double().t().reshape(-1, 3, 3)
        R = _bmm33(M, W) - W * L[:, None, :]
        fro = torch.linalg.matrix_norm(M)
        r = torch.linalg.matrix_norm(R)
        res[s:e] = torch.where(fro > 0, r / torch.where(fro > 0, fro, torch.ones_like(fro)), r)
        G = _bmm33(W.transpose(1, 2), W) - torch.eye(3, dtype=torch.float64,
                                                       device=a.device)
        orth[s:e] = torch.linalg.matrix_norm(G)
    return res, orth


def sample_indices(n, k, seed, cat=None):
    """k random indices, plus up to k/8 from every category if given."""
    g = np.random.default_rng(seed)
    idx = [g.choice(n, size=min(k, n), replace=False)]
    if cat is not None:
        c = cat.cpu().numpy() if hasattr(cat, "cpu") else cat
        for v in np.unique(c):
            w = np.flatnonzero(c == v)
            idx.append(g.choice(w, size=min(len(w), max(1, k // 8)), replace=False))
    return np.unique(np.concatenate(idx))


def check_vs_oracle(A, lam, V, f32=False, sample=None, seed=0, label=""):
    """Results of the GPU path against the CPU oracle on the same input, at
    the acceptance bars: FP64 16 eps ||A||_F (eigenvalues, residual) and
    16 eps (orthogonality); FP32 storage (refined) 1 eps32 ||A||_F,
    3 eps32 ||A||_F and 3 eps32, against the FP64 oracle on the FP32 values
    widened exactly.  A (6, n) SoA, lam (3, n), V (9, n) or None, on any
    device and of the input's dtype.  sample: check only that many matrices
    (drawn at random with `seed`); None: all.  Returns the worst errors in
    units of the eps of the dtype."""
    import checks
    import oracle
    n = A.shape[1]
    idx = None
    if sample is not None and n > sample:
        idx = torch.from_numpy(np.sort(np.random.default_rng(seed).choice(n, sample,
                                                                           replace=False)))
    def take(t):
        t = t.detach().to("cpu")
        return t[:, idx] if idx is not None else t
    A6 = take(A).double().t().contiguous().numpy()
    l = take(lam).double().t().numpy()
    lam_o, _ = oracle.solve(A6)
    unit = EPS32 / EPS64 if f32 else 1.0
    bar = {"lam": 1.0, "res": 3.0, "orth": 3.0} if f32 else {"lam": 16.0, "res": 16.0,
                                                               "orth": 16.0}
    e = checks.eig_error(A6, l, lam_o).max() / unit
    out = {"lam": e}
    if V is not None:
        v = take(V).double().t().numpy().reshape(-1, 3, 3)
        out["res"] = checks.residual(A6, l, v).max() / unit
        out["orth"] = checks.orthogonality(v).max() / unit
    print(f"  {label} n={n} checked {A6.shape[0]} vs oracle: "
          + ", ".join(f"{k} {x:.2f}" for k, x in out.items())
          + (" eps32" if f32 else " eps"), flush=True)
    for k, x in out.items():
        assert x <= bar[k], f"{label}: {k} error {x:.2f} above {bar[k]}"
    return out
