"""The accuracy experiment of Sec. 1.5 of the paper, re-run on the GPU.

    python -m paper_1806_06698_amd.accuracy [--n 100000] [--seed 0] [--json out.json]

For each entry distribution the paper uses (U(0,1), N(0,1), chi-square with
one degree of freedom), draw n random symmetric 3x3 matrices T, solve them
with this library (FP64, on the GPU) and with LAPACK (numpy.linalg.eigh, the
routine family behind Matlab's eig, which the paper compares against), and
compute per matrix the paper's two measures:

    ||I - V^T V||_F     orthogonality of the computed eigenvectors
    ||T V - V Lambda||_F  accuracy of the spectral factorisation

The measures are evaluated in 80-bit extended precision (numpy.longdouble) so
that differences at the level of one ulp are resolved.  As in the paper, the
per-matrix differences (LAPACK minus ours: negative where ours is worse) are
sorted; the report gives their quantiles and the fractions of matrices where
ours is better, equal, or worse.  The paper's figures are not available, so
there is no printed curve to compare with; its claim is qualitative.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import gen, syev3

DISTS = ("uniform", "normal", "chi2")


def full_ld(A6: np.ndarray) -> np.ndarray:
    """(n, 6) -> (n, 3, 3) symmetric, longdouble."""
    idx = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
    T = np.empty((A6.shape[0], 3, 3), dtype=np.longdouble)
    for k, (i, j) in enumerate(idx):
        T[:, i, j] = A6[:, k]
        T[:, j, i] = A6[:, k]
    return T


def measures(A6: np.ndarray, lam: np.ndarray, V: np.ndarray):
    """The paper's two measures per matrix, in extended precision."""
    T = full_ld(A6)
    Vl = V.astype(np.longdouble)
    Ll = lam.astype(np.longdouble)
    G = np.einsum("nij,nik->njk", Vl, Vl) - np.eye(3, dtype=np.longdouble)
    orth = np.sqrt((G * G).sum(axis=(1, 2)))
    R = np.einsum("nij,njk->nik", T, Vl) - Vl * Ll[:, None, :]
    res = np.sqrt((R * R).sum(axis=(1, 2)))
    return orth.astype(np.float64), res.astype(np.float64)


def _summary(diff: np.ndarray) -> dict:
    d = np.sort(diff)
    q = [0.0, 0.01, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99, 1.0]
    return {"ours_better": float(np.mean(d > 0)), "equal": float(np.mean(d == 0)),
            "ours_worse": float(np.mean(d < 0)),
            "sorted_diff_quantiles_eps": {str(p): float(np.quantile(d, p)) / 2.0 ** -52
                                          for p in q}}


def run(n: int = 100_000, seed: int = 0, device: str = "cuda") -> dict:
    out = {"n": n, "seed": seed, "solver": "libsyev3 FP64 (GPU)",
           "reference": "LAPACK via numpy.linalg.eigh (FP64)",
           "diff": "LAPACK measure minus ours, per matrix (positive: ours better)"}
    for k, dist in enumerate(DISTS):
        A = gen.paper_dist(n, dist, seed=seed + k, device="cpu")
        lam_d, V_d = syev3(A.to(device))
        torch.cuda.synchronize()
        lam = lam_d.t().cpu().numpy()
        V = V_d.t().cpu().numpy().reshape(-1, 3, 3)
        A6 = gen.to_aos(A).numpy()
        w, Q = np.linalg.eigh(full_ld(A6).astype(np.float64))
        o_ours, r_ours = measures(A6, lam, V)
        o_lap, r_lap = measures(A6, w, Q)
        eps = 2.0 ** -52
        out[dist] = {
            "orthogonality": {"ours_median_eps": float(np.median(o_ours)) / eps,
                              "ours_max_eps": float(o_ours.max()) / eps,
                              "lapack_median_eps": float(np.median(o_lap)) / eps,
                              "lapack_max_eps": float(o_lap.max()) / eps,
                              "lapack_minus_ours": _summary(o_lap - o_ours)},
            "residual": {"ours_median_eps": float(np.median(r_ours)) / eps,
                         "ours_max_eps": float(r_ours.max()) / eps,
                         "lapack_median_eps": float(np.median(r_lap)) / eps,
                         "lapack_max_eps": float(r_lap.max()) / eps,
                         "lapack_minus_ours": _summary(r_lap - r_ours)},
        }
    return out


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--n", type=int, default=100_000)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--json", default=None)
    a = p.parse_args()
    res = run(a.n, a.seed)
    for dist in DISTS:
        for m in ("orthogonality", "residual"):
            r = res[dist][m]
            s = r["lapack_minus_ours"]
            print(f"{dist:8s} {m:13s} ours median {r['ours_median_eps']:.3f} eps "
                  f"(max {r['ours_max_eps']:.2f}); LAPACK median {r['lapack_median_eps']:.3f} "
                  f"(max {r['lapack_max_eps']:.2f}); ours better {s['ours_better']:.3f}, "
                  f"equal {s['equal']:.3f}, worse {s['ours_worse']:.3f}")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
