"""Closed-form eigendecompositions (tests/golden/closed_forms.json) against
the oracle (no GPU) and the library (GPU).

The fixtures come from mathematics, not from either implementation: each
case cites the fact that gives its eigenvalues and eigenvectors, and the
first test checks every case's own consistency (A v = lambda v, to 50
digits) before any solver is trusted with it.  Each case is also run scaled
by 2^600 and 2^-600 (exact), which exercises the power-of-two scaling.

Bars (per case, eps = 2^-52):
  |lambda_i - exact_i| <= 4 eps ||A||_F       (oracle; 16 for the GPU path)
  simple eigenvalue:  ||v -+ v_exact|| <= 8 eps ||A||_F / gap
  double eigenvalue:  ||P - P_exact||_F <= 8 eps ||A||_F / gap
(the eigenvector bounds are Davis-Kahan's sin(theta) <= ||residual|| / gap
with the residual at the bars above).
"""
import json
import os

import mpmath
import numpy as np
import pytest

import oracle

EPS = 2.0 ** -52
HERE = os.path.dirname(os.path.abspath(__file__))
# working precision of every mpmath evaluation here, set per use (workdps)
# so that no other test module's precision leaks in or out
DPS = 50


def _cases():
    with open(os.path.join(HERE, "golden", "closed_forms.json")) as fh:
        return json.load(fh)["cases"]


CASES = _cases()
SCALES = [0, 600, -600]


_NAMES = {"sqrt": mpmath.sqrt, "sin": mpmath.sin, "cos": mpmath.cos, "pi": mpmath.pi}


def _value(expr):
    """An expression of the fixture file (numbers, + - * /, sqrt, sin, cos,
    pi), evaluated in the caller's working precision (DPS digits)."""
    return mpmath.mpf(eval(expr, {"__builtins__": {}}, dict(_NAMES)))


def _exact(case):
    with mpmath.workdps(DPS):
        lam = [_value(e) for e in case["lambda"]]
        vecs = []
        for v in case["vectors"]:
            if v is None:
                vecs.append(None)
                continue
            u = mpmath.matrix([_value(e) for e in v])
            vecs.append(u / mpmath.norm(u))
    return lam, vecs


def _full(A6):
    a = A6
    return np.array([[a[0], a[1], a[2]], [a[1], a[3], a[4]], [a[2], a[4], a[5]]], dtype=float)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_fixture_is_consistent(case):
    with mpmath.workdps(DPS):
        lam, vecs = _exact(case)
        A = mpmath.matrix(_full(case["A6"]).tolist())
        assert lam == sorted(lam)
        assert abs(sum(lam) - sum(A[i, i] for i in range(3))) < mpmath.mpf(10) ** -40
        for l, v in zip(lam, vecs):
            if v is not None:
                assert mpmath.norm(A * v - l * v) < mpmath.mpf(10) ** -40
        # eigenvalues against the characteristic polynomial's roots, by mpmath
        ev = sorted(mpmath.eigsy(A)[0])
        for a, b in zip(ev, lam):
            assert abs(a - b) < mpmath.mpf(10) ** -40


def _check(case, scale, lam, V, tol):
    """lam (3,), V (3, 3) columns, for A scaled by 2^scale."""
    lam_e, vecs = _exact(case)
    A = _full(case["A6"])
    fro = np.linalg.norm(A)
    lam_u = np.ldexp(np.asarray(lam, dtype=float), -scale)
    lam_e = np.array([float(x) for x in lam_e])
    err = np.abs(lam_u - lam_e) / (EPS * fro)
    assert err.max() <= tol, (case["name"], scale, err)
    for i, v in enumerate(vecs):
        if v is None:
            continue
        ve = np.array([float(x) for x in v])
        others = [lam_e[j] for j in range(3) if j != i]
        gap = min(abs(lam_e[i] - o) for o in others)
        d = min(np.linalg.norm(V[:, i] - ve), np.linalg.norm(V[:, i] + ve))
        assert d <= 2 * tol * EPS * fro / gap, (case["name"], scale, i, d)
        # a double eigenvalue: its computed eigenspace is the complement of ve
        if sum(1 for x in vecs if x is None) == 2:
            P = np.eye(3) - np.outer(ve, ve)
            cols = [j for j in range(3) if j != i]
            Pc = V[:, cols] @ V[:, cols].T
            assert np.linalg.norm(Pc - P) <= 2 * tol * EPS * fro / gap


@pytest.mark.parametrize("scale", SCALES)
@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_oracle_matches_closed_form(oracle_mod, case, scale):
    A6 = np.ldexp(np.array([case["A6"]], dtype=float), scale)
    lam, V = oracle_mod.solve(A6)
    _check(case, scale, lam[0], V[0], 4.0)


@pytest.mark.gpu
@pytest.mark.parametrize("scale", SCALES)
def test_library_matches_closed_form(scale):
    import torch
    from gpu_common import need_gpu
    need_gpu()
    import paper_1806_06698_amd as s3
    A6 = np.ldexp(np.array([c["A6"] for c in CASES], dtype=float), scale)
    lam, V = s3.syev3(torch.from_numpy(A6).cuda().contiguous(), layout="aos")
    torch.cuda.synchronize()
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    for k, case in enumerate(CASES):
        _check(case, scale, lam[k], V[k], 16.0)
