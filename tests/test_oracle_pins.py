"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test pins one part of the oracle to something other than itself:
exact special cases the paper states (Sec. 1.1), closed forms of the 2x2
problem, Cauchy interlacing for the arrow reduction (Sec. 1), the properties
of the spectral function and of both zero finders (Sec. 1.4), the
orthogonality bound (Sec. 1.3), the characteristic-polynomial invariants, the
paper's two accuracy measures (Sec. 1.5), LAPACK (the paper's own comparison)
and a brute-force cyclic Jacobi.  No GPU.
"""
import numpy as np
import pytest
import torch

import checks
from deflation_cases import DEFLATION_BRANCHES, DEFLATION_CASES
from paper_1806_06698_amd import gen

EPS = 2.0 ** -52
TOL = 16.0  # acceptance bound, in eps (times ||A||_F where it applies)


def _aos(A_soa):
    return gen.to_aos(A_soa).numpy()


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# Exact cases (Sec. 1.1: h = 0 means diagonal; beta- and combo-deflation)
# --------------------------------------------------------------------------

def test_diagonal_input_is_exact(oracle_mod):
    rng = _rng(1)
    n = 2000
    A = np.zeros((n, 6))
    d = rng.standard_normal((n, 3))
    d[::7, 1] = d[::7, 0]           # ties
    d[::11, 2] = 0.0
    A[:, 0], A[:, 3], A[:, 5] = d[:, 0], d[:, 1], d[:, 2]
    lam, V, info = oracle_mod.solve(A, return_info=True)
    assert np.array_equal(lam, np.sort(d, axis=1))
    assert np.all(info[:, 0] == oracle_mod.BR_DIAGONAL)
    # V is a signed permutation, bitwise
    assert np.all(np.isin(V, (-1.0, 0.0, 1.0)))
    assert np.all(np.abs(V).sum(axis=1) == 1.0)
    assert np.all(np.abs(V).sum(axis=2) == 1.0)
    # and it maps the diagonal onto the sorted eigenvalues
    assert np.all(checks.residual(A, lam, V) == 0.0)


def _closed_form_2x2(p, q, r):
    m = 0.5 * (p + q)
    h = np.hypot(0.5 * (p - q), r)
    return m - h, m + h


@pytest.mark.parametrize("zero_entry", [2, 4])  # a13 = 0 or a23 = 0
def test_beta_deflation_is_exact(oracle_mod, zero_entry):
    rng = _rng(2 + zero_entry)
    n = 3000
    A = rng.standard_normal((n, 6))
    A[:, 1] = 0.0                    # a12 = 0: already an arrow
    A[:, zero_entry] = 0.0           # one beta exactly zero
    lam, V, info = oracle_mod.solve(A, return_info=True)
    assert np.all(info[:, 0] == oracle_mod.BR_DEFLATED)
    # the deflated eigenvalue is the matching diagonal entry, bitwise
    keep = 0 if zero_entry == 2 else 3
    assert np.all((lam == A[:, [keep]]).any(axis=1))
    # the other two: textbook 2x2 closed form of the remaining block
    if zero_entry == 2:
        p, q, r = A[:, 3], A[:, 5], A[:, 4]
    else:
        p, q, r = A[:, 0], A[:, 5], A[:, 2]
    lo, hi = _closed_form_2x2(p, q, r)
    fro = np.linalg.norm(checks.full(A), axis=(1, 2))
    for i in range(n):
        rest = list(lam[i])
        rest.remove(A[i, keep])
        rest = sorted(rest)
        assert abs(rest[0] - lo[i]) <= 4 * EPS * fro[i]
        assert abs(rest[1] - hi[i]) <= 4 * EPS * fro[i]
    assert checks.residual(A, lam, V).max() <= TOL


def test_combo_deflation_is_exact(oracle_mod):
    rng = _rng(5)
    n = 3000
    A = rng.standard_normal((n, 6))
    A[:, 1] = 0.0
    A[:, 3] = A[:, 0]                # alpha1 == alpha2
    lam, V, info = oracle_mod.solve(A, return_info=True)
    assert np.all(info[:, 0] == oracle_mod.BR_DEFLATED)
    assert np.all((lam == A[:, [0]]).any(axis=1))
    assert checks.residual(A, lam, V).max() <= TOL
    assert checks.orthogonality(V).max() <= TOL




def test_deflation_and_h_tests_decide_as_stated(oracle_mod):
    """Each deflation test and the h guard take the branch that the stated
    inequality gives, with margins of a factor 20 or more; every branch
    gives eigenvalues within 1 eps ||A|| of LAPACK's."""
    A = DEFLATION_CASES
    ref = checks.lapack_eigvals(A)
    for flags, want in DEFLATION_BRANCHES.items():
        lam, V, info = oracle_mod.solve(A, flags=flags, return_info=True)
        assert info[:, 0].tolist() == want, flags
        assert checks.eig_error(A, lam, ref).max() <= 1.0
        assert checks.residual(A, lam, V).max() <= TOL
        assert checks.orthogonality(V).max() <= TOL


def test_zero_and_scalar_identity(oracle_mod):
    A = np.zeros((4, 6))
    for i, s in enumerate([0.0, 3.5, -1e-300, 7e250]):
        A[i, 0] = A[i, 3] = A[i, 5] = s
    lam, V = oracle_mod.solve(A)
    for i in range(4):
        assert np.all(lam[i] == A[i, 0])
        assert np.array_equal(V[i], np.eye(3))


def test_nonfinite_input_gives_nan(oracle_mod):
    A = np.ones((3, 6))
    A[0, 2] = np.nan
    A[1, 4] = np.inf
    A[2, 0] = -np.inf
    lam, V, info = oracle_mod.solve(A, return_info=True)
    assert np.all(np.isnan(lam)) and np.all(np.isnan(V))
    assert np.all(info[:, 0] == oracle_mod.BR_NONFINITE)


def test_power_of_two_scaling_is_bitwise(oracle_mod):
    """lambda(2^j A) = 2^j lambda(A) and V(2^j A) = V(A), bitwise, wherever
    no entry of 2^j A leaves the normal range."""
    A_soa, _ = gen.stress_mix(3000, seed=11)
    A = _aos(A_soa)
    A = A[np.abs(A).min(axis=1) > 1e-30]      # keep 2^j A normal below
    lam0, V0 = oracle_mod.solve(A)
    for j in (-900, -301, -1, 1, 77, 900):
        lam, V = oracle_mod.solve(np.ldexp(A, j))
        assert np.array_equal(lam, np.ldexp(lam0, j)), j
        assert np.array_equal(V, V0), j


# --------------------------------------------------------------------------
# Sec. 1: arrow reduction
# --------------------------------------------------------------------------

def test_arrow_reduction_and_interlacing(oracle_mod):
    rng = _rng(7)
    A = rng.standard_normal((500, 6))
    lam_np = checks.lapack_eigvals(A)
    fro = np.linalg.norm(checks.full(A), axis=(1, 2))
    for i in range(A.shape[0]):
        (a1, a2, b1, b2, g), J = oracle_mod.arrow(A[i])
        B = np.array([[A[i, 0], A[i, 1]], [A[i, 1], A[i, 3]]])
        # J orthogonal, J^T B J = diag(a1, a2) with a1 >= a2
        assert np.abs(J.T @ J - np.eye(2)).max() <= 2 * EPS
        D = J.T @ B @ J
        assert abs(D[0, 1]) <= 4 * EPS * np.abs(B).max()
        assert a1 >= a2
        lo, hi = _closed_form_2x2(B[0, 0], B[1, 1], B[0, 1])
        assert abs(a1 - hi) <= 4 * EPS * np.abs(B).max()
        assert abs(a2 - lo) <= 4 * EPS * np.abs(B).max()
        # beta = J^T (a13, a23), gamma = a33
        bb = J.T @ np.array([A[i, 2], A[i, 4]])
        assert np.allclose([b1, b2], bb, rtol=0, atol=2 * EPS * np.abs(bb).max())
        assert g == A[i, 5]
        # Cauchy interlacing: l3 <= a2 <= l2 <= a1 <= l1
        l3, l2, l1 = lam_np[i]
        t = 4 * EPS * fro[i]
        assert l3 <= a2 + t and a2 <= l2 + t and l2 <= a1 + t and a1 <= l1 + t


# --------------------------------------------------------------------------
# Sec. 1.4: spectral function and zero finders
# --------------------------------------------------------------------------

def _reduced_arrows(oracle_mod, n, seed):
    """Fully reduced arrows (b1, b2, abar, gbar) taken from random matrices
    and from the near-deflation slice of the stress mix."""
    A_soa, _ = gen.stress_mix(n, seed=seed)
    A = _aos(A_soa)
    _, _, info = oracle_mod.solve(A, return_info=True)
    out = []
    for i in np.where(info[:, 0] == oracle_mod.BR_REDUCED)[0]:
        a = np.ldexp(A[i], -int(info[i, 3]))
        (a1, a2, b1, b2, g), _ = oracle_mod.arrow(a)
        out.append((b1, b2, a1 - a2, g - a1))   # mu problem
        out.append((b2, b1, a1 - a2, a2 - g))   # nu problem
    return out


def _f_noise(b1, b2, ab, gb, x):
    """Rounding floor of a computed zero of f: the sum of the magnitudes of
    the terms of f divided by f'."""
    terms = abs(x) + abs(gb) + b1 * b1 / x + b2 * b2 / (x + ab)
    fp = 1.0 + (b1 / x) ** 2 + (b2 / (x + ab)) ** 2
    return terms / fp


def test_spectral_function_shape(oracle_mod):
    """f' >= 1 and f' strictly decreasing on (0, inf) (f'' < 0)."""
    arrows = _reduced_arrows(oracle_mod, 400, 21)
    xs = np.logspace(-12, 3, 60)
    for b1, b2, ab, gb in arrows[:200]:
        fp = np.array([oracle_mod.spec_fp(b1, b2, ab, x) for x in xs])
        assert np.all(fp >= 1.0)
        assert np.all(np.diff(fp) <= 0.0)


def test_bg_monotone_from_right(oracle_mod):
    arrows = _reduced_arrows(oracle_mod, 3000, 22)
    assert len(arrows) > 1000
    for b1, b2, ab, gb in arrows:
        x, it, tr = oracle_mod.bg_root(b1, b2, ab, gb, trace_cap=64)
        xn, _, _ = oracle_mod.newton_root(b1, b2, ab, gb)
        # x0 is the positive zero of the model from +infinity,
        # x^2 - gb x - (b1^2 + b2^2) = 0 (Sec. 1.4.1)
        x0, H = tr[0], b1 * b1 + b2 * b2
        assert x0 > 0
        assert abs(x0 * x0 - gb * x0 - H) <= 8 * EPS * (x0 * x0 + abs(gb) * x0 + H)
        # start to the right of the root, iterates strictly decreasing
        assert tr[0] >= x
        assert np.all(np.diff(tr) < 0)
        # f > 0 at every iterate before the last (right of the root)
        for xj in tr[:-1]:
            assert oracle_mod.spec_f(b1, b2, ab, gb, xj) > 0
        # a second method reaches the same zero, to within what rounding in
        # the evaluation of f allows: |dx| <= eps * sum|terms of f| / f'
        assert abs(x - xn) <= 8 * EPS * max(x, _f_noise(b1, b2, ab, gb, x))


def test_bg_cubic_convergence(oracle_mod):
    """Sec. 1.4.1: the order estimate log(e2/e1)/log(e1/e0) from three
    successive relative errors is 3 (whatever the asymptotic constant).  The
    errors are measured against the largest eigenvalue of the fully reduced
    arrow from a 40-digit library eigensolver, and only above the rounding
    floor of the evaluation of f."""
    mpmath = pytest.importorskip("mpmath")
    arrows = _reduced_arrows(oracle_mod, 1500, 22)
    orders = []
    for b1, b2, ab, gb in arrows:
        x, _, tr = oracle_mod.bg_root(b1, b2, ab, gb, trace_cap=64)
        if len(tr) < 3:
            continue
        # 40 digits for this test only (workdps restores the caller's)
        with mpmath.workdps(40):
            M = mpmath.matrix([[0, 0, b1], [0, -ab, b2], [b1, b2, gb]])
            root = max(mpmath.eigsy(M, eigvals_only=True))
            e = [float(abs((mpmath.mpf(float(t)) - root) / root)) for t in tr]
        floor = 1e3 * EPS * max(1.0, _f_noise(b1, b2, ab, gb, x) / x)
        for j in range(len(e) - 2):
            if e[j] < 0.5 and e[j + 2] > floor:
                orders.append(np.log(e[j + 2] / e[j + 1])
                              / np.log(e[j + 1] / e[j]))
    assert len(orders) >= 20
    assert min(orders) > 2.5 and np.median(orders) > 2.8


def test_bg_root_matches_lapack(oracle_mod):
    """The BG zero is the largest eigenvalue of the fully reduced arrow."""
    arrows = _reduced_arrows(oracle_mod, 1500, 23)
    for b1, b2, ab, gb in arrows:
        M = np.array([[0, 0, b1], [0, -ab, b2], [b1, b2, gb]])
        top = np.linalg.eigvalsh(M)[-1]
        x, _, _ = oracle_mod.bg_root(b1, b2, ab, gb)
        assert abs(x - top) <= 8 * EPS * np.linalg.norm(M)


def test_newton_monotone_from_left(oracle_mod):
    arrows = _reduced_arrows(oracle_mod, 2000, 24)
    for b1, b2, ab, gb in arrows:
        x, it, tr = oracle_mod.newton_root(b1, b2, ab, gb, trace_cap=64)
        assert np.all(np.diff(tr) > 0)
        for xj in tr[:-1]:
            assert oracle_mod.spec_f(b1, b2, ab, gb, xj) < 0


def test_near_pole_roots_keep_relative_accuracy(oracle_mod):
    """Arrows with one beta just above the deflation threshold have a root
    next to the pole at 0 (~1e-30 here).  Newton from the left never
    cancels; BG must reach the same root to high relative precision."""
    cases = [(1.296e-15, 9.766e-04, 0.735, 0.5587 - 1.400),
             (7.0e-15, 0.5543, 2.38, 0.7081 - 1.661),
             (2.168e-01, 1.489e-11, 1.593, -1.317 - 1.484)]
    for b1, b2, ab, gb in cases:
        for bb1, bb2, g in ((b1, b2, gb), (b2, b1, -gb - ab)):
            x, _, tr = oracle_mod.bg_root(bb1, bb2, ab, g, trace_cap=64)
            xn, _, _ = oracle_mod.newton_root(bb1, bb2, ab, g)
            assert x > 0 and abs(x - xn) <= 4 * EPS * x


# --------------------------------------------------------------------------
# Whole-solve pins: invariants, orthogonality, paper measures, LAPACK, Jacobi
# --------------------------------------------------------------------------

WORKLOADS = [("normal", 0), ("stress_mix", 1), ("spd_fe", 2),
             ("wide_range", 4), ("uniform", 5), ("chi2", 6)]


@pytest.mark.parametrize("kind,seed", WORKLOADS)
def test_paper_measures_and_invariants(oracle_mod, kind, seed):
    A_soa, _ = gen.make(kind, 20000, seed)
    A = _aos(A_soa)
    lam, V = oracle_mod.solve(A)
    assert np.all(np.diff(lam, axis=1) >= 0)
    assert checks.residual(A, lam, V).max() <= TOL
    assert checks.orthogonality(V).max() <= TOL
    e_tr, e_m, e_det, e_cp = checks.invariants(A, lam)
    assert e_tr.max() <= 51
    assert e_m.max() <= 100
    assert e_det.max() <= 100
    assert e_cp.max() <= 80
    assert checks.eig_error(A, lam, checks.lapack_eigvals(A)).max() <= TOL


def test_u1_u3_orthogonality_bound(oracle_mod):
    """Sec. 1.3: |u1^T u3| <= 2 eps + O(eps^2) on reduced arrows.  The
    columns of V for lambda1 and lambda3 carry the back-transform rounding
    too, so the bound checked is 4 eps."""
    A_soa, _ = gen.stress_mix(20000, seed=31)
    A = _aos(A_soa)
    lam, V, info = oracle_mod.solve(A, return_info=True)
    red = info[:, 0] == oracle_mod.BR_REDUCED
    dots = np.abs(np.einsum("ni,ni->n", V[red, :, 0], V[red, :, 2]))
    assert dots.max() <= 4 * EPS


@pytest.mark.parametrize("kind,seed", WORKLOADS)
def test_against_cyclic_jacobi(oracle_mod, kind, seed):
    A_soa, cat = gen.make(kind, 6000, seed + 100)
    A = _aos(A_soa)
    lam, V = oracle_mod.solve(A)
    lj, Vj, sweeps = oracle_mod.jacobi_cyclic(A)
    assert sweeps.max() < 100
    # the brute force is itself accurate
    assert checks.residual(A, lj, Vj).max() <= TOL
    assert checks.eig_error(A, lam, lj).max() <= TOL


def test_branches_all_reached_by_stress_mix(oracle_mod):
    A_soa, cat = gen.stress_mix(20000, seed=1)
    _, _, info = oracle_mod.solve(_aos(A_soa), return_info=True)
    counts = np.bincount(info[:, 0], minlength=5)
    assert counts[oracle_mod.BR_DIAGONAL] > 0
    assert counts[oracle_mod.BR_DEFLATED] > 0
    assert counts[oracle_mod.BR_REDUCED] > 0
    # near-threshold arrows take both branches
    arrow = cat.numpy() == gen.CAT_ARROW
    b = np.bincount(info[arrow, 0], minlength=5)
    assert b[oracle_mod.BR_DEFLATED] > 0 and b[oracle_mod.BR_REDUCED] > 0


@pytest.mark.parametrize("flags", ["SIMPLIFIED_DEFLATION", "NO_H_GUARD",
                                   "NEWTON"])
def test_flag_variants_meet_bounds(oracle_mod, flags):
    """The simplified deflation test (Sec. 1.1), the literal h == 0 exit and
    the Newton zero finder (Sec. 1.4.2) give results within the same bounds
    on generic input."""
    f = getattr(oracle_mod, flags)
    for kind, seed in (("normal", 40), ("spd_fe", 41), ("uniform", 42)):
        A = _aos(gen.make(kind, 5000, seed)[0])
        lam0, _ = oracle_mod.solve(A)
        lam, V = oracle_mod.solve(A, flags=f)
        assert checks.residual(A, lam, V).max() <= TOL
        assert checks.orthogonality(V).max() <= TOL
        assert checks.eig_error(A, lam, lam0).max() <= TOL


def test_newton_flag_on_stress_mix(oracle_mod):
    A = _aos(gen.stress_mix(20000, seed=43)[0])
    lam, V = oracle_mod.solve(A, flags=oracle_mod.NEWTON)
    assert checks.residual(A, lam, V).max() <= TOL
    assert checks.orthogonality(V).max() <= TOL


def test_threads_do_not_change_results(oracle_mod):
    A = _aos(gen.stress_mix(5000, seed=44)[0])
    l1, V1 = oracle_mod.solve(A, nthreads=1)
    l8, V8 = oracle_mod.solve(A, nthreads=7)
    assert np.array_equal(l1, l8) and np.array_equal(V1, V8)
