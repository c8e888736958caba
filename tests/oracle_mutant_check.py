"""Run a compact set of the oracle's pins against an oracle library given on
the command line; exit 0 if every pin holds, 1 otherwise.  Used by
test_oracle_mutants.py (in a child process, since a planted mistake may also
crash the library)."""
import ctypes
import sys

import numpy as np

import checks
from paper_1806_06698_amd import gen

EPS = 2.0 ** -52


def main(path):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_solve_batch.argtypes = [ctypes.c_int64, dp, dp, dp,
                                       ctypes.c_uint, ip, ctypes.c_int]
    for nm in ("oracle_bg_root", "oracle_newton_root"):
        getattr(lib, nm).argtypes = [ctypes.c_double] * 4 + [ip, dp, ctypes.c_int]
        getattr(lib, nm).restype = ctypes.c_double

    def solve(A, flags=0):
        A = np.ascontiguousarray(A, dtype=np.float64)
        lam = np.empty((A.shape[0], 3))
        V = np.empty((A.shape[0], 3, 3))
        lib.oracle_solve_batch(A.shape[0], A.ctypes.data_as(dp),
                               lam.ctypes.data_as(dp), V.ctypes.data_as(dp),
                               flags, ip(), 1)
        return lam, V

    def branches(A, flags):
        A = np.ascontiguousarray(A, dtype=np.float64)
        lam = np.empty((A.shape[0], 3))
        V = np.empty((A.shape[0], 3, 3))
        info = np.empty((A.shape[0], 4), dtype=np.int32)
        lib.oracle_solve_batch(A.shape[0], A.ctypes.data_as(dp),
                               lam.ctypes.data_as(dp), V.ctypes.data_as(dp),
                               flags, info.ctypes.data_as(ip), 1)
        return info[:, 0].tolist()

    fails = []
    # the deflation tests and the h guard decide as their inequalities state
    from deflation_cases import DEFLATION_BRANCHES, DEFLATION_CASES
    for flags, want in DEFLATION_BRANCHES.items():
        if branches(DEFLATION_CASES, flags) != want:
            fails.append(f"deflation-branches/flags={flags}")
    for kind, seed, n in (("stress_mix", 1, 3000), ("normal", 0, 2000),
                          ("wide_range", 4, 1000), ("spd_fe", 2, 1000)):
        A = gen.to_aos(gen.make(kind, n, seed)[0]).numpy()
        for flags in (0, 4):
            lam, V = solve(A, flags)
            ok = np.all(np.isfinite(lam)) and np.all(np.diff(lam, axis=1) >= 0)
            ok = ok and checks.residual(A, lam, V).max() <= 16
            ok = ok and checks.orthogonality(V).max() <= 16
            ok = ok and checks.eig_error(A, lam, checks.lapack_eigvals(A)).max() <= 16
            if not ok:
                fails.append(f"{kind}/flags={flags}")
    # exact cases
    rng = np.random.default_rng(3)
    D = np.zeros((500, 6))
    D[:, [0, 3, 5]] = rng.standard_normal((500, 3))
    lam, V = solve(D)
    if not np.array_equal(lam, np.sort(D[:, [0, 3, 5]], axis=1)):
        fails.append("diagonal")
    B = rng.standard_normal((500, 6))
    B[:, 1] = 0.0
    B[:, 2] = 0.0
    lam, V = solve(B)
    if not np.all((lam == B[:, [0]]).any(axis=1)):
        fails.append("beta-deflation")
    # zero finders against LAPACK on fully reduced arrows
    for i in range(300):
        b1, b2 = rng.standard_normal(2)
        ab = abs(rng.standard_normal()) + 0.01
        gb = rng.standard_normal()
        M = np.array([[0, 0, b1], [0, -ab, b2], [b1, b2, gb]])
        top = np.linalg.eigvalsh(M)[-1]
        for nm in ("oracle_bg_root", "oracle_newton_root"):
            x = getattr(lib, nm)(b1, b2, ab, gb, ip(), dp(), 0)
            if not abs(x - top) <= 8 * EPS * np.linalg.norm(M):
                fails.append(nm)
                break
        else:
            continue
        break
    # BG start (zero of the model from +infinity) and cubic order
    try:
        import mpmath
        mpmath.mp.dps = 40
    except ImportError:
        mpmath = None
    orders = []
    tr = np.zeros(64)
    it = np.zeros(1, dtype=np.int32)
    for i in range(200):
        b1, b2 = rng.standard_normal(2)
        ab = abs(rng.standard_normal()) + 0.01
        gb = rng.standard_normal()
        x = lib.oracle_bg_root(b1, b2, ab, gb, it.ctypes.data_as(ip),
                               tr.ctypes.data_as(dp), 64)
        x0, H = tr[0], b1 * b1 + b2 * b2
        if not abs(x0 * x0 - gb * x0 - H) <= 8 * EPS * (x0 * x0 + abs(gb) * x0 + H):
            fails.append("bg-start")
            break
        if mpmath is None or it[0] < 3:
            continue
        M = mpmath.matrix([[0, 0, b1], [0, -ab, b2], [b1, b2, gb]])
        root = max(mpmath.eigsy(M, eigvals_only=True))
        e = [float(abs((mpmath.mpf(float(t)) - root) / root)) for t in tr[:it[0]]]
        for j in range(len(e) - 2):
            if e[j] < 0.5 and e[j + 2] > 1e3 * EPS:
                orders.append(np.log(e[j + 2] / e[j + 1]) / np.log(e[j + 1] / e[j]))
    if mpmath is not None and (len(orders) < 5 or min(orders) < 2.5):
        fails.append("bg-cubic-order")
    if fails:
        print("pins failed:", ", ".join(sorted(set(fails))))
        return 1
    print("all pins hold")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
