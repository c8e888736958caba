"""Plant plausible mistakes in a copy of the oracle and check that its pins
catch every one (a dropped term, a wrong sign or index, a transposed operand,
a wrong constant).  Each mutant is compiled from a patched copy of the source
in a temporary directory and checked in a child process.  No GPU."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "syev3_oracle.c")

MUTANTS = {
    "f drops the b2 term":
        ("return x - gb - b1 * b1 / x - b2 * b2 / (x + ab);",
         "return x - gb - b1 * b1 / x;"),
    "f' squares the wrong factor":
        ("return 1.0 + b1 * b1 / (x * x) + b2 * b2 / (p * p);",
         "return 1.0 + b1 * b1 / (x * x) + b2 * b2 / p;"),
    "u3 third component sign":
        ("U[2][2] = -nu * (nu + ab);", "U[2][2] = nu * (nu + ab);"),
    "u2 uses beta2 for beta1":
        ("U[1][1] = be1 * nu * (mu + ab);", "U[1][1] = be2 * nu * (mu + ab);"),
    "trace identity sign":
        ("l[1] = nu - mu + ga;", "l[1] = nu + mu + ga;"),
    "back-transform with J transposed":
        ("W[c][0] = J[0] * U[c][0] + J[1] * U[c][1];",
         "W[c][0] = J[0] * U[c][0] + J[2] * U[c][1];"),
    "beta = J a instead of J^T a":
        ("arrow[2] = J[0] * a[2] + J[2] * a[4];",
         "arrow[2] = J[0] * a[2] + J[1] * a[4];"),
    "deflated eigenvector (s, -c)":
        ("U[0][0] = cg; U[0][1] = -sg; U[0][2] = 0.0;",
         "U[0][0] = sg; U[0][1] = -cg; U[0][2] = 0.0;"),
    "d1 and d2 exchanged":
        ("d1 = (al1 * be2 * be2 + al2 * be1 * be1) / (h * h);",
         "d1 = (al1 * be1 * be1 + al2 * be2 * be2) / (h * h);"),
    "BG start: conjugate form sign":
        ("x = H / (-g2 + sqrt(g2 * g2 + H));",
         "x = H / (g2 + sqrt(g2 * g2 + H));"),
    "omega0 drops abar":
        ("double w0 = 1.0 + b2 * b2 * ab / (p * p * p);",
         "double w0 = 1.0 + b2 * b2 / (p * p * p);"),
    "increment halved":
        ("double F = 2.0 * f / b;", "double F = f / b;"),
    "descending sort":
        ("while (j >= 0 && l[ord[j]] > l[key])",
         "while (j >= 0 && l[ord[j]] < l[key])"),
    "eigenvalues not unscaled":
        ("for (int i = 0; i < 3; ++i) l[i] = ldexp(l[i], k);",
         "for (int i = 0; i < 3; ++i) l[i] = l[i];"),
    "Jacobi rotation sign":
        ("double sg = (tau >= 0.0) ? 1.0 : -1.0;",
         "double sg = (tau >= 0.0) ? -1.0 : 1.0;"),
    "deflation test inverted":
        ("deflate = (lhs <= rhs);", "deflate = (lhs >= rhs);"),
    "h guard far too loose":
        ("diagonal = (h <= EPS * (fabs(al1) + fabs(al2) + fabs(ga)));",
         "diagonal = (h <= 1e-8 * (fabs(al1) + fabs(al2) + fabs(ga)));"),
    "nu problem without the beta swap":
        ("nu = oracle_bg_root(be2, be1, ab, al2 - ga, &it_nu, NULL, 0);",
         "nu = oracle_bg_root(be1, be2, ab, al2 - ga, &it_nu, NULL, 0);"),
    "normalisation skipped":
        ("u[0] = v0 / nrm; u[1] = v1 / nrm; u[2] = v2 / nrm;",
         "u[0] = v0; u[1] = v1; u[2] = v2;"),
    "Newton step sign":
        ("double xn = x - f / fp;", "double xn = x + f / fp;"),
    "simplified deflation bound uses alpha1 - alpha2":
        ("rhs = C_DEFL * EPS * fabs(al1 + al2) * h * h;",
         "rhs = C_DEFL * EPS * fabs(al1 - al2) * h * h;"),
    "h guard applied only when it is switched off":
        ("if (!diagonal && !(flags & ORACLE_NO_H_GUARD))",
         "if (!diagonal && (flags & ORACLE_NO_H_GUARD))"),
    "Newton starts from the two-pole model (right of the root)":
        ("    x = g2 + sqrt(g2 * g2 + b1 * b1);\n  else\n    x = b1 * b1 / (-g2 + sqrt(g2 * g2 + b1 * b1));",
         "    x = g2 + sqrt(g2 * g2 + b1 * b1 + b2 * b2);\n  else\n    x = (b1 * b1 + b2 * b2) / (-g2 + sqrt(g2 * g2 + b1 * b1 + b2 * b2));"),
    "vectors not permuted with the sorted eigenvalues":
        ("V[3 * r + c] = W[ord[c]][r];", "V[3 * r + c] = W[c][r];"),
    "d2 drops a term":
        ("d2 = (al1 * be1 * be1 + al2 * be2 * be2) / (h * h);",
         "d2 = (al1 * be1 * be1) / (h * h);"),
    "back-transform row 2 uses the wrong rotation entry":
        ("W[c][1] = J[2] * U[c][0] + J[3] * U[c][1];",
         "W[c][1] = J[1] * U[c][0] + J[3] * U[c][1];"),
}


def _build_and_check(tmp, name, patch):
    src = open(SRC).read()
    if patch is not None:
        old, new = patch
        assert src.count(old) == 1, f"mutation site not unique: {name}"
        src = src.replace(old, new)
    d = tempfile.mkdtemp(dir=tmp)
    c = os.path.join(d, "syev3_oracle.c")
    with open(c, "w") as fh:
        fh.write(src)
    so = os.path.join(d, "liboracle_mut.so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", so, c,
                           os.path.join(ROOT, "oracle", "jacobi_cyclic.c"),
                           "-lm"])
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([ROOT, HERE]))
    p = subprocess.run([sys.executable, os.path.join(HERE, "oracle_mutant_check.py"), so],
                       env=env, capture_output=True, text=True, timeout=600)
    return p.returncode, p.stdout + p.stderr


def test_unmutated_oracle_passes_the_compact_pins(tmp_path):
    rc, out = _build_and_check(str(tmp_path), "none", None)
    assert rc == 0, out


def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(_build_and_check, str(tmp_path), name, patch)
                for name, patch in MUTANTS.items()}
        results = {name: f.result() for name, f in futs.items()}
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"mutants not caught by the pins: {survivors}"
