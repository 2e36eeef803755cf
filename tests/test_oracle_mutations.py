"""Planted mistakes in the oracle (on the CPU, in a copy of it): each one
must make a pin fail.  The pins are what the oracle is trusted on, so a
plausible mistake anywhere in its arithmetic -- a dropped term, a wrong sign,
index, conjugate or constant -- has to be caught by one of them.

A C case copies oracle/ref.c, applies one textual change, compiles it the way
oracle.build does, and runs the named pin file in a child process whose oracle
module loads the mutated library.  A Python case copies the oracle package,
changes one of its modules and runs the pin file in a child process that
imports the copy.  Unchanged copies run the same way pass the same files (the
controls)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (label, original text, mutated text, pin file that must fail)
MUTATIONS = [
    ("backward hop reads the link of x, not of x - mu",
     "u = conj(U[((mu * V + nb) * 3 + b) * 3 + a]);", "u = conj(U[((mu * V + s) * 3 + b) * 3 + a]);",
     "tests/test_oracle_operator.py"),
    ("no antiperiodic sign across the time boundary",
     "if (mu == 3 && antiperiodic_t) *sign = -1.0;", "(void)0;",
     "tests/test_oracle_operator.py"),
    ("Newton recurrence with the wrong sign",
     "w[i] = w[i] - t * aw[i];", "w[i] = w[i] + t * aw[i];",
     "tests/test_oracle_poly.py"),
    ("double polynomial without its final p_in factor",
     "newton_poly(wilson_op, &w, n, n_in, inv_in, z, Y + r * n);", "memcpy(Y + r * n, z, sizeof(cplx) * n);",
     "tests/test_oracle_poly.py"),
    ("Z4 code 1 mapped to -i instead of i",
     "case 1: b = I; break;", "case 1: b = -I; break;",
     "tests/test_oracle_noise.py"),
    ("one entry of gamma_2 with the wrong sign",
     "{{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}}",
     "{{0, 0, 0, 1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}}",
     "tests/test_oracle_operator.py"),
    ("a SplitMix64 multiplier off by one bit",
     "0xBF58476D1CE4E5B9ULL", "0xBF58476D1CE4E5B8ULL",
     "tests/test_oracle_noise.py"),
    ("the hopping term added instead of subtracted (kappa sign)",
     "x[12 * s + 3 * sp + a] - kappa * acc[sp][a];", "x[12 * s + 3 * sp + a] + kappa * acc[sp][a];",
     "tests/test_oracle_operator.py"),
]

# (label, module, original text, mutated text, pin file that must fail)
PY_MUTATIONS = [
    ("sample variance over n instead of n - 1", "estimator.py",
     "np.sum(np.abs(s - mean) ** 2) / (n - 1)", "np.sum(np.abs(s - mean) ** 2) / n",
     "tests/test_oracle_estimator.py"),
    ("level 2 checked from 2 samples instead of 3", "estimator.py",
     "return list(range(3, nmax + 1, 3))", "return list(range(2, nmax + 1, 3))",
     "tests/test_oracle_estimator.py"),
    ("first level's share of eps over sqrt(2) instead of sqrt(3)", "estimator.py",
     "t1 = eps / np.sqrt(3.0)", "t1 = eps / np.sqrt(2.0)",
     "tests/test_oracle_estimator.py"),
    ("deflation term added to the sample", "estimator.py",
     's = s - np.einsum("i,ir,ir->r", np.asarray(c), np.conj(zeta), omega)',
     's = s + np.einsum("i,ir,ir->r", np.asarray(c), np.conj(zeta), omega)',
     "tests/test_oracle_deflation.py"),
    ("left vectors scaled by d instead of conj(d)", "deflation.py",
     "return U / np.conj(d)[:, None]", "return U / d[:, None]",
     "tests/test_oracle_deflation.py"),
    ("zeta = V^T b instead of V^H b", "deflation.py",
     "return Z.conj() @ B.T, U.conj() @ B.T", "return Z @ B.T, U.conj() @ B.T",
     "tests/test_oracle_deflation.py"),
    ("harmonic Ritz with H^-T e_m instead of H^-H e_m", "krylov.py",
     "f = np.linalg.solve(Hm.conj().T, em)", "f = np.linalg.solve(Hm.T, em)",
     "tests/test_oracle_poly.py"),
    ("harmonic Ritz with |h| instead of |h|^2", "krylov.py",
     "np.linalg.eigvals(Hm + (abs(h) ** 2) * np.outer(f, em))", "np.linalg.eigvals(Hm + abs(h) * np.outer(f, em))",
     "tests/test_oracle_poly.py"),
    ("Leja order by summed distances instead of their product", "krylov.py",
     "score[i] += np.log(abs(th[i] - last))", "score[i] += abs(th[i] - last)",
     "tests/test_oracle_poly.py"),
    ("selection's left residual without g5", "krylov.py",
     "        u = gamma5(Z[src])\n        u = u / np.linalg.norm(u)", "        u = Z[src]\n        u = u / np.linalg.norm(u)",
     "tests/test_oracle_selection.py"),
    ("colouring one step too short", "probing.py",
     "torus_distance(dims, s, t) <= d", "torus_distance(dims, s, t) < d",
     "tests/test_oracle_probing.py"),
    ("site distance without the periodic wrap", "probing.py",
     "out += min(da, L - da)", "out += da",
     "tests/test_oracle_probing.py"),
    ("top-level sample b^H x + b^H Q b", "solve.py",
     'np.einsum("ri,ri->r", B2.conj(), X2) - np.einsum("ri,ri->r", B2.conj(), Q2)',
     'np.einsum("ri,ri->r", B2.conj(), X2) + np.einsum("ri,ri->r", B2.conj(), Q2)',
     "tests/test_oracle_deflation.py::test_top_level_trace_identity"),
    ("solve residual b + A x", "solve.py",
     "R = B2 - lat.apply(X2)", "R = B2 + lat.apply(X2)",
     "tests/test_oracle_deflation.py::test_top_level_trace_identity"),
]

# the child processes: point the oracle at the given source and library, or
# import the oracle package from the given directory; then run pytest
RUNNER = ("import sys, oracle; oracle._SRC, oracle._LIB = sys.argv[1], sys.argv[2]; "
          "import pytest; sys.exit(pytest.main(sys.argv[3:]))")
PY_RUNNER = ("import sys; sys.path.insert(0, sys.argv[1]); import oracle; "
             "assert oracle.__file__.startswith(sys.argv[1]), oracle.__file__; "
             "import pytest; sys.exit(pytest.main(sys.argv[2:]))")
PIN_ARGS = ["-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]


def _build(tmp_path, text):
    src = tmp_path / "ref.c"
    src.write_text(text)
    lib = tmp_path / "liboracle.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-fPIC",
                           "-shared", "-o", str(lib), str(src), "-lm"])
    return src, lib


def _run_pins(src, lib, files):
    r = subprocess.run([sys.executable, "-c", RUNNER, str(src), str(lib), *PIN_ARGS, *files], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-3000:] + r.stderr[-2000:]


def _copy_package(tmp_path):
    shutil.copytree(os.path.join(ROOT, "oracle"), tmp_path / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.tmp*"))
    return tmp_path / "oracle"


def _run_pins_on_copy(tmp_path, files):
    r = subprocess.run([sys.executable, "-c", PY_RUNNER, str(tmp_path), *PIN_ARGS, *files], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-3000:] + r.stderr[-2000:]


def test_unchanged_copy_passes_the_pins(tmp_path):
    src, lib = _build(tmp_path, open(os.path.join(ROOT, "oracle", "ref.c")).read())
    files = sorted({m[3] for m in MUTATIONS})
    rc, out = _run_pins(src, lib, files)
    assert rc == 0, out


@pytest.mark.parametrize("label,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, label, old, new, pins):
    text = open(os.path.join(ROOT, "oracle", "ref.c")).read()
    assert old in text, label
    src, lib = _build(tmp_path, text.replace(old, new))
    rc, out = _run_pins(src, lib, [pins])
    # 1: the tests ran and at least one failed (anything else is a harness error)
    assert rc == 1, out


def test_unchanged_package_copy_passes_the_pins(tmp_path):
    _copy_package(tmp_path)
    rc, out = _run_pins_on_copy(tmp_path, sorted({m[4] for m in PY_MUTATIONS if "::" not in m[4]}) +
                                ["tests/test_oracle_deflation.py::test_top_level_trace_identity"])
    assert rc == 0, out


@pytest.mark.parametrize("label,module,old,new,pins", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_planted_mistake_in_a_module_fails_a_pin(tmp_path, label, module, old, new, pins):
    pkg = _copy_package(tmp_path)
    path = pkg / module
    text = path.read_text()
    assert text.count(old) == 1, label
    path.write_text(text.replace(old, new))
    rc, out = _run_pins_on_copy(tmp_path, [pins])
    assert rc == 1, out
