"""Planted mistakes in the oracle (on the CPU, in a copy of its C source):
each one must make a pin fail.  The pins are what the oracle is trusted on,
so a plausible mistake anywhere in its arithmetic -- a dropped term, a wrong
sign, index or constant -- has to be caught by one of them.

Each case copies oracle/ref.c, applies one textual change, compiles it the
way oracle.build does, and runs the named pin file in a child process whose
oracle module loads the mutated library.  An unchanged copy run the same way
passes the same files (the control)."""
import os
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

# the child process: point the oracle at the given source and library, then run pytest
RUNNER = ("import sys, oracle; oracle._SRC, oracle._LIB = sys.argv[1], sys.argv[2]; "
          "import pytest; sys.exit(pytest.main(sys.argv[3:]))")


def _build(tmp_path, text):
    src = tmp_path / "ref.c"
    src.write_text(text)
    lib = tmp_path / "liboracle.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-fPIC",
                           "-shared", "-o", str(lib), str(src), "-lm"])
    return src, lib


def _run_pins(src, lib, files):
    r = subprocess.run([sys.executable, "-c", RUNNER, str(src), str(lib), "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *files], cwd=ROOT, capture_output=True, text=True, timeout=600)
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
