"""Host-side logic of the product's GPU set-up (small dense algebra only)
checked against the oracle's independent implementation.  No GPU: the module
is imported without touching the device."""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle  # noqa: F401
from oracle import deflation, krylov as okr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pk():
    # load krylov.py's host helpers; its binding import needs the built library
    pytest.importorskip("torch")
    if not os.path.exists(os.path.join(ROOT, "paper_2306_09559_amd", "libmpmc.so")):
        pytest.skip("libmpmc.so not built")
    from paper_2306_09559_amd import krylov
    return krylov


def _hess(n, seed):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((n + 1, n)) + 1j * rng.standard_normal((n + 1, n)), -1)
    H += 3 * np.eye(n + 1, n)
    return H


@pytest.mark.parametrize("m", [1, 5, 17])
def test_harmonic_ritz_matches_oracle(pk, m):
    H = _hess(20, m)
    a = np.sort_complex(pk.harmonic_ritz_values(H, m))
    b = np.sort_complex(okr.harmonic_ritz(H, m))
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_leja_matches_oracle(pk):
    rng = np.random.default_rng(4)
    th = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    th = np.append(th, [th[5], th[5]])
    assert np.array_equal(pk.leja(th), okr.leja_order(th))


def test_newton_value_matches_oracle(pk):
    rng = np.random.default_rng(5)
    t = 1.0 / (2 + rng.standard_normal(12) + 1j * rng.standard_normal(12))
    lam = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    assert np.allclose(pk.newton_value(t, lam), deflation.poly_eval(t, lam), rtol=1e-13)


@pytest.mark.parametrize("m", [3, 11])
def test_gmres_residual_matches_oracle(pk, m):
    H = _hess(15, m + 7)
    _, res = okr.gmres_ls(H, 2.5, m)
    assert pk.gmres_residual(H, 2.5, m) == pytest.approx(res, rel=1e-10)
