"""Pins of the oracle's Z4 noise generator (Sec. 1: entries 1, -1, i, -i) and
of the Hutchinson estimator statistics.  No GPU."""
import os

import numpy as np

import oracle
from oracle import estimator

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_reference_outputs():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 9
    for state, k, out in rows:
        assert oracle.splitmix64(int(state), int(k)) == int(out)


def test_z4_values_and_reproducibility():
    z = oracle.z4(5, 1, 2, 0, 3, 64)
    vals = {1 + 0j, -1 + 0j, 1j, -1j}
    assert set(np.unique(z).tolist()) <= vals
    assert np.array_equal(z, oracle.z4(5, 1, 2, 0, 3, 64))
    # sample r of a batch equals the same sample drawn alone
    assert np.array_equal(z[2], oracle.z4(5, 1, 2, 2, 1, 64)[0])
    # different streams differ
    assert not np.array_equal(z[0], oracle.z4(5, 1, 3, 0, 1, 64)[0])
    assert not np.array_equal(z[0], z[1])


def test_z4_uniform_and_moments():
    n_s, V = 64, 32
    z = oracle.z4(11, 0, 0, 0, n_s, V)
    counts = np.array([np.sum(z == v) for v in (1, 1j, -1, -1j)])
    N = z.size
    chi2 = np.sum((counts - N / 4) ** 2 / (N / 4))
    assert chi2 < 16.3          # 3 d.o.f., p ~ 0.001
    # E[b b^H] = I, E[b b^T] = 0 (Sec. 1 with the conjugate transpose)
    bbH = z.T @ z.conj() / n_s
    bbT = z.T @ z / n_s
    off = bbH - np.diag(np.diag(bbH))
    assert np.allclose(np.diag(bbH), 1.0)
    assert np.abs(off).mean() < 3.0 / np.sqrt(n_s)
    assert np.abs(bbT).mean() < 3.0 / np.sqrt(n_s)


def test_hutchinson_mean_and_variance_closed_form():
    rng = np.random.default_rng(0)
    n = 48
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ns = 4000
    B = oracle.z4(21, 0, 0, 0, ns, n // 12)
    s = np.einsum("ri,ij,rj->r", B.conj(), M, B)
    var_pred = estimator.z4_variance(M)
    est = estimator.level_estimate(s)
    assert abs(est.mean - np.trace(M)) < 4.5 * np.sqrt(var_pred / ns)
    # sample variance of ns samples: relative sd about sqrt(2/ns) ~ 2%
    assert abs(est.var / var_pred - 1.0) < 0.1
    # b^T M b (no conjugate) has expectation 0, not Tr M
    s_t = np.einsum("ri,ij,rj->r", B, M, B)
    assert abs(s_t.mean()) < 4.5 * np.sqrt(np.sum(np.abs(M) ** 2) / ns) * 2
