"""Pins of the host deflation diagnostics (Example 1 of Sec. 4.1).  The
paper's figures have no seed, so their values are not matched; these tests
check the quantities against identities that fix them.  No GPU."""
import numpy as np

from paper_2306_09559_amd import diagnostics as dg
from paper_2306_09559_amd.krylov import newton_value


def test_svd_deflation_closed_form_and_optimality():
    A = dg.shifted_random(80, 5.0, 3)
    s = np.linalg.svd(A, compute_uv=False)
    sv = dg.svd_deflation_norms(A, 10)
    ev = dg.eigen_deflation_norms(A, 10)
    # removing the k smallest singular components leaves 1 / sigma_{k+1} (smallest first)
    assert np.allclose(sv, 1.0 / s[::-1][:11], rtol=1e-10)
    # Eckart-Young: no rank-k correction (eigencomponents included) does better in the 2-norm
    assert np.all(sv <= ev * (1 + 1e-10))
    assert ev[0] == sv[0]


def test_eigen_triplets_and_full_deflation():
    A = dg.shifted_random(40, 4.0, 5)
    e = dg.eigen(A)
    assert np.allclose(e.W @ e.Z, np.eye(40), atol=1e-10)
    assert np.allclose(A @ e.Z, e.Z * e.lam, atol=1e-9)
    assert np.all(np.diff(np.abs(e.lam)) >= 0)
    full = dg.eigen_deflation_norms(A, 40, e)
    assert full[-1] < 1e-10 * full[0]


def test_gmres_polynomial_minimises_the_residual():
    """||b - A p_d(A) b|| equals the least-squares minimum over the Krylov
    space span{b, Ab, ..., A^d b} (a direct lstsq, no Arnoldi)."""
    A = dg.shifted_random(60, 6.0, 7)
    b = np.random.default_rng(8).standard_normal(60).astype(np.complex128)
    for d in (3, 8):
        t = dg.gmres_inverse_roots(A, d, b)
        assert len(t) == d + 1
        # p_d(A) b by the Newton form on vectors
        w, y = b.copy(), np.zeros_like(b)
        for tj in t:
            y = y + tj * w
            w = w - tj * (A @ w)
        K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(d + 1)], axis=1)
        c = np.linalg.lstsq(A @ K, b, rcond=None)[0]
        best = np.linalg.norm(b - A @ (K @ c))
        assert abs(np.linalg.norm(b - A @ y) - best) <= 1e-8 * np.linalg.norm(b)


def test_poly_difference_spectrum_and_norm():
    """p_hi(A) - p_lo(A) formed as a matrix by the Newton recurrence has the
    eigenvalues p_hi(lambda) - p_lo(lambda), and its 2-norm is the k = 0 entry."""
    A = dg.shifted_random(50, 6.0, 11)
    b = np.random.default_rng(12).standard_normal(50).astype(np.complex128)
    e = dg.eigen(A)
    c, order, norms = dg.poly_difference_deflation_norms(A, 12, 6, 5, b, e)

    def mat(t):
        W, Y = np.eye(50, dtype=np.complex128), np.zeros((50, 50), dtype=np.complex128)
        for tj in t:
            Y = Y + tj * W
            W = W - tj * (A @ W)
        return Y

    P = mat(dg.gmres_inverse_roots(A, 12, b)) - mat(dg.gmres_inverse_roots(A, 6, b))
    ev = np.linalg.eigvals(P)
    for x in c:
        assert np.min(np.abs(ev - x)) < 1e-8 * np.max(np.abs(c))
    assert abs(norms[0] - np.linalg.norm(P, 2)) < 1e-8 * norms[0]
    assert np.all(np.abs(c[order[:-1]]) >= np.abs(c[order[1:]]))
    assert np.allclose(c, newton_value(dg.gmres_inverse_roots(A, 12, b), e.lam)
                       - newton_value(dg.gmres_inverse_roots(A, 6, b), e.lam))
