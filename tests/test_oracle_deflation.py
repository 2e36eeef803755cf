"""Pins of the oracle's deflation (Sec. 2.1 Left-right Projection, Sec. 4 left
vectors from gamma_5, Sec. 4.1 Monte Carlo deflation, Sec. 4.3 deflated
polynomial) and of the multilevel telescoping (eq. multpolytr).  No GPU."""
import numpy as np
import pytest

import oracle
import synth
from oracle import deflation, dense, estimator, krylov


@pytest.fixture(scope="module")
def small():
    dims = (2, 2, 2, 2)
    lat = oracle.Lattice(dims, 0.16, synth.gauge_links(dims, 0.5, 21))
    A = dense.dense_matrix(lat)
    lam, Z, pair = deflation.dense_triplets(A, 6, lat.gamma5)
    U = deflation.left_vectors(Z, pair, lat.gamma5)
    return lat, A, lam, Z, pair, U


def test_gamma5_rule_gives_lapack_left_vectors(small):
    lat, A, lam, Z, pair, U = small
    # left eigenvectors: eigenvectors of A^H with eigenvalue conj(lambda)
    mu, L = np.linalg.eig(A.conj().T)
    for i in range(len(lam)):
        j = np.argmin(np.abs(mu - np.conj(lam[i])))
        l = L[:, j] / np.linalg.norm(L[:, j])
        u = U[i] / np.linalg.norm(U[i])
        assert abs(abs(np.vdot(l, u)) - 1.0) < 1e-10
        assert np.linalg.norm(A.conj().T @ U[i] - np.conj(lam[i]) * U[i]) < 1e-10 * np.linalg.norm(U[i])
    assert np.allclose(np.einsum("ij,ij->i", U.conj(), Z), 1.0)


def test_projection_matrix_diagonal(small):
    lat, A, lam, Z, pair, U = small
    H = deflation.projection_matrix(lat.apply, Z, U)
    assert np.allclose(H, np.diag(lam), atol=1e-10)


def test_left_right_projection_removes_components(small):
    lat, A, lam, Z, pair, U = small
    H = deflation.projection_matrix(lat.apply, Z, U)
    r0 = synth.gaussian_start(lat.n, 30)
    xh, r = deflation.left_right_projection(lat.apply, Z, U, H, r0)
    assert np.linalg.norm(U.conj() @ r) < 1e-12 * np.linalg.norm(r0)
    assert np.linalg.norm(r - (r0 - A @ xh)) < 1e-13


def test_deflated_poly_operator_eigen(small):
    lat, A, lam, Z, pair, U = small
    H = deflation.projection_matrix(lat.apply, Z, U)
    ps = krylov.gmres_polys(lat.apply, synth.gaussian_start(lat.n, 31), [6])
    Q = deflation.DeflatedPoly(lat.apply, Z, U, H, lambda v: lat.poly_apply(ps.inv_roots[6], v)[0])
    for i in range(len(lam)):
        assert np.linalg.norm(Q.apply(Z[i]) - Z[i] / lam[i]) < 1e-10


def test_deflation_unbiased_identity(small):
    lat, A, lam, Z, pair, U = small
    rng = np.random.default_rng(3)
    M = rng.standard_normal(A.shape) + 1j * rng.standard_normal(A.shape)
    c = rng.standard_normal(len(lam)) + 1j * rng.standard_normal(len(lam))
    D = np.einsum("i,ia,ib->ab", c, Z, U.conj())
    # Tr(M - D) + sum c_i u_i^* z_i = Tr M for any c
    uz = np.einsum("ij,ij->i", U.conj(), Z)
    assert abs(np.trace(M - D) + np.sum(c * uz) - np.trace(M)) < 1e-10
    # sample form: b^* D b = sum c_i conj(zeta_i) omega_i
    b = oracle.z4(1, 0, 0, 0, 3, lat.V)
    zeta, omega = deflation.projection_coefficients(Z, U, b)
    s = estimator.level_samples(np.einsum("ri,ij,rj->r", b.conj(), M, b), None, zeta, omega, c)
    direct = np.einsum("ri,ij,rj->r", b.conj(), M - D, b)
    assert np.allclose(s, direct, rtol=1e-12)


def test_deflation_reduces_level_variance(small):
    # Sec. 4.1: polynomials differ mostly at the small eigenvalues, so
    # deflating them lowers the Z4 variance of the difference level
    lat, A, lam, Z, pair, U = small
    ps = krylov.gmres_polys(lat.apply, synth.gaussian_start(lat.n, 32), [12, 3])
    P12, _ = lat.poly_apply(ps.inv_roots[12], np.eye(lat.n))
    P3, _ = lat.poly_apply(ps.inv_roots[3], np.eye(lat.n))
    M = (P12 - P3).T
    c = deflation.deflation_coefficients(lam, lambda l: deflation.poly_eval(ps.inv_roots[12], l),
                                         lambda l: deflation.poly_eval(ps.inv_roots[3], l))
    D = np.einsum("i,ia,ib->ab", c, Z, U.conj())
    assert estimator.z4_variance(M - D) < estimator.z4_variance(M)


def test_telescoping_levels_sum_to_trace_inverse(small):
    lat, A, lam, Z, pair, U = small
    ps = krylov.gmres_polys(lat.apply, synth.gaussian_start(lat.n, 33), [15, 6, 2])
    P = {d: lat.poly_apply(ps.inv_roots[d], np.eye(lat.n))[0].T for d in (15, 6, 2)}
    Ainv = np.linalg.inv(A)
    levels = [np.trace(Ainv - P[15]), np.trace(P[15] - P[6]), np.trace(P[6] - P[2]), np.trace(P[2])]
    assert abs(sum(levels) - np.trace(Ainv)) < 1e-11 * abs(np.trace(Ainv))


@pytest.mark.slow
def test_mc_levels_within_4_sigma_of_exact():
    """Sampled multilevel estimate vs exact dense level traces (C1 shape)."""
    from synth.configs import C1
    lat = oracle.Lattice(C1.dims, C1.kappa, synth.gauge_links(C1.dims, C1.eps, C1.seed_links))
    ps = krylov.gmres_polys(lat.apply, synth.gaussian_start(lat.n, C1.seed_start), [20, 5])
    ev = np.linalg.eigvals(dense.dense_matrix(lat))
    exact = {d: np.sum(deflation.poly_eval(ps.inv_roots[d], ev)) for d in (20, 5)}
    for lvl, (hi, lo) in enumerate([(20, 5), (5, None)]):
        b = oracle.z4(C1.seed_noise, C1.lattice_id, lvl, 0, 100, lat.V)
        _, h = lat.poly_apply(ps.inv_roots[hi], b)
        l = lat.poly_apply(ps.inv_roots[lo], b)[1] if lo else None
        est = estimator.level_estimate(estimator.level_samples(h, l))
        target = exact[hi] - (exact[lo] if lo else 0)
        assert abs(est.estimate - target) < 4 * est.stderr


def test_top_level_trace_identity(small):
    """Tr(A^{-1} - Q) summed from unit-vector samples b^H A^{-1} b - b^H Q b
    (dense solve, deflated composite Q) equals sum over the eigenvalues not
    deflated of 1/lambda - p_1(lambda) (LAPACK spectrum): Q is 1/lambda_i on
    the deflated z_i and p_1(lambda_j) on every other eigenvector."""
    from oracle import solve
    lat, A, lam, Z, pair, U = small
    H = deflation.projection_matrix(lat.apply, Z, U)
    rng = np.random.default_rng(5)
    inv_in = 0.4 + 0.3 * rng.standard_normal(4) + 0.1j * rng.standard_normal(4)
    inv_out = 0.5 + 0.2 * rng.standard_normal(3) + 0.1j * rng.standard_normal(3)
    Q = deflation.DeflatedPoly(lat.apply, Z, U, H, lambda v: lat.composite_apply(inv_in, inv_out, v)[0])
    E = np.eye(lat.n, dtype=np.complex128)
    X = solve.dense_solve(lat, E)
    QE = np.array([Q.apply(e) for e in E])
    s = solve.top_level_samples(E, X, QE)
    mu = np.linalg.eigvals(A)
    keep = np.ones(len(mu), dtype=bool)
    for l in lam:
        keep[np.argmin(np.abs(mu - l) + (~keep) * 1e9)] = False
    want = np.sum(1.0 / mu[keep] - deflation.composite_eval(inv_in, inv_out, mu[keep]))
    assert abs(np.sum(s) - want) < 1e-9 * np.sum(np.abs(1.0 / mu))
    assert np.max(solve.residual(lat, E[:5], X[:5])) < 1e-13
