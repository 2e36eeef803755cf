"""Pins of the oracle's GMRES polynomials (Sec. 2.3, Sec. 3.1) and composite
polynomial (Sec. 2.4, Sec. 3.2): the roots are harmonic Ritz values, so the
Newton form reproduces the GMRES iterate; a full Krylov space gives the
exact inverse; the scalar and matrix forms agree with independent routes.
No GPU."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense, krylov
from oracle.deflation import composite_eval, poly_eval, residual_poly_eval


def _lat(dims, kappa=0.15, eps=0.5, seed=7):
    return oracle.Lattice(dims, kappa, synth.gauge_links(dims, eps, seed))


def test_scalar_newton_form():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(9) + 1j * rng.standard_normal(9) + 2.0
    t = 1.0 / krylov.leja_order(theta)
    # p(theta_j) = 1/theta_j because pi(theta_j) = 0
    assert np.allclose(poly_eval(t, 1.0 / t), t, rtol=1e-13)
    lam = rng.standard_normal(20) + 1j * rng.standard_normal(20)
    # pi(lambda) = 1 - lambda p(lambda)
    assert np.allclose(1.0 - lam * poly_eval(t, lam), residual_poly_eval(t, lam), rtol=1e-12, atol=1e-12)


def test_leja_order_properties():
    rng = np.random.default_rng(2)
    th = rng.standard_normal(15) + 1j * rng.standard_normal(15)
    th = np.append(th, th[3])                           # an exact duplicate
    L = krylov.leja_order(th)
    assert sorted(L.tolist(), key=lambda z: (z.real, z.imag)) == sorted(th.tolist(), key=lambda z: (z.real, z.imag))
    assert abs(L[0]) == np.max(np.abs(th))
    for k in range(1, len(L) - 1):
        score = lambda z: np.sum(np.log(np.abs(z - L[:k])))
        with np.errstate(divide="ignore"):
            assert score(L[k]) >= max(score(z) for z in L[k:]) - 1e-12
    assert L[-1] == th[3]


@pytest.mark.parametrize("dims,deg", [((2, 2, 2, 2), 10), ((4, 4, 4, 4), 20)])
def test_harmonic_ritz_roots_reproduce_gmres(dims, deg):
    lat = _lat(dims)
    r0 = synth.gaussian_start(lat.n, 3)
    ps = krylov.gmres_polys(lat.apply, r0, [deg])
    m = deg + 1
    y, res = krylov.gmres_ls(ps.arn.Hbar, ps.arn.beta, m)
    x_gmres = ps.arn.Vb[:m].T @ y
    x_newton, _ = lat.poly_apply(ps.inv_roots[deg], r0)
    assert np.linalg.norm(x_newton - x_gmres) <= 1e-12 * np.linalg.norm(x_gmres)
    rn = np.linalg.norm(r0 - lat.apply(x_newton))
    assert abs(rn - res) <= 1e-10 * max(res, 1e-300) + 1e-14
    # the residual polynomial applied to r0 is the GMRES residual
    rp = lat.residual_poly_apply(ps.inv_roots[deg], r0)
    assert np.linalg.norm(rp - (r0 - lat.apply(x_newton))) <= 1e-12 * np.linalg.norm(r0)


def test_full_krylov_space_gives_inverse():
    dims = (1, 1, 1, 1)                                  # n = 12
    lat = _lat(dims, kappa=0.2)
    r0 = synth.gaussian_start(lat.n, 4)
    arn = krylov.arnoldi(lat.apply, r0, 12)
    th = krylov.leja_order(krylov.harmonic_ritz(arn.Hbar, arn.m))
    A = dense.dense_matrix(lat)
    X, _ = lat.poly_apply(1.0 / th, np.eye(12))
    assert np.linalg.norm(X.T - np.linalg.inv(A)) <= 1e-10 * np.linalg.norm(np.linalg.inv(A))


def test_newton_vs_dense_residual_route():
    # p(A) v = A^{-1} (v - pi(A) v), independent of the Newton recurrence
    lat = _lat((2, 2, 2, 2))
    rng = np.random.default_rng(5)
    th = 1.0 + 0.5 * (rng.standard_normal(8) + 1j * rng.standard_normal(8))
    t = 1.0 / krylov.leja_order(th)
    v = synth.random_fields(2, lat.V, 6).reshape(2, -1)
    A = dense.dense_matrix(lat)
    P = np.eye(lat.n, dtype=complex)
    for tj in t:
        P = P @ (np.eye(lat.n) - tj * A)
    ref = np.linalg.solve(A, (v - (P @ v.T).T).T).T
    y, bhy = lat.poly_apply(t, v)
    assert np.linalg.norm(y - ref) <= 1e-11 * np.linalg.norm(ref)
    assert np.allclose(bhy, np.einsum("ri,ri->r", v.conj(), y), rtol=1e-14)


def test_free_field_polynomial_trace():
    dims, kappa = (2, 2, 2, 4), 0.12
    lat = oracle.Lattice(dims, kappa, synth.unit_links(dims))
    r0 = synth.gaussian_start(lat.n, 8)
    ps = krylov.gmres_polys(lat.apply, r0, [6])
    t = ps.inv_roots[6]
    P, _ = lat.poly_apply(t, np.eye(lat.n))
    tr = np.trace(P)
    ff = dense.free_field_trace_fn(dims, kappa, lambda z: poly_eval(t, z))
    assert abs(tr - ff) <= 1e-12 * abs(ff)


def test_composite_scalar_identity():
    rng = np.random.default_rng(9)
    t_in = 1.0 / krylov.leja_order(1 + rng.standard_normal(5) + 1j * rng.standard_normal(5))
    t_out = 1.0 / krylov.leja_order(1 + rng.standard_normal(4) + 1j * rng.standard_normal(4))
    lam = 0.5 * (rng.standard_normal(30) + 1j * rng.standard_normal(30))
    p1 = composite_eval(t_in, t_out, lam)
    # 1 - a p_1(a) = pi_out(a p_in(a))
    rhs = residual_poly_eval(t_out, lam * poly_eval(t_in, lam))
    assert np.allclose(1 - lam * p1, rhs, rtol=1e-12, atol=1e-12)
    # degree of p_1: the residual polynomial has n_in*n_out roots -> p_1 has degree n_in*n_out - 1
    roots = np.roots(np.polyfit(lam[:21], 1 - lam[:21] * p1[:21], 20))
    assert len(roots) == 20 == len(t_in) * len(t_out)


def test_composite_reproduces_pp_gmres():
    # PP-GMRES on B = A p_in(A): x = p_in(A) p_out(B) r0 has residual pi_out(B) r0,
    # whose norm is the PP-GMRES least-squares residual (Sec. 3.2)
    lat = _lat((2, 2, 2, 2), kappa=0.16)
    r0 = synth.gaussian_start(lat.n, 10)
    ps = krylov.gmres_polys(lat.apply, r0, [4])
    t_in = ps.inv_roots[4]
    opB = krylov.pp_operator(lat.apply, t_in, lambda t, v: lat.poly_apply(t, v)[0])
    t_out, arn = krylov.pp_gmres_roots(opB, r0, n_out=6)
    y, res = krylov.gmres_ls(arn.Hbar, arn.beta, 6)
    x, _ = lat.composite_apply(t_in, t_out, r0)
    assert np.linalg.norm(r0 - lat.apply(x)) == pytest.approx(res, rel=1e-9)
    # and x equals p_in(A) applied to the PP-GMRES iterate
    z = arn.Vb[:6].T @ y
    x2, _ = lat.poly_apply(t_in, z)
    assert np.linalg.norm(x - x2) <= 1e-11 * np.linalg.norm(x)
    # composite application equals the dense-evaluated composite polynomial
    A = dense.dense_matrix(lat)
    ev, R = np.linalg.eig(A)
    xd = R @ (composite_eval(t_in, t_out, ev) * np.linalg.solve(R, r0))
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(x)




@pytest.mark.parametrize("rtol", [1e-3, 1e-6])
def test_pp_gmres_rtol_stops_at_first_crossing(rtol):
    """rtolpoly1 (Sec. 5 step 2c): the outer PP-GMRES stops at the first step
    whose residual r0 - B x_j, formed explicitly from the Krylov basis and B,
    is at most rtol ||ref||; the step before it is still above."""
    lat = _lat((2, 2, 2, 2), kappa=0.16)
    r0 = synth.gaussian_start(lat.n, 12)
    ps = krylov.gmres_polys(lat.apply, r0, [3])
    t_in = ps.inv_roots[3]
    opB = krylov.pp_operator(lat.apply, t_in, lambda t, v: lat.poly_apply(t, v)[0])
    ref = 2.0 * np.linalg.norm(r0)
    _, arn = krylov.pp_gmres_roots(opB, r0, rtol=rtol, rnorm_ref=ref)
    m = arn.m

    def explicit(j):
        y, _ = krylov.gmres_ls(arn.Hbar, arn.beta, j)
        return np.linalg.norm(r0 - opB(arn.Vb[:j].T @ y))

    assert explicit(m) <= rtol * ref * (1 + 1e-9)
    assert m == 1 or explicit(m - 1) > rtol * ref


def test_pp_arnoldi_rtolev_stops_at_first_crossing():
    """rtolev (Sec. 5 step 2b): PP-Arnoldi stops at the first step where the
    PP-GMRES solution of B y = r0 on its basis has relative residual <= rtolev."""
    lat = _lat((2, 2, 2, 2), kappa=0.16)
    r0 = synth.gaussian_start(lat.n, 13)
    ps = krylov.gmres_polys(lat.apply, r0, [3])
    opB = krylov.pp_operator(lat.apply, ps.inv_roots[3], lambda t, v: lat.poly_apply(t, v)[0])
    lam, Z, AZ, arn = krylov.pp_arnoldi_ritz(opB, lat.apply, r0, 200, 8, rtol=1e-8)
    m = arn.m

    def explicit(j):
        y, _ = krylov.gmres_ls(arn.Hbar, arn.beta, j)
        return np.linalg.norm(r0 - opB(arn.Vb[:j].T @ y)) / np.linalg.norm(r0)

    assert m < 200
    assert explicit(m) <= 1e-8 * (1 + 1e-6)
    assert explicit(m - 1) > 1e-8
