"""Pins of the oracle's Wilson-Dirac operator against facts fixed by the
mathematics: the Dirac algebra, the free-field closed-form spectrum,
gamma_5-hermiticity (Sec. 4: left vectors from gamma_5), gauge covariance and
dense LU traces.  No GPU."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense


def test_gamma_algebra():
    G = [oracle.gamma(m) for m in range(4)]
    I4 = np.eye(4)
    for a in range(4):
        assert np.allclose(G[a], G[a].conj().T)
        for b in range(4):
            anti = G[a] @ G[b] + G[b] @ G[a]
            assert np.allclose(anti, 2 * I4 * (a == b))
    # chiral basis: gamma_5 diagonal
    assert np.allclose(oracle.gamma5_matrix(), np.diag([1, 1, -1, -1]))
    assert np.allclose(G[0] @ G[1] @ G[2] @ G[3], np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims,antiperiodic", [((2, 2, 2, 4), True), ((2, 2, 2, 4), False),
                                               ((4, 2, 2, 2), True), ((1, 1, 1, 1), True)])
def test_free_field_spectrum(dims, antiperiodic):
    kappa = 0.15
    lat = oracle.Lattice(dims, kappa, synth.unit_links(dims), antiperiodic_t=antiperiodic)
    A = dense.dense_matrix(lat)
    ev = np.linalg.eigvals(A)
    ff = dense.free_field_eigenvalues(dims, kappa, antiperiodic)
    # match as multisets: sort by (real, imag) after rounding away noise
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    assert np.allclose(sorted(ev, key=key), sorted(ff, key=key), atol=1e-12)
    tr = np.trace(np.linalg.inv(A))
    assert abs(tr - dense.free_field_trace_inverse(dims, kappa, antiperiodic)) < 1e-12 * abs(tr)


def test_free_field_trace_value_2x2x2x4():
    # closed form sum_p 12a/(a^2+b^2) at kappa 0.15, antiperiodic t
    assert abs(dense.free_field_trace_inverse((2, 2, 2, 4), 0.15) - 340.5579036128) < 1e-9


def _random_lattice(dims, kappa=0.15, eps=0.5, seed=7):
    return oracle.Lattice(dims, kappa, synth.gauge_links(dims, eps, seed))


def test_links_su3():
    U = synth.gauge_links((2, 2, 2, 2), 0.5, 1).reshape(-1, 3, 3)
    I3 = np.eye(3)
    assert np.allclose(np.einsum("kab,kcb->kac", U, U.conj()), I3, atol=1e-14)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-13)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_gamma5_hermiticity(dims):
    lat = _random_lattice(dims)
    x = synth.random_fields(1, lat.V, 11).reshape(-1)
    y = synth.random_fields(1, lat.V, 12).reshape(-1)
    lhs = np.vdot(y, lat.apply(x))
    rhs = np.vdot(lat.gamma5(lat.apply(lat.gamma5(y))), x)
    assert abs(lhs - rhs) <= 1e-14 * np.linalg.norm(x) * np.linalg.norm(y) * 10


def test_spectrum_closed_under_conjugation():
    lat = _random_lattice((2, 2, 2, 2))
    ev = np.linalg.eigvals(dense.dense_matrix(lat))
    for z in ev:
        assert np.min(np.abs(ev - np.conj(z))) < 1e-10


def test_gauge_covariance():
    dims = (2, 2, 4, 2)
    lat = _random_lattice(dims, seed=3)
    G = synth.random_su3(lat.V, 99)
    # U'_mu(x) = G(x) U_mu(x) G(x+mu)^H ; site index s = x + Lx(y + Ly(z + Lz t))
    L = dims
    coords = np.array(np.unravel_index(np.arange(lat.V), (L[3], L[2], L[1], L[0]))[::-1]).T
    Up = np.empty_like(lat.U)
    for mu in range(4):
        c = coords.copy()
        c[:, mu] = (c[:, mu] + 1) % L[mu]
        nb = c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))
        Up[mu] = G @ lat.U[mu] @ np.conj(np.swapaxes(G[nb], 1, 2))
    latp = oracle.Lattice(dims, lat.kappa, Up)
    psi = synth.random_fields(1, lat.V, 5)[0]              # (V, 4, 3)
    gpsi = np.einsum("sab,spb->spa", G, psi)
    lhs = latp.apply(gpsi.reshape(-1)).reshape(lat.V, 4, 3)
    rhs = np.einsum("sab,spb->spa", G, lat.apply(psi.reshape(-1)).reshape(lat.V, 4, 3))
    assert np.linalg.norm(lhs - rhs) <= 1e-14 * np.linalg.norm(rhs) * 10


def test_dense_lu_trace_matches_eigenvalues():
    lat = _random_lattice((2, 2, 2, 2), kappa=0.12)
    A = dense.dense_matrix(lat)
    tr_lu = np.trace(np.linalg.solve(A, np.eye(lat.n)))
    tr_ev = np.sum(1.0 / np.linalg.eigvals(A))
    assert abs(tr_lu - tr_ev) <= 1e-12 * abs(tr_lu)
    # gamma_5-hermiticity makes the trace of the inverse real
    assert abs(tr_lu.imag) <= 1e-12 * abs(tr_lu)


def test_batch_apply_matches_single():
    lat = _random_lattice((2, 2, 2, 2))
    X = synth.random_fields(3, lat.V, 4).reshape(3, -1)
    Y = lat.apply(X)
    for r in range(3):
        assert np.array_equal(Y[r], lat.apply(X[r]))
