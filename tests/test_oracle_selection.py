"""Pins of the oracle's eigenvalue selection (the enumerated algorithm of
Sec. 4: imaglim, evectol, left vectors from gamma_5) and of its PP-Arnoldi
Ritz extraction (Sec. 4, setup step 2(b) of Sec. 5).  No GPU.

The selection is pinned on hand-built candidates whose residuals are set by
construction, so the accepted set, the pair map and the biorthonormal left
vectors are known in advance: gamma_5 swaps the two vectors of a conjugate
pair, A z_i = lambda_i z_i + r_i e, and A^H acts on u as conj(lambda) u plus a
chosen component along another unit vector.  A random unitary rotation of the
whole space leaves every residual unchanged and makes the vectors dense.  The
Ritz extraction is pinned against LAPACK: with a full Krylov space the Ritz
pairs of B = A p_in(A) are exact eigenpairs of A.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import deflation, dense, krylov

IMAGLIM, EVECTOL = 2e-4, 1e-3


def _hand_built(cases, seed=0):
    """cases: list of (lambda, right residual, left residual, partner) with
    partner = index of the other member of a conjugate pair (gamma_5 swaps the
    two), or None for a value gamma_5 maps to itself.  Returns the inputs of
    select_eigs and the rotation Q."""
    k = len(cases)
    n = k + 2                                     # two spare directions carry the residuals
    e_r, e_l = n - 1, n - 2
    lam = np.array([c[0] for c in cases], dtype=np.complex128)
    Z = np.eye(n, dtype=np.complex128)[:k]
    AZ = np.zeros((k, n), dtype=np.complex128)
    for i, (l, rr, _rl, _p) in enumerate(cases):
        AZ[i, i] = l
        AZ[i, e_r] = rr
    G5 = np.eye(n, dtype=np.complex128)
    for i, c in enumerate(cases):
        p = c[3]
        if p is not None:
            G5[i, i] = 0.0
            G5[p, i] = -1.0                         # gamma_5 e_i = -e_p: an involution with a sign
        elif i % 2:
            G5[i, i] = -1.0
    assert np.allclose(G5 @ G5, np.eye(n))
    # A^H: the left vector of candidate i is u = gamma_5 z_partner = -e_i (or
    # gamma_5 z_i = +-e_i for a value gamma_5 maps to itself), so A^H e_i =
    # conj(lambda_i) e_i + rl_i e_l gives candidate i the left residual rl_i
    MH = np.zeros((n, n), dtype=np.complex128)
    for i, (l, _rr, rl, _p) in enumerate(cases):
        MH[i, i] = np.conj(l)
        MH[e_l, i] = rl
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Zq, AZq = Z @ Q.T, AZ @ Q.T
    g5 = lambda v: Q @ (G5 @ (Q.conj().T @ v))
    ah = lambda v: Q @ (MH @ (Q.conj().T @ v))
    return lam, Zq, AZq, g5, ah, Q


# walk order of select_eigs: candidates sorted by |lambda| (as pp_arnoldi_ritz returns them)
CASES = [
    (0.010 + 1.9e-4j, 1e-5, 2e-5, None),          # 0 real: |Im| just inside imaglim -> accepted
    (0.020 + 2.1e-4j, 1e-5, 1e-5, None),          # 1 |Im| just outside, next is no partner -> skipped
    (0.030 + 0.010j, 3e-5, 4e-5, 3),              # 2, 3 exact conjugate pair -> both accepted
    (0.030 - 0.010j, 5e-5, 6e-5, 2),
    (0.050 + 0.020j, 1e-5, 2e-3, 5),              # 4, 5 pair, one left residual above evectol -> both rejected
    (0.050 - 0.020j, 1e-5, 1e-5, 4),
    (0.060, 2e-3, 1e-5, None),                    # 6 real, right residual above evectol -> rejected
    (0.070, 1e-5, 1.01e-3, None),                 # 7 real, left residual just above evectol -> rejected
    (0.080 - 1.9e-4j, 0.99e-3, 0.98e-3, None),    # 8 real, both residuals just below evectol -> accepted
    (0.090 + 0.030j, 2e-5, 3e-5, 10),             # 9, 10 near pair: |l10 - conj(l9)| = 1.5e-4 -> accepted
    (0.090 - 0.030j + 1.5e-4, 4e-5, 5e-5, 9),
    (0.100 + 0.050j, 1e-5, 1e-5, None),           # 11 complex, next value is not its conjugate -> skipped
    (0.100 + 0.0501j, 1e-5, 1e-5, None),          # 12 complex, last, unpaired -> skipped
]


def test_selection_hand_built_outcome():
    lam, Z, AZ, g5, ah, Q = _hand_built(CASES)
    assert np.all(np.diff(np.abs(lam)) >= 0)
    tr = krylov.select_eigs(lam, Z, AZ, g5, ah, IMAGLIM, EVECTOL)
    acc = [0, 2, 3, 8, 9, 10]
    assert np.array_equal(tr.lam, lam[acc])
    assert np.array_equal(tr.Z, Z[acc])
    # pair map: position of the partner among the accepted values
    assert tr.pair.tolist() == [0, 2, 1, 3, 5, 4]
    # residuals as built (rounding of the rotation only)
    assert np.allclose(tr.res_right, [CASES[i][1] for i in acc], rtol=1e-9)
    assert np.allclose(tr.res_left, [CASES[i][2] for i in acc], rtol=1e-9)
    # left vectors: u_q = gamma_5 z_partner scaled so u_q^H z_q = 1; here that is the rotated e_q
    assert np.allclose(np.einsum("ij,ij->i", tr.U.conj(), tr.Z), 1.0, rtol=0, atol=1e-13)
    want_U = (Q @ np.eye(Q.shape[0])[:, acc]).T
    assert np.max(np.abs(tr.U - want_U)) < 1e-13


@pytest.mark.parametrize("mutate,expect", [
    # moving a value across imaglim changes the walk: a real value becomes an unpaired complex one
    (lambda c: c.__setitem__(0, (0.010 + 2.05e-4j,) + c[0][1:]), [2, 3, 8, 9, 10]),
    # a pair separated by more than imaglim is two unpaired complex values
    (lambda c: c.__setitem__(10, (0.090 - 0.030j + 2.5e-4,) + c[10][1:]), [0, 2, 3, 8]),
    # every residual of the rejected pair below evectol -> the pair is accepted
    (lambda c: c.__setitem__(4, (0.050 + 0.020j, 1e-5, 1e-5, 5)), [0, 2, 3, 4, 5, 8, 9, 10]),
])
def test_selection_hand_built_thresholds(mutate, expect):
    cases = list(CASES)
    mutate(cases)
    lam, Z, AZ, g5, ah, Q = _hand_built(cases, seed=1)
    tr = krylov.select_eigs(lam, Z, AZ, g5, ah, IMAGLIM, EVECTOL)
    assert np.array_equal(tr.lam, lam[expect])
    assert np.allclose(np.einsum("ij,ij->i", tr.U.conj(), tr.Z), 1.0, atol=1e-13)


def test_selection_on_exact_triplets_gives_lapack_left_vectors():
    """Exact eigenpairs of a gamma_5-hermitian matrix (2^4 lattice): every
    candidate passes, and the selected left vectors are LAPACK's left
    eigenvectors (up to the biorthonormal scale)."""
    dims = (2, 2, 2, 2)
    lat = oracle.Lattice(dims, 0.16, synth.gauge_links(dims, 0.5, 21))
    A = dense.dense_matrix(lat)
    mu, X = np.linalg.eig(A)
    order = np.argsort(np.abs(mu), kind="stable")[:24]
    lam, Z = mu[order], (X[:, order] / np.linalg.norm(X[:, order], axis=0)).T
    AZ = Z @ A.T
    tr = krylov.select_eigs(lam, Z, AZ, lat.gamma5, lambda v: A.conj().T @ v, IMAGLIM, EVECTOL)
    npair = int(np.sum(np.arange(len(tr.pair)) != tr.pair))
    assert len(tr.lam) >= 20 and npair >= 2
    for q in range(len(tr.lam)):
        u = tr.U[q]
        assert np.linalg.norm(A.conj().T @ u - np.conj(tr.lam[q]) * u) < 1e-10 * np.linalg.norm(u)
        assert abs(np.vdot(u, tr.Z[q]) - 1.0) < 1e-12
    # biorthogonality across different eigenvalues: u_p^H z_q = 0
    G = tr.U.conj() @ tr.Z.T
    assert np.max(np.abs(G - np.eye(len(tr.lam)))) < 1e-9


def test_pp_arnoldi_ritz_against_lapack():
    """With a full Krylov space the Ritz pairs of B = A p_in(A) are exact, so
    pp_arnoldi_ritz returns eigenpairs of A (LAPACK), namely the nev whose
    B-eigenvalue lambda p_in(lambda) is smallest in modulus, sorted by |lambda|."""
    dims = (2, 2, 2, 2)
    lat = oracle.Lattice(dims, 0.16, synth.gauge_links(dims, 0.5, 21))
    A = dense.dense_matrix(lat)
    r0 = synth.gaussian_start(lat.n, 4)
    t_in = krylov.gmres_polys(lat.apply, r0, [3]).inv_roots[3]    # a low degree: |lambda p(lambda)| order != |lambda| order
    opB = krylov.pp_operator(lat.apply, t_in, lambda t, v: lat.poly_apply(t, v)[0])
    nev = 16
    lam, Z, AZ, arn = krylov.pp_arnoldi_ritz(opB, lat.apply, r0, lat.n, nev)
    assert arn.m >= lat.n - 1
    mu = np.linalg.eigvals(A)
    beta = mu * deflation.poly_eval(t_in, mu)
    want = mu[np.argsort(np.abs(beta), kind="stable")[:nev]]
    # the chosen set differs from the nev smallest |lambda| (so the ordering key is checked)
    smallest = mu[np.argsort(np.abs(mu))[:nev]]
    assert max(np.min(np.abs(smallest - w)) for w in want) > 1e-6
    for l in want:
        assert np.min(np.abs(lam - l)) < 1e-10
    assert np.all(np.diff(np.abs(lam)) >= 0)
    for i in range(nev):
        assert abs(np.linalg.norm(Z[i]) - 1.0) < 1e-13
        assert np.linalg.norm(AZ[i] - A @ Z[i]) < 1e-12
        assert np.linalg.norm(A @ Z[i] - lam[i] * Z[i]) < 1e-9
