"""The tiled-link generator of the near-critical 16^3x32 workloads: with
periodic boundaries every eigenpair of the base lattice's operator is one of
the tiled lattice's (its eigenvector repeated), checked on small lattices
against dense eigenvalues.  No GPU."""
import numpy as np

import oracle
import synth
from oracle import dense


def test_tiled_links_repeat_the_base():
    base, dims = (2, 2, 2, 2), (4, 2, 2, 4)
    U = synth.tiled_links(dims, base, 0.3, 5)
    B = synth.gauge_links(base, 0.3, 5)
    lx, ly, lz, _ = dims
    for s in range(synth.volume(dims)):
        x, y, z, t = s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)
        bs = (x % 2) + 2 * ((y % 2) + 2 * ((z % 2) + 2 * (t % 2)))
        assert np.array_equal(U[:, s], B[:, bs])


def test_tiled_operator_contains_the_base_spectrum():
    base, dims, kappa = (2, 2, 2, 2), (4, 2, 2, 4), 0.16
    ob = oracle.Lattice(base, kappa, synth.gauge_links(base, 0.3, 5), False)
    ot = oracle.Lattice(dims, kappa, synth.tiled_links(dims, base, 0.3, 5), False)
    eb = np.linalg.eigvals(dense.dense_matrix(ob))
    et = np.linalg.eigvals(dense.dense_matrix(ot))
    for l in eb:
        assert np.min(np.abs(et - l)) < 1e-9
    # the base eigenvector repeated over the tiles is an eigenvector of the tiled operator
    w, R = np.linalg.eig(dense.dense_matrix(ob))
    i = int(np.argmin(np.abs(w)))
    zb = R[:, i].reshape(synth.volume(base), 12)
    lx, ly, lz, _ = dims
    s = np.arange(synth.volume(dims))
    x, y, z, t = s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)
    bs = (x % 2) + 2 * ((y % 2) + 2 * ((z % 2) + 2 * (t % 2)))
    zt = zb[bs].reshape(-1)
    assert np.linalg.norm(ot.apply(zt) - w[i] * zt) < 1e-10 * np.linalg.norm(zt)


def test_monomial_links_are_su3_with_exact_row_two():
    """Permutation-with-phases links: unitary, determinant 1, entries in
    {0, 1, i, -1, -i}, and row 2 = conj(row 0 x row 1) holds exactly (the
    two-row storage rebuilds them without rounding)."""
    U = synth.monomial_links((4, 2, 3, 5), 3).reshape(-1, 3, 3)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-15)
    assert np.array_equal(U @ U.conj().transpose(0, 2, 1), np.broadcast_to(np.eye(3), U.shape))
    assert set(np.unique(U)) <= {0, 1, -1, 1j, -1j}
    assert np.array_equal(np.conj(np.cross(U[:, 0, :], U[:, 1, :])), U[:, 2, :])
