"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds no arithmetic of the trace-estimation method itself: only
random gauge links, random start vectors and random test fields, all drawn
from numpy's PCG64 generator with an explicit seed, in the canonical layouts
both sides agree on:

* site index      s = x + Lx*(y + Ly*(z + Lz*t))
* vector index    i = 12*s + 3*spin + colour   (n = 12*V entries per vector)
* gauge field     complex128 array (4, V, 3, 3): U[mu, s, row, col], mu = x,y,z,t
* spinor batches  complex128 array (N, V, 4, 3), i.e. (N, n) row-major

The gauge configurations of the paper (quenched beta = 6.0 ensembles, Sec. 5
Example 2 and Example 3) are not available; these links stand in for them.
"""
from __future__ import annotations

import numpy as np

from .configs import CONFIGS, LatticeConfig  # noqa: F401


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gauge_links(dims, eps: float, seed: int) -> np.ndarray:
    """SU(3) links U = exp(i*eps*H), one per (mu, site).

    H = (M + M^H)/2 - Tr(.)/3 * I with M_ab = (g1 + i g2)/sqrt(2), g ~ N(0,1):
    a traceless Hermitian Gaussian matrix, so U is unitary with det U = 1.
    eps = 0 gives the free field U = 1.  Computed through the eigen-
    decomposition H = Q diag(h) Q^H, U = Q diag(exp(i eps h)) Q^H.
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, 4, V, 3, 3))
    M = (g[0] + 1j * g[1]) / np.sqrt(2.0)
    H = 0.5 * (M + np.conj(np.swapaxes(M, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    h, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * h)
    U = np.einsum("...ab,...b,...cb->...ac", Q, ph, np.conj(Q))
    return np.ascontiguousarray(U.astype(np.complex128))


def tiled_links(dims, base_dims, eps: float, seed: int) -> np.ndarray:
    """gauge_links(base_dims, eps, seed) repeated periodically over `dims`
    (every extent a multiple of the base's): the link at (x, y, z, t) is the
    base link at (x mod bx, y mod by, z mod bz, t mod bt).  With periodic
    boundaries in every direction each eigenpair of the base operator gives
    one of the tiled operator (the eigenvector repeated), so the tiled
    lattice keeps the base's spectral edge at any size."""
    if any(d % b for d, b in zip(dims, base_dims)):
        raise ValueError(f"{dims} is not a multiple of {base_dims}")
    base = gauge_links(base_dims, eps, seed)
    lx, ly, lz, lt = dims
    bx, by, bz, bt = base_dims
    s = np.arange(volume(dims))
    x, y, z, t = s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)
    bs = (x % bx) + bx * ((y % by) + by * ((z % bz) + bz * (t % bt)))
    return np.ascontiguousarray(base[:, bs])


def config_links(cfg) -> np.ndarray:
    """The links of a workload configuration: tiled from a smaller lattice
    when its `extra` names one ("tile_from"), else gauge_links."""
    tile = cfg.extra.get("tile_from") if cfg.extra else None
    if tile is not None:
        return tiled_links(cfg.dims, tuple(tile), cfg.eps, cfg.seed_links)
    return gauge_links(cfg.dims, cfg.eps, cfg.seed_links)


def unit_links(dims) -> np.ndarray:
    """The free field: every link is the 3x3 identity."""
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def monomial_links(dims, seed: int) -> np.ndarray:
    """SU(3) links that are permutation matrices with phases in {1, i, -1, -i}
    (determinant 1).  Products with them only move and re-sign entries, so
    operator applications to Gaussian-integer fields are exact in floating
    point: inputs for bit-exact comparisons at full size."""
    rng = np.random.default_rng(seed)
    count = 4 * volume(dims)
    perms = np.array([(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)])
    odd = np.array([0, 0, 0, 1, 1, 1])                       # the last three are transpositions
    phase = np.array([1, 1j, -1, -1j], dtype=np.complex128)  # i^q, exactly
    which = rng.integers(0, 6, count)
    q = rng.integers(0, 4, (count, 3))
    # det = sign(perm) i^(q0 + q1 + q2) = 1
    q[:, 2] = (-q[:, 0] - q[:, 1] - 2 * odd[which]) % 4
    U = np.zeros((count, 3, 3), dtype=np.complex128)
    rows = np.arange(count)
    for a in range(3):
        U[rows, a, perms[which, a]] = phase[q[:, a]]
    return U.reshape(4, -1, 3, 3)


def random_su3(count: int, seed: int) -> np.ndarray:
    """`count` Haar-ish random SU(3) matrices (QR of a complex Gaussian,
    phases fixed, determinant divided out).  Used for gauge transformations."""
    rng = np.random.default_rng(seed)
    Z = (rng.standard_normal((count, 3, 3)) + 1j * rng.standard_normal((count, 3, 3))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q = Q / (det ** (1.0 / 3.0))[:, None, None]
    return np.ascontiguousarray(Q)


def gaussian_start(n: int, seed: int) -> np.ndarray:
    """Random normal start vector of norm one (complex: i.i.d. N(0,1) real and
    imaginary parts, then normalised).  The Krylov setup starts from it."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return v / np.linalg.norm(v)


def random_fields(nrhs: int, V: int, seed: int) -> np.ndarray:
    """A batch of complex Gaussian spinor fields, shape (nrhs, V, 4, 3)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nrhs, V, 4, 3)) + 1j * rng.standard_normal((nrhs, V, 4, 3))
    return np.ascontiguousarray(x)
