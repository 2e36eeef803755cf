"""Oracle of the top level Tr(A^{-1} - p_1(A)) (Sec. 5 step 3a): test
infrastructure only, never imported by the product.

The level's samples are s = b^H A^{-1} b - b^H Q b, with Q the deflated
double polynomial of Sec. 4.3 (or p_1(A) itself without deflation).  The
product approximates A^{-1} b with a deflated polynomial-preconditioned
GMRES to a relative residual rtolle; the oracle uses the definition itself:

* dense_solve   x = A^{-1} b by an LU factorisation of the dense matrix
                (tiny lattices only);
* residual      ||b - A x|| / ||b|| through the oracle operator, the
                property the product's solutions are checked against at
                any lattice size;
* top_level_samples  s_r = b_r^H x_r - b_r^H (Q b)_r.
"""
from __future__ import annotations

import numpy as np

from . import dense


def dense_solve(lat, B: np.ndarray) -> np.ndarray:
    """X with A X_r = B_r for a batch B (N, n) (or one vector)."""
    A = dense.dense_matrix(lat)
    B2 = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    X = np.linalg.solve(A, B2.T).T
    return X.reshape(np.shape(B))


def residual(lat, B: np.ndarray, X: np.ndarray) -> np.ndarray:
    """||b_r - A x_r|| / ||b_r|| per vector, with the oracle operator."""
    B2 = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    X2 = np.atleast_2d(np.asarray(X, dtype=np.complex128))
    R = B2 - lat.apply(X2)
    return np.linalg.norm(R, axis=1) / np.linalg.norm(B2, axis=1)


def top_level_samples(B: np.ndarray, X: np.ndarray, QB: np.ndarray) -> np.ndarray:
    """s_r = b_r^H x_r - b_r^H (Q b)_r for batches of shape (N, n)."""
    B2, X2, Q2 = (np.atleast_2d(np.asarray(a, dtype=np.complex128)) for a in (B, X, QB))
    return np.einsum("ri,ri->r", B2.conj(), X2) - np.einsum("ri,ri->r", B2.conj(), Q2)
