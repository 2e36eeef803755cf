"""Oracle deflation pieces (FP64, numpy): test infrastructure only.

* Left-right Projection (Sec. 2.1): H = U^* A V, c = U^* r_0, H d = c,
  x_hat = V d, r = r_0 - A V d.
* Left eigenvectors from gamma_5 (Sec. 4): u_i = g5 z_i for a real
  eigenvalue; u_i = g5 z_{i+1}, u_{i+1} = g5 z_i for a near-conjugate pair.
* Deflation of a polynomial-difference level (Sec. 4.1):
  Tr(M - sum_i c_i z_i u_i^*) + sum_i c_i u_i^* z_i with c_i = p_hi(l_i) - p_lo(l_i).
* Deflated polynomial operator (Sec. 4.3): one projection, then p_1 on the
  projected residual: Q b = V H^{-1} U^* b + p_1(A) (b - A V H^{-1} U^* b).
* Scalar polynomial values p(lambda) from the same Newton form.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np


def poly_eval(inv_roots: np.ndarray, lam) -> np.ndarray:
    """p(lambda) = sum_j t_j prod_{i<j} (1 - lambda t_i), t_j = theta_j^{-1}
    (the scalar version of the Newton recurrence of Sec. 3.1)."""
    lam = np.asarray(lam, dtype=np.complex128)
    w = np.ones_like(lam)
    y = np.zeros_like(lam)
    for t in np.asarray(inv_roots, dtype=np.complex128):
        y = y + t * w
        w = w - t * lam * w
    return y


def residual_poly_eval(inv_roots: np.ndarray, lam) -> np.ndarray:
    """pi(lambda) = prod_j (1 - lambda/theta_j)."""
    lam = np.asarray(lam, dtype=np.complex128)
    out = np.ones_like(lam)
    for t in np.asarray(inv_roots, dtype=np.complex128):
        out = out * (1.0 - lam * t)
    return out


def composite_eval(inv_in: np.ndarray, inv_out: np.ndarray, lam) -> np.ndarray:
    """p_1(lambda) = p_in(lambda) p_out(lambda p_in(lambda)) (Sec. 2.4)."""
    pin = poly_eval(inv_in, lam)
    return pin * poly_eval(inv_out, np.asarray(lam) * pin)


def left_vectors(Z: np.ndarray, pair: np.ndarray, gamma5: Callable) -> np.ndarray:
    """u_i = g5 z_{pair[i]}, scaled so that u_i^* z_i = 1."""
    U = np.stack([gamma5(Z[pair[i]]) for i in range(len(pair))])
    d = np.einsum("ij,ij->i", U.conj(), Z)
    return U / np.conj(d)[:, None]


def projection_matrix(apply_A: Callable, Z: np.ndarray, U: np.ndarray) -> np.ndarray:
    """H = U^* A V with V = [z_1 .. z_k] (k x k)."""
    AZ = np.stack([apply_A(z) for z in Z])
    return U.conj() @ AZ.T


def left_right_projection(apply_A: Callable, Z: np.ndarray, U: np.ndarray, H: np.ndarray,
                          r0: np.ndarray):
    """Left-right Projection (Sec. 2.1, steps 2-4) for A (x - x0) = r0.
    Returns (x_hat, r): correction V d and new residual r0 - A V d."""
    c = U.conj() @ r0
    d = np.linalg.solve(H, c)
    xh = Z.T @ d
    r = r0 - apply_A(xh)
    return xh, r


@dataclass
class DeflatedPoly:
    """The deflated polynomial operator Q of Sec. 4.3 (projection first)."""
    apply_A: Callable
    Z: np.ndarray
    U: np.ndarray
    H: np.ndarray
    apply_p1: Callable            # v -> p_1(A) v

    def apply(self, b: np.ndarray) -> np.ndarray:
        xh, r = left_right_projection(self.apply_A, self.Z, self.U, self.H, b)
        return xh + self.apply_p1(r)


def deflation_coefficients(lam: np.ndarray, f_hi: Callable, f_lo: Optional[Callable]) -> np.ndarray:
    """c_i = f_hi(lambda_i) - f_lo(lambda_i) (Sec. 4.1)."""
    c = np.asarray(f_hi(lam), dtype=np.complex128)
    if f_lo is not None:
        c = c - np.asarray(f_lo(lam), dtype=np.complex128)
    return c


def dense_triplets(Adense: np.ndarray, k: int, gamma5: Callable, imaglim: float = 1e-8):
    """Exact triplets of a small dense A: the k eigenvalues nearest the origin
    (completing a conjugate pair if the k-th splits one), right vectors from
    LAPACK, left vectors by the gamma_5 rule of Sec. 4.  Returns
    (lam, Z, pair) with unit-norm rows of Z."""
    lam, R = np.linalg.eig(Adense)
    order = np.argsort(np.abs(lam), kind="stable")
    lam, R = lam[order], R[:, order]
    Z = (R / np.linalg.norm(R, axis=0)).T
    pair = []
    i = 0
    while i < len(lam) and len(pair) < k:
        if abs(lam[i].imag) < imaglim:
            pair.append(i)
            i += 1
        else:
            j = i + 1
            if j < len(lam) and abs(lam[j] - np.conj(lam[i])) < 1e-8 * max(1.0, abs(lam[i])):
                pair += [j, i]
                i += 2
            else:
                raise ValueError("unpaired complex eigenvalue in the gamma_5-hermitian spectrum")
    kk = len(pair)
    return lam[:kk], Z[:kk], np.array(pair, dtype=np.int64)


def projection_coefficients(Z: np.ndarray, U: np.ndarray, B: np.ndarray):
    """zeta = V^* b and omega = U^* b for a batch B of shape (N, n);
    returns two (k, N) arrays (Sec. 2.1 step 2, Sec. 4.1)."""
    B = np.atleast_2d(B)
    return Z.conj() @ B.T, U.conj() @ B.T
