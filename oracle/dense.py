"""Oracle dense checks for tiny lattices (numpy): test infrastructure only.

* The dense matrix A, column by column from the oracle operator.
* The free field (all links 1): plane waves diagonalise the operator.  With
  p_mu = 2 pi n_mu / L_mu (x, y, z) and p_t = pi (2 n_t + 1) / L_t for an
  antiperiodic time direction, each momentum gives the eigenvalues
      a +- i |b|,  a = 1 - 2 kappa sum_mu cos p_mu,
                   |b| = 2 kappa sqrt(sum_mu sin^2 p_mu),
  each 6-fold (2 spin x 3 colour).  Hence
      Tr(A^{-1}) = sum_p 12 a / (a^2 + |b|^2),
      Tr(f(A))   = 6 sum_p [ f(a + i|b|) + f(a - i|b|) ].
"""
from __future__ import annotations

import itertools

import numpy as np


def dense_matrix(lat) -> np.ndarray:
    """A as an (n, n) complex128 array, built from A e_j."""
    E = np.eye(lat.n, dtype=np.complex128)
    cols = lat.apply(E)          # row j holds A e_j
    return np.ascontiguousarray(cols.T)


def free_field_eigenvalues(dims, kappa: float, antiperiodic_t: bool = True) -> np.ndarray:
    """All n eigenvalues of the free-field operator, with multiplicity."""
    lx, ly, lz, lt = dims
    out = []
    for nx, ny, nz, nt in itertools.product(range(lx), range(ly), range(lz), range(lt)):
        p = [2 * np.pi * nx / lx, 2 * np.pi * ny / ly, 2 * np.pi * nz / lz,
             (np.pi * (2 * nt + 1) / lt) if antiperiodic_t else (2 * np.pi * nt / lt)]
        a = 1.0 - 2.0 * kappa * sum(np.cos(q) for q in p)
        b = 2.0 * kappa * np.sqrt(sum(np.sin(q) ** 2 for q in p))
        out += [a + 1j * b] * 6 + [a - 1j * b] * 6
    return np.array(out, dtype=np.complex128)


def free_field_trace_inverse(dims, kappa: float, antiperiodic_t: bool = True) -> float:
    lam = free_field_eigenvalues(dims, kappa, antiperiodic_t)[::6]   # one per 6-fold block
    a, b = lam.real, np.abs(lam.imag)
    # each (a + i b, a - i b) pair appears as two consecutive entries of lam
    return float(np.sum(6.0 * a / (a ** 2 + b ** 2)))


def free_field_trace_fn(dims, kappa: float, f, antiperiodic_t: bool = True) -> complex:
    lam = free_field_eigenvalues(dims, kappa, antiperiodic_t)
    return complex(np.sum(f(lam)))
