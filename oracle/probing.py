"""Oracle of the exact lowest level by probing (Sec. 5 step 3d): test
infrastructure only, never imported by the product.

p(A) of degree d couples sites within taxicab distance d of the periodic
lattice; with a colouring in which sites of one colour are more than d apart,
Tr p(A) = sum over colours c and unknowns k of b^H p(A) b, b the indicator of
unknown k on the sites of colour c.  The oracle builds its own colouring by
brute force (every pair of sites, plain loops) and applies p(A) with its own
Newton recurrence; tiny lattices only.
"""
from __future__ import annotations

import numpy as np


def torus_distance(dims, a: int, b: int) -> int:
    """Taxicab distance between sites a and b (site = x + Lx(y + Ly(z + Lz t)))."""
    out, ra, rb = 0, a, b
    for L in dims:
        da = abs(ra % L - rb % L)
        out += min(da, L - da)
        ra //= L
        rb //= L
    return out


def distance_colouring(dims, d: int) -> np.ndarray:
    """Greedy colouring: each site takes the smallest colour no earlier site
    within distance d has."""
    V = int(np.prod(dims))
    col = [-1] * V
    for s in range(V):
        taken = {col[t] for t in range(s) if torus_distance(dims, s, t) <= d}
        c = 0
        while c in taken:
            c += 1
        col[s] = c
    return np.array(col, dtype=np.int64)


def probe_trace(lat, inv_roots, col: np.ndarray) -> complex:
    """sum_{c,k} b_{c,k}^H p(A) b_{c,k} with the oracle's Newton form."""
    V = lat.V
    ncol = int(col.max()) + 1
    B = np.zeros((12 * ncol, V, 12), dtype=np.complex128)
    for c in range(ncol):
        for k in range(12):
            B[12 * c + k, col == c, k] = 1.0
    _, bhy = lat.poly_apply(inv_roots, B.reshape(12 * ncol, 12 * V))
    return complex(np.sum(bhy))
