"""Exact trace of a low-degree polynomial by probing (Sec. 3.1; Sec. 5 step 3d).

A couples nearest-neighbour sites, so p(A) of degree d couples only sites
within taxicab distance d on the periodic lattice.  Given a colouring in
which any two sites of one colour are more than d apart, the probe vectors
b_{c,k} -- 1 on unknown k (spin, colour index) of every site of colour c --
give Tr p(A) = sum_{c,k} b_{c,k}^H p(A) b_{c,k} exactly: the cross terms
between distinct sites of one colour vanish.  This replaces the Hutchinson
estimate of the lowest level of the multilevel formula.

The paper calls for a distance-d colouring of the lattice graph without
giving an algorithm.  Here: greedy colouring in site order over the
distance-d ball; a lattice whose extents are all divisible by some m > 2d
reuses the greedy colouring of the m^4 torus (two distinct sites within
distance d differ by less than m in every coordinate, so their images on the
small torus are distinct and within distance d there too).

The probe vectors are generated on the device -- inside the t-sweep from the
colouring (mpmc_noise.probe_colour), or by mpmc_probe_fill -- and applied in
scalar mode; the host sums the FP64 results in a fixed order.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def ball_offsets(d: int) -> np.ndarray:
    """All nonzero integer 4-vectors with taxicab length <= d."""
    r = range(-d, d + 1)
    off = [o for o in itertools.product(r, r, r, r) if 0 < sum(abs(v) for v in o) <= d]
    return np.array(off, dtype=np.int64)


def _coords(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    s = np.arange(lx * ly * lz * lt)
    return np.stack([s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)], axis=1)


def _index(dims, c: np.ndarray) -> np.ndarray:
    lx, ly, lz, lt = dims
    c = c % np.array(dims)
    return c[..., 0] + lx * (c[..., 1] + ly * (c[..., 2] + lz * c[..., 3]))


def greedy_colouring(dims, d: int) -> np.ndarray:
    """Greedy distance-d colouring of the periodic lattice, sites in order."""
    V = int(np.prod(dims))
    xyz = _coords(dims)
    off = ball_offsets(d)
    col = np.full(V, -1, dtype=np.int64)
    for s in range(V):
        nb = _index(dims, xyz[s] + off)
        used = col[nb]
        used = used[used >= 0]
        mark = np.zeros(len(used) + 1, dtype=bool)
        mark[used[used <= len(used)]] = True
        col[s] = int(np.argmin(mark))
    return col.astype(np.int32)


_CACHE = {}


def colouring(dims, d: int, max_greedy: int = 1 << 17) -> np.ndarray:
    """A distance-d colouring: tiled from the smallest m^4 torus (m > 2d
    dividing every extent) when that is smaller than the lattice, else greedy
    on the whole lattice.  Computed once per (lattice, d) and kept."""
    dims = tuple(int(v) for v in dims)
    key = (dims, int(d))
    if key not in _CACHE:
        _CACHE[key] = _colouring(dims, int(d), max_greedy)
    return _CACHE[key]


def _colouring(dims, d: int, max_greedy: int) -> np.ndarray:
    V = int(np.prod(dims))
    for m in range(2 * d + 1, min(dims) + 1):
        if all(L_ % m == 0 for L_ in dims) and m ** 4 < V:
            tile = greedy_colouring((m, m, m, m), d)
            c = _coords(dims) % m
            return tile[c[:, 0] + m * (c[:, 1] + m * (c[:, 2] + m * c[:, 3]))].astype(np.int32)
    if V > max_greedy:
        raise ValueError(f"no tiled colouring for {dims} at distance {d} and the lattice is too large for greedy")
    return greedy_colouring(dims, d)


def is_valid(dims, d: int, col: np.ndarray) -> bool:
    """No two distinct sites within distance d share a colour."""
    dims = tuple(int(v) for v in dims)
    xyz = _coords(dims)
    s = np.arange(len(col))
    for o in ball_offsets(d):
        nb = _index(dims, xyz + o)
        bad = (nb != s) & (col[nb] == col)
        if bad.any():
            return False
    return True


@dataclass
class ProbeResult:
    trace: complex
    ncolours: int
    probes: int
    batches: int


def probe_trace(dl: L.DeviceLattice, poly: L.DevicePoly, colour: np.ndarray, nrhs: int = 256, rb: int = 1,
                in_kernel: Optional[bool] = None) -> ProbeResult:
    """Tr p(A) = sum over probes of b^H p(A) b, probes in batches of nrhs.

    Where the t-sweep applies, the probe vectors are generated inside it
    from the colouring (like Z4 noise: never stored, no dot-vector reads);
    otherwise each batch is written by mpmc_probe_fill and applied as a
    field, laid out with block width rb = 1 (the sweep reads its input and
    dot vector site by site within one vector, coalesced only at rb = 1).
    in_kernel forces one of the two."""
    col = np.ascontiguousarray(colour, dtype=np.int32)
    ncol = int(col.max()) + 1
    nprobe = 12 * ncol
    nb = (nprobe + nrhs - 1) // nrhs
    dev_col = torch.from_numpy(col).cuda()
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
    if in_kernel is None:
        in_kernel = poly.inv_out is None and poly.inv_in.numel() >= 2 and L.sweep_plan(dl, nrhs, rb)["ok"]
    # every batch writes its b^H p(A) b into its own slice; one copy to the host at the end
    bhy = torch.empty((nb, nrhs), dtype=torch.complex128, device="cuda")
    field = None if in_kernel else L.empty_field(dl.V, nrhs, rb, dl.prec)
    for i in range(nb):
        if in_kernel:
            L.poly_apply(dl, poly, nrhs, rb, None, L.Noise(0, 0, 0, i * nrhs, probe_colour=dev_col), None, bhy[i], ws)
        else:
            L.probe_fill(dl.dims, dl.prec, dev_col, i * nrhs, field)
            L.poly_apply(dl, poly, nrhs, rb, field, None, None, bhy[i], ws)
    vals = bhy.cpu().numpy().reshape(-1)[:nprobe]      # probes past the last colour are zero vectors
    return ProbeResult(complex(np.sum(vals)), ncol, nprobe, nb)
