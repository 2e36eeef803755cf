"""Oracle: the plain CPU FP64 definition of every step on the trace-estimation
hot path (arXiv 2306.09559, "Multipolynomial Monte Carlo for Trace
Estimation in Lattice QCD").

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import or run anything in this package.
The product path (`paper_2306_09559_amd`) never imports it and shares no code
with it; the only common inputs come from `synth` (seeded random numbers).

Contents
  ref.c          operator, Z4 generator, Newton / composite polynomial (C, FP64)
  __init__.py    ctypes wrapper returning numpy arrays in canonical layout
  krylov.py      Arnoldi/GMRES, harmonic Ritz roots, Leja order, PP-GMRES,
                 PP-Arnoldi eigenpairs, eigenvalue selection
  deflation.py   left vectors from gamma_5, Left-right Projection, deflated
                 polynomial operator, deflation coefficients
  estimator.py   level samples, level estimates, stopping rule, cost formula
  dense.py       dense matrices and free-field closed forms for tiny lattices
  solve.py       the top level Tr(A^{-1} - p_1(A)): dense solves, residuals,
                 top-level samples
  probing.py     exact Tr p(A) by probing with a brute-force distance colouring
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ref.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ref.c with gcc (FP64, no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, i64, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
            L.ora_gamma.argtypes = [i32, P]
            L.ora_gamma5_matrix.argtypes = [P]
            L.ora_wilson_apply.argtypes = [P, i32, f64, P, P, P, i32]
            L.ora_gamma5.argtypes = [i64, P, P, i32]
            L.ora_splitmix64.argtypes = [u64, u64]
            L.ora_splitmix64.restype = u64
            L.ora_noise_key.argtypes = [u64, u64, u64]
            L.ora_noise_key.restype = u64
            L.ora_z4_fill.argtypes = [u64, u64, u64, u64, i32, i64, P]
            L.ora_poly_apply.argtypes = [P, i32, f64, P, i32, P, P, P, P, i32]
            L.ora_composite_apply.argtypes = [P, i32, f64, P, i32, P, i32, P, P, P, P, i32]
            L.ora_residual_poly_apply.argtypes = [P, i32, f64, P, i32, P, P, P, i32]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _batch(x, n):
    x = _c128(x)
    if x.ndim == 1:
        return x.reshape(1, n), True
    return x.reshape(-1, n), False


class Lattice:
    """Geometry, boundary condition, hopping parameter and gauge links."""

    def __init__(self, dims, kappa: float, U: np.ndarray, antiperiodic_t: bool = True):
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.U = _c128(U).reshape(4, -1, 3, 3)
        self.antiperiodic_t = bool(antiperiodic_t)
        self.V = int(np.prod(self.dims))
        self.n = 12 * self.V
        assert self.U.shape[1] == self.V

    # -- operator -----------------------------------------------------
    def apply(self, x: np.ndarray) -> np.ndarray:
        """A x for one vector (n,) or a batch (N, n) / (N, V, 4, 3)."""
        shape = np.shape(x)
        xb, single = _batch(x, self.n)
        y = np.empty_like(xb)
        lib().ora_wilson_apply(_ptr(_dims(self.dims)), int(self.antiperiodic_t), self.kappa,
                               _ptr(self.U), _ptr(xb), _ptr(y), xb.shape[0])
        return y.reshape(shape)

    def gamma5(self, x: np.ndarray) -> np.ndarray:
        shape = np.shape(x)
        xb, _ = _batch(x, self.n)
        y = np.empty_like(xb)
        lib().ora_gamma5(self.V, _ptr(xb), _ptr(y), xb.shape[0])
        return y.reshape(shape)

    # -- polynomials --------------------------------------------------
    def poly_apply(self, inv_roots, b):
        """(p(A) b, b^H p(A) b) for the Newton form over `inv_roots` (Sec. 3.1)."""
        shape = np.shape(b)
        bb, _ = _batch(b, self.n)
        ir = _c128(inv_roots)
        y = np.empty_like(bb)
        bhy = np.empty(bb.shape[0], dtype=np.complex128)
        lib().ora_poly_apply(_ptr(_dims(self.dims)), int(self.antiperiodic_t), self.kappa, _ptr(self.U),
                             len(ir), _ptr(ir), _ptr(bb), _ptr(y), _ptr(bhy), bb.shape[0])
        return y.reshape(shape), bhy

    def composite_apply(self, inv_in, inv_out, b):
        """(p_1(A) b, b^H p_1(A) b) with p_1(A) = p_in(A) p_out(A p_in(A)) (Sec. 3.2)."""
        shape = np.shape(b)
        bb, _ = _batch(b, self.n)
        a_in, a_out = _c128(inv_in), _c128(inv_out)
        y = np.empty_like(bb)
        bhy = np.empty(bb.shape[0], dtype=np.complex128)
        lib().ora_composite_apply(_ptr(_dims(self.dims)), int(self.antiperiodic_t), self.kappa,
                                  _ptr(self.U), len(a_in), _ptr(a_in), len(a_out), _ptr(a_out),
                                  _ptr(bb), _ptr(y), _ptr(bhy), bb.shape[0])
        return y.reshape(shape), bhy

    def residual_poly_apply(self, inv_roots, b):
        """prod_j (I - A/theta_j) b, the GMRES residual polynomial."""
        shape = np.shape(b)
        bb, _ = _batch(b, self.n)
        ir = _c128(inv_roots)
        y = np.empty_like(bb)
        lib().ora_residual_poly_apply(_ptr(_dims(self.dims)), int(self.antiperiodic_t), self.kappa,
                                      _ptr(self.U), len(ir), _ptr(ir), _ptr(bb), _ptr(y), bb.shape[0])
        return y.reshape(shape)


def gamma(mu: int) -> np.ndarray:
    out = np.empty(32, dtype=np.float64)
    lib().ora_gamma(mu, _ptr(out))
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4)


def gamma5_matrix() -> np.ndarray:
    out = np.empty(32, dtype=np.float64)
    lib().ora_gamma5_matrix(_ptr(out))
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4)


def splitmix64(state: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 from `state`."""
    return int(lib().ora_splitmix64(ctypes.c_uint64(state), ctypes.c_uint64(k)))


def noise_key(seed: int, lattice: int, level: int) -> int:
    return int(lib().ora_noise_key(seed, lattice, level))


def z4(seed: int, lattice: int, level: int, first: int, nsamples: int, V: int) -> np.ndarray:
    """Z4 noise vectors, shape (nsamples, 12V) (Sec. 1: entries 1, -1, i, -i)."""
    n = 12 * V
    out = np.empty((nsamples, n), dtype=np.complex128)
    lib().ora_z4_fill(seed, lattice, level, first, nsamples, n, _ptr(out))
    return out
