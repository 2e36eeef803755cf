"""MI355X (gfx950) hot path of Multipolynomial Monte Carlo trace estimation
(Lashomb, Morgan, Whyte, Wilcox, arXiv:2306.09559).

    libmpmc.so   HIP kernels behind the C ABI of include/mpmc.h
    _lib         ctypes binding (same entry-point names, marshalling only)
    build        compiles libmpmc.so in-tree for gfx950
    krylov       GPU setup: GMRES/Arnoldi roots and PP-Arnoldi eigenvectors
    driver       per-lattice state and the multilevel sampling loop

The binding is imported lazily so that `build` works on a machine without a
GPU; using any entry point requires the built library.
"""
import importlib

__all__ = ["_lib", "build", "krylov", "driver"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
