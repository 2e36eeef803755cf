"""MI355X (gfx950) hot path of Multipolynomial Monte Carlo trace estimation
(Lashomb, Morgan, Whyte, Wilcox, arXiv:2306.09559).

    libmpmc.so   HIP kernels behind the C ABI of include/mpmc.h
    _lib         ctypes binding (same entry-point names, marshalling only)
    build        compiles libmpmc.so in-tree for gfx950
    krylov       GPU setup: GMRES/Arnoldi roots and PP-Arnoldi eigenvectors
    solve        deflated PP-GMRES for the top level (FP32 inner, FP64 refinement)
    driver       per-lattice state, the multilevel sampling loop, the adaptive
                 stopping rule, checkpoint / resume
    batch        several lattices' steps as one HIP graph; shape autotuner
    probing      exact low-degree traces by probing with a distance colouring
    diagnostics  deflation diagnostics (how many eigenvectors to deflate)

The binding is imported lazily so that `build` works on a machine without a
GPU; using any entry point requires the built library.
"""
import importlib

__all__ = ["_lib", "build", "krylov", "solve", "driver", "batch", "probing", "diagnostics"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
