"""The five synthetic workloads (lattice, links, kappa, polynomial levels,
sample counts, deflation size, seeds).

Levels are listed top (highest degree) to bottom.  A level is a pair of
operators (hi, lo) whose trace difference is estimated with Hutchinson
samples; lo = None marks the last level Tr(p_lo(A)) estimated on its own.
Degrees follow the GMRES convention: a polynomial of degree d has d+1
residual-polynomial roots and costs d matrix-vector products per application
(Sec. 3.1).  A composite polynomial is written (n_in, n_out): n_in inner
roots (p_in of degree n_in-1) and n_out outer roots, total degree
n_in*n_out - 1 (Sec. 3.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple, Union

Poly = Union[int, Tuple[int, int], str]  # degree of a single polynomial, (n_in, n_out) composite, or SOLVE

# The operator A^{-1} of the top level Tr(A^{-1} - p_1(A)) (Sec. 5 step 3a):
# its samples b^H A^{-1} b need a linear solve per noise vector.
SOLVE = "solve"


@dataclass(frozen=True)
class Level:
    hi: Poly
    lo: Optional[Poly]
    samples: int
    deflated: bool = False


@dataclass(frozen=True)
class LatticeConfig:
    name: str
    dims: Tuple[int, int, int, int]   # Lx, Ly, Lz, Lt
    eps: float                        # link roughness, U = exp(i eps H)
    kappa: float
    levels: Tuple[Level, ...]
    k_defl: int = 0                   # deflation eigenvectors
    antiperiodic_t: bool = True
    seed_links: int = 0
    seed_start: int = 0
    seed_noise: int = 0
    lattice_id: int = 0
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def volume(self) -> int:
        lx, ly, lz, lt = self.dims
        return lx * ly * lz * lt

    @property
    def n(self) -> int:
        return 12 * self.volume


C1 = LatticeConfig(
    name="C1", dims=(4, 4, 4, 4), eps=0.5, kappa=0.150,
    levels=(Level(20, 5, 100), Level(5, None, 100)),
    seed_links=101, seed_start=102, seed_noise=103, lattice_id=1,
    description="4^4 lattice, n=3072, polys deg 20 and 5, 2-level MLMC, 100 Z4 vectors, dense-LU exact trace check",
)

# kappa for C2 puts the eigenvalue of A nearest the origin at |lambda| = 1e-3.
# It was found once from the largest-real-part eigenvalues of the hopping term
# on these links (tests/golden/tune_kappa.py).  Time is periodic here: with
# an antiperiodic time direction the edge of the hopping spectrum of these
# smooth links is a complex pair far from the real axis and no kappa brings
# an eigenvalue of A within 1e-3 of the origin.
C2 = LatticeConfig(
    name="C2", dims=(8, 8, 8, 8), eps=0.3, kappa=0.13241373193166625, antiperiodic_t=False,
    levels=(Level(150, 30, 256, deflated=True), Level(30, 8, 256, deflated=True), Level(8, None, 256)),
    k_defl=20, seed_links=201, seed_start=202, seed_noise=203, lattice_id=2,
    description="8^4 lattice, n=49152, 3 levels deg 150/30/8, 20 deflated eigenvectors, 256 Z4 vectors, plain FP64",
)

C3 = LatticeConfig(
    name="C3", dims=(16, 16, 16, 32), eps=0.5, kappa=0.150,
    levels=(Level(SOLVE, (20, 15), 64, deflated=True),),
    k_defl=32, seed_links=301, seed_start=302, seed_noise=303, lattice_id=3,
    description="16^3x32, n=1.57M, composite poly 20x15 (deg 299), 64 RHS, FP32 bulk / FP64 sums",
)

# Near-critical 16^3x32 top level (n = 1.57M): the links of the 8^4 workload
# tiled 2x2x2x4 with its periodic time and kappa, so the eigenvalue of A
# nearest the origin keeps modulus 1e-3 (every eigenpair of the 8^4 operator
# is one of the tiled one).  Two set-ups of the deflation, after Example 3 and
# Sec. 6.1: "regular" runs PP(50)-Arnoldi until its PP-GMRES residual is
# 1e-12 (rtolev, Example 2); "extra" runs PP(70)-Arnoldi for a fixed 150
# steps.  Both test the 60 Ritz pairs nearest the origin, grow the outer
# polynomial of the deflated p_1 = p_in(A) p_out(A p_in(A)) until its PP-GMRES
# residual is 1e-5 (rtolpoly1, at most 50 roots) and solve with
# PP(dp_in+1)-GMRES(50) to 1e-6 (rtolle).
_C3N = dict(dims=(16, 16, 16, 32), eps=0.3, kappa=0.13241373193166625, antiperiodic_t=False, k_defl=60,
            seed_links=201, seed_start=302, seed_noise=303, lattice_id=6)
C3R = LatticeConfig(
    name="C3R", levels=(Level(SOLVE, (50, 50), 64, deflated=True),), **_C3N,
    description="near-critical 16^3x32 (8^4 links tiled), top level, regular deflation: PP(50)-Arnoldi to 1e-12",
    extra={"tile_from": (8, 8, 8, 8), "arnoldi_m": 250, "rtolev": 1e-12, "nev": 60, "rtolpoly1": 1e-5,
           "gmres_m": 50},
)
C3X = LatticeConfig(
    name="C3X", levels=(Level(SOLVE, (70, 50), 64, deflated=True),), **_C3N,
    description="near-critical 16^3x32 (8^4 links tiled), top level, extra deflation: PP(70)-Arnoldi(150)",
    extra={"tile_from": (8, 8, 8, 8), "arnoldi_m": 150, "nev": 60, "rtolpoly1": 1e-5, "gmres_m": 50},
)

C4 = LatticeConfig(
    name="C4", dims=(24, 24, 24, 48), eps=0.5, kappa=0.150,
    levels=(Level((20, 15), 60, 32, deflated=True), Level(60, 15, 128, deflated=True),
            Level(15, 4, 512, deflated=True), Level(4, None, 2048)),
    k_defl=128, seed_links=401, seed_start=402, seed_noise=403, lattice_id=4,
    description="24^3x48, n=7.96M complex64, 4 levels 299/60/15/4, at most 128 eigvecs, 32/128/512/2048 samples",
    extra={"arnoldi_m": 255, "nev": 240},
)

C5 = tuple(
    LatticeConfig(name=f"C5.{i}", dims=d, eps=0.5, kappa=kap, levels=(Level(deg, None, ns),),
                  seed_links=501 + i, seed_start=511 + i, seed_noise=521 + i, lattice_id=50 + i,
                  description="mixed batch of independent lattices")
    for i, (d, kap, deg, ns) in enumerate([
        ((8, 8, 8, 8), 0.145, 10, 64),
        ((12, 12, 12, 12), 0.149, 50, 32),
        ((16, 16, 16, 16), 0.153, 100, 16),
        ((12, 12, 12, 24), 0.157, 200, 8),
    ])
)

CONFIGS = {"C1": C1, "C2": C2, "C3": C3, "C3R": C3R, "C3X": C3X, "C4": C4}
