"""Deflation diagnostics: how many eigenvectors to deflate (Sec. 4.1, Example 1).

* `example1` reproduces the random-matrix study of Sec. 4.1 on the host:
  A = B + 21 I with B an n x n matrix of Normal(0, 1) entries.  It reports
  the 2-norm of A^{-1} after removing the k eigencomponents nearest the
  origin (right and left eigenvectors, z_i u_i^* / lambda_i), the same norm
  after removing the k smallest singular components, the overlaps
  |z_j^H z_i| of one eigenvector with its neighbours, and the norm of
  p_hi(A) - p_lo(A) (GMRES polynomials of degree 200 and 100) with its
  largest eigencomponents removed one by one.  Dense linear algebra on a
  500 x 500 matrix; the paper gives no seed, so the figures it shows are
  matched in kind, not in value.
* `level_variance_profile` asks the same question of a GPU workload in the
  terms that matter there: the Hutchinson sample variance of a deflated
  level with only its first k deflation terms c_i conj(zeta_i) omega_i
  subtracted, k = 0 .. ndefl.  One batch of the level's samples and
  zeta = V^H b, omega = U^H b of the same noise come from the library; the
  profile at k = ndefl must reproduce the level's own deflated samples.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L
from .krylov import harmonic_ritz_values, leja, newton_value


# ------------------------------------------------------------------ Example 1
def shifted_random(n: int = 500, shift: float = 21.0, seed: int = 0) -> np.ndarray:
    """A = B + shift I, B with i.i.d. Normal(0, 1) entries (real)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + shift * np.eye(n)


@dataclass
class Eigen:
    lam: np.ndarray      # eigenvalues, nearest the origin first
    Z: np.ndarray        # unit right eigenvectors as columns
    W: np.ndarray        # rows u_i^*: left eigenvectors with u_i^* z_j = delta_ij


def eigen(A: np.ndarray) -> Eigen:
    lam, Z = np.linalg.eig(A)
    order = np.argsort(np.abs(lam), kind="stable")
    lam, Z = lam[order], Z[:, order]
    Z = Z / np.linalg.norm(Z, axis=0, keepdims=True)
    return Eigen(lam, Z, np.linalg.inv(Z))


def eigen_deflation_norms(A: np.ndarray, kmax: int, eig: Optional[Eigen] = None) -> np.ndarray:
    """|| A^{-1} - sum_{i<k} z_i u_i^* / lambda_i ||_2 for k = 0 .. kmax."""
    e = eig or eigen(A)
    M = np.linalg.inv(A).astype(np.complex128)
    out = [np.linalg.norm(M, 2)]
    for i in range(kmax):
        M = M - np.outer(e.Z[:, i], e.W[i]) / e.lam[i]
        out.append(np.linalg.norm(M, 2))
    return np.array(out)


def svd_deflation_norms(A: np.ndarray, kmax: int) -> np.ndarray:
    """|| A^{-1} - sum over the k smallest singular triplets v sigma^{-1} u^H ||_2."""
    U, s, Vh = np.linalg.svd(A)
    M = np.linalg.inv(A).astype(np.complex128)
    n = len(s)
    out = [np.linalg.norm(M, 2)]
    for j in range(kmax):
        i = n - 1 - j
        M = M - np.outer(Vh[i].conj(), U[:, i].conj()) / s[i]
        out.append(np.linalg.norm(M, 2))
    return np.array(out)


def eigvec_overlaps(eig: Eigen, j: int, count: int) -> np.ndarray:
    """|z_j^H z_i| for i = 0 .. count-1 (unit vectors)."""
    return np.abs(eig.Z[:, :count].conj().T @ eig.Z[:, j])


def gmres_inverse_roots(A: np.ndarray, d: int, start: np.ndarray) -> np.ndarray:
    """Leja-ordered inverse roots of the degree-d GMRES polynomial p_d ~ A^{-1}
    (Sec. 2.3): harmonic Ritz values of d+1 Arnoldi steps (CGS2) from start."""
    n = A.shape[0]
    m = d + 1
    Q = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    Q[:, 0] = start / np.linalg.norm(start)
    for j in range(m):
        w = A @ Q[:, j]
        for _ in range(2):
            h = Q[:, : j + 1].conj().T @ w
            w = w - Q[:, : j + 1] @ h
            H[: j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        Q[:, j + 1] = w / H[j + 1, j]
    return 1.0 / leja(harmonic_ritz_values(H, m))


def poly_difference_deflation_norms(A: np.ndarray, d_hi: int, d_lo: int, kmax: int, start: np.ndarray,
                                    eig: Optional[Eigen] = None):
    """Eigenvalues of p_hi(A) - p_lo(A) (= p_hi(lambda) - p_lo(lambda)) and the
    2-norm of the difference with its k largest eigencomponents removed."""
    e = eig or eigen(A)
    c = newton_value(gmres_inverse_roots(A, d_hi, start), e.lam) - \
        newton_value(gmres_inverse_roots(A, d_lo, start), e.lam)
    order = np.argsort(-np.abs(c), kind="stable")
    out = []
    for k in range(kmax + 1):
        ck = c.copy()
        ck[order[:k]] = 0.0
        out.append(np.linalg.norm((e.Z * ck) @ e.W, 2))
    return c, order, np.array(out)


def example1(n: int = 500, shift: float = 21.0, seed: int = 0, kmax: int = 30, d_hi: int = 200,
             d_lo: int = 100) -> dict:
    """The quantities of Figures 1-3 of Sec. 4.1 for one seeded matrix."""
    A = shifted_random(n, shift, seed)
    e = eigen(A)
    start = np.random.default_rng(seed + 1).standard_normal(n).astype(np.complex128)
    c, order, pnorm = poly_difference_deflation_norms(A, d_hi, d_lo, 10, start, e)
    return {"lambda_nearest": e.lam[:kmax], "eigen_deflation": eigen_deflation_norms(A, kmax, e),
            "svd_deflation": svd_deflation_norms(A, kmax),
            "overlaps_z3": eigvec_overlaps(e, 2, kmax), "overlaps_z19": eigvec_overlaps(e, 18, kmax),
            "poly_difference_eigs": c[order[:10]], "poly_difference_deflation": pnorm}


# ------------------------------------------------------------------ GPU workloads
@dataclass
class VarianceProfile:
    k: np.ndarray              # 0 .. ndefl
    variance: np.ndarray       # sample variance with the first k deflation terms subtracted
    lam: np.ndarray            # deflated eigenvalues, in deflation order
    c: np.ndarray              # their coefficients p_hi(lambda) - p_lo(lambda)
    nsamples: int
    reproduction_error: float  # max |profile sample at k = ndefl - level sample| / max |level sample|


def level_variance_profile(run, level: int, nsamples: Optional[int] = None, first: int = 0) -> VarianceProfile:
    """Sample variance of a deflated polynomial level against the number of
    deflated eigenvectors, from one batch of the level's noise (samples
    first .. first+nsamples-1).  Runs the level kernel and the deflation
    projection on the device; the partial sums are formed on the host."""
    lv = run.levels[level]
    if lv.solver is not None or lv.c is None:
        raise ValueError(f"level {level} is not a deflated polynomial level")
    N = int(nsamples or lv.batch)
    rb = run.level_rb(level)
    if N % rb:
        raise ValueError(f"nsamples {N} is not a multiple of the level's block width {rb}")
    nz = L.Noise(run.cfg.seed_noise, run.cfg.lattice_id, lv.index, first)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(run.dl, lv.device, N, rb))
    L.mlmc_level_estimate(run.dl, lv.device, N, rb, nz, samples, acc, ws)
    defl = run.defl.device
    k = defl.k
    zeta = torch.empty((k, N), dtype=torch.complex128, device="cuda")
    omega = torch.empty((k, N), dtype=torch.complex128, device="cuda")
    wsd = L.workspace(L.deflate_workspace_size(run.dl, defl, N, rb))
    L.deflate_project(run.dl, defl, L.DEFL_COEFF, N, rb, None, nz, zeta, omega, None, None, wsd)
    S = samples.cpu().numpy()
    s_level = S[:, 0] + 1j * S[:, 1]
    raw = (S[:, 2] + 1j * S[:, 3]) - (S[:, 4] + 1j * S[:, 5])
    c = np.asarray(lv.c)
    terms = c[:, None] * np.conj(zeta.cpu().numpy()) * omega.cpu().numpy()
    partial = raw[None, :] - np.concatenate([np.zeros((1, N), dtype=np.complex128), np.cumsum(terms, axis=0)])
    mean = partial.mean(axis=1, keepdims=True)
    var = np.sum(np.abs(partial - mean) ** 2, axis=1) / (N - 1)
    err = float(np.max(np.abs(partial[-1] - s_level)) / max(np.max(np.abs(s_level)), 1e-300))
    return VarianceProfile(np.arange(k + 1), var, np.asarray(run.defl.lam), c, N, err)


def main(argv: Optional[List[str]] = None) -> None:
    import argparse
    ap = argparse.ArgumentParser(description="Deflation diagnostics of Sec. 4.1 (Example 1)")
    ap.add_argument("--n", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--kmax", type=int, default=30)
    a = ap.parse_args(argv)
    r = example1(a.n, seed=a.seed, kmax=a.kmax)
    print(" k   |lambda_k|   ||A^-1 - eig defl||   ||A^-1 - svd defl||   |z3^H z_k|  |z19^H z_k|")
    for k in range(a.kmax + 1):
        lam = f"{abs(r['lambda_nearest'][k - 1]):10.4f}" if k else " " * 10
        ov = (f"{r['overlaps_z3'][k - 1]:10.3f} {r['overlaps_z19'][k - 1]:10.3f}" if k else "")
        print(f"{k:3d} {lam}   {r['eigen_deflation'][k]:18.4f}   {r['svd_deflation'][k]:18.4f}   {ov}")
    print("largest eigenvalues of p_200(A) - p_100(A):", np.round(np.abs(r["poly_difference_eigs"]), 3))
    print("||p_200 - p_100|| with k removed:", np.round(r["poly_difference_deflation"], 4))


if __name__ == "__main__":
    main()
