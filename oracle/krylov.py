"""Oracle Krylov machinery (FP64, numpy): test infrastructure only.

* Arnoldi with modified Gram-Schmidt and one full reorthogonalisation pass.
* GMRES polynomials from one GMRES run: the residual polynomial of GMRES at
  iteration m has the harmonic Ritz values as its roots, and a degree-d
  polynomial p is read off at iteration d+1 (Sec. 3.1, setup step 2(a) of
  the algorithm in Sec. 5).
* Leja ordering of the roots (the order both sides apply them in).
* PP-GMRES / PP-Arnoldi on B = A p_in(A) (Sec. 2.4, Sec. 4, setup step 2(b)).
* Selection of eigenvalues for deflation (the enumerated algorithm of Sec. 4).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

Op = Callable[[np.ndarray], np.ndarray]


@dataclass
class Arnoldi:
    Vb: np.ndarray      # (m+1, n) orthonormal basis rows
    Hbar: np.ndarray    # (m+1, m) upper Hessenberg
    beta: float         # norm of the start vector
    m: int              # iterations actually taken (< requested on breakdown)
    breakdown: bool


def arnoldi(op: Op, r0: np.ndarray, m: int, breakdown_tol: float = 1e-13,
            on_step: Optional[Callable[[int, np.ndarray, float], bool]] = None) -> Arnoldi:
    """m steps of Arnoldi from r0.  on_step(j, Hbar[:j+2,:j+1], beta) may
    return True to stop after step j (used for residual-tolerance stops)."""
    n = r0.shape[0]
    beta = float(np.linalg.norm(r0))
    Vb = np.zeros((m + 1, n), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    Vb[0] = r0 / beta
    taken = m
    broke = False
    for j in range(m):
        w = op(Vb[j])
        for _pass in range(2):                    # MGS, then one reorthogonalisation
            for i in range(j + 1):
                h = np.vdot(Vb[i], w)
                H[i, j] += h
                w = w - h * Vb[i]
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        if hn <= breakdown_tol * max(1.0, float(np.abs(H[: j + 1, j]).max())):
            taken, broke = j + 1, True
            break
        Vb[j + 1] = w / hn
        if on_step is not None and on_step(j, H[: j + 2, : j + 1], beta):
            taken = j + 1
            break
    return Arnoldi(Vb[: taken + 1], H[: taken + 1, :taken], beta, taken, broke)


def harmonic_ritz(Hbar: np.ndarray, m: int) -> np.ndarray:
    """Harmonic Ritz values (target 0) after m Arnoldi steps:
    eigenvalues of H_m + |h_{m+1,m}|^2 f e_m^T with f = H_m^{-H} e_m.  These are
    the roots of the GMRES residual polynomial of iteration m."""
    Hm = Hbar[:m, :m]
    if Hbar.shape[0] <= m:                        # breakdown: Krylov space invariant
        return np.linalg.eigvals(Hm)
    h = Hbar[m, m - 1]
    em = np.zeros(m, dtype=np.complex128)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.conj().T, em)
    return np.linalg.eigvals(Hm + (abs(h) ** 2) * np.outer(f, em))


def leja_order(theta: Sequence[complex]) -> np.ndarray:
    """Leja order: start with the root of largest modulus, then repeatedly take
    the remaining root maximising the product of distances to those already
    taken (sum of logs).  Ties go to the lowest original index; exact
    duplicates of a taken root have distance 0 and so come last."""
    th = np.asarray(theta, dtype=np.complex128)
    n = len(th)
    order: List[int] = []
    left = list(range(n))
    first = max(left, key=lambda i: (abs(th[i]), -i))
    order.append(first)
    left.remove(first)
    score = np.zeros(n)
    with np.errstate(divide="ignore"):
        while left:
            last = th[order[-1]]
            for i in left:
                score[i] += np.log(abs(th[i] - last))
            best = max(left, key=lambda i: (score[i], -i))
            order.append(best)
            left.remove(best)
    return th[np.array(order, dtype=np.int64)]


def gmres_ls(Hbar: np.ndarray, beta: float, m: int):
    """GMRES iterate coefficients y_m = argmin ||beta e_1 - Hbar_m y|| and the
    least-squares residual norm."""
    Hb = Hbar[: m + 1, :m]
    rhs = np.zeros(Hb.shape[0], dtype=np.complex128)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(Hb, rhs, rcond=None)
    return y, float(np.linalg.norm(rhs - Hb @ y))


@dataclass
class PolySet:
    inv_roots: Dict[int, np.ndarray]   # degree -> Leja-ordered theta^{-1}
    roots: Dict[int, np.ndarray]       # degree -> Leja-ordered theta
    arn: Arnoldi


def gmres_polys(op: Op, r0: np.ndarray, degrees: Sequence[int]) -> PolySet:
    """One GMRES(maxit) cycle, maxit = max(d)+1; the degree-d polynomial has
    the d+1 harmonic Ritz values of iteration d+1 as residual roots."""
    maxit = max(degrees) + 1
    arn = arnoldi(op, r0, maxit)
    inv, rts = {}, {}
    for d in degrees:
        m = min(d + 1, arn.m)
        th = leja_order(harmonic_ritz(arn.Hbar, m))
        rts[d] = th
        inv[d] = 1.0 / th
    return PolySet(inv, rts, arn)


def pp_operator(apply_A: Op, inv_in: np.ndarray, poly_apply: Callable) -> Op:
    """B v = A p_in(A) v (polynomial preconditioned operator, Sec. 2.3)."""
    def op(v):
        pv = poly_apply(inv_in, v)
        return apply_A(pv)
    return op


def pp_gmres_roots(opB: Op, r0: np.ndarray, n_out: Optional[int] = None,
                   rtol: Optional[float] = None, rnorm_ref: Optional[float] = None,
                   maxit: int = 400):
    """Roots of p_out: PP-GMRES on B without restarting, either for a fixed
    n_out iterations (n_out roots) or until the GMRES relative residual falls
    below rtol (relative to rnorm_ref, default ||r0||).  Returns
    (Leja-ordered phi^{-1}, Arnoldi)."""
    ref = float(np.linalg.norm(r0)) if rnorm_ref is None else float(rnorm_ref)

    def stop(j, Hb, beta):
        if rtol is None:
            return False
        _, res = gmres_ls(Hb, beta, j + 1)
        return res <= rtol * ref

    arn = arnoldi(opB, r0, n_out if n_out is not None else maxit, on_step=stop)
    m = arn.m
    phi = leja_order(harmonic_ritz(arn.Hbar, m))
    return 1.0 / phi, arn


@dataclass
class Triplets:
    lam: np.ndarray        # (k,) eigenvalues of A
    Z: np.ndarray          # (k, n) right eigenvectors, unit norm
    pair: np.ndarray       # (k,) index j such that u_i = gamma_5 z_j (scaled)
    U: np.ndarray          # (k, n) left eigenvectors, scaled so u_i^H z_i = 1
    res_right: np.ndarray
    res_left: np.ndarray


def pp_arnoldi_ritz(opB: Op, apply_A: Op, r0: np.ndarray, m: int, nev: int,
                    rtol: Optional[float] = None):
    """PP-Arnoldi (Sec. 4, setup step 2(b)): Arnoldi on B = A p_in(A), regular
    Ritz pairs of H_m; B shares eigenvectors with A, so each Ritz vector z
    gives lambda = z^H A z (unit z).  Returns the nev pairs nearest the
    origin (by |Ritz value of B|), sorted by |lambda|."""
    def stop(j, Hb, beta):
        if rtol is None:
            return False
        _, res = gmres_ls(Hb, beta, j + 1)
        return res <= rtol * beta
    arn = arnoldi(opB, r0, m, on_step=stop)
    mm = arn.m
    mu, G = np.linalg.eig(arn.Hbar[:mm, :mm])
    idx = np.argsort(np.abs(mu))[:nev]
    Z = (G[:, idx].T @ arn.Vb[:mm])
    Z = Z / np.linalg.norm(Z, axis=1, keepdims=True)
    AZ = np.stack([apply_A(z) for z in Z])
    lam = np.einsum("ij,ij->i", Z.conj(), AZ)
    order = np.argsort(np.abs(lam), kind="stable")
    return lam[order], Z[order], AZ[order], arn


def select_eigs(lam: np.ndarray, Z: np.ndarray, AZ: np.ndarray, gamma5: Op, apply_AH: Op,
                imaglim: float = 2e-4, evectol: float = 1e-3) -> Triplets:
    """Eigenvalue selection for deflation (enumerated algorithm of Sec. 4).

    Walk from the value nearest the origin.  |Im lambda| < imaglim: treat as
    real; accept if ||Az - lambda z|| < evectol and the left vector u = g5 z
    has ||A^H u - conj(lambda) u|| < evectol.  Otherwise, if the next value is
    within imaglim of conj(lambda), treat the two as a pair with
    u_i = g5 z_{i+1}, u_{i+1} = g5 z_i and accept both if all four residuals
    are below evectol.  Left vectors are finally scaled so u_i^H z_i = 1."""
    k = len(lam)
    acc: List[int] = []
    pair: List[int] = []
    rr: List[float] = []
    rl: List[float] = []
    i = 0

    def res_r(j):
        return float(np.linalg.norm(AZ[j] - lam[j] * Z[j]))

    def res_l(j, src):
        u = gamma5(Z[src])
        u = u / np.linalg.norm(u)
        return float(np.linalg.norm(apply_AH(u) - np.conj(lam[j]) * u))

    while i < k:
        if abs(lam[i].imag) < imaglim:
            a, b = res_r(i), res_l(i, i)
            if a < evectol and b < evectol:
                acc.append(i); pair.append(i); rr.append(a); rl.append(b)
            i += 1
        elif i + 1 < k and abs(lam[i + 1] - np.conj(lam[i])) < imaglim:
            a1, a2 = res_r(i), res_r(i + 1)
            b1, b2 = res_l(i, i + 1), res_l(i + 1, i)
            if max(a1, a2, b1, b2) < evectol:
                acc += [i, i + 1]; pair += [i + 1, i]
                rr += [a1, a2]; rl += [b1, b2]
            i += 2
        else:
            i += 1
    sel = np.array(acc, dtype=np.int64)
    pos = {j: q for q, j in enumerate(acc)}
    pr = np.array([pos[p] for p in pair], dtype=np.int64)
    lam_s, Z_s = lam[sel], Z[sel]
    U = np.stack([gamma5(Z_s[pr[q]]) for q in range(len(sel))]) if len(sel) else np.zeros((0, Z.shape[1]), complex)
    # biorthonormal scaling: u_i <- u_i / conj(u_i^H z_i)
    d = np.einsum("ij,ij->i", U.conj(), Z_s)
    U = U / np.conj(d)[:, None]
    return Triplets(lam_s, Z_s, pr, U, np.array(rr), np.array(rl))
