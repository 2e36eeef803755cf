"""GPU set-up of the multipolynomial method (Sec. 5, setup step 2):
GMRES polynomial roots and deflation eigen-triplets.

Every operation on n-vectors runs in libmpmc's kernels (operator, polynomial,
MFMA basis products, FP64 reductions); the host only handles the small
Hessenberg matrices (harmonic Ritz values, Ritz pairs, Leja order, least
squares) in FP64 with numpy.

* GMRES(maxit) from a unit random-normal start vector; the degree-d
  polynomial has as residual roots the d+1 harmonic Ritz values of step d+1
  (Sec. 3.1; all degrees from one run, setup step 2(a)).
* PP-Arnoldi on B = A p_in(A) (Sec. 4, setup step 2(b)): regular Ritz pairs
  of B nearest the origin; B shares eigenvectors with A, so each unit Ritz
  vector z gives lambda = z^H A z.
* Eigenvalue selection of Sec. 4 (imaglim / evectol), left vectors from
  gamma_5 (u_i = g5 z_i, or g5 z_{i+1} and g5 z_i for a pair) scaled so
  u_i^H z_i = 1, and H = U^H A V for the Left-right Projection (Sec. 2.1).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

F64 = L.F64


def _pad16(k: int) -> int:
    """Batch width holding k vectors: a power of two, at least 16 (the batch
    layout needs a power-of-two block width; the MFMA tiles need 16 | width)."""
    w = 16
    while w < k:
        w *= 2
    return w


def _c(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).cuda()


class DeviceArnoldi:
    """Arnoldi with classical Gram-Schmidt and one full re-orthogonalisation
    (CGS2) on the device, basis held as a batch of width mpad."""

    def __init__(self, dl: L.DeviceLattice, m: int):
        if dl.prec != F64:
            raise ValueError("the Krylov set-up runs in FP64")
        self.dl, self.m = dl, m
        self.dims, self.V = dl.dims, dl.V
        self.mpad = _pad16(m + 1)
        if self.mpad > 256:
            raise ValueError("basis wider than 256 vectors")
        self.Q = torch.zeros((1, 12, self.V, self.mpad), dtype=torch.complex128, device="cuda")
        self.w = L.empty_field(self.V, 1, 1, F64)
        self.v = L.empty_field(self.V, 1, 1, F64)
        self.x = L.empty_field(self.V, 1, 1, F64)
        self.h = torch.empty((self.mpad, 1), dtype=torch.complex128, device="cuda")
        self.nrm = torch.empty(1, dtype=torch.complex128, device="cuda")
        self.pair = torch.arange(self.mpad, dtype=torch.int32, device="cuda")
        self.ones = torch.ones(self.mpad, dtype=torch.complex128, device="cuda")
        self.minus1 = _c([-1.0])
        self.one = _c([1.0])
        probe = L.DeviceDefl(self.mpad, self.Q, self.pair, self.ones, None)
        self.ws = L.workspace(max(L.deflate_workspace_size(dl, probe, 1, 1),
                                  L.field_dot_workspace_size(self.dims, 1, 1)))

    def _basis(self, k: int) -> L.DeviceDefl:
        return L.DeviceDefl(k, self.Q, self.pair, self.ones, None)

    def _norm(self, f) -> float:
        L.field_dot(self.dims, F64, f, f, self.nrm, self.ws)
        return float(np.sqrt(max(self.nrm.cpu().numpy()[0].real, 0.0)))

    def run(self, apply_op: Callable, start: np.ndarray, stop: Optional[Callable] = None,
            breakdown_tol: float = 1e-13):
        """apply_op(x, y): y = Op x on single-vector fields.  start: canonical
        (n,) complex.  stop(j, Hbar, beta) -> bool ends the run after step j.
        Returns (Hbar (m'+1, m'), beta, m', breakdown)."""
        dims, V, m = self.dims, self.V, self.m
        canon = torch.from_numpy(np.ascontiguousarray(start.reshape(1, V, 4, 3).astype(np.complex128))).cuda()
        L.pack_fields(dims, F64, canon, self.w)
        beta = self._norm(self.w)
        L.field_axpby(dims, F64, _c([1.0 / beta]), self.w, None, self.w)
        L.field_copy_vector(dims, F64, self.w, 0, self.Q, 0)
        # v holds the newest basis vector as its own contiguous field (the
        # basis column it equals is strided by the basis width)
        self.v, self.w = self.w, self.v
        H = np.zeros((m + 1, m), dtype=np.complex128)
        taken, broke = m, False
        for j in range(m):
            apply_op(self.v, self.w)
            basis = self._basis(j + 1)
            hcol = np.zeros(j + 1, dtype=np.complex128)
            for _ in range(2):
                L.deflate_project(self.dl, basis, L.DEFL_COEFF, 1, 1, self.w, None, self.h, None, None, None, self.ws)
                L.deflate_project(self.dl, basis, L.DEFL_RECON, 1, 1, None, None, None, None, self.h, self.x,
                                  self.ws)
                L.field_axpby(dims, F64, self.minus1, self.x, self.one, self.w)
                hcol += self.h[: j + 1, 0].cpu().numpy()
            hn = self._norm(self.w)
            H[: j + 1, j] = hcol
            H[j + 1, j] = hn
            if hn <= breakdown_tol * max(1.0, float(np.abs(hcol).max())):
                taken, broke = j + 1, True
                break
            L.field_axpby(dims, F64, _c([1.0 / hn]), self.w, None, self.w)
            L.field_copy_vector(dims, F64, self.w, 0, self.Q, j + 1)
            self.v, self.w = self.w, self.v
            if stop is not None and stop(j, H[: j + 2, : j + 1], beta):
                taken = j + 1
                break
        return H[: taken + 1, :taken], beta, taken, broke


# ------------------------------------------------------------------ small dense algebra
def harmonic_ritz_values(Hbar: np.ndarray, m: int) -> np.ndarray:
    """Roots of the GMRES residual polynomial after m steps: eigenvalues of
    H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^T (or of H_m after a breakdown)."""
    Hm = np.array(Hbar[:m, :m])
    if Hbar.shape[0] > m:
        em = np.zeros(m, dtype=np.complex128)
        em[m - 1] = 1.0
        g = np.linalg.solve(Hm.conj().T, em)
        Hm[:, m - 1] += abs(Hbar[m, m - 1]) ** 2 * g
    return np.linalg.eigvals(Hm)


def leja(points: Sequence[complex]) -> np.ndarray:
    """Leja ordering: largest modulus first, then each next point maximises the
    product of distances to the points already chosen (log-sum, ties to the
    lower index; exact repeats of chosen points are taken last)."""
    z = np.asarray(points, dtype=np.complex128)
    n = len(z)
    chosen = np.zeros(n, dtype=bool)
    order = []
    first = int(np.argmax(np.abs(z)))        # argmax returns the lowest index on ties
    order.append(first)
    chosen[first] = True
    logd = np.zeros(n)
    for _ in range(n - 1):
        with np.errstate(divide="ignore"):
            logd = logd + np.log(np.abs(z - z[order[-1]]))
        cand = np.where(chosen, -np.inf, logd)
        if np.all(np.isneginf(cand[~chosen])):
            nxt = int(np.flatnonzero(~chosen)[0])
        else:
            nxt = int(np.argmax(cand))
        order.append(nxt)
        chosen[nxt] = True
    return z[np.array(order)]


def gmres_residual(Hbar: np.ndarray, beta: float, m: int) -> float:
    """min_y || beta e_1 - Hbar_m y || via a QR factorisation."""
    Hb = Hbar[: m + 1, :m]
    Qr, Rr = np.linalg.qr(Hb, mode="complete")
    g = beta * Qr.conj().T[:, 0]
    return float(abs(g[m])) if Hb.shape[0] > m else 0.0


def newton_value(inv_roots: np.ndarray, lam) -> np.ndarray:
    """p(lambda) from the Newton form used on vectors: w <- w - t w lambda,
    y <- y + t w, over the inverse roots in their application order."""
    lam = np.asarray(lam, dtype=np.complex128)
    acc = np.zeros_like(lam)
    w = np.ones_like(lam)
    for t in inv_roots:
        acc += t * w
        w = w * (1.0 - t * lam)
    return acc


def composite_value(inv_in: np.ndarray, inv_out: np.ndarray, lam) -> np.ndarray:
    """p_1(lambda) = p_in(lambda) p_out(lambda p_in(lambda)) (Sec. 3.2)."""
    pin = newton_value(inv_in, lam)
    return pin * newton_value(inv_out, np.asarray(lam) * pin)


# ------------------------------------------------------------------ operators
class Operators:
    """A and B = A p_in(A) on single vectors, through the library."""

    def __init__(self, dl: L.DeviceLattice):
        self.dl = dl
        self.tmp = L.empty_field(dl.V, 1, 1, dl.prec)
        self._ws = None
        self._poly = None

    def A(self, x, y):
        L.wilson_apply(self.dl, x, y)

    def set_pin(self, poly: L.DevicePoly):
        self._poly = poly
        self._ws = L.workspace(L.poly_workspace_size(self.dl, poly, 1, 1))

    def B(self, x, y):
        L.poly_apply(self.dl, self._poly, 1, 1, x, None, self.tmp, None, self._ws)
        L.wilson_apply(self.dl, self.tmp, y)


@dataclass
class RootSet:
    inv_roots: Dict[int, np.ndarray]        # degree -> Leja-ordered 1/theta (host)
    device: Dict[int, L.DevicePoly]
    residual: Dict[int, float]              # GMRES relative residual at step d+1


def gmres_roots(dl: L.DeviceLattice, degrees: Sequence[int], start: np.ndarray) -> RootSet:
    """Setup step 2(a): one GMRES(maxit) run, maxit = max(d)+1."""
    ops = Operators(dl)
    arn = DeviceArnoldi(dl, max(degrees) + 1)
    H, beta, m, _ = arn.run(ops.A, start)
    inv, dev, res = {}, {}, {}
    for d in degrees:
        mm = min(d + 1, m)
        th = leja(harmonic_ritz_values(H, mm))
        inv[d] = 1.0 / th
        dev[d] = L.DevicePoly(_c(inv[d]))
        res[d] = gmres_residual(H, beta, mm) / beta
    return RootSet(inv, dev, res)


def select_eigenvalues(lam: np.ndarray, right_res: np.ndarray, left_res: Callable[[int, int], float],
                       imaglim: float, evectol: float, kmax: int):
    """The selection walk of Sec. 4 over candidates sorted by |lambda|.

    A value with |Im lambda| < imaglim is taken as real: accepted when its
    right residual ||A z - lambda z|| and the left residual of u = g5 z are
    both below evectol.  Otherwise, when the next value lies within imaglim of
    conj(lambda), the two are a conjugate pair whose left vectors are g5 of
    the partner's right vector: both are accepted when all four residuals are
    below evectol.  Any other value is skipped.  At most kmax values are
    accepted (a pair only as a whole).

    right_res[i] is the right residual of candidate i; left_res(i, src) the
    residual ||A^H u - conj(lambda_i) u|| of the unit vector u = g5 z_src.
    Returns the accepted candidate indices, each one's partner index (itself
    for a real value), and their right and left residuals."""
    acc: List[int] = []
    pair: List[int] = []
    rrs: List[float] = []
    rls: List[float] = []
    i, k = 0, len(lam)
    while i < k and len(acc) < kmax:
        l = lam[i]
        if abs(l.imag) < imaglim:
            if right_res[i] < evectol and left_res(i, i) < evectol:
                acc.append(i); pair.append(i); rrs.append(float(right_res[i])); rls.append(left_res(i, i))
            i += 1
        elif i + 1 < k and abs(lam[i + 1] - np.conj(l)) < imaglim:
            if len(acc) + 2 <= kmax:
                r1, r2 = float(right_res[i]), float(right_res[i + 1])
                b1, b2 = left_res(i, i + 1), left_res(i + 1, i)
                if max(r1, r2, b1, b2) < evectol:
                    acc += [i, i + 1]; pair += [i + 1, i]; rrs += [r1, r2]; rls += [b1, b2]
            i += 2
        else:
            i += 1
    return acc, pair, rrs, rls


@dataclass
class Deflation:
    device: L.DeviceDefl
    lam: np.ndarray          # accepted eigenvalues (k,)
    pair: np.ndarray
    res_right: np.ndarray
    res_left: np.ndarray
    candidates: int
    arnoldi_steps: int = 0       # PP-Arnoldi steps taken
    arnoldi_residual: float = float("nan")   # PP-GMRES relative residual on that basis
    ritz: Optional[dict] = None  # with keep_candidates: the Ritz pairs the selection walked


def pp_arnoldi_deflation(dl: L.DeviceLattice, pin: L.DevicePoly, start: np.ndarray, m: int, nev: int,
                         kmax: int, imaglim: float = 2e-4, evectol: float = 1e-3,
                         rtolev: Optional[float] = None, keep_candidates: bool = False) -> Deflation:
    """Setup step 2(b): PP-Arnoldi, Ritz pairs nearest the origin, selection.
    The Arnoldi run takes m steps, or stops earlier once the relative residual
    of the PP-GMRES solution of B y = start on the same basis is at most
    rtolev (the paper's stopping rule; a fixed step count is its "extra
    deflation" set-up, Sec. 6.1)."""
    dims, V = dl.dims, dl.V
    ops = Operators(dl)
    ops.set_pin(pin)
    arn = DeviceArnoldi(dl, m)
    stop = None
    if rtolev is not None:
        def stop(j, Hb, b):
            return gmres_residual(Hb, b, j + 1) <= rtolev * b
    H, beta, mm, _ = arn.run(ops.B, start, stop)
    mu, G = np.linalg.eig(H[:mm, :mm])
    idx = np.argsort(np.abs(mu))[:nev]
    kp = _pad16(nev)
    # Ritz vectors Z = Q_m G (MFMA reconstruction into a batch of width kp)
    Gp = np.zeros((arn.mpad, kp), dtype=np.complex128)
    Gp[:mm, : len(idx)] = G[:, idx]
    Zb = torch.zeros((1, 12, V, kp), dtype=torch.complex128, device="cuda")
    basis = arn._basis(mm)
    wsr = L.workspace(L.deflate_workspace_size(dl, basis, kp, kp))
    L.deflate_project(dl, basis, L.DEFL_RECON, kp, kp, None, None, None, None, _c(Gp[:mm]), Zb, wsr)
    wsd = L.workspace(L.field_dot_workspace_size(dims, kp, kp))
    nrm = torch.empty(kp, dtype=torch.complex128, device="cuda")
    L.field_dot(dims, F64, Zb, Zb, nrm, wsd)
    nn = np.sqrt(np.maximum(nrm.cpu().numpy().real, 1e-300))
    alpha = np.where(np.arange(kp) < len(idx), 1.0 / nn, 0.0)
    L.field_axpby(dims, F64, _c(alpha), Zb, None, Zb)
    # lambda = z^H A z and residual norms from batched operator applications
    AZ = torch.empty_like(Zb)
    L.wilson_apply(dl, Zb, AZ)
    zaz = torch.empty(kp, dtype=torch.complex128, device="cuda")
    L.field_dot(dims, F64, Zb, AZ, zaz, wsd)
    lam_all = zaz.cpu().numpy()[: len(idx)]
    order = np.argsort(np.abs(lam_all), kind="stable")

    one = (L.empty_field(V, 1, 1, F64), L.empty_field(V, 1, 1, F64))   # the single-candidate residuals

    def resid(coef: np.ndarray, src_perm: np.ndarray) -> np.ndarray:
        """|| A z_p - coef_i z_p || for p = src_perm[i]: for several
        candidates in the batch's own column order (one coefficient per
        column, no vector moved), for one candidate on single-vector fields."""
        if len(src_perm) == 1:
            P, R = one
            L.field_copy_vector(dims, F64, Zb, int(src_perm[0]), P, 0)
            L.field_copy_vector(dims, F64, AZ, int(src_perm[0]), R, 0)
            cpad = np.array([-complex(coef[0])])
            sel = np.array([0])
            w = 1
        else:
            P, R = Zb, AZ.clone()
            w = kp
            cpad = np.zeros(w, dtype=np.complex128)
            cpad[np.asarray(src_perm)] = -np.asarray(coef)
            sel = np.asarray(src_perm)
        L.field_axpby(dims, F64, _c(cpad), P, _c(np.ones(w)), R)
        out = torch.empty(w, dtype=torch.complex128, device="cuda")
        L.field_dot(dims, F64, R, R, out, wsd)
        return np.sqrt(np.maximum(out.cpu().numpy().real[sel], 0.0))

    lam_s = lam_all[order]
    rr_all = resid(lam_s, order)
    left_cache: Dict[tuple, float] = {}

    def left_res(a: int, src: int) -> float:
        # A^H g5 z = g5 A z, so ||A^H u - conj(l) u|| = ||A z_src - conj(l) z_src|| for unit u = g5 z_src
        key = (a, src)
        if key not in left_cache:
            left_cache[key] = float(resid(np.array([np.conj(lam_s[a])]), np.array([order[src]]))[0])
        return left_cache[key]

    acc, pair, rrs, rls = select_eigenvalues(lam_s, rr_all, left_res, imaglim, evectol, kmax)
    if not acc:
        raise RuntimeError("no eigenvalue passed the deflation selection")
    arnoldi_steps = mm
    ka = len(acc)
    kpa = _pad16(ka)
    pos = {a: q for q, a in enumerate(acc)}
    pr = np.array([pos[p] for p in pair], dtype=np.int32)
    Vf = torch.zeros((1, 12, V, kpa), dtype=torch.complex128, device="cuda")
    for q, a in enumerate(acc):
        L.field_copy_vector(dims, F64, Zb, int(order[a]), Vf, q)
    lam = lam_s[np.array(acc)]
    # scaling: u_i = s_i g5 z_pair(i), u_i^H z_i = 1 -> s_i = 1 / conj(z_pair(i)^H g5 z_i)
    ident = L.DeviceDefl(ka, Vf, torch.arange(kpa, dtype=torch.int32, device="cuda"),
                         torch.ones(kpa, dtype=torch.complex128, device="cuda"), None)
    wsc = L.workspace(L.deflate_workspace_size(dl, ident, kpa, kpa))
    G5 = torch.empty((ka, kpa), dtype=torch.complex128, device="cuda")
    L.deflate_project(dl, ident, L.DEFL_COEFF, kpa, kpa, Vf, None, None, G5, None, None, wsc)
    g5 = G5.cpu().numpy()
    gii = np.array([g5[pr[q], q] for q in range(ka)])
    scale = 1.0 / np.conj(gii)
    # H = U^H A V
    defl = L.DeviceDefl(ka, Vf, torch.from_numpy(pr).cuda(), _c(scale), None)
    AV = torch.empty_like(Vf)
    L.wilson_apply(dl, Vf, AV)
    UAV = torch.empty((ka, kpa), dtype=torch.complex128, device="cuda")
    L.deflate_project(dl, defl, L.DEFL_COEFF, kpa, kpa, AV, None, None, UAV, None, None, wsc)
    Hm = UAV.cpu().numpy()[:, :ka]
    defl.hinv = _c(L.small_inverse(Hm))       # MpmcError(ESINGULAR) for a singular U^H A V
    torch.cuda.synchronize()
    ritz = None
    if keep_candidates:
        # lam: candidates in walk order; Z: unit Ritz vectors (batch of width kp), candidate i at column order[i]
        ritz = dict(lam=lam_s, Z=Zb, order=order, right_res=rr_all)
    return Deflation(defl, lam, pr, np.array(rrs), np.array(rls), len(order), arnoldi_steps,
                     gmres_residual(H, beta, mm) / beta, ritz)


@dataclass
class OuterRoots:
    inv_roots: np.ndarray        # Leja-ordered 1/phi (host)
    device: L.DevicePoly         # composite p_in(A) p_out(A p_in(A))
    residual: float              # PP-GMRES relative residual after the steps taken

    @property
    def n_out(self) -> int:
        return len(self.inv_roots)


def pp_outer_roots(dl: L.DeviceLattice, pin: L.DevicePoly, inv_in: np.ndarray, defl: Optional[Deflation],
                   n_out: int, noise: L.Noise, rtol: Optional[float] = None) -> OuterRoots:
    """Setup step 2(c): the deflated double polynomial.  A Z4 start vector is
    deflated with one Left-right Projection (Sec. 2.1) when triplets are
    given, then n_out steps of PP-GMRES on B = A p_in(A) from it -- or fewer:
    with rtol (the paper's rtolpoly1) the run stops at the first step whose
    GMRES residual is at most rtol times the norm of the Z4 vector.  The
    harmonic Ritz values of the last step are the roots phi_j of the outer
    residual polynomial pi_out(beta), beta = a p_in(a) (Sec. 3.2, Sec. 4.3)."""
    dims, V = dl.dims, dl.V
    b = L.empty_field(V, 1, 1, F64)
    L.z4_fill(dims, F64, noise, b)
    ref = float(np.sqrt(12.0 * V))               # || Z4 vector ||: every entry has modulus 1
    if defl is not None:
        r = L.empty_field(V, 1, 1, F64)
        d = torch.empty((defl.device.k, 1), dtype=torch.complex128, device="cuda")
        ws = L.workspace(L.deflate_workspace_size(dl, defl.device, 1, 1))
        L.deflate_project(dl, defl.device, L.DEFL_PROJECT, 1, 1, b, None, None, None, d, r, ws)
        b = r
    canon = torch.empty((1, V, 4, 3), dtype=torch.complex128, device="cuda")
    L.unpack_fields(dims, F64, b, canon)
    start = canon.cpu().numpy().reshape(-1)
    ops = Operators(dl)
    ops.set_pin(pin)
    arn = DeviceArnoldi(dl, n_out)
    stop = None
    if rtol is not None:
        def stop(j, Hb, bt):
            return gmres_residual(Hb, bt, j + 1) <= rtol * ref
    H, beta, m, _ = arn.run(ops.B, start, stop)
    phi = leja(harmonic_ritz_values(H, m))
    inv = 1.0 / phi
    return OuterRoots(inv, L.DevicePoly(_c(inv_in), _c(inv)), gmres_residual(H, beta, m) / ref)
