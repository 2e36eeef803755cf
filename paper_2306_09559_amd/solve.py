"""Linear solves A x = b for the top level Tr(A^{-1} - p_1(A)) (Sec. 5 step 3a).

Each noise vector's solution comes from deflated polynomial-preconditioned
GMRES(m): a Left-right Projection over the accepted eigen-triplets (Sec. 2.1)
before every cycle (Sec. 4.2), then one cycle of GMRES on the right-
preconditioned operator A p_in(A), x = p_in(A) y (Sec. 2.2), with p_in the
polynomial of the PP-Arnoldi set-up.

Precision: the cycles run on FP32 fields, links and eigenvectors inside an
iterative refinement whose residual b - A x and solution update x += d are
FP64, so the solution reaches the FP64 tolerance (rtolle, Sec. 5 Example 2)
although every inner operation is FP32.  Every vector of the batch has its
own Krylov basis; the bases live on the device and are orthogonalised with
classical Gram-Schmidt and one re-orthogonalisation (CGS2) through
mpmc_field_block_dot / mpmc_field_block_axpy.  The host only solves the
small per-vector Hessenberg least-squares problems.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L


def _c(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).cuda()


@dataclass
class SolveStats:
    outer: int = 0                       # refinement steps
    cycles: int = 0                      # inner GMRES cycles (all vectors together)
    arnoldi_steps: int = 0               # Arnoldi steps over all cycles
    mvps: int = 0                        # operator applications per vector
    rel_res: Optional[np.ndarray] = None  # final ||b - A x|| / ||b|| per vector (FP64)
    history: List[float] = field(default_factory=list)   # max relative residual after each outer step
    converged: bool = False               # every vector reached the tolerance
    tol: float = 0.0


class SolveNotConverged(L.MpmcError):
    """A top-level solve ended above its tolerance (its samples would be
    biased); status MPMC_ENOTCONVERGED."""

    def __init__(self, stats: "SolveStats"):
        RuntimeError.__init__(self, f"PP-GMRES did not converge: max relative residual "
                                    f"{float(np.max(stats.rel_res)):.3e} > tolerance {stats.tol:.1e} after "
                                    f"{stats.outer} refinement steps, {stats.cycles} cycles "
                                    f"({L.status_string(L.ENOTCONVERGED)})")
        self.status = L.ENOTCONVERGED
        self.stats = stats


class MixedPPGMRES:
    """x = A^{-1} b for a batch of N vectors.

    lat64    FP64 lattice (outer residual)
    lat_in   lattice of the inner cycles (FP32 for mixed precision, or FP64)
    pin      p_in (single polynomial, its inverse roots) of the preconditioner
    defl_in  eigen-triplets in the inner precision (with H^{-1}), or None
    m        GMRES restart length
    """

    def __init__(self, lat64: L.DeviceLattice, lat_in: L.DeviceLattice, pin: L.DevicePoly,
                 defl_in: Optional[L.DeviceDefl], m: int, nrhs: int, rb: int):
        if pin.inv_out is not None:
            raise ValueError("the preconditioner is a single polynomial")
        self.l64, self.li, self.pin, self.defl = lat64, lat_in, pin, defl_in
        self.m, self.N, self.rb = int(m), int(nrhs), int(rb)
        self.dims, self.V = lat64.dims, lat64.V
        self.pi = lat_in.prec
        self.deg_in = int(pin.inv_in.numel()) - 1
        V, N = self.V, self.N
        ct = L.complex_dtype(self.pi)
        self.basis = torch.empty((self.m + 1, N // rb, 12, V, rb), dtype=ct, device="cuda")
        self.w = L.empty_field(V, N, rb, self.pi)
        self.z = L.empty_field(V, N, rb, self.pi)
        self.t = L.empty_field(V, N, rb, self.pi)
        self.rho = L.empty_field(V, N, rb, self.pi)
        self.delta = L.empty_field(V, N, rb, self.pi)
        self.r64 = L.empty_field(V, N, rb, L.F64)
        self.t64 = L.empty_field(V, N, rb, L.F64)
        self.h = torch.empty((self.m + 1, N), dtype=torch.complex128, device="cuda")
        self.nrm = torch.empty(N, dtype=torch.complex128, device="cuda")
        self.ones = _c(np.ones(N))
        self.minus1 = _c(-np.ones(N))
        ws = [L.field_dot_workspace_size(self.dims, N, rb),
              L.field_block_dot_workspace_size(self.dims, N, rb, self.m + 1),
              L.poly_workspace_size(lat_in, pin, N, rb)]
        if defl_in is not None:
            ws.append(L.deflate_workspace_size(lat_in, defl_in, N, rb))
            self.d = torch.empty((defl_in.k, N), dtype=torch.complex128, device="cuda")
        self.ws = L.workspace(max(ws))

    # -- small helpers -----------------------------------------------------
    def _norms(self, prec, f) -> np.ndarray:
        L.field_dot(self.dims, prec, f, f, self.nrm, self.ws)
        return np.sqrt(np.maximum(self.nrm.cpu().numpy().real, 0.0))

    def _B(self, x, y):
        """y = A p_in(A) x (inner precision)."""
        L.poly_apply(self.li, self.pin, self.N, self.rb, x, None, self.t, None, self.ws)
        L.wilson_apply(self.li, self.t, y)

    # -- one inner solve: A delta ~ rho, rho of unit norm per vector --------
    def _inner(self, tol: float, max_cycles: int, stats: SolveStats):
        dims, pi, N, m = self.dims, self.pi, self.N, self.m
        first = True
        for _ in range(max_cycles):
            # Left-right Projection of the current residual (Sec. 2.1): d = H^{-1} U^H rho,
            # rho <- rho - A V d, delta <- delta + V d
            if self.defl is not None:
                L.deflate_project(self.li, self.defl, L.DEFL_PROJECT, N, self.rb, self.rho, None, None, None,
                                  self.d, self.w, self.ws)
                L.deflate_project(self.li, self.defl, L.DEFL_RECON, N, self.rb, None, None, None, None, self.d,
                                  self.z, self.ws)
                L.field_axpby(dims, pi, self.ones, self.w, None, self.rho)
                L.field_axpby(dims, pi, self.ones, self.z, None if first else self.ones, self.delta)
                stats.mvps += 1
                first = False
            beta = self._norms(pi, self.rho)
            if np.all(beta <= tol):
                break
            # one GMRES(m) cycle on B = A p_in(A) from rho
            safe = np.where(beta > 0, beta, 1.0)
            L.field_axpby(dims, pi, _c(1.0 / safe), self.rho, None, self.basis[0])
            Hs = np.zeros((m + 1, m, N), dtype=np.complex128)
            taken = m
            done = beta <= tol
            for j in range(m):
                self._B(self.basis[j], self.w)
                stats.mvps += self.deg_in + 1
                stats.arnoldi_steps += 1
                hj = np.zeros((j + 1, N), dtype=np.complex128)
                for _ in range(2):       # CGS2
                    L.field_block_dot(dims, pi, self.basis, j + 1, self.w, self.h, self.ws)
                    hc = self.h[: j + 1].cpu().numpy()
                    L.field_block_axpy(dims, pi, self.basis, j + 1, _c(-hc), self.w, True)
                    hj += hc
                hn = self._norms(pi, self.w)
                Hs[: j + 1, j] = hj
                Hs[j + 1, j] = hn
                inv = np.where(hn > 1e-30 * np.maximum(1.0, np.abs(hj).max(axis=0)), 1.0 / np.maximum(hn, 1e-300), 0.0)
                L.field_axpby(dims, pi, _c(inv), self.w, None, self.basis[j + 1])
                # per-vector least-squares residual of this cycle
                res = np.array([self._ls(Hs[: j + 2, : j + 1, r], beta[r])[1] for r in range(N)])
                if np.all(done | (res <= tol)):
                    taken = j + 1
                    break
            stats.cycles += 1
            Y = np.zeros((taken, N), dtype=np.complex128)
            for r in range(N):
                if beta[r] > 0:
                    Y[:, r] = self._ls(Hs[: taken + 1, :taken, r], beta[r])[0]
            # delta += p_in(A) sum_i y_i v_i ;  rho -= A p_in(A) sum_i y_i v_i
            L.field_block_axpy(dims, pi, self.basis, taken, _c(Y), self.z, False)
            L.poly_apply(self.li, self.pin, N, self.rb, self.z, None, self.t, None, self.ws)
            L.wilson_apply(self.li, self.t, self.w)
            stats.mvps += self.deg_in + 1
            L.field_axpby(dims, pi, self.ones, self.t, None if first else self.ones, self.delta)
            first = False
            L.field_axpby(dims, pi, self.minus1, self.w, self.ones, self.rho)
        if first:   # nothing was added: delta = 0
            L.field_axpby(dims, pi, _c(np.zeros(N)), self.rho, None, self.delta)

    @staticmethod
    def _ls(Hbar: np.ndarray, beta: float):
        """min_y || beta e_1 - Hbar y || (FP64, small)."""
        rhs = np.zeros(Hbar.shape[0], dtype=np.complex128)
        rhs[0] = beta
        y, *_ = np.linalg.lstsq(Hbar, rhs, rcond=None)
        return y, float(np.linalg.norm(rhs - Hbar @ y))

    # -- the refinement loop ----------------------------------------------
    def solve(self, b64: torch.Tensor, x64: torch.Tensor, tol: float = 1e-6, inner_tol: float = 1e-4,
              max_outer: int = 10, max_cycles: int = 20) -> SolveStats:
        """x64 = A^{-1} b64 to ||b - A x|| <= tol ||b|| per vector (FP64 fields
        of the batch shape).  x64 is overwritten."""
        dims, N = self.dims, self.N
        stats = SolveStats()
        bn = self._norms(L.F64, b64)
        bn = np.where(bn > 0, bn, 1.0)
        L.field_axpby(dims, L.F64, self.ones, b64, None, self.r64)          # r = b, x = 0
        have_x = False
        for _ in range(max_outer):
            rn = self._norms(L.F64, self.r64)
            rel = rn / bn
            if have_x:
                stats.history.append(float(rel.max()))
            if np.all(rel <= tol):
                break
            stats.outer += 1
            # FP32 inner solve of A delta = r / ||r||, only as far as this step needs:
            # the outer residual must fall from rel to tol
            safe = np.where(rn > 0, rn, 1.0)
            L.field_axpby_mixed(dims, _c(1.0 / safe), self.r64, None, self.rho)
            self._inner(max(inner_tol, 0.5 * tol / float(rel.max())), max_cycles, stats)
            # x += ||r|| delta ; r = b - A x   (FP64)
            L.field_axpby_mixed(dims, _c(rn), self.delta, self.ones if have_x else None, x64)
            have_x = True
            L.wilson_apply(self.l64, x64, self.t64)
            stats.mvps += 1
            L.field_axpby(dims, L.F64, self.ones, b64, None, self.r64)
            L.field_axpby(dims, L.F64, self.minus1, self.t64, self.ones, self.r64)
        if not have_x:
            L.field_axpby(dims, L.F64, _c(np.zeros(N)), b64, None, x64)
        stats.rel_res = self._norms(L.F64, self.r64) / bn
        stats.tol = float(tol)
        stats.converged = bool(np.all(stats.rel_res <= tol))
        return stats
