"""Oracle estimators (FP64, numpy): test infrastructure only.

* Hutchinson samples b^* M b with Z4 noise (Sec. 1).  With E[b b^*] = I and
  E[b b^T] = 0 the expectation is Tr(M) (the conjugate transpose is meant).
* Level samples of the multilevel formula (eq. multpolytr, Sec. 3.1) with
  the deflation of Sec. 4.1:
      s = b^* P_hi b - b^* P_lo b - sum_i c_i conj(zeta_i) omega_i,
      zeta = V^* b, omega = U^* b,
  level estimate mean(s) + sum_i c_i u_i^* z_i.
* Standard error S / sqrt(N) with the (N-1) sample variance of the complex
  samples.
* Stopping tolerances and check cadence of the algorithm in Sec. 5, step 3.
* The multilevel cost formula of Sec. 5 (eq. mlevcost).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


def level_samples(hi: np.ndarray, lo: Optional[np.ndarray], zeta: Optional[np.ndarray] = None,
                  omega: Optional[np.ndarray] = None, c: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-sample values.  hi, lo: (N,) b^* P b values; zeta, omega: (k, N);
    c: (k,)."""
    s = np.asarray(hi, dtype=np.complex128).copy()
    if lo is not None:
        s = s - np.asarray(lo, dtype=np.complex128)
    if c is not None and len(c):
        s = s - np.einsum("i,ir,ir->r", np.asarray(c), np.conj(zeta), omega)
    return s


@dataclass
class LevelEstimate:
    n: int
    mean: complex
    var: float            # (N-1) sample variance of the complex samples
    stderr: float
    estimate: complex     # mean + deflation correction


def level_estimate(samples: np.ndarray, c: Optional[np.ndarray] = None,
                   uz: Optional[np.ndarray] = None) -> LevelEstimate:
    s = np.asarray(samples, dtype=np.complex128)
    n = len(s)
    mean = complex(s.mean())
    var = float(np.sum(np.abs(s - mean) ** 2) / (n - 1)) if n > 1 else float("nan")
    corr = 0.0
    if c is not None and len(c):
        corr = complex(np.sum(np.asarray(c) * (np.ones(len(c)) if uz is None else np.asarray(uz))))
    return LevelEstimate(n, mean, var, float(np.sqrt(var / n)) if n > 1 else float("nan"), mean + corr)


def z4_variance(M: np.ndarray) -> float:
    """Var(b^* M b) for Z4 noise: ||M||_F^2 - sum_i |M_ii|^2.

    Derivation: b^* M b - Tr M = sum_{i != j} conj(b_i) M_ij b_j; the terms
    are uncorrelated with E|conj(b_i) b_j|^2 = 1 and, for Z4, E[conj(b_i) b_j
    conj(conj(b_k) b_l)] = 0 unless (k,l) = (i,j) (the (k,l) = (j,i) term
    averages conj(b_i)^2 b_j^2, whose expectation is 0 for Z4)."""
    d = np.diagonal(M)
    return float(np.sum(np.abs(M) ** 2) - np.sum(np.abs(d) ** 2))


def cost_formula(variances: Sequence[float], costs: Sequence[float], eps: float) -> float:
    """C = eps^-2 (sum_l sqrt(V_l C_l))^2 (eq. mlevcost of Sec. 5)."""
    return float(sum(np.sqrt(v * c) for v, c in zip(variances, costs)) ** 2 / eps ** 2)


def hutchinson_cost(variance: float, cost: float, eps: float) -> float:
    """C = eps^-2 V_0 C_0."""
    return float(variance * cost / eps ** 2)


def epsilon_for_volume(V: int) -> float:
    """eps = 0.0005 * V, V the number of lattice sites (Sec. 5, Example 2)."""
    return 0.0005 * V


def level_tolerances(eps: float, currerr: Sequence[float]):
    """Standard-error targets of the three Monte Carlo steps of Sec. 5 step 3:
    eps/sqrt(3); then sqrt(eps^2 - e^2)/sqrt(2); then sqrt(eps^2 - e^2), with
    e the combined standard error so far (square root of the sum of squares)."""
    t1 = eps / np.sqrt(3.0)
    e1 = float(np.sqrt(np.sum(np.square(currerr[:1])))) if len(currerr) >= 1 else 0.0
    t2 = np.sqrt(max(eps ** 2 - e1 ** 2, 0.0)) / np.sqrt(2.0)
    e2 = float(np.sqrt(np.sum(np.square(currerr[:2])))) if len(currerr) >= 2 else e1
    t3 = np.sqrt(max(eps ** 2 - e2 ** 2, 0.0))
    return t1, t2, t3


def check_points(level: int, nmax: int):
    """Sample counts at which the standard error is checked (Sec. 5 step 3):
    level 1 from 2 noises on, after every noise; level 2 at 3 then every 3;
    level 3 at 6 then every 3."""
    if level == 1:
        return list(range(2, nmax + 1))
    if level == 2:
        return list(range(3, nmax + 1, 3))
    return list(range(6, nmax + 1, 3))
