"""Derive the hopping parameter of the 8^4 workload (eps = 0.3 links, seed
201) so that the eigenvalue of A = I - kappa*D nearest the origin has
modulus 1e-3, as that workload asks.

D = (I - A)/kappa is kappa-independent.  For an eigenvalue mu = a + ib of D
the eigenvalue of A is 1 - kappa*mu; the critical mode is the eigenvalue of
D with the largest real part.  |1 - kappa mu| = t has a real solution iff
|b| <= t |mu|; the smaller root kappa = (a - sqrt(t^2 |mu|^2 - b^2)) / |mu|^2
keeps the rest of the spectrum on the right of the origin.  With an
antiperiodic time direction these links have |b| ~ 0.7 at the edge (no
solution); with a periodic one the edge pair has |b|/|mu| ~ 6e-4, so the
workload uses periodic time.  Calls only the oracle.

usage: python tests/golden/tune_kappa.py   (writes tests/golden/c2_kappa.txt)
"""
import os
import sys

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402
from synth.configs import C2  # noqa: E402


def main():
    U = synth.gauge_links(C2.dims, C2.eps, C2.seed_links)
    k0 = 0.1
    lat = oracle.Lattice(C2.dims, k0, U, False)
    D = LinearOperator((lat.n, lat.n), matvec=lambda x: (x - lat.apply(x)) / k0, dtype=np.complex128)
    mu = eigs(D, k=16, which="LR", ncv=96, tol=1e-12, maxiter=20000, return_eigenvectors=False)
    mu = mu[np.argsort(-mu.real)]
    top = mu[0]
    target = 1e-3
    disc = target ** 2 * abs(top) ** 2 - top.imag ** 2
    if disc >= 0:
        kappa = (top.real - np.sqrt(disc)) / abs(top) ** 2
    else:
        kappa = top.real / abs(top) ** 2
    lam = 1.0 - kappa * mu
    lines = [f"# largest-real-part eigenvalues of D (8^4, eps=0.3, seed {C2.seed_links}, periodic t)"]
    lines += [f"# mu = {m.real:.15f} {m.imag:+.3e}i" for m in mu]
    lines += [f"# min |1 - kappa mu| over these = {np.min(np.abs(lam)):.6e}", repr(float(kappa))]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_kappa.txt")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
