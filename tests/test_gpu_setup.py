"""The product's GPU set-up (Sec. 5 setup step 2): GMRES roots and
PP-Arnoldi deflation triplets, checked against the oracle's independent set-up
from the same start vector and against identities the set-up must satisfy."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import deflation, dense, krylov as okr

from gpu_helpers import device_lattice, lib, pack, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _matched(a, b):
    """max distance between two root sets matched greedily (nearest first)."""
    b = list(b)
    worst = 0.0
    for z in sorted(a, key=lambda z: -abs(z)):
        j = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b[j]))
        b.pop(j)
    return worst


def test_gmres_roots_c1():
    from paper_2306_09559_amd import krylov
    from synth.configs import C1
    L = lib()
    dl, ol = device_lattice(C1.dims, C1.kappa, C1.eps, C1.seed_links, True)
    start = synth.gaussian_start(ol.n, C1.seed_start)
    rs = krylov.gmres_roots(dl, [5, 20], start)
    ps = okr.gmres_polys(ol.apply, start, [5, 20])
    for d in (5, 20):
        th_gpu, th_ora = 1.0 / rs.inv_roots[d], ps.roots[d]
        assert _matched(th_gpu, th_ora) < 1e-8 * np.max(np.abs(th_ora))
        # the Newton polynomial of the GPU roots reproduces the GPU GMRES residual
        x = pack(C1.dims, start.reshape(1, -1), 1, 0)
        y = torch.empty_like(x)
        ws = L.workspace(L.poly_workspace_size(dl, rs.device[d], 1, 1))
        L.poly_apply(dl, rs.device[d], 1, 1, x, None, y, None, ws)
        Ay = torch.empty_like(y)
        L.wilson_apply(dl, y, Ay)
        r = start - unpack(C1.dims, Ay, 0)[0]
        assert np.linalg.norm(r) / np.linalg.norm(start) == pytest.approx(rs.residual[d], rel=1e-6)


def test_pp_arnoldi_deflation_small():
    from paper_2306_09559_amd import krylov
    dims = (2, 2, 2, 4)
    dl, ol = device_lattice(dims, 0.16, 0.5, 21, True)
    start = synth.gaussian_start(ol.n, 3)
    rs = krylov.gmres_roots(dl, [6], start)
    df = krylov.pp_arnoldi_deflation(dl, rs.device[6], start, 60, 16, 8)
    ev = np.linalg.eigvals(dense.dense_matrix(ol))
    k = df.device.k
    assert k >= 4
    for l in df.lam:
        assert np.min(np.abs(ev - l)) < 1e-6
    assert np.all(df.res_right < 1e-3) and np.all(df.res_left < 1e-3)
    # biorthonormal left vectors: u_i^H z_i = 1 and H = U^H A V ~ diag(lambda)
    H = np.linalg.inv(df.device.hinv.cpu().numpy())
    assert np.allclose(np.diag(H), df.lam, atol=1e-6)
    assert np.max(np.abs(H - np.diag(np.diag(H)))) < 1e-5
