"""The level entry point that allocates nothing (static device scratch)
against the allocating one, through the C ABI: two calls in a row, the
second with a smaller batch, give the same samples and accumulators bit for
bit (same kernels, same order of sums); a level too large for the scratch
is refused before anything runs."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import dev_c128, device_lattice, lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _levels(L, ol, dl):
    """A deflated polynomial-difference level and a deflated-operator level.
    The two entry points run the same kernels, so any well-conditioned
    triplets serve: orthonormal random vectors, g5-rule left vectors with
    their biorthonormal scale, H = U^H A V from the oracle operator."""
    from oracle import deflation, krylov
    from gpu_helpers import device_defl
    ps = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 3), [12, 4])
    k = 6
    Q, _ = np.linalg.qr(synth.random_fields(k, ol.V, 9).reshape(k, -1).T)
    Z = np.ascontiguousarray(Q.T)
    pair = np.arange(k)
    U = deflation.left_vectors(Z, pair, ol.gamma5)
    H = deflation.projection_matrix(ol.apply, Z, U)
    D = device_defl(dl.dims, Z, pair, U, H, prec=dl.prec)
    hi, lo = L.DevicePoly(dev_c128(ps.inv_roots[12])), L.DevicePoly(dev_c128(ps.inv_roots[4]))
    c = np.linspace(0.5, 1.5, k) + 0.25j
    return [L.DeviceLevel(L.OP_POLY, hi, L.OP_POLY, lo, D, True, dev_c128(c)),
            L.DeviceLevel(L.OP_DEFLATED_POLY, hi, L.OP_POLY, lo, D, False)]


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_allocating_entry_point(prec):
    L = lib()
    dims = (4, 4, 4, 8)
    dl, ol = device_lattice(dims, 0.15, 0.5, 61, True, prec=prec)
    for lvl in _levels(L, ol, dl):
        acc_a = torch.zeros(8, dtype=torch.float64, device="cuda")
        acc_b = torch.zeros(8, dtype=torch.float64, device="cuda")
        for call, (nrhs, rb) in enumerate(((48, 16), (16, 4))):      # the second call is smaller
            assert L.level_workspace_size(dl, lvl, nrhs, rb) <= L.noalloc_scratch_bytes()
            nz = L.Noise(71, 5, 2, 1000 * call)
            sa = torch.full((nrhs, 6), float("nan"), dtype=torch.float64, device="cuda")
            sb = torch.full((nrhs, 6), float("nan"), dtype=torch.float64, device="cuda")
            ws = L.workspace(L.level_workspace_size(dl, lvl, nrhs, rb))
            L.mlmc_level_estimate(dl, lvl, nrhs, rb, nz, sa, acc_a, ws)
            L.mlmc_level_estimate_noalloc(dl, lvl, nrhs, rb, nz, sb, acc_b)
            torch.cuda.synchronize()
            a, b = sa.cpu().numpy(), sb.cpu().numpy()
            assert np.all(np.isfinite(a)), call
            assert np.array_equal(a, b), (call, np.max(np.abs(a - b)))
            assert np.array_equal(acc_a.cpu().numpy(), acc_b.cpu().numpy()), call


def test_noalloc_refuses_levels_beyond_the_scratch():
    L = lib()
    dims = (8, 8, 8, 8)
    dl, ol = device_lattice(dims, 0.13, 0.3, 62, False)
    lvl = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(np.array([0.9, 0.8, 0.7]))))
    nrhs = 256
    assert L.level_workspace_size(dl, lvl, nrhs, 16) > L.noalloc_scratch_bytes()
    s = torch.zeros((nrhs, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(L.MpmcError) as e:
        L.mlmc_level_estimate_noalloc(dl, lvl, nrhs, 16, L.Noise(1, 1, 1, 0), s, acc)
    assert e.value.status == L.EWORKSPACE
    torch.cuda.synchronize()
    assert not acc.any()
