"""Failure handling on the device path: a non-finite link is counted in the
level accumulator instead of crashing, an exact Krylov breakdown (kappa = 0,
A = I) ends the polynomial at its exact degree, and a top-level solve that
misses its tolerance is reported rather than sampled."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev_c128, device_lattice, lib, pack, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("sweep", [0, 1])
def test_nonfinite_link_is_counted(sweep):
    L = lib()
    dims, N = (8, 8, 8, 4), 32
    dl, ol = device_lattice(dims, 0.14, 0.4, 41, True)
    dl.gauge[5] = float("nan")                     # one link element of one site
    poly = L.DevicePoly(dev_c128(np.array([0.6, 0.5 + 0.1j, 0.4, 0.3j, 0.2])))
    lvl = L.DeviceLevel(L.OP_POLY, poly)
    L.set_option(L.OPT_PLANE_SWEEP, sweep)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lvl, N, 16))
    L.mlmc_level_estimate(dl, lvl, N, 16, L.Noise(1, 1, 0, 0), samples, acc, ws)
    torch.cuda.synchronize()
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    a = acc.cpu().numpy()
    assert a[0] == N and a[4] == N                 # every sample sees the NaN within 4 hops
    assert not np.isfinite(a[1])                   # the mean carries it: the flag is sticky


def test_exact_breakdown_gives_the_exact_polynomial():
    """kappa = 0: A = I, the Krylov space of any start vector has dimension 1,
    GMRES stops after one step with the exact inverse p(A) = I."""
    L = lib()
    from paper_2306_09559_amd import krylov
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.0, 0.4, 41, True)
    rs = krylov.gmres_roots(dl, [1, 5], synth.gaussian_start(ol.n, 2))
    for d in (1, 5):
        assert len(rs.inv_roots[d]) == 1 and abs(rs.inv_roots[d][0] - 1.0) < 1e-12
        assert rs.residual[d] < 1e-12
    N = 16
    lvl = L.DeviceLevel(L.OP_POLY, rs.device[5])
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lvl, N, 16))
    L.mlmc_level_estimate(dl, lvl, N, 16, L.Noise(1, 1, 0, 0), samples, acc, ws)
    torch.cuda.synchronize()
    S = samples.cpu().numpy()
    assert np.allclose(S[:, 0], 12 * dl.V, rtol=1e-14) and np.allclose(S[:, 1], 0, atol=1e-9)   # b^H b


def test_unconverged_top_level_solve_is_reported():
    L = lib()
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.solve import SolveNotConverged
    from synth.configs import C1, Level, SOLVE
    cfg = dataclasses.replace(C1, name="C1S", levels=(Level(SOLVE, (4, 3), 16, deflated=False),), k_defl=0)
    run = driver.build(cfg, prec=L.F32, rb=16)
    lv = run.levels[0]
    # one FP64 refinement step around an FP32 inner solve cannot reach 1e-12
    L.z4_fill(cfg.dims, L.F64, run.noise(0), lv.b64)
    st = lv.solver.solve(lv.b64, lv.x64, tol=1e-12, max_outer=1, max_cycles=1)
    assert not st.converged and np.max(st.rel_res) > 1e-12
    lv.solve_tol = 1e-30                           # unreachable: the draw must refuse to sample
    with pytest.raises(SolveNotConverged):
        run.draw(0, 16)
    assert lv.drawn == 0 and lv.acc.cpu().numpy()[0] == 0
