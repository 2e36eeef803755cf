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


@pytest.mark.parametrize("dims,prec,nrhs,rb", [
    ((8, 8, 8, 8), 0, 64, 16),      # FP64 whole-plane t-sweep
    ((8, 8, 8, 8), 1, 64, 16),      # FP32 whole-plane t-sweep (own backward products)
    ((16, 16, 16, 2), 1, 32, 4),    # FP32 blocks with a halo
])
def test_kappa_zero_polynomial_is_p_of_one(dims, prec, nrhs, rb):
    """kappa = 0 gives A = I, so b^H p(A) b = p(1) b^H b = 12 V p(1) for every
    Z4 sample, with p(1) from the scalar Newton form of the oracle.  A 5-root
    polynomial runs 4 Newton steps on the t-sweep (every kappa t_j is 0) and
    on the streaming kernel; vector mode gives y = p(1) b."""
    from oracle import deflation
    L = lib()
    dl, ol = device_lattice(dims, 0.0, 0.4, 43, True, prec=prec)
    assert L.sweep_plan(dl, nrhs, rb)["ok"] and L.sweep_plan(dl, nrhs, 1)["ok"]
    t = np.array([0.6, 0.5 + 0.1j, 0.4, 0.3j, 0.2])
    p1 = complex(deflation.poly_eval(t, 1.0))
    poly = L.DevicePoly(dev_c128(t))
    want = 12 * dl.V * p1
    # amplification of the recurrence: max_j |prod_{i<j} (1 - t_i)|
    kN = max(1.0, max(abs(np.prod(1.0 - t[:j])) for j in range(1, len(t))))
    tol = 1e-13 if prec == 0 else 8 * len(t) * kN * 2.0 ** -24
    nz = L.Noise(3, 1, 0, 0)
    for sweep in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, sweep)
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
        ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
        L.poly_apply(dl, poly, nrhs, rb, None, nz, None, bhy, ws)
        y = L.empty_field(dl.V, nrhs, 1, prec)
        ws1 = L.workspace(L.poly_workspace_size(dl, poly, nrhs, 1))
        L.poly_apply(dl, poly, nrhs, 1, None, nz, y, None, ws1)
        torch.cuda.synchronize()
        got = bhy.cpu().numpy()
        assert np.all(np.isfinite(got)), sweep
        assert np.max(np.abs(got - want)) <= tol * abs(want), (sweep, got[:3], want)
        Y = unpack(dims, y, prec)
        B = oracle.z4(3, 1, 0, 0, nrhs, dl.V)
        for r in (0, nrhs - 1):
            assert np.max(np.abs(Y[r] - p1 * B[r])) <= tol * abs(p1), (sweep, r)
    L.set_option(L.OPT_PLANE_SWEEP, 1)


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_inverse_root_on_the_sweep(prec):
    """An inverse root t_j = 0 makes kappa t_j = 0 with kappa != 0: that Newton
    step is w_{j+1} = w_j.  The t-sweep agrees with the oracle (and with the
    streaming kernel) on the 8^4 lattice."""
    L = lib()
    dims, nrhs, rb = (8, 8, 8, 8), 32, 16
    dl, ol = device_lattice(dims, 0.12, 0.4, 44, True, prec=prec)
    t = np.array([0.9, 0.0, 0.7 + 0.2j, 0.0, 0.5 - 0.1j, 0.8])
    poly = L.DevicePoly(dev_c128(t))
    B = oracle.z4(9, 2, 0, 0, nrhs, dl.V)
    _, ref = ol.poly_apply(t, B)
    tol = 1e-12 if prec == 0 else 8 * len(t) * 4 * 2.0 ** -24
    out = {}
    for sweep in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, sweep)
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
        ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
        L.poly_apply(dl, poly, nrhs, rb, None, L.Noise(9, 2, 0, 0), None, bhy, ws)
        torch.cuda.synchronize()
        out[sweep] = bhy.cpu().numpy()
        assert np.max(np.abs(out[sweep] - ref) / np.abs(ref)) < tol, sweep
    L.set_option(L.OPT_PLANE_SWEEP, 1)
