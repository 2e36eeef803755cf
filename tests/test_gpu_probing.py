"""Exact lowest level by probing on the GPU (Sec. 5 step 3d): probe vectors
bit-exact, the probing trace against the oracle's (its own colouring), and on
the 8^4 workload against a Hutchinson estimate of the same trace."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import krylov, probing as oprobe
from gpu_helpers import dev_c128, device_lattice, lib, unpack

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_probe_fill_exact():
    L = lib()
    dims, nrhs, rb = (4, 2, 2, 3), 40, 8
    V = int(np.prod(dims))
    rng = np.random.default_rng(1)
    col = rng.integers(0, 5, V).astype(np.int32)
    f = L.empty_field(V, nrhs, rb, 0)
    L.probe_fill(dims, 0, torch.from_numpy(col).cuda(), 17, f)
    got = unpack(dims, f, 0).reshape(nrhs, V, 12)
    for r in range(nrhs):
        p = 17 + r
        want = np.zeros((V, 12))
        want[col == p // 12, p % 12] = 1.0
        assert np.array_equal(got[r], want)


@pytest.mark.parametrize("prec,rb,in_kernel", [(0, 16, False), (1, 16, False), (0, 1, False), (1, 1, False),
                                               (0, 1, True), (1, 1, True)])
def test_probe_trace_matches_oracle(prec, rb, in_kernel):
    L = lib()
    from paper_2306_09559_amd import probing
    dims, deg = (4, 4, 4, 4), 3
    dl, ol = device_lattice(dims, 0.14, 0.5, 21, True, prec)
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 2), [deg]).inv_roots[deg]
    res = probing.probe_trace(dl, L.DevicePoly(dev_c128(t)), probing.colouring(dims, deg), nrhs=64, rb=rb,
                              in_kernel=in_kernel)
    want = oprobe.probe_trace(ol, t, oprobe.distance_colouring(dims, deg))
    tol = 1e-12 if prec == 0 else 8 * deg * 10 * U32
    assert abs(res.trace - want) <= tol * abs(want), (res.trace, want)


def test_probing_agrees_with_hutchinson_on_the_8x4_workload():
    """Tr p_8(A) of the 8^4 workload: exact by probing (1024 colours) and the
    Hutchinson mean of 2048 Z4 samples agree within 5 standard errors."""
    L = lib()
    from paper_2306_09559_amd import driver, probing
    from synth.configs import C2
    run = driver.build(C2, prec=L.F64, rb=16)
    li = len(run.levels) - 1
    run.reset()
    for _ in range(8):
        run.draw(li, 256)
    e = run.estimates()[li]
    res = probing.probe_trace(run.dl, run.levels[li].device.poly_hi, probing.colouring(C2.dims, 8))
    # probes written as a field (block width 16) instead of generated in the sweep: the same trace
    res16 = probing.probe_trace(run.dl, run.levels[li].device.poly_hi, probing.colouring(C2.dims, 8), rb=16,
                                in_kernel=False)
    assert abs(res16.trace - res.trace) <= 1e-14 * abs(res.trace)
    print(f"probing {res.trace:.6f} ({res.ncolours} colours); Hutchinson {e['estimate']:.3f} +- {e['stderr']:.3f}")
    assert abs(res.trace - e["estimate"]) <= 5 * e["stderr"] * np.sqrt(2)


@pytest.mark.parametrize("prec", [0, 1])
def test_probes_in_kernel_equal_filled_probes(prec):
    """Probe vectors generated inside the t-sweep give the trace of the same
    probes written by mpmc_probe_fill and read as a field."""
    L = lib()
    from paper_2306_09559_amd import probing
    dims, deg = (8, 8, 8, 4), 3
    dl, ol = device_lattice(dims, 0.14, 0.5, 23, True, prec)
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 3), [deg]).inv_roots[deg]
    poly = L.DevicePoly(dev_c128(t))
    col = probing.colouring(dims, deg)
    # the filled probes on the same kernel (at 64 vectors the automatic choice streams them)
    L.set_option(L.OPT_PLANE_SWEEP, L.SWEEP_ALWAYS)
    try:
        a = probing.probe_trace(dl, poly, col, nrhs=64, in_kernel=True)
        b = probing.probe_trace(dl, poly, col, nrhs=64, in_kernel=False)
    finally:
        L.set_option(L.OPT_PLANE_SWEEP, L.SWEEP_AUTO)
    print(f"prec {prec}: in kernel {a.trace}, filled {b.trace}, equal {a.trace == b.trace}")
    assert abs(a.trace - b.trace) <= 1e-14 * abs(b.trace)
    if prec == 0:
        want = oprobe.probe_trace(ol, t, oprobe.distance_colouring(dims, deg))
        assert abs(a.trace - want) <= 1e-12 * abs(want)


def test_probe_noise_is_rejected_elsewhere():
    """Only the scalar t-sweep of mpmc_poly_apply takes probe vectors."""
    L = lib()
    from paper_2306_09559_amd import probing
    dims = (8, 8, 8, 4)
    dl, ol = device_lattice(dims, 0.14, 0.5, 23, True, 0)
    col = torch.from_numpy(probing.colouring(dims, 2)).cuda()
    nz = L.Noise(0, 0, 0, 0, probe_colour=col)
    f = L.empty_field(dl.V, 16, 16, 0)
    with pytest.raises(L.MpmcError, match="status -2"):
        L.z4_fill(dims, 0, nz, f)
    poly = L.DevicePoly(dev_c128(np.array([0.5, 0.4, 0.3], complex)))
    ws = L.workspace(L.poly_workspace_size(dl, poly, 16, 16))
    with pytest.raises(L.MpmcError, match="status -2"):      # vector mode
        L.poly_apply(dl, poly, 16, 16, None, nz, L.empty_field(dl.V, 16, 16, 0), None, ws)
    comp = L.DevicePoly(dev_c128(np.array([0.5, 0.4], complex)), dev_c128(np.array([0.7, 0.6], complex)))
    wsc = L.workspace(L.poly_workspace_size(dl, comp, 16, 16))
    with pytest.raises(L.MpmcError, match="status -2"):      # double polynomial
        L.poly_apply(dl, comp, 16, 16, None, nz, None, torch.empty(16, dtype=torch.complex128, device="cuda"), wsc)
    lvl = L.DeviceLevel(L.OP_POLY, poly, L.OP_NONE, None)
    wsl = L.workspace(L.level_workspace_size(dl, lvl, 16, 16))
    with pytest.raises(L.MpmcError, match="status -2"):
        L.mlmc_level_estimate(dl, lvl, 16, 16, nz, torch.empty((16, 6), dtype=torch.float64, device="cuda"),
                              torch.zeros(8, dtype=torch.float64, device="cuda"), wsl)
