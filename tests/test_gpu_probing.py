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


@pytest.mark.parametrize("prec,rb", [(0, 16), (1, 16), (0, 1), (1, 1)])
def test_probe_trace_matches_oracle(prec, rb):
    L = lib()
    from paper_2306_09559_amd import probing
    dims, deg = (4, 4, 4, 4), 3
    dl, ol = device_lattice(dims, 0.14, 0.5, 21, True, prec)
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 2), [deg]).inv_roots[deg]
    res = probing.probe_trace(dl, L.DevicePoly(dev_c128(t)), probing.colouring(dims, deg), nrhs=64, rb=rb)
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
    # the probe batch layout changes only the speed: the sweep sums sites in a fixed order
    res16 = probing.probe_trace(run.dl, run.levels[li].device.poly_hi, probing.colouring(C2.dims, 8), rb=16)
    assert res16.trace == res.trace
    print(f"probing {res.trace:.6f} ({res.ncolours} colours); Hutchinson {e['estimate']:.3f} +- {e['stderr']:.3f}")
    assert abs(res.trace - e["estimate"]) <= 5 * e["stderr"] * np.sqrt(2)
