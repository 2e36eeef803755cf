"""Mixed precision (FP32 fields, links, eigenvectors and vector updates; FP64
roots, dots, samples and accumulators) against the FP64 oracle on the 4^4
two-level workload: every sample constituent within 8 * d * kappa_N * u32,
and each level mean within 0.1 of its FP64 standard error."""
import numpy as np
import pytest
import torch

import oracle
from oracle import estimator

from gpu_helpers import build_from_oracle_set_up, oracle_set_up

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_mixed_levels_c1(tmp_path):
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    from synth.configs import C1
    # both runs on the oracle's own GMRES roots, resumed into the FP64 run and taken over by the FP32 one
    su = oracle_set_up(C1, [lv.hi for lv in C1.levels])
    run64 = build_from_oracle_set_up(C1, su, tmp_path / "c1_oracle_setup.npz", prec=L.F64, rb=4)
    run32 = driver.build(C1, prec=L.F32, rb=4, reuse=run64)
    ol = su.ol
    for run in (run64, run32):
        run.reset()
        run.step()
    torch.cuda.synchronize()
    e64, e32 = run64.estimates(), run32.estimates()
    for lvl, lv in enumerate(C1.levels):
        S = run32.levels[lvl].samples.cpu().numpy()
        hi = S[:, 2] + 1j * S[:, 3]
        B = oracle.z4(C1.seed_noise, C1.lattice_id, lvl, 0, lv.samples, ol.V)
        t = su.ps.inv_roots[lv.hi]
        _, rh = ol.poly_apply(t, B)
        # amplification of rounding through the Newton recurrence
        kN = 1.0
        for b in B[:4]:
            w = b.copy()
            for tj in t[:-1]:
                w = w - tj * ol.apply(w)
                kN = max(kN, np.linalg.norm(w) / np.linalg.norm(b))
        bound = 8 * lv.hi * kN * U32
        assert np.max(np.abs(hi - rh) / np.abs(rh)) < bound
        assert abs(e32[lvl]["estimate"] - e64[lvl]["estimate"]) < 0.1 * e64[lvl]["stderr"]


def test_mixed_levels_c2_within_target():
    """The 8^4 three-level workload: with the same noise, each mixed level
    mean is within 0.1 of that level's standard-error target (eps = 0.0005 V
    split over the levels as in Sec. 5), the FP64 GPU run as reference."""
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    from synth.configs import C2
    run64 = driver.build(C2, prec=L.F64, rb=16)
    run32 = driver.build(C2, prec=L.F32, rb=16, reuse=run64)
    for run in (run64, run32):
        run.reset()
        run.step()
        run.step()
    torch.cuda.synchronize()
    e64, e32 = run64.estimates(), run32.estimates()
    eps = estimator.epsilon_for_volume(int(np.prod(C2.dims)))
    targets = estimator.level_tolerances(eps, [e["stderr"] for e in e64])
    for lvl in range(len(C2.levels)):
        err = abs(e32[lvl]["estimate"] - e64[lvl]["estimate"])
        print(f"level {lvl}: |T32 - T64| = {err:.3g}, target {targets[lvl]:.3g}, stderr {e64[lvl]['stderr']:.3g}")
        assert err <= 0.1 * targets[lvl]
