"""The deflation variance profile of a GPU workload: one batch of a deflated
level's samples with the first k deflation terms subtracted; at full k it
must reproduce the level's own deflated samples (the same noise, the level
kernel vs the projection kernel)."""
import numpy as np
import pytest
import torch

from gpu_helpers import lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", [0, 1])
def test_level_variance_profile_c2(prec):
    L = lib()
    from paper_2306_09559_amd import diagnostics, driver
    from synth.configs import C2
    run = driver.build(C2, prec=prec, rb=16)
    for li in (0, 1):
        p = diagnostics.level_variance_profile(run, li, 256)
        print(f"prec {prec} level {li}: variance k=0 {p.variance[0]:.4g} -> k={p.k[-1]} {p.variance[-1]:.4g}, "
              f"reproduction {p.reproduction_error:.1e}")
        assert p.reproduction_error < (1e-12 if prec == 0 else 1e-6)
        assert np.all(np.isfinite(p.variance)) and len(p.variance) == run.defl.device.k + 1
        assert p.variance[-1] < p.variance[0]
