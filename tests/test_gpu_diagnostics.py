"""The deflation variance profile of a GPU workload (the diagnostic behind
Sec. 4.1's deflation count): one batch of a deflated level's samples with the
first k deflation terms subtracted, for every k.  The 8^4 workload runs on the
oracle's own set-up (its GMRES roots and accepted eigen-triplets resumed into
the product's run): at full k the profile must reproduce the level's own
deflated samples (the level kernel against the projection kernel), and on
the first 16 samples of the top level every variance must equal the oracle's,
whose samples come from its own polynomial applications and coefficients."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import build_from_oracle_set_up, lib, oracle_set_up

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", [0, 1])
def test_level_variance_profile_c2(prec, tmp_path):
    L = lib()
    from oracle import deflation, estimator
    from paper_2306_09559_amd import diagnostics
    from synth.configs import C2
    su = oracle_set_up(C2, [150, 30, 8], pin_degree=30)
    run = build_from_oracle_set_up(C2, su, tmp_path / "c2_oracle_setup.npz", prec=prec, rb=16)
    for li in (0, 1):
        p = diagnostics.level_variance_profile(run, li, 256)
        print(f"prec {prec} level {li}: variance k=0 {p.variance[0]:.4g} -> k={p.k[-1]} {p.variance[-1]:.4g}, "
              f"reproduction {p.reproduction_error:.1e}")
        assert p.reproduction_error < (1e-12 if prec == 0 else 1e-6)
        assert np.all(np.isfinite(p.variance)) and len(p.variance) == run.defl.device.k + 1
        assert p.variance[-1] < p.variance[0]
    if prec != 0:
        return
    # the oracle's profile of the first 16 samples of the top level, Tr(p150 - p30)
    n, ol, tri = 16, su.ol, su.tri
    p = diagnostics.level_variance_profile(run, 0, n)
    t150, t30 = su.ps.inv_roots[150], su.ps.inv_roots[30]
    B = oracle.z4(C2.seed_noise, C2.lattice_id, run.levels[0].index, 0, n, ol.V)
    _, hi = ol.poly_apply(t150, B)
    _, lo = ol.poly_apply(t30, B)
    c = deflation.poly_eval(t150, tri.lam) - deflation.poly_eval(t30, tri.lam)
    zeta, omega = tri.Z.conj() @ B.T, tri.U.conj() @ B.T
    want = np.array([estimator.level_estimate(estimator.level_samples(hi, lo, zeta[:k], omega[:k], c[:k])).var
                     for k in range(len(c) + 1)])
    # each partial sample within delta (1e-12 of the sample's scale): a variance
    # over n samples then moves by at most 4 delta (sqrt(var) + delta) n / (n - 1)
    terms = np.abs(c[:, None] * np.conj(zeta) * omega)
    delta = 1e-12 * float(np.max(np.abs(hi) + np.abs(lo) + terms.sum(axis=0)))
    bound = 4 * delta * (np.sqrt(want) + delta) * n / (n - 1)
    err = np.abs(p.variance - want)
    print(f"oracle profile: variance k=0 {want[0]:.6g} -> k={len(c)} {want[-1]:.6g}, "
          f"max err / bound {np.max(err / bound):.2e}")
    assert np.all(err <= bound)
