"""Checkpoint and resume: a run saved mid-way and resumed from the file in a
new set-up continues with exactly the samples of the uninterrupted run (the
noise is counter-based), so the level accumulators agree bit for bit --
eagerly and through a captured HIP graph."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_helpers import lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _accs(run):
    torch.cuda.synchronize()
    return [lv.acc.cpu().numpy().copy() for lv in run.levels]


@pytest.mark.parametrize("prec", [0, 1])
def test_resume_eager_is_bit_exact(tmp_path, prec):
    L = lib()
    from paper_2306_09559_amd import driver
    from synth.configs import C2
    a = driver.build(C2, prec=prec, rb=16)
    a.step()
    a.step()
    path = str(tmp_path / "c2.npz")
    driver.save_checkpoint(a, path)
    a.step()
    want = _accs(a)
    b = driver.build(C2, prec=prec, rb=16, resume=path)
    assert [lv.drawn for lv in b.levels] == [2 * lv.batch for lv in a.levels]
    assert np.array_equal(b.roots.inv_roots[150], a.roots.inv_roots[150])
    b.step()
    got = _accs(b)
    for x, y in zip(got, want):
        assert np.array_equal(x, y)
    assert [e["estimate"] for e in b.estimates()] == [e["estimate"] for e in a.estimates()]


def test_resume_through_a_graph(tmp_path):
    L = lib()
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    from synth.configs import C1
    a = driver.build(C1, prec=0, rb=4)
    ga = GraphStep([a])
    ga.replay(2)
    ga.sync_drawn()
    path = str(tmp_path / "c1.npz")
    driver.save_checkpoint(a, path)
    ga.replay(1)
    want = _accs(a)
    b = driver.build(C1, prec=0, rb=4, resume=path)
    gb = GraphStep([b], keep_state=True)
    gb.replay(1)
    gb.sync_drawn()
    for x, y in zip(_accs(b), want):
        assert np.array_equal(x, y)
    assert [lv.drawn for lv in b.levels] == [3 * lv.batch for lv in a.levels]


def test_resume_refuses_another_workload(tmp_path):
    L = lib()
    from paper_2306_09559_amd import driver
    from synth.configs import C1
    a = driver.build(C1, prec=0, rb=4)
    path = str(tmp_path / "c1.npz")
    driver.save_checkpoint(a, path)
    other = dataclasses.replace(C1, kappa=0.151)
    with pytest.raises(ValueError, match="another workload"):
        driver.build(other, prec=0, rb=4, resume=path)
