"""Batched execution: a whole multilevel step of one or several lattices
captured as one HIP graph must reproduce the eager step bit for bit on
every replay (the sample index comes from a device counter the graph
advances), with eager work and synchronisation between replays; the
autotuner's shape choice changes only the speed, not the values beyond
the order of floating-point sums."""
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


def _small_cfgs():
    from synth.configs import C1, Level
    a = C1
    b = dataclasses.replace(C1, name="C1b", dims=(4, 4, 4, 2), kappa=0.14, levels=(Level(12, None, 24),),
                            seed_links=111, seed_start=112, seed_noise=113, lattice_id=11)
    return a, b


def _eager_steps(run, steps):
    out = []
    run.reset()
    for _ in range(steps):
        run.step()
        torch.cuda.synchronize()
        out.append([lv.samples[: run.cfg.levels[i].samples].cpu().numpy().copy() for i, lv in enumerate(run.levels)])
    accs = [lv.acc.cpu().numpy().copy() for lv in run.levels]
    return out, accs


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager(prec):
    L = lib()
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    ca, cb = _small_cfgs()
    runs = [driver.build(ca, prec=prec, rb=4), driver.build(cb, prec=prec, rb=8)]
    steps = 3
    eager = [_eager_steps(r, steps) for r in runs]
    gs = GraphStep(runs, parallel=True)
    other = L.empty_field(runs[0].dl.V, 4, 4, prec)
    scratch = L.empty_field(runs[0].dl.V, 4, 4, prec)
    L.z4_fill(runs[0].dl.dims, prec, L.Noise(9, 9, 9, 0), scratch)
    for k in range(steps):
        gs.replay()
        torch.cuda.synchronize()
        for ri, run in enumerate(runs):
            for li, lv in enumerate(run.levels):
                got = lv.samples[: run.cfg.levels[li].samples].cpu().numpy()
                assert np.array_equal(got, eager[ri][0][k][li]), (ri, li, k)
        # the program's own eager work between replays
        L.wilson_apply(runs[0].dl, scratch, other)
        torch.cuda.synchronize()
    for ri, run in enumerate(runs):
        for li, lv in enumerate(run.levels):
            assert np.array_equal(lv.acc.cpu().numpy(), eager[ri][1][li])
    assert gs.samples_drawn()[(0, 0)] == steps * ca.levels[0].samples


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager_on_the_8x4_workload(prec):
    """The full 8^4 three-level workload (256 samples per level and step, the
    two polynomial-difference levels deflated with 20 eigenvectors: the MFMA
    GEMMs inside the recording) as one graph with a branch per level: every
    replay gives
    every level's samples of the eager step bit for bit, and the accumulators
    match after two steps."""
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    from synth.configs import C2
    run = driver.build(C2, prec=prec, rb=16)
    assert any(lv.deflated for lv in C2.levels)
    steps = 2
    eager, accs = _eager_steps(run, steps)
    gs = GraphStep([run], level_branches=True)
    for k in range(steps):
        gs.replay()
        torch.cuda.synchronize()
        for li, lv in enumerate(run.levels):
            got = lv.samples[: C2.levels[li].samples].cpu().numpy()
            assert np.array_equal(got, eager[k][li]), (li, k)
    for li, lv in enumerate(run.levels):
        assert np.array_equal(lv.acc.cpu().numpy(), accs[li]), li


def test_graph_serial_equals_parallel():
    """One branch in order, one per lattice and one per level give the same
    accumulators bit for bit."""
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    ca, cb = _small_cfgs()
    runs = [driver.build(ca, prec=0, rb=4), driver.build(cb, prec=0, rb=8)]
    res = []
    for kw in (dict(parallel=False), dict(parallel=True), dict(level_branches=True)):
        gs = GraphStep(runs, **kw)
        gs.replay(2)
        torch.cuda.synchronize()
        res.append([[lv.acc.cpu().numpy().copy() for lv in r.levels] for r in runs])
    for other in res[1:]:
        for a, b in zip(res[0], other):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_autotune_keeps_values(tmp_path):
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import autotune
    from synth.configs import C1
    run = driver.build(C1, prec=0, rb=4)
    run.reset()
    run.step()
    ref = [run.estimates()[i]["estimate"] for i in range(len(run.levels))]
    res = autotune(run, reps=1, cache_path=str(tmp_path / "tune.json"))
    assert set(res.choice) == {0, 1}
    run.step()
    got = [run.estimates()[i]["estimate"] for i in range(len(run.levels))]
    for a, b in zip(got, ref):
        assert abs(a - b) <= 1e-12 * abs(b)
    # second call is served from the cache
    res2 = autotune(run, reps=1, cache_path=str(tmp_path / "tune.json"))
    assert all(res2.cached.values()) and res2.choice == res.choice


def test_autotune_offers_the_blocked_sweep(tmp_path):
    """On an FP32 lattice whose xyz-plane exceeds one workgroup (16^3 planes:
    the t-sweep cuts them into blocks with a halo), mpmc_autotune times the
    blocked t-sweep with its best-ranked blocks next to the streaming kernel,
    and keeps the sweep when it is the faster shape; the chosen block rank
    changes the plan's block and leaves the level's values alone."""
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import autotune
    from synth.configs import Level
    L = lib()
    cfg = dataclasses.replace(_small_cfgs()[0], name="C1p", dims=(16, 16, 16, 4), kappa=0.14,
                              levels=(Level(12, None, 64),), seed_links=121, lattice_id=12)
    run = driver.build(cfg, prec=L.F32, rb=16)
    assert L.sweep_plan(run.dl, 64, 16)["halo"]
    L.set_option(L.OPT_SWEEP_RANK, 1)
    second = L.sweep_plan(run.dl, 64, 16)
    L.set_option(L.OPT_SWEEP_RANK, 0)
    assert second["ok"] and second["block"] != L.sweep_plan(run.dl, 64, 16)["block"]
    run.step()
    torch.cuda.synchronize()
    ref = run.levels[0].samples.cpu().numpy().copy()
    res = autotune(run, reps=3, use_cache=False, cache_path=str(tmp_path / "t.json"))
    t = res.timings[0]
    print(t)
    assert {"rb16", "rb16-sweep", "rb16-sweep1"} <= set(t)
    # streaming candidates are labelled rbN alone ("-auto" is the level's current shape, the plan's choice)
    best_sweep = min(v for k, v in t.items() if "-sweep" in k)
    best_stream = min(v for k, v in t.items() if "-sweep" not in k and "-auto" not in k)
    # the blocked sweep moves ~1.7x the streaming kernel's bytes per second on these planes
    assert best_sweep < best_stream
    assert res.choice[0][1]
    run.step()
    torch.cuda.synchronize()
    got = run.levels[0].samples.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_autotune_with_a_current_shape_wider_than_its_candidates():
    """A level run at block width 64, wider than the tuner's candidates (its
    workspace covers rb <= 32): mpmc_autotune times only the candidates,
    returns the fastest of them and never the untimed current shape."""
    from paper_2306_09559_amd import driver
    from synth.configs import Level
    L = lib()
    cfg = dataclasses.replace(_small_cfgs()[0], name="C1w", levels=(Level(6, None, 64),), lattice_id=14)
    run = driver.build(cfg, prec=L.F64, rb=16)
    lv = run.levels[0]
    nz = L.Noise(cfg.seed_noise, cfg.lattice_id, lv.index, 0)
    best, secs, cached, table = L.autotune_level(L.Handle(), run.dl, lv.device, 64, nz, (64, 0, 0, 0), reps=1)
    print(best, secs, table)
    assert not cached and secs > 0 and table
    assert all(c[0] <= 32 for c, _ in table)
    assert best in [c for c, _ in table] and secs == min(t for _, t in table)


def test_a_level_runs_the_kernel_family_it_was_tuned_with(tmp_path, monkeypatch):
    """The tuner times forced kernel families (0 streaming, 1 t-sweep) next to
    the level's current shape as it runs (family 2: the plan decides); the
    level then runs with exactly the chosen family.  A t-sweep in 2 t-chunks
    on 8^4 x 64 vectors (128 workgroups for 256 CUs, where the plan's own
    test would fall back to streaming) still runs as a t-sweep."""
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import autotune
    from synth.configs import Level
    L = lib()
    cfg = dataclasses.replace(_small_cfgs()[0], name="C1f", dims=(8, 8, 8, 8), kappa=0.14,
                              levels=(Level(6, None, 64),), seed_links=141, lattice_id=15)
    run = driver.build(cfg, prec=L.F64, rb=16)
    calls = []
    set_option = L.set_option

    def record(opt, value):
        calls.append((opt, value))
        return set_option(opt, value)
    monkeypatch.setattr(L, "set_option", record)
    run.draw(0, 64)
    assert calls[:3] == [(L.OPT_PLANE_SWEEP, L.SWEEP_AUTO), (L.OPT_SWEEP_RANK, 0), (L.OPT_SWEEP_CHUNKS, 0)]
    calls.clear()
    run.set_level_shape(0, 16, True, 0, 2)
    run.draw(0, 64)
    assert calls[:3] == [(L.OPT_PLANE_SWEEP, L.SWEEP_ALWAYS), (L.OPT_SWEEP_RANK, 0), (L.OPT_SWEEP_CHUNKS, 2)]
    run.set_level_shape(0, 16, L.SWEEP_AUTO)
    res = autotune(run, reps=1, use_cache=False, cache_path=str(tmp_path / "t.json"))
    print(res.timings[0], res.choice[0])
    assert "rb16-auto" in res.timings[0]              # the current shape, timed as it runs
    rb, family, rank, chunks = res.choice[0]
    calls.clear()
    run.draw(0, 64)
    assert calls[:3] == [(L.OPT_PLANE_SWEEP, family), (L.OPT_SWEEP_RANK, rank), (L.OPT_SWEEP_CHUNKS, chunks)]
    torch.cuda.synchronize()


def test_a_recorded_step_outlives_a_reshaped_level():
    """A recorded step keeps the buffers it was recorded with: after the
    level is reshaped (a new workspace; the old one would go back to torch's
    allocator), a tensor of the old workspace's size filled with a constant
    stays untouched by replays, and the replays still give the recorded
    shape's samples bit for bit.  The adaptive loop's recorded steps of a
    reshaped level are dropped, to be recorded again with its new shape."""
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    L = lib()
    cfg = _small_cfgs()[1]
    run = driver.build(cfg, prec=L.F64, rb=4)
    lv = run.levels[0]
    run.reset()
    run.step()
    torch.cuda.synchronize()
    ref = lv.samples.cpu().numpy().copy()
    gs = GraphStep([run])
    driver.prepare_adaptive(run)
    assert any(k[0] == "step" and k[1] == 0 for k in run.adaptive)
    old_bytes = lv.ws.numel()
    run.set_level_shape(0, 8, L.SWEEP_OFF)
    assert not any(k[0] == "step" and k[1] == 0 for k in run.adaptive)
    filler = torch.full((old_bytes,), 7, dtype=torch.uint8, device="cuda")
    gs.reset()
    gs.replay()
    torch.cuda.synchronize()
    assert bool((filler == 7).all())
    assert np.array_equal(lv.samples.cpu().numpy(), ref)


def test_autotune_offers_t_chunks(tmp_path):
    """On 8^4 planes with 64 vectors the plan cuts the whole-plane t-sweep
    into 4 t-chunks (64 workgroups would leave three CUs in four idle);
    mpmc_autotune also times the neighbouring chunk count, 2.  A level forced
    to 2 chunks gives the samples of the plan's 4 up to the order of FP64
    sums, and the same level recorded as a HIP graph (the chunk count carried
    by the batch item) replays the eager samples bit for bit."""
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep, autotune
    from synth.configs import Level
    L = lib()
    cfg = dataclasses.replace(_small_cfgs()[0], name="C1t", dims=(8, 8, 8, 8), kappa=0.14,
                              levels=(Level(12, None, 64),), seed_links=131, lattice_id=13)
    run = driver.build(cfg, prec=L.F64, rb=16)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    L.set_option(L.OPT_SWEEP_CHUNKS, 0)
    assert L.sweep_plan(run.dl, 64, 16)["chunks"] == 4
    L.set_option(L.OPT_PLANE_SWEEP, 2)
    res = autotune(run, reps=2, use_cache=False, cache_path=str(tmp_path / "t.json"))
    t = res.timings[0]
    print(t)
    assert {"rb16", "rb16-sweep", "rb16-sweep-t2"} <= set(t)
    samples = {}
    for chunks in (0, 2):
        run.set_level_shape(0, 16, True, 0, chunks)
        eager, _ = _eager_steps(run, 1)
        samples[chunks] = eager[0][0]
        gs = GraphStep([run])
        gs.replay()
        torch.cuda.synchronize()
        assert np.array_equal(run.levels[0].samples[:64].cpu().numpy(), samples[chunks]), chunks
    assert L.sweep_plan(run.dl, 64, 16)["chunks"] == 4     # eager steps leave the options as they found them
    a, b = samples[0], samples[2]
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_batch_entry_points_validate(tmp_path):
    """mpmc_batch_build rejects a solve level, a missing counter and a short
    workspace before recording anything; mpmc_batch_launch needs a built step."""
    from paper_2306_09559_amd import driver
    L = lib()
    run = driver.build(_small_cfgs()[1], prec=0, rb=8)
    lv = run.levels[0]
    h = L.Handle()
    with pytest.raises(L.MpmcError) as e:
        L.batch_launch(h)
    assert e.value.status == L.EINVAL
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    good = dict(lat=run.dl, level=lv.device, nrhs=lv.batch, rb=8, noise=L.Noise(1, 2, 3, 0), counter=ctr,
                batches=1, samples=lv.samples, acc=lv.acc, ws=lv.ws)
    with pytest.raises(L.MpmcError) as e:
        L.batch_build(h, [L.BatchItem(**dict(good, ws=lv.ws[:16]))])
    assert e.value.status == L.EWORKSPACE
    solve = L.DeviceLevel(L.OP_SOLVE, None, solve_x=lv.samples)
    with pytest.raises(L.MpmcError) as e:
        L.batch_build(h, [L.BatchItem(**dict(good, level=solve))])
    assert e.value.status == L.EUNSUPPORTED
    L.batch_build(h, [L.BatchItem(**good)])
    h.close()
