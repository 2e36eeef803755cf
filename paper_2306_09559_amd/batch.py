"""Batched execution of the multilevel sampling: HIP-graph capture of whole
steps over several lattices, and an autotuner for the kernel shape.

A step is every polynomial level of every lattice drawing its batch of Z4
samples (eq. multpolytr, Sec. 3.1; Sec. 5 step 3).  `GraphStep` records one
step of a list of `LatticeRun`s as a single HIP graph: each lattice gets
its own branch (a forked stream), so independent lattices of uneven size,
degree and sample count run concurrently instead of one after the other,
and a replay costs one graph launch instead of one host launch per kernel.
Each level's noise takes its sample index from a device counter that the
graph advances by the batch size (mpmc_counter_add), so every replay draws
new samples and the level accumulators keep merging them on the device.
Solve levels (host-driven GMRES) are not captured.

`autotune` times each level's candidate shapes -- RHS block width and the
t-sweep vs the streaming kernel -- on the real workload and keeps the
fastest; results are cached in a JSON file keyed by (gfx arch, lattice,
batch size, precision, polynomial).
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib as L
from .driver import LatticeRun


@dataclass
class _Item:
    run: LatticeRun
    level: int
    nsamples: int          # vectors per batch
    repeats: int           # batches per replay
    counter: torch.Tensor


class GraphStep:
    """One step of several lattice runs captured as one HIP graph."""

    def __init__(self, runs: Sequence[LatticeRun], batch: Optional[Dict[Tuple[int, int], int]] = None,
                 parallel: bool = True, warmup: int = 1, only: Optional[Sequence[Tuple[int, int]]] = None,
                 keep_state: bool = False):
        """runs: the lattices; batch: samples per (run, level), default the
        configured batch; only: restrict to these (run, level) pairs;
        keep_state: continue the levels' accumulators and sample counts (a
        run resumed from a checkpoint) instead of starting from zero."""
        self.runs = list(runs)
        self.parallel = parallel
        self.items: List[List[_Item]] = []
        sel = set(only) if only is not None else None
        for ri, run in enumerate(self.runs):
            row = []
            for li, lv in enumerate(run.levels):
                if lv.solver is not None or (sel is not None and (ri, li) not in sel):
                    continue
                if batch is not None and (ri, li) in batch:
                    n, reps = batch[(ri, li)], 1
                else:
                    n, reps = lv.batch, run.batches(li)
                row.append(_Item(run, li, n, reps, torch.zeros(1, dtype=torch.int64, device="cuda")))
            self.items.append(row)
        self.replays = 0
        saved = None
        if keep_state:
            torch.cuda.synchronize()
            saved = [[(it.run.levels[it.level].acc.clone(), it.run.levels[it.level].drawn) for it in row]
                     for row in self.items]
        self._side = [torch.cuda.Stream() for _ in self.runs] if parallel else []
        # eager warm-up: sets kernel attributes and touches every buffer before capture
        for _ in range(warmup):
            self._enqueue_all(torch.cuda.current_stream())
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=cap):
            self._enqueue_all(cap)
        torch.cuda.synchronize()
        if saved is None:
            self.reset()
        else:
            for row, srow in zip(self.items, saved):
                for it, (acc, drawn) in zip(row, srow):
                    it.run.levels[it.level].acc.copy_(acc)
                    it.run.levels[it.level].drawn = drawn
                    it.counter.fill_(drawn)
            torch.cuda.synchronize()

    def _enqueue_run(self, row: List[_Item]):
        for it in row:
            # the sample index is the counter alone: replay k draws samples k*N .. k*N+N-1
            nz = L.Noise(it.run.cfg.seed_noise, it.run.cfg.lattice_id, it.run.levels[it.level].index, 0,
                         it.counter)
            for _ in range(it.repeats):
                it.run.enqueue(it.level, it.nsamples, nz)
                L.counter_add(it.counter, it.nsamples)

    def _enqueue_all(self, main: torch.cuda.Stream):
        if not self.parallel:
            for row in self.items:
                self._enqueue_run(row)
            return
        for row, side in zip(self.items, self._side):
            side.wait_stream(main)
            with torch.cuda.stream(side):
                self._enqueue_run(row)
        for side in self._side:
            main.wait_stream(side)

    def reset(self):
        """Zero the accumulators and the sample counters (outside the graph)."""
        for row in self.items:
            for it in row:
                it.counter.zero_()
                it.run.levels[it.level].acc.zero_()
                it.run.levels[it.level].drawn = 0
        torch.cuda.synchronize()
        self.replays = 0

    def replay(self, times: int = 1):
        for _ in range(times):
            self.graph.replay()
        self.replays += times

    def sync_drawn(self):
        """Set every level's sample count from its device counter (the replays
        advance only the counters), e.g. before driver.save_checkpoint."""
        torch.cuda.synchronize()
        for row in self.items:
            for it in row:
                it.run.levels[it.level].drawn = int(it.counter.item())

    def samples_drawn(self) -> Dict[Tuple[int, int], int]:
        return {(ri, it.level): it.nsamples * it.repeats * self.replays
                for ri, row in enumerate(self.items) for it in row}


# ------------------------------------------------------------------ autotuner
_CACHE = os.environ.get("MPMC_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mpmc_autotune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:       # noqa: BLE001 - device query only labels the cache entry
        return "unknown"


def _key(run: LatticeRun, level: int) -> str:
    lv = run.cfg.levels[level]
    return json.dumps([_arch(), list(run.cfg.dims), int(run.prec), int(lv.samples), str(lv.hi), str(lv.lo),
                       bool(lv.deflated)])


def _candidates(run: LatticeRun, level: int) -> List[Tuple[int, bool]]:
    """(rb, sweep) shapes to time for one level: every block width dividing
    the batch on the streaming kernel, and on the t-sweep wherever the
    library's plan takes it (whole planes, or FP32 blocks with a halo); the
    level's current shape is always among them."""
    N = run.levels[level].batch
    rbs = [rb for rb in (1, 2, 4, 8, 16, 32) if N % rb == 0]
    out = [(rb, False) for rb in rbs]
    # the sweep reads the noise itself: rb only shapes the first step's input, so wide blocks suffice
    out += [(rb, True) for rb in rbs if rb >= 8 and L.sweep_plan(run.dl, N, rb)["ok"]]
    current = (run.level_rb(level), bool(run.levels[level].sweep))
    if current not in out:
        out.append(current)
    return out


def _time_level(run: LatticeRun, level: int, reps: int) -> float:
    N = run.levels[level].batch
    s = torch.cuda.current_stream()
    run.draw(level, N)                 # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run.draw(level, N)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


@dataclass
class TuneResult:
    choice: Dict[int, Tuple[int, bool]] = field(default_factory=dict)
    timings: Dict[int, Dict[str, float]] = field(default_factory=dict)
    cached: Dict[int, bool] = field(default_factory=dict)


def autotune(run: LatticeRun, reps: int = 3, use_cache: bool = True, cache_path: Optional[str] = None,
             keep_within: float = 0.03) -> TuneResult:
    """Pick (rb, sweep) per polynomial level of `run` by timing; applies the
    choice to the run and resets its accumulators.  The level's current shape
    is kept unless another candidate is faster by more than keep_within (a
    shape the kernel ignores, such as rb under the t-sweep, would otherwise
    be chosen by timing noise)."""
    path = cache_path or _CACHE
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    res = TuneResult()
    for li, lv in enumerate(run.levels):
        if lv.solver is not None:
            continue
        key = _key(run, li)
        if use_cache and key in cache:
            rb, sw = cache[key]["rb"], cache[key]["sweep"]
            run.set_level_shape(li, rb, sw)
            res.choice[li] = (rb, sw)
            res.cached[li] = True
            continue
        best, times = None, {}
        current = (run.level_rb(li), lv.sweep)
        t_current = None
        for rb, sw in _candidates(run, li):
            run.set_level_shape(li, rb, sw)
            t = _time_level(run, li, reps)
            times[f"rb{rb}{'-sweep' if sw else ''}"] = t
            if (rb, sw) == current:
                t_current = t
            if best is None or t < best[0]:
                best = (t, rb, sw)
        if t_current is not None and t_current <= best[0] * (1.0 + keep_within):
            best = (t_current,) + current
        _, rb, sw = best
        run.set_level_shape(li, rb, sw)
        res.choice[li] = (rb, sw)
        res.timings[li] = times
        res.cached[li] = False
        cache[key] = {"rb": rb, "sweep": sw, "seconds": best[0], "when": time.strftime("%Y-%m-%d")}
    run.reset()
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return res
