"""Batched execution of the multilevel sampling through the library's
batched-step entry points, and the kernel-shape autotuner.

A step is every polynomial level of every lattice drawing its batch of Z4
samples (eq. multpolytr, Sec. 3.1; Sec. 5 step 3).  `GraphStep` hands one
step of a list of `LatticeRun`s to `mpmc_batch_build`, which records it as
a single HIP graph: each lattice gets its own branch, so independent
lattices of uneven size, degree and sample count run concurrently, and a
replay (`mpmc_batch_launch`) is one graph launch instead of one host launch
per kernel.  Each level's noise takes its sample index from a device
counter that the graph advances by the batch size, so every replay draws
new samples and the level accumulators keep merging them on the device.
Solve levels (host-driven GMRES) are not batched.

`autotune` asks `mpmc_autotune` to time each level's candidate shapes --
RHS block width, the t-sweep or the streaming kernel, and on FP32 planes cut
into blocks the block shape -- on the real workload, keeps the fastest, and
persists the choices in a JSON file keyed by (gfx arch, lattice, batch size,
precision, polynomial).
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
    """One step of several lattice runs recorded by the library as one HIP graph."""

    def __init__(self, runs: Sequence[LatticeRun], batch: Optional[Dict[Tuple[int, int], int]] = None,
                 parallel: bool = True, only: Optional[Sequence[Tuple[int, int]]] = None,
                 keep_state: bool = False, level_branches: bool = False):
        """runs: the lattices; batch: samples per (run, level), default the
        configured batch; parallel: one graph branch per lattice (else one
        branch in order); level_branches: one branch per level of every
        lattice (the levels hold separate buffers, so their launches may
        overlap); only: restrict to these (run, level) pairs; keep_state:
        continue the levels' accumulators and sample counts (a run resumed
        from a checkpoint) instead of starting from zero."""
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
        self.handle = L.Handle()
        citems = []
        nb = 0
        for ri, row in enumerate(self.items):
            for it in row:
                if level_branches:
                    branch = nb
                    nb += 1
                else:
                    branch = ri if parallel else 0
                run, lv = it.run, it.run.levels[it.level]
                cfg = run.cfg
                # the sample index is the counter alone: replay k draws samples k*N .. k*N+N-1
                cfg_noise = L.Noise(cfg.seed_noise, cfg.lattice_id, lv.index, 0)
                citems.append(L.BatchItem(run.dl, lv.device, it.nsamples, run.level_rb(it.level), cfg_noise,
                                          it.counter, it.repeats, lv.samples[: it.nsamples], lv.acc, lv.ws,
                                          branch=branch,
                                          plane_sweep=int(lv.sweep),
                                          sweep_rank=int(lv.sweep_rank), sweep_chunks=int(lv.sweep_chunks)))
        L.batch_build(self.handle, citems)
        if keep_state:
            torch.cuda.synchronize()
            for row in self.items:
                for it in row:
                    it.counter.fill_(it.run.levels[it.level].drawn)
            torch.cuda.synchronize()
        else:
            self.reset()

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
            L.batch_launch(self.handle)
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


@dataclass
class TuneResult:
    # level -> (rb, kernel family 0/1/2 as MPMC_OPT_PLANE_SWEEP, block rank, t-chunks)
    choice: Dict[int, Tuple[int, int, int, int]] = field(default_factory=dict)
    timings: Dict[int, Dict[str, float]] = field(default_factory=dict)
    cached: Dict[int, bool] = field(default_factory=dict)


def _label(choice) -> str:
    rb, sw, rank, chunks = choice
    if not sw:
        return f"rb{rb}"
    return f"rb{rb}-{'sweep' if sw == 1 else 'auto'}{'' if rank == 0 else rank}{'' if chunks == 0 else f'-t{chunks}'}"


def autotune(run: LatticeRun, reps: int = 3, use_cache: bool = True, cache_path: Optional[str] = None,
             keep_within: float = 0.03, handle: Optional[L.Handle] = None) -> TuneResult:
    """Pick (rb, kernel family, block rank, t-chunks) per polynomial level of
    `run` with mpmc_autotune; applies the choice to the run and resets its
    accumulators.  The level's current shape (initially the plan's choice of
    kernel, family 2) is timed as it runs and kept unless another is faster
    by more than keep_within; a chosen candidate runs exactly as it was
    timed (family 0 or 1, never re-decided by the plan).  Choices persist in
    a JSON file."""
    path = cache_path or _CACHE
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    h = handle or L.Handle()
    res = TuneResult()
    for li, lv in enumerate(run.levels):
        if lv.solver is not None:
            continue
        key = _key(run, li)
        if use_cache and key in cache:
            c = cache[key]
            rb, sw, rank, chunks = int(c["rb"]), int(c["sweep"]), int(c.get("rank", 0)), int(c.get("chunks", 0))
            run.set_level_shape(li, rb, sw, rank, chunks)
            res.choice[li] = (rb, sw, rank, chunks)
            res.cached[li] = True
            continue
        N = lv.batch
        cur = (run.level_rb(li), int(lv.sweep), int(lv.sweep_rank), int(lv.sweep_chunks))
        nz = L.Noise(run.cfg.seed_noise, run.cfg.lattice_id, lv.index, 0)
        best, secs, _hit, table = L.autotune_level(h, run.dl, lv.device, N, nz, cur, reps=reps,
                                                   keep_within=keep_within)
        rb, sw, rank, chunks = best
        run.set_level_shape(li, rb, sw, rank, chunks)
        res.choice[li] = (rb, sw, rank, chunks)
        res.timings[li] = {_label(c): t for c, t in table}
        res.cached[li] = False
        cache[key] = {"rb": rb, "sweep": sw, "rank": rank, "chunks": chunks, "seconds": secs,
                      "when": time.strftime("%Y-%m-%d")}
    run.reset()
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return res
