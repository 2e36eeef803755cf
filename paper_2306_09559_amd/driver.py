"""Per-lattice state and the multilevel sampling loop on the GPU.

A `LatticeRun` owns the device lattice, the polynomial roots and the
deflation triplets of one workload, builds one `DeviceLevel` per term of the
multilevel formula (eq. multpolytr, Sec. 3.1) with Monte Carlo deflation on
the polynomial-difference levels (Sec. 4.1), and draws batches of Z4
samples through `mpmc_mlmc_level_estimate`.

Levels are numbered from the top (0 = highest degree).  The estimate of a
level is the accumulator mean plus the exact deflation correction sum_i c_i
(u_i^H z_i = 1 by the scaling, Sec. 4.1).
"""
from __future__ import annotations

import json
import os
import time
import types
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

import synth
from synth.configs import LatticeConfig

from synth.configs import SOLVE

from . import _lib as L
from . import krylov, probing
from .solve import MixedPPGMRES, SolveNotConverged, SolveStats


def poly_mvps(p) -> int:
    """Operator applications of one polynomial application (Sec. 3.1, Sec. 3.2):
    d for a single polynomial of degree d, n_in n_out - 1 for a double one
    given as (n_in, n_out), none for a level without a polynomial or a solve
    (whose cost depends on its convergence and is counted by the solver)."""
    if p is None or p == SOLVE:
        return 0
    if isinstance(p, tuple):
        n_in, n_out = p
        return n_in * n_out - 1
    return int(p)


@dataclass
class LevelState:
    index: int
    device: L.DeviceLevel
    mvps_per_sample: int
    c: Optional[np.ndarray]
    acc: torch.Tensor
    samples: torch.Tensor
    ws: torch.Tensor
    drawn: int = 0
    # top level Tr(A^{-1} - p_1(A)): the solver and its batch fields
    solver: Optional[MixedPPGMRES] = None
    b64: Optional[torch.Tensor] = None
    x64: Optional[torch.Tensor] = None
    xl: Optional[torch.Tensor] = None       # x in the level precision
    last_solve: Optional[SolveStats] = None
    solve_tol: float = 1e-6
    rb: int = 0                             # RHS block width of this level (0: the run's)
    batch: int = 0                          # vectors per batch (device buffers); samples per step / batch draws
    sweep: int = L.SWEEP_AUTO               # kernel family (MPMC_OPT_PLANE_SWEEP: 0 streaming, 1 t-sweep, 2 plan's choice)
    sweep_rank: int = 0                     # block choice of a blocked t-sweep (MPMC_OPT_SWEEP_RANK)
    sweep_chunks: int = 0                   # t-chunks of the sweep (MPMC_OPT_SWEEP_CHUNKS; 0: the plan's)


@dataclass
class LatticeRun:
    cfg: LatticeConfig
    prec: int
    rb: int
    dl: L.DeviceLattice
    roots: krylov.RootSet
    defl: Optional[krylov.Deflation]
    levels: List[LevelState] = field(default_factory=list)
    setup_seconds: float = 0.0
    defl64_V: Optional[torch.Tensor] = None     # FP64 eigenvectors of the set-up
    composites: Dict[tuple, krylov.OuterRoots] = field(default_factory=dict)
    # adaptive loop: per-level device stopping state and recorded one-batch steps (kept across calls)
    adaptive: Dict[tuple, object] = field(default_factory=dict)

    # -- sampling --------------------------------------------------------
    def noise(self, level: int, sample_offset: Optional[torch.Tensor] = None) -> L.Noise:
        lv = self.levels[level]
        return L.Noise(self.cfg.seed_noise, self.cfg.lattice_id, lv.index, lv.drawn, sample_offset)

    def level_rb(self, level: int) -> int:
        return self.levels[level].rb or self.rb

    def enqueue(self, level: int, nsamples: int, nz: L.Noise):
        """Enqueue one batch of a polynomial level with an explicit noise
        descriptor (used by graph capture, where the sample index comes from a
        device counter)."""
        lv = self.levels[level]
        # the level's kernel selection for this call only (the options are
        # process-wide; mpmc_batch_build scopes them per item the same way):
        # the caller's values are restored afterwards
        opts = (L.OPT_PLANE_SWEEP, L.OPT_SWEEP_RANK, L.OPT_SWEEP_CHUNKS)
        prev = [L.get_option(o) for o in opts]
        for o, v in zip(opts, (lv.sweep, lv.sweep_rank, lv.sweep_chunks)):
            L.set_option(o, int(v))
        try:
            L.mlmc_level_estimate(self.dl, lv.device, nsamples, self.level_rb(level), nz, lv.samples[:nsamples],
                                  lv.acc, lv.ws)
        finally:
            for o, v in zip(opts, prev):
                L.set_option(o, v)

    def draw(self, level: int, nsamples: int):
        """Enqueue nsamples more samples of one level (one batch)."""
        lv = self.levels[level]
        nz = self.noise(level)
        if lv.solver is not None:
            # x = A^{-1} b for this batch's noise, then b^H x - b^H P_lo b
            if nsamples != lv.solver.N:
                raise ValueError(f"level {level} solves batches of {lv.solver.N} vectors")
            L.z4_fill(self.cfg.dims, L.F64, nz, lv.b64)
            lv.last_solve = lv.solver.solve(lv.b64, lv.x64, tol=lv.solve_tol)
            if not lv.last_solve.converged:
                raise SolveNotConverged(lv.last_solve)
            if lv.xl is not lv.x64:
                L.field_axpby_mixed(self.cfg.dims, lv.solver.ones, lv.x64, None, lv.xl)
        self.enqueue(level, nsamples, nz)
        lv.drawn += nsamples

    def batches(self, level: int) -> int:
        """Batches per step of a level: its configured samples / its batch size."""
        return self.cfg.levels[level].samples // self.levels[level].batch

    def step(self, batch: Optional[Dict[int, int]] = None):
        """One pass of the hot path: every level draws its configured samples
        (in batches of its buffer size), or `batch[level]` samples."""
        for i, lv in enumerate(self.levels):
            if batch is not None and i in batch:
                self.draw(i, batch[i])
                continue
            for _ in range(self.batches(i)):
                self.draw(i, lv.batch)

    def reset(self):
        for lv in self.levels:
            lv.acc.zero_()
            lv.drawn = 0

    def set_level_shape(self, level: int, rb: int, sweep, rank: int = 0, chunks: int = 0):
        """Choose the RHS block width, kernel family, blocked-sweep block rank
        and t-chunk count (0: the plan's) of one level (the autotuner's
        knobs); resizes the level's workspace.  sweep is the kernel family as
        MPMC_OPT_PLANE_SWEEP takes it (0 streaming, 1 the t-sweep wherever the
        lattice admits one, 2 the plan's choice); True means 1, False 0."""
        lv = self.levels[level]
        if lv.solver is not None:
            raise ValueError("the block width of a solve level is fixed by its solver")
        N = lv.batch
        if N % rb:
            raise ValueError(f"rb={rb} does not divide {N}")
        mode = int(sweep)
        if mode not in (L.SWEEP_OFF, L.SWEEP_ALWAYS, L.SWEEP_AUTO):
            raise ValueError(f"kernel family {sweep!r} is not 0, 1 or 2")
        lv.rb, lv.sweep, lv.sweep_rank, lv.sweep_chunks = int(rb), mode, int(rank), int(chunks)
        lv.ws = L.workspace(L.level_workspace_size(self.dl, lv.device, N, rb))
        # the adaptive loop's recorded one-batch steps of this level have the old shape
        for key in [k for k in self.adaptive if k[0] == "step" and k[1] == level]:
            del self.adaptive[key]

    def estimates(self):
        """Per-level (estimate, stderr, variance, n) on the host."""
        out = []
        for lv in self.levels:
            a = lv.acc.cpu().numpy()
            n = a[0]
            mean = a[1] + 1j * a[2]
            var = a[3] / (n - 1) if n > 1 else float("nan")
            corr = complex(np.sum(lv.c)) if lv.c is not None else 0.0
            out.append(dict(estimate=mean + corr, stderr=float(np.sqrt(var / n)) if n > 1 else float("nan"),
                            variance=float(var), n=int(n), nonfinite=int(a[4])))
        return out

    # -- work accounting -------------------------------------------------
    def bytes_per_step(self) -> int:
        """Algorithmic HBM bytes of the operator applications of one step."""
        return sum(lv.mvps_per_sample * launch_bytes(self.dl.V, self.cfg.levels[i].samples, self.prec)
                   for i, lv in enumerate(self.levels))

    def mvp_rhs_per_step(self) -> int:
        return sum(lv.mvps_per_sample * self.cfg.levels[i].samples for i, lv in enumerate(self.levels))


def launch_bytes(V: int, nrhs: int, prec: int) -> int:
    """Algorithmic HBM bytes of one operator application to nrhs vectors:
    read w and write w' (2 x 12 complex per site and vector) and read the
    links once (4 x 9 complex per site); the noise b of the fused dot is
    regenerated in registers and costs no traffic."""
    c = 16 if prec == L.F64 else 8
    return V * nrhs * 24 * c + V * 36 * c


def _batch_size(samples: int, rb: int, max_batch: int) -> int:
    """Largest multiple of rb that divides samples and is at most max_batch."""
    if samples % rb:
        raise ValueError(f"rb={rb} does not divide the level's {samples} samples")
    best = rb
    for b in range(rb, min(samples, max_batch) + 1, rb):
        if samples % b == 0:
            best = b
    return best


def _device_poly(roots: krylov.RootSet, comps: Dict[tuple, krylov.OuterRoots], p) -> L.DevicePoly:
    if isinstance(p, tuple):
        return comps[p].device
    return roots.device[p]


def _poly_value(roots: krylov.RootSet, comps: Dict[tuple, krylov.OuterRoots], p, lam) -> np.ndarray:
    if isinstance(p, tuple):
        return krylov.composite_value(roots.inv_roots[p[0] - 1], comps[p].inv_roots, lam)
    return krylov.newton_value(roots.inv_roots[p], lam)


# set-up parameters (Sec. 5 step 2) and their defaults; a configuration may
# set any of them in its `extra` dict, an argument of build() overrides both
SETUP_DEFAULTS = {
    "pin_degree": None,    # degree of p_in for PP-Arnoldi (dp_in); default: the composite's, else a middle degree
    "arnoldi_m": 90,       # PP-Arnoldi steps at most
    "rtolev": None,        # stop PP-Arnoldi at this PP-GMRES relative residual (None: run arnoldi_m steps)
    "nev": 40,             # Ritz pairs nearest the origin tested for deflation (nevch)
    "rtolpoly1": None,     # stop the outer PP-GMRES of a double polynomial here (None: the configured n_out)
    "gmres_m": 30,         # restart length of the top-level PP-GMRES
    "solve_tol": 1e-6,     # rtolle
    "solve_rb": 1,         # block width of a top level's fields (1: its polynomials run on the t-sweep)
}


def build(cfg: LatticeConfig, prec: int = L.F64, rb: int = 16, pin_degree: Optional[int] = None,
          arnoldi_m: Optional[int] = None, nev: Optional[int] = None, verbose: bool = False,
          reuse: Optional["LatticeRun"] = None, gmres_m: Optional[int] = None, solve_tol: Optional[float] = None,
          two_row_links: bool = True, max_batch: int = 1 << 30, rtolev: Optional[float] = None,
          rtolpoly1: Optional[float] = None, resume: Optional[str] = None) -> LatticeRun:
    """Set up a lattice workload: links, GMRES roots, PP-Arnoldi deflation,
    outer roots of composite polynomials (FP64 on the GPU, Sec. 5 setup
    step 2) and the level descriptors in precision `prec`.  With `reuse`,
    the roots and eigen-triplets of an earlier set-up of the same workload
    are taken over (the set-up is always FP64).  A top level with hi = SOLVE
    gets a deflated PP-GMRES(gmres_m) solver (FP32 inner cycles when prec is
    FP32, FP64 residual) converging to solve_tol (rtolle).  Links that are
    SU(3) to 1e-12 are read as two rows (two_row_links).  A level's device
    buffers hold at most max_batch vectors; a step draws its samples in
    samples / batch batches.  Set-up parameters not given here come from
    cfg.extra, else SETUP_DEFAULTS.  With `resume`, a checkpoint written by
    save_checkpoint supplies the set-up and every level's Monte Carlo state
    (see there)."""
    t0 = time.perf_counter()
    state = None
    if resume is not None:
        reuse, state = _load_checkpoint(resume, cfg)
    given = dict(pin_degree=pin_degree, arnoldi_m=arnoldi_m, rtolev=rtolev, nev=nev, rtolpoly1=rtolpoly1,
                 gmres_m=gmres_m, solve_tol=solve_tol, solve_rb=None)
    prm = {k: (given[k] if given[k] is not None else cfg.extra.get(k, d)) for k, d in SETUP_DEFAULTS.items()}
    pin_degree, arnoldi_m, rtolev, nev = prm["pin_degree"], prm["arnoldi_m"], prm["rtolev"], prm["nev"]
    rtolpoly1, gmres_m, solve_tol = prm["rtolpoly1"], prm["gmres_m"], prm["solve_tol"]
    U = synth.config_links(cfg)
    canon = torch.from_numpy(U).cuda()
    V = cfg.volume

    # SU(3) links need only two rows in the kernels (row 2 = conj(row 0 x row 1))
    g64 = torch.empty(36 * V, dtype=torch.complex128, device="cuda")
    L.pack_gauge(cfg.dims, L.F64, canon, g64)
    du, dd = L.gauge_unitarity(cfg.dims, L.F64, g64)
    link_rows = 2 if (two_row_links and max(du, dd) <= 1e-12) else 3

    def lattice(p):
        if p == L.F64:
            g = g64
        else:
            g = torch.empty(36 * V, dtype=L.complex_dtype(p), device="cuda")
            L.pack_gauge(cfg.dims, p, canon, g)
        return L.DeviceLattice(tuple(cfg.dims), cfg.kappa, cfg.antiperiodic_t, p, g, link_rows)

    polys = [p for lv in cfg.levels for p in (lv.hi, lv.lo) if p is not None and p != SOLVE]
    comp_keys = sorted({p for p in polys if isinstance(p, tuple)})
    degrees = sorted({p for p in polys if isinstance(p, int)} | {p[0] - 1 for p in comp_keys})
    if comp_keys and pin_degree is None:
        pin_degree = comp_keys[0][0] - 1          # PP(dp_in + 1) of the composite (Sec. 5 step 2b)
    comps: Dict[tuple, krylov.OuterRoots] = {}
    if reuse is not None:
        roots = reuse.roots
        defl = None
        if reuse.defl is not None:
            d0 = reuse.defl
            defl = krylov.Deflation(L.DeviceDefl(d0.device.k, reuse.defl64_V, d0.device.pair, d0.device.scale,
                                                 d0.device.hinv), d0.lam, d0.pair, d0.res_right, d0.res_left,
                                    d0.candidates, d0.arnoldi_steps, d0.arnoldi_residual)
        comps = reuse.composites
        dl64 = None
    else:
        dl64 = lattice(L.F64)
        start = synth.gaussian_start(cfg.n, cfg.seed_start)
        roots = krylov.gmres_roots(dl64, degrees, start)
        defl = None
        if cfg.k_defl > 0:
            pd = pin_degree if pin_degree is not None else degrees[len(degrees) // 2]
            if pd not in roots.device:
                extra = krylov.gmres_roots(dl64, [pd], start)
                roots.inv_roots[pd], roots.device[pd] = extra.inv_roots[pd], extra.device[pd]
            defl = krylov.pp_arnoldi_deflation(dl64, roots.device[pd], start, arnoldi_m, nev, cfg.k_defl,
                                               rtolev=rtolev)
        for key in comp_keys:
            n_in, n_out = key
            comps[key] = krylov.pp_outer_roots(dl64, roots.device[n_in - 1], roots.inv_roots[n_in - 1], defl,
                                               n_out, L.Noise(cfg.seed_noise, cfg.lattice_id, 1000, 0),
                                               rtol=rtolpoly1)
    defl64_V = defl.device.V if defl is not None else None
    dl = dl64 if (prec == L.F64 and dl64 is not None) else lattice(prec)
    if defl is not None and prec != L.F64:
        kp = defl.device.kpad
        canon_v = torch.empty((kp, V, 4, 3), dtype=torch.complex128, device="cuda")
        L.unpack_fields(cfg.dims, L.F64, defl.device.V, canon_v)
        Vp = torch.empty((1, 12, V, kp), dtype=L.complex_dtype(prec), device="cuda")
        L.pack_fields(cfg.dims, prec, canon_v, Vp)    # eigenvectors rounded to the field precision
        defl.device = L.DeviceDefl(defl.device.k, Vp, defl.device.pair, defl.device.scale, defl.device.hinv)
    run = LatticeRun(cfg, prec, rb, dl, roots, defl)
    run.defl64_V = defl64_V
    run.composites = comps
    run.setup_params = prm

    def mvps(p) -> int:
        # a double polynomial stopped by rtolpoly1 has fewer outer roots than configured
        if isinstance(p, tuple):
            return p[0] * comps[p].n_out - 1
        return poly_mvps(p)
    for i, lv in enumerate(cfg.levels):
        if lv.hi == SOLVE:
            srb = int(prm["solve_rb"])
            N = _batch_size(lv.samples, srb, max_batch)
            # Tr(A^{-1} - Q) with Q the deflated p_1 (Sec. 4.3): the deflation is in Q,
            # so the samples carry no Monte Carlo deflation term
            lo = _device_poly(roots, comps, lv.lo)
            kind_lo = L.OP_DEFLATED_POLY if (lv.deflated and defl is not None) else L.OP_POLY
            x64 = L.empty_field(V, N, srb, L.F64)
            xl = x64 if prec == L.F64 else L.empty_field(V, N, srb, prec)
            dlev = L.DeviceLevel(L.OP_SOLVE, None, kind_lo, lo, defl.device if defl is not None else None,
                                 False, None, xl)
            n_in = lv.lo[0] if isinstance(lv.lo, tuple) else (pin_degree or lv.lo) + 1
            l64 = dl64 if dl64 is not None else (dl if prec == L.F64 else lattice(L.F64))
            dl64 = l64
            solver = MixedPPGMRES(l64, dl, roots.device[n_in - 1], defl.device if defl is not None else None,
                                  gmres_m, N, srb)
            ws = L.workspace(L.level_workspace_size(dl, dlev, N, srb))
            st = LevelState(i, dlev, mvps(lv.lo), None, torch.zeros(8, dtype=torch.float64, device="cuda"),
                            torch.empty((N, 6), dtype=torch.float64, device="cuda"), ws, solver=solver,
                            b64=L.empty_field(V, N, srb, L.F64), x64=x64, xl=xl, solve_tol=solve_tol, batch=N,
                            rb=srb)
            run.levels.append(st)
            continue
        N = _batch_size(lv.samples, rb, max_batch)
        hi = _device_poly(roots, comps, lv.hi)
        lo = _device_poly(roots, comps, lv.lo) if lv.lo is not None else None
        c = None
        if lv.deflated and defl is not None:
            c = _poly_value(roots, comps, lv.hi, defl.lam)
            if lv.lo is not None:
                c = c - _poly_value(roots, comps, lv.lo, defl.lam)
        dlev = L.DeviceLevel(L.OP_POLY, hi, L.OP_POLY if lo is not None else L.OP_NONE, lo,
                             defl.device if c is not None else None, c is not None,
                             krylov._c(c) if c is not None else None)
        ws = L.workspace(L.level_workspace_size(dl, dlev, N, rb))
        run.levels.append(LevelState(i, dlev, mvps(lv.hi) + mvps(lv.lo), c,
                                     torch.zeros(8, dtype=torch.float64, device="cuda"),
                                     torch.empty((N, 6), dtype=torch.float64, device="cuda"), ws, batch=N))
    if state is not None:
        acc, drawn = state
        if len(acc) != len(run.levels):
            raise ValueError(f"checkpoint has {len(acc)} levels, the workload {len(run.levels)}")
        for lv, a, n in zip(run.levels, acc, drawn):
            lv.acc.copy_(torch.from_numpy(np.ascontiguousarray(a)))
            lv.drawn = int(n)
    torch.cuda.synchronize()
    run.setup_seconds = time.perf_counter() - t0
    if verbose:
        print(f"setup {cfg.name}: {run.setup_seconds:.1f} s, k_defl={defl.device.k if defl else 0}, "
              f"GMRES residuals {roots.residual}", flush=True)
    return run


# ------------------------------------------------------------------ checkpoint / resume
CHECKPOINT_VERSION = 1


def _identity(cfg: LatticeConfig) -> dict:
    return {"name": cfg.name, "dims": list(cfg.dims), "kappa": cfg.kappa, "eps": cfg.eps,
            "antiperiodic_t": bool(cfg.antiperiodic_t), "seed_links": cfg.seed_links, "seed_start": cfg.seed_start,
            "seed_noise": cfg.seed_noise, "lattice_id": cfg.lattice_id,
            "levels": [[str(lv.hi), str(lv.lo), int(lv.samples), bool(lv.deflated)] for lv in cfg.levels]}


def save_checkpoint(run: LatticeRun, path: str) -> None:
    """Write a run's Monte Carlo state and set-up to `path` (numpy .npz, no
    pickled objects): per level the FP64 accumulator (n, mean, M2,
    non-finite count) and the next sample index; the GMRES roots, the
    deflation triplets (FP64 right eigenvectors, pair, scale, H^{-1},
    eigenvalues) and the outer roots of the double polynomials.  The noise
    is counter-based, so build(cfg, resume=path) continues with exactly the
    samples the uninterrupted run would have drawn and merges them into the
    same accumulators."""
    torch.cuda.synchronize()
    d = {"meta": np.array(json.dumps({"version": CHECKPOINT_VERSION, "config": _identity(run.cfg)}))}
    degs = sorted(run.roots.inv_roots)
    d["root_degrees"] = np.array(degs, dtype=np.int64)
    d["root_residuals"] = np.array([run.roots.residual[k] for k in degs], dtype=np.float64)
    for k in degs:
        d[f"root_{k}"] = np.asarray(run.roots.inv_roots[k], dtype=np.complex128)
    keys = sorted(run.composites)
    d["composite_keys"] = np.array(keys, dtype=np.int64).reshape(-1, 2)
    d["composite_residuals"] = np.array([run.composites[k].residual for k in keys], dtype=np.float64)
    for k in keys:
        d[f"outer_{k[0]}_{k[1]}"] = np.asarray(run.composites[k].inv_roots, dtype=np.complex128)
    if run.defl is not None:
        df = run.defl
        d["defl_V"] = run.defl64_V.cpu().numpy()
        d["defl_pair"] = df.device.pair.cpu().numpy()
        d["defl_scale"] = df.device.scale.cpu().numpy()
        d["defl_hinv"] = df.device.hinv.cpu().numpy()
        d["defl_lam"] = np.asarray(df.lam)
        d["defl_res"] = np.stack([np.asarray(df.res_right), np.asarray(df.res_left)])
        d["defl_counts"] = np.array([df.device.k, df.candidates, df.arnoldi_steps], dtype=np.int64)
        d["defl_arnoldi_residual"] = np.array(df.arnoldi_residual)
    d["acc"] = np.stack([lv.acc.cpu().numpy() for lv in run.levels])
    d["drawn"] = np.array([lv.drawn for lv in run.levels], dtype=np.int64)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **d)
    os.replace(tmp, path)


def _load_checkpoint(path: str, cfg: LatticeConfig):
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        if meta.get("version") != CHECKPOINT_VERSION:
            raise ValueError(f"{path}: checkpoint version {meta.get('version')}, expected {CHECKPOINT_VERSION}")
        if meta["config"] != json.loads(json.dumps(_identity(cfg))):
            raise ValueError(f"{path} was written for another workload: {meta['config']['name']}")
        degs = [int(k) for k in z["root_degrees"]]
        inv = {k: z[f"root_{k}"].copy() for k in degs}
        roots = krylov.RootSet(inv, {k: L.DevicePoly(krylov._c(inv[k])) for k in degs},
                               {k: float(r) for k, r in zip(degs, z["root_residuals"])})
        comps = {}
        for (n_in, n_out), res in zip(z["composite_keys"], z["composite_residuals"]):
            key = (int(n_in), int(n_out))
            out = z[f"outer_{key[0]}_{key[1]}"].copy()
            comps[key] = krylov.OuterRoots(out, L.DevicePoly(krylov._c(inv[key[0] - 1]), krylov._c(out)), float(res))
        saved = types.SimpleNamespace(roots=roots, composites=comps, defl=None, defl64_V=None)
        if "defl_V" in z:
            k, cand, steps = (int(v) for v in z["defl_counts"])
            V64 = torch.from_numpy(z["defl_V"].copy()).cuda()
            dev = L.DeviceDefl(k, V64, torch.from_numpy(z["defl_pair"].copy()).cuda(),
                               torch.from_numpy(z["defl_scale"].copy()).cuda(),
                               torch.from_numpy(z["defl_hinv"].copy()).cuda())
            saved.defl = krylov.Deflation(dev, z["defl_lam"].copy(), z["defl_pair"].copy(), z["defl_res"][0].copy(),
                                          z["defl_res"][1].copy(), cand, steps, float(z["defl_arnoldi_residual"]))
            saved.defl64_V = V64
        return saved, (z["acc"].copy(), z["drawn"].copy())


def time_to_error(variances, seconds_per_sample, eps: float) -> float:
    """Wall time to a combined standard error eps with the optimal sample
    allocation of multilevel Monte Carlo: T = eps^-2 (sum_l sqrt(V_l t_l))^2
    (the cost formula eq. mlevcost of Sec. 5 with measured time as cost)."""
    s = sum(np.sqrt(max(v, 0.0) * t) for v, t in zip(variances, seconds_per_sample))
    return float(s * s / eps ** 2)


def level_targets(eps: float, stderrs) -> List[float]:
    """Standard-error targets of the levels, top first, for a total error eps
    (Sec. 5 step 3): level l gets sqrt(eps^2 - e^2) / sqrt(L - l), e^2 the
    summed squared standard errors of the levels before it.  With three
    levels this is eps/sqrt(3), then sqrt(eps^2 - e_1^2)/sqrt(2), then
    sqrt(eps^2 - e_1^2 - e_2^2)."""
    nl = len(stderrs)
    out, e2 = [], 0.0
    for l in range(nl):
        out.append(float(np.sqrt(max(eps * eps - e2, 0.0)) / np.sqrt(nl - l)))
        e2 += float(stderrs[l]) ** 2
    return out


def check_points(level: int, nmax: int) -> List[int]:
    """Sample counts at which a level's standard error is checked (Sec. 5
    step 3): the first Monte Carlo from 2 noises after every noise, the second
    at 3 and then every 3, every later one at 6 and then every 3."""
    if level == 0:
        return list(range(2, nmax + 1))
    if level == 1:
        return list(range(3, nmax + 1, 3))
    return list(range(6, nmax + 1, 3))


def stopping_index(s: np.ndarray, target: float, level: int, start: int = 0) -> Optional[int]:
    """Smallest check point n > start (within len(s)) at which the standard
    error of the first n complex samples, sqrt(sum |s - mean|^2 / (n-1) / n),
    is at most target; None if there is none yet."""
    s = np.asarray(s, dtype=np.complex128)
    if len(s) == 0:
        return None
    s = s - s[0]           # the variance is shift-invariant; the shift keeps the running sums small
    c1 = np.cumsum(s)
    c2 = np.cumsum(np.abs(s) ** 2)
    for n in check_points(level, len(s)):
        if n <= start:
            continue
        mean = c1[n - 1] / n
        m2 = max(c2[n - 1] - n * abs(mean) ** 2, 0.0)
        if np.sqrt(m2 / (n - 1) / n) <= target:
            return n
    return None


@dataclass
class AdaptiveLevel:
    n: int                 # samples the estimate uses (the stopping point)
    drawn: int             # samples computed on the GPU (whole batches)
    estimate: complex
    stderr: float
    target: float
    seconds: float


def check_rule(level: int):
    """(first, every) of a level's check points (check_points)."""
    if level == 0:
        return 2, 1
    if level == 1:
        return 3, 3
    return 6, 3


def run_to_tolerance(run: LatticeRun, eps: float, first_batch: int = 32,
                     max_samples: int = 1 << 20, probe_last: bool = False, graphs: bool = False,
                     lookahead: int = 1) -> List[AdaptiveLevel]:
    """The multilevel Monte Carlo of Sec. 5 step 3 on the GPU: levels top
    first, each drawing batches of Z4 samples until its standard error falls
    to its share of eps (level_targets, given the errors of the levels before
    it) at one of its check points.  The check runs on the device after every
    batch (mpmc_level_stop_check: one sample at a time, so the estimate uses
    exactly the samples up to the stopping point, as the paper's loop would);
    the host reads back 128 bytes per batch.  Up to `lookahead` further
    batches are enqueued before a batch's check is read, but only while the
    running error predicts that the samples already enqueued fall short of
    the target (a batch enqueued after the stop would be wasted work, not a
    wrong result).  Batches start at first_batch and double up to the level's
    configured batch (a solve level always draws its full batch).  With
    graphs, each batch of a polynomial level is one launch of a step
    recorded by the library (mpmc_batch_build: the level, its stopping check
    and its sample counter).  With probe_last, the last level Tr p_d(A) is
    computed exactly by probing with a distance-d colouring (Sec. 5 step 3d;
    its standard error is 0) and eps is split over the Monte Carlo levels
    only.  Returns one AdaptiveLevel per level."""
    out: List[AdaptiveLevel] = []
    errs: List[float] = []
    nl = len(run.levels)
    last = run.cfg.levels[-1]
    if probe_last and not (last.lo is None and isinstance(last.hi, int)):
        raise ValueError("probing needs a last level Tr p_d(A) of a single polynomial")
    nmc = nl - 1 if probe_last else nl
    run.reset()
    host = torch.zeros((lookahead + 1, 16), dtype=torch.float64, pin_memory=True)
    for li, lv in enumerate(run.levels):
        if li == nmc:
            t0 = time.perf_counter()
            col = probing.colouring(run.cfg.dims, int(last.hi))
            pr = probing.probe_trace(run.dl, lv.device.poly_hi, col, nrhs=lv.batch)
            out.append(AdaptiveLevel(pr.probes, pr.probes, pr.trace, 0.0, 0.0, time.perf_counter() - t0))
            break
        target = level_targets(eps, errs + [0.0] * (nmc - len(errs)))[li]
        first, every = check_rule(li)
        N = lv.batch
        rb = run.level_rb(li)
        batch = N if lv.solver is not None else max(rb, min(N, (first_batch // rb) * rb or rb))
        state = run.adaptive.setdefault(("state", li), torch.zeros(16, dtype=torch.float64, device="cuda"))
        state.zero_()
        state[7] = float(target)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending: List[tuple] = []
        have, k, stopped = 0, 0, False
        need = None             # samples the running error predicts, from the last state read
        while True:
            # enqueue when nothing is in flight, or (pipelined) when the samples already enqueued
            # are predicted not to reach the target, so the next batch is not wasted work
            more = have < max_samples and (not pending or (len(pending) <= lookahead and need is not None
                                                            and need > have))
            if more:
                if graphs and lv.solver is None:
                    key = ("step", li, batch, first, every)
                    if key not in run.adaptive:
                        run.adaptive[key] = _stop_step(run, li, batch, state, first, every)
                    h, ctr = run.adaptive[key]
                    ctr.fill_(have)
                    L.batch_launch(h)
                    lv.drawn += batch
                else:
                    run.draw(li, batch)
                    L.level_stop_check(lv.samples, batch, first, every, state)
                slot = host[k % (lookahead + 1)]
                slot.copy_(state, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record()
                pending.append((ev, slot))
                have += batch
                k += 1
                if lv.solver is None and batch < N:
                    batch = min(N, 2 * batch)
                continue
            if not pending:
                break
            ev, slot = pending.pop(0)
            ev.synchronize()
            if slot[4].item() != 0.0:
                stopped = True
                break
            n_read, m2 = float(slot[0].item()), float(slot[3].item())
            if n_read >= 2 and target > 0:
                need = int(np.ceil(m2 / (n_read - 1) / target ** 2))     # n with stderr^2 = var / n = target^2
        torch.cuda.synchronize()
        st = state.cpu().numpy()
        if stopped or st[4] != 0.0:
            n, mean, m2 = int(st[5]), complex(st[8], st[9]), float(st[10])
        else:
            n, mean, m2 = int(st[0]), complex(st[1], st[2]), float(st[3])
        corr = complex(np.sum(lv.c)) if lv.c is not None else 0.0
        se = float(np.sqrt(m2 / (n - 1) / n)) if n > 1 else float("inf")
        errs.append(se)
        out.append(AdaptiveLevel(n, have, mean + corr, se, float(target), time.perf_counter() - t0))
    return out


def prepare_adaptive(run: LatticeRun, first_batch: int = 32):
    """Record, ahead of a timed run_to_tolerance(graphs=True), every
    one-batch step the adaptive loop can launch (batch sizes first_batch
    doubling to each polynomial level's batch): recording is set-up."""
    for li, lv in enumerate(run.levels):
        if lv.solver is not None:
            continue
        state = run.adaptive.setdefault(("state", li), torch.zeros(16, dtype=torch.float64, device="cuda"))
        first, every = check_rule(li)
        rb, N = run.level_rb(li), lv.batch
        batch = max(rb, min(N, (first_batch // rb) * rb or rb))
        while True:
            key = ("step", li, batch, first, every)
            if key not in run.adaptive:
                run.adaptive[key] = _stop_step(run, li, batch, state, first, every)
            if batch >= N:
                break
            batch = min(N, 2 * batch)


def _stop_step(run: LatticeRun, level: int, batch: int, state: torch.Tensor, first: int, every: int):
    """A recorded one-level step for the adaptive loop: one batch of `batch`
    samples starting at the sample counter, its stopping check, the counter
    advanced (mpmc_batch_build)."""
    lv = run.levels[level]
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    h = L.Handle()
    item = L.BatchItem(run.dl, lv.device, batch, run.level_rb(level),
                       L.Noise(run.cfg.seed_noise, run.cfg.lattice_id, lv.index, 0), ctr, 1, lv.samples[:batch],
                       lv.acc, lv.ws, 0, int(lv.sweep), int(lv.sweep_rank),
                       int(lv.sweep_chunks),
                       state, first, every)
    L.batch_build(h, [item])
    return h, ctr

