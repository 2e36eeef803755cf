"""Benchmark of the multipolynomial Monte Carlo hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f64|f32]

Workload: the 8^4 Wilson-Dirac lattice (n = 49152, eps = 0.3 links, periodic
time, kappa with |lambda_min| = 1e-3), three levels Tr(p150 - p30) and
Tr(p30 - p8) with 20 deflation eigenvectors and Tr(p8), 256 Z4 samples per
level, FP64.  A step is one pass of every level over its batch: noise
generation, deflation coefficient GEMMs, the polynomial applications (fused
Wilson-Dirac + Newton + FP64 dot kernels) and the FP64 level reductions.
Set-up (GMRES roots, PP-Arnoldi eigenvectors, on the GPU) is done before the
timed region and reported separately.

Prints one JSON line (rank 0): value = algorithmic HBM GB/s of the operator
applications of the whole step, a roofline object for the dominant kernel
(the fused Newton step) and a cpu_baseline object (the FP64 oracle on a
bounded sample of the same workload, on the host cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL = "k_sweep (t-sweep Wilson-Dirac + Newton step + FP64 b^H w partial)"
KERNEL_SOURCES = ("sweep.hip", "common.hpp")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--rb", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-bulk (mixed) comparison run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched independent lattices and the top-level solve measurements")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the 24^3x48 four-level workload (set-up ~20 s, ~190 GiB of HBM)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="print only the oracle's CPU rate (used for the one-thread figure)")
    ap.add_argument("--probe", choices=["gemm", "hop", "sweep"], default=None,
                    help="measurement helper for profiling runs: time the deflation GEMMs at the 8^4 and "
                         "24^3x48 workloads' sizes (gemm), the streaming kernel on the 16^4 / 12^3x24 / "
                         "24^3x48 lattices (hop), or the blocked FP32 t-sweep on 24^3x48 and 16^4 (sweep), "
                         "then exit")
    ap.add_argument("--reps", type=int, default=10, help="repetitions of each probe call")
    ap.add_argument("--hop-orders", default="0,1",
                    help="work orders (MPMC_OPT_HOP_SLAB values) the hop probe times, comma-separated")
    ap.add_argument("--c4-only", action="store_true", help="run only the 24^3x48 workload (profiling runs)")
    ap.add_argument("--c5-only", action="store_true",
                    help="run only the four independent lattices in one graph (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2306_09559_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(prec: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), if it
    was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"k_sweep_c2_{prec}_traffic.md")
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def calibrate_copy():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB), three times:
    the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def copy_bandwidth_gbs(reps: int = 10) -> float:
    """Measured HBM bandwidth of a plain device copy on this GPU (the
    library's streaming copy, mpmc_field_copy_bytes): 1 GiB read and 1 GiB
    written per copy, timed with HIP events over `reps` copies."""
    import torch
    from paper_2306_09559_amd import _lib as L
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    L.field_copy_bytes(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        L.field_copy_bytes(a, b)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2 * (1 << 30) / sec / 1e9


def cpu_baseline(cfg, run_prec: str):
    """The oracle (plain C FP64, OpenMP over sites) on a bounded sample of the
    same workload: rounds of one Z4 sample per level (every polynomial of
    the level applied) until about 12 s have passed, roots from the oracle's
    own GMRES (not timed).  Scaled to the metric's unit (algorithmic GB/s)."""
    import numpy as np
    import oracle
    import synth
    from oracle import krylov as okr
    U = synth.gauge_links(cfg.dims, cfg.eps, cfg.seed_links)
    lat = oracle.Lattice(cfg.dims, cfg.kappa, U, cfg.antiperiodic_t)
    degs = sorted({d for lv in cfg.levels for d in (lv.hi, lv.lo) if isinstance(d, int)})
    ps = okr.gmres_polys(lat.apply, synth.gaussian_start(lat.n, cfg.seed_start), degs)
    t0 = time.perf_counter()
    mvps = 0
    nsamp = 0
    while time.perf_counter() - t0 < 12.0 and nsamp < cfg.levels[0].samples:
        for li, lv in enumerate(cfg.levels):
            b = oracle.z4(cfg.seed_noise, cfg.lattice_id, li, nsamp, 1, lat.V)
            lat.poly_apply(ps.inv_roots[lv.hi], b)
            mvps += lv.hi
            if lv.lo is not None:
                lat.poly_apply(ps.inv_roots[lv.lo], b)
                mvps += lv.lo
        nsamp += 1
    dt = time.perf_counter() - t0
    # the same algorithmic bytes per MVP on one vector as the GPU metric counts
    # for the workload's batches of N vectors (FP64)
    N = cfg.levels[0].samples
    byts = mvps * lat.V * (24 * 16 + 36 * 16 / N)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(byts / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsamp} Z4 samples of each level (p150, p30, p8 Newton applications, {mvps} MVPs), "
                      f"no deflation GEMM, FP64; {dt:.1f} s"}


def probe_gemm(reps: int):
    """The deflation GEMMs (k_coeff: zeta = V^H b and omega = U^H b with the
    Z4 noise b regenerated; k_recon: X = V d) at the 8^4 workload's size
    (FP64, k = 20 padded to 32, 256 vectors) and the 24^3x48 workload's size
    (FP32, k = 128, 128 vectors); Z4 vectors stand in for the eigenvectors
    (the GEMMs do not depend on the values).  Algorithmic flops 8 n k N."""
    import numpy as np
    import torch
    from paper_2306_09559_amd import _lib as L
    cases = [("8^4 f64", (8, 8, 8, 8), L.F64, 20, 32, 256, 16), ("24^3x48 f32", (24, 24, 24, 48), L.F32, 128, 128, 128, 16)]
    out = []
    for name, dims, prec, k, kpad, N, rb in cases:
        V = int(np.prod(dims))
        n = 12 * V
        g = torch.zeros(36 * V, dtype=L.complex_dtype(prec), device="cuda")
        dl = L.DeviceLattice(dims, 0.13, True, prec, g, 3)
        Vf = L.empty_field(V, kpad, kpad, prec)
        L.z4_fill(dims, prec, L.Noise(5, 6, 7, 0), Vf)
        D = L.DeviceDefl(k, Vf, torch.arange(k, dtype=torch.int32, device="cuda"),
                         torch.ones(k, dtype=torch.complex128, device="cuda"), None)
        ws = L.workspace(L.deflate_workspace_size(dl, D, N, rb))
        zeta = torch.empty((k, N), dtype=torch.complex128, device="cuda")
        omega = torch.empty((k, N), dtype=torch.complex128, device="cuda")
        d = torch.ones((k, N), dtype=torch.complex128, device="cuda")
        X = L.empty_field(V, N, rb, prec)
        nz = L.Noise(1, 2, 3, 0)
        row = {"case": name, "n": n, "k": k, "kpad": kpad, "N": N}
        for mode, label in ((L.DEFL_COEFF, "coeff"), (L.DEFL_RECON, "recon")):
            def call():
                if mode == L.DEFL_COEFF:
                    L.deflate_project(dl, D, mode, N, rb, None, nz, zeta, omega, None, None, ws)
                else:
                    L.deflate_project(dl, D, mode, N, rb, None, None, None, None, d, X, ws)
            call()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / reps
            row[label] = {"ms": round(sec * 1e3, 4), "TFLOPs": round(8.0 * n * k * N / sec / 1e12, 2)}
        out.append(row)
        del Vf, X, ws
        torch.cuda.empty_cache()
    return out


def probe_hop(reps: int, orders=(0, 1)):
    """The streaming kernel (k_hop, scalar-mode Newton steps of a degree-10
    polynomial, t-sweep off) on the lattices it runs: 16^4 x 16 and
    12^3x24 x 8 vectors (FP32), 24^3x48 x 1 vector (FP64, the set-up's
    operator), 24^3x48 x 128 and 8^4 x 256 vectors (FP32), each in the plain
    and the slab work order (MPMC_OPT_HOP_SLAB 0, 1; `orders`).
    Algorithmic bytes per launch: the spinors in and out (V N 24 c, the first
    step V N 12 c: its input is drawn in the kernel) and the two-row links
    (V 24 c); the mean over the 10 launches of a polynomial is reported."""
    import numpy as np
    import torch
    import synth
    from paper_2306_09559_amd import _lib as L
    cases = [((16, 16, 16, 16), L.F32, 16, 16), ((12, 12, 12, 24), L.F32, 8, 8), ((24, 24, 24, 48), L.F64, 1, 1),
             ((24, 24, 24, 48), L.F32, 128, 16), ((8, 8, 8, 8), L.F32, 256, 16)]
    prev = L.get_option(L.OPT_PLANE_SWEEP)
    L.set_option(L.OPT_PLANE_SWEEP, 0)
    out = []
    for dims, prec, N, rb in cases:
        V = int(np.prod(dims))
        csz = 16 if prec == L.F64 else 8
        U = synth.gauge_links(dims, 0.5, 7)
        g = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
        L.pack_gauge(dims, prec, torch.from_numpy(U).cuda(), g)
        del U
        dl = L.DeviceLattice(dims, 0.14, True, prec, g, 2)
        poly = L.DevicePoly(torch.from_numpy(np.linspace(0.3, 0.9, 11) + 0.05j).cuda())
        ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
        bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
        nz = L.Noise(1, 2, 3, 0)
        byts = (9 * V * N * 24 * csz + V * N * 12 * csz) // 10 + V * 24 * csz
        for slab in orders:
            L.set_option(L.OPT_HOP_SLAB, slab)
            L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / (reps * 10)
            out.append({"dims": list(dims), "prec": "f64" if prec == L.F64 else "f32", "N": N, "rb": rb,
                        "order": slab, "bytes_per_launch": byts, "us_per_launch": round(us, 2),
                        "GBps": round(byts / us / 1e3, 1)})
            print(json.dumps(out[-1]), file=sys.stderr, flush=True)
        del ws, g
        torch.cuda.empty_cache()
    L.set_option(L.OPT_HOP_SLAB, 1)
    L.set_option(L.OPT_PLANE_SWEEP, prev)
    return out


def probe_sweep(reps: int):
    """The blocked FP32 t-sweep (scalar-mode Newton steps of a degree-10
    polynomial) on the 24^3x48 lattice at 256 and 32 vectors and on 16^4 x
    16 vectors, for each of the first three ranked blocks
    (MPMC_OPT_SWEEP_RANK).  Algorithmic bytes as for the streaming probe."""
    import numpy as np
    import torch
    import synth
    from paper_2306_09559_amd import _lib as L
    cases = [((24, 24, 24, 48), 256, 16), ((24, 24, 24, 48), 32, 16), ((16, 16, 16, 16), 16, 16)]
    prev = L.get_option(L.OPT_PLANE_SWEEP)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    out = []
    for dims, N, rb in cases:
        V = int(np.prod(dims))
        csz = 8
        U = synth.gauge_links(dims, 0.5, 7)
        g = torch.empty(36 * V, dtype=L.complex_dtype(L.F32), device="cuda")
        L.pack_gauge(dims, L.F32, torch.from_numpy(U).cuda(), g)
        del U
        dl = L.DeviceLattice(dims, 0.14, True, L.F32, g, 2)
        poly = L.DevicePoly(torch.from_numpy(np.linspace(0.3, 0.9, 11) + 0.05j).cuda())
        ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
        bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
        nz = L.Noise(1, 2, 3, 0)
        byts = (9 * V * N * 24 * csz + V * N * 12 * csz) // 10 + V * 24 * csz
        for rank in (0, 1, 2):
            L.set_option(L.OPT_SWEEP_RANK, rank)
            plan = L.sweep_plan(dl, N, rb)
            L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / (reps * 10)
            out.append({"dims": list(dims), "N": N, "rb": rb, "rank": rank, "plan": plan,
                        "bytes_per_launch": byts, "us_per_launch": round(us, 2), "GBps": round(byts / us / 1e3, 1)})
            print(json.dumps(out[-1]), file=sys.stderr, flush=True)
        del ws, g
        torch.cuda.empty_cache()
    L.set_option(L.OPT_SWEEP_RANK, 0)
    L.set_option(L.OPT_PLANE_SWEEP, prev)
    return out


def cpu_baseline_one_thread():
    """The same oracle sample on one host thread (a child process with
    OMP_NUM_THREADS=1; about 12 s)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-baseline-only"], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def timed_steps(run, steps, stream):
    """Run `steps` steps from sample 0 with per-level HIP events on `stream`.
    Returns (wall seconds, per-level milliseconds summed over steps)."""
    import numpy as np
    import torch
    nl = len(run.levels)
    run.reset()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nl)]
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        for i in range(nl):
            ev[k][i][0].record(stream)
            for _ in range(run.batches(i)):
                run.draw(i, run.levels[i].batch)
            ev[k][i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lvl_ms = np.array([sum(ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(steps)) for i in range(nl)])
    return wall, lvl_ms


def kernel_launch_seconds(run, steps: int, stream) -> float:
    """Average duration of one launch of the dominant kernel, from HIP events
    on `stream`: scalar-mode applications of the top level's high-degree
    polynomial (one t-sweep launch per operator application, plus one tiny
    reduction) to the level's batch of Z4 vectors."""
    import torch
    from paper_2306_09559_amd import _lib as L
    lv = run.levels[0]
    poly = lv.device.poly_hi
    prev = L.get_option(L.OPT_PLANE_SWEEP)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    N = run.cfg.levels[0].samples
    ws = L.workspace(L.poly_workspace_size(run.dl, poly, N, run.rb))
    bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
    nz = L.Noise(run.cfg.seed_noise, run.cfg.lattice_id, 99, 0)
    L.poly_apply(run.dl, poly, N, run.rb, None, nz, None, bhy, ws)      # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        L.poly_apply(run.dl, poly, N, run.rb, None, nz, None, bhy, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    L.set_option(L.OPT_PLANE_SWEEP, prev)
    launches = steps * (int(poly.inv_in.numel()) - 1)
    return e0.elapsed_time(e1) * 1e-3 / launches


def graph_level_seconds(run, reps: int):
    """Per-sample seconds of each level when its batch is replayed as a HIP graph."""
    import torch
    from paper_2306_09559_amd.batch import GraphStep
    out = []
    for li in range(len(run.levels)):
        gs = GraphStep([run], parallel=False, only=[(0, li)])
        gs.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gs.replay(reps)
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) * 1e-3 / (reps * run.cfg.levels[li].samples))
    run.reset()
    return out


def batched_c5(steps: int):
    """The mixed batch of independent lattices (8^4, 12^4, 16^4, 12^3x24; own
    kappa, degree and sample count), FP32 bulk: serial eager steps against one
    graph whose branches run the lattices concurrently."""
    import time
    import torch
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    from synth.configs import C5
    t0 = time.perf_counter()
    runs = [driver.build(c, prec=L.F32, rb=8) for c in C5]
    setup = time.perf_counter() - t0
    for r in runs:
        r.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in runs:
            r.step()
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / steps
    gs = GraphStep(runs, parallel=True)
    gs.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs.replay(steps)
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / steps
    # the same graph after the library's autotuner picked every lattice's shape
    from paper_2306_09559_amd.batch import autotune
    t0 = time.perf_counter()
    tunes = [autotune(r, reps=3, use_cache=False) for r in runs]
    tune_s = time.perf_counter() - t0
    gt = GraphStep(runs, parallel=True)
    gt.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gt.replay(steps)
    torch.cuda.synchronize()
    tuned = (time.perf_counter() - t0) / steps
    mvp = sum(r.mvp_rhs_per_step() for r in runs)
    byts = sum(r.bytes_per_step() for r in runs)
    return {"lattices": [f"{'x'.join(map(str, c.dims))} k={c.kappa} deg {c.levels[0].hi} N={c.levels[0].samples}"
                         for c in C5],
            "prec": "f32", "setup_s": round(setup, 2), "mvp_rhs_per_step": mvp,
            "eager_serial_ms_per_step": round(eager * 1e3, 3), "graph_parallel_ms_per_step": round(graph * 1e3, 3),
            "speedup": round(eager / graph, 3), "graph_GBps": round(byts / graph / 1e9, 1),
            "autotuned": {"tune_s": round(tune_s, 2), "graph_parallel_ms_per_step": round(tuned * 1e3, 3),
                          "graph_GBps": round(byts / tuned / 1e9, 1),
                          "shapes": [{"rb": t.choice[0][0], "sweep": t.choice[0][1], "block_rank": t.choice[0][2],
                                      "t_chunks": t.choice[0][3]}
                                     for t in tunes]}}


def fp64_level_errors(run32, levels, nsamp: int, targets):
    """Each level's error against FP64 on the same noise: the mixed-precision
    run and an FP64 run built on the same set-up (roots, eigen-triplets,
    outer roots) each draw samples 0 .. nsamp-1 of the level; reported are the
    largest per-sample error of s relative to |b^H P_hi b| + |b^H P_lo b| and
    |mean_mixed - mean_FP64| against the level's standard-error target (the
    bound is 0.1 of it).  Also returns the FP64 run for reuse."""
    import numpy as np
    import torch
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    run64 = driver.build(run32.cfg, prec=L.F64, rb=run32.rb, reuse=run32, max_batch=nsamp)
    out = []
    for li, t in zip(levels, targets):
        res = []
        for r in (run32, run64):
            r.levels[li].drawn = 0
            r.draw(li, nsamp)
            torch.cuda.synchronize()
            res.append(r.levels[li].samples[:nsamp].cpu().numpy().copy())
        a, b = res
        s32, s64 = a[:, 0] + 1j * a[:, 1], b[:, 0] + 1j * b[:, 1]
        scale = np.abs(b[:, 2] + 1j * b[:, 3]) + np.abs(b[:, 4] + 1j * b[:, 5])
        err = abs(s32.mean() - s64.mean())
        out.append({"level": li, "samples": nsamp, "max_rel_sample_error": float(f"{np.max(np.abs(s32 - s64) / scale):.3g}"),
                    "mean_error": float(f"{err:.4g}"), "target": round(float(t), 4),
                    "error_over_target": float(f"{err / t:.3g}"), "bound_met": bool(err <= 0.1 * t)})
    return out, run64


def top_level_c3(cfg=None, fp64_check=False):
    """The top level Tr(A^{-1} - p_1) of the 16^3x32 workload: one batch of 64
    Z4 vectors solved by deflated PP-GMRES (FP32 inner cycles, FP64 residual)
    and sampled against the deflated double polynomial p_1.  cfg: the regular
    set-up (default, PP(20)x15 = degree 299) or the extra-deflation one."""
    import time
    import torch
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    from synth.configs import C3
    cfg = cfg or C3
    t0 = time.perf_counter()
    run = driver.build(cfg, prec=L.F32, rb=16)
    setup = time.perf_counter() - t0
    torch.cuda.synchronize()
    N = cfg.levels[0].samples
    t0 = time.perf_counter()
    run.draw(0, N)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = run.levels[0].last_solve
    e = run.estimates()[0]
    key = cfg.levels[0].lo
    comp = run.composites[key]
    prm = run.setup_params
    var = e["stderr"] ** 2 * N
    target = 0.0005 * cfg.volume / 3 ** 0.5
    links = ("links of the 8^4 workload tiled" if cfg.extra.get("tile_from") else "eps=%g links" % cfg.eps)
    fp64 = None
    if fp64_check:
        # the top level solved and sampled in FP64 throughout, same noise, same set-up
        fp64, run64 = fp64_level_errors(run, [0], N, [target])
        del run64
        torch.cuda.empty_cache()
    return {"fp64_error": fp64, "workload": "%s %s n=%d, kappa=%.6g, %s; Tr(A^-1 - Q), Q = deflated double polynomial PP(%d)x%d "
                        "(deg %d), k=%d" % (cfg.name, "x".join(map(str, cfg.dims)), cfg.n, cfg.kappa, links, key[0],
                                            comp.n_out, key[0] * comp.n_out - 1, run.defl.device.k),
            "setup": {"seconds": round(setup, 2), "pin_degree": key[0] - 1, "arnoldi_steps": run.defl.arnoldi_steps,
                      "arnoldi_gmres_residual": float(f"{run.defl.arnoldi_residual:.3g}"),
                      "ritz_tested": run.defl.candidates, "accepted": run.defl.device.k,
                      "accepted_abs_lambda": [float(f"{abs(l):.3g}") for l in sorted(run.defl.lam, key=abs)],
                      "p1_outer_roots": comp.n_out, "p1_residual": float(f"{comp.residual:.3g}"),
                      "gmres_m": prm["gmres_m"]},
            "batch": N, "batch_s": round(dt, 3),
            "solve": {"outer_fp64": st.outer, "inner_cycles": st.cycles, "arnoldi_steps": st.arnoldi_steps,
                      "mvps_per_vector": st.mvps, "max_rel_residual": float(f"{st.rel_res.max():.3g}"),
                      "rtolle": prm["solve_tol"]},
            "estimate": [round(e["estimate"].real, 4), round(e["estimate"].imag, 4)], "stderr": round(e["stderr"], 4),
            "sample_variance": round(var, 2), "target_stderr": round(target, 3),
            # time for this level alone to reach its share eps/sqrt(3) of eps = 0.0005 V: the samples
            # that variance needs, and at least the two the first check is taken at (Sec. 5 step 3a)
            "seconds_to_target": round(max(2, math.ceil(var / target ** 2)) * dt / N, 3)}


def c4_step(steps: int = 2):
    """The 24^3x48 workload (n = 7.96M, FP32 bulk): levels Tr(p_1 - p_60),
    Tr(p_60 - p_15), Tr(p_15 - p_4) deflated and Tr(p_4), with 32 / 128 / 512
    / 2048 samples drawn in batches of at most 256 vectors, the whole step one
    HIP graph recorded by the library; then every level against FP64 on its
    first 16 samples."""
    import time
    import numpy as np
    import torch
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep
    from synth.configs import C4
    t0 = time.perf_counter()
    run = driver.build(C4, prec=L.F32, rb=16, max_batch=256)
    setup = time.perf_counter() - t0
    # one graph branch per level: launches of different levels fill each other's tails
    # (2.32 -> 2.22 s per step, same estimates)
    gs = GraphStep([run], level_branches=True)
    gs.replay()
    torch.cuda.synchronize()
    gs.reset()
    t0 = time.perf_counter()
    gs.replay(steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    est = run.estimates()
    eps = 0.0005 * C4.volume
    targets = driver.level_targets(eps, [e["stderr"] for e in est])
    del gs
    errs, run64 = fp64_level_errors(run, list(range(len(run.levels))), 16, targets)
    del run64
    torch.cuda.empty_cache()
    d = run.defl
    return {"workload": "24^3x48 n=7962624, kappa=0.15, eps=0.5 links; levels (20x15 composite)-p60, p60-p15, "
                        "p15-p4 deflated (k=%d), p4; 32/128/512/2048 samples" % d.device.k,
            "prec": "f32", "setup_s": round(setup, 1), "graph_step_s": round(dt, 3), "steps": steps,
            "mvp_rhs_per_step": run.mvp_rhs_per_step(), "GBps": round(run.bytes_per_step() / dt / 1e9, 1),
            "pct_peak": round(100 * run.bytes_per_step() / dt / 1e9 / HBM_PEAK_GBS, 2),
            "deflation": {"configured_k": C4.k_defl, "accepted_k": d.device.k, "ritz_tested": d.candidates,
                          "arnoldi_steps": d.arnoldi_steps,
                          "accepted_max_right_residual": float(f"{np.max(d.res_right):.3g}")},
            "levels": [{"estimate": [round(e["estimate"].real, 2), round(e["estimate"].imag, 2)],
                        "stderr": round(e["stderr"], 3), "n": e["n"]} for e in est],
            "level_error_vs_fp64": errs, "eps": eps}


def main():
    args = parse()
    if args.cpu_baseline_only:
        from synth.configs import C2
        print(json.dumps(cpu_baseline(C2, args.prec)), flush=True)
        return
    if args.c4_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"c4": c4_step(max(1, args.steps))}), flush=True)
        return
    if args.c5_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"batched_lattices": batched_c5(max(1, args.steps))}), flush=True)
        return
    if args.probe:
        import torch
        torch.cuda.set_device(0)
        if args.probe == "gemm":
            res = probe_gemm(args.reps)
        elif args.probe == "sweep":
            res = probe_sweep(args.reps)
        else:
            res = probe_hop(args.reps, tuple(int(v) for v in args.hop_orders.split(",")))
        print(json.dumps({"probe": args.probe, "results": res}), flush=True)
        if args.calibrate_copy:
            calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: --gpus must be 1 "
                          "(sample-parallel sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2306_09559_amd import _lib as L
    from paper_2306_09559_amd import driver
    from paper_2306_09559_amd.batch import GraphStep, autotune
    from synth.configs import C2

    torch.cuda.set_device(0)
    prec = L.F64 if args.prec == "f64" else L.F32
    run = driver.build(C2, prec=prec, rb=args.rb)
    V, N = run.dl.V, C2.levels[0].samples
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        run.step()
    torch.cuda.synchronize()
    wall, lvl_ms = timed_steps(run, args.steps, stream)
    ms_per_step = wall / args.steps * 1e3
    byts = run.bytes_per_step()
    value = byts * args.steps / wall / 1e9

    # dominant kernel: the t-sweep launch (one per operator application)
    launch_s = kernel_launch_seconds(run, args.steps, stream)
    per_launch_bytes = driver.launch_bytes(V, N, prec)
    achieved = per_launch_bytes / launch_s / 1e9
    traffic = measured_traffic(args.prec)
    copy_gbs = copy_bandwidth_gbs()

    est = run.estimates()
    eps = 0.0005 * V
    per_sample_s = [lvl_ms[i] * 1e-3 / (args.steps * C2.levels[i].samples) for i in range(len(run.levels))]
    t_eps = driver.time_to_error([e["variance"] for e in est], per_sample_s, eps)
    out = {
        "metric": "p(A)B dslash HBM GB/s (% peak); time to fixed trace std-error, mixed vs FP64",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "8^4 Wilson-Dirac n=49152, eps=0.3 links, periodic t, kappa=%.6f; levels "
                               "Tr(p150-p30) & Tr(p30-p8) deflated (k=%d), Tr(p8); %d Z4 samples per level"
                               % (C2.kappa, run.defl.device.k if run.defl else 0, N),
                   "rb": args.rb, "prec": args.prec},
        "pct_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": KERNEL, "bytes_per_launch": per_launch_bytes,
                     "avg_launch_us": round(launch_s * 1e6, 3),
                     "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "time_to_eps_s": round(t_eps, 4),
        "eps": eps,
        "levels": [{"estimate": [round(e["estimate"].real, 6), round(e["estimate"].imag, 6)],
                    "stderr": e["stderr"], "n": e["n"]} for e in est],
        "mvp_rhs_per_step": run.mvp_rhs_per_step(),
        "setup_s": round(run.setup_seconds, 2),
    }
    if not args.no_mixed and prec == L.F64:
        # mixed precision: FP32 fields, links, eigenvectors and vector updates,
        # FP64 roots, dots, samples and accumulators; same set-up, same samples
        run32 = driver.build(C2, prec=L.F32, rb=args.rb, reuse=run)
        for _ in range(args.warmup):
            run32.step()
        wall32, lvl_ms32 = timed_steps(run32, args.steps, stream)
        est32 = run32.estimates()
        targets = driver.level_targets(eps, [e["stderr"] for e in est])
        ps32 = [lvl_ms32[i] * 1e-3 / (args.steps * C2.levels[i].samples) for i in range(len(run32.levels))]
        out["mixed"] = {
            "value": round(run32.bytes_per_step() * args.steps / wall32 / 1e9, 2), "unit": "GB/s",
            "ms_per_step": round(wall32 / args.steps * 1e3, 3),
            "time_to_eps_s": round(driver.time_to_error([e["variance"] for e in est32], ps32, eps), 4),
            "level_error": [float(f"{abs(a['estimate'] - b['estimate']):.4g}") for a, b in zip(est32, est)],
            "level_target": [round(t, 4) for t in targets],
            "level_error_over_target": [round(abs(a["estimate"] - b["estimate"]) / t, 5)
                                        for a, b, t in zip(est32, est, targets)],
            "level_error_over_stderr": [round(abs(a["estimate"] - b["estimate"]) / b["stderr"], 5)
                                        for a, b in zip(est32, est)],
            "bound": "per level |T_mixed - T_fp64| <= 0.1 x the level's standard-error target "
                     "(eps = 0.0005 V split over the levels), same noise",
            "bound_met": all(abs(a["estimate"] - b["estimate"]) <= 0.1 * t for a, b, t in zip(est32, est, targets)),
        }
        # mixed + batched: the library's autotuner picks every level's shape; each batch of
        # the adaptive loop is then one launch of a step the library recorded as a HIP graph
        tune = autotune(run32, reps=4, use_cache=False)
        gps = graph_level_seconds(run32, args.steps)
        gs = GraphStep([run32], level_branches=True)
        gs.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs.replay(args.steps)
        torch.cuda.synchronize()
        gstep = (time.perf_counter() - t0) / args.steps
        del gs
        t_mb = driver.time_to_error([e["variance"] for e in est32], gps, eps)
        # the measured time to eps: the multilevel Monte Carlo of Sec. 5 step 3 run to
        # completion (levels top first, each to its share of eps at its check points, the
        # check on the device); every leg is warmed up once, then the legs are timed in
        # alternating order and the median of `rounds` runs is reported
        driver.prepare_adaptive(run32)
        legs = {"f64": (run, False), "mixed": (run32, False), "mixed_batched": (run32, True)}
        for r, g in legs.values():
            driver.run_to_tolerance(r, eps, graphs=g)
        rounds = 3
        tot = {k: [] for k in legs}
        lsum = {k: [] for k in legs}
        last = {}
        for k in range(rounds):
            names = list(legs) if k % 2 == 0 else list(reversed(list(legs)))
            for name in names:
                r, g = legs[name]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = driver.run_to_tolerance(r, eps, graphs=g)
                torch.cuda.synchronize()
                tot[name].append(time.perf_counter() - t0)
                lsum[name].append(sum(x.seconds for x in res))
                last[name] = res
        out["adaptive"] = {}
        for name in legs:
            res = last[name]
            med = float(np.median(tot[name]))
            out["adaptive"][name] = {
                "seconds": round(med, 4), "level_seconds": round(float(np.median(lsum[name])), 4),
                "runs": [round(x, 4) for x in tot[name]],
                "stderr": round(float(np.sqrt(sum(x.stderr ** 2 for x in res))), 4), "eps": eps,
                "trace_estimate": [round(sum(x.estimate for x in res).real, 3),
                                   round(sum(x.estimate for x in res).imag, 3)],
                "levels": [{"n": x.n, "drawn": x.drawn, "stderr": round(x.stderr, 4), "target": round(x.target, 4),
                            "seconds": round(x.seconds, 4)} for x in res]}
        ad = out["adaptive"]
        ad["speedup_mixed_vs_f64"] = round(ad["f64"]["seconds"] / ad["mixed"]["seconds"], 3)
        ad["speedup_mixed_batched_vs_f64"] = round(ad["f64"]["seconds"] / ad["mixed_batched"]["seconds"], 3)
        out["mixed_batched"] = {
            "ms_per_step": round(gstep * 1e3, 3),
            "value": round(run32.bytes_per_step() / gstep / 1e9, 2), "unit": "GB/s",
            "time_to_eps_s": ad["mixed_batched"]["seconds"],
            "speedup_vs_f64": ad["speedup_mixed_batched_vs_f64"],
            "shapes": {str(k): {"rb": v[0], "sweep": v[1], "block_rank": v[2], "t_chunks": v[3]}
                       for k, v in tune.choice.items()},
        }
        # measured seconds to eps (the adaptive runs above); the MLMC-optimal cost formula with measured
        # per-sample times is kept beside them as a model
        out["time_to_eps_s"] = {"f64": ad["f64"]["seconds"], "mixed": ad["mixed"]["seconds"],
                                "mixed_batched": ad["mixed_batched"]["seconds"],
                                "model": {"f64": out["time_to_eps_s"], "mixed": out["mixed"]["time_to_eps_s"],
                                          "mixed_batched": round(t_mb, 4)}}
        # the paper's lowest level exact by probing (Sec. 5 step 3d), eps over the Monte Carlo levels;
        # the colouring is set-up (once per lattice and degree) and timed apart
        from paper_2306_09559_amd import probing
        t0 = time.perf_counter()
        col = probing.colouring(C2.dims, int(C2.levels[-1].hi))
        out["adaptive"]["colouring"] = {"distance": int(C2.levels[-1].hi), "colours": int(col.max()) + 1,
                                        "setup_s": round(time.perf_counter() - t0, 3)}
        for r in (run, run32):
            driver.run_to_tolerance(r, eps, probe_last=True)          # warm-up (probe kernels, colouring upload)
        for name, r in (("f64_probing", run), ("mixed_probing", run32)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = driver.run_to_tolerance(r, eps, probe_last=True)
            torch.cuda.synchronize()
            tot = time.perf_counter() - t0
            out["adaptive"][name] = {
                "seconds": round(tot, 4), "stderr": round(float(np.sqrt(sum(x.stderr ** 2 for x in res))), 4),
                "trace_estimate": [round(sum(x.estimate for x in res).real, 3),
                                   round(sum(x.estimate for x in res).imag, 3)],
                "levels": [{"n": x.n, "stderr": round(x.stderr, 4), "seconds": round(x.seconds, 4)} for x in res]}
    if not args.no_extra:
        # variance of the deflated levels against the number of deflated eigenvectors (Sec. 4.1)
        from paper_2306_09559_amd import diagnostics
        prof = {}
        for li in (0, 1):
            p = diagnostics.level_variance_profile(run, li, run.levels[li].batch)
            prof[f"level{li}"] = {"variance_vs_k": [float(f"{v:.4g}") for v in p.variance],
                                  "reproduction_error": float(f"{p.reproduction_error:.2g}")}
        out["deflation_profile"] = prof
        out["batched_lattices"] = batched_c5(args.steps)
        out["top_level"] = top_level_c3(fp64_check=True)
        # a near-critical 16^3x32 top level with the regular and the extra-deflation set-up (Sec. 6.1)
        from synth.configs import C3R, C3X
        out["deflation_setups"] = {"regular": top_level_c3(C3R), "extra": top_level_c3(C3X)}
    if not args.no_c4:
        torch.cuda.empty_cache()
        out["c4"] = c4_step()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(C2, args.prec)
        out["cpu_baseline"]["one_thread"] = cpu_baseline_one_thread()
    if args.calibrate_copy:
        calibrate_copy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
