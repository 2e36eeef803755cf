"""Full-size parity in the launch configuration bench.py times.

* 8^4 workload (n = 49152, 256 Z4 vectors, rb = 16, the t-sweep kernel):
  every sample of the top polynomial-difference level is computed on the
  GPU, and sampled vectors are recomputed one by one by the oracle with its
  own GMRES roots.  FP64 within 1e-12 relative (the workload is
  near-critical: the amplification kappa_N of the Newton recurrence is
  measured and reported); FP32 within 8 d kappa_N u32.
* bit-exact, in the same launch configuration (8^4 x 256, rb = 16, FP64
  t-sweep, two-row links) and on the 24^3 x 48 lattice (FP32 blocked t-sweep
  and streaming kernel): with monomial SU(3) links (permutations with phases
  in {1, i, -1, -i}), kappa = 1/8 and dyadic inverse roots every product and
  sum of the Newton recurrence and of b^H w is exact in the kernels' and the
  oracle's arithmetic, so the samples must equal the oracle's bit for bit --
  an indexing, layout or spin-algebra mistake anywhere fails, whatever the
  rounding.
* the same level deflated as the workload runs it (FP64), on the oracle's own
  set-up: its GMRES roots and the first 20 eigen-triplets its PP(31)-Arnoldi
  and selection accept, written as a checkpoint of the product's run and
  resumed, so no root or eigenvector comes from the HIP path.  All 256
  deflated samples b^H p150 b - b^H p30 b - sum_i c_i conj(zeta_i) omega_i,
  with zeta = V^H b, the left vectors, their biorthonormal scaling and
  c_i = p150(lambda_i) - p30(lambda_i) formed by the oracle, within 1e-12 of
  each sample's scale, and the level's FP64 accumulator (n, mean, M2) against
  the oracle's estimate of the same samples.
* 24^3 x 48 workload (n = 7.96M, the largest): its lowest level's polynomial
  (degree 4, GMRES roots at full size) over 16 Z4 vectors in FP32 on the
  blocked t-sweep (24 x 4 x 4 blocks of the 24^3 plane with a one-site halo)
  and on the streaming kernel; the first and last samples are recomputed by
  the oracle at full size, within 8 d kappa_N u32.
* the 24^3 x 48 workload's second level, Tr(p60 - p15), as it is launched
  (128 samples, block width 16, FP32 level kernel on the blocked t-sweep),
  on roots the oracle computes on an 8^4 lattice of the same ensemble:
  samples 0 and 127 of both polynomials within 8 d kappa_N u32.
* the deflation coefficients V^H b and U^H b over the 24^3 x 48 lattice's
  n = 7.96M rows in FP32 on MFMA (k = 20 padded to 32, 128 Z4 vectors):
  eigenvector entries in {-1, 0, 1} + i{-1, 0, 1} and left vectors g5 z / 2
  make every product and partial sum exact in FP32, so sampled columns must
  equal the oracle's exactly, whatever the summation order.
* 16^3 x 32 workload (n = 1.57M, 64 vectors): its double polynomial
  p_1 = p_in(A) p_out(A p_in(A)) (PP(20) x 15, degree 299, the oracle's own
  GMRES and PP-GMRES roots) in FP32 scalar mode, the inner chains on the
  blocked t-sweep and the outer update on the streaming kernel; samples 0 and
  63 recomputed by the oracle at full size, within 8 d kappa_N u32 with
  kappa_N the measured growth of the double polynomial's intermediate vectors.
* 16^3 x 32 workload (n = 1.57M, 64 vectors): the top-level solutions of one
  batch satisfy ||b - A x|| <= 1e-6 ||b|| through the oracle operator, for
  sampled vectors (a property that holds at any size).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import krylov, solve as osolve
from gpu_helpers import build_from_oracle_set_up, composite_amplification, dev_c128, lib, oracle_set_up, pack, unpack

pytestmark = pytest.mark.gpu

U32, U64 = 2.0 ** -24, 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def c2():
    from synth.configs import C2
    U = synth.gauge_links(C2.dims, C2.eps, C2.seed_links)
    ol = oracle.Lattice(C2.dims, C2.kappa, U, C2.antiperiodic_t)
    ps = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, C2.seed_start), [150, 30])
    return C2, U, ol, ps


def _kappa_N(ol, t, b):
    w = b.copy()
    nb = np.linalg.norm(b)
    out = 1.0
    for tj in t[:-1]:
        w = w - tj * ol.apply(w)
        out = max(out, np.linalg.norm(w) / nb)
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_c2_top_level_sampled_vs_oracle(c2, prec):
    L = lib()
    C2, U, ol, ps = c2
    dims, N, rb = C2.dims, C2.levels[0].samples, 16
    V = int(np.prod(dims))
    gauge = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
    L.pack_gauge(dims, prec, torch.from_numpy(U).cuda(), gauge)
    dl = L.DeviceLattice(tuple(dims), C2.kappa, C2.antiperiodic_t, prec, gauge)
    t150, t30 = ps.inv_roots[150], ps.inv_roots[30]
    lvl = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(t150)), L.OP_POLY, L.DevicePoly(dev_c128(t30)))
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    nz = L.Noise(C2.seed_noise, C2.lattice_id, 0, 0)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lvl, N, rb))
    L.mlmc_level_estimate(dl, lvl, N, rb, nz, samples, acc, ws)
    S = samples.cpu().numpy()
    hi, lo = S[:, 2] + 1j * S[:, 3], S[:, 4] + 1j * S[:, 5]
    assert np.all(np.isfinite(S)) and acc.cpu().numpy()[0] == N
    for r in (0, 131, 255):
        b = oracle.z4(C2.seed_noise, C2.lattice_id, 0, r, 1, V)[0]
        _, rh = ol.poly_apply(t150, b)
        _, rl = ol.poly_apply(t30, b)
        for got, want, t, d in ((hi[r], rh[0], t150, 150), (lo[r], rl[0], t30, 30)):
            kN = _kappa_N(ol, t, b)
            bound = 1e-12 if prec == 0 else 8 * d * kN * U32
            err = abs(got - want) / abs(want)
            print(f"prec {prec} r {r} d {d}: rel err {err:.2e}, kappa_N {kN:.3g}, bound {bound:.2e}")
            assert err <= bound


# dyadic inverse roots: with kappa = 1/8 every Newton step w - t A w of a
# Gaussian-integer field is exact (few fraction bits per step)
T_EXACT_HI = np.array([1.0, 0.5 + 0.5j, 0.5, 1.0, 0.5 - 0.5j])
T_EXACT_LO = np.array([0.5, 1.0, 0.5 + 0.5j])


def _exact_lattice(L, dims, prec, apbc, seed):
    U = synth.monomial_links(dims, seed)
    ol = oracle.Lattice(dims, 0.125, U, apbc)
    V = int(np.prod(dims))
    gauge = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
    L.pack_gauge(dims, prec, torch.from_numpy(U).cuda(), gauge)
    return ol, L.DeviceLattice(tuple(dims), 0.125, apbc, prec, gauge, 2)


@pytest.mark.parametrize("prec", [0, 1])
def test_c2_launch_bit_exact_with_monomial_links(prec):
    """FP64 (the bench's level kernel) and FP32 (its mixed-precision run, the
    whole-plane sweep with the link prefetch; degree 3 so that every FP32
    entry stays within 24 bits)."""
    L = lib()
    from synth.configs import C2
    dims, N, rb, V = C2.dims, C2.levels[0].samples, 16, C2.volume
    ol, dl = _exact_lattice(L, dims, prec, C2.antiperiodic_t, 5)
    assert L.sweep_plan(dl, N, 1)["ok"]
    t_hi = T_EXACT_HI if prec == 0 else T_EXACT_HI[:4]
    lvl = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(t_hi)), L.OP_POLY, L.DevicePoly(dev_c128(T_EXACT_LO)))
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lvl, N, rb))
    L.mlmc_level_estimate(dl, lvl, N, rb, L.Noise(C2.seed_noise, C2.lattice_id, 0, 0), samples, acc, ws)
    S = samples.cpu().numpy()
    s, hi, lo = S[:, 0] + 1j * S[:, 1], S[:, 2] + 1j * S[:, 3], S[:, 4] + 1j * S[:, 5]
    B = oracle.z4(C2.seed_noise, C2.lattice_id, 0, 0, N, V)
    _, rh = ol.poly_apply(t_hi, B)
    _, rl = ol.poly_apply(T_EXACT_LO, B)
    print("prec", prec, "hi up to", np.max(np.abs(rh)), "mismatches", np.count_nonzero(hi != rh), np.count_nonzero(lo != rl))
    assert np.array_equal(hi, rh) and np.array_equal(lo, rl) and np.array_equal(s, rh - rl)


def test_c4_lattice_bit_exact_with_monomial_links():
    L = lib()
    from synth.configs import C4
    dims, N, rb, V = C4.dims, 16, 1, C4.volume
    ol, dl = _exact_lattice(L, dims, 1, C4.antiperiodic_t, 6)
    assert L.sweep_plan(dl, N, rb)["halo"]
    t = T_EXACT_HI[:4]
    poly = L.DevicePoly(dev_c128(t))
    ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
    nz = L.Noise(C4.seed_noise, C4.lattice_id, 3, 0)
    out = {}
    for opt in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, opt)
        bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
        torch.cuda.synchronize()
        out[opt] = bhy.cpu().numpy()
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    assert np.array_equal(out[1], out[0])
    for r in (0, N - 1):
        b = oracle.z4(C4.seed_noise, C4.lattice_id, 3, r, 1, V)[0]
        _, want = ol.poly_apply(t, b)
        print(f"r {r}: {want[0]} sweep {out[1][r]} streaming {out[0][r]}")
        assert out[1][r] == want[0]


def test_c2_double_polynomial_bit_exact_with_monomial_links():
    """The double polynomial in scalar mode on the 8^4 x 256 launch: inner
    chains on the FP64 t-sweep, the outer update on the streaming kernel."""
    L = lib()
    from synth.configs import C2
    dims, N, rb, V = C2.dims, 256, 16, C2.volume
    ol, dl = _exact_lattice(L, dims, 0, C2.antiperiodic_t, 8)
    t_in, t_out = np.array([1.0, 0.5]), np.array([1.0, 0.5 + 0.5j])
    poly = L.DevicePoly(dev_c128(t_in), dev_c128(t_out))
    ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
    bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    L.poly_apply(dl, poly, N, rb, None, L.Noise(9, 2, 4, 0), None, bhy, ws)
    got = bhy.cpu().numpy()
    _, want = ol.composite_apply(t_in, t_out, oracle.z4(9, 2, 4, 0, N, V))
    print("double polynomial: mismatches", np.count_nonzero(got != want), "of", N)
    assert np.array_equal(got, want)


def test_c3_vector_mode_bit_exact_with_monomial_links():
    """y = p(A) b materialised (vector mode at block width 1, the top-level
    solver's p_in) on the 16^3 x 32 lattice in FP32: the blocked t-sweep
    accumulates y in the same launches; whole output vectors compared."""
    L = lib()
    from synth.configs import C3
    dims, N, V = C3.dims, C3.levels[0].samples, C3.volume
    ol, dl = _exact_lattice(L, dims, 1, C3.antiperiodic_t, 9)
    assert L.sweep_plan(dl, N, 1)["halo"]
    t = T_EXACT_HI[:4]
    poly = L.DevicePoly(dev_c128(t))
    ws = L.workspace(L.poly_workspace_size(dl, poly, N, 1))
    y = L.empty_field(V, N, 1, 1)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    L.poly_apply(dl, poly, N, 1, None, L.Noise(21, 3, 0, 0), y, None, ws)
    one = L.empty_field(V, 1, 1, 1)
    for r in (0, N - 1):
        L.field_copy_vector(dims, 1, y, r, one, 0)
        got = unpack(dims, one, 1)[0]
        want, _ = ol.poly_apply(t, oracle.z4(21, 3, 0, r, 1, V)[0])
        print(f"vector mode r {r}: mismatches {np.count_nonzero(got != want)} of {got.size}")
        assert np.array_equal(got, want)


def test_c2_deflated_level_bit_exact_with_monomial_links():
    """The deflated level kernel on the 8^4 x 256 launch: b^H p_hi b - b^H p_lo b
    - sum_i c_i conj(zeta_i) omega_i with 20 Gaussian-integer vectors in the
    place of eigenvectors (k padded to 32, as the workload runs it), left
    vectors g5 z / 2 and dyadic c: every sample equals the oracle's exactly."""
    L = lib()
    from oracle import estimator
    from synth.configs import C2
    dims, N, rb, V = C2.dims, C2.levels[0].samples, 16, C2.volume
    n, k, kpad = 12 * V, 20, 32
    ol, dl = _exact_lattice(L, dims, 0, C2.antiperiodic_t, 10)
    rng = np.random.default_rng(12)
    Z = (rng.integers(-1, 2, (k, n)) + 1j * rng.integers(-1, 2, (k, n))).astype(np.complex128)
    Uv = 0.5 * np.stack([ol.gamma5(Z[i]) for i in range(k)])
    Zp = np.zeros((kpad, n), dtype=np.complex128)
    Zp[:k] = Z
    D = L.DeviceDefl(k, pack(dims, Zp, kpad, 0), torch.arange(k, dtype=torch.int32, device="cuda"),
                     dev_c128(np.full(k, 0.5)), None)
    c = (rng.integers(-4, 5, k) + 1j * rng.integers(-4, 5, k)) / 8.0
    lvl = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(T_EXACT_HI)), L.OP_POLY, L.DevicePoly(dev_c128(T_EXACT_LO)),
                        D, True, dev_c128(c))
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lvl, N, rb))
    L.mlmc_level_estimate(dl, lvl, N, rb, L.Noise(C2.seed_noise, C2.lattice_id, 1, 0), samples, acc, ws)
    S = samples.cpu().numpy()
    got = S[:, 0] + 1j * S[:, 1]
    B = oracle.z4(C2.seed_noise, C2.lattice_id, 1, 0, N, V)
    _, rh = ol.poly_apply(T_EXACT_HI, B)
    _, rl = ol.poly_apply(T_EXACT_LO, B)
    zeta, omega = Z.conj() @ B.T, Uv.conj() @ B.T
    want = estimator.level_samples(rh, rl, zeta, omega, c)
    print("deflated level: mismatches", np.count_nonzero(got != want), "of", N)
    assert np.array_equal(got, want)


def test_c2_probing_bit_exact_with_monomial_links():
    """Tr p(A) by probing on the 8^4 lattice (degree 4: a distance-4
    colouring, probe vectors generated inside the FP64 t-sweep, 256 per
    launch): the trace equals the oracle's probe sum over the same colouring
    exactly."""
    L = lib()
    from paper_2306_09559_amd import probing
    from oracle import probing as oprobe
    from synth.configs import C2
    dims = C2.dims
    ol, dl = _exact_lattice(L, dims, 0, C2.antiperiodic_t, 11)
    t = T_EXACT_HI
    d = len(t) - 1
    col = probing.colouring(dims, d)
    res = probing.probe_trace(dl, L.DevicePoly(dev_c128(t)), col, nrhs=256, rb=1, in_kernel=True)
    want = oprobe.probe_trace(ol, t, col.astype(np.int64))
    print(f"probing: {res.ncolours} colours, {res.probes} probes, trace {res.trace} oracle {want}")
    assert res.trace == want


@pytest.mark.parametrize("prec", [0, 1])
def test_c4_lattice_operator_bit_exact_with_monomial_links(prec):
    """A x through mpmc_wilson_apply (the streaming kernel) on the 24^3 x 48
    lattice, 16 Z4 vectors at block width 16: whole output vectors equal the
    oracle's entry for entry."""
    L = lib()
    from synth.configs import C4
    dims, N, rb, V = C4.dims, 16, 16, C4.volume
    ol, dl = _exact_lattice(L, dims, prec, C4.antiperiodic_t, 12)
    x = L.empty_field(V, N, rb, prec)
    L.z4_fill(dims, prec, L.Noise(31, 4, 0, 0), x)
    y = L.empty_field(V, N, rb, prec)
    L.wilson_apply(dl, x, y)
    one = L.empty_field(V, 1, 1, prec)
    for r in (0, 9, N - 1):
        L.field_copy_vector(dims, prec, y, r, one, 0)
        got = unpack(dims, one, prec)[0]
        want = ol.apply(oracle.z4(31, 4, 0, r, 1, V)[0])
        assert np.array_equal(got, want), (r, np.count_nonzero(got != want))


def test_c2_deflated_level_every_sample_vs_oracle(tmp_path):
    L = lib()
    from oracle import deflation, estimator
    from synth.configs import C2
    su = oracle_set_up(C2, [150, 30, 8], pin_degree=30)
    ol, tri = su.ol, su.tri
    run = build_from_oracle_set_up(C2, su, tmp_path / "c2_oracle_setup.npz", prec=L.F64, rb=16)
    lv = run.levels[0]
    assert lv.c is not None and run.defl.device.k == len(tri.lam) == C2.k_defl
    N, rb, V = lv.batch, run.level_rb(0), C2.volume
    nz = L.Noise(C2.seed_noise, C2.lattice_id, lv.index, 0)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(run.dl, lv.device, N, rb))
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    L.mlmc_level_estimate(run.dl, lv.device, N, rb, nz, samples, acc, ws)
    S = samples.cpu().numpy()
    got = S[:, 0] + 1j * S[:, 1]
    t150, t30 = su.ps.inv_roots[150], su.ps.inv_roots[30]
    c = deflation.poly_eval(t150, tri.lam) - deflation.poly_eval(t30, tri.lam)
    # every sample of the batch, by the oracle (a batch of N Newton applications per polynomial)
    B = oracle.z4(C2.seed_noise, C2.lattice_id, lv.index, 0, N, V)
    _, hi = ol.poly_apply(t150, B)
    _, lo = ol.poly_apply(t30, B)
    zeta, omega = tri.Z.conj() @ B.T, tri.U.conj() @ B.T
    terms = c[:, None] * np.conj(zeta) * omega
    want = estimator.level_samples(hi, lo, zeta, omega, c)
    scale = np.abs(hi) + np.abs(lo) + np.sum(np.abs(terms), axis=0)
    err = np.abs(got - want) / scale
    kN = max(_kappa_N(ol, t150, B[0]), _kappa_N(ol, t30, B[0]))
    r = int(np.argmax(err))
    print(f"{N} deflated samples: max error / scale {err[r]:.2e} (sample {r}), kappa_N of sample 0 {kN:.3g}")
    assert np.all(err <= 1e-12)
    # the level's FP64 accumulator: n, mean and M2 of exactly these samples
    est = estimator.level_estimate(want)
    A = acc.cpu().numpy()
    assert A[0] == N and A[4] == 0
    # with every sample within delta = 1e-12 of its scale, the mean moves by at most
    # that and the variance by 4 delta (sqrt(var) + delta) N / (N - 1); plus FP64 summation order
    delta = 1e-12 * float(np.max(scale))
    assert abs(complex(A[1], A[2]) - est.mean) <= delta
    assert abs(A[3] / (N - 1) - est.var) <= 4 * delta * (np.sqrt(est.var) + delta) * N / (N - 1) + 1e-13 * est.var


def test_c4_planes_blocked_sweep_sampled_vs_oracle():
    L = lib()
    from synth.configs import C4
    dims, V, N, rb, prec = C4.dims, C4.volume, 16, 1, 1
    U = synth.gauge_links(dims, C4.eps, C4.seed_links)
    ol = oracle.Lattice(dims, C4.kappa, U, C4.antiperiodic_t)
    d = C4.levels[3].hi
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, C4.seed_start), [d]).inv_roots[d]
    gauge = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
    L.pack_gauge(dims, prec, torch.from_numpy(U).cuda(), gauge)
    del U
    dl = L.DeviceLattice(tuple(dims), C4.kappa, C4.antiperiodic_t, prec, gauge)
    plan = L.sweep_plan(dl, N, rb)
    assert plan["ok"] and plan["halo"], plan
    print("block", plan["block"], "halo sites", plan["halo_sites"])
    poly = L.DevicePoly(dev_c128(t))
    ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
    nz = L.Noise(C4.seed_noise, C4.lattice_id, 3, 0)
    out = {}
    for opt in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, opt)
        bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
        torch.cuda.synchronize()
        out[opt] = bhy.cpu().numpy()
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    del ws, gauge
    for r in (0, N - 1):
        b = oracle.z4(C4.seed_noise, C4.lattice_id, 3, r, 1, V)[0]
        _, want = ol.poly_apply(t, b)
        kN = _kappa_N(ol, t, b)
        bound = 8 * d * kN * U32
        for opt in (1, 0):
            err = abs(out[opt][r] - want[0]) / abs(want[0])
            print(f"r {r} {'sweep' if opt else 'streaming'}: rel err {err:.2e}, kappa_N {kN:.3g}, bound {bound:.2e}")
            assert err <= bound


def test_c4_level_at_its_degrees_sampled_vs_oracle():
    """The 24^3 x 48 workload's second level, Tr(p60 - p15), as the workload
    launches it: 128 samples, block width 16, FP32, two-row links, the level
    kernel on the blocked t-sweep.  The roots are the oracle's GMRES roots of
    degrees 60 and 15 on an 8^4 lattice with the same kappa, link ensemble and
    seeds (the oracle's Arnoldi at n = 7.96M is too slow for a test; any roots
    serve, the oracle applying the same ones).  Samples 0 and 127, both
    polynomials, are recomputed by the oracle at full size within
    8 d kappa_N u32."""
    L = lib()
    from synth.configs import C4
    from gpu_helpers import device_lattice, newton_amplification
    li = 1
    hi, lo, N = C4.levels[li].hi, C4.levels[li].lo, C4.levels[li].samples
    small = (8, 8, 8, 8)
    ols = oracle.Lattice(small, C4.kappa, synth.gauge_links(small, C4.eps, C4.seed_links), C4.antiperiodic_t)
    ps = krylov.gmres_polys(ols.apply, synth.gaussian_start(ols.n, C4.seed_start), [hi, lo])
    del ols
    dl, ol = device_lattice(C4.dims, C4.kappa, C4.eps, C4.seed_links, C4.antiperiodic_t, L.F32, link_rows=2)
    rb, V = 16, C4.volume
    plan = L.sweep_plan(dl, N, rb)
    assert plan["ok"] and plan["halo"], plan
    print("block", plan["block"], "chunks", plan["chunks"])
    lev = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(ps.inv_roots[hi])), L.OP_POLY,
                        L.DevicePoly(dev_c128(ps.inv_roots[lo])))
    nz = L.Noise(C4.seed_noise, C4.lattice_id, li, 0)
    samples = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lev, N, rb))
    L.set_option(L.OPT_PLANE_SWEEP, L.SWEEP_AUTO)
    L.mlmc_level_estimate(dl, lev, N, rb, nz, samples, acc, ws)
    S = samples.cpu().numpy()
    del ws
    assert np.all(np.isfinite(S))
    B = oracle.z4(C4.seed_noise, C4.lattice_id, li, 0, N, V)[[0, N - 1]]
    for d, col in ((hi, 2), (lo, 4)):
        t = ps.inv_roots[d]
        _, want = ol.poly_apply(t, B)
        kN = newton_amplification(ol.apply, t, B)
        bound = 8 * d * kN * U32
        for j, r in enumerate((0, N - 1)):
            got = S[r, col] + 1j * S[r, col + 1]
            err = abs(got - want[j]) / abs(want[j])
            print(f"p{d} r {r}: rel err {err:.2e}, kappa_N {kN:.3g}, bound {bound:.2e}")
            assert err <= bound
        # the level's sample is the difference of the two constituents
    assert np.array_equal(S[:, 0], S[:, 2] - S[:, 4]) and np.array_equal(S[:, 1], S[:, 3] - S[:, 5])


@pytest.mark.parametrize("i,plan_want", [(0, (False, 4)), (1, (True, 3)), (2, (True, 2)), (3, None)])
def test_c5_lattices_sampled_vs_oracle(i, plan_want):
    """The four independent lattices of the mixed batch at their sizes and
    batch widths (8^4 x 64, 12^4 x 32, 16^4 x 16, 12^3x24 x 8 vectors, FP32,
    block width 8) on the kernel the default plan picks: the whole-plane
    t-sweep in 4 t-chunks, blocked sweeps in 3 and 2 t-chunks, and the
    streaming kernel for the 12^3x24 batch.  A degree-12 GMRES polynomial of
    each lattice's own operator; samples 0 and N-1 against the oracle."""
    L = lib()
    from synth.configs import C5
    cfg = C5[i]
    dims, V, N, rb, prec = cfg.dims, cfg.volume, cfg.levels[0].samples, 8, 1
    U = synth.gauge_links(dims, cfg.eps, cfg.seed_links)
    ol = oracle.Lattice(dims, cfg.kappa, U, cfg.antiperiodic_t)
    d = 12
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, cfg.seed_start), [d]).inv_roots[d]
    gauge = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
    L.pack_gauge(dims, prec, torch.from_numpy(U).cuda(), gauge)
    del U
    dl = L.DeviceLattice(tuple(dims), cfg.kappa, cfg.antiperiodic_t, prec, gauge)
    L.set_option(L.OPT_PLANE_SWEEP, 2)
    L.set_option(L.OPT_SWEEP_CHUNKS, 0)
    plan = L.sweep_plan(dl, N, rb)
    print(dims, N, plan)
    if plan_want is None:
        assert not plan["ok"]
    else:
        assert plan["ok"] and (plan["halo"], plan["chunks"]) == plan_want, plan
    poly = L.DevicePoly(dev_c128(t))
    ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
    nz = L.Noise(cfg.seed_noise, cfg.lattice_id, 0, 0)
    bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
    L.poly_apply(dl, poly, N, rb, None, nz, None, bhy, ws)
    torch.cuda.synchronize()
    got = bhy.cpu().numpy()
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    del ws, gauge
    for r in (0, N - 1):
        b = oracle.z4(cfg.seed_noise, cfg.lattice_id, 0, r, 1, V)[0]
        _, want = ol.poly_apply(t, b)
        kN = _kappa_N(ol, t, b)
        bound = 8 * d * kN * U32
        err = abs(got[r] - want[0]) / abs(want[0])
        print(f"r {r}: rel err {err:.2e}, kappa_N {kN:.3g}, bound {bound:.2e}")
        assert err <= bound


def test_c4_size_deflation_coefficients_exact():
    L = lib()
    dims = (24, 24, 24, 48)
    V = int(np.prod(dims))
    n, k, kpad, N, rb = 12 * V, 20, 32, 128, 16
    rng = np.random.default_rng(11)
    Z = (rng.integers(-1, 2, (k, n)) + 1j * rng.integers(-1, 2, (k, n))).astype(np.complex128)
    ol = oracle.Lattice(dims, 0.15, synth.unit_links(dims))
    U = 0.5 * np.stack([ol.gamma5(Z[i]) for i in range(k)])
    # u_i = scale_i g5 z_i with scale_i = 1/2 exactly (a ratio of two inner products
    # computed in complex arithmetic can come out one unit in the last place off)
    Zp = np.zeros((kpad, n), dtype=np.complex128)
    Zp[:k] = Z
    D = L.DeviceDefl(k, pack(dims, Zp, kpad, 1), torch.arange(k, dtype=torch.int32, device="cuda"),
                     dev_c128(np.full(k, 0.5)), None)
    del Zp
    gauge = torch.zeros(36 * V, dtype=L.complex_dtype(1), device="cuda")
    dl = L.DeviceLattice(dims, 0.15, True, 1, gauge)
    nz = L.Noise(17, 9, 1, 0)
    zeta = torch.empty((k, N), dtype=torch.complex128, device="cuda")
    omega = torch.empty_like(zeta)
    ws = L.workspace(L.deflate_workspace_size(dl, D, N, rb))
    L.deflate_project(dl, D, L.DEFL_COEFF, N, rb, None, nz, zeta, omega, None, None, ws)
    zg, og = zeta.cpu().numpy(), omega.cpu().numpy()
    del D, ws
    for r in (0, 77, N - 1):
        b = oracle.z4(17, 9, 1, r, 1, V)[0]
        rz, ro = Z.conj() @ b, U.conj() @ b
        print(f"r {r}: |zeta| up to {np.max(np.abs(rz)):.0f}, max |diff| {np.max(np.abs(zg[:, r] - rz)):.1e} / "
              f"{np.max(np.abs(og[:, r] - ro)):.1e}")
        assert np.array_equal(zg[:, r], rz) and np.array_equal(og[:, r], ro)


def test_c4_size_reconstruction_and_projection_exact():
    """X = V d (RECON) and the Left-right Projection X = b - A V H^{-1} U^H b
    (PROJECT) on the 24^3 x 48 lattice in FP32 (k = 20 padded to 32, 16
    vectors): Gaussian-integer vectors, dyadic d and H^{-1}, monomial links
    and kappa = 1/8 keep every step exact, so sampled output vectors equal the
    oracle's entry for entry."""
    L = lib()
    from synth.configs import C4
    dims, V = C4.dims, C4.volume
    n, k, kpad, N, rb = 12 * V, 20, 32, 16, 16
    ol, dl = _exact_lattice(L, dims, 1, C4.antiperiodic_t, 13)
    rng = np.random.default_rng(14)
    Z = (rng.integers(-1, 2, (k, n)) + 1j * rng.integers(-1, 2, (k, n))).astype(np.complex128)
    Uv = 0.5 * np.stack([ol.gamma5(Z[i]) for i in range(k)])
    hinv = (rng.integers(-2, 3, (k, k)) + 1j * rng.integers(-2, 3, (k, k))) / 4.0
    Zp = np.zeros((kpad, n), dtype=np.complex128)
    Zp[:k] = Z
    D = L.DeviceDefl(k, pack(dims, Zp, kpad, 1), torch.arange(k, dtype=torch.int32, device="cuda"),
                     dev_c128(np.full(k, 0.5)), dev_c128(hinv))
    del Zp
    ws = L.workspace(L.deflate_workspace_size(dl, D, N, rb))
    X = L.empty_field(V, N, rb, 1)
    one = L.empty_field(V, 1, 1, 1)
    d = (rng.integers(-8, 9, (k, N)) + 1j * rng.integers(-8, 9, (k, N))) / 8.0
    L.deflate_project(dl, D, L.DEFL_RECON, N, rb, None, None, None, None, dev_c128(d), X, ws)
    for r in (0, N - 1):
        L.field_copy_vector(dims, 1, X, r, one, 0)
        assert np.array_equal(unpack(dims, one, 1)[0], Z.T @ d[:, r]), ("recon", r)
    nz = L.Noise(41, 4, 2, 0)
    dd = torch.empty((k, N), dtype=torch.complex128, device="cuda")
    L.deflate_project(dl, D, L.DEFL_PROJECT, N, rb, None, nz, None, None, dd, X, ws)
    ddh = dd.cpu().numpy()
    for r in (0, N - 1):
        b = oracle.z4(41, 4, 2, r, 1, V)[0]
        dr = hinv @ (Uv.conj() @ b)
        assert np.array_equal(ddh[:, r], dr), ("d", r)
        L.field_copy_vector(dims, 1, X, r, one, 0)
        want = b - ol.apply(Z.T @ dr)
        got = unpack(dims, one, 1)[0]
        print(f"projection r {r}: mismatches {np.count_nonzero(got != want)} of {got.size}")
        assert np.array_equal(got, want)


def test_c3_double_polynomial_sampled_vs_oracle():
    L = lib()
    from synth.configs import C3
    from gpu_helpers import device_lattice
    n_in, n_out = C3.levels[0].lo
    dl, ol = device_lattice(C3.dims, C3.kappa, C3.eps, C3.seed_links, C3.antiperiodic_t, L.F32, link_rows=2)
    # the oracle's roots: GMRES p_in of degree n_in - 1, then PP-GMRES on A p_in(A) for p_out
    start = synth.gaussian_start(ol.n, C3.seed_start)
    t_in = krylov.gmres_polys(ol.apply, start, [n_in - 1]).inv_roots[n_in - 1]
    opB = krylov.pp_operator(ol.apply, t_in, lambda t, v: ol.poly_apply(t, v)[0])
    t_out, _ = krylov.pp_gmres_roots(opB, start, n_out=n_out)
    comp = L.DevicePoly(dev_c128(t_in), dev_c128(t_out))
    N, rb, V = C3.levels[0].samples, 16, C3.volume
    assert L.sweep_plan(dl, N, 1)["halo"]
    nz = L.Noise(C3.seed_noise, C3.lattice_id, 5, 0)
    ws = L.workspace(L.poly_workspace_size(dl, comp, N, rb))
    bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    L.poly_apply(dl, comp, N, rb, None, nz, None, bhy, ws)
    torch.cuda.synchronize()
    got = bhy.cpu().numpy()
    del ws
    assert np.all(np.isfinite(got))
    key = (n_in, n_out)
    d = len(t_in) * len(t_out) - 1
    for r in (0, N - 1):
        b = oracle.z4(C3.seed_noise, C3.lattice_id, 5, r, 1, V)[0]
        _, want = ol.composite_apply(t_in, t_out, b)
        kN = composite_amplification(ol.apply, t_in, t_out, b[None, :])
        bound = 8 * d * kN * U32
        err = abs(got[r] - want[0]) / abs(want[0])
        print(f"{key} degree {d} r {r}: rel err {err:.2e}, kappa_N {kN:.3g}, bound {bound:.2e}")
        assert err <= bound


def test_c3_top_level_solutions_full_size():
    L = lib()
    from paper_2306_09559_amd import driver
    from synth.configs import C3
    run = driver.build(C3, prec=L.F32, rb=16)
    N = C3.levels[0].samples
    run.draw(0, N)
    torch.cuda.synchronize()
    lv = run.levels[0]
    st = lv.last_solve
    assert np.max(st.rel_res) <= 1e-6
    V = C3.volume
    ol = oracle.Lattice(C3.dims, C3.kappa, synth.gauge_links(C3.dims, C3.eps, C3.seed_links), C3.antiperiodic_t)
    canon = torch.empty((N, V, 4, 3), dtype=torch.complex128, device="cuda")
    L.unpack_fields(C3.dims, L.F64, lv.x64, canon)
    for r in (0, 37, 63):
        x = canon[r].cpu().numpy().reshape(-1)
        b = oracle.z4(C3.seed_noise, C3.lattice_id, 0, r, 1, V)[0]
        res = osolve.residual(ol, b, x)[0]
        print(f"C3 vector {r}: residual {res:.2e} (solver {st.rel_res[r]:.2e})")
        assert res <= 1e-6
        assert abs(res - st.rel_res[r]) <= 1e-3 * st.rel_res[r] + 1e-12
    e = run.estimates()[0]
    assert e["n"] == N and np.isfinite(e["estimate"])
