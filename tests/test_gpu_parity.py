"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 bar: 1e-12 relative (normwise for vectors; per constituent for sample
values), bit-exact for noise.  FP32 bar: the stated mixed-precision bound
8 * d * kappa_N * u32 per constituent (kappa_N = max_j ||w_j|| / ||b||).
Sizes span several workgroups and ragged tails (V * rb not a multiple of 256).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import deflation, dense, estimator, krylov

from gpu_helpers import (composite_amplification, dev_c128, device_defl, device_lattice, lib,
                         newton_amplification, pack, rel, unpack)

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib()


# ------------------------------------------------------------------ noise / layout
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dims,nrhs,rb", [((4, 4, 4, 4), 12, 4), ((3, 2, 2, 5), 8, 8), ((2, 2, 2, 2), 5, 1)])
def test_z4_bit_exact(dims, nrhs, rb, prec):
    L = lib()
    V = int(np.prod(dims))
    f = L.empty_field(V, nrhs, rb, prec)
    nz = L.Noise(777, 3, 2, 40)
    L.z4_fill(dims, prec, nz, f)
    got = unpack(dims, f, prec)
    ref = oracle.z4(777, 3, 2, 40, nrhs, V)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, 3 << 24])
def test_copy_bytes_bit_exact(nbytes):
    """The plain streaming copy moves every byte (sizes below one workgroup,
    ragged, and larger than its grid-stride cap), and leaves the bytes past
    the end untouched."""
    L = lib()
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    L.field_copy_bytes(src, dst[:nbytes])
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].sum()) == 0


@pytest.mark.parametrize("prec", [0, 1])
def test_pack_roundtrip(prec):
    dims = (4, 2, 2, 6)
    V = int(np.prod(dims))
    X = synth.random_fields(6, V, 3).reshape(6, -1)
    f = pack(dims, X, 2, prec)
    back = unpack(dims, f, prec)
    if prec == 0:
        assert np.array_equal(back, X)
    else:
        assert np.array_equal(back, X.astype(np.complex64).astype(np.complex128))


# ------------------------------------------------------------------ operator
@pytest.mark.parametrize("dims,nrhs,rb,ap", [
    ((4, 4, 4, 4), 16, 16, True),      # C1 geometry
    ((4, 4, 4, 4), 12, 4, False),
    ((3, 2, 2, 5), 8, 2, True),        # odd extents, ragged last workgroup
    ((2, 4, 2, 2), 3, 1, True),
    ((8, 4, 4, 4), 64, 64, True),      # one site per workgroup quarter
    ((4, 4, 2, 2), 256, 256, True),    # the largest block width: one site per workgroup
])
def test_wilson_apply_f64(dims, nrhs, rb, ap):
    L = lib()
    dl, ol = device_lattice(dims, 0.137, 0.5, 11, ap, prec=0)
    X = synth.random_fields(nrhs, dl.V, 5).reshape(nrhs, -1)
    x = pack(dims, X, rb, 0)
    y = torch.empty_like(x)
    L.wilson_apply(dl, x, y)
    got = unpack(dims, y, 0)
    ref = ol.apply(X)
    for r in range(nrhs):
        assert rel(got[r], ref[r]) < 1e-12


def test_wilson_apply_f32():
    L = lib()
    dims = (4, 4, 4, 6)
    dl, ol = device_lattice(dims, 0.15, 0.5, 12, True, prec=1)
    X = synth.random_fields(8, dl.V, 6).reshape(8, -1)
    x = pack(dims, X, 8, 1)
    y = torch.empty_like(x)
    L.wilson_apply(dl, x, y)
    got = unpack(dims, y, 1)
    ref = ol.apply(X)
    # each output is a 9-term sum of O(1) products: a few units of FP32 rounding
    assert rel(got, ref) < 30 * U32


def test_wilson_free_field_plane_wave():
    """Free field: a plane wave is mapped to its closed-form eigen-combination."""
    L = lib()
    dims, kappa = (4, 4, 2, 4), 0.13
    dl, _ = device_lattice(dims, kappa, 0.0, 1, True, prec=0)
    lat = oracle.Lattice(dims, kappa, synth.unit_links(dims))
    A = dense.dense_matrix(lat)
    ev, R = np.linalg.eig(A)
    X = R[:, :4].T.copy()
    x = pack(dims, X, 4, 0)
    y = torch.empty_like(x)
    L.wilson_apply(dl, x, y)
    got = unpack(dims, y, 0)
    for i in range(4):
        assert rel(got[i], ev[i] * X[i]) < 1e-12


# ------------------------------------------------------------------ polynomials
def _roots(ol, degs, seed=3):
    ps = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, seed), degs)
    return ps


@pytest.mark.parametrize("deg,nrhs,rb,z4", [(0, 4, 4, True), (1, 4, 2, False), (5, 12, 4, True),
                                            (20, 16, 16, True), (20, 6, 2, False),
                                            (5, 256, 256, False)])      # the largest block width
def test_poly_apply_f64(deg, nrhs, rb, z4):
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 101, True)
    ps = _roots(ol, [max(deg, 1)])
    t = ps.inv_roots[max(deg, 1)][: deg + 1]
    poly = L.DevicePoly(dev_c128(t))
    if z4:
        nz = L.Noise(5, 1, 0, 10)
        B = oracle.z4(5, 1, 0, 10, nrhs, dl.V)
        xin = None
    else:
        nz = None
        B = synth.random_fields(nrhs, dl.V, 9).reshape(nrhs, -1)
        xin = pack(dims, B, rb, 0)
    y = L.empty_field(dl.V, nrhs, rb, 0)
    bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
    L.poly_apply(dl, poly, nrhs, rb, xin, nz, y, bhy, ws)
    ref_y, ref_bhy = ol.poly_apply(t, B)
    got = unpack(dims, y, 0)
    gb = bhy.cpu().numpy()
    for r in range(nrhs):
        assert rel(got[r], ref_y[r]) < 1e-12
        assert abs(gb[r] - ref_bhy[r]) <= 1e-12 * abs(ref_bhy[r])


def test_poly_scalar_mode_matches_vector_mode():
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 101, True)
    t = _roots(ol, [12]).inv_roots[12]
    poly = L.DevicePoly(dev_c128(t))
    nz = L.Noise(9, 1, 1, 0)
    ws = L.workspace(L.poly_workspace_size(dl, poly, 32, 16))
    b1 = torch.empty(32, dtype=torch.complex128, device="cuda")
    b2 = torch.empty_like(b1)
    L.poly_apply(dl, poly, 32, 16, None, nz, None, b1, ws)
    L.poly_apply(dl, poly, 32, 16, None, nz, L.empty_field(dl.V, 32, 16, 0), b2, ws)
    # scalar mode may run the t-sweep kernel: same values up to summation order
    assert torch.allclose(b1, b2, rtol=1e-13, atol=0)
    _, ref = ol.poly_apply(t, oracle.z4(9, 1, 1, 0, 32, dl.V))
    assert np.max(np.abs(b1.cpu().numpy() - ref) / np.abs(ref)) < 1e-12


@pytest.mark.parametrize("n_in,n_out,nrhs,rb", [(4, 3, 8, 4), (5, 1, 4, 4), (1, 4, 4, 2), (6, 5, 16, 16)])
def test_composite_f64(n_in, n_out, nrhs, rb):
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 101, True)
    r0 = synth.gaussian_start(ol.n, 4)
    ps = krylov.gmres_polys(ol.apply, r0, [max(n_in - 1, 1)])
    t_in = ps.inv_roots[max(n_in - 1, 1)][:n_in]
    opB = krylov.pp_operator(ol.apply, t_in, lambda t, v: ol.poly_apply(t, v)[0])
    t_out, _ = krylov.pp_gmres_roots(opB, r0, n_out=n_out)
    poly = L.DevicePoly(dev_c128(t_in), dev_c128(t_out))
    nz = L.Noise(21, 1, 0, 0)
    B = oracle.z4(21, 1, 0, 0, nrhs, dl.V)
    y = L.empty_field(dl.V, nrhs, rb, 0)
    bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
    L.poly_apply(dl, poly, nrhs, rb, None, nz, y, bhy, ws)
    ref_y, ref_b = ol.composite_apply(t_in, t_out, B)
    got = unpack(dims, y, 0)
    gb = bhy.cpu().numpy()
    for r in range(nrhs):
        assert rel(got[r], ref_y[r]) < 1e-12
        assert abs(gb[r] - ref_b[r]) <= 1e-12 * abs(ref_b[r])


def test_poly_apply_f32_bound():
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 101, True, prec=1)
    deg = 20
    t = _roots(ol, [deg]).inv_roots[deg]
    poly = L.DevicePoly(dev_c128(t))
    nrhs = 8
    nz = L.Noise(5, 1, 0, 0)
    B = oracle.z4(5, 1, 0, 0, nrhs, dl.V)
    bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, 8))
    L.poly_apply(dl, poly, nrhs, 8, None, nz, None, bhy, ws)
    _, ref = ol.poly_apply(t, B)
    kN = newton_amplification(ol.apply, t, B[:2])
    bound = 8 * deg * kN * U32
    err = np.abs(bhy.cpu().numpy() - ref) / np.abs(ref)
    assert np.max(err) < bound, (np.max(err), bound)


# ------------------------------------------------------------------ deflation
@pytest.fixture(scope="module")
def small_defl():
    dims = (2, 2, 2, 4)
    dl, ol = device_lattice(dims, 0.16, 0.5, 21, True)
    A = dense.dense_matrix(ol)
    lam, Z, pair = deflation.dense_triplets(A, 10, ol.gamma5)
    U = deflation.left_vectors(Z, pair, ol.gamma5)
    H = deflation.projection_matrix(ol.apply, Z, U)
    return dims, dl, ol, lam, Z, pair, U, H


def _device_defl(dims, Z, pair, U, H, prec=0, kpad=16):
    return device_defl(dims, Z, pair, U, H, prec, kpad)


@pytest.mark.parametrize("nrhs,rb,z4", [(8, 4, True), (5, 1, False), (40, 8, True),
                                        (1, 1, True), (1, 1, False)])     # one vector: the vector-unit kernel
def test_deflate_coeff(small_defl, nrhs, rb, z4):
    L = lib()
    dims, dl, ol, lam, Z, pair, U, H = small_defl
    D = _device_defl(dims, Z, pair, U, H)
    if z4:
        nz = L.Noise(3, 2, 1, 0)
        B = oracle.z4(3, 2, 1, 0, nrhs, dl.V)
        bf = None
    else:
        nz = None
        B = synth.random_fields(nrhs, dl.V, 2).reshape(nrhs, -1)
        bf = pack(dims, B, rb, 0)
    k = D.k
    zeta = torch.empty((k, nrhs), dtype=torch.complex128, device="cuda")
    omega = torch.empty_like(zeta)
    ws = L.workspace(L.deflate_workspace_size(dl, D, nrhs, rb))
    L.deflate_project(dl, D, L.DEFL_COEFF, nrhs, rb, bf, nz, zeta, omega, None, None, ws)
    rz, ro = deflation.projection_coefficients(Z, U, B)
    nb = np.linalg.norm(B, axis=1)
    assert np.max(np.abs(zeta.cpu().numpy() - rz) / nb) < 1e-12
    assert np.max(np.abs(omega.cpu().numpy() - ro) / (nb * np.linalg.norm(U, axis=1)[:, None])) < 1e-12


@pytest.mark.parametrize("nrhs,rb", [(100, 4), (1, 1)])
def test_deflate_coeff_large_random(nrhs, rb):
    """Tall-skinny V^H b over 4^4 x 12 rows with k = 20 padded to 32, ragged N;
    one vector (the Gram-Schmidt case) on the vector-unit kernel."""
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 5, True)
    k, n = 20, 12 * dl.V
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
    pair = np.arange(k)
    U = np.stack([ol.gamma5(Z[i]) for i in range(k)]) * 0.5
    D = _device_defl(dims, Z, pair, U, None, kpad=32)
    nz = L.Noise(8, 1, 2, 100)
    B = oracle.z4(8, 1, 2, 100, nrhs, dl.V)
    zeta = torch.empty((k, nrhs), dtype=torch.complex128, device="cuda")
    omega = torch.empty_like(zeta)
    ws = L.workspace(L.deflate_workspace_size(dl, D, nrhs, rb))
    L.deflate_project(dl, D, L.DEFL_COEFF, nrhs, rb, None, nz, zeta, omega, None, None, ws)
    rz, ro = deflation.projection_coefficients(Z, U, B)
    scale = np.linalg.norm(Z, axis=1)[:, None] * np.linalg.norm(B, axis=1)[None, :]
    assert np.max(np.abs(zeta.cpu().numpy() - rz) / scale) < 1e-13
    assert np.max(np.abs(omega.cpu().numpy() - ro) / scale) < 1e-13


@pytest.mark.parametrize("prec", [0, 1])
def test_deflate_at_the_largest_width(prec):
    """The deflation GEMMs at their largest width, kpad = 256 with a ragged
    k = 250 (pairs swapped, left vectors g5 z_pair / 2), on 4^4 x 12 rows:
    V^H b and U^H b for 48 Z4 vectors and X = V d, against the oracle's
    dense products (FP64 1e-13 of the terms' scale; FP32 operands and
    accumulation: the summation bound 4 m u32 sum|products|, m the number of
    complex terms, 12 V for the coefficients and k + 2 for X, d rounded
    once)."""
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 5, True, prec=prec)
    k, kpad, n = 250, 256, 12 * dl.V
    rng = np.random.default_rng(11)
    Z = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
    if prec == 1:
        Z = Z.astype(np.complex64).astype(np.complex128)     # the field-precision eigenvectors
    pair = np.arange(k)
    pair[0:2] = [1, 0]
    U = np.stack([ol.gamma5(Z[pair[i]]) for i in range(k)]) * 0.5
    D = device_defl(dims, Z, pair, U, None, prec, kpad)
    nrhs, rb = 48, 16
    nz = L.Noise(8, 1, 3, 7)
    B = oracle.z4(8, 1, 3, 7, nrhs, dl.V)
    zeta = torch.empty((k, nrhs), dtype=torch.complex128, device="cuda")
    omega = torch.empty_like(zeta)
    ws = L.workspace(L.deflate_workspace_size(dl, D, nrhs, rb))
    L.deflate_project(dl, D, L.DEFL_COEFF, nrhs, rb, None, nz, zeta, omega, None, None, ws)
    rz, ro = deflation.projection_coefficients(Z, U, B)
    if prec == 0:
        scale = np.linalg.norm(Z, axis=1)[:, None] * np.linalg.norm(B, axis=1)[None, :]
        assert np.max(np.abs(zeta.cpu().numpy() - rz) / scale) < 1e-13
        assert np.max(np.abs(omega.cpu().numpy() - ro) / scale) < 1e-13
    else:
        # a complex product is two real ones in each of Re and Im (2n real terms per sum):
        # |zeta - zeta*| <= gamma_2n (|Re| + |Im| parts) <= 4 n u32 sum|z||b|
        bz = 4 * n * U32 * (np.abs(Z) @ np.abs(B).T)
        assert np.all(np.abs(zeta.cpu().numpy() - rz) <= bz)
        assert np.all(np.abs(omega.cpu().numpy() - ro) <= 0.5 * bz[pair])
    d = rng.standard_normal((k, nrhs)) + 1j * rng.standard_normal((k, nrhs))
    X = L.empty_field(dl.V, nrhs, rb, prec)
    L.deflate_project(dl, D, L.DEFL_RECON, nrhs, rb, None, None, None, None, dev_c128(d), X, ws)
    ref = (Z.T @ d).T
    got = unpack(dims, X, prec)
    for r in (0, nrhs // 2, nrhs - 1):
        if prec == 0:
            assert rel(got[r], ref[r]) < 1e-13
        else:
            bx = 4 * (k + 2) * U32 * (np.abs(Z).T @ np.abs(d[:, r]))   # d rounded to FP32, k products summed
            assert np.all(np.abs(got[r] - ref[r]) <= bx)


def test_deflate_recon_and_project(small_defl):
    L = lib()
    dims, dl, ol, lam, Z, pair, U, H = small_defl
    D = _device_defl(dims, Z, pair, U, H)
    nrhs, rb = 6, 2
    k = D.k
    rng = np.random.default_rng(1)
    d = rng.standard_normal((k, nrhs)) + 1j * rng.standard_normal((k, nrhs))
    X = L.empty_field(dl.V, nrhs, rb, 0)
    ws = L.workspace(L.deflate_workspace_size(dl, D, nrhs, rb))
    L.deflate_project(dl, D, L.DEFL_RECON, nrhs, rb, None, None, None, None, dev_c128(d), X, ws)
    ref = (Z.T @ d).T
    assert rel(unpack(dims, X, 0), ref) < 1e-13
    # projection of Z4 vectors
    nz = L.Noise(4, 4, 4, 0)
    B = oracle.z4(4, 4, 4, 0, nrhs, dl.V)
    dd = torch.empty((k, nrhs), dtype=torch.complex128, device="cuda")
    L.deflate_project(dl, D, L.DEFL_PROJECT, nrhs, rb, None, nz, None, None, dd, X, ws)
    got = unpack(dims, X, 0)
    for r in range(nrhs):
        _, rr = deflation.left_right_projection(ol.apply, Z, U, H, B[r])
        assert rel(got[r], rr) < 1e-12
        assert np.linalg.norm(U.conj() @ got[r]) < 1e-11 * np.linalg.norm(B[r])


# ------------------------------------------------------------------ levels
def _run_level(dl, level, nrhs, rb, nz):
    L = lib()
    samples = torch.empty((nrhs, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, level, nrhs, rb))
    L.mlmc_level_estimate(dl, level, nrhs, rb, nz, samples, acc, ws)
    torch.cuda.synchronize()
    s = samples.cpu().numpy()
    return s[:, 0] + 1j * s[:, 1], s[:, 2] + 1j * s[:, 3], s[:, 4] + 1j * s[:, 5], acc.cpu().numpy()


def test_level_c1_two_levels():
    """C1 geometry: Tr(p20 - p5) and Tr(p5), 100 samples each, per-sample parity."""
    from synth.configs import C1
    L = lib()
    dl, ol = device_lattice(C1.dims, C1.kappa, C1.eps, C1.seed_links, True)
    ps = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, C1.seed_start), [20, 5])
    p20, p5 = L.DevicePoly(dev_c128(ps.inv_roots[20])), L.DevicePoly(dev_c128(ps.inv_roots[5]))
    for lvl, level in enumerate([L.DeviceLevel(L.OP_POLY, p20, L.OP_POLY, p5), L.DeviceLevel(L.OP_POLY, p5)]):
        nz = L.Noise(C1.seed_noise, C1.lattice_id, lvl, 0)
        s, hi, lo, acc = _run_level(dl, level, 100, 4, nz)
        B = oracle.z4(C1.seed_noise, C1.lattice_id, lvl, 0, 100, dl.V)
        _, rh = ol.poly_apply(ps.inv_roots[20 if lvl == 0 else 5], B)
        rl = ol.poly_apply(ps.inv_roots[5], B)[1] if lvl == 0 else np.zeros(100)
        assert np.max(np.abs(hi - rh) / np.abs(rh)) < 1e-12
        if lvl == 0:
            assert np.max(np.abs(lo - rl) / np.abs(rl)) < 1e-12
        rs = estimator.level_samples(rh, rl if lvl == 0 else None)
        assert np.max(np.abs(s - rs) / (np.abs(rh) + np.abs(rl))) < 1e-12
        est = estimator.level_estimate(rs)
        assert acc[0] == 100
        assert abs(acc[1] + 1j * acc[2] - est.mean) <= 1e-12 * (np.abs(rh).mean() + np.abs(rl).mean())
        assert abs(acc[3] / 99 - est.var) <= 1e-9 * est.var
        assert acc[4] == 0


def test_level_deflated_and_q_operator(small_defl):
    L = lib()
    dims, dl, ol, lam, Z, pair, U, H = small_defl
    D = _device_defl(dims, Z, pair, U, H)
    ps = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 7), [12, 3])
    t12, t3 = ps.inv_roots[12], ps.inv_roots[3]
    nrhs, rb = 24, 8
    # (a) Tr(p12 - p3) with Monte Carlo deflation
    c = deflation.deflation_coefficients(lam, lambda l: deflation.poly_eval(t12, l),
                                         lambda l: deflation.poly_eval(t3, l))
    lvl = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(t12)), L.OP_POLY, L.DevicePoly(dev_c128(t3)), D, True,
                        dev_c128(c))
    nz = L.Noise(1, 9, 1, 0)
    s, hi, lo, acc = _run_level(dl, lvl, nrhs, rb, nz)
    B = oracle.z4(1, 9, 1, 0, nrhs, dl.V)
    _, rh = ol.poly_apply(t12, B)
    _, rl = ol.poly_apply(t3, B)
    zeta, omega = deflation.projection_coefficients(Z, U, B)
    rs = estimator.level_samples(rh, rl, zeta, omega, c)
    scale = np.abs(rh) + np.abs(rl) + np.einsum("i,ir->r", np.abs(c), np.abs(zeta) * np.abs(omega))
    assert np.max(np.abs(s - rs) / scale) < 1e-12
    # (b) Tr(Q - p3): Q the deflated polynomial built on p12
    cq = deflation.deflation_coefficients(lam, lambda l: 1.0 / l, lambda l: deflation.poly_eval(t3, l))
    lq = L.DeviceLevel(L.OP_DEFLATED_POLY, L.DevicePoly(dev_c128(t12)), L.OP_POLY, L.DevicePoly(dev_c128(t3)), D,
                       True, dev_c128(cq))
    s2, hi2, lo2, _ = _run_level(dl, lq, nrhs, rb, nz)
    Q = deflation.DeflatedPoly(ol.apply, Z, U, H, lambda v: ol.poly_apply(t12, v)[0])
    rq = np.array([np.vdot(B[r], Q.apply(B[r])) for r in range(nrhs)])
    assert np.max(np.abs(hi2 - rq) / np.abs(rq)) < 1e-12
    rs2 = estimator.level_samples(rq, rl, zeta, omega, cq)
    scale2 = np.abs(rq) + np.abs(rl) + np.einsum("i,ir->r", np.abs(cq), np.abs(zeta) * np.abs(omega))
    assert np.max(np.abs(s2 - rs2) / scale2) < 1e-12


def test_level_accumulates_batches_and_is_deterministic():
    L = lib()
    dims = (4, 4, 4, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 101, True)
    t = _roots(ol, [6]).inv_roots[6]
    level = L.DeviceLevel(L.OP_POLY, L.DevicePoly(dev_c128(t)))
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    samples = torch.empty((32, 6), dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, level, 32, 8))
    allS = []
    for b in range(3):
        L.mlmc_level_estimate(dl, level, 32, 8, L.Noise(2, 1, 0, 32 * b), samples, acc, ws)
        allS.append(samples.clone())
    torch.cuda.synchronize()
    S = torch.cat(allS).cpu().numpy()
    s = S[:, 0] + 1j * S[:, 1]
    est = estimator.level_estimate(s)
    a = acc.cpu().numpy()
    assert a[0] == 96
    assert abs(a[1] + 1j * a[2] - est.mean) < 1e-12 * np.abs(s).mean()
    assert abs(a[3] / 95 - est.var) < 1e-10 * est.var
    # same inputs -> bitwise identical samples
    L.mlmc_level_estimate(dl, level, 32, 8, L.Noise(2, 1, 0, 0), samples, acc, ws)
    torch.cuda.synchronize()
    assert np.array_equal(samples.cpu().numpy(), S[:32])


# ------------------------------------------------------------------ t-sweep vs streaming kernel
@pytest.mark.parametrize("dims,ap,prec,nrhs,rb,z4", [
    ((8, 8, 8, 8), False, 0, 24, 8, True),     # the 8^4 workload geometry
    ((4, 4, 4, 4), True, 0, 12, 4, False),     # field input in a blocked layout
    ((4, 4, 4, 6), True, 0, 5, 1, True),
    ((8, 4, 2, 3), True, 0, 4, 2, True),       # odd Lt
    ((4, 4, 4, 1), True, 0, 4, 4, True),       # Lt = 1: the t-neighbours are the site itself
    ((8, 8, 8, 4), True, 1, 16, 16, True),     # FP32
    # planes larger than one workgroup: xyz-blocks with a halo (FP32), with
    # enough vectors for a workgroup's worth of threads per CU (256 CUs)
    ((8, 8, 16, 4), True, 1, 128, 4, True),    # 8 x 8 x 8 blocks, cut in z
    ((16, 8, 8, 3), True, 1, 128, 2, False),   # 16-wide 512-site blocks, field input, odd Lt
    ((12, 12, 12, 2), True, 1, 80, 8, True),   # 12 x 4 x 4 blocks, cut in y and z
    ((16, 16, 16, 2), False, 1, 32, 4, True),  # eight 16 x 8 x 4 blocks of a 16^3 plane
    ((32, 8, 8, 2), True, 1, 64, 16, True),    # 16-wide 512-site blocks, cut in x
])
def test_sweep_matches_oracle_and_streaming(dims, ap, prec, nrhs, rb, z4):
    L = lib()
    dl, ol = device_lattice(dims, 0.14, 0.4, 33, ap, prec=prec)
    plan = L.sweep_plan(dl, nrhs, rb)
    P = dims[0] * dims[1] * dims[2]
    assert plan["ok"] and plan["halo"] == (P > 512), plan
    print(dims, "block", plan["block"], "halo sites", plan["halo_sites"])
    deg = 9
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 1), [deg]).inv_roots[deg]
    poly = L.DevicePoly(dev_c128(t))
    if z4:
        nz, xin = L.Noise(4, 2, 0, 7), None
        B = oracle.z4(4, 2, 0, 7, nrhs, dl.V)
    else:
        nz = None
        B = synth.random_fields(nrhs, dl.V, 8).reshape(nrhs, -1)
        xin = pack(dims, B, rb, prec)
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
    out = {}
    for opt in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, opt)
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, nrhs, rb, xin, nz, None, bhy, ws)
        torch.cuda.synchronize()
        out[opt] = bhy.cpu().numpy()
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    _, ref = ol.poly_apply(t, B)
    tol = 1e-12 if prec == 0 else 8 * deg * newton_amplification(ol.apply, t, B[:2]) * U32
    for opt in (1, 0):
        assert np.max(np.abs(out[opt] - ref) / np.abs(ref)) < tol, opt


# ------------------------------------------------------------------ SU(3) links read as two rows
@pytest.mark.parametrize("dims,ap", [((4, 4, 4, 4), True), ((8, 8, 8, 2), False)])
def test_two_row_links_match_oracle(dims, ap):
    """link_rows = 2 (row 2 rebuilt as conj(row 0 x row 1)) gives the full-link
    operator to FP64 rounding for SU(3) links: A x, and scalar-mode
    polynomials on both the t-sweep and the streaming kernel."""
    L = lib()
    dl, ol = device_lattice(dims, 0.14, 0.5, 77, ap, 0, link_rows=2)
    V = dl.V
    X = synth.random_fields(8, V, 3).reshape(8, 12 * V)
    x = pack(dims, X, 4, 0)
    y = L.empty_field(V, 8, 4, 0)
    L.wilson_apply(dl, x, y)
    Y = unpack(dims, y, 0)
    R = ol.apply(X)
    for r in range(8):
        assert rel(Y[r], R[r]) < 1e-13
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 5), [9]).inv_roots[9]
    B = oracle.z4(5, 6, 7, 0, 16, V)
    _, ref = ol.poly_apply(t, B)
    for sweep in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, sweep)
        poly = L.DevicePoly(dev_c128(t))
        bhy = torch.empty(16, dtype=torch.complex128, device="cuda")
        ws = L.workspace(L.poly_workspace_size(dl, poly, 16, 8))
        L.poly_apply(dl, poly, 16, 8, None, L.Noise(5, 6, 7, 0), None, bhy, ws)
        assert np.max(np.abs(bhy.cpu().numpy() - ref) / np.abs(ref)) < 1e-12
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    # FP32 two-row links: the FP32 operator bound
    dl32, _ = device_lattice(dims, 0.14, 0.5, 77, ap, 1, link_rows=2)
    x32 = pack(dims, X, 4, 1)
    y32 = L.empty_field(V, 8, 4, 1)
    L.wilson_apply(dl32, x32, y32)
    Y32 = unpack(dims, y32, 1)
    for r in range(8):
        assert rel(Y32[r], R[r]) < 1e-6


def test_gauge_unitarity_check():
    L = lib()
    dims = (4, 4, 2, 4)
    U = synth.gauge_links(dims, 0.5, 8)
    V = int(np.prod(dims))
    for scale, prec in ((1.0, 0), (1.01, 0), (1.0, 1)):
        Us = U * scale
        g = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
        L.pack_gauge(dims, prec, torch.from_numpy(np.ascontiguousarray(Us)).cuda(), g)
        du, dd = L.gauge_unitarity(dims, prec, g)
        M = Us.reshape(-1, 3, 3)
        if prec == 1:
            M = M.astype(np.complex64).astype(np.complex128)
        want_u = np.max(np.abs(M @ np.conj(np.swapaxes(M, 1, 2)) - np.eye(3)))
        want_d = np.max(np.abs(np.linalg.det(M) - 1.0))
        assert abs(du - want_u) <= 1e-12 + 1e-9 * want_u and abs(dd - want_d) <= 1e-12 + 1e-9 * want_d
        if scale == 1.0:
            assert max(du, dd) < (1e-13 if prec == 0 else 1e-6)
        else:
            assert abs(du - (1.01 ** 2 - 1)) < 1e-9 and abs(dd - (1.01 ** 3 - 1)) < 1e-9


def test_link_rows_validated():
    L = lib()
    dl, _ = device_lattice((2, 2, 2, 4), 0.1, 0.5, 1, True, 0, link_rows=5)
    x = L.empty_field(dl.V, 1, 1, 0)
    y = L.empty_field(dl.V, 1, 1, 0)
    with pytest.raises(L.MpmcError):
        L.wilson_apply(dl, x, y)


def test_blocked_sweep_two_row_links():
    """xyz-blocks with a halo and two-row SU(3) links against the oracle."""
    L = lib()
    dims = (16, 16, 16, 2)
    dl, ol = device_lattice(dims, 0.14, 0.4, 35, True, prec=1, link_rows=2)
    N = 32
    assert L.sweep_plan(dl, N, 8)["halo"]
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 2), [6]).inv_roots[6]
    poly = L.DevicePoly(dev_c128(t))
    ws = L.workspace(L.poly_workspace_size(dl, poly, N, 8))
    bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
    L.poly_apply(dl, poly, N, 8, None, L.Noise(6, 6, 6, 0), None, bhy, ws)
    B = oracle.z4(6, 6, 6, 0, N, dl.V)
    _, ref = ol.poly_apply(t, B)
    assert np.max(np.abs(bhy.cpu().numpy() - ref) / np.abs(ref)) < 8 * 6 * newton_amplification(ol.apply, t, B[:2]) * U32


@pytest.mark.parametrize("dims,prec,nrhs,rb,field_in,n_in,n_out", [
    ((4, 4, 4, 4), 0, 16, 16, False, 4, 3),     # whole plane, noise input
    ((4, 4, 4, 4), 0, 8, 4, True, 3, 4),        # field input at block width 4, dot against the noise
    ((8, 8, 8, 4), 1, 16, 16, False, 5, 2),     # FP32
    ((16, 8, 8, 2), 1, 128, 8, True, 3, 3),     # FP32 blocks with a halo, field input
])
def test_scalar_composite_sweep(dims, prec, nrhs, rb, field_in, n_in, n_out):
    """Scalar-mode double polynomial b^H p_in(A) p_out(A p_in(A)) x against the
    noise b: the inner chains on the t-sweep (block width 1 inside) agree with
    the streaming kernel and with the oracle."""
    L = lib()
    dl, ol = device_lattice(dims, 0.14, 0.4, 35, True, prec=prec)
    r0 = synth.gaussian_start(ol.n, 6)
    ps = krylov.gmres_polys(ol.apply, r0, [n_in - 1])
    t_in = ps.inv_roots[n_in - 1]
    opB = krylov.pp_operator(ol.apply, t_in, lambda t, v: ol.poly_apply(t, v)[0])
    t_out, _ = krylov.pp_gmres_roots(opB, r0, n_out=n_out)
    poly = L.DevicePoly(dev_c128(t_in), dev_c128(t_out))
    nz = L.Noise(13, 4, 2, 5)
    B = oracle.z4(13, 4, 2, 5, nrhs, dl.V)
    if field_in:
        X = synth.random_fields(nrhs, dl.V, 12).reshape(nrhs, -1)
        xin = pack(dims, X, rb, prec)
    else:
        X, xin = B, None
    if dl.dims[0] * dl.dims[1] * dl.dims[2] > 512:
        assert L.sweep_plan(dl, nrhs, 1)["halo"]
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
    out = {}
    for opt in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, opt)
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, nrhs, rb, xin, nz, None, bhy, ws)
        torch.cuda.synchronize()
        out[opt] = bhy.cpu().numpy()
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    ref_y, _ = ol.composite_apply(t_in, t_out, X)
    ref = np.einsum("rn,rn->r", B.conj(), ref_y)
    d = n_in * n_out
    tol = 1e-12 if prec == 0 else 8 * d * composite_amplification(ol.apply, t_in, t_out, X[:2]) * U32
    for opt in (1, 0):
        err = np.max(np.abs(out[opt] - ref) / np.abs(ref))
        print(dims, "sweep" if opt else "streaming", f"rel err {err:.2e}")
        assert err < tol, opt
    if prec == 0:
        assert np.max(np.abs(out[1] - out[0]) / np.abs(out[0])) < 1e-13


@pytest.mark.parametrize("dims,prec,nrhs,field_in,dot", [
    ((8, 8, 8, 8), 0, 256, False, True),      # whole plane, noise input, y and b^H y
    ((8, 8, 8, 4), 1, 256, True, False),      # FP32, field input, y only
    ((16, 8, 8, 2), 1, 128, False, False),    # FP32 blocks with a halo
])
def test_vector_mode_sweep(dims, prec, nrhs, field_in, dot):
    """Vector mode y = p(A) x at block width 1 on the t-sweep (y accumulated
    in the same launches) against the streaming kernel and, for sampled
    vectors, the oracle."""
    L = lib()
    dl, ol = device_lattice(dims, 0.14, 0.4, 37, True, prec=prec)
    plan = L.sweep_plan(dl, nrhs, 1)
    assert plan["ok"]
    deg = 6
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 2), [deg]).inv_roots[deg]
    poly = L.DevicePoly(dev_c128(t))
    nz = L.Noise(17, 5, 1, 3)
    if field_in:
        X = synth.random_fields(nrhs, dl.V, 14).reshape(nrhs, -1)
        xin = pack(dims, X, 1, prec)
    else:
        X, xin = None, None
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, 1))
    yt, ys, bs = {}, {}, {}
    for opt in (1, 0):
        L.set_option(L.OPT_PLANE_SWEEP, opt)
        yt[opt] = L.empty_field(dl.V, nrhs, 1, prec)
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda") if dot else None
        L.poly_apply(dl, poly, nrhs, 1, xin, None if field_in else nz, yt[opt], bhy, ws)
        torch.cuda.synchronize()
        ys[opt] = yt[opt].cpu().numpy()
        bs[opt] = bhy.cpu().numpy() if dot else None
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    scale = np.max(np.abs(ys[0]))
    x0 = X[0] if field_in else oracle.z4(17, 5, 1, 3, 1, dl.V)[0]
    kN = newton_amplification(ol.apply, t, x0[None, :])
    tol_same = 1e-13 if prec == 0 else 8 * deg * kN * U32
    assert np.max(np.abs(ys[1] - ys[0])) <= tol_same * scale
    Y = unpack(dims, yt[1], prec)
    for r in (0, nrhs // 2 + 1, nrhs - 1):
        x = X[r] if field_in else oracle.z4(17, 5, 1, 3 + r, 1, dl.V)[0]
        want, _ = ol.poly_apply(t, x)
        err = rel(Y[r], want)
        print(dims, "vector", r, f"rel err {err:.2e}")
        assert err < (1e-12 if prec == 0 else 8 * deg * newton_amplification(ol.apply, t, x[None, :]) * U32)
        if dot:
            assert abs(bs[1][r] - np.vdot(x, want)) <= 1e-12 * abs(np.vdot(x, want))


@pytest.mark.parametrize("dims,prec,nrhs,rb,chunks", [
    ((8, 8, 8, 8), 0, 32, 8, (2, 4, 8)),        # whole plane, down to one plane per chunk
    ((4, 4, 4, 6), 0, 5, 1, (2, 3, 6)),         # whole plane, odd chunk lengths, 5 vectors
    ((8, 8, 8, 8), 1, 64, 16, (2, 4)),          # FP32 whole plane (own backward-hop products)
    # blocked planes are offered only when the unchunked launch already
    # covers the CUs: 32 x 8 workgroups of 512 sites, 64 x 9 of 192 (two per CU)
    ((16, 16, 16, 8), 1, 32, 8, (2, 4, 8)),     # FP32 16 x 8 x 4 blocks with a halo
    ((12, 12, 12, 4), 1, 64, 8, (2, 4)),        # FP32 12 x 4 x 4 blocks, cut in y and z
])
def test_sweep_t_chunks(dims, prec, nrhs, rb, chunks):
    """The t-sweep cut into k t-chunks (each workgroup walks Lt / k planes,
    starting from a prologue that forms the -t term of its first plane from
    the plane before; the partial sums of every (chunk, block) are summed
    after the launch), with an inverse root 0 among the roots (a step without
    hops): scalar mode on Z4 noise and vector mode y = p(A) b with b^H y,
    against the oracle and against the unchunked sweep, for every k."""
    L = lib()
    dl, ol = device_lattice(dims, 0.14, 0.4, 57, True, prec=prec)
    deg = 7
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 4), [deg]).inv_roots[deg]
    t = np.insert(t, 3, 0.0)
    poly = L.DevicePoly(dev_c128(t))
    nz = L.Noise(8, 3, 0, 5)
    B = oracle.z4(8, 3, 0, 5, nrhs, dl.V)
    _, ref = ol.poly_apply(t, B)
    kN = newton_amplification(ol.apply, t, B[:2])
    tol = 1e-12 if prec == 0 else 8 * len(t) * kN * U32
    ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, rb))
    ws1 = L.workspace(L.poly_workspace_size(dl, poly, nrhs, 1))
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    got = {}
    try:
        for k in (1,) + tuple(chunks):
            L.set_option(L.OPT_SWEEP_CHUNKS, k)
            plan = L.sweep_plan(dl, nrhs, rb)
            assert plan["ok"] and plan["chunks"] == k and plan["halo"] == (dl.V // dims[3] > 512), plan
            assert L.sweep_plan(dl, nrhs, 1)["chunks"] == k
            bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
            L.poly_apply(dl, poly, nrhs, rb, None, nz, None, bhy, ws)
            y = L.empty_field(dl.V, nrhs, 1, prec)
            bhy1 = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
            L.poly_apply(dl, poly, nrhs, 1, None, nz, y, bhy1, ws1)
            torch.cuda.synchronize()
            got[k] = (bhy.cpu().numpy(), unpack(dims, y, prec), bhy1.cpu().numpy())
    finally:
        L.set_option(L.OPT_SWEEP_CHUNKS, 0)
    for k, (s, Y, s1) in got.items():
        err = np.max(np.abs(s - ref) / np.abs(ref))
        print(dims, "chunks", k, f"scalar rel err {err:.2e}")
        assert err < tol, k
        assert np.max(np.abs(s1 - ref) / np.abs(ref)) < tol, k
        for r in (0, nrhs - 1):
            want, _ = ol.poly_apply(t, B[r])
            assert rel(Y[r], want) < tol, (k, r)
        # against the unchunked sweep: the same site arithmetic, partial sums
        # grouped differently
        s0, Y0, _ = got[1]
        assert np.max(np.abs(s - s0) / np.abs(s0)) < (1e-13 if prec == 0 else tol), k
        assert np.max(np.abs(Y - Y0)) <= (1e-13 if prec == 0 else tol) * np.max(np.abs(Y0)), k


@pytest.mark.parametrize("chunks", [2, 4])
def test_t_chunks_in_probing_composite_and_identity(chunks):
    """The t-chunked sweep (FP64, 4^4, chunks of 2 and 1 planes) on its three
    other paths: probe vectors generated inside the kernel (the exact trace of
    a degree-3 polynomial against the oracle's brute-force colouring), the
    double polynomial's inner chains (scalar mode against the oracle's
    composite polynomial), and steps without hops (kappa = 0, A = I: every
    sample equals 12 V p(1))."""
    L = lib()
    from oracle import probing as oprobe
    from paper_2306_09559_amd import probing
    dims = (4, 4, 4, 4)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    L.set_option(L.OPT_SWEEP_CHUNKS, chunks)
    try:
        # probe vectors drawn in the kernel
        dl, ol = device_lattice(dims, 0.14, 0.5, 21, True)
        assert L.sweep_plan(dl, 64, 1)["chunks"] == chunks
        deg = 3
        t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 2), [deg]).inv_roots[deg]
        res = probing.probe_trace(dl, L.DevicePoly(dev_c128(t)), probing.colouring(dims, deg), nrhs=64, rb=1,
                                  in_kernel=True)
        want = oprobe.probe_trace(ol, t, oprobe.distance_colouring(dims, deg))
        assert abs(res.trace - want) <= 1e-12 * abs(want), (res.trace, want)
        # the double polynomial's inner chains
        dl, ol = device_lattice(dims, 0.14, 0.4, 35, True)
        r0 = synth.gaussian_start(ol.n, 6)
        t_in = krylov.gmres_polys(ol.apply, r0, [3]).inv_roots[3]
        opB = krylov.pp_operator(ol.apply, t_in, lambda tt, v: ol.poly_apply(tt, v)[0])
        t_out, _ = krylov.pp_gmres_roots(opB, r0, n_out=3)
        nrhs = 16
        assert L.sweep_plan(dl, nrhs, 1)["chunks"] == chunks
        poly = L.DevicePoly(dev_c128(t_in), dev_c128(t_out))
        ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, 4))
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, nrhs, 4, None, L.Noise(13, 4, 2, 5), None, bhy, ws)
        torch.cuda.synchronize()
        B = oracle.z4(13, 4, 2, 5, nrhs, dl.V)
        ref_y, _ = ol.composite_apply(t_in, t_out, B)
        ref = np.einsum("rn,rn->r", B.conj(), ref_y)
        assert np.max(np.abs(bhy.cpu().numpy() - ref) / np.abs(ref)) < 1e-12
        # steps without hops
        dl, _ = device_lattice(dims, 0.0, 0.4, 43, True)
        tz = np.array([0.6, 0.5 + 0.1j, 0.4, 0.3j, 0.2])
        p1 = complex(deflation.poly_eval(tz, 1.0))
        poly = L.DevicePoly(dev_c128(tz))
        ws = L.workspace(L.poly_workspace_size(dl, poly, nrhs, 4))
        bhy = torch.empty(nrhs, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, nrhs, 4, None, L.Noise(3, 1, 0, 0), None, bhy, ws)
        torch.cuda.synchronize()
        assert np.max(np.abs(bhy.cpu().numpy() - 12 * dl.V * p1)) <= 1e-13 * abs(12 * dl.V * p1)
    finally:
        L.set_option(L.OPT_SWEEP_CHUNKS, 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_streaming_link_load_paths(prec):
    """The streaming kernel's two ways of reading the links (buffer loads
    below 4 GiB, 64-bit flat addresses otherwise): A x and a scalar-mode
    polynomial agree with the oracle on both, and with each other to the
    rounding the FMA contraction of each path allows."""
    L = lib()
    dims, N, rb = (8, 8, 8, 6), 32, 16
    dl, ol = device_lattice(dims, 0.14, 0.4, 91, True, prec=prec)
    V = dl.V
    X = synth.random_fields(N, V, 92).reshape(N, -1)
    x = pack(dims, X, rb, prec)
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 93), [6]).inv_roots[6]
    poly = L.DevicePoly(dev_c128(t))
    L.set_option(L.OPT_PLANE_SWEEP, 0)
    got = {}
    for buf in (1, 0):
        L.set_option(L.OPT_LINK_BUF, buf)
        y = L.empty_field(V, N, rb, prec)
        L.wilson_apply(dl, x, y)
        ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
        bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
        L.poly_apply(dl, poly, N, rb, None, L.Noise(9, 1, 2, 0), None, bhy, ws)
        torch.cuda.synchronize()
        got[buf] = (unpack(dims, y, prec), bhy.cpu().numpy())
    L.set_option(L.OPT_LINK_BUF, 1)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    R = ol.apply(X)
    _, ref = ol.poly_apply(t, oracle.z4(9, 1, 2, 0, N, V))
    bound = 1e-12 if prec == 0 else 8 * 6 * newton_amplification(ol.apply, t, oracle.z4(9, 1, 2, 0, 2, V)) * U32
    for buf in (1, 0):
        for r in (0, N // 2, N - 1):
            assert rel(got[buf][0][r], R[r]) < (1e-13 if prec == 0 else 1e-6)
        assert np.max(np.abs(got[buf][1] - ref) / np.abs(ref)) < bound
    assert np.max(np.abs(got[1][1] - got[0][1]) / np.abs(got[0][1])) < bound


@pytest.mark.parametrize("prec", [0, 1])
def test_streaming_work_order_changes_no_value(prec):
    """The streaming kernel's slab work order (each XCD a z-slab swept along
    t) only reorders workgroups: A x, scalar-mode and vector-mode polynomials
    and the double polynomial are bit-identical to the plain order, and
    match the oracle."""
    L = lib()
    # 16 tiles per xyz-plane (the slab order applies), 9 RHS blocks
    dims, N, rb = (8, 8, 8, 6), 72, 8
    dl, ol = device_lattice(dims, 0.14, 0.4, 81, True, prec=prec)
    V = dl.V
    X = synth.random_fields(N, V, 82).reshape(N, -1)
    x = pack(dims, X, rb, prec)
    t = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, 83), [5]).inv_roots[5]
    t_out = np.array([0.7, 0.5 + 0.1j, 0.9])
    single, comp = L.DevicePoly(dev_c128(t)), L.DevicePoly(dev_c128(t), dev_c128(t_out))
    L.set_option(L.OPT_PLANE_SWEEP, 0)
    got = {}
    for slab in (0, 1):
        L.set_option(L.OPT_HOP_SLAB, slab)
        y = L.empty_field(V, N, rb, prec)
        L.wilson_apply(dl, x, y)
        ys, bs, bc = L.empty_field(V, N, rb, prec), [], []
        for poly, out in ((single, bs), (comp, bc)):
            ws = L.workspace(L.poly_workspace_size(dl, poly, N, rb))
            bhy = torch.empty(N, dtype=torch.complex128, device="cuda")
            L.poly_apply(dl, poly, N, rb, None, L.Noise(8, 1, 2, 0), ys if poly is single else None, bhy, ws)
            torch.cuda.synchronize()
            out.append(bhy.cpu().numpy())
        got[slab] = (unpack(dims, y, prec), unpack(dims, ys, prec), bs[0], bc[0])
    L.set_option(L.OPT_HOP_SLAB, 1)
    L.set_option(L.OPT_PLANE_SWEEP, 1)
    for a, b in zip(got[0], got[1]):
        assert np.array_equal(a, b)
    R = ol.apply(X)
    for r in (0, N - 1):
        assert rel(got[1][0][r], R[r]) < (1e-13 if prec == 0 else 1e-6)
    _, ref = ol.poly_apply(t, oracle.z4(8, 1, 2, 0, N, V))
    bound = 1e-12 if prec == 0 else 8 * 5 * newton_amplification(ol.apply, t, oracle.z4(8, 1, 2, 0, 2, V)) * U32
    assert np.max(np.abs(got[1][2] - ref) / np.abs(ref)) < bound
