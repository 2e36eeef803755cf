"""The top level Tr(A^{-1} - p_1(A)) on the GPU (Sec. 5 step 3a): Krylov-basis
block kernels, the deflated PP-GMRES solver with FP64-outer / FP32-inner
iterative refinement, and the SOLVE level against the oracle.  Inputs come
from `synth` and roots / triplets from the oracle; expected values from the
oracle (dense solves on lattices small enough) or from properties that hold
at any size (the FP64 residual through the oracle operator)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import deflation, dense, krylov, solve as osolve
from gpu_helpers import dev_c128, device_defl, device_lattice, lib, pack, rel, unpack

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# ------------------------------------------------------------------ block kernels
@pytest.mark.parametrize("prec,dims,k,nrhs,rb", [(0, (4, 4, 2, 3), 1, 4, 4), (0, (3, 4, 4, 5), 9, 8, 2),
                                                  (1, (4, 4, 2, 3), 8, 16, 16), (1, (5, 3, 4, 4), 17, 6, 2),
                                                  (0, (2, 2, 2, 2), 3, 1, 1)])
def test_block_dot_and_axpy(prec, dims, k, nrhs, rb):
    L = lib()
    V = int(np.prod(dims))
    n = 12 * V
    X = synth.random_fields(nrhs, V, 5).reshape(nrhs, n)
    Bs = synth.random_fields(k * nrhs, V, 6).reshape(k, nrhs, n)
    xf = pack(dims, X, rb, prec)
    basis = torch.stack([pack(dims, Bs[i], rb, prec) for i in range(k)]).contiguous()
    # the values the device holds (rounded to the field precision)
    Xr = unpack(dims, xf, prec)
    Br = np.stack([unpack(dims, basis[i], prec) for i in range(k)])
    out = torch.empty((k, nrhs), dtype=torch.complex128, device="cuda")
    ws = L.workspace(L.field_block_dot_workspace_size(dims, nrhs, rb, k))
    L.field_block_dot(dims, prec, basis, k, xf, out, ws)
    want = np.einsum("irn,rn->ir", Br.conj(), Xr)
    scale = np.einsum("irn,rn->ir", np.abs(Br), np.abs(Xr))
    assert np.max(np.abs(out.cpu().numpy() - want) / scale) < 1e-13
    rng = np.random.default_rng(7)
    coeff = rng.standard_normal((k, nrhs)) + 1j * rng.standard_normal((k, nrhs))
    for acc in (False, True):
        y = pack(dims, X, rb, prec)
        L.field_block_axpy(dims, prec, basis, k, dev_c128(coeff), y, acc)
        got = unpack(dims, y, prec)
        want = np.einsum("ir,irn->rn", coeff, Br) + (Xr if acc else 0)
        mag = np.einsum("ir,irn->rn", np.abs(coeff), np.abs(Br)) + (np.abs(Xr) if acc else 0)
        # summed in FP64 and rounded once to the field precision
        tol = 1e-14 if prec == 0 else 1.01 * U32
        assert np.max(np.abs(got - want) / (mag + np.abs(want))) < tol


def test_axpby_mixed_roundtrip():
    L = lib()
    dims, nrhs, rb = (4, 4, 4, 2), 8, 4
    V = int(np.prod(dims))
    X = synth.random_fields(nrhs, V, 9).reshape(nrhs, 12 * V)
    x64 = pack(dims, X, rb, 0)
    x32 = L.empty_field(V, nrhs, rb, 1)
    alpha = np.arange(1, nrhs + 1) * (0.5 - 0.25j)
    L.field_axpby_mixed(dims, dev_c128(alpha), x64, None, x32)
    got = unpack(dims, x32, 1)
    want = alpha[:, None] * X
    assert np.max(np.abs(got - want) / np.abs(want).max(axis=1, keepdims=True)) < 1.01 * U32
    # back to FP64, accumulated: y = 2 x32 + 1 * y
    y64 = pack(dims, X, rb, 0)
    L.field_axpby_mixed(dims, dev_c128(2 * np.ones(nrhs)), x32, dev_c128(np.ones(nrhs)), y64)
    assert rel(unpack(dims, y64, 0), 2 * got + X) < 1e-15


# ------------------------------------------------------------------ the solver
def _pin_roots(ol, n_in, seed):
    ps = krylov.gmres_polys(ol.apply, synth.gaussian_start(ol.n, seed), [n_in - 1])
    return ps.inv_roots[n_in - 1]


def _oracle_defl(dims, ol, k, prec):
    A = dense.dense_matrix(ol)
    lam, Z, pair = deflation.dense_triplets(A, k, ol.gamma5)
    U = deflation.left_vectors(Z, pair, ol.gamma5)
    H = deflation.projection_matrix(ol.apply, Z, U)
    return lam, Z, pair, U, H, device_defl(dims, Z, pair, U, H, prec=prec)


@pytest.mark.parametrize("inner_prec,deflated", [(0, False), (1, False), (1, True)])
def test_solver_reaches_rtolle(inner_prec, deflated):
    """x = A^{-1} b to 1e-6 in FP64 through the oracle operator; the mixed
    solver needs more than one refinement step to get there, and x matches
    the dense LU solution to the conditioning of the residual."""
    L = lib()
    from paper_2306_09559_amd.solve import MixedPPGMRES
    dims = (4, 4, 2, 4)
    dl64, ol = device_lattice(dims, 0.15, 0.5, 101, True, 0)
    dli = dl64 if inner_prec == 0 else device_lattice(dims, 0.15, 0.5, 101, True, 1)[0]
    t_in = _pin_roots(ol, 6, 3)
    D = _oracle_defl(dims, ol, 8, inner_prec)[-1] if deflated else None
    nrhs, rb = 8, 4
    nz = L.Noise(31, 3, 0, 0)
    b = L.empty_field(dl64.V, nrhs, rb, 0)
    L.z4_fill(dims, 0, nz, b)
    x = L.empty_field(dl64.V, nrhs, rb, 0)
    sol = MixedPPGMRES(dl64, dli, L.DevicePoly(dev_c128(t_in)), D, 12, nrhs, rb)
    st = sol.solve(b, x, tol=1e-6)
    B = oracle.z4(31, 3, 0, 0, nrhs, dl64.V)
    X = unpack(dims, x, 0)
    res = osolve.residual(ol, B, X)
    print(f"outer {st.outer} cycles {st.cycles} steps {st.arnoldi_steps} mvps {st.mvps} res {res.max():.2e}")
    assert np.max(res) <= 1e-6
    assert np.allclose(res, st.rel_res, rtol=1e-6, atol=1e-15)
    if inner_prec == 1:
        assert st.outer >= 2        # the FP32 cycles alone cannot reach 1e-6 at inner_tol 1e-4
    Xs = osolve.dense_solve(ol, B)
    cond = np.linalg.cond(dense.dense_matrix(ol))
    for r in range(nrhs):
        assert rel(X[r], Xs[r]) <= cond * 1e-6


# ------------------------------------------------------------------ the SOLVE level
@pytest.mark.parametrize("prec", [0, 1])
def test_top_level_samples_match_oracle(prec):
    """s = b^H x - b^H Q b with Q the deflated composite p_1 (Sec. 4.3):
    each sample within |b^H (x - x*)| (the solve tolerance, bounded through
    the dense solution x*) plus the polynomial's rounding bound."""
    L = lib()
    from paper_2306_09559_amd.solve import MixedPPGMRES
    dims = (4, 4, 2, 4)
    dl64, ol = device_lattice(dims, 0.15, 0.5, 101, True, 0)
    dl = dl64 if prec == 0 else device_lattice(dims, 0.15, 0.5, 101, True, 1)[0]
    n_in, n_out = 5, 3
    t_in = _pin_roots(ol, n_in, 3)
    opB = krylov.pp_operator(ol.apply, t_in, lambda t, v: ol.poly_apply(t, v)[0])
    t_out, _ = krylov.pp_gmres_roots(opB, synth.gaussian_start(ol.n, 4), n_out=n_out)
    lam, Z, pair, U, H, D = _oracle_defl(dims, ol, 8, prec)
    nrhs, rb = 8, 8
    nz = L.Noise(41, 3, 0, 0)
    b = L.empty_field(dl64.V, nrhs, rb, 0)
    L.z4_fill(dims, 0, nz, b)
    x64 = L.empty_field(dl64.V, nrhs, rb, 0)
    sol = MixedPPGMRES(dl64, dl, L.DevicePoly(dev_c128(t_in)), D, 12, nrhs, rb)
    sol.solve(b, x64, tol=1e-6)
    xl = x64
    if prec == 1:
        xl = L.empty_field(dl64.V, nrhs, rb, 1)
        L.field_axpby_mixed(dims, dev_c128(np.ones(nrhs)), x64, None, xl)
    lvl = L.DeviceLevel(L.OP_SOLVE, None, L.OP_DEFLATED_POLY, L.DevicePoly(dev_c128(t_in), dev_c128(t_out)), D,
                        False, None, xl)
    samples = torch.empty((nrhs, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(L.level_workspace_size(dl, lvl, nrhs, rb))
    L.mlmc_level_estimate(dl, lvl, nrhs, rb, nz, samples, acc, ws)
    S = samples.cpu().numpy()
    s, hi, lo = S[:, 0] + 1j * S[:, 1], S[:, 2] + 1j * S[:, 3], S[:, 4] + 1j * S[:, 5]
    B = oracle.z4(41, 3, 0, 0, nrhs, dl64.V)
    Xs = osolve.dense_solve(ol, B)
    Q = deflation.DeflatedPoly(ol.apply, Z, U, H, lambda v: ol.composite_apply(t_in, t_out, v)[0])
    QB = np.array([Q.apply(bb) for bb in B])
    rs = osolve.top_level_samples(B, Xs, QB)
    X = unpack(dims, x64, 0)
    nb = np.linalg.norm(B, axis=1)
    solve_err = nb * np.linalg.norm(X - Xs, axis=1)
    rhi = np.einsum("ri,ri->r", B.conj(), Xs)
    rlo = np.einsum("ri,ri->r", B.conj(), QB)
    if prec == 0:
        assert np.all(np.abs(hi - rhi) <= solve_err + 1e-12 * np.abs(rhi))
        assert np.max(np.abs(lo - rlo) / np.abs(rlo)) < 1e-12
        assert np.all(np.abs(s - rs) <= solve_err + 1e-12 * (np.abs(rhi) + np.abs(rlo)))
    else:
        # x rounded to FP32 for the dot; Q b with FP32 entries: composite degree d and
        # the projection, bounded with the Cauchy-Schwarz scale |b| |Q b|
        d = n_in * n_out - 1 + 1
        hi_b = solve_err + nb * np.linalg.norm(Xs, axis=1) * U32
        lo_b = 8 * d * U32 * nb * np.linalg.norm(QB, axis=1)
        assert np.all(np.abs(hi - rhi) <= hi_b)
        assert np.all(np.abs(lo - rlo) <= lo_b)
        assert np.all(np.abs(s - rs) <= hi_b + lo_b)
    a = acc.cpu().numpy()
    assert a[0] == nrhs and abs(a[1] + 1j * a[2] - s.mean()) < 1e-12 * np.abs(s).max()


def test_solve_level_rejects_missing_solution():
    L = lib()
    dims = (2, 2, 2, 4)
    dl, ol = device_lattice(dims, 0.15, 0.5, 101, True, 0)
    t = _pin_roots(ol, 3, 3)
    lvl = L.DeviceLevel(L.OP_SOLVE, None, L.OP_POLY, L.DevicePoly(dev_c128(t)), None, False, None, None)
    samples = torch.empty((4, 6), dtype=torch.float64, device="cuda")
    acc = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = L.workspace(1 << 20)
    with pytest.raises(L.MpmcError):
        L.mlmc_level_estimate(dl, lvl, 4, 4, L.Noise(1, 1, 1, 0), samples, acc, ws)
