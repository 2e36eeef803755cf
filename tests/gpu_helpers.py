"""Shared set-up for the GPU parity tests: synthetic inputs from `synth`,
expected values from `oracle`, device calls through the C ABI binding."""
import numpy as np
import torch

import oracle
import synth


def lib():
    from paper_2306_09559_amd import _lib
    return _lib


def device_lattice(dims, kappa, eps, seed, antiperiodic=True, prec=0, link_rows=3):
    L = lib()
    U = synth.unit_links(dims) if eps == 0 else synth.gauge_links(dims, eps, seed)
    canon = torch.from_numpy(U).cuda()
    V = int(np.prod(dims))
    gauge = torch.empty(36 * V, dtype=L.complex_dtype(prec), device="cuda")
    L.pack_gauge(dims, prec, canon, gauge)
    dl = L.DeviceLattice(tuple(dims), kappa, antiperiodic, prec, gauge, link_rows)
    ol = oracle.Lattice(dims, kappa, U, antiperiodic)
    return dl, ol


def pack(dims, X: np.ndarray, rb: int, prec: int) -> torch.Tensor:
    L = lib()
    V = int(np.prod(dims))
    N = X.shape[0]
    canon = torch.from_numpy(np.ascontiguousarray(X.reshape(N, V, 4, 3).astype(np.complex128))).cuda()
    f = L.empty_field(V, N, rb, prec)
    L.pack_fields(dims, prec, canon, f)
    return f


def unpack(dims, f: torch.Tensor, prec: int) -> np.ndarray:
    L = lib()
    V = int(np.prod(dims))
    N = f.shape[0] * f.shape[3]
    canon = torch.empty((N, V, 4, 3), dtype=torch.complex128, device="cuda")
    L.unpack_fields(dims, prec, f, canon)
    torch.cuda.synchronize()
    return canon.cpu().numpy().reshape(N, 12 * V)


def dev_c128(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).cuda()


def rel(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def device_defl(dims, Z, pair, U, H, prec=0, kpad=16):
    """Oracle triplets (rows of Z, left vectors U, H = U^H A V) as a DeviceDefl."""
    L = lib()
    k, n = Z.shape
    Zp = np.zeros((kpad, n), dtype=np.complex128)
    Zp[:k] = Z
    Vf = pack(dims, Zp, kpad, prec)
    # scale_i: u_i = scale_i * g5 z_pair(i)
    g5 = np.array([1] * 6 + [-1] * 6, dtype=float)
    V = n // 12
    g5z = (Z.reshape(k, V, 12) * g5).reshape(k, n)
    scale = np.array([np.vdot(g5z[pair[i]], U[i]) / np.vdot(g5z[pair[i]], g5z[pair[i]]) for i in range(k)])
    assert np.allclose(U, scale[:, None] * g5z[pair])
    return L.DeviceDefl(k, Vf, torch.from_numpy(pair.astype(np.int32)).cuda(), dev_c128(scale),
                        dev_c128(np.linalg.inv(H)) if H is not None else None)


def newton_amplification(apply, t, B) -> float:
    """kappa_N = max_j ||w_j|| / ||b|| over the Newton recurrence
    w_{j+1} = w_j - t_j A w_j (rows b of B): the growth that multiplies the
    rounding errors of a polynomial application.  At least 1."""
    out = 1.0
    for b in np.atleast_2d(B):
        w = b.copy()
        nb = np.linalg.norm(b)
        for tj in t[:-1]:
            w = w - tj * apply(w)
            out = max(out, float(np.linalg.norm(w) / nb))
    return out


def composite_amplification(apply, t_in, t_out, B) -> float:
    """kappa_N of the double polynomial p_in(A) p_out(A p_in(A)) b as the
    library evaluates it: the outer Newton recurrence over B = I - pi_in(A),
    each application a product chain prod_i (1 - t_i A) w, then p_in(A) on the
    outer sum.  Max over every intermediate vector of ||.|| / ||b||."""
    out = 1.0
    for b in np.atleast_2d(B):
        nb = np.linalg.norm(b)
        w, y = b.copy(), np.zeros_like(b)
        for j, ph in enumerate(t_out):
            y = y + ph * w
            out = max(out, float(np.linalg.norm(y) / nb))
            if j + 1 == len(t_out):
                break
            v = w.copy()
            for ti in t_in:
                v = v - ti * apply(v)
                out = max(out, float(np.linalg.norm(v) / nb))
            w = w - ph * (w - v)
            out = max(out, float(np.linalg.norm(w) / nb))
        out = max(out, newton_amplification(apply, t_in, y[None, :]) * float(np.linalg.norm(y) / nb))
    return out


_SETUPS = {}


def oracle_set_up(cfg, degrees, pin_degree=None, arnoldi_m=90, nev=40, imaglim=2e-4, evectol=1e-3):
    """The oracle's own set-up of a workload (Sec. 5 setup step 2) from the
    workload's seeded links and start vector: GMRES roots of the given degrees
    and, with pin_degree, the PP(pin_degree + 1)-Arnoldi Ritz pairs nearest
    the origin put through the selection of Sec. 4, of which the first
    cfg.k_defl accepted are kept (a conjugate pair whole).  Cached for the
    test process.  Returns a namespace (ol, start, ps, tri)."""
    import types
    from oracle import krylov as okr
    key = (cfg.name, tuple(sorted(degrees)), pin_degree, arnoldi_m, nev, imaglim, evectol)
    if key in _SETUPS:
        return _SETUPS[key]
    ol = oracle.Lattice(cfg.dims, cfg.kappa, synth.config_links(cfg), cfg.antiperiodic_t)
    start = synth.gaussian_start(ol.n, cfg.seed_start)
    ps = okr.gmres_polys(ol.apply, start, sorted(set(degrees) | ({pin_degree} - {None})))
    tri = None
    if pin_degree is not None:
        opB = okr.pp_operator(ol.apply, ps.inv_roots[pin_degree], lambda t, v: ol.poly_apply(t, v)[0])
        lam, Z, AZ, _ = okr.pp_arnoldi_ritz(opB, ol.apply, start, arnoldi_m, nev)
        tri = okr.select_eigs(lam, Z, AZ, ol.gamma5, lambda v: ol.gamma5(ol.apply(ol.gamma5(v))), imaglim, evectol)
        k = min(cfg.k_defl, len(tri.lam))
        if k < len(tri.lam) and tri.pair[k - 1] == k:      # the last kept value's partner would be cut off
            k -= 1
        assert k > 0 and np.all(tri.pair[:k] < k)
        tri = okr.Triplets(tri.lam[:k], tri.Z[:k], tri.pair[:k], tri.U[:k], tri.res_right[:k], tri.res_left[:k])
    su = types.SimpleNamespace(ol=ol, start=start, ps=ps, tri=tri)
    _SETUPS[key] = su
    return su


def build_from_oracle_set_up(cfg, su, path, prec=0, rb=16):
    """The product's run of a workload whose set-up is the oracle's: the
    roots and deflation triplets of `su` written in the product's checkpoint
    format (fresh Monte Carlo state) and resumed with driver.build, so that
    the GPU levels use no root or eigenvector the HIP path produced."""
    import json
    from paper_2306_09559_amd import driver
    from oracle import krylov as okr
    ps, tri, ol = su.ps, su.tri, su.ol
    beta = ps.arn.beta
    degs = sorted(ps.inv_roots)
    d = {"meta": np.array(json.dumps({"version": driver.CHECKPOINT_VERSION, "config": driver._identity(cfg)})),
         "root_degrees": np.array(degs, dtype=np.int64),
         "root_residuals": np.array([okr.gmres_ls(ps.arn.Hbar, beta, min(k + 1, ps.arn.m))[1] / beta for k in degs]),
         "composite_keys": np.zeros((0, 2), dtype=np.int64), "composite_residuals": np.zeros(0)}
    for k in degs:
        d[f"root_{k}"] = np.asarray(ps.inv_roots[k], dtype=np.complex128)
    if tri is not None:
        k = len(tri.lam)
        kpad = 16
        while kpad < k:
            kpad *= 2
        Zp = np.zeros((kpad, ol.n), dtype=np.complex128)
        Zp[:k] = tri.Z
        # u_i = scale_i g5 z_pair(i) with u_i^H z_i = 1
        g5z = np.stack([ol.gamma5(z) for z in tri.Z])
        scale = 1.0 / np.conj(np.einsum("ij,ij->i", g5z[tri.pair].conj(), tri.Z))
        assert np.allclose(tri.U, scale[:, None] * g5z[tri.pair])
        H = tri.U.conj() @ np.stack([ol.apply(z) for z in tri.Z]).T
        d.update(defl_V=pack(cfg.dims, Zp, kpad, 0).cpu().numpy(), defl_pair=tri.pair.astype(np.int32),
                 defl_scale=scale, defl_hinv=np.linalg.inv(H), defl_lam=np.asarray(tri.lam),
                 defl_res=np.stack([tri.res_right, tri.res_left]),
                 defl_counts=np.array([k, len(tri.lam), 0], dtype=np.int64), defl_arnoldi_residual=np.array(0.0))
    d["acc"] = np.zeros((len(cfg.levels), 8))
    d["drawn"] = np.zeros(len(cfg.levels), dtype=np.int64)
    np.savez(path, **d)
    return driver.build(cfg, prec=prec, rb=rb, resume=str(path))
