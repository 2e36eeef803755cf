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
