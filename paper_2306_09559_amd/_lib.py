"""ctypes binding of libmpmc.so (the C ABI declared in include/mpmc.h).

Argument marshalling only: torch tensors are passed as device pointers,
torch's current HIP stream as the stream; every operation runs in the
library's HIP kernels.  Importing this module raises if libmpmc.so has not
been built (there is no fallback path).

Field tensors use the library's field layout as a complex tensor of shape
(nrhs/rb, 12, V, rb): complex128 for MPMC_F64, complex64 for MPMC_F32.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_09559_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, EUNSUPPORTED, EWORKSPACE, EHIP, ESINGULAR, ENOTCONVERGED = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
DEFL_COEFF, DEFL_RECON, DEFL_PROJECT = 0, 1, 2
OP_NONE, OP_POLY, OP_DEFLATED_POLY, OP_SOLVE = 0, 1, 2, 3
OPT_PLANE_SWEEP, OPT_SWEEP_RANK, OPT_HOP_SLAB, OPT_LINK_BUF, OPT_SWEEP_CHUNKS = 1, 2, 3, 4, 5
# MPMC_OPT_PLANE_SWEEP values: never, whenever the lattice admits one, when the batch keeps half the CUs busy
SWEEP_OFF, SWEEP_ALWAYS, SWEEP_AUTO = 0, 1, 2

c_i32, c_u64, c_f64, c_vp, c_size = ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class mpmc_lattice(ctypes.Structure):
    _fields_ = [("dims", c_i32 * 4), ("antiperiodic_t", c_i32), ("prec", c_i32), ("kappa", c_f64),
                ("gauge", c_vp), ("link_rows", c_i32)]


class mpmc_shape(ctypes.Structure):
    _fields_ = [("nrhs", c_i32), ("rb", c_i32)]


class mpmc_noise(ctypes.Structure):
    _fields_ = [("seed", c_u64), ("lattice", c_u64), ("level", c_u64), ("first_sample", c_u64),
                ("sample_offset", c_vp), ("probe_colour", c_vp)]


class mpmc_poly(ctypes.Structure):
    _fields_ = [("n_in", c_i32), ("n_out", c_i32), ("inv_roots_in", c_vp), ("inv_roots_out", c_vp)]


class mpmc_defl(ctypes.Structure):
    _fields_ = [("k", c_i32), ("kpad", c_i32), ("V", c_vp), ("pair", c_vp), ("scale", c_vp), ("hinv", c_vp)]


class mpmc_level(ctypes.Structure):
    _fields_ = [("kind_hi", c_i32), ("kind_lo", c_i32), ("poly_hi", mpmc_poly), ("poly_lo", mpmc_poly),
                ("defl", ctypes.POINTER(mpmc_defl)), ("deflate_samples", c_i32), ("c", c_vp), ("solve_x", c_vp)]


class mpmc_batch_item(ctypes.Structure):
    _fields_ = [("lat", ctypes.POINTER(mpmc_lattice)), ("level", ctypes.POINTER(mpmc_level)), ("shape", mpmc_shape),
                ("noise", mpmc_noise), ("counter", c_vp), ("batches", c_i32), ("samples", c_vp), ("acc", c_vp),
                ("ws", c_vp), ("ws_bytes", c_size), ("branch", c_i32), ("plane_sweep", c_i32),
                ("sweep_rank", c_i32), ("sweep_chunks", c_i32), ("stop_state", c_vp), ("stop_first", c_i32),
                ("stop_every", c_i32)]


class mpmc_tune_choice(ctypes.Structure):
    _fields_ = [("rb", c_i32), ("plane_sweep", c_i32), ("sweep_rank", c_i32), ("sweep_chunks", c_i32)]


class mpmc_tune_result(ctypes.Structure):
    _fields_ = [("choice", mpmc_tune_choice), ("seconds", c_f64)]


P = ctypes.POINTER
_sig = {
    "mpmc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mpmc_build_info": (ctypes.c_char_p, []),
    "mpmc_set_option": (ctypes.c_int, [c_i32, c_i32]),
    "mpmc_counter_add": (ctypes.c_int, [c_vp, c_u64, c_vp]),
    "mpmc_probe_fill": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_vp, ctypes.c_int64, c_vp, c_vp]),
    "mpmc_sweep_plan": (ctypes.c_int, [P(mpmc_lattice), mpmc_shape, P(c_i32)]),
    "mpmc_gauge_unitarity": (ctypes.c_int, [P(c_i32), c_i32, c_vp, c_vp, c_vp]),
    "mpmc_pack_gauge": (ctypes.c_int, [P(c_i32), c_i32, c_vp, c_vp, c_vp]),
    "mpmc_pack_fields": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_vp, c_vp, c_vp]),
    "mpmc_unpack_fields": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_vp, c_vp, c_vp]),
    "mpmc_z4_fill": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, P(mpmc_noise), c_vp, c_vp]),
    "mpmc_field_axpby": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "mpmc_field_dot_workspace_size": (c_size, [P(c_i32), mpmc_shape]),
    "mpmc_field_dot": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]),
    "mpmc_field_copy_vector": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_vp, c_i32, mpmc_shape, c_vp, c_i32,
                                              c_vp]),
    "mpmc_field_copy_bytes": (ctypes.c_int, [c_vp, c_vp, c_size, c_vp]),
    "mpmc_field_axpby_mixed": (ctypes.c_int, [P(c_i32), mpmc_shape, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "mpmc_field_block_dot_workspace_size": (c_size, [P(c_i32), mpmc_shape, c_i32]),
    "mpmc_field_block_dot": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_i32, c_vp, c_vp, c_vp, c_vp, c_size,
                                            c_vp]),
    "mpmc_field_block_axpy": (ctypes.c_int, [P(c_i32), c_i32, mpmc_shape, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp]),
    "mpmc_wilson_apply": (ctypes.c_int, [P(mpmc_lattice), mpmc_shape, c_vp, c_vp, c_vp]),
    "mpmc_poly_workspace_size": (c_size, [P(mpmc_lattice), P(mpmc_poly), mpmc_shape]),
    "mpmc_poly_apply": (ctypes.c_int, [P(mpmc_lattice), P(mpmc_poly), mpmc_shape, c_vp, P(mpmc_noise), c_vp,
                                       c_vp, c_vp, c_size, c_vp]),
    "mpmc_deflate_workspace_size": (c_size, [P(mpmc_lattice), P(mpmc_defl), mpmc_shape]),
    "mpmc_deflate_project": (ctypes.c_int, [P(mpmc_lattice), P(mpmc_defl), c_i32, mpmc_shape, c_vp,
                                            P(mpmc_noise), c_vp, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]),
    "mpmc_level_workspace_size": (c_size, [P(mpmc_lattice), P(mpmc_level), mpmc_shape]),
    "mpmc_mlmc_level_estimate": (ctypes.c_int, [P(mpmc_lattice), P(mpmc_level), mpmc_shape, P(mpmc_noise), c_vp,
                                                c_vp, c_vp, c_size, c_vp]),
    "mpmc_handle_create": (ctypes.c_int, [P(c_vp)]),
    "mpmc_handle_destroy": (ctypes.c_int, [c_vp]),
    "mpmc_batch_build": (ctypes.c_int, [c_vp, P(mpmc_batch_item), c_i32]),
    "mpmc_batch_launch": (ctypes.c_int, [c_vp, c_vp]),
    "mpmc_autotune_workspace_size": (c_size, [P(mpmc_lattice), P(mpmc_level), c_i32]),
    "mpmc_autotune": (ctypes.c_int, [c_vp, P(mpmc_lattice), P(mpmc_level), c_i32, P(mpmc_noise), c_i32, c_f64, c_vp,
                                     c_size, P(mpmc_tune_choice), P(c_f64), P(c_i32), P(mpmc_tune_result), c_i32,
                                     P(c_i32), c_vp]),
    "mpmc_small_inverse": (ctypes.c_int, [c_i32, c_vp, c_f64, c_vp]),
    "mpmc_level_stop_check": (ctypes.c_int, [c_vp, c_i32, c_i32, c_i32, c_vp, c_vp]),
    "mpmc_noalloc_scratch_bytes": (c_size, []),
    "mpmc_mlmc_level_estimate_noalloc": (ctypes.c_int, [P(mpmc_lattice), P(mpmc_level), mpmc_shape, P(mpmc_noise),
                                                        c_vp, c_vp, c_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class MpmcError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: status {status} ({status_string(status)})")
        self.status = status


def status_string(status: int) -> str:
    return _lib.mpmc_status_string(int(status)).decode()


def build_info() -> str:
    return _lib.mpmc_build_info().decode()


# the library's process-wide options as last set through this binding (their
# defaults in the library until then)
_OPTIONS = {OPT_PLANE_SWEEP: SWEEP_AUTO, OPT_SWEEP_RANK: 0, OPT_HOP_SLAB: 1, OPT_LINK_BUF: 1, OPT_SWEEP_CHUNKS: 0}


def set_option(option: int, value: int):
    _check("mpmc_set_option", _lib.mpmc_set_option(int(option), int(value)))
    _OPTIONS[int(option)] = int(value)


def get_option(option: int) -> int:
    """The value of a process-wide option as last set through set_option."""
    return _OPTIONS[int(option)]


def _check(fn: str, st: int):
    if st != OK:
        raise MpmcError(fn, st)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dims(d: Sequence[int]):
    return (c_i32 * 4)(*[int(x) for x in d])


# ------------------------------------------------------------------ descriptors
def complex_dtype(prec: int):
    return torch.complex128 if prec == F64 else torch.complex64


@dataclass
class Noise:
    seed: int
    lattice: int
    level: int
    first_sample: int = 0
    sample_offset: Optional[torch.Tensor] = None   # device int64 (1,) counter added to first_sample
    probe_colour: Optional[torch.Tensor] = None    # device int32 (V,): probe vectors instead of Z4 noise

    def c(self) -> mpmc_noise:
        return mpmc_noise(self.seed, self.lattice, self.level, self.first_sample, _ptr(self.sample_offset),
                          _ptr(self.probe_colour))


@dataclass
class DeviceLattice:
    """Geometry, hopping parameter and the packed gauge field on the device."""
    dims: tuple
    kappa: float
    antiperiodic_t: bool
    prec: int
    gauge: torch.Tensor
    link_rows: int = 3          # 2: SU(3) links, row 2 rebuilt in the kernels

    @property
    def V(self) -> int:
        lx, ly, lz, lt = self.dims
        return lx * ly * lz * lt

    def c(self) -> mpmc_lattice:
        return mpmc_lattice(_dims(self.dims), int(self.antiperiodic_t), int(self.prec), float(self.kappa),
                            self.gauge.data_ptr(), int(self.link_rows))


@dataclass
class DevicePoly:
    """Inverse roots (complex128 device tensors) of p, or of p_in and p_out."""
    inv_in: torch.Tensor
    inv_out: Optional[torch.Tensor] = None

    def c(self) -> mpmc_poly:
        n_out = 0 if self.inv_out is None else int(self.inv_out.numel())
        return mpmc_poly(int(self.inv_in.numel()), n_out, self.inv_in.data_ptr(),
                         None if self.inv_out is None else self.inv_out.data_ptr())


@dataclass
class DeviceDefl:
    """Right eigenvectors V (field layout, nrhs = rb = kpad), pair, scale, H^{-1}."""
    k: int
    V: torch.Tensor
    pair: torch.Tensor            # int32 (k,)
    scale: torch.Tensor           # complex128 (k,)
    hinv: Optional[torch.Tensor]  # complex128 (k, k)

    @property
    def kpad(self) -> int:
        return int(self.V.shape[-1])

    def c(self) -> mpmc_defl:
        return mpmc_defl(int(self.k), self.kpad, self.V.data_ptr(), self.pair.data_ptr(), self.scale.data_ptr(),
                         None if self.hinv is None else self.hinv.data_ptr())


@dataclass
class DeviceLevel:
    kind_hi: int
    poly_hi: Optional[DevicePoly]       # None for OP_SOLVE
    kind_lo: int = OP_NONE
    poly_lo: Optional[DevicePoly] = None
    defl: Optional[DeviceDefl] = None
    deflate_samples: bool = False
    c: Optional[torch.Tensor] = None   # complex128 (k,)
    solve_x: Optional[torch.Tensor] = None   # field of the batch (OP_SOLVE)

    def cstruct(self):
        dref = self.defl.c() if self.defl is not None else None
        hi = self.poly_hi.c() if self.poly_hi is not None else mpmc_poly(0, 0, None, None)
        lo = self.poly_lo.c() if self.poly_lo is not None else mpmc_poly(0, 0, None, None)
        lv = mpmc_level(int(self.kind_hi), int(self.kind_lo), hi, lo,
                        ctypes.pointer(dref) if dref is not None else None, int(self.deflate_samples),
                        None if self.c is None else self.c.data_ptr(), _ptr(self.solve_x))
        return lv, dref


def field_shape(t: torch.Tensor) -> mpmc_shape:
    nb, twelve, _V, rb = t.shape
    assert twelve == 12
    return mpmc_shape(int(nb * rb), int(rb))


def empty_field(V: int, nrhs: int, rb: int, prec: int, device="cuda") -> torch.Tensor:
    assert nrhs % rb == 0
    return torch.empty((nrhs // rb, 12, V, rb), dtype=complex_dtype(prec), device=device)


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ entry points
def sweep_plan(lat: "DeviceLattice", nrhs: int, rb: int) -> dict:
    """The t-sweep a scalar-mode polynomial would use on this lattice and batch."""
    out = (c_i32 * 9)()
    L = lat.c()
    _check("mpmc_sweep_plan", _lib.mpmc_sweep_plan(ctypes.byref(L), mpmc_shape(nrhs, rb), out))
    v = list(out)
    return dict(ok=bool(v[0]), halo=bool(v[1]), block=tuple(v[2:5]), sites=v[5], halo_sites=v[6], blocks=v[7],
                chunks=v[8])


def probe_fill(dims, prec: int, colour: torch.Tensor, first_probe: int, field: torch.Tensor):
    """Probe vectors first_probe .. + N-1 (colour c = p // 12, unknown p % 12)."""
    assert colour.dtype == torch.int32 and colour.is_contiguous()
    _check("mpmc_probe_fill", _lib.mpmc_probe_fill(_dims(dims), prec, field_shape(field), _ptr(colour),
                                                   int(first_probe), _ptr(field), _stream()))


def counter_add(counter: torch.Tensor, increment: int):
    """counter[0] += increment on the device (int64 tensor; capturable)."""
    assert counter.dtype == torch.int64
    _check("mpmc_counter_add", _lib.mpmc_counter_add(_ptr(counter), int(increment), _stream()))


def gauge_unitarity(dims, prec: int, gauge: torch.Tensor) -> tuple:
    """(max |U U^H - I|, max |det U - 1|) over the packed links (synchronises)."""
    out = torch.empty(2, dtype=torch.float64, device=gauge.device)
    _check("mpmc_gauge_unitarity", _lib.mpmc_gauge_unitarity(_dims(dims), prec, _ptr(gauge), _ptr(out), _stream()))
    o = out.cpu().numpy()
    return float(o[0]), float(o[1])


def pack_gauge(dims, prec: int, canon: torch.Tensor, gauge: torch.Tensor):
    assert canon.dtype == torch.complex128 and canon.is_contiguous()
    _check("mpmc_pack_gauge", _lib.mpmc_pack_gauge(_dims(dims), prec, _ptr(canon), _ptr(gauge), _stream()))


def pack_fields(dims, prec: int, canon: torch.Tensor, field: torch.Tensor):
    assert canon.dtype == torch.complex128 and canon.is_contiguous()
    _check("mpmc_pack_fields", _lib.mpmc_pack_fields(_dims(dims), prec, field_shape(field), _ptr(canon),
                                                     _ptr(field), _stream()))


def unpack_fields(dims, prec: int, field: torch.Tensor, canon: torch.Tensor):
    _check("mpmc_unpack_fields", _lib.mpmc_unpack_fields(_dims(dims), prec, field_shape(field), _ptr(field),
                                                         _ptr(canon), _stream()))


def z4_fill(dims, prec: int, noise: Noise, field: torch.Tensor):
    nz = noise.c()
    _check("mpmc_z4_fill", _lib.mpmc_z4_fill(_dims(dims), prec, field_shape(field), ctypes.byref(nz), _ptr(field),
                                             _stream()))


def field_axpby(dims, prec: int, alpha: torch.Tensor, x: torch.Tensor, beta: Optional[torch.Tensor],
                y: torch.Tensor):
    """y_r = alpha_r x_r + beta_r y_r (alpha, beta: complex128 device (N,))."""
    _check("mpmc_field_axpby", _lib.mpmc_field_axpby(_dims(dims), prec, field_shape(x), _ptr(alpha), _ptr(x),
                                                     _ptr(beta), _ptr(y), _stream()))


def field_dot_workspace_size(dims, nrhs: int, rb: int) -> int:
    return int(_lib.mpmc_field_dot_workspace_size(_dims(dims), mpmc_shape(nrhs, rb)))


def field_dot(dims, prec: int, x: torch.Tensor, y: torch.Tensor, out: torch.Tensor, ws: torch.Tensor):
    """out_r = x_r^H y_r in FP64 (out: complex128 device (N,))."""
    _check("mpmc_field_dot", _lib.mpmc_field_dot(_dims(dims), prec, field_shape(x), _ptr(x), _ptr(y), _ptr(out),
                                                 _ptr(ws), ws.numel(), _stream()))


def field_copy_vector(dims, prec: int, src: torch.Tensor, src_index: int, dst: torch.Tensor, dst_index: int):
    _check("mpmc_field_copy_vector", _lib.mpmc_field_copy_vector(
        _dims(dims), prec, field_shape(src), _ptr(src), int(src_index), field_shape(dst), _ptr(dst),
        int(dst_index), _stream()))


def field_copy_bytes(src: torch.Tensor, dst: torch.Tensor):
    """dst = src for two contiguous device tensors of the same byte size."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("field_copy_bytes needs contiguous tensors of equal byte size")
    _check("mpmc_field_copy_bytes", _lib.mpmc_field_copy_bytes(_ptr(src), _ptr(dst), nb, _stream()))


def field_axpby_mixed(dims, alpha: torch.Tensor, x: torch.Tensor, beta: Optional[torch.Tensor], y: torch.Tensor):
    """y_r = alpha_r x_r + beta_r y_r with x, y of different precisions."""
    xp, yp = _prec_of(x), _prec_of(y)
    _check("mpmc_field_axpby_mixed", _lib.mpmc_field_axpby_mixed(
        _dims(dims), field_shape(x), xp, _ptr(alpha), _ptr(x), yp, _ptr(beta), _ptr(y), _stream()))


def field_block_dot_workspace_size(dims, nrhs: int, rb: int, k: int) -> int:
    return int(_lib.mpmc_field_block_dot_workspace_size(_dims(dims), mpmc_shape(nrhs, rb), int(k)))


def field_block_dot(dims, prec: int, basis: torch.Tensor, k: int, x: torch.Tensor, out: torch.Tensor,
                    ws: torch.Tensor):
    """out[i, r] = (basis_i)_r^H x_r for i < k (basis: (K, nb, 12, V, rb); out complex128 (k, N))."""
    assert basis.is_contiguous() and basis.shape[0] >= k and basis.shape[1:] == x.shape
    _check("mpmc_field_block_dot", _lib.mpmc_field_block_dot(
        _dims(dims), prec, field_shape(x), int(k), _ptr(basis), _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
        _stream()))


def field_block_axpy(dims, prec: int, basis: torch.Tensor, k: int, coeff: torch.Tensor, y: torch.Tensor,
                     accumulate: bool = True):
    """y_r = [y_r +] sum_{i<k} coeff[i, r] (basis_i)_r (coeff complex128 (k, N))."""
    assert basis.is_contiguous() and basis.shape[0] >= k and basis.shape[1:] == y.shape
    assert coeff.is_contiguous() and coeff.shape[0] >= k
    _check("mpmc_field_block_axpy", _lib.mpmc_field_block_axpy(
        _dims(dims), prec, field_shape(y), int(k), _ptr(basis), _ptr(coeff), int(bool(accumulate)), _ptr(y),
        _stream()))


def _prec_of(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return F64
    if t.dtype == torch.complex64:
        return F32
    raise TypeError(f"field dtype {t.dtype}")


def wilson_apply(lat: DeviceLattice, x: torch.Tensor, y: torch.Tensor):
    L = lat.c()
    _check("mpmc_wilson_apply", _lib.mpmc_wilson_apply(ctypes.byref(L), field_shape(x), _ptr(x), _ptr(y),
                                                       _stream()))


def poly_workspace_size(lat: DeviceLattice, poly: DevicePoly, nrhs: int, rb: int) -> int:
    L, Pl = lat.c(), poly.c()
    return int(_lib.mpmc_poly_workspace_size(ctypes.byref(L), ctypes.byref(Pl), mpmc_shape(nrhs, rb)))


def poly_apply(lat: DeviceLattice, poly: DevicePoly, nrhs: int, rb: int, x: Optional[torch.Tensor],
               noise: Optional[Noise], y: Optional[torch.Tensor], bhy: Optional[torch.Tensor],
               ws: torch.Tensor):
    L, Pl = lat.c(), poly.c()
    nz = noise.c() if noise is not None else None
    _check("mpmc_poly_apply", _lib.mpmc_poly_apply(
        ctypes.byref(L), ctypes.byref(Pl), mpmc_shape(nrhs, rb), _ptr(x), ctypes.byref(nz) if nz else None,
        _ptr(y), _ptr(bhy), _ptr(ws), ws.numel(), _stream()))


def deflate_workspace_size(lat: DeviceLattice, defl: DeviceDefl, nrhs: int, rb: int) -> int:
    L, D = lat.c(), defl.c()
    return int(_lib.mpmc_deflate_workspace_size(ctypes.byref(L), ctypes.byref(D), mpmc_shape(nrhs, rb)))


def deflate_project(lat: DeviceLattice, defl: DeviceDefl, mode: int, nrhs: int, rb: int,
                    b: Optional[torch.Tensor], noise: Optional[Noise], zeta: Optional[torch.Tensor],
                    omega: Optional[torch.Tensor], d: Optional[torch.Tensor], X: Optional[torch.Tensor],
                    ws: torch.Tensor):
    L, D = lat.c(), defl.c()
    nz = noise.c() if noise is not None else None
    _check("mpmc_deflate_project", _lib.mpmc_deflate_project(
        ctypes.byref(L), ctypes.byref(D), int(mode), mpmc_shape(nrhs, rb), _ptr(b),
        ctypes.byref(nz) if nz else None, _ptr(zeta), _ptr(omega), _ptr(d), _ptr(X), _ptr(ws), ws.numel(),
        _stream()))


def noalloc_scratch_bytes() -> int:
    return int(_lib.mpmc_noalloc_scratch_bytes())


def mlmc_level_estimate_noalloc(lat: DeviceLattice, level: DeviceLevel, nrhs: int, rb: int, noise: Noise,
                                samples: torch.Tensor, acc: torch.Tensor):
    """mpmc_mlmc_level_estimate with the library's static device scratch as
    the workspace (no allocation; calls on one GPU must not overlap)."""
    L = lat.c()
    lv, _keep = level.cstruct()
    nz = noise.c()
    _check("mpmc_mlmc_level_estimate_noalloc", _lib.mpmc_mlmc_level_estimate_noalloc(
        ctypes.byref(L), ctypes.byref(lv), mpmc_shape(nrhs, rb), ctypes.byref(nz), _ptr(samples), _ptr(acc),
        _stream()))


def level_workspace_size(lat: DeviceLattice, level: DeviceLevel, nrhs: int, rb: int) -> int:
    L = lat.c()
    lv, _keep = level.cstruct()
    return int(_lib.mpmc_level_workspace_size(ctypes.byref(L), ctypes.byref(lv), mpmc_shape(nrhs, rb)))


def mlmc_level_estimate(lat: DeviceLattice, level: DeviceLevel, nrhs: int, rb: int, noise: Noise,
                        samples: torch.Tensor, acc: torch.Tensor, ws: torch.Tensor):
    L = lat.c()
    lv, _keep = level.cstruct()
    nz = noise.c()
    _check("mpmc_mlmc_level_estimate", _lib.mpmc_mlmc_level_estimate(
        ctypes.byref(L), ctypes.byref(lv), mpmc_shape(nrhs, rb), ctypes.byref(nz), _ptr(samples), _ptr(acc),
        _ptr(ws), ws.numel(), _stream()))


# ------------------------------------------------------------------ batched steps and the autotuner
class Handle:
    """Owner of a recorded step (HIP graph), its streams and the tuner's cache
    (mpmc_handle_create / mpmc_handle_destroy)."""

    def __init__(self):
        h = c_vp()
        _check("mpmc_handle_create", _lib.mpmc_handle_create(ctypes.byref(h)))
        self._h = h
        self._keep = []          # C descriptors referenced by the recorded step

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib.mpmc_handle_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:       # noqa: BLE001 - interpreter shutdown
            pass


@dataclass
class BatchItem:
    """One level of one lattice in a batched step (mpmc_batch_item)."""
    lat: DeviceLattice
    level: DeviceLevel
    nrhs: int
    rb: int
    noise: Noise                  # seed, lattice, level id, first sample (its sample_offset is not used)
    counter: torch.Tensor         # device int64 (1,)
    batches: int
    samples: torch.Tensor
    acc: torch.Tensor
    ws: torch.Tensor
    branch: int = 0
    plane_sweep: int = SWEEP_AUTO
    sweep_rank: int = 0
    sweep_chunks: int = 0                        # t-chunks of the sweep (0: the plan's choice)
    stop_state: Optional[torch.Tensor] = None    # device float64 (16,): mpmc_level_stop_check after each batch
    stop_first: int = 2
    stop_every: int = 1


def batch_build(h: Handle, items: Sequence[BatchItem]):
    """Record the step (mpmc_batch_build); nothing runs."""
    keep = []
    arr = (mpmc_batch_item * len(items))()
    for i, it in enumerate(items):
        L = it.lat.c()
        lv, dref = it.level.cstruct()
        # the C descriptors and every device buffer the recorded graph uses stay
        # alive with the handle (a level reshaped later gets a new workspace;
        # the graph keeps writing its own)
        keep += [L, lv, dref, it.lat, it.level, it.counter, it.samples, it.acc, it.ws, it.stop_state]
        assert it.counter.dtype == torch.int64 and it.counter.is_cuda
        arr[i] = mpmc_batch_item(ctypes.pointer(L), ctypes.pointer(lv), mpmc_shape(it.nrhs, it.rb), it.noise.c(),
                                 it.counter.data_ptr(), int(it.batches), it.samples.data_ptr(), it.acc.data_ptr(),
                                 it.ws.data_ptr(), it.ws.numel(), int(it.branch), int(it.plane_sweep),
                                 int(it.sweep_rank), int(it.sweep_chunks),
                                 None if it.stop_state is None else it.stop_state.data_ptr(),
                                 int(it.stop_first), int(it.stop_every))
    _check("mpmc_batch_build", _lib.mpmc_batch_build(h.ptr, arr, len(items)))
    h._keep = keep


def batch_launch(h: Handle):
    _check("mpmc_batch_launch", _lib.mpmc_batch_launch(h.ptr, _stream()))


def autotune_workspace_size(lat: DeviceLattice, level: DeviceLevel, nrhs: int) -> int:
    L = lat.c()
    lv, _keep = level.cstruct()
    return int(_lib.mpmc_autotune_workspace_size(ctypes.byref(L), ctypes.byref(lv), int(nrhs)))


def autotune_level(h: Handle, lat: DeviceLattice, level: DeviceLevel, nrhs: int, noise: Noise, current: tuple,
                   reps: int = 3, keep_within: float = 0.03, ws: Optional[torch.Tensor] = None):
    """mpmc_autotune for one level.  current = (rb, plane_sweep, sweep_rank, sweep_chunks).
    Returns (choice tuple, seconds per call, cached flag, [(choice, seconds)...])."""
    L = lat.c()
    lv, _keep = level.cstruct()
    nz = noise.c()
    if ws is None:
        ws = workspace(autotune_workspace_size(lat, level, nrhs))
    best = mpmc_tune_choice(*[int(x) for x in current])
    secs, cached, nres = c_f64(), c_i32(), c_i32()
    res = (mpmc_tune_result * 64)()
    _check("mpmc_autotune", _lib.mpmc_autotune(
        h.ptr, ctypes.byref(L), ctypes.byref(lv), int(nrhs), ctypes.byref(nz), int(reps), float(keep_within),
        _ptr(ws), ws.numel(), ctypes.byref(best), ctypes.byref(secs), ctypes.byref(cached), res, 64,
        ctypes.byref(nres), _stream()))
    table = [((r.choice.rb, r.choice.plane_sweep, r.choice.sweep_rank, r.choice.sweep_chunks), r.seconds)
             for r in res[: nres.value]]
    return (best.rb, best.plane_sweep, best.sweep_rank, best.sweep_chunks), secs.value, bool(cached.value), table


def level_stop_check(samples: torch.Tensor, nrhs: int, first: int, every: int, state: torch.Tensor):
    """mpmc_level_stop_check: the stopping rule on the device (state float64 (16,))."""
    assert state.dtype == torch.float64 and state.numel() >= 16
    _check("mpmc_level_stop_check", _lib.mpmc_level_stop_check(_ptr(samples), int(nrhs), int(first), int(every),
                                                               _ptr(state), _stream()))


def small_inverse(a, tiny: float = 1e-14):
    """Inverse of a small complex FP64 matrix on the host (mpmc_small_inverse);
    raises MpmcError(ESINGULAR) for a zero pivot."""
    import numpy as np
    m = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    k = m.shape[0]
    assert m.shape == (k, k)
    out = np.empty_like(m)
    _check("mpmc_small_inverse", _lib.mpmc_small_inverse(k, m.ctypes.data_as(c_vp), float(tiny),
                                                         out.ctypes.data_as(c_vp)))
    return out
