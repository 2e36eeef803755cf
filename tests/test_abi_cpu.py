"""The C ABI library loads, exports every entry point declared in
include/mpmc.h, and rejects invalid arguments on the host with status codes
before touching a device.  No GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpmc.h")


@pytest.fixture(scope="module")
def L():
    from paper_2306_09559_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpmc_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 13
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_status_strings(L):
    texts = [L.status_string(st) for st in (L.OK, L.EINVAL, L.EUNSUPPORTED, L.EWORKSPACE, L.EHIP, L.ESINGULAR,
                                            L.ENOTCONVERGED)]
    assert len(set(texts)) == len(texts) and "unknown" not in " ".join(texts)
    assert "gfx950" in L.build_info()


def _lat(L, dims=(4, 4, 4, 4), prec=0, gauge=1):
    return L.mpmc_lattice((ctypes.c_int32 * 4)(*dims), 1, prec, 0.15, gauge)


def test_validation_without_device(L):
    lib = L._lib
    sh = L.mpmc_shape(8, 4)
    x, y = ctypes.c_void_p(16), ctypes.c_void_p(32)
    assert lib.mpmc_wilson_apply(None, sh, x, y, None) == L.EINVAL
    lat = _lat(L)
    assert lib.mpmc_wilson_apply(ctypes.byref(lat), L.mpmc_shape(8, 3), x, y, None) == L.EINVAL   # rb not 2^k
    assert lib.mpmc_wilson_apply(ctypes.byref(lat), L.mpmc_shape(6, 4), x, y, None) == L.EINVAL   # rb !| N
    assert lib.mpmc_wilson_apply(ctypes.byref(lat), L.mpmc_shape(8, 512), x, y, None) == L.EINVAL
    assert lib.mpmc_wilson_apply(ctypes.byref(lat), sh, x, x, None) == L.EINVAL                   # aliasing
    bad = _lat(L, prec=7)
    assert lib.mpmc_wilson_apply(ctypes.byref(bad), sh, x, y, None) == L.EUNSUPPORTED
    zero = _lat(L, dims=(4, 0, 4, 4))
    assert lib.mpmc_wilson_apply(ctypes.byref(zero), sh, x, y, None) == L.EINVAL
    nog = _lat(L, gauge=None)
    assert lib.mpmc_wilson_apply(ctypes.byref(nog), sh, x, y, None) == L.EINVAL
    # an empty or negative batch (the header requires N >= 1) is an argument error, not a no-op launch
    for n in (0, -4):
        assert lib.mpmc_wilson_apply(ctypes.byref(lat), L.mpmc_shape(n, 4), x, y, None) == L.EINVAL
        assert lib.mpmc_z4_fill((ctypes.c_int32 * 4)(4, 4, 4, 4), 0, L.mpmc_shape(n, 1),
                                ctypes.byref(L.mpmc_noise(1, 2, 3, 0)), x, None) == L.EINVAL
    # plain copy: zero bytes is a no-op; ragged sizes, misaligned or overlapping ranges are rejected
    assert lib.mpmc_field_copy_bytes(None, None, 0, None) == L.OK
    assert lib.mpmc_field_copy_bytes(ctypes.c_void_p(4096), ctypes.c_void_p(1 << 20), 24, None) == L.EINVAL
    assert lib.mpmc_field_copy_bytes(ctypes.c_void_p(4104), ctypes.c_void_p(1 << 20), 32, None) == L.EINVAL
    assert lib.mpmc_field_copy_bytes(ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 64), 128, None) == L.EINVAL
    assert lib.mpmc_field_copy_bytes(None, ctypes.c_void_p(4096), 32, None) == L.EINVAL
    # polynomial: no roots, no outputs, workspace too small
    roots = ctypes.c_void_p(64)
    p0 = L.mpmc_poly(0, 0, roots, None)
    assert lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(p0), sh, x, None, y, None, None, 0, None) == L.EINVAL
    p = L.mpmc_poly(5, 0, roots, None)
    assert lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(p), sh, x, None, None, None, None, 0, None) == L.EINVAL
    assert lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(p), sh, None, None, y, None, None, 0, None) == L.EINVAL
    need = lib.mpmc_poly_workspace_size(ctypes.byref(lat), ctypes.byref(p), sh)
    assert need > 0
    assert lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(p), sh, x, None, y, None,
                               ctypes.c_void_p(128), need - 1, None) == L.EWORKSPACE
    pc = L.mpmc_poly(5, 3, roots, None)   # composite without outer roots
    assert lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(pc), sh, x, None, y, None, None, 0, None) == L.EINVAL
    # deflation: kpad not a multiple of 16, unknown mode, PROJECT without H^{-1}
    d = L.mpmc_defl(4, 8, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), None)
    z = ctypes.c_void_p(256)
    assert lib.mpmc_deflate_project(ctypes.byref(lat), ctypes.byref(d), 0, sh, x, None, z, z, None, None, None, 0,
                                    None) == L.EINVAL
    d16 = L.mpmc_defl(4, 16, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), None)
    assert lib.mpmc_deflate_project(ctypes.byref(lat), ctypes.byref(d16), 9, sh, x, None, z, z, None, None, None, 0,
                                    None) == L.EUNSUPPORTED
    assert lib.mpmc_deflate_project(ctypes.byref(lat), ctypes.byref(d16), 2, sh, x, None, z, z, z, y, None, 0,
                                    None) == L.EINVAL
    # level: NONE as the high operator, deflated samples without c
    lv = L.mpmc_level(0, 0, p, p, None, 0, None)
    nz = L.mpmc_noise(1, 2, 3, 0)
    assert lib.mpmc_mlmc_level_estimate(ctypes.byref(lat), ctypes.byref(lv), sh, ctypes.byref(nz), z, z, None, 0,
                                        None) == L.EUNSUPPORTED
    lv2 = L.mpmc_level(1, 0, p, p, ctypes.pointer(d16), 1, None)
    assert lib.mpmc_mlmc_level_estimate(ctypes.byref(lat), ctypes.byref(lv2), sh, ctypes.byref(nz), z, z, None, 0,
                                        None) == L.EINVAL
    # no samples
    lv1 = L.mpmc_level(1, 0, p, p, None, 0, None)
    assert lib.mpmc_mlmc_level_estimate(ctypes.byref(lat), ctypes.byref(lv1), L.mpmc_shape(0, 1), ctypes.byref(nz),
                                        z, z, None, 0, None) == L.EINVAL
    assert lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(p), L.mpmc_shape(0, 1), x, None, y, None, None, 0,
                               None) == L.EINVAL


def test_workspace_sizes_scale(L):
    lib = L._lib
    lat = _lat(L)
    roots = ctypes.c_void_p(64)
    single = L.mpmc_poly(21, 0, roots, None)
    comp = L.mpmc_poly(20, 15, roots, roots)
    sh = L.mpmc_shape(64, 16)
    a = lib.mpmc_poly_workspace_size(ctypes.byref(lat), ctypes.byref(single), sh)
    b = lib.mpmc_poly_workspace_size(ctypes.byref(lat), ctypes.byref(comp), sh)
    field = 256 * 12 * 64 * 16
    assert a >= 2 * field and b >= 5 * field
    lat32 = _lat(L, prec=1)
    assert lib.mpmc_poly_workspace_size(ctypes.byref(lat32), ctypes.byref(single), sh) < a


def test_workspace_too_small_is_rejected_on_the_host(L):
    """A workspace one byte short of the *_workspace_size result returns
    MPMC_EWORKSPACE before anything is enqueued (fake device pointers: the
    host never dereferences them)."""
    lib = L._lib
    lat = _lat(L)
    roots = ctypes.c_void_p(64)
    poly = L.mpmc_poly(4, 0, roots, None)
    sh = L.mpmc_shape(8, 4)
    need = lib.mpmc_poly_workspace_size(ctypes.byref(lat), ctypes.byref(poly), sh)
    assert need > 0
    x, y, ws = ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(4096)
    st = lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(poly), sh, x, None, y, None, ws, need - 1, None)
    assert st == L.EWORKSPACE
    # probe noise outside the scalar t-sweep is refused on the host too
    col = ctypes.c_void_p(8192)
    nz = L.mpmc_noise(0, 0, 0, 0, None, col)
    st = lib.mpmc_poly_apply(ctypes.byref(lat), ctypes.byref(poly), sh, None, ctypes.byref(nz), y, None, ws, need,
                             None)
    assert st == L.EUNSUPPORTED


def test_small_inverse(L):
    """mpmc_small_inverse (host): the inverse of a random complex matrix, a
    pivot that needs row exchanges, and ESINGULAR for a rank-deficient one."""
    import numpy as np
    rng = np.random.default_rng(4)
    a = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    assert np.max(np.abs(L.small_inverse(a) @ a - np.eye(20))) < 1e-12
    p = np.array([[0, 1j], [2.0, 0]])
    assert np.allclose(L.small_inverse(p) @ p, np.eye(2), atol=1e-15)
    s = a.copy()
    s[3] = 2.0 * s[7]
    with pytest.raises(L.MpmcError) as e:
        L.small_inverse(s)
    assert e.value.status == L.ESINGULAR


def test_batch_and_tuner_reject_on_host(L):
    """mpmc_batch_build, mpmc_batch_launch and mpmc_autotune validate their
    arguments before any device work."""
    h = L.Handle()
    assert L._lib.mpmc_batch_launch(h.ptr, None) == L.EINVAL
    assert L._lib.mpmc_batch_build(h.ptr, None, 1) == L.EINVAL
    items = (L.mpmc_batch_item * 1)()
    assert L._lib.mpmc_batch_build(h.ptr, items, 1) == L.EINVAL          # no lattice
    assert L._lib.mpmc_batch_build(None, items, 1) == L.EINVAL
    assert L._lib.mpmc_autotune(None, None, None, 1, None, 1, 0.0, None, 0, None, None, None, None, 0, None,
                                None) == L.EINVAL
    # a current shape outside the options' ranges (t-chunks above 1024, a kernel selection above 2)
    fake = ctypes.c_void_p(256)                      # never dereferenced: the argument checks come first
    lat = L.mpmc_lattice((ctypes.c_int32 * 4)(8, 8, 8, 8), 0, L.F64, 0.13, fake, 3)
    lv = L.mpmc_level(L.OP_POLY, L.OP_NONE, L.mpmc_poly(3, 0, fake, None), L.mpmc_poly(0, 0, None, None), None,
                      0, None, None)
    nz = L.mpmc_noise(1, 1, 1, 0, None, None)
    for bad in (L.mpmc_tune_choice(16, 2, 0, 1025), L.mpmc_tune_choice(16, 3, 0, 0), L.mpmc_tune_choice(16, 1, 64, 0)):
        assert L._lib.mpmc_autotune(h.ptr, ctypes.byref(lat), ctypes.byref(lv), 64, ctypes.byref(nz), 1, 0.0,
                                    fake, 1 << 30, ctypes.byref(bad), None, None, None, 0, None, None) == L.EINVAL
    # a batch item with t-chunks out of range
    item = L.mpmc_batch_item()
    item.lat, item.level, item.counter, item.batches = ctypes.pointer(lat), ctypes.pointer(lv), fake, 1
    item.shape = L.mpmc_shape(64, 16)
    item.plane_sweep, item.sweep_chunks = 2, 2000
    assert L._lib.mpmc_batch_build(h.ptr, ctypes.byref(item), 1) == L.EINVAL
    item.sweep_chunks = 0                            # in range: the next check is the (missing) workspace
    assert L._lib.mpmc_batch_build(h.ptr, ctypes.byref(item), 1) == L.EWORKSPACE
    h.close()


def test_noalloc_rejects_a_level_beyond_its_scratch(L):
    """The no-allocation level entry point refuses, on the host, a level whose
    workspace exceeds its static scratch (8^4 x 256 vectors in FP64)."""
    c_i32 = ctypes.c_int32
    fake = ctypes.c_void_p(256)                      # never dereferenced: the size check comes first
    lat = L.mpmc_lattice((c_i32 * 4)(8, 8, 8, 8), 0, L.F64, 0.13, fake, 3)
    poly = L.mpmc_poly(3, 0, fake, None)
    lv = L.mpmc_level(L.OP_POLY, L.OP_NONE, poly, L.mpmc_poly(0, 0, None, None), None, 0, None, None)
    shape = L.mpmc_shape(256, 16)
    need = L._lib.mpmc_level_workspace_size(ctypes.byref(lat), ctypes.byref(lv), shape)
    assert need > L.noalloc_scratch_bytes() == 64 << 20
    nz = L.mpmc_noise(1, 1, 1, 0, None, None)
    st = L._lib.mpmc_mlmc_level_estimate_noalloc(ctypes.byref(lat), ctypes.byref(lv), shape, ctypes.byref(nz),
                                                 fake, fake, None)
    assert st == L.EWORKSPACE


def test_set_option_checks_its_arguments(L):
    """Every kernel-selection option takes its documented values, rejects
    others with EINVAL, and an unknown option is EUNSUPPORTED; the defaults
    are restored afterwards (the options are process-wide)."""
    lib = L._lib
    ranges = {L.OPT_PLANE_SWEEP: (0, 2, 2), L.OPT_SWEEP_RANK: (0, 63, 0), L.OPT_HOP_SLAB: (0, 1, 1),
              L.OPT_LINK_BUF: (0, 1, 1), L.OPT_SWEEP_CHUNKS: (0, 1024, 0)}
    for opt, (lo, hi, default) in ranges.items():
        assert lib.mpmc_set_option(opt, lo) == L.OK
        assert lib.mpmc_set_option(opt, hi) == L.OK
        assert lib.mpmc_set_option(opt, lo - 1) == L.EINVAL
        assert lib.mpmc_set_option(opt, hi + 1) == L.EINVAL
        assert lib.mpmc_set_option(opt, default) == L.OK
    assert lib.mpmc_set_option(0, 1) == L.EUNSUPPORTED
    assert lib.mpmc_set_option(max(ranges) + 1, 1) == L.EUNSUPPORTED


def test_binding_tracks_the_options_it_sets(L):
    """set_option records what the library accepted, so that a call that
    scopes an option (a level's kernel selection) can restore the caller's
    value; a rejected value leaves the record alone."""
    assert L.get_option(L.OPT_PLANE_SWEEP) == L.SWEEP_AUTO and L.get_option(L.OPT_SWEEP_CHUNKS) == 0
    try:
        L.set_option(L.OPT_SWEEP_CHUNKS, 4)
        assert L.get_option(L.OPT_SWEEP_CHUNKS) == 4
        with pytest.raises(L.MpmcError):
            L.set_option(L.OPT_SWEEP_CHUNKS, 2000)
        assert L.get_option(L.OPT_SWEEP_CHUNKS) == 4
    finally:
        L.set_option(L.OPT_SWEEP_CHUNKS, 0)
