"""Pins of the oracle's probing trace (Sec. 5 step 3d) and of the product's
colouring (host logic).  No GPU."""
import numpy as np
import pytest

import oracle
import synth
from oracle import deflation, dense, krylov, probing


def _random_roots(n, seed):
    rng = np.random.default_rng(seed)
    return 0.5 + 0.2 * rng.standard_normal(n) + 0.1j * rng.standard_normal(n)


@pytest.mark.parametrize("dims,deg", [((2, 2, 2, 4), 2), ((4, 2, 2, 4), 3), ((4, 4, 2, 2), 1)])
def test_probe_trace_equals_spectral_trace(dims, deg):
    """Probing with a distance-deg colouring gives sum_i p(lambda_i) (LAPACK)."""
    lat = oracle.Lattice(dims, 0.14, synth.gauge_links(dims, 0.5, 3), True)
    t = _random_roots(deg + 1, deg)
    col = probing.distance_colouring(dims, deg)
    got = probing.probe_trace(lat, t, col)
    lam = np.linalg.eigvals(dense.dense_matrix(lat))
    want = np.sum(deflation.poly_eval(t, lam))
    assert abs(got - want) < 1e-10 * np.sum(np.abs(deflation.poly_eval(t, lam)))


def test_probe_trace_free_field_closed_form():
    dims, deg = (4, 4, 4, 4), 3
    lat = oracle.Lattice(dims, 0.13, synth.unit_links(dims), True)
    t = _random_roots(deg + 1, 11)
    got = probing.probe_trace(lat, t, probing.distance_colouring(dims, deg))
    want = dense.free_field_trace_fn(dims, 0.13, lambda l: deflation.poly_eval(t, l), True)
    assert abs(got - want) < 1e-10 * abs(want)


def test_too_coarse_colouring_is_wrong():
    """A colouring one step too short misses couplings: the trace is off."""
    dims, deg = (4, 2, 2, 4), 3
    lat = oracle.Lattice(dims, 0.14, synth.gauge_links(dims, 0.5, 3), True)
    t = _random_roots(deg + 1, 5)
    good = probing.probe_trace(lat, t, probing.distance_colouring(dims, deg))
    bad = probing.probe_trace(lat, t, probing.distance_colouring(dims, deg - 1))
    assert abs(bad - good) > 1e-6 * abs(good)


@pytest.fixture(scope="module")
def pp():
    pytest.importorskip("torch")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists(os.path.join(root, "paper_2306_09559_amd", "libmpmc.so")):
        pytest.skip("libmpmc.so not built")
    from paper_2306_09559_amd import probing as pprobe
    return pprobe


@pytest.mark.parametrize("dims,d", [((4, 4, 2, 4), 2), ((4, 4, 4, 4), 3), ((6, 4, 4, 2), 4)])
def test_product_colouring_is_a_distance_colouring(pp, dims, d):
    """Every pair of same-coloured sites is more than d apart (brute force
    over all pairs with the oracle's torus distance), and the colouring is not
    valid one step further (the check has teeth)."""
    col = pp.colouring(dims, d)
    V = len(col)
    for a in range(V):
        for b in range(a + 1, V):
            if col[a] == col[b]:
                assert probing.torus_distance(dims, a, b) > d
    assert pp.is_valid(dims, d, col) and not pp.is_valid(dims, d + 1, col)


def test_product_tiled_colouring_sampled(pp):
    """The tiled colouring of a large lattice: same-coloured sites are more
    than d apart for random pairs within a window (brute-force distances)."""
    dims, d = (24, 24, 24, 48), 4
    col = pp.colouring(dims, d)
    V = len(col)
    rng = np.random.default_rng(0)
    lx, ly, lz = dims[:3]
    for a in rng.integers(0, V, 400):
        x, y, z, t = a % lx, (a // lx) % ly, (a // (lx * ly)) % lz, a // (lx * ly * lz)
        for _ in range(200):
            o = rng.integers(-d, d + 1, 4)
            if 0 < np.abs(o).sum() <= d:
                b = ((x + o[0]) % lx) + lx * (((y + o[1]) % ly) + ly * (((z + o[2]) % lz) + lz * ((t + o[3]) % dims[3])))
                assert col[a] != col[b]
