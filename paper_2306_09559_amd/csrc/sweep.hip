// Newton step of a GMRES polynomial (Sec. 3.1) as a t-sweep: one workgroup
// owns one vector and one whole xyz-plane of the lattice (one thread per
// (x, y, z)), and marches through t = 0 .. Lt-1 (or, for larger planes, an
// xyz-block of it with a halo; for small batches, one t-chunk of the planes,
// started from the plane before it).
//
//   * The current plane is staged in LDS; the +-x, +-y, +-z neighbours are
//     read from there (periodic wrap inside the plane).
//   * The +t neighbour is the next plane, prefetched into registers one
//     step ahead; the -t term of a site is formed one step early from the
//     plane below it and carried as a spin-projected half spinor.
//   * Every spinor of the input is therefore read from HBM once and the
//     output written once (plus one re-read of plane 0 for the periodic
//     wrap): the compulsory traffic of the step.
//
// The step computes out = (1 - t_j) w + kappa t_j D w and the FP64 partial
// t_{j+1} b^H out (plus t_0 b^H w on the first step) of the scalar-mode
// Newton recurrence, exactly as the streaming kernel does; only the order of
// the floating-point sums inside a site differs.
#include "common.hpp"
#include <algorithm>
#include <cmath>
#include "internal.hpp"

namespace mpmc {

template <typename T> struct SweepArgs {
    int L[4];
    int P, V;                  // plane sites Lx*Ly*Lz, volume
    int apbc;
    const cplx_t<T> *in;       // input field (layout rb_in), unused for noise input
    int rb_in;
    cplx_t<T> *out;            // output field, rb = 1
    const cplx_t<T> *gauge;    // [mu][9][V]
    int two_rows;              // links special unitary: row 2 rebuilt from rows 0, 1
    const double2 *troots;
    int j;
    double kappa;
    uint64_t key, first;       // noise (input when IN_Z4; dot vector when bvec == nullptr)
    const uint64_t *off;       // device sample counter added to first, or nullptr
    const int32_t *colour;     // probe vectors of this colouring instead of Z4 noise, or nullptr
    const cplx_t<T> *bvec;     // dot vector field (layout rb_b), or nullptr
    int rb_b;
    double2 *part;             // partial sums, one per (vector, t-chunk, block)
    double2 *bhy;              // final sums (last step, whole planes in one t-chunk only), or nullptr
    int dot_first;
    // xyz-blocks (HALO): block extents, sites, halo sites, blocks per plane
    int B[3];
    int Pb, Hb, nbp;
    // t-chunks: a workgroup walks Lt / nch planes (nch divides Lt)
    int nch;
    // vector mode (YACC): y (block width 1) accumulates t_j w_j, zeroed first, + t_{j+1} w_{j+1} last
    cplx_t<T> *y;
    int y_first, y_last;
};

namespace {

template <typename T> __device__ __forceinline__ cplx_t<T> neg(cplx_t<T> a) { return mk<T>(-a.x, -a.y); }

// Every spinor of a sweep is read once, so the plane loads carry the
// nontemporal hint: they stream through L2 without evicting the links, which
// every workgroup of the launch reads again (measured: 139 -> 110 us per FP64
// launch at 8^4 x 256 vectors, loads and stores nontemporal).  The stores are
// plain: the step's next link wait also waits for them (vector memory
// operations complete in issue order), and plain stores complete sooner
// (FP64 106 -> 102 us at 8^4 x 256 vectors, 74 -> 72 us at 64; FP32 even).
// Component c of vector r of a batch with block width rb, site s, lives at
// byte  cbase(r, c) + s * rb * sizeof(C)  where cbase is wavefront-uniform
// (scalar registers) and the per-site offset fits 32 bits (V * rb * sizeof(C)
// < 4 GiB is checked on the host).
template <typename T> struct Plane {
    const char *base;   // vector r, component 0
    size_t cstride;     // bytes between components
    uint32_t sstride;   // bytes between sites
    __device__ __forceinline__ cplx_t<T> ld(int c, int s) const {
        const T *p = (const T *)(base + (size_t)c * cstride + (uint32_t)s * sstride);
        return mk<T>(__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + 1));
    }
    __device__ __forceinline__ void st(int c, int s, cplx_t<T> v) const {
        T *p = (T *)(const_cast<char *>(base) + (size_t)c * cstride + (uint32_t)s * sstride);
        p[0] = v.x;
        p[1] = v.y;
    }
};

template <typename T> __device__ __forceinline__ Plane<T> plane_of(const void *f, int r, int V, int rb) {
    Plane<T> p;
    const size_t csz = sizeof(cplx_t<T>);
    p.cstride = (size_t)V * (size_t)rb * csz;
    p.sstride = (uint32_t)(rb * csz);
    p.base = (const char *)f + (size_t)(r / rb) * 12 * p.cstride + (size_t)(r % rb) * csz;
    return p;
}

// the noise of one vector: Z4 from its sample state S, or, with a colouring,
// the probe vector b_{cg, kk} (1 at unknown kk of the sites of colour cg)
struct NoiseSrc {
    uint64_t S;
    const int32_t *colour;
    long long cg;
    int kk;
};

template <typename T, bool PROBE>
__device__ __forceinline__ void noise_site(const NoiseSrc &ns, int s, cplx_t<T> (&p)[12]) {
    if constexpr (PROBE) {
        const bool on = (long long)ns.colour[s] == ns.cg;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = mk<T>((on && c == ns.kk) ? T(1) : T(0), T(0));
    } else {
        const uint32_t codes = z4_site_codes(ns.S, (unsigned)s);
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = z4_value<T>((codes >> (2 * c)) & 3u);
    }
}

template <typename T, bool PROBE = false>
__device__ __forceinline__ void load_plane_site(const Plane<T> &in, bool z4, const NoiseSrc &ns, int s,
                                                cplx_t<T> (&p)[12]) {
    if (z4) {
        noise_site<T, PROBE>(ns, s, p);
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = in.ld(c, s);
    }
}

template <typename T>
__device__ __forceinline__ void load_link(const char *g, size_t estride, int site, bool two_rows, cplx_t<T> (&U)[9]) {
    load_su3<T>(g, estride, (uint32_t)site * (uint32_t)sizeof(cplx_t<T>), two_rows, U);
}

// half spinor h (2 x 3) <- U h or U^H h
template <typename T, bool HERM>
__device__ __forceinline__ void mul_link(const cplx_t<T> (&U)[9], cplx_t<T> (&h)[2][3]) {
    cplx_t<T> o[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx_t<T> t = mk<T>(T(0), T(0));
#pragma unroll
            for (int b = 0; b < 3; ++b) t = HERM ? cfmaconj<T>(U[3 * b + a], h[sp][b], t) : cfma<T>(U[3 * a + b], h[sp][b], t);
            o[sp][a] = t;
        }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[sp][a] = o[sp][a];
}

// spin projections (1 -+ g_mu) to a half spinor and the matching
// reconstruction; DeGrand-Rossi basis (same algebra as the streaming kernel)
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void proj(const cplx_t<T> (&p)[12], cplx_t<T> (&h)[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx_t<T> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
        if (MU == 0) {
            h[0][a] = FWD ? cadd<T>(p0, mul_mi<T>(p3)) : cadd<T>(p0, mul_i<T>(p3));
            h[1][a] = FWD ? cadd<T>(p1, mul_mi<T>(p2)) : cadd<T>(p1, mul_i<T>(p2));
        } else if (MU == 1) {
            h[0][a] = FWD ? cadd<T>(p0, p3) : csub<T>(p0, p3);
            h[1][a] = FWD ? csub<T>(p1, p2) : cadd<T>(p1, p2);
        } else if (MU == 2) {
            h[0][a] = FWD ? cadd<T>(p0, mul_mi<T>(p2)) : cadd<T>(p0, mul_i<T>(p2));
            h[1][a] = FWD ? cadd<T>(p1, mul_i<T>(p3)) : cadd<T>(p1, mul_mi<T>(p3));
        } else {
            h[0][a] = FWD ? csub<T>(p0, p2) : cadd<T>(p0, p2);
            h[1][a] = FWD ? csub<T>(p1, p3) : cadd<T>(p1, p3);
        }
    }
}

template <typename T, int MU, bool FWD>
__device__ __forceinline__ void recon(const cplx_t<T> (&h)[2][3], cplx_t<T> (&acc)[12]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx_t<T> h0 = h[0][a], h1 = h[1][a];
        acc[a] = cadd<T>(acc[a], h0);
        acc[3 + a] = cadd<T>(acc[3 + a], h1);
        cplx_t<T> r2, r3;
        if (MU == 0) {
            r2 = FWD ? mul_i<T>(h1) : mul_mi<T>(h1);
            r3 = FWD ? mul_i<T>(h0) : mul_mi<T>(h0);
        } else if (MU == 1) {
            r2 = FWD ? neg<T>(h1) : h1;
            r3 = FWD ? h0 : neg<T>(h0);
        } else if (MU == 2) {
            r2 = FWD ? mul_i<T>(h0) : mul_mi<T>(h0);
            r3 = FWD ? mul_mi<T>(h1) : mul_i<T>(h1);
        } else {
            r2 = FWD ? neg<T>(h0) : h0;
            r3 = FWD ? neg<T>(h1) : h1;
        }
        acc[6 + a] = cadd<T>(acc[6 + a], r2);
        acc[9 + a] = cadd<T>(acc[9 + a], r3);
    }
}

// one spatial hop read from the LDS plane (component-major: lds[c*P + q])
// projection read straight from the LDS plane, one spin pair at a time
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void proj_lds(const cplx_t<T> *lds, int P, int q, cplx_t<T> (&h)[2][3]) {
    // partner spin of spin 0 and of spin 1 under g_mu
    constexpr int k0 = (MU == 0 || MU == 1) ? 3 : 2;
    constexpr int k1 = (MU == 0 || MU == 1) ? 2 : 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx_t<T> p0 = lds[a * P + q], pk = lds[(3 * k0 + a) * P + q];
        if (MU == 0) h[0][a] = FWD ? cadd<T>(p0, mul_mi<T>(pk)) : cadd<T>(p0, mul_i<T>(pk));
        else if (MU == 1) h[0][a] = FWD ? cadd<T>(p0, pk) : csub<T>(p0, pk);
        else if (MU == 2) h[0][a] = FWD ? cadd<T>(p0, mul_mi<T>(pk)) : cadd<T>(p0, mul_i<T>(pk));
        else h[0][a] = FWD ? csub<T>(p0, pk) : cadd<T>(p0, pk);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx_t<T> p1 = lds[(3 + a) * P + q], pk = lds[(3 * k1 + a) * P + q];
        if (MU == 0) h[1][a] = FWD ? cadd<T>(p1, mul_mi<T>(pk)) : cadd<T>(p1, mul_i<T>(pk));
        else if (MU == 1) h[1][a] = FWD ? csub<T>(p1, pk) : cadd<T>(p1, pk);
        else if (MU == 2) h[1][a] = FWD ? cadd<T>(p1, mul_i<T>(pk)) : cadd<T>(p1, mul_mi<T>(pk));
        else h[1][a] = FWD ? csub<T>(p1, pk) : cadd<T>(p1, pk);
    }
}

// accumulate the reconstruction of colour a of the rotated half spinor (g0, g1)
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void recon_a(int a, cplx_t<T> g0, cplx_t<T> g1, cplx_t<T> (&acc)[12]) {
    acc[a] = cadd<T>(acc[a], g0);
    acc[3 + a] = cadd<T>(acc[3 + a], g1);
    cplx_t<T> r2, r3;
    if (MU == 0) {
        r2 = FWD ? mul_i<T>(g1) : mul_mi<T>(g1);
        r3 = FWD ? mul_i<T>(g0) : mul_mi<T>(g0);
    } else if (MU == 1) {
        r2 = FWD ? neg<T>(g1) : g1;
        r3 = FWD ? g0 : neg<T>(g0);
    } else if (MU == 2) {
        r2 = FWD ? mul_i<T>(g0) : mul_mi<T>(g0);
        r3 = FWD ? mul_mi<T>(g1) : mul_i<T>(g1);
    } else {
        r2 = FWD ? neg<T>(g0) : g0;
        r3 = FWD ? neg<T>(g1) : g1;
    }
    acc[6 + a] = cadd<T>(acc[6 + a], r2);
    acc[9 + a] = cadd<T>(acc[9 + a], r3);
}

// one spatial hop: projection from LDS, then the link applied one output
// colour at a time (row a of U, or column a of U for U^H) straight into acc
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void plane_hop(const cplx_t<T> *lds, int P, int q, const char *glmu, size_t estride,
                                          int gsite, bool two_rows, cplx_t<T> (&acc)[12]) {
    cplx_t<T> h[2][3];
    proj_lds<T, MU, FWD>(lds, P, q, h);
    cplx_t<T> U[9];
    load_link<T>(glmu, estride, gsite, two_rows, U);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cplx_t<T> u[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) u[b] = U[FWD ? 3 * a + b : 3 * b + a];
        cplx_t<T> g0 = mk<T>(T(0), T(0)), g1 = mk<T>(T(0), T(0));
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (FWD) {
                g0 = cfma<T>(u[b], h[0][b], g0);
                g1 = cfma<T>(u[b], h[1][b], g1);
            } else {
                g0 = cfmaconj<T>(u[b], h[0][b], g0);
                g1 = cfmaconj<T>(u[b], h[1][b], g1);
            }
        }
        recon_a<T, MU, FWD>(a, g0, g1, acc);
    }
}

// link elements as stored (two rows when TWO), and the rebuild of row 2
template <typename T, bool TWO>
__device__ __forceinline__ void link_raw(const char *g, size_t estride, int site, cplx_t<T> (&U)[9]) {
    const uint32_t off = (uint32_t)site * (uint32_t)sizeof(cplx_t<T>);
#pragma unroll
    for (int e = 0; e < (TWO ? 6 : 9); ++e) U[e] = *(const cplx_t<T> *)(g + (size_t)e * estride + off);
}
template <typename T, bool TWO> __device__ __forceinline__ void link_complete(cplx_t<T> (&U)[9]) {
    if (TWO) {
        const cplx_t<T> c0 = csub<T>(cmul<T>(U[1], U[5]), cmul<T>(U[2], U[4]));
        const cplx_t<T> c1 = csub<T>(cmul<T>(U[2], U[3]), cmul<T>(U[0], U[5]));
        const cplx_t<T> c2 = csub<T>(cmul<T>(U[0], U[4]), cmul<T>(U[1], U[3]));
        U[6] = mk<T>(c0.x, -c0.y);
        U[7] = mk<T>(c1.x, -c1.y);
        U[8] = mk<T>(c2.x, -c2.y);
    }
}

// plane_hop with the link already in registers
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void plane_hop_u(const cplx_t<T> *lds, int P, int q, const cplx_t<T> (&U)[9],
                                            cplx_t<T> (&acc)[12]) {
    cplx_t<T> h[2][3];
    proj_lds<T, MU, FWD>(lds, P, q, h);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cplx_t<T> u[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) u[b] = U[FWD ? 3 * a + b : 3 * b + a];
        cplx_t<T> g0 = mk<T>(T(0), T(0)), g1 = mk<T>(T(0), T(0));
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (FWD) {
                g0 = cfma<T>(u[b], h[0][b], g0);
                g1 = cfma<T>(u[b], h[1][b], g1);
            } else {
                g0 = cfmaconj<T>(u[b], h[0][b], g0);
                g1 = cfmaconj<T>(u[b], h[1][b], g1);
            }
        }
        recon_a<T, MU, FWD>(a, g0, g1, acc);
    }
}

// FP32 whole planes: the backward-hop product U_mu(x)^H (1 + g_mu) w(x) of
// this site's own link, left in LDS (bwl[(mu * 6 + 3 sp + a) * Pb + q]) for
// the neighbour x + mu
template <typename T, int MU>
__device__ __forceinline__ void own_backward(const cplx_t<T> (&w)[12], const cplx_t<T> (&U)[9], cplx_t<T> *bwl,
                                             int Pb, int q) {
    cplx_t<T> h[2][3];
    proj<T, MU, false>(w, h);
    mul_link<T, true>(U, h);
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) bwl[(MU * 6 + sp * 3 + a) * Pb + q] = h[sp][a];
}

// the forward hop with this site's link U_mu(x), then the backward hop
// from the product the neighbour x - mu (LDS slot qb) left
template <typename T, int MU>
__device__ __forceinline__ void own_hops(const cplx_t<T> *lds, int Sl, int qf, int qb, const cplx_t<T> (&U)[9],
                                         const cplx_t<T> *bwl, int Pb, cplx_t<T> (&acc)[12]) {
    plane_hop_u<T, MU, true>(lds, Sl, qf, U, acc);
    cplx_t<T> g[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) g[sp][a] = bwl[(MU * 6 + sp * 3 + a) * Pb + qb];
    recon<T, MU, false>(g, acc);
}

__device__ __forceinline__ double2 zmul2(double2 a, double2 b) {
    double2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

template <typename T>
__device__ __forceinline__ void dot_acc(const cplx_t<T> (&b)[12], const cplx_t<T> (&w)[12], double &re, double &im) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double br = (double)b[c].x, bi = (double)b[c].y, wr = (double)w[c].x, wi = (double)w[c].y;
        re += br * wr + bi * wi;
        im += br * wi - bi * wr;
    }
}

// The scalar-mode dot of one launch: t_{j+1} b^H w_{j+1} (+ t_j b^H w_j on the
// first step) from each thread's FP64 partial, summed over the block in a
// fixed-order tree (LDS plane buffer reused) and added to the vector's (or
// block's) running partial.
template <typename T, bool FIRST, bool HALO>
__device__ __forceinline__ void sweep_dot_finish(const SweepArgs<T> &a, int r, size_t pi, int q, int Pb, double2 tj,
                                                 double dre, double dim, double d0re, double d0im,
                                                 unsigned char *smem) {
    double2 *red = reinterpret_cast<double2 *>(smem);
    double2 v = zmul2(a.troots[a.j + 1], make_double2(dre, dim));
    if (FIRST) {
        const double2 v0 = zmul2(tj, make_double2(d0re, d0im));
        v.x += v0.x;
        v.y += v0.y;
    }
    red[q] = v;
    __syncthreads();
    int n = Pb;
    while (n > 1) {
        const int h = (n + 1) >> 1;
        if (q < n - h) {
            red[q].x += red[q + h].x;
            red[q].y += red[q + h].y;
        }
        __syncthreads();
        n = h;
    }
    if (q == 0) {
        // one partial per (vector, t-chunk, block); a whole plane in one
        // t-chunk also writes b^H y at the end
        double2 tot = red[0];
        if (!FIRST) {
            tot.x += a.part[pi].x;
            tot.y += a.part[pi].y;
        }
        a.part[pi] = tot;
        if (!HALO && a.bhy) a.bhy[r] = tot;
    }
}

// A step with kappa t_j = 0 (kappa = 0, i.e. A = I, or an inverse root 0):
// w_{j+1} = (1 - t_j) w_j involves no hop.  The main path forms
// kappa t_j ((1 - t_j) / (kappa t_j) w + D w), which does not exist here, so
// such a launch takes this separate path at entry: each thread scales its own
// sites plane by plane, with the same dot, vector-mode update and reduction.
// Taken at entry, its registers are not live in the main loop (folded into
// the step's epilogue instead, the same update cost 2% per FP64 launch at
// 8^4 x 256 vectors; as an out-of-line call it made every variant spill).
template <typename T, bool IN_Z4, bool DOT, bool FIRST, bool BFIELD, bool HALO, bool YACC, bool PROBE>
__device__ __forceinline__ void sweep_step_no_hop(const SweepArgs<T> &a, int r, size_t pi, int t0, int t1, int q,
                                                  int Pb, int gq,
                                               NoiseSrc S, unsigned char *smem) {
    using C = cplx_t<T>;
    const int P = a.P;
    const double2 tj = a.troots[a.j];
    const double2 alpha = make_double2(1.0 - tj.x, -tj.y);
    const Plane<T> inp = plane_of<T>(a.in, r, a.V, a.rb_in);
    const Plane<T> outp = plane_of<T>(a.out, r, a.V, 1);
    double dre = 0.0, dim = 0.0, d0re = 0.0, d0im = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int s = gq + t * P;
        C w[12], o[12];
        load_plane_site<T, PROBE>(inp, IN_Z4, S, s, w);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            o[c] = cmul_d<T>(alpha, w[c]);
            outp.st(c, s, o[c]);
        }
        if (DOT) {
            C b[12];
            if (!BFIELD) {
                noise_site<T, PROBE>(S, s, b);
            } else {
                const Plane<T> bp = plane_of<T>(a.bvec, r, a.V, a.rb_b);
#pragma unroll
                for (int c = 0; c < 12; ++c) b[c] = bp.ld(c, s);
            }
            if (FIRST) dot_acc<T>(b, w, d0re, d0im);
            dot_acc<T>(b, o, dre, dim);
        }
        if constexpr (YACC) {
            const Plane<T> yp = plane_of<T>(a.y, r, a.V, 1);
            const double2 tn = a.y_last ? a.troots[a.j + 1] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                C yv = a.y_first ? mk<T>(T(0), T(0)) : yp.ld(c, s);
                yv = axpy_d<T>(tj, w[c], yv);
                if (a.y_last) yv = axpy_d<T>(tn, o[c], yv);
                yp.st(c, s, yv);
            }
        }
    }
    if (DOT) sweep_dot_finish<T, FIRST, HALO>(a, r, pi, q, Pb, tj, dre, dim, d0re, d0im, smem);
}

}  // namespace

// IN_Z4: the input is the noise itself; FIRST: also accumulate t_0 b^H w
// (first Newton step); BFIELD: the dot vector b is a field, not the noise;
// TWO: the links are read as two rows (SU(3), row 2 rebuilt) -- a template
// parameter because a run-time flag cost 6% (FP64) and 14% (FP32) per launch;
// HALO: a workgroup owns an xyz-block of the plane (the plane is too large
// for one workgroup's LDS) and stages a one-site halo of the neighbouring
// blocks next to it; without HALO the block is the whole plane and the x, y,
// z neighbours wrap inside it.
template <typename T, bool IN_Z4, bool DOT, bool FIRST, bool BFIELD, bool TWO, bool HALO, bool YACC = false,
          bool PROBE = false>
__global__ void __launch_bounds__(512) k_sweep(SweepArgs<T> a) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int P = a.P, Lt = a.L[3];
    const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
    const int q = (int)threadIdx.x;               // site within the block
    int r, blk = 0, ch;
    int x, y, z, bx, by, bz, Pb, Hb;
    if (HALO) {
        // the blocks of one (vector, t-chunk) are consecutive logical ids: one
        // XCD, shared halos in its L2
        const unsigned lg = xcd_remap(blockIdx.x, gridDim.x);
        blk = (int)(lg % (unsigned)a.nbp);
        const unsigned rc = lg / (unsigned)a.nbp;
        r = (int)(rc / (unsigned)a.nch);
        ch = (int)(rc % (unsigned)a.nch);
        bx = a.B[0];
        by = a.B[1];
        bz = a.B[2];
        Pb = a.Pb;
        Hb = a.Hb;
        const int nbx = Lx / bx, nby = Ly / by;
        x = (blk % nbx) * bx + q % bx;
        y = ((blk / nbx) % nby) * by + (q / bx) % by;
        z = (blk / (nbx * nby)) * bz + q / (bx * by);
    } else {
        r = (int)(blockIdx.x / (unsigned)a.nch);
        ch = (int)(blockIdx.x % (unsigned)a.nch);
        bx = Lx;
        by = Ly;
        bz = Lz;
        Pb = P;
        Hb = 0;
        x = q % Lx;
        y = (q / Lx) % Ly;
        z = q / (Lx * Ly);
    }
    const int Sl = Pb + Hb;                       // LDS sites: block, then halo
    const int lx = q % bx, ly = (q / bx) % by, lz = q / (bx * by);
    const int gq = x + Lx * (y + Ly * z);         // plane index of this site
    // plane indices of the backward neighbours (periodic), for their links
    const int gxm = x == 0 ? gq + Lx - 1 : gq - 1;
    const int gym = y == 0 ? gq + (Ly - 1) * Lx : gq - Lx;
    const int gzm = z == 0 ? gq + (Lz - 1) * Lx * Ly : gq - Lx * Ly;
    // LDS slots of the six neighbours: inside the block, wrapped inside it
    // when the block spans the dimension, else on the halo face
    const bool hx = bx < Lx, hy = by < Ly, hz = bz < Lz;
    const int Fx = by * bz, Fy = bx * bz, Fz = bx * by;
    const int o_xm = 0, o_xp = hx ? Fx : 0, o_ym = hx ? 2 * Fx : 0;
    const int o_yp = o_ym + (hy ? Fy : 0), o_zm = o_ym + (hy ? 2 * Fy : 0), o_zp = o_zm + (hz ? Fz : 0);
    const int sxp = lx + 1 < bx ? q + 1 : (!hx ? q - lx : Pb + o_xp + ly + by * lz);
    const int sxm = lx > 0 ? q - 1 : (!hx ? q + bx - 1 : Pb + o_xm + ly + by * lz);
    const int syp = ly + 1 < by ? q + bx : (!hy ? q - ly * bx : Pb + o_yp + lx + bx * lz);
    const int sym = ly > 0 ? q - bx : (!hy ? q + (by - 1) * bx : Pb + o_ym + lx + bx * lz);
    const int szp = lz + 1 < bz ? q + bx * by : (!hz ? q - lz * bx * by : Pb + o_zp + lx + bx * ly);
    const int szm = lz > 0 ? q - bx * by : (!hz ? q + (bz - 1) * bx * by : Pb + o_zm + lx + bx * ly);
    // the halo site this thread stages (threads q < Hb), as a plane index
    int ghq = 0;
    if (HALO && q < Hb) {
        const int x0 = x - lx, y0 = y - ly, z0 = z - lz;
        int hx_, hy_, hz_, f;
        if (q < o_ym) {                           // x faces
            f = q < o_xp ? q : q - o_xp;
            hx_ = q < o_xp ? (x0 == 0 ? Lx - 1 : x0 - 1) : (x0 + bx == Lx ? 0 : x0 + bx);
            hy_ = y0 + f % by;
            hz_ = z0 + f / by;
        } else if (q < o_zm) {                    // y faces
            const bool minus = q < o_yp;
            f = minus ? q - o_ym : q - o_yp;
            hx_ = x0 + f % bx;
            hy_ = minus ? (y0 == 0 ? Ly - 1 : y0 - 1) : (y0 + by == Ly ? 0 : y0 + by);
            hz_ = z0 + f / bx;
        } else {                                  // z faces
            const bool minus = q < o_zp;
            f = minus ? q - o_zm : q - o_zp;
            hx_ = x0 + f % bx;
            hy_ = y0 + f / bx;
            hz_ = minus ? (z0 == 0 ? Lz - 1 : z0 - 1) : (z0 + bz == Lz ? 0 : z0 + bz);
        }
        ghq = hx_ + Lx * (hy_ + Ly * hz_);
    }
    const size_t V = (size_t)a.V;
    const size_t estride = V * sizeof(C);
    constexpr bool two = TWO;
    const char *g0 = (const char *)a.gauge;
    const char *gx = g0, *gy = g0 + 9 * estride, *gz = g0 + 18 * estride, *gt = g0 + 27 * estride;

    const double2 tj = a.troots[a.j];
    const double2 beta = make_double2(a.kappa * tj.x, a.kappa * tj.y);   // kappa t_j
    const uint64_t g = sample_base(a.first, a.off) + (uint64_t)r;      // global sample (or probe) index
    const NoiseSrc S{PROBE ? 0ull : sample_state(a.key, g), a.colour, (long long)(g / 12u), (int)(g % 12u)};
    // this workgroup's planes t0 .. t1-1 and its partial sum
    const int tc = Lt / a.nch, t0 = ch * tc, t1 = t0 + tc;
    const size_t pidx = ((size_t)r * (size_t)a.nch + (size_t)ch) * (size_t)a.nbp + (size_t)blk;
    if (a.kappa * (tj.x * tj.x + tj.y * tj.y) == 0.0) {   // kappa t_j = 0 (uniform over the launch)
        sweep_step_no_hop<T, IN_Z4, DOT, FIRST, BFIELD, HALO, YACC, PROBE>(a, r, pidx, t0, t1, q, Pb, gq, S, smem);
        return;
    }
    const Plane<T> inp = plane_of<T>(a.in, r, a.V, a.rb_in);
    const Plane<T> outp = plane_of<T>(a.out, r, a.V, 1);

    // The -t term of the next plane is carried in LDS behind the plane (as the
    // colour-rotated half spinor (1 + g_t) U_t^H psi, sign included), which
    // keeps it out of the registers during the hops.
    C *stl = lds + 12 * Sl;
    // FP32 whole planes after the first step: every site forms the
    // backward-hop products of its own x-, y- and z-links, U_mu(x)^H (1 + g_mu)
    // w(x), and leaves them in LDS (bwl, 144 B per site) for its neighbours
    // x + mu, which then load 5 links per step instead of 8; links are read as
    // three rows, so nothing is rebuilt (68.5 -> 61.7 us per launch at 8^4 x
    // 256 vectors).  FP64 has no LDS left for it; on blocks with a halo the
    // halo sites' products would not fit either; the first-step kernels keep
    // the general path (its registers are already at their limit).
    constexpr bool OWN = sizeof(T) == 4 && !HALO && !FIRST;
    constexpr bool TWOL = OWN ? false : TWO;
    C *bwl = stl + 6 * Pb;
    // prologue: -t term of plane t0 from plane t0-1 (Lt-1 for t0 = 0, across
    // the boundary); cur (and halo) = plane t0
    C stash[2][3];
    {
        C p[12];
        const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
        load_plane_site<T, PROBE>(inp, IN_Z4, S, gq + tp * P, p);
        proj<T, 3, false>(p, stash);
        C U[9];
        load_link<T>(gt, estride, gq + tp * P, two, U);
        mul_link<T, true>(U, stash);
        const T sg = (t0 == 0 && a.apbc) ? T(-1) : T(1);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) stl[(sp * 3 + aa) * Pb + q] = mk<T>(sg * stash[sp][aa].x, sg * stash[sp][aa].y);
    }
    // Vector memory operations complete in issue order, so a wait for a link
    // (an L2 hit) also waits for every HBM load and store issued before it.
    // The links a step needs first are therefore requested ahead of the plane
    // traffic: the -t link of the next step before this step's stores, the
    // first spatial hop's link before the next plane's loads (measured at
    // 8^4 x 256 vectors FP64, with the hops unrolled: 112 -> 106 us per launch;
    // at 64 vectors 83 -> 75 us).
    C Ust[9];
    link_raw<T, TWOL>(gt, estride, gq + t0 * P, Ust);
    C cur[12];
    load_plane_site<T, PROBE>(inp, IN_Z4, S, gq + t0 * P, cur);
    C hcur[12];
    if constexpr (HALO) {
        if (q < Hb) load_plane_site<T, PROBE>(inp, IN_Z4, S, ghq + t0 * P, hcur);
    }

    // out = alpha w + beta D w is formed as beta * ((alpha/beta) w + D w): the
    // current spinor then enters the accumulator at the start of the step and
    // is dead during the hops (beta = kappa t_j = 0 took the path above)
    double2 aob;
    {
        // (1 - t) / (kappa t) = (1 - t) conj(t) / (kappa |t|^2)
        const double den = a.kappa * (tj.x * tj.x + tj.y * tj.y);
        const double ar = 1.0 - tj.x, ai = -tj.y;
        aob.x = (ar * tj.x + ai * tj.y) / den;
        aob.y = (ai * tj.x - ar * tj.y) / den;
    }

    double dre = 0.0, dim = 0.0, d0re = 0.0, d0im = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int s = gq + t * P;
        const T sg = (t + 1 == Lt && a.apbc) ? T(-1) : T(1);
#pragma unroll
        for (int c = 0; c < 12; ++c) lds[c * Sl + q] = cur[c];
        if constexpr (HALO) {
            if (q < Hb) {
#pragma unroll
                for (int c = 0; c < 12; ++c) lds[c * Sl + Pb + q] = hcur[c];
            }
        }
        // accumulator: (alpha/beta) w + the -t term carried from plane t-1
        C acc[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = cmul_d<T>(aob, cur[c]);
        {
            C st[2][3];
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) st[sp][aa] = stl[(sp * 3 + aa) * Pb + q];
            recon<T, 3, false>(st, acc);
        }
        // the -t term of (x, t+1): (1 + g_t) U_t(x, t)^H w(x, t)
        {
            C st[2][3];
            link_complete<T, TWOL>(Ust);
            proj<T, 3, false>(cur, st);
            mul_link<T, true>(Ust, st);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) stl[(sp * 3 + aa) * Pb + q] = mk<T>(sg * st[sp][aa].x, sg * st[sp][aa].y);
        }
        if (DOT && FIRST) {
            C b[12];
            if (!BFIELD) {
                noise_site<T, PROBE>(S, s, b);
            } else {
                const Plane<T> bp = plane_of<T>(a.bvec, r, a.V, a.rb_b);
#pragma unroll
                for (int c = 0; c < 12; ++c) b[c] = bp.ld(c, s);
            }
            dot_acc<T>(b, cur, d0re, d0im);
        }
        // the first spatial hop's link, then the +t plane (plane 0 again after
        // the last one) and its halo
        C U0[9];
        link_raw<T, TWOL>(gx, estride, s, U0);
        C Uy[OWN ? 9 : 1], Uz[OWN ? 9 : 1];   // the y- and z-links (OWN only)
        if constexpr (OWN) {
            link_raw<T, false>(gy, estride, s, Uy);
            link_raw<T, false>(gz, estride, s, Uz);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (OWN) {
            own_backward<T, 0>(cur, U0, bwl, Pb, q);
            own_backward<T, 1>(cur, Uy, bwl, Pb, q);
            own_backward<T, 2>(cur, Uz, bwl, Pb, q);
            __builtin_amdgcn_sched_barrier(0);
        }
        const int tn = t + 1 == Lt ? 0 : t + 1;
        C nxt[12];
        load_plane_site<T, PROBE>(inp, IN_Z4, S, gq + tn * P, nxt);
        C hnx[12];
        if constexpr (HALO) {
            if (q < Hb) load_plane_site<T, PROBE>(inp, IN_Z4, S, ghq + tn * P, hnx);
        }
        __syncthreads();

        if constexpr (OWN) {
            // forward hops with this site's links; backward hops read the
            // products the neighbours x - mu left in LDS
            own_hops<T, 0>(lds, Sl, sxp, sxm, U0, bwl, Pb, acc);
            __builtin_amdgcn_sched_barrier(0);
            own_hops<T, 1>(lds, Sl, syp, sym, Uy, bwl, Pb, acc);
            __builtin_amdgcn_sched_barrier(0);
            own_hops<T, 2>(lds, Sl, szp, szm, Uz, bwl, Pb, acc);
            __builtin_amdgcn_sched_barrier(0);
            // +t hop: (1 - g_t) U_t(x, t) w(x, t+1), the stash's link
            C h[2][3];
            proj<T, 3, true>(nxt, h);
            mul_link<T, false>(Ust, h);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) h[sp][aa] = mk<T>(sg * h[sp][aa].x, sg * h[sp][aa].y);
            recon<T, 3, true>(h, acc);
        } else if constexpr (sizeof(T) == 4 && !FIRST) {
            // FP32 after the first step: the link of each hop is loaded one hop
            // ahead (the +t link during the -z hop), a (+mu, -mu) pair per
            // rolled iteration.  This kernel has the registers for the second
            // link and is bound by instruction issue once the link latency is
            // hidden (measured: 79 -> 69 us per launch at 8^4 x 256 vectors).
            // The FP64 kernel and the first-step kernels have no registers to
            // spare: there the prefetch spills, and FP64 without the spills
            // measured no faster.
            C Ua[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) Ua[e] = U0[e];
#pragma nounroll
            for (int k2 = 0; k2 < 3; ++k2) {
                C Ub[9];
                int qf = k2 == 0 ? sxp : k2 == 1 ? syp : szp;
                int qb = k2 == 0 ? sxm : k2 == 1 ? sym : szm;
                int sb = (k2 == 0 ? gxm : k2 == 1 ? gym : gzm) + t * P;
                const char *gm = opaque_ptr(k2 == 0 ? gx : k2 == 1 ? gy : gz);
                asm volatile("" : "+v"(qf), "+v"(qb), "+v"(sb));
                link_raw<T, TWO>(gm, estride, sb, Ub);
                link_complete<T, TWO>(Ua);
                switch (k2) {
                case 0: plane_hop_u<T, 0, true>(lds, Sl, qf, Ua, acc); break;
                case 1: plane_hop_u<T, 1, true>(lds, Sl, qf, Ua, acc); break;
                default: plane_hop_u<T, 2, true>(lds, Sl, qf, Ua, acc); break;
                }
                int sn = s;
                const char *gn = opaque_ptr(k2 == 0 ? gy : k2 == 1 ? gz : gt);
                asm volatile("" : "+v"(sn));
                link_raw<T, TWO>(gn, estride, sn, Ua);
                link_complete<T, TWO>(Ub);
                switch (k2) {
                case 0: plane_hop_u<T, 0, false>(lds, Sl, qb, Ub, acc); break;
                case 1: plane_hop_u<T, 1, false>(lds, Sl, qb, Ub, acc); break;
                default: plane_hop_u<T, 2, false>(lds, Sl, qb, Ub, acc); break;
                }
            }
            // +t hop: (1 - g_t) U_t(x, t) w(x, t+1), its link already in Ua
            link_complete<T, TWO>(Ua);
            C h[2][3];
            proj<T, 3, true>(nxt, h);
            mul_link<T, false>(Ua, h);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) h[sp][aa] = mk<T>(sg * h[sp][aa].x, sg * h[sp][aa].y);
            recon<T, 3, true>(h, acc);
        } else {
        // The six spatial hops in sequence, with scheduling barriers between
        // them so that the compiler cannot interleave them (which bounds the
        // live registers).  Unrolled they cost no loop overhead: a rolled loop
        // over a switch spent ~230 of ~1750 instructions per site and step on
        // dispatch and on copying the accumulator (83 -> 77 us at 64 vectors).
        link_complete<T, TWO>(U0);
        plane_hop_u<T, 0, true>(lds, Sl, sxp, U0, acc);
        __builtin_amdgcn_sched_barrier(0);
        plane_hop<T, 0, false>(lds, Sl, sxm, gx, estride, gxm + t * P, two, acc);
        __builtin_amdgcn_sched_barrier(0);
        plane_hop<T, 1, true>(lds, Sl, syp, gy, estride, s, two, acc);
        __builtin_amdgcn_sched_barrier(0);
        plane_hop<T, 1, false>(lds, Sl, sym, gy, estride, gym + t * P, two, acc);
        __builtin_amdgcn_sched_barrier(0);
        plane_hop<T, 2, true>(lds, Sl, szp, gz, estride, s, two, acc);
        __builtin_amdgcn_sched_barrier(0);
        plane_hop<T, 2, false>(lds, Sl, szm, gz, estride, gzm + t * P, two, acc);
        __builtin_amdgcn_sched_barrier(0);
        // +t hop: (1 - g_t) U_t(x, t) w(x, t+1)
        {
            C U[9];
            int ss = s;
            asm volatile("" : "+v"(ss));
            load_link<T>(gt, estride, ss, two, U);
            C h[2][3];
            proj<T, 3, true>(nxt, h);
            mul_link<T, false>(U, h);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) h[sp][aa] = mk<T>(sg * h[sp][aa].x, sg * h[sp][aa].y);
            recon<T, 3, true>(h, acc);
        }
        }
        // the next step's -t link ahead of the stores (the site clamped on the
        // last step: a conditional load here made the compiler spill)
        link_raw<T, TWOL>(gt, estride, t + 1 < Lt ? s + P : s, Ust);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            acc[c] = cmul_d<T>(beta, acc[c]);
            outp.st(c, s, acc[c]);
        }
        if (DOT) {
            C b[12];
            if (!BFIELD) {
                noise_site<T, PROBE>(S, s, b);
            } else {
                const Plane<T> bp = plane_of<T>(a.bvec, r, a.V, a.rb_b);
#pragma unroll
                for (int c = 0; c < 12; ++c) b[c] = bp.ld(c, s);
            }
            dot_acc<T>(b, acc, dre, dim);
        }
        if constexpr (YACC) {
            // y += t_j w_j (+ t_{j+1} w_{j+1} after the last step); w_j is still
            // this site's entry of the LDS plane, so it costs no registers
            const Plane<T> yp = plane_of<T>(a.y, r, a.V, 1);
            const double2 tn = a.y_last ? a.troots[a.j + 1] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                C yv = a.y_first ? mk<T>(T(0), T(0)) : yp.ld(c, s);
                yv = axpy_d<T>(tj, lds[c * Sl + q], yv);
                if (a.y_last) yv = axpy_d<T>(tn, acc[c], yv);
                yp.st(c, s, yv);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 12; ++c) cur[c] = nxt[c];
        if constexpr (HALO) {
            if (q < Hb) {
#pragma unroll
                for (int c = 0; c < 12; ++c) hcur[c] = hnx[c];
            }
        }
    }

    if (DOT) sweep_dot_finish<T, FIRST, HALO>(a, r, pidx, q, Pb, tj, dre, dim, d0re, d0im, smem);
}

// b^H y of a blocked or t-chunked sweep: the (t-chunk, block) partials of each
// vector in a fixed order
__global__ void k_sweep_sum(const double2 *part, int nbp, int nrhs, double2 *bhy) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= nrhs) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nbp; ++b) {
        re += part[(size_t)r * nbp + b].x;
        im += part[(size_t)r * nbp + b].y;
    }
    bhy[r] = make_double2(re, im);
}

// ------------------------------------------------------------------ host side

SweepPlan sweep_plan(const mpmc_lattice &lat, mpmc_shape sh) {
    SweepPlan p;
    const int Lx = lat.dims[0], Ly = lat.dims[1], Lz = lat.dims[2], Lt = lat.dims[3];
    const int P = Lx * Ly * Lz;
    const size_t csz = lat.prec == MPMC_F64 ? 16 : 8;
    const size_t V = (size_t)P * (size_t)Lt;
    if (36 * V * csz >= ((size_t)1 << 32)) return p;          // 32-bit link offsets
    const size_t kLds = 160 * 1024;
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return p;
    if (!cus[dev] && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return p;
    const size_t min_threads = (size_t)cus[dev] * 512;
    // partial sums the polynomial workspace holds
    const size_t avail = poly_part_count(V, sh.nrhs, sh.rb);
    // t-chunks.  A workgroup walks the Lt / k planes of its chunk, starting
    // from a prologue that forms the -t term of its first plane from the
    // plane before, so k chunks give k times the workgroups for one more plane
    // read per chunk.  Of the k that divide Lt (chunks of at least min_len
    // planes, partial sums within the workspace), the plan takes the one with
    // the least modelled time, rounds of workgroups (C at a time) times
    // (planes per chunk + 2), among those whose launch gives every CU a
    // workgroup; if none does, the sweep is not worth its launch (`fill`
    // false) and the cheapest k is kept for callers that force it.  Measured
    // per launch (FP32 unless noted; sweep with k chunks against streaming):
    // 8^4 x 64 vectors k = 1 / 2 / 4: 56.7 / 33.6 / 23.7 us, streaming 32.5
    // (FP64 74.9 / 45.0 / 36.1, streaming 52.6); 16^4 x 16 k = 2 / 4 / 8:
    // 86.3 / 96.0 / 112.4, streaming 112.2; 24^3x48 x 32 k = 1 / 2 / 4:
    // 2059 / 1916 / 1970, streaming 2032; 8^4 x 256 k = 1 / 2 / 4: 67.1 /
    // 73.2 / 82.1, streaming 109.9.
    struct Chunks {
        int k;
        bool fill;
    };
    auto chunks = [&](size_t W, size_t C, int min_len) {
        if (g_opt_sweep_chunks > 0) {
            const size_t f = (size_t)g_opt_sweep_chunks;
            const size_t k = (Lt % g_opt_sweep_chunks == 0 && W * f <= avail) ? f : 1;
            return Chunks{(int)k, W * k >= C};
        }
        Chunks best{1, W >= C}, any{1, W >= C};
        double tbest = 1e300, tany = 1e300;
        for (int k = 1; k <= Lt; ++k) {
            if (Lt % k || (k > 1 && Lt / k < min_len) || W * (size_t)k > avail) continue;
            const double t = (double)((W * (size_t)k + C - 1) / C) * (double)(Lt / k + 2);
            if (t < tany) {
                tany = t;
                any = Chunks{k, W * (size_t)k >= C};
            }
            if (W * (size_t)k >= C && t < tbest) {
                tbest = t;
                best = Chunks{k, true};
            }
        }
        return tbest < 1e300 ? best : any;
    };
    // A whole-plane sweep runs one workgroup per (vector, t-chunk) for the
    // whole launch, so a launch that leaves CUs idle takes about as long as
    // one that does not, while the streaming kernel's time grows with the
    // vectors: the sweep applies when its workgroups, chunked, cover the CUs
    // (one per CU: the LDS holds one plane).
    const size_t whole = (lat.prec == MPMC_F32 ? 36 : 18) * (size_t)P * csz;
    if (P >= 64 && P <= 512 && P % 64 == 0 && whole <= kLds) {
        // the whole xyz-plane in one workgroup (neighbours wrap inside it)
        const Chunks c = chunks((size_t)sh.nrhs, (size_t)cus[dev], 2);
        p.nch = c.k;
        p.busy = c.fill;
        p.fills = (size_t)sh.nrhs * (size_t)P * (size_t)c.k >= min_threads;
        p.ok = true;
        p.B[0] = Lx;
        p.B[1] = Ly;
        p.B[2] = Lz;
        p.Pb = P;
        p.lds = whole;
        return p;
    }
    if (lat.prec != MPMC_F32) return p;                        // FP64 blocks + halo exceed the registers
    // A blocked sweep pays only when its launch, chunked in t (chunks of at
    // least 4 planes), gives every CU a workgroup; small batches on large
    // planes stay on the streaming kernel (12^3x24 x 8 vectors would need
    // 2-plane chunks: 48.2 us per launch against 42.6 streaming).
    // Sites are x-fastest over the whole lattice, so a block reads and writes
    // its rows (and its halo rows, and its links) bx sites at a time: whole
    // 128-byte lines only when bx spans the x extent or a multiple of a line.
    // The plan minimises the input bytes per block site over the compulsory
    // ones, (1 + halo / block sites) / line efficiency, then takes the larger
    // block, then the one longer in y (measured: 4x8x16 -> 16x4x8 blocks of
    // 16^3 planes 1.2 -> 2.8 TB/s, 8x8x8 -> 24x4x4 of 24^3 planes 1.8 -> 2.2
    // TB/s; of the equal-cost 16x4x8 and 16x8x4, the latter is 5% faster on
    // 16^4 x 16 vectors and 0-1% on 16^3x32).  The candidates are
    // ranked by that cost; the kernel-selection option MPMC_OPT_SWEEP_RANK
    // picks a lower-ranked block (the autotuner times a few).
    auto cost = [&](int bx, int Pb, int Hb) {
        const double row = (double)bx * (double)csz;
        const double eff = bx == Lx ? 1.0 : row / (128.0 * std::ceil(row / 128.0));
        return (1.0 + (double)Hb / (double)Pb) / eff;
    };
    struct Cand {
        double cost;
        int bx, by, bz, Pb, Hb;
        size_t lds;
    };
    Cand cands[64];
    int nc = 0;
    for (int bx = 1; bx <= Lx; ++bx) {
        if (Lx % bx) continue;
        for (int by = 1; by <= Ly; ++by) {
            if (Ly % by) continue;
            for (int bz = 1; bz <= Lz; ++bz) {
                if (Lz % bz) continue;
                const int Pb = bx * by * bz;
                if (Pb < 64 || Pb > 512 || Pb % 64) continue;
                const int Hb = 2 * ((bx < Lx ? by * bz : 0) + (by < Ly ? bx * bz : 0) + (bz < Lz ? bx * by : 0));
                if (Hb > Pb) continue;                          // one halo site per thread at most
                const size_t lds = (12 * (size_t)(Pb + Hb) + 6 * (size_t)Pb) * csz;
                if (lds > kLds) continue;
                if ((size_t)sh.nrhs * (size_t)(P / Pb) > avail) continue;
                const Cand c{cost(bx, Pb, Hb), bx, by, bz, Pb, Hb, lds};
                // keep the 64 best by (cost, larger block, longer y extent first), insertion-sorted
                int at = nc < 64 ? nc : 64;
                while (at > 0 && (c.cost < cands[at - 1].cost - 1e-9 ||
                                  (c.cost < cands[at - 1].cost + 1e-9 &&
                                   (c.Pb > cands[at - 1].Pb || (c.Pb == cands[at - 1].Pb && c.by > cands[at - 1].by)))))
                    --at;
                if (at >= 64) continue;
                for (int m = (nc < 64 ? nc : 63); m > at; --m) cands[m] = cands[m - 1];
                cands[at] = c;
                if (nc < 64) ++nc;
            }
        }
    }
    if (nc == 0) return p;
    // the plan's choice is the cheapest block; a tuner may ask for the rank-th (clamped)
    const Cand &c = cands[g_opt_sweep_rank < nc ? g_opt_sweep_rank : nc - 1];
    p.ok = true;
    p.halo = true;
    p.busy = true;    // blocked planes take the sweep only when the batch fills the GPU (above)
    p.B[0] = c.bx;
    p.B[1] = c.by;
    p.B[2] = c.bz;
    p.Pb = c.Pb;
    p.Hb = c.Hb;
    p.nbp = P / c.Pb;
    // workgroups resident per CU: the LDS's limit and two waves per SIMD
    // (the kernels take over 128 VGPRs)
    const size_t wpc = std::max<size_t>(1, std::min<size_t>(kLds / c.lds, 512 / (size_t)c.Pb));
    const Chunks ck = chunks((size_t)sh.nrhs * (size_t)p.nbp, (size_t)cus[dev] * wpc, 4);
    if (!ck.fill) {
        p.ok = false;
        p.halo = false;
        return p;
    }
    p.nch = ck.k;
    p.fills = true;
    p.lds = c.lds;
    p.nranked = nc;
    return p;
}

// kernel of one launch: v = 0 noise input (first step), 1 field input (first
// step), 2 a later step; dot: accumulate b^H w partials (b the noise, or the
// field bvec when bf); yacc: vector mode.  Blocks with a halo are FP32 only;
// vector mode has no field dot vector.
template <typename T, bool Y, bool D, bool BF, bool TW, bool H> static const void *sweep_kernel_v(int v) {
    if (v == 0) return (const void *)k_sweep<T, true, D, true, BF, TW, H, Y>;
    if (v == 1) return (const void *)k_sweep<T, false, D, true, BF, TW, H, Y>;
    return (const void *)k_sweep<T, false, D, false, BF, TW, H, Y>;
}
template <typename T, bool Y, bool D, bool BF> static const void *sweep_kernel_h(bool tw, bool h, int v) {
    if (h) {
        if constexpr (sizeof(T) == 4)
            return tw ? sweep_kernel_v<T, Y, D, BF, true, true>(v) : sweep_kernel_v<T, Y, D, BF, false, true>(v);
        return nullptr;
    }
    return tw ? sweep_kernel_v<T, Y, D, BF, true, false>(v) : sweep_kernel_v<T, Y, D, BF, false, false>(v);
}
// probe vectors instead of Z4 noise: scalar mode, noise input (first step) or later steps
template <typename T, bool TW, bool H> static const void *sweep_probe_v(int v) {
    if (v == 0) return (const void *)k_sweep<T, true, true, true, false, TW, H, false, true>;
    if (v == 2) return (const void *)k_sweep<T, false, true, false, false, TW, H, false, true>;
    return nullptr;
}
template <typename T> static const void *sweep_probe_kernel(bool tw, bool h, int v) {
    if (h) {
        if constexpr (sizeof(T) == 4) return tw ? sweep_probe_v<T, true, true>(v) : sweep_probe_v<T, false, true>(v);
        return nullptr;
    }
    return tw ? sweep_probe_v<T, true, false>(v) : sweep_probe_v<T, false, false>(v);
}
template <typename T> static const void *sweep_kernel(bool yacc, bool dot, bool bf, bool tw, bool h, int v) {
    if (!dot && !yacc && v < 2) return nullptr;   // the plain chain has no first-step variants
    if (yacc) {
        if (bf) return nullptr;
        return dot ? sweep_kernel_h<T, true, true, false>(tw, h, v) : sweep_kernel_h<T, true, false, false>(tw, h, v);
    }
    if (!dot) return bf ? nullptr : sweep_kernel_h<T, false, false, false>(tw, h, v);
    return bf ? sweep_kernel_h<T, false, true, true>(tw, h, v) : sweep_kernel_h<T, false, true, false>(tw, h, v);
}
// the kernels use up to 160 KB of dynamic LDS: allowed once per kernel
static int ensure_lds_attr(const void *k) {
    static const void *done[256];
    static int ndone = 0;
    for (int i = 0; i < ndone; ++i)
        if (done[i] == k) return MPMC_OK;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) return MPMC_EHIP;
    if (ndone < 256) done[ndone++] = k;
    return MPMC_OK;
}

template <typename T> static int prepare_kernels_t() {
    for (int m = 0; m < 2 * 2 * 2 * 2 * 2 * 3; ++m) {
        const int v = m % 3, h = (m / 3) % 2, tw = (m / 6) % 2, bf = (m / 12) % 2, d = (m / 24) % 2, y = m / 48;
        const void *k = sweep_kernel<T>(y, d, bf, tw, h, v);
        if (k && ensure_lds_attr(k) != MPMC_OK) return MPMC_EHIP;
        const void *kp = (y || bf || !d) ? nullptr : sweep_probe_kernel<T>(tw, h, v);
        if (kp && ensure_lds_attr(kp) != MPMC_OK) return MPMC_EHIP;
    }
    return MPMC_OK;
}

// Sets the dynamic-LDS limit of every t-sweep kernel up front, so that work
// captured into a HIP graph makes no attribute calls.
int sweep_prepare_kernels() {
    const int st = prepare_kernels_t<double>();
    return st != MPMC_OK ? st : prepare_kernels_t<float>();
}

template <typename T>
static SweepArgs<T> sweep_args(const mpmc_lattice &lat, const SweepPlan &plan, const double *troots) {
    SweepArgs<T> a{};
    for (int d = 0; d < 4; ++d) a.L[d] = lat.dims[d];
    a.P = lat.dims[0] * lat.dims[1] * lat.dims[2];
    a.V = a.P * lat.dims[3];
    a.apbc = lat.antiperiodic_t;
    a.gauge = (const cplx_t<T> *)lat.gauge;
    a.two_rows = lat.link_rows == 2;
    a.troots = (const double2 *)troots;
    a.kappa = lat.kappa;
    for (int d = 0; d < 3; ++d) a.B[d] = plan.B[d];
    a.Pb = plan.Pb;
    a.Hb = plan.Hb;
    a.nbp = plan.nbp;
    a.nch = plan.nch;
    return a;
}

template <typename T>
int sweep_newton_t(const mpmc_lattice &lat, mpmc_shape sh, const SweepPlan &plan, int n, const double *troots,
                   const void *x, bool x_is_noise, const void *bvec, uint64_t key, uint64_t first, const uint64_t *off,
                   double2 *part, double2 *bhy, void *w0, void *w1, void *yacc, void *stream,
                   const int32_t *colour) {
    SweepArgs<T> a = sweep_args<T>(lat, plan, troots);
    a.colour = colour;
    a.key = key;
    a.first = first;
    a.off = off;
    a.bvec = (const cplx_t<T> *)bvec;
    a.rb_b = sh.rb;
    a.part = part;
    a.y = (cplx_t<T> *)yacc;
    const bool h = plan.halo, tw = lat.link_rows == 2, bf = bvec != nullptr, dot = bhy != nullptr;
    const bool y = yacc != nullptr;
    if (!dot && !y) return MPMC_EINVAL;
    const int d = n - 1;
    const dim3 grid((unsigned)(sh.nrhs * plan.nbp * plan.nch)), block((unsigned)plan.Pb);
    // b^H y straight from the kernel only when one workgroup covers a vector
    const bool sum_after = plan.halo || plan.nch > 1;
    for (int j = 0; j < d; ++j) {
        a.j = j;
        const bool first_step = (j == 0);
        a.in = (const cplx_t<T> *)(first_step ? x : (((j - 1) % 2 == 0) ? w0 : w1));
        a.rb_in = first_step ? sh.rb : 1;
        a.out = (cplx_t<T> *)(j % 2 == 0 ? w0 : w1);
        a.dot_first = first_step;
        a.bhy = (j == d - 1 && !sum_after) ? bhy : nullptr;
        a.y_first = first_step;
        a.y_last = (j == d - 1);
        const int v = first_step ? (x_is_noise ? 0 : 1) : 2;
        const void *k = colour ? ((y || bf || !dot) ? nullptr : sweep_probe_kernel<T>(tw, h, v))
                               : sweep_kernel<T>(y, dot, bf, tw, h, v);
        if (!k) return MPMC_EUNSUPPORTED;
        if (ensure_lds_attr(k) != MPMC_OK) return MPMC_EHIP;
        void *args[] = {&a};
        if (hipLaunchKernel(k, grid, block, args, plan.lds, (hipStream_t)stream) != hipSuccess) return MPMC_EHIP;
        if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    }
    if (sum_after && bhy) {
        hipLaunchKernelGGL(k_sweep_sum, dim3((sh.nrhs + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)part, plan.nbp * plan.nch, sh.nrhs, bhy);
        if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    }
    return MPMC_OK;
}

template <typename T>
int sweep_chain_t(const mpmc_lattice &lat, mpmc_shape sh, const SweepPlan &plan, int count, const double *troots,
                  const void *in, int rb_in, void *w0, void *w1, const void **out, void *stream) {
    *out = in;
    if (count <= 0) return MPMC_OK;
    SweepArgs<T> a = sweep_args<T>(lat, plan, troots);
    const void *k = sweep_kernel<T>(false, false, false, lat.link_rows == 2, plan.halo, 2);
    if (!k) return MPMC_EUNSUPPORTED;
    if (ensure_lds_attr(k) != MPMC_OK) return MPMC_EHIP;
    const dim3 grid((unsigned)(sh.nrhs * plan.nbp * plan.nch)), block((unsigned)plan.Pb);
    const void *cur = in;
    for (int j = 0; j < count; ++j) {
        a.j = j;
        a.in = (const cplx_t<T> *)cur;
        a.rb_in = j == 0 ? rb_in : 1;
        void *o = (j % 2 == 0) ? w0 : w1;
        a.out = (cplx_t<T> *)o;
        void *args[] = {&a};
        if (hipLaunchKernel(k, grid, block, args, plan.lds, (hipStream_t)stream) != hipSuccess) return MPMC_EHIP;
        if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
        cur = o;
    }
    *out = cur;
    return MPMC_OK;
}

template int sweep_chain_t<double>(const mpmc_lattice &, mpmc_shape, const SweepPlan &, int, const double *,
                                   const void *, int, void *, void *, const void **, void *);
template int sweep_chain_t<float>(const mpmc_lattice &, mpmc_shape, const SweepPlan &, int, const double *,
                                  const void *, int, void *, void *, const void **, void *);

template int sweep_newton_t<double>(const mpmc_lattice &, mpmc_shape, const SweepPlan &, int, const double *,
                                    const void *, bool, const void *, uint64_t, uint64_t, const uint64_t *, double2 *,
                                    double2 *, void *, void *, void *, void *, const int32_t *);
template int sweep_newton_t<float>(const mpmc_lattice &, mpmc_shape, const SweepPlan &, int, const double *,
                                   const void *, bool, const void *, uint64_t, uint64_t, const uint64_t *, double2 *,
                                   double2 *, void *, void *, void *, void *, const int32_t *);

}  // namespace mpmc
