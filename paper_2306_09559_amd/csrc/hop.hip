// Multi-RHS Wilson-Dirac hopping kernel and the polynomial drivers built on it.
//
// One thread owns one (site, vector) pair and produces all 12 unknowns of
// that site.  Each of the 8 neighbours is spin-projected to a half spinor
// (2 spins x 3 colours) before the SU(3) product, then reconstructed; the
// projector algebra below is that of the DeGrand-Rossi gamma matrices.
// A workgroup covers 256/rb consecutive sites of one RHS block, lanes
// walking the rb vectors of a site fastest, so every field access of a
// wavefront is one contiguous run and the links of a site are shared by its
// rb lanes.  Workgroups are remapped so each XCD sweeps a contiguous range
// of tiles (its L2 then holds the neighbours).
//
// The same kernel body serves every operator application of the hot path:
//   out = alpha * in + beta * D in  (+ b)            D = hopping term
// with (alpha, beta) = (1, -kappa) for A itself, (1 - t, kappa t) for a
// Newton / product-chain step w -> w - t A w (Sec. 3.1), (-1, kappa) plus b
// for the projected residual b - A x (Sec. 2.1 step 4), and optional fused
// epilogues: the Newton accumulator y += t w, the FP64 partial of b^H w,
// and the outer Newton update of the composite polynomial (Sec. 3.2).
#include "common.hpp"
#include "internal.hpp"

namespace mpmc {

template <typename T> struct HopArgs {
    Geo g;
    int rb, spw, nblk;
    unsigned G;                 // workgroups of the launch
    // work order (see hop_tile): slab = 1 when each XCD sweeps t over its own
    // z-slab of the xyz-plane: tps tiles per xyz-plane, chunk of them per XCD
    int slab, tps, chunk;
    const cplx_t<T> *in;        // input field; unused when the input is noise
    cplx_t<T> *out;
    const cplx_t<T> *gauge;     // [mu][9][V]
    int two_rows;               // links special unitary: row 2 rebuilt from rows 0, 1
    int gbuf;                   // the links take buffer loads (whole array below 4 GiB)
    // step coefficients: t = troots[j] if troots, else (alpha, beta) given
    const double2 *troots;
    int j;
    double kappa;
    double2 alpha, beta;
    // noise (input when IN_Z4, dot/add vector when bvec == nullptr)
    uint64_t key, first;
    const uint64_t *off;       // device sample counter added to first, or nullptr
    const cplx_t<T> *bvec;
    // Newton accumulator y (YACC)
    cplx_t<T> *y;
    int y_first, y_last;
    // dot partials (DOT): part[L*rb + lane] accumulates sum_j t_j b^H w_j
    double2 *part;
    int dot_first;
    // composite outer step (OUTER): u_next = (1-phi) u + phi * out
    const cplx_t<T> *u;
    cplx_t<T> *u_next;
    const double2 *phi;
    int jo, jo_last;
};

namespace {

template <typename T> struct Half { cplx_t<T> h[2][3]; };

// A field restricted to one RHS block: component c of the thread's vector at
// site s lives at base + c*cstride + (s*rb + j)*sizeof(C).  base and cstride
// are wavefront-uniform (scalar registers); the per-site byte offset fits in
// 32 bits because V*rb*sizeof(C) < 4 GiB is checked on the host.
template <typename T> struct Blk {
    const char *base;
    size_t cstride;
    __device__ __forceinline__ cplx_t<T> ld(int c, uint32_t off) const {
        return *(const cplx_t<T> *)(base + (size_t)c * cstride + off);
    }
    // outputs are read again only by the next launch: stream them past L2
    __device__ __forceinline__ void st(int c, uint32_t off, cplx_t<T> v) const {
        T *p = (T *)(const_cast<char *>(base) + (size_t)c * cstride + off);
        __builtin_nontemporal_store(v.x, p);
        __builtin_nontemporal_store(v.y, p + 1);
    }
};

template <typename T> __device__ __forceinline__ Blk<T> blk(const void *f, int nbk, int V, int rb) {
    Blk<T> b;
    b.cstride = (size_t)V * (size_t)rb * sizeof(cplx_t<T>);
    b.base = (const char *)f + (size_t)nbk * 12 * b.cstride;
    return b;
}

// byte offset of (site s, lane j) inside a component plane
template <typename T> __device__ __forceinline__ uint32_t site_off(int s, int rb, int j) {
    return (uint32_t)(s * rb + j) * (uint32_t)sizeof(cplx_t<T>);
}

template <typename T>
__device__ __forceinline__ void load_site(const Blk<T> &in, int rb, int jr, bool z4, uint64_t S, int s, T sign,
                                          cplx_t<T> (&p)[12]) {
    if (z4) {
        const uint32_t codes = z4_site_codes(S, (unsigned)s);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            cplx_t<T> v = z4_value<T>((codes >> (2 * c)) & 3u);
            p[c] = mk<T>(sign * v.x, sign * v.y);
        }
    } else {
        const uint32_t off = site_off<T>(s, rb, jr);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            cplx_t<T> v = in.ld(c, off);
            p[c] = mk<T>(sign * v.x, sign * v.y);
        }
    }
}

// (1 - g_mu) psi  (FWD) or (1 + g_mu) psi (!FWD) as a half spinor (spins 0, 1)
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void project(const cplx_t<T> (&p)[12], cplx_t<T> (&h)[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx_t<T> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
        if (MU == 0) {        // g1: h0 = p0 -+ i p3, h1 = p1 -+ i p2
            h[0][a] = FWD ? cadd<T>(p0, mul_mi<T>(p3)) : cadd<T>(p0, mul_i<T>(p3));
            h[1][a] = FWD ? cadd<T>(p1, mul_mi<T>(p2)) : cadd<T>(p1, mul_i<T>(p2));
        } else if (MU == 1) { // g2: h0 = p0 +- p3, h1 = p1 -+ p2
            h[0][a] = FWD ? cadd<T>(p0, p3) : csub<T>(p0, p3);
            h[1][a] = FWD ? csub<T>(p1, p2) : cadd<T>(p1, p2);
        } else if (MU == 2) { // g3: h0 = p0 -+ i p2, h1 = p1 +- i p3
            h[0][a] = FWD ? cadd<T>(p0, mul_mi<T>(p2)) : cadd<T>(p0, mul_i<T>(p2));
            h[1][a] = FWD ? cadd<T>(p1, mul_i<T>(p3)) : cadd<T>(p1, mul_mi<T>(p3));
        } else {              // g4: h0 = p0 -+ p2, h1 = p1 -+ p3
            h[0][a] = FWD ? csub<T>(p0, p2) : cadd<T>(p0, p2);
            h[1][a] = FWD ? csub<T>(p1, p3) : cadd<T>(p1, p3);
        }
    }
}

// accumulate the reconstructed 4-spinor of the (colour-rotated) half spinor
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void reconstruct(const cplx_t<T> (&h)[2][3], cplx_t<T> (&acc)[12]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx_t<T> h0 = h[0][a], h1 = h[1][a];
        acc[a] = cadd<T>(acc[a], h0);
        acc[3 + a] = cadd<T>(acc[3 + a], h1);
        cplx_t<T> r2, r3;
        if (MU == 0) {        // (1-g1): r2 = i h1, r3 = i h0 ; (1+g1): -i h1, -i h0
            r2 = FWD ? mul_i<T>(h1) : mul_mi<T>(h1);
            r3 = FWD ? mul_i<T>(h0) : mul_mi<T>(h0);
        } else if (MU == 1) { // (1-g2): r2 = -h1, r3 = h0 ; (1+g2): h1, -h0
            r2 = FWD ? mk<T>(-h1.x, -h1.y) : h1;
            r3 = FWD ? h0 : mk<T>(-h0.x, -h0.y);
        } else if (MU == 2) { // (1-g3): r2 = i h0, r3 = -i h1 ; (1+g3): -i h0, i h1
            r2 = FWD ? mul_i<T>(h0) : mul_mi<T>(h0);
            r3 = FWD ? mul_mi<T>(h1) : mul_i<T>(h1);
        } else {              // (1-g4): r2 = -h0, r3 = -h1 ; (1+g4): h0, h1
            r2 = FWD ? mk<T>(-h0.x, -h0.y) : h0;
            r3 = FWD ? mk<T>(-h1.x, -h1.y) : h1;
        }
        acc[6 + a] = cadd<T>(acc[6 + a], r2);
        acc[9 + a] = cadd<T>(acc[9 + a], r3);
    }
}

// Links through buffer loads when the link array is below 4 GiB (measured
// on the FP32 kernel: 133.7 -> 116.1 us per launch at 16^4 x 16 vectors,
// 9.16 -> 7.85 ms at 24^3x48 x 128; FP64, and the spinor loads as buffer
// loads too, within 1%).
// h <- U h (FWD, U = U_mu(x)) or h <- U^H h (!FWD, U = U_mu(x - mu))
template <typename T, bool FWD>
__device__ __forceinline__ void su3_mul(const HopArgs<T> &ha, int mu, int site, cplx_t<T> (&h)[2][3]) {
    cplx_t<T> U[9];
    if (ha.gbuf) {
        load_su3_buf<T>(link_buf<T>(ha.gauge, ha.g.V, mu), site, ha.two_rows != 0, U);
    } else {
        const size_t estride = (size_t)ha.g.V * sizeof(cplx_t<T>);
        load_su3<T>((const char *)ha.gauge + (size_t)mu * 9 * estride, estride,
                    (uint32_t)site * (uint32_t)sizeof(cplx_t<T>), ha.two_rows != 0, U);
    }
    cplx_t<T> o[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx_t<T> t = mk<T>(T(0), T(0));
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (FWD) t = cfma<T>(U[3 * a + b], h[sp][b], t);
                else t = cfmaconj<T>(U[3 * b + a], h[sp][b], t);
            }
            o[sp][a] = t;
        }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[sp][a] = o[sp][a];
}

// one neighbour hop: direction MU, forward (x + mu) or backward (x - mu)
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void hop_one(const HopArgs<T> &a, const Blk<T> &in, int jr, bool z4, uint64_t S, int s,
                                        const int (&x)[4], cplx_t<T> (&acc)[12]) {
    const bool wrap = FWD ? (x[MU] == a.g.L[MU] - 1) : (x[MU] == 0);
    const int step = FWD ? a.g.st[MU] : -a.g.st[MU];
    const int nb = wrap ? s - (a.g.L[MU] - 1) * step : s + step;
    const T sign = (MU == 3 && wrap && a.g.apbc) ? T(-1) : T(1);
    cplx_t<T> p[12];
    load_site<T>(in, a.rb, jr, z4, S, nb, sign, p);
    Half<T> h;
    project<T, MU, FWD>(p, h.h);
    // forward: U_mu(x) h ; backward: U_mu(x - mu)^H h
    su3_mul<T, FWD>(a, MU, FWD ? s : nb, h.h);
    reconstruct<T, MU, FWD>(h.h, acc);
}

// both hops of direction MU, the two neighbours' loads issued before either
// is used (FP64, see hop_all)
template <typename T, int MU>
__device__ __forceinline__ void hop_pair(const HopArgs<T> &a, const Blk<T> &in, int jr, bool z4, uint64_t S, int s,
                                         const int (&x)[4], cplx_t<T> (&acc)[12]) {
    const bool wf = x[MU] == a.g.L[MU] - 1, wb = x[MU] == 0;
    const int st = a.g.st[MU];
    const int nf = wf ? s - (a.g.L[MU] - 1) * st : s + st;
    const int nb = wb ? s + (a.g.L[MU] - 1) * st : s - st;
    const T sf = (MU == 3 && wf && a.g.apbc) ? T(-1) : T(1);
    const T sb = (MU == 3 && wb && a.g.apbc) ? T(-1) : T(1);
    cplx_t<T> pf[12], pb[12];
    load_site<T>(in, a.rb, jr, z4, S, nf, sf, pf);
    load_site<T>(in, a.rb, jr, z4, S, nb, sb, pb);
    {
        Half<T> h;
        project<T, MU, true>(pf, h.h);
        su3_mul<T, true>(a, MU, s, h.h);
        reconstruct<T, MU, true>(h.h, acc);
    }
    {
        Half<T> h;
        project<T, MU, false>(pb, h.h);
        su3_mul<T, false>(a, MU, nb, h.h);
        reconstruct<T, MU, false>(h.h, acc);
    }
}

// acc = D psi at site s: the hops run as a rolled loop so that only one
// neighbour's (FP32) or one direction's (FP64) loads and products are live at
// a time (bounded registers); acc is carried in registers.  FP64 takes the
// two hops of a direction per iteration, both neighbours requested together:
// 159 -> 243 VGPRs (3 -> 2 waves per SIMD) and faster all the same (24^3x48 x
// 1 vector 176 -> 159 us per launch, 8^4 x 64 even); FP32 kept one hop per
// iteration (103 -> 144 VGPRs with pairs, 4-8% slower).
template <typename T>
__device__ __forceinline__ void hop_all(const HopArgs<T> &a, const Blk<T> &in, int jr, bool z4, uint64_t S, int s,
                                        const int (&x)[4], cplx_t<T> (&acc)[12]) {
    if constexpr (sizeof(T) == 8) {
#pragma nounroll
        for (int d = 0; d < 4; ++d) {
            // opaque copies of the loop-invariant inputs (see below)
            int sl = s, xl[4] = {x[0], x[1], x[2], x[3]};
            asm volatile("" : "+v"(sl), "+v"(xl[0]), "+v"(xl[1]), "+v"(xl[2]), "+v"(xl[3]));
            Blk<T> il = in;
            il.base = opaque_ptr(il.base);
            switch (d) {
            case 0: hop_pair<T, 0>(a, il, jr, z4, S, sl, xl, acc); break;
            case 1: hop_pair<T, 1>(a, il, jr, z4, S, sl, xl, acc); break;
            case 2: hop_pair<T, 2>(a, il, jr, z4, S, sl, xl, acc); break;
            default: hop_pair<T, 3>(a, il, jr, z4, S, sl, xl, acc); break;
            }
        }
        return;
    }
#pragma nounroll
    for (int d = 0; d < 8; ++d) {
        // Opaque copies of the loop-invariant inputs: without them the
        // compiler hoists every direction's address arithmetic out of the
        // loop and keeps it all live, which defeats the rolled loop.
        int sl = s, xl[4] = {x[0], x[1], x[2], x[3]};
        asm volatile("" : "+v"(sl), "+v"(xl[0]), "+v"(xl[1]), "+v"(xl[2]), "+v"(xl[3]));
        Blk<T> il = in;
        il.base = opaque_ptr(il.base);
        switch (d) {
        case 0: hop_one<T, 0, true>(a, il, jr, z4, S, sl, xl, acc); break;
        case 1: hop_one<T, 0, false>(a, il, jr, z4, S, sl, xl, acc); break;
        case 2: hop_one<T, 1, true>(a, il, jr, z4, S, sl, xl, acc); break;
        case 3: hop_one<T, 1, false>(a, il, jr, z4, S, sl, xl, acc); break;
        case 4: hop_one<T, 2, true>(a, il, jr, z4, S, sl, xl, acc); break;
        case 5: hop_one<T, 2, false>(a, il, jr, z4, S, sl, xl, acc); break;
        case 6: hop_one<T, 3, true>(a, il, jr, z4, S, sl, xl, acc); break;
        default: hop_one<T, 3, false>(a, il, jr, z4, S, sl, xl, acc); break;
        }
    }
}

template <typename T>
__device__ __forceinline__ void get_b(const HopArgs<T> &a, int nbk, int jr, uint64_t S, int s, cplx_t<T> (&b)[12]) {
    if (a.bvec == nullptr) {
        const uint32_t codes = z4_site_codes(S, (unsigned)s);
#pragma unroll
        for (int c = 0; c < 12; ++c) b[c] = z4_value<T>((codes >> (2 * c)) & 3u);
    } else {
        const Blk<T> bb = blk<T>(a.bvec, nbk, a.g.V, a.rb);
        const uint32_t off = site_off<T>(s, a.rb, jr);
#pragma unroll
        for (int c = 0; c < 12; ++c) b[c] = bb.ld(c, off);
    }
}

// sum_c conj(b_c) w_c in FP64
template <typename T>
__device__ __forceinline__ double2 dot12(const cplx_t<T> (&b)[12], const cplx_t<T> (&w)[12]) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double br = (double)b[c].x, bi = (double)b[c].y, wr = (double)w[c].x, wi = (double)w[c].y;
        re += br * wr + bi * wi;
        im += br * wi - bi * wr;
    }
    double2 r;
    r.x = re;
    r.y = im;
    return r;
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    double2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

}  // namespace

// The tile (RHS block nbk, site tile sblk) of hardware workgroup h, and
// whether h has one.  A tile is spw consecutive sites of one RHS block.
// Workgroups are dispatched round-robin over the 8 XCDs, and each XCD works
// through its own ones in order.  With slab = 1 the tiles of each xyz-plane
// are cut into 8 chunks (a z-slab each) and XCD x walks t = 0, 1, .. over its
// chunk, so the +-t neighbours of the sites it runs were read just before (or
// are read just after) by the same XCD and hit its L2; only the slab's two
// z-faces come from another XCD.  (A plain range of tiles in site order per
// XCD, the order without slab, evicts the t-neighbours: they are a whole
// xyz-plane of reads apart.)
template <typename T>
__device__ __forceinline__ bool hop_tile(const HopArgs<T> &a, unsigned h, int &nbk, int &sblk) {
    if (!a.slab) {
        const unsigned L = xcd_remap(h, a.G);
        nbk = (int)(L / (unsigned)a.nblk);
        sblk = (int)(L % (unsigned)a.nblk);
        return true;
    }
    const unsigned x = h % kXcds, k = h / kXcds;
    const unsigned per_t = (unsigned)a.chunk, per_blk = (unsigned)a.g.L[3] * per_t;
    nbk = (int)(k / per_blk);
    const unsigned rem = k % per_blk;
    const int t = (int)(rem / per_t);
    const int tile = (int)(x * per_t + rem % per_t);
    sblk = t * a.tps + tile;
    return tile < a.tps;
}

template <typename T, bool IN_Z4, bool DOT, bool YACC, bool OUTER, bool ADDB>
__global__ void __launch_bounds__(kBlock) k_hop(HopArgs<T> a) {
    using C = cplx_t<T>;
    __shared__ double2 red[DOT ? kBlock : 1];
    int nbk, sblk;
    if (!hop_tile<T>(a, blockIdx.x, nbk, sblk)) return;    // a padding workgroup (uniform)
    const unsigned L = (unsigned)nbk * (unsigned)a.nblk + (unsigned)sblk;
    const int lane = (int)threadIdx.x;
    const int jr = lane & (a.rb - 1), ls = lane / a.rb;
    const int s = sblk * a.spw + ls;
    const bool valid = s < a.g.V;
    const uint64_t r_global = sample_base(a.first, a.off) + (uint64_t)(nbk * a.rb + jr);
    const Blk<T> in = blk<T>(a.in, nbk, a.g.V, a.rb);

    // step coefficients
    // step coefficients, kept in FP64 (applied through cmul_d / lin2_d)
    double2 alpha, beta;
    double2 t_cur;
    t_cur.x = 0.0;
    t_cur.y = 0.0;
    if (a.troots != nullptr) {
        t_cur = a.troots[a.j];
        alpha = make_double2(1.0 - t_cur.x, -t_cur.y);
        beta = make_double2(a.kappa * t_cur.x, a.kappa * t_cur.y);
    } else {
        alpha = a.alpha;
        beta = a.beta;
    }

    double2 contrib;
    contrib.x = 0.0;
    contrib.y = 0.0;
    if (valid) {
        const uint64_t S = (IN_Z4 || ((DOT || ADDB) && a.bvec == nullptr)) ? sample_state(a.key, r_global) : 0ull;
        int x[4];
        {
            int r = s;
            x[0] = r % a.g.L[0];
            r /= a.g.L[0];
            x[1] = r % a.g.L[1];
            r /= a.g.L[1];
            x[2] = r % a.g.L[2];
            x[3] = r / a.g.L[2];
        }
        C acc[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = mk<T>(T(0), T(0));
        hop_all<T>(a, in, jr, IN_Z4, S, s, x, acc);

        const uint32_t off = site_off<T>(s, a.rb, jr);
        C w[12];
        load_site<T>(in, a.rb, jr, IN_Z4, S, s, T(1), w);
        C o[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = lin2_d<T>(alpha, w[c], beta, acc[c]);
        if (ADDB) {
            C b[12];
            get_b<T>(a, nbk, jr, S, s, b);
#pragma unroll
            for (int c = 0; c < 12; ++c) o[c] = cadd<T>(o[c], b[c]);
        }
        if (OUTER) {
            // composite: u_next = (1 - phi) u + phi * pi_in(A) u ; y (+)= phi u [+ phi' u_next]
            const Blk<T> u = blk<T>(a.u, nbk, a.g.V, a.rb);
            const Blk<T> un = blk<T>(a.u_next, nbk, a.g.V, a.rb);
            const Blk<T> y = blk<T>(a.y, nbk, a.g.V, a.rb);
            const double2 ph = a.phi[a.jo];
            const double2 omp = make_double2(1.0 - ph.x, -ph.y);
            const double2 p2 = a.jo_last ? a.phi[a.jo + 1] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const C uo = u.ld(c, off);
                const C unew = lin2_d<T>(ph, o[c], omp, uo);
                un.st(c, off, unew);
                C yv = a.y_first ? mk<T>(T(0), T(0)) : y.ld(c, off);
                yv = axpy_d<T>(ph, uo, yv);
                if (a.jo_last) yv = axpy_d<T>(p2, unew, yv);
                y.st(c, off, yv);
            }
        } else {
            const Blk<T> out = blk<T>(a.out, nbk, a.g.V, a.rb);
#pragma unroll
            for (int c = 0; c < 12; ++c) out.st(c, off, o[c]);
            if (YACC) {
                const Blk<T> y = blk<T>(a.y, nbk, a.g.V, a.rb);
                const double2 tn = a.y_last ? a.troots[a.j + 1] : make_double2(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    C yv = a.y_first ? mk<T>(T(0), T(0)) : y.ld(c, off);
                    yv = axpy_d<T>(t_cur, w[c], yv);
                    if (a.y_last) yv = axpy_d<T>(tn, o[c], yv);
                    y.st(c, off, yv);
                }
            }
            if (DOT) {
                C b[12];
                get_b<T>(a, nbk, jr, S, s, b);
                contrib = zmul(a.troots[a.j + 1], dot12<T>(b, o));
                if (a.dot_first) {
                    const double2 d0 = zmul(t_cur, dot12<T>(b, w));
                    contrib.x += d0.x;
                    contrib.y += d0.y;
                }
            }
        }
    }
    if (DOT) {
        // fixed-order tree over the sites of the workgroup, per vector
        red[lane] = contrib;
        __syncthreads();
        for (int stride = a.spw >> 1; stride > 0; stride >>= 1) {
            if (ls < stride) {
                const double2 o2 = red[lane + stride * a.rb];
                red[lane].x += o2.x;
                red[lane].y += o2.y;
            }
            __syncthreads();
        }
        if (ls == 0) {
            double2 *p = a.part + (size_t)L * (size_t)a.rb + (size_t)jr;
            double2 v = red[lane];
            if (!a.dot_first) {
                const double2 old = *p;
                v.x += old.x;
                v.y += old.y;
            }
            *p = v;
        }
    }
}

// degree-0 polynomial p = t_0: y = t_0 x and part = t_0 b^H x
template <typename T, bool IN_Z4>
__global__ void __launch_bounds__(kBlock) k_scale_dot(HopArgs<T> a) {
    using C = cplx_t<T>;
    __shared__ double2 red[kBlock];
    int nbk, sblk;
    if (!hop_tile<T>(a, blockIdx.x, nbk, sblk)) return;    // a padding workgroup (uniform)
    const unsigned L = (unsigned)nbk * (unsigned)a.nblk + (unsigned)sblk;
    const int lane = (int)threadIdx.x;
    const int jr = lane & (a.rb - 1), ls = lane / a.rb;
    const int s = sblk * a.spw + ls;
    const uint64_t r_global = sample_base(a.first, a.off) + (uint64_t)(nbk * a.rb + jr);
    const double2 t0 = a.troots[a.j];
    const Blk<T> in = blk<T>(a.in, nbk, a.g.V, a.rb);
    double2 contrib;
    contrib.x = contrib.y = 0.0;
    if (s < a.g.V) {
        const uint64_t S = sample_state(a.key, r_global);
        C w[12];
        load_site<T>(in, a.rb, jr, IN_Z4, S, s, T(1), w);
        if (a.y != nullptr) {
            const Blk<T> y = blk<T>(a.y, nbk, a.g.V, a.rb);
            const uint32_t off = site_off<T>(s, a.rb, jr);
#pragma unroll
            for (int c = 0; c < 12; ++c) y.st(c, off, cmul_d<T>(t0, w[c]));
        }
        if (a.part != nullptr) {
            C b[12];
            get_b<T>(a, nbk, jr, S, s, b);
            contrib = zmul(t0, dot12<T>(b, w));
        }
    }
    if (a.part != nullptr) {
        red[lane] = contrib;
        __syncthreads();
        for (int stride = a.spw >> 1; stride > 0; stride >>= 1) {
            if (ls < stride) {
                const double2 o2 = red[lane + stride * a.rb];
                red[lane].x += o2.x;
                red[lane].y += o2.y;
            }
            __syncthreads();
        }
        if (ls == 0) a.part[(size_t)L * (size_t)a.rb + (size_t)jr] = red[lane];
    }
}

// bhy[r] = sum over site blocks of part, fixed order: one 64-lane workgroup per vector
__global__ void __launch_bounds__(kSumLanes) k_reduce_part(const double2 *part, int nblk, int rb, double2 *bhy) {
    const int r = (int)blockIdx.x;
    const int nbk = r / rb, jr = r % rb;
    const double2 *p = part + (size_t)nbk * (size_t)nblk * (size_t)rb + (size_t)jr;
    double2 tot[1];
    sum_fixed<1>(nblk, [&](int b, double2 (&v)[1]) { v[0] = p[(size_t)b * (size_t)rb]; }, tot);
    if (threadIdx.x == 0) bhy[r] = tot[0];
}

// ------------------------------------------------------------------ host side

template <typename T> static HopArgs<T> base_args(const mpmc_lattice &lat, mpmc_shape sh) {
    HopArgs<T> a{};
    a.g = make_geo(lat.dims, lat.antiperiodic_t);
    const FieldTiling t = make_tiling(a.g.V, sh.nrhs, sh.rb);
    a.rb = t.rb;
    a.spw = t.spw;
    a.nblk = t.nblk;
    a.G = t.groups();
    // slab order when whole tiles cover an xyz-plane at least once per XCD
    const int P = lat.dims[0] * lat.dims[1] * lat.dims[2];
    if (g_opt_hop_slab && P % t.spw == 0 && P / t.spw >= kXcds) {
        a.slab = 1;
        a.tps = P / t.spw;
        a.chunk = (a.tps + kXcds - 1) / kXcds;
        a.G = (unsigned)kXcds * (unsigned)t.nb * (unsigned)lat.dims[3] * (unsigned)a.chunk;
    }
    a.gauge = (const cplx_t<T> *)lat.gauge;
    a.two_rows = lat.link_rows == 2;
    a.gbuf = g_opt_link_buf && 36ull * (unsigned long long)a.g.V * sizeof(cplx_t<T>) < (1ull << 32);
    a.kappa = lat.kappa;
    return a;
}

#define MPMC_LAUNCH(KERNEL, a, stream)                                                       \
    do {                                                                                     \
        hipLaunchKernelGGL((KERNEL), dim3((a).G), dim3(kBlock), 0, (hipStream_t)(stream), a); \
    } while (0)

template <typename T>
static void launch_hop(const HopArgs<T> &a, bool in_z4, bool dot, bool yacc, bool outer, bool addb, void *stream) {
    if (outer) { MPMC_LAUNCH((k_hop<T, false, false, false, true, false>), a, stream); return; }
    if (addb) { MPMC_LAUNCH((k_hop<T, false, false, false, false, true>), a, stream); return; }
    if (in_z4) {
        if (dot && yacc) MPMC_LAUNCH((k_hop<T, true, true, true, false, false>), a, stream);
        else if (dot) MPMC_LAUNCH((k_hop<T, true, true, false, false, false>), a, stream);
        else if (yacc) MPMC_LAUNCH((k_hop<T, true, false, true, false, false>), a, stream);
        else MPMC_LAUNCH((k_hop<T, true, false, false, false, false>), a, stream);
    } else {
        if (dot && yacc) MPMC_LAUNCH((k_hop<T, false, true, true, false, false>), a, stream);
        else if (dot) MPMC_LAUNCH((k_hop<T, false, true, false, false, false>), a, stream);
        else if (yacc) MPMC_LAUNCH((k_hop<T, false, false, true, false, false>), a, stream);
        else MPMC_LAUNCH((k_hop<T, false, false, false, false, false>), a, stream);
    }
}

template <typename T>
int wilson_apply_t(const mpmc_lattice &lat, mpmc_shape sh, const void *x, void *y, void *stream) {
    HopArgs<T> a = base_args<T>(lat, sh);
    a.in = (const cplx_t<T> *)x;
    a.out = (cplx_t<T> *)y;
    a.alpha.x = 1.0;
    a.alpha.y = 0.0;
    a.beta.x = -lat.kappa;
    a.beta.y = 0.0;
    launch_hop<T>(a, false, false, false, false, false, stream);
    return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

template <typename T>
int residual_apply_t(const mpmc_lattice &lat, mpmc_shape sh, const void *x, const void *b, uint64_t key,
                     uint64_t first, const uint64_t *off, void *out, void *stream) {
    // out = b - A x
    HopArgs<T> a = base_args<T>(lat, sh);
    a.in = (const cplx_t<T> *)x;
    a.out = (cplx_t<T> *)out;
    a.alpha.x = -1.0;
    a.alpha.y = 0.0;
    a.beta.x = lat.kappa;
    a.beta.y = 0.0;
    a.bvec = (const cplx_t<T> *)b;
    a.key = key;
    a.first = first;
    a.off = off;
    launch_hop<T>(a, false, false, false, false, true, stream);
    return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

// Newton-form single polynomial over n roots (n-1 operator applications).
//   x == nullptr: input is the noise; bvec == nullptr: dot vector is the noise.
template <typename T>
static int newton_t(const mpmc_lattice &lat, mpmc_shape sh, int n, const double *troots, const void *x, bool x_is_noise,
                    const void *bvec, uint64_t key, uint64_t first, const uint64_t *off, void *y, double2 *part, void *w0, void *w1,
                    void *stream) {
    HopArgs<T> a = base_args<T>(lat, sh);
    a.troots = (const double2 *)troots;
    a.key = key;
    a.first = first;
    a.off = off;
    a.bvec = (const cplx_t<T> *)bvec;
    a.part = part;
    a.y = (cplx_t<T> *)y;
    const bool dot = part != nullptr, yacc = y != nullptr;
    if (n == 1) {
        a.j = 0;
        a.in = (const cplx_t<T> *)x;
        if (x_is_noise) hipLaunchKernelGGL((k_scale_dot<T, true>), dim3(a.G), dim3(kBlock), 0, (hipStream_t)stream, a);
        else hipLaunchKernelGGL((k_scale_dot<T, false>), dim3(a.G), dim3(kBlock), 0, (hipStream_t)stream, a);
        return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
    }
    const int d = n - 1;
    for (int j = 0; j < d; ++j) {
        a.j = j;
        a.in = (j == 0) ? (const cplx_t<T> *)x : (const cplx_t<T> *)((j - 1) % 2 == 0 ? w0 : w1);
        a.out = (cplx_t<T> *)(j % 2 == 0 ? w0 : w1);
        a.y_first = (j == 0);
        a.y_last = (j == d - 1);
        a.dot_first = (j == 0);
        launch_hop<T>(a, j == 0 && x_is_noise, dot, yacc, false, false, stream);
        if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    }
    return MPMC_OK;
}

// b^H p_in(A) p_out(A p_in(A)) b for the noise b, the input (x, or b when x
// is null) moved to block width 1 first; see poly_apply_t
template <typename T>
static int composite_sweep_t(const mpmc_lattice &lat, const mpmc_poly &poly, mpmc_shape sh, mpmc_shape sh1,
                             const SweepPlan &plan, const void *x, uint64_t key, uint64_t first, const uint64_t *off,
                             double *bhy, const PolyWs &ws, void *stream) {
    void *U0 = ws.f[0], *U1 = ws.f[1], *V0 = ws.f[2], *V1 = ws.f[3], *Y = ws.f[4];
    const int32_t prec = sizeof(T) == 8 ? MPMC_F64 : MPMC_F32;
    int st;
    if (x != nullptr)
        st = field_relayout_impl(lat.dims, prec, sh.nrhs, x, sh.rb, U0, 1, stream);
    else
        st = copy_or_noise_t<T>(lat, sh1, nullptr, key, first, off, U0, stream);
    if (st != MPMC_OK) return st;
    HopArgs<T> a = base_args<T>(lat, sh1);
    a.troots = (const double2 *)poly.inv_roots_in;
    a.phi = (const double2 *)poly.inv_roots_out;
    void *ucur = U0, *unext = U1;
    const int n_in = poly.n_in, n_out = poly.n_out;
    for (int jo = 0; jo + 1 < n_out; ++jo) {
        const void *vin = nullptr;
        st = sweep_chain_t<T>(lat, sh1, plan, n_in - 1, poly.inv_roots_in, ucur, 1, V0, V1, &vin, stream);
        if (st != MPMC_OK) return st;
        // last inner step with the outer update: u_next, y (the chain left V0 or V1 free)
        a.j = n_in - 1;
        a.in = (const cplx_t<T> *)vin;
        a.u = (const cplx_t<T> *)ucur;
        a.u_next = (cplx_t<T> *)unext;
        a.y = (cplx_t<T> *)Y;
        a.jo = jo;
        a.y_first = (jo == 0);
        a.jo_last = (jo + 2 == n_out);
        launch_hop<T>(a, false, false, false, true, false, stream);
        if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
        void *tmp = ucur;
        ucur = unext;
        unext = tmp;
    }
    // final p_in(A) applied to y_out, dot against the noise
    return sweep_newton_t<T>(lat, sh1, plan, n_in, poly.inv_roots_in, Y, false, nullptr, key, first, off,
                             (double2 *)ws.part, (double2 *)bhy, V0, V1, nullptr, stream);
}

template <typename T>
int poly_apply_t(const mpmc_lattice &lat, const mpmc_poly &poly, mpmc_shape sh, const void *x, const mpmc_noise *noise,
                 void *y, double *bhy, const PolyWs &ws, void *stream) {
    const uint64_t key = noise ? noise_key(*noise) : 0ull;
    const uint64_t first = noise ? noise->first_sample : 0ull;
    const uint64_t *off = noise ? noise->sample_offset : nullptr;
    const bool x_noise = (x == nullptr);
    // dot vector: the noise if given, else x itself
    const void *bvec = noise ? nullptr : x;
    double2 *part = bhy ? (double2 *)ws.part : nullptr;
    const FieldTiling t = make_tiling(lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3], sh.nrhs, sh.rb);
    int st;
    const int32_t *colour = noise ? noise->probe_colour : nullptr;
    if (poly.n_out == 0 && y == nullptr && bhy != nullptr && poly.n_in >= 2 && (g_opt_sweep || colour)) {
        // scalar mode: t-sweep over xyz-blocks when the lattice admits one
        // (option 2: and the batch keeps half the CUs busy; probe vectors
        // are generated only by the sweep and always take it)
        const SweepPlan plan = sweep_plan(lat, sh);
        if (plan.ok && (plan.busy || g_opt_sweep == 1 || colour))
            return sweep_newton_t<T>(lat, sh, plan, poly.n_in, poly.inv_roots_in, x, x_noise, bvec, key, first, off,
                                     part, (double2 *)bhy, ws.f[0], ws.f[1], nullptr, stream, colour);
    }
    if (colour) return MPMC_EUNSUPPORTED;                          // probe vectors: the t-sweep only
    if (poly.n_out == 0 && poly.n_in >= 2 && y != nullptr && sh.rb == 1 && (noise != nullptr || bhy == nullptr) &&
        g_opt_sweep) {
        // vector mode on the t-sweep: y (block width 1, like the sweep's own
        // outputs) accumulates t_j w_j in the same launches; when the batch,
        // chunked in t, fills the GPU (option 1: whenever the lattice admits a
        // sweep)
        const SweepPlan plan = sweep_plan(lat, sh);
        if (plan.ok && (plan.fills || g_opt_sweep == 1))
            return sweep_newton_t<T>(lat, sh, plan, poly.n_in, poly.inv_roots_in, x, x_noise, bhy ? bvec : nullptr,
                                     key, first, off, bhy ? part : nullptr, (double2 *)bhy, ws.f[0], ws.f[1], y,
                                     stream);
    }
    if (poly.n_out >= 2 && poly.n_in >= 2 && y == nullptr && bhy != nullptr && noise != nullptr && g_opt_sweep) {
        // scalar-mode double polynomial against the noise: the n_in - 1 plain
        // steps of every inner chain and the final p_in run as t-sweeps, the
        // fused outer update on the streaming kernel, all at block width 1
        const mpmc_shape sh1{sh.nrhs, 1};
        const SweepPlan plan = sweep_plan(lat, sh1);
        if (plan.ok && (plan.busy || g_opt_sweep == 1)) return composite_sweep_t<T>(lat, poly, sh, sh1, plan, x, key, first, off, bhy, ws, stream);
    }
    if (poly.n_out == 0) {
        st = newton_t<T>(lat, sh, poly.n_in, poly.inv_roots_in, x, x_noise, bvec, key, first, off, y, part, ws.f[0],
                         ws.f[1], stream);
        if (st != MPMC_OK) return st;
    } else {
        // composite p_in(A) p_out(B), B = A p_in(A) = I - pi_in(A) (Sec. 3.2)
        HopArgs<T> a = base_args<T>(lat, sh);
        void *U0 = ws.f[0], *U1 = ws.f[1], *V0 = ws.f[2], *V1 = ws.f[3], *Y = ws.f[4];
        // u_0 = x
        st = copy_or_noise_t<T>(lat, sh, x, key, first, off, U0, stream);
        if (st != MPMC_OK) return st;
        void *ucur = U0, *unext = U1;
        const int n_in = poly.n_in, n_out = poly.n_out;
        a.troots = (const double2 *)poly.inv_roots_in;
        a.phi = (const double2 *)poly.inv_roots_out;
        if (n_out == 1) {
            HopArgs<T> s1 = base_args<T>(lat, sh);
            s1.troots = (const double2 *)poly.inv_roots_out;
            s1.j = 0;
            s1.in = (const cplx_t<T> *)ucur;
            s1.y = (cplx_t<T> *)Y;
            hipLaunchKernelGGL((k_scale_dot<T, false>), dim3(s1.G), dim3(kBlock), 0, (hipStream_t)stream, s1);
        }
        for (int jo = 0; jo + 1 < n_out; ++jo) {
            const void *vin = ucur;
            for (int i = 0; i < n_in; ++i) {
                a.j = i;
                a.in = (const cplx_t<T> *)vin;
                if (i + 1 < n_in) {
                    void *vout = (i % 2 == 0) ? V0 : V1;
                    a.out = (cplx_t<T> *)vout;
                    launch_hop<T>(a, false, false, false, false, false, stream);
                    vin = vout;
                } else {
                    a.u = (const cplx_t<T> *)ucur;
                    a.u_next = (cplx_t<T> *)unext;
                    a.y = (cplx_t<T> *)Y;
                    a.jo = jo;
                    a.y_first = (jo == 0);
                    a.jo_last = (jo + 2 == n_out);
                    launch_hop<T>(a, false, false, false, true, false, stream);
                    void *tmp = ucur;
                    ucur = unext;
                    unext = tmp;
                }
                if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
            }
        }
        // final p_in(A) applied to y_out, dot against b
        const void *bv = noise ? nullptr : x;
        st = newton_t<T>(lat, sh, n_in, poly.inv_roots_in, Y, false, bv, key, first, off, y, part, V0, V1, stream);
        if (st != MPMC_OK) return st;
    }
    if (bhy) {
        hipLaunchKernelGGL(k_reduce_part, dim3(sh.nrhs), dim3(kSumLanes), 0, (hipStream_t)stream,
                           (const double2 *)ws.part, t.nblk, sh.rb, (double2 *)bhy);
        if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    }
    return MPMC_OK;
}

template int wilson_apply_t<double>(const mpmc_lattice &, mpmc_shape, const void *, void *, void *);
template int wilson_apply_t<float>(const mpmc_lattice &, mpmc_shape, const void *, void *, void *);
template int residual_apply_t<double>(const mpmc_lattice &, mpmc_shape, const void *, const void *, uint64_t, uint64_t,
                                      const uint64_t *, void *, void *);
template int residual_apply_t<float>(const mpmc_lattice &, mpmc_shape, const void *, const void *, uint64_t, uint64_t,
                                     const uint64_t *, void *, void *);
template int poly_apply_t<double>(const mpmc_lattice &, const mpmc_poly &, mpmc_shape, const void *, const mpmc_noise *,
                                  void *, double *, const PolyWs &, void *);
template int poly_apply_t<float>(const mpmc_lattice &, const mpmc_poly &, mpmc_shape, const void *, const mpmc_noise *,
                                 void *, double *, const PolyWs &, void *);

}  // namespace mpmc
