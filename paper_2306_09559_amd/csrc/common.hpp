// Device-side building blocks shared by the libmpmc kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpmc.h"

namespace mpmc {

// ---------------------------------------------------------------- complex
template <typename T> struct c2;
template <> struct c2<double> { using type = double2; };
template <> struct c2<float> { using type = float2; };
template <typename T> using cplx_t = typename c2<T>::type;

template <typename T> __device__ __forceinline__ cplx_t<T> mk(T re, T im) {
    cplx_t<T> z;
    z.x = re;
    z.y = im;
    return z;
}
template <typename T> __device__ __forceinline__ cplx_t<T> cadd(cplx_t<T> a, cplx_t<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx_t<T> csub(cplx_t<T> a, cplx_t<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
// a * b
template <typename T> __device__ __forceinline__ cplx_t<T> cmul(cplx_t<T> a, cplx_t<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
template <typename T> __device__ __forceinline__ cplx_t<T> cfma(cplx_t<T> a, cplx_t<T> b, cplx_t<T> acc) {
    return mk<T>(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
// acc + conj(a) * b
template <typename T> __device__ __forceinline__ cplx_t<T> cfmaconj(cplx_t<T> a, cplx_t<T> b, cplx_t<T> acc) {
    return mk<T>(acc.x + a.x * b.x + a.y * b.y, acc.y + a.x * b.y - a.y * b.x);
}
// Products with a coefficient held in FP64.  The step coefficients of a
// polynomial (t_j, kappa t_j, phi_j, ...) are never rounded to the field
// precision: in FP32 mode the entries are widened, combined in FP64 and
// rounded once, so the polynomial applied is exactly the FP64 one and only
// the vector entries carry FP32 rounding (a rounded coefficient would shift
// every sample's result the same way).
// a * x
template <typename T> __device__ __forceinline__ cplx_t<T> cmul_d(double2 a, cplx_t<T> x) {
    const double xr = (double)x.x, xi = (double)x.y;
    return mk<T>((T)(a.x * xr - a.y * xi), (T)(a.x * xi + a.y * xr));
}
// a * x + b * y
template <typename T>
__device__ __forceinline__ cplx_t<T> lin2_d(double2 a, cplx_t<T> x, double2 b, cplx_t<T> y) {
    const double xr = (double)x.x, xi = (double)x.y, yr = (double)y.x, yi = (double)y.y;
    return mk<T>((T)(a.x * xr - a.y * xi + (b.x * yr - b.y * yi)), (T)(a.x * xi + a.y * xr + (b.x * yi + b.y * yr)));
}
// y + a * x
template <typename T> __device__ __forceinline__ cplx_t<T> axpy_d(double2 a, cplx_t<T> x, cplx_t<T> y) {
    const double xr = (double)x.x, xi = (double)x.y;
    return mk<T>((T)((double)y.x + (a.x * xr - a.y * xi)), (T)((double)y.y + (a.x * xi + a.y * xr)));
}

// p advanced by an offset the compiler cannot see (zero): address arithmetic
// built on the result stays inside a rolled loop instead of being hoisted.
// Hiding the pointer itself would also hide that it points to global memory,
// and its loads would become flat loads, which hold up every LDS wait.
template <typename P> __device__ __forceinline__ P *opaque_ptr(P *p) {
    long z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

// i * a and -i * a
template <typename T> __device__ __forceinline__ cplx_t<T> mul_i(cplx_t<T> a) { return mk<T>(-a.y, a.x); }
template <typename T> __device__ __forceinline__ cplx_t<T> mul_mi(cplx_t<T> a) { return mk<T>(a.y, -a.x); }

// One link U (row-major, entry (a, b) at gl + (3a + b) * estride + off).
// two_rows: U is special unitary and only rows 0 and 1 are read; row 2 is
// rebuilt as the complex conjugate of row 0 x row 1 (for U in SU(3) the
// rows are orthonormal and det U = 1, so row 2 = conj(r0 x r1) exactly).
template <typename T>
__device__ __forceinline__ void load_su3(const char *gl, size_t estride, uint32_t off, bool two_rows,
                                         cplx_t<T> (&U)[9]) {
#pragma unroll
    for (int e = 0; e < 6; ++e) U[e] = *(const cplx_t<T> *)(gl + (size_t)e * estride + off);
    if (two_rows) {
        const cplx_t<T> c0 = csub<T>(cmul<T>(U[1], U[5]), cmul<T>(U[2], U[4]));
        const cplx_t<T> c1 = csub<T>(cmul<T>(U[2], U[3]), cmul<T>(U[0], U[5]));
        const cplx_t<T> c2 = csub<T>(cmul<T>(U[0], U[4]), cmul<T>(U[1], U[3]));
        U[6] = mk<T>(c0.x, -c0.y);
        U[7] = mk<T>(c1.x, -c1.y);
        U[8] = mk<T>(c2.x, -c2.y);
    } else {
#pragma unroll
        for (int e = 6; e < 9; ++e) U[e] = *(const cplx_t<T> *)(gl + (size_t)e * estride + off);
    }
}

// Buffer loads of the links: a resource over the whole link array (4 scalar
// registers for the launch), each element's byte offset (mu, e) in a scalar
// register and the site's 32-bit offset in the lane: one load instruction
// per element.  Flat loads from a 64-bit base put every element's address in
// a register pair instead: a chain of 64-bit vector adds, or with scalar
// bases per element, spilled scalar registers.  Needs the link array below
// 4 GiB (36 V sizeof(complex) bytes).  The streaming kernel takes them; the
// t-sweeps keep flat loads, measured faster there (FP32 whole planes 60.8
// against 64.5 us per launch at 8^4 x 256 vectors, blocked 4%, FP64 even).
constexpr int kBufWord3 = 0x00020000;    // raw buffer access (gfx9 descriptor word 3)

template <typename T>
__device__ __forceinline__ cplx_t<T> buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(cplx_t<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    } else {
        return __builtin_bit_cast(cplx_t<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
}

// the links of direction mu: element e of a site at base + e * es + site * sizeof(complex)
template <typename T> struct LinkBuf {
    __amdgpu_buffer_rsrc_t r;
    uint32_t base, es;
};
template <typename T> __device__ __forceinline__ LinkBuf<T> link_buf(const void *gauge, int V, int mu) {
    LinkBuf<T> l;
    l.es = (uint32_t)V * (uint32_t)sizeof(cplx_t<T>);
    l.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(gauge), (short)0, (int)(36u * l.es), kBufWord3);
    l.base = (uint32_t)mu * 9u * l.es;
    return l;
}
template <typename T> __device__ __forceinline__ cplx_t<T> link_el(const LinkBuf<T> &l, int e, int site) {
    return buf_ld<T>(l.r, (uint32_t)site * (uint32_t)sizeof(cplx_t<T>), l.base + (uint32_t)e * l.es);
}

// load_su3 through a LinkBuf
template <typename T>
__device__ __forceinline__ void load_su3_buf(const LinkBuf<T> &l, int site, bool two_rows, cplx_t<T> (&U)[9]) {
#pragma unroll
    for (int e = 0; e < 6; ++e) U[e] = link_el<T>(l, e, site);
    if (two_rows) {
        const cplx_t<T> c0 = csub<T>(cmul<T>(U[1], U[5]), cmul<T>(U[2], U[4]));
        const cplx_t<T> c1 = csub<T>(cmul<T>(U[2], U[3]), cmul<T>(U[0], U[5]));
        const cplx_t<T> c2 = csub<T>(cmul<T>(U[0], U[4]), cmul<T>(U[1], U[3]));
        U[6] = mk<T>(c0.x, -c0.y);
        U[7] = mk<T>(c1.x, -c1.y);
        U[8] = mk<T>(c2.x, -c2.y);
    } else {
#pragma unroll
        for (int e = 6; e < 9; ++e) U[e] = link_el<T>(l, e, site);
    }
}

// ---------------------------------------------------------------- geometry
struct Geo {
    int L[4];      // Lx, Ly, Lz, Lt
    int st[4];     // site strides 1, Lx, Lx*Ly, Lx*Ly*Lz
    int V;
    int apbc;      // antiperiodic time
};

inline Geo make_geo(const int32_t dims[4], int apbc) {
    Geo g;
    for (int d = 0; d < 4; ++d) g.L[d] = dims[d];
    g.st[0] = 1;
    g.st[1] = dims[0];
    g.st[2] = dims[0] * dims[1];
    g.st[3] = dims[0] * dims[1] * dims[2];
    g.V = g.st[3] * dims[3];
    g.apbc = apbc;
    return g;
}

// ---------------------------------------------------------------- Z4 noise
// SplitMix64 (Steele, Lea & Flood 2014): output k of state x = mix(x + k*gamma).
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

__host__ __device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t sm_out(uint64_t x, uint64_t k) { return sm_mix(x + k * kGolden); }

// Global index of vector 0 of a noise batch: first_sample, plus the device
// counter sample_offset when one is given (read by the kernels, so a captured
// graph draws new samples on every replay once the counter is advanced).
__device__ __forceinline__ uint64_t sample_base(uint64_t first, const uint64_t *off) {
    return off ? first + *off : first;
}

inline uint64_t noise_key(const mpmc_noise &nz) {
    uint64_t k = sm_out(nz.seed, 1);
    k = sm_out(k ^ nz.lattice, 1);
    return sm_out(k ^ nz.level, 1);
}

// per-sample generator state
__device__ __forceinline__ uint64_t sample_state(uint64_t key, uint64_t sample) { return sm_out(key ^ sample, 1); }

// 2-bit code q of unknown i of the sample with state S
__device__ __forceinline__ unsigned z4_code(uint64_t S, unsigned i) {
    const uint64_t w = sm_out(S, (uint64_t)(i >> 5) + 1);
    return (unsigned)(w >> (2 * (i & 31))) & 3u;
}

// the 12 codes of site s (unknowns 12s .. 12s+11) packed 2 bits each
__device__ __forceinline__ uint32_t z4_site_codes(uint64_t S, unsigned s) {
    const unsigned i0 = 12u * s;
    const unsigned w0 = i0 >> 5, sh = 2u * (i0 & 31u);
    const uint64_t a = sm_out(S, (uint64_t)w0 + 1);
    uint64_t bits = a >> sh;
    if (sh > 40u) {  // the 24 bits straddle two 64-bit words
        const uint64_t b = sm_out(S, (uint64_t)w0 + 2);
        bits |= b << (64u - sh);
    }
    return (uint32_t)(bits & 0xFFFFFFu);
}

template <typename T> __device__ __forceinline__ cplx_t<T> z4_value(unsigned q) {
    // q = 0, 1, 2, 3 -> 1, i, -1, -i
    const T re = (q == 0u) ? T(1) : ((q == 2u) ? T(-1) : T(0));
    const T im = (q == 1u) ? T(1) : ((q == 3u) ? T(-1) : T(0));
    return mk<T>(re, im);
}

// ---------------------------------------------------------------- partial sums
// out[m] = sum over b < n of term(b)[m], in a fixed order, by one 64-lane
// workgroup (launch with blockDim.x = kSumLanes): lane j adds the terms
// j, j + 64, ... in turn, then a fixed tree combines the lanes.  Every lane
// returns the total.  The order depends only on n, never on timing.
constexpr int kSumLanes = 64;
template <int M, typename F> __device__ __forceinline__ void sum_fixed(int n, F term, double2 (&out)[M]) {
    __shared__ double2 red[M][kSumLanes];
    const int j = (int)threadIdx.x;
    double2 acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = make_double2(0.0, 0.0);
    for (int b = j; b < n; b += kSumLanes) {
        double2 v[M];
        term(b, v);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            acc[m].x += v[m].x;
            acc[m].y += v[m].y;
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) red[m][j] = acc[m];
    __syncthreads();
    for (int h = kSumLanes / 2; h > 0; h >>= 1) {
        if (j < h) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                red[m][j].x += red[m][j + h].x;
                red[m][j].y += red[m][j + h].y;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < M; ++m) out[m] = red[m][0];
}

// ---------------------------------------------------------------- launch shape
constexpr int kBlock = 256;   // threads per workgroup of the field kernels
constexpr int kXcds = 8;      // MI355X: 8 XCDs, workgroups dispatched round-robin

// Map the hardware workgroup index to a logical index so that each XCD
// (hardware index mod 8) receives one contiguous range of logical work:
// neighbouring tiles then share that XCD's L2.  A bijection on [0, G).
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned G) {
    const unsigned x = bid % kXcds, slot = bid / kXcds;
    const unsigned q = G / kXcds, rem = G % kXcds;
    return x * q + (x < rem ? x : rem) + slot;
}

// Field-kernel work decomposition: a workgroup covers spw = 256/rb sites of
// one RHS block, all rb vectors of that block.
struct FieldTiling {
    int rb, spw, nblk, nb;   // nblk site blocks per RHS block, nb RHS blocks
    unsigned groups() const { return (unsigned)(nblk * nb); }
};

inline FieldTiling make_tiling(int V, int nrhs, int rb) {
    FieldTiling t;
    t.rb = rb;
    t.spw = kBlock / rb;
    t.nblk = (V + t.spw - 1) / t.spw;
    t.nb = nrhs / rb;
    return t;
}

}  // namespace mpmc
