// Deflation products on the matrix cores (Sec. 2.1 Left-right Projection,
// Sec. 4.1 Monte Carlo deflation, Sec. 4.3 deflated polynomial).
//
// Coefficients.  zeta = V^H b and omega = U^H b with u_i = scale_i g5 z_pair(i)
// need only the two half products over the upper spins (c < 6) and the lower
// spins (c >= 6): V^H b = up + dn and V^H g5 b = up - dn, so omega_i =
// conj(scale_i) (up - dn)[pair_i] and U is never stored.  Each wavefront
// accumulates one 16 x 16 (eigenvector x vector) tile over a slice of the
// lattice with the 16x16x4 MFMA (FP64 operands in FP64 mode, FP32 operands
// and accumulation in FP32 mode) in the complex "4 real products" form; the
// slices are summed in FP64 in a fixed order.  Z4 operands are regenerated
// in registers.
//
// Reconstruction.  X = V d (n x N) with the same MFMA, d rounded to the
// field precision.
#include "common.hpp"
#include "internal.hpp"

namespace mpmc {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Operand layout (both): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
// Accumulator element v of lane l is D[row(l, v)][l % 16], where the row
// mapping differs between the FP64 and FP32 instructions (measured on gfx950).
template <> struct Mfma<double> {
    using acc_t = d4_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return l / 16 + 4 * v; }
};
template <> struct Mfma<float> {
    using acc_t = f4_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l / 16) + v; }
};

constexpr int kWaves = 4;   // wavefronts per workgroup in the GEMM kernels

template <typename T> struct CoeffArgs {
    int Vol, kpad, nrhs, rb, ntr;      // ntr: 16-wide vector tiles
    int sites_per_split;               // multiple of 16
    const cplx_t<T> *V;                // [12][Vol][kpad]
    const cplx_t<T> *b;                // field, or nullptr -> Z4
    uint64_t key, first;
    const uint64_t *off;
    double2 *part;                     // [split][2][kpad][ntr*16]
};

// grid: x = eigen tile * ntr + vector tile, y = split
template <typename T>
__global__ void __launch_bounds__(kWaves * 64) k_coeff(CoeffArgs<T> a) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    __shared__ double2 red[kWaves][2][64][4];
    const int wave = (int)threadIdx.x / 64, l = (int)threadIdx.x % 64;
    const int kk = l / 16, m = l % 16;
    const int ti = (int)blockIdx.x / a.ntr, tr = (int)blockIdx.x % a.ntr;
    const int i = ti * 16 + m;                  // eigenvector row of the A operand
    const int r = tr * 16 + m;                  // vector column of the B operand
    const bool rvalid = r < a.nrhs;
    const int s_begin = (int)blockIdx.y * a.sites_per_split;
    const int s_end = min(s_begin + a.sites_per_split, a.Vol);
    uint64_t S = 0;
    size_t bfb = 0;
    if (rvalid) {
        if (a.b == nullptr) S = sample_state(a.key, sample_base(a.first, a.off) + (uint64_t)r);
        else bfb = (size_t)(r / a.rb) * 12 * (size_t)a.Vol * (size_t)a.rb + (size_t)(r % a.rb);
    }
    acc_t cre[2], cim[2];
    for (int h = 0; h < 2; ++h)
        for (int v = 0; v < 4; ++v) cre[h][v] = cim[h][v] = T(0);

    for (int s0 = s_begin + wave * 4; s0 < s_end; s0 += kWaves * 4) {
        const int s = s0 + kk;
        const bool sv = s < s_end;
        uint32_t codes = 0;
        if (sv && rvalid && a.b == nullptr) codes = z4_site_codes(S, (unsigned)s);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            T vr = T(0), vi = T(0), br = T(0), bi = T(0);
            if (sv) {
                const cplx_t<T> v = a.V[((size_t)c * a.Vol + (size_t)s) * (size_t)a.kpad + (size_t)i];
                vr = v.x;
                vi = v.y;
                if (rvalid) {
                    cplx_t<T> bb;
                    if (a.b == nullptr) bb = z4_value<T>((codes >> (2 * c)) & 3u);
                    else bb = a.b[bfb + ((size_t)c * a.Vol + (size_t)s) * (size_t)a.rb];
                    br = bb.x;
                    bi = bb.y;
                }
            }
            const int h = c < 6 ? 0 : 1;
            // conj(v) b = (vr br + vi bi) + i (vr bi - vi br)
            cre[h] = M::run(vr, br, cre[h]);
            cre[h] = M::run(vi, bi, cre[h]);
            cim[h] = M::run(vr, bi, cim[h]);
            cim[h] = M::run(-vi, br, cim[h]);
        }
    }
    // fixed-order sum of the wavefronts' tiles
    for (int h = 0; h < 2; ++h)
        for (int v = 0; v < 4; ++v) {
            double2 z;
            z.x = (double)cre[h][v];
            z.y = (double)cim[h][v];
            red[wave][h][l][v] = z;
        }
    __syncthreads();
    if (wave == 0) {
        for (int h = 0; h < 2; ++h)
            for (int v = 0; v < 4; ++v) {
                double2 z = red[0][h][l][v];
                for (int w = 1; w < kWaves; ++w) {
                    z.x += red[w][h][l][v].x;
                    z.y += red[w][h][l][v].y;
                }
                const int row = ti * 16 + M::row(l, v);
                const int col = tr * 16 + (l % 16);
                const size_t ldr = (size_t)a.ntr * 16;
                a.part[(((size_t)blockIdx.y * 2 + h) * (size_t)a.kpad + (size_t)row) * ldr + (size_t)col] = z;
            }
    }
}

// One vector (the Gram-Schmidt steps of the set-up's Arnoldi runs): the same
// partial sums as k_coeff, on the vector units.  The MFMA tiles would pad the
// vector to 16 columns and do 16 times the products, which bounds that kernel
// on the matrix cores (FP64 at 24^3x48, 128 basis vectors: ~1.7 ms of MFMA
// per call against ~3 ms to read the basis); here every lane (eigenvector
// row m, site kk of four) forms conj(v) b for its sites in FP64, and the
// partials are summed over the sites of a wave and the waves in a fixed
// order.  Only column 0 of the partial rows is written (ntr = 1).
template <typename T>
__global__ void __launch_bounds__(kWaves * 64) k_coeff_one(CoeffArgs<T> a) {
    __shared__ double2 red[kWaves][2][64];
    const int wave = (int)threadIdx.x / 64, l = (int)threadIdx.x % 64;
    const int kk = l / 16, m = l % 16;
    const int i = (int)blockIdx.x * 16 + m;
    const int s_begin = (int)blockIdx.y * a.sites_per_split;
    const int s_end = min(s_begin + a.sites_per_split, a.Vol);
    const uint64_t S = a.b == nullptr ? sample_state(a.key, sample_base(a.first, a.off)) : 0ull;
    double ur = 0.0, ui = 0.0, dr = 0.0, di = 0.0;
    for (int s0 = s_begin + wave * 4; s0 < s_end; s0 += kWaves * 4) {
        const int s = s0 + kk;
        if (s >= s_end) continue;
        const uint32_t codes = a.b == nullptr ? z4_site_codes(S, (unsigned)s) : 0u;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cplx_t<T> v = a.V[((size_t)c * a.Vol + (size_t)s) * (size_t)a.kpad + (size_t)i];
            const cplx_t<T> bb = a.b == nullptr ? z4_value<T>((codes >> (2 * c)) & 3u)
                                                : a.b[((size_t)c * a.Vol + (size_t)s) * (size_t)a.rb];
            const double vr = (double)v.x, vi = (double)v.y, br = (double)bb.x, bi = (double)bb.y;
            // conj(v) b = (vr br + vi bi) + i (vr bi - vi br)
            if (c < 6) {
                ur += vr * br + vi * bi;
                ui += vr * bi - vi * br;
            } else {
                dr += vr * br + vi * bi;
                di += vr * bi - vi * br;
            }
        }
    }
    red[wave][0][l] = make_double2(ur, ui);
    red[wave][1][l] = make_double2(dr, di);
    __syncthreads();
    if (threadIdx.x < 32) {
        const int h = (int)threadIdx.x / 16, mm = (int)threadIdx.x % 16;
        double2 z = make_double2(0.0, 0.0);
        for (int w = 0; w < kWaves; ++w)
            for (int q = 0; q < 4; ++q) {
                z.x += red[w][h][q * 16 + mm].x;
                z.y += red[w][h][q * 16 + mm].y;
            }
        const int row = (int)blockIdx.x * 16 + mm;
        a.part[(((size_t)blockIdx.y * 2 + h) * (size_t)a.kpad + (size_t)row) * 16] = z;
    }
}

// zeta = up + dn, omega_i = conj(scale_i) (up - dn)[pair_i]; fixed split order
// one 64-lane workgroup per (eigenvector, vector): the four split sums in a fixed order (sum_fixed)
__global__ void __launch_bounds__(kSumLanes) k_coeff_finish(const double2 *part, int nsplit, int kpad, int ldr, int k,
                                                            int nrhs, const int32_t *pair, const double2 *scale,
                                                            double2 *zeta, double2 *omega) {
    const int e = (int)blockIdx.x;
    const int i = e / nrhs, r = e % nrhs;
    const int pr = pair[i];
    const bool pair_ok = pr >= 0 && pr < k;     // a bad pair entry yields NaN, never a stray read
    const int pi = pair_ok ? pr : i;
    double2 s4[4];
    sum_fixed<4>(nsplit, [&](int p, double2 (&v)[4]) {
        const double2 *b0 = part + ((size_t)p * 2) * (size_t)kpad * (size_t)ldr;
        const double2 *b1 = b0 + (size_t)kpad * (size_t)ldr;
        v[0] = b0[(size_t)i * ldr + r];
        v[1] = b1[(size_t)i * ldr + r];
        v[2] = b0[(size_t)pi * ldr + r];
        v[3] = b1[(size_t)pi * ldr + r];
    }, s4);
    if (threadIdx.x != 0) return;
    const double2 u = s4[0], d = s4[1], up = s4[2], dp = s4[3];
    if (zeta) {
        double2 z;
        z.x = u.x + d.x;
        z.y = u.y + d.y;
        zeta[(size_t)i * nrhs + r] = z;
    }
    if (omega) {
        const double xr = up.x - dp.x, xi = up.y - dp.y;
        const double2 sc = scale[i];
        double2 o;   // conj(sc) * xi
        o.x = sc.x * xr + sc.y * xi;
        o.y = sc.x * xi - sc.y * xr;
        if (!pair_ok) o.x = o.y = __builtin_nan("");
        omega[(size_t)i * nrhs + r] = o;
    }
}

// d = H^{-1} omega  (k x k times k x N, FP64)
__global__ void k_small_gemm(const double2 *hinv, const double2 *omega, int k, int nrhs, double2 *d) {
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= k * nrhs) return;
    const int i = e / nrhs, r = e % nrhs;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < k; ++j) {
        const double2 h = hinv[(size_t)i * k + j], w = omega[(size_t)j * nrhs + r];
        re += h.x * w.x - h.y * w.y;
        im += h.x * w.y + h.y * w.x;
    }
    double2 o;
    o.x = re;
    o.y = im;
    d[(size_t)i * nrhs + r] = o;
}

template <typename T> struct ReconArgs {
    int Vol, kpad, k, nrhs, rb, ntr, nts;   // nts: 16-site tiles
    int kact;                               // columns summed: k rounded up to the MFMA depth 4
    const cplx_t<T> *V;
    const double2 *d;                       // k x nrhs
    cplx_t<T> *X;                           // field
};

// grid: x = (site tile * 12 + c) / kWaves groups, y = vector tile
template <typename T>
__global__ void __launch_bounds__(kWaves * 64) k_recon(ReconArgs<T> a) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    const int wave = (int)threadIdx.x / 64, l = (int)threadIdx.x % 64;
    const int kk = l / 16, m = l % 16;
    const int tile = (int)blockIdx.x * kWaves + wave;      // (site tile, c) pair
    if (tile >= a.nts * 12) return;
    const int c = tile % 12, ts = tile / 12;
    const int tr = (int)blockIdx.y;
    const int s = ts * 16 + m;                 // site row of the A operand
    const int r = tr * 16 + m;                 // vector column of the B operand
    acc_t xr, xi;
    for (int v = 0; v < 4; ++v) xr[v] = xi[v] = T(0);
    for (int i0 = 0; i0 < a.kact; i0 += 4) {
        const int i = i0 + kk;
        T vr = T(0), vi = T(0), dr = T(0), di = T(0);
        if (s < a.Vol) {
            const cplx_t<T> v = a.V[((size_t)c * a.Vol + (size_t)s) * (size_t)a.kpad + (size_t)i];
            vr = v.x;
            vi = v.y;
        }
        if (i < a.k && r < a.nrhs) {
            const double2 dd = a.d[(size_t)i * a.nrhs + r];
            dr = (T)dd.x;
            di = (T)dd.y;
        }
        // v d = (vr dr - vi di) + i (vr di + vi dr)
        xr = M::run(vr, dr, xr);
        xr = M::run(-vi, di, xr);
        xi = M::run(vr, di, xi);
        xi = M::run(vi, dr, xi);
    }
    const int col = tr * 16 + (l % 16);
    if (col >= a.nrhs) return;
    const size_t fb = (size_t)(col / a.rb) * 12 * (size_t)a.Vol * (size_t)a.rb + (size_t)(col % a.rb);
    for (int v = 0; v < 4; ++v) {
        const int row = ts * 16 + M::row(l, v);
        if (row < a.Vol) a.X[fb + ((size_t)c * a.Vol + (size_t)row) * (size_t)a.rb] = mk<T>(xr[v], xi[v]);
    }
}

// ------------------------------------------------------------------ host side

namespace {

struct CoeffPlan {
    int ntr, nti, nti_run, nsplit, sites_per_split, ldr;
    size_t part_bytes;
};

// kpad: the row length of V (and of the partial sums); k: the columns in use.
// The split over the lattice (and so the workspace) follows kpad; only the
// eigenvector tiles holding columns below k are launched, so a basis filled
// column by column (the Arnoldi runs) is read only as far as it is filled;
// the finish reads rows below k.
CoeffPlan plan_coeff(int Vol, int kpad, int k, int nrhs) {
    CoeffPlan p;
    p.ntr = (nrhs + 15) / 16;
    p.nti = kpad / 16;
    p.nti_run = (k + 15) / 16;
    p.ldr = p.ntr * 16;
    const int tiles = p.ntr * p.nti;
    int want = (2048 + tiles - 1) / tiles;
    int maxsplit = (Vol + 63) / 64;
    p.nsplit = want < 1 ? 1 : (want > maxsplit ? maxsplit : want);
    int sps = (Vol + p.nsplit - 1) / p.nsplit;
    p.sites_per_split = (sps + 15) / 16 * 16;
    p.nsplit = (Vol + p.sites_per_split - 1) / p.sites_per_split;
    p.part_bytes = (size_t)p.nsplit * 2 * (size_t)kpad * (size_t)p.ldr * sizeof(double2);
    return p;
}

template <typename T>
int coeff_t(const mpmc_lattice &lat, const mpmc_defl &df, mpmc_shape sh, const void *b, const mpmc_noise *noise,
            double *zeta, double *omega, void *ws, void *stream) {
    const int Vol = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3];
    const CoeffPlan p = plan_coeff(Vol, df.kpad, df.k, sh.nrhs);
    CoeffArgs<T> a;
    a.Vol = Vol;
    a.kpad = df.kpad;
    a.nrhs = sh.nrhs;
    a.rb = sh.rb;
    a.ntr = p.ntr;
    a.sites_per_split = p.sites_per_split;
    a.V = (const cplx_t<T> *)df.V;
    a.b = (const cplx_t<T> *)b;
    a.key = noise ? noise_key(*noise) : 0ull;
    a.first = noise ? noise->first_sample : 0ull;
    a.off = noise ? noise->sample_offset : nullptr;
    a.part = (double2 *)ws;
    if (sh.nrhs == 1)
        hipLaunchKernelGGL(k_coeff_one<T>, dim3(p.nti_run, p.nsplit), dim3(kWaves * 64), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_coeff<T>, dim3(p.nti_run * p.ntr, p.nsplit), dim3(kWaves * 64), 0, (hipStream_t)stream,
                           a);
    if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    const int tot = df.k * sh.nrhs;
    hipLaunchKernelGGL(k_coeff_finish, dim3((unsigned)tot), dim3(kSumLanes), 0, (hipStream_t)stream,
                       (const double2 *)ws, p.nsplit, df.kpad, p.ldr, df.k, sh.nrhs, df.pair,
                       (const double2 *)df.scale, (double2 *)zeta, (double2 *)omega);
    return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

template <typename T>
int recon_t(const mpmc_lattice &lat, const mpmc_defl &df, mpmc_shape sh, const double *d, void *X, void *stream) {
    ReconArgs<T> a;
    a.Vol = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3];
    a.kpad = df.kpad;
    a.k = df.k;
    a.kact = (df.k + 3) / 4 * 4;
    a.nrhs = sh.nrhs;
    a.rb = sh.rb;
    a.ntr = (sh.nrhs + 15) / 16;
    a.nts = (a.Vol + 15) / 16;
    a.V = (const cplx_t<T> *)df.V;
    a.d = (const double2 *)d;
    a.X = (cplx_t<T> *)X;
    const int groups = (a.nts * 12 + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_recon<T>, dim3(groups, a.ntr), dim3(kWaves * 64), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

}  // namespace

size_t defl_ws_bytes(const mpmc_lattice &lat, const mpmc_defl &df, mpmc_shape sh) {
    const int Vol = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3];
    const CoeffPlan p = plan_coeff(Vol, df.kpad, df.k, sh.nrhs);
    // partials, then (PROJECT) omega/zeta scratch and the field V d
    return align256(p.part_bytes) + 2 * align256((size_t)df.k * sh.nrhs * sizeof(double2)) +
           align256(field_bytes(lat.dims, lat.prec, sh.nrhs));
}

int deflate_impl(const mpmc_lattice &lat, const mpmc_defl &df, int32_t mode, mpmc_shape sh, const void *b,
                 const mpmc_noise *noise, double *zeta, double *omega, double *d, void *X, void *ws, void *stream) {
    const int Vol = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3];
    const CoeffPlan p = plan_coeff(Vol, df.kpad, df.k, sh.nrhs);
    char *w = (char *)ws;
    void *part = w;
    w += align256(p.part_bytes);
    double *zs = (double *)w;
    w += align256((size_t)df.k * sh.nrhs * sizeof(double2));
    double *os = (double *)w;
    w += align256((size_t)df.k * sh.nrhs * sizeof(double2));
    void *xh = w;
    const bool f64 = lat.prec == MPMC_F64;
    int st = MPMC_OK;
    if (mode == MPMC_DEFL_COEFF) {
        return f64 ? coeff_t<double>(lat, df, sh, b, noise, zeta, omega, part, stream)
                   : coeff_t<float>(lat, df, sh, b, noise, zeta, omega, part, stream);
    }
    if (mode == MPMC_DEFL_RECON) {
        return f64 ? recon_t<double>(lat, df, sh, d, X, stream) : recon_t<float>(lat, df, sh, d, X, stream);
    }
    // PROJECT: zeta, omega; d = H^{-1} omega; xh = V d; X = b - A xh
    double *z = zeta ? zeta : zs;
    double *o = omega ? omega : os;
    st = f64 ? coeff_t<double>(lat, df, sh, b, noise, z, o, part, stream)
             : coeff_t<float>(lat, df, sh, b, noise, z, o, part, stream);
    if (st != MPMC_OK) return st;
    const int tot = df.k * sh.nrhs;
    hipLaunchKernelGGL(k_small_gemm, dim3((tot + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (const double2 *)df.hinv, (const double2 *)o, df.k, sh.nrhs, (double2 *)d);
    if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    st = f64 ? recon_t<double>(lat, df, sh, d, xh, stream) : recon_t<float>(lat, df, sh, d, xh, stream);
    if (st != MPMC_OK) return st;
    const uint64_t key = noise ? noise_key(*noise) : 0ull;
    const uint64_t first = noise ? noise->first_sample : 0ull;
    const uint64_t *off = noise ? noise->sample_offset : nullptr;
    return f64 ? residual_apply_t<double>(lat, sh, xh, b, key, first, off, X, stream)
               : residual_apply_t<float>(lat, sh, xh, b, key, first, off, X, stream);
}

}  // namespace mpmc
