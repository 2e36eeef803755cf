// Field utilities for the Krylov set-up (Sec. 5, setup step 2): y = a x + b y
// per vector, FP64 inner products with a fixed-order reduction, and copies
// of single vectors between batches of different layouts (an Arnoldi basis
// is a batch with nrhs = rb = its padded width).
#include "common.hpp"
#include "internal.hpp"

namespace mpmc {

namespace {

// index of unknown (c, s) of vector r in a batch of block width rb
__device__ __forceinline__ size_t fidx(int r, int c, int s, int V, int rb) {
    return ((size_t)(r / rb) * 12 + (size_t)c) * (size_t)V * (size_t)rb + (size_t)s * (size_t)rb + (size_t)(r % rb);
}

// Element-wise kernels run on a grid (element of a component plane, component
// c, RHS block nbk): a plane of one RHS block holds V * rb elements (fewer
// than 2^29, the byte offsets of a plane fit 32 bits), rb is a power of two,
// so every index is formed without division (a 64-bit division per element,
// emulated in software, held a one-vector FP64 axpby on 24^3x48 to 0.2 TB/s).
struct PlaneIdx {
    size_t e;      // element index in the batch
    int r;         // vector
    unsigned i;    // element within the plane: site i >> lrb, lane i & (rb - 1)
    bool ok;
};
__device__ __forceinline__ PlaneIdx plane_idx(int V, int lrb) {
    PlaneIdx p;
    const unsigned per = (unsigned)V << lrb;
    p.i = blockIdx.x * blockDim.x + threadIdx.x;
    p.ok = p.i < per;
    const unsigned c = blockIdx.y, nbk = blockIdx.z;
    p.e = ((size_t)nbk * 12 + c) * (size_t)per + p.i;
    p.r = (int)((nbk << lrb) + (p.i & ((1u << lrb) - 1u)));
    return p;
}
// (at most 65535 RHS blocks: the launches check it)
inline dim3 plane_grid(int V, int rb, int nrhs) {
    return dim3((unsigned)(((size_t)V * rb + 255) / 256), 12u, (unsigned)(nrhs / rb));
}
inline int log2_pow2(int rb) {
    int l = 0;
    while ((1 << l) < rb) ++l;
    return l;
}

template <typename T>
__global__ void k_axpby(const double2 *alpha, const cplx_t<T> *x, const double2 *beta, cplx_t<T> *y, int V, int lrb) {
    const PlaneIdx q = plane_idx(V, lrb);
    if (!q.ok) return;
    const size_t e = q.e;
    const int r = q.r;
    const double2 a = alpha[r];
    const cplx_t<T> xv = x[e];
    y[e] = beta != nullptr ? lin2_d<T>(a, xv, beta[r], y[e]) : cmul_d<T>(a, xv);
}

constexpr int kDotRun = 4096;

// partial inner products: workgroup b of an RHS block covers the site tiles
// b, b + nrun, .. (256/rb sites each), so that an RHS block leaves at most
// nrun partials per vector (at block width 256 one site per tile: a partial
// per site made the finish read V strided values per vector)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot_part(const cplx_t<T> *x, const cplx_t<T> *y, int V, int rb, int spw,
                                                     int nblk, int nrun, double2 *part) {
    __shared__ double2 red[kBlock];
    const int L = (int)blockIdx.x;
    const int nbk = L / nrun, b0 = L % nrun;
    const int lane = (int)threadIdx.x, jr = lane & (rb - 1), ls = lane / rb;
    const int r = nbk * rb + jr;
    double re = 0.0, im = 0.0;
    for (int sblk = b0; sblk < nblk; sblk += nrun) {
        const int s = sblk * spw + ls;
        if (s >= V) break;
        for (int c = 0; c < 12; ++c) {
            const size_t ix = fidx(r, c, s, V, rb);
            const double xr = (double)x[ix].x, xi = (double)x[ix].y, yr = (double)y[ix].x, yi = (double)y[ix].y;
            re += xr * yr + xi * yi;
            im += xr * yi - xi * yr;
        }
    }
    red[lane].x = re;
    red[lane].y = im;
    __syncthreads();
    for (int stride = spw >> 1; stride > 0; stride >>= 1) {
        if (ls < stride) {
            red[lane].x += red[lane + stride * rb].x;
            red[lane].y += red[lane + stride * rb].y;
        }
        __syncthreads();
    }
    if (ls == 0) part[(size_t)L * rb + jr] = red[lane];
}

// one 64-lane workgroup per vector (sum_fixed)
__global__ void __launch_bounds__(kSumLanes) k_dot_finish(const double2 *part, int nblk, int rb, double2 *out) {
    const int r = (int)blockIdx.x;
    const int nbk = r / rb, jr = r % rb;
    const double2 *p = part + (size_t)nbk * (size_t)nblk * (size_t)rb + (size_t)jr;
    double2 tot[1];
    sum_fixed<1>(nblk, [&](int b, double2 (&v)[1]) { v[0] = p[(size_t)b * (size_t)rb]; }, tot);
    if (threadIdx.x == 0) out[r] = tot[0];
}

template <typename T>
__global__ void k_copy_vector(const cplx_t<T> *src, int src_rb, int src_r, cplx_t<T> *dst, int dst_rb, int dst_r, int V) {
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= 12 * V) return;
    const int c = e / V, s = e % V;
    dst[fidx(dst_r, c, s, V, dst_rb)] = src[fidx(src_r, c, s, V, src_rb)];
}

// a whole batch from block width src_rb to dst_rb, one thread per destination element
template <typename T>
__global__ void k_relayout(const cplx_t<T> *src, int lsrc, cplx_t<T> *dst, int ldst, int V) {
    const PlaneIdx q = plane_idx(V, ldst);
    if (!q.ok) return;
    const int s = (int)(q.i >> ldst), c = (int)blockIdx.y;
    const size_t per = (size_t)V << lsrc;
    const size_t from = ((size_t)(q.r >> lsrc) * 12 + (size_t)c) * per + ((size_t)s << lsrc) +
                        (size_t)(q.r & ((1 << lsrc) - 1));
    dst[q.e] = src[from];
}

// y = alpha x + beta y across precisions, coefficients applied in FP64
template <typename TX, typename TY>
__global__ void k_axpby_mixed(const double2 *alpha, const cplx_t<TX> *x, const double2 *beta, cplx_t<TY> *y, int V,
                              int lrb) {
    const PlaneIdx q = plane_idx(V, lrb);
    if (!q.ok) return;
    const size_t e = q.e;
    const int r = q.r;
    const double2 a = alpha[r];
    const double xr = (double)x[e].x, xi = (double)x[e].y;
    double re = a.x * xr - a.y * xi, im = a.x * xi + a.y * xr;
    if (beta != nullptr) {
        const double2 b = beta[r];
        const double yr = (double)y[e].x, yi = (double)y[e].y;
        re += b.x * yr - b.y * yi;
        im += b.x * yi + b.y * yr;
    }
    y[e] = mk<TY>((TY)re, (TY)im);
}

// Block inner products out[i][r] = (v_i)_r^H x_r: a workgroup covers the
// sites of tiles sb, sb + SB, ... of one RHS block for basis vectors
// i0 .. i0+7 (blockIdx.y = chunk), holding x in registers while it streams
// the basis vectors; partials per (RHS block, sb, i) are summed by
// k_block_dot_finish in a fixed order.
constexpr int kDotChunk = 8;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_block_dot(const cplx_t<T> *basis, size_t F, int k, const cplx_t<T> *x,
                                                      int V, int rb, int SB, double2 *part) {
    __shared__ double2 red[kBlock];
    const int spw = kBlock / rb;
    const int ntiles = (V + spw - 1) / spw;
    const int nbk = (int)blockIdx.x / SB, sb = (int)blockIdx.x % SB;
    const int i0 = (int)blockIdx.y * kDotChunk;
    const int lane = (int)threadIdx.x, jr = lane & (rb - 1), ls = lane / rb;
    const int r = nbk * rb + jr;
    double2 acc[kDotChunk];
#pragma unroll
    for (int ii = 0; ii < kDotChunk; ++ii) acc[ii] = make_double2(0.0, 0.0);
    for (int t = sb; t < ntiles; t += SB) {
        const int s = t * spw + ls;
        if (s >= V) continue;
        cplx_t<T> xv[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) xv[c] = x[fidx(r, c, s, V, rb)];
#pragma unroll
        for (int ii = 0; ii < kDotChunk; ++ii) {
            if (i0 + ii < k) {
                const cplx_t<T> *v = basis + (size_t)(i0 + ii) * F;
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const cplx_t<T> vv = v[fidx(r, c, s, V, rb)];
                    const double vr = (double)vv.x, vi = (double)vv.y, xr = (double)xv[c].x, xi = (double)xv[c].y;
                    re += vr * xr + vi * xi;
                    im += vr * xi - vi * xr;
                }
                acc[ii].x += re;
                acc[ii].y += im;
            }
        }
    }
    for (int ii = 0; ii < kDotChunk; ++ii) {
        if (i0 + ii >= k) break;   // uniform across the workgroup
        red[lane] = acc[ii];
        __syncthreads();
        for (int stride = spw >> 1; stride > 0; stride >>= 1) {
            if (ls < stride) {
                red[lane].x += red[lane + stride * rb].x;
                red[lane].y += red[lane + stride * rb].y;
            }
            __syncthreads();
        }
        if (ls == 0) part[(((size_t)nbk * SB + sb) * k + (i0 + ii)) * rb + jr] = red[lane];
        __syncthreads();
    }
}

// one 64-lane workgroup per (basis vector, vector) (sum_fixed)
__global__ void __launch_bounds__(kSumLanes) k_block_dot_finish(const double2 *part, int k, int rb, int nrhs, int SB,
                                                                double2 *out) {
    const int e = (int)blockIdx.x;
    const int i = e / nrhs, r = e % nrhs;
    const int nbk = r / rb, jr = r % rb;
    double2 tot[1];
    sum_fixed<1>(SB, [&](int sb, double2 (&v)[1]) { v[0] = part[(((size_t)nbk * SB + sb) * k + i) * rb + jr]; },
                 tot);
    if (threadIdx.x == 0) out[e] = tot[0];
}

// y = [y +] sum_i coeff[i][r] (v_i)_r, in FP64, rounded once
template <typename T>
__global__ void k_block_axpy(const cplx_t<T> *basis, size_t F, int k, const double2 *coeff, int accumulate,
                             cplx_t<T> *y, int V, int lrb, int nrhs) {
    const PlaneIdx q = plane_idx(V, lrb);
    if (!q.ok) return;
    const size_t e = q.e;
    const int r = q.r;
    double re = 0.0, im = 0.0;
    if (accumulate) {
        re = (double)y[e].x;
        im = (double)y[e].y;
    }
    for (int i = 0; i < k; ++i) {
        const double2 a = coeff[(size_t)i * nrhs + r];
        const cplx_t<T> v = basis[(size_t)i * F + e];
        const double vr = (double)v.x, vi = (double)v.y;
        re += a.x * vr - a.y * vi;
        im += a.x * vi + a.y * vr;
    }
    y[e] = mk<T>((T)re, (T)im);
}

// site-block groups of the block dot: enough workgroups to fill the chip
int block_dot_groups(int V, mpmc_shape sh, int k) {
    const int spw = kBlock / sh.rb;
    const int ntiles = (V + spw - 1) / spw;
    const int nb = sh.nrhs / sh.rb;
    const int chunks = (k + kDotChunk - 1) / kDotChunk;
    int SB = 2048 / (nb * chunks);
    if (SB < 1) SB = 1;
    if (SB > ntiles) SB = ntiles;
    return SB;
}

inline int st() { return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP; }

}  // namespace

int field_axpby_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const double *alpha, const void *x,
                     const double *beta, void *y, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    if (sh.nrhs / sh.rb > 65535) return MPMC_EUNSUPPORTED;
    const dim3 g = plane_grid(V, sh.rb, sh.nrhs);
    const int lrb = log2_pow2(sh.rb);
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_axpby<double>, g, dim3(256), 0, (hipStream_t)stream, (const double2 *)alpha,
                           (const double2 *)x, (const double2 *)beta, (double2 *)y, V, lrb);
    else
        hipLaunchKernelGGL(k_axpby<float>, g, dim3(256), 0, (hipStream_t)stream, (const double2 *)alpha,
                           (const float2 *)x, (const double2 *)beta, (float2 *)y, V, lrb);
    return st();
}

// workgroups per RHS block of the inner products (and partials per vector)
static int dot_nrun(const FieldTiling &t) { return t.nblk < kDotRun ? t.nblk : kDotRun; }

size_t field_dot_ws_bytes(const int32_t dims[4], mpmc_shape sh) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const FieldTiling t = make_tiling(V, sh.nrhs, sh.rb);
    return align256((size_t)t.nb * dot_nrun(t) * sh.rb * sizeof(double2));
}

int field_dot_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const void *x, const void *y, double *out,
                   void *ws, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const FieldTiling t = make_tiling(V, sh.nrhs, sh.rb);
    const int nrun = dot_nrun(t);
    const dim3 grid((unsigned)(t.nb * nrun));
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_dot_part<double>, grid, dim3(kBlock), 0, (hipStream_t)stream, (const double2 *)x,
                           (const double2 *)y, V, sh.rb, t.spw, t.nblk, nrun, (double2 *)ws);
    else
        hipLaunchKernelGGL(k_dot_part<float>, grid, dim3(kBlock), 0, (hipStream_t)stream, (const float2 *)x,
                           (const float2 *)y, V, sh.rb, t.spw, t.nblk, nrun, (double2 *)ws);
    if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    hipLaunchKernelGGL(k_dot_finish, dim3(sh.nrhs), dim3(kSumLanes), 0, (hipStream_t)stream, (const double2 *)ws,
                       nrun, sh.rb, (double2 *)out);
    return st();
}

int field_axpby_mixed_impl(const int32_t dims[4], mpmc_shape sh, int32_t xp, const double *alpha, const void *x,
                           int32_t yp, const double *beta, void *y, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    if (sh.nrhs / sh.rb > 65535) return MPMC_EUNSUPPORTED;
    const dim3 g = plane_grid(V, sh.rb, sh.nrhs);
    const int lrb = log2_pow2(sh.rb);
    const double2 *a = (const double2 *)alpha, *b = (const double2 *)beta;
    hipStream_t s = (hipStream_t)stream;
    if (xp == MPMC_F64 && yp == MPMC_F64)
        hipLaunchKernelGGL((k_axpby_mixed<double, double>), g, dim3(256), 0, s, a, (const double2 *)x, b,
                           (double2 *)y, V, lrb);
    else if (xp == MPMC_F64)
        hipLaunchKernelGGL((k_axpby_mixed<double, float>), g, dim3(256), 0, s, a, (const double2 *)x, b,
                           (float2 *)y, V, lrb);
    else if (yp == MPMC_F64)
        hipLaunchKernelGGL((k_axpby_mixed<float, double>), g, dim3(256), 0, s, a, (const float2 *)x, b,
                           (double2 *)y, V, lrb);
    else
        hipLaunchKernelGGL((k_axpby_mixed<float, float>), g, dim3(256), 0, s, a, (const float2 *)x, b,
                           (float2 *)y, V, lrb);
    return st();
}

size_t block_dot_ws_bytes(const int32_t dims[4], mpmc_shape sh, int k) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const int SB = block_dot_groups(V, sh, k);
    return align256((size_t)(sh.nrhs / sh.rb) * SB * (size_t)k * sh.rb * sizeof(double2));
}

int field_block_dot_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, int k, const void *basis, const void *x,
                         double *out, void *ws, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t F = (size_t)sh.nrhs * 12 * (size_t)V;
    const int SB = block_dot_groups(V, sh, k);
    const dim3 grid((unsigned)((sh.nrhs / sh.rb) * SB), (unsigned)((k + kDotChunk - 1) / kDotChunk));
    hipStream_t s = (hipStream_t)stream;
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_block_dot<double>, grid, dim3(kBlock), 0, s, (const double2 *)basis, F, k,
                           (const double2 *)x, V, sh.rb, SB, (double2 *)ws);
    else
        hipLaunchKernelGGL(k_block_dot<float>, grid, dim3(kBlock), 0, s, (const float2 *)basis, F, k,
                           (const float2 *)x, V, sh.rb, SB, (double2 *)ws);
    if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    hipLaunchKernelGGL(k_block_dot_finish, dim3((unsigned)(k * sh.nrhs)), dim3(kSumLanes), 0, s,
                       (const double2 *)ws, k, sh.rb, sh.nrhs, SB, (double2 *)out);
    return st();
}

int field_block_axpy_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, int k, const void *basis,
                          const double *coeff, int accumulate, void *y, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t F = (size_t)sh.nrhs * 12 * (size_t)V;
    if (sh.nrhs / sh.rb > 65535) return MPMC_EUNSUPPORTED;
    const dim3 g = plane_grid(V, sh.rb, sh.nrhs);
    const int lrb = log2_pow2(sh.rb);
    hipStream_t s = (hipStream_t)stream;
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_block_axpy<double>, g, dim3(256), 0, s, (const double2 *)basis, F, k,
                           (const double2 *)coeff, accumulate, (double2 *)y, V, lrb, sh.nrhs);
    else
        hipLaunchKernelGGL(k_block_axpy<float>, g, dim3(256), 0, s, (const float2 *)basis, F, k,
                           (const double2 *)coeff, accumulate, (float2 *)y, V, lrb, sh.nrhs);
    return st();
}

int field_relayout_impl(const int32_t dims[4], int32_t prec, int32_t nrhs, const void *src, int32_t src_rb, void *dst,
                        int32_t dst_rb, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    if (nrhs / dst_rb > 65535) return MPMC_EUNSUPPORTED;
    const dim3 g = plane_grid(V, dst_rb, nrhs);
    const int ls = log2_pow2(src_rb), ld = log2_pow2(dst_rb);
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_relayout<double>, g, dim3(256), 0, (hipStream_t)stream, (const double2 *)src, ls,
                           (double2 *)dst, ld, V);
    else
        hipLaunchKernelGGL(k_relayout<float>, g, dim3(256), 0, (hipStream_t)stream, (const float2 *)src, ls,
                           (float2 *)dst, ld, V);
    return st();
}

// 16-byte elements i < n, grid-stride: four workgroups per CU streaming
// with the nontemporal hint measured fastest for large copies (5.9 TB/s at
// 1 GiB against 4.6-5.4 TB/s with more workgroups or cached accesses)
__global__ void __launch_bounds__(256) k_copy_bytes(const double2 *__restrict__ x, double2 *__restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double2 v;
        v.x = __builtin_nontemporal_load(&x[i].x);
        v.y = __builtin_nontemporal_load(&x[i].y);
        __builtin_nontemporal_store(v.x, &y[i].x);
        __builtin_nontemporal_store(v.y, &y[i].y);
    }
}

int field_copy_bytes_impl(const void *src, void *dst, size_t bytes, void *stream) {
    const size_t n = bytes / 16;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;                       // the grid size only: four workgroups per CU of an MI355X
    const size_t want = (n + 255) / 256, cap = (size_t)4 * (size_t)(cus > 0 ? cus : 256);
    const unsigned g = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(k_copy_bytes, dim3(g), dim3(256), 0, (hipStream_t)stream, (const double2 *)src, (double2 *)dst,
                       n);
    return st();
}

int field_copy_vector_impl(const int32_t dims[4], int32_t prec, mpmc_shape ssh, const void *src, int32_t si,
                           mpmc_shape dsh, void *dst, int32_t di, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const unsigned g = (unsigned)((12 * V + 255) / 256);
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_copy_vector<double>, dim3(g), dim3(256), 0, (hipStream_t)stream, (const double2 *)src,
                           ssh.rb, si, (double2 *)dst, dsh.rb, di, V);
    else
        hipLaunchKernelGGL(k_copy_vector<float>, dim3(g), dim3(256), 0, (hipStream_t)stream, (const float2 *)src,
                           ssh.rb, si, (float2 *)dst, dsh.rb, di, V);
    return st();
}

}  // namespace mpmc
