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

template <typename T>
__global__ void k_axpby(const double2 *alpha, const cplx_t<T> *x, const double2 *beta, cplx_t<T> *y, int V, int rb,
                        int nrhs) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nrhs * 12 * (size_t)V;
    if (e >= total) return;
    const int j = (int)(e % (size_t)rb);
    const int nbk = (int)(e / ((size_t)rb * 12 * (size_t)V));
    const int r = nbk * rb + j;
    const double2 a = alpha[r];
    const cplx_t<T> xv = x[e];
    y[e] = beta != nullptr ? lin2_d<T>(a, xv, beta[r], y[e]) : cmul_d<T>(a, xv);
}

// partial inner products: workgroup covers 256/rb sites of one RHS block
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot_part(const cplx_t<T> *x, const cplx_t<T> *y, int V, int rb, int spw,
                                                     int nblk, double2 *part) {
    __shared__ double2 red[kBlock];
    const int L = (int)blockIdx.x;
    const int nbk = L / nblk, sblk = L % nblk;
    const int lane = (int)threadIdx.x, jr = lane & (rb - 1), ls = lane / rb;
    const int s = sblk * spw + ls;
    double re = 0.0, im = 0.0;
    if (s < V) {
        const int r = nbk * rb + jr;
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

__global__ void k_dot_finish(const double2 *part, int nblk, int rb, int nrhs, double2 *out) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= nrhs) return;
    const int nbk = r / rb, jr = r % rb;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double2 v = part[((size_t)nbk * nblk + b) * rb + jr];
        re += v.x;
        im += v.y;
    }
    out[r].x = re;
    out[r].y = im;
}

template <typename T>
__global__ void k_copy_vector(const cplx_t<T> *src, int src_rb, int src_r, cplx_t<T> *dst, int dst_rb, int dst_r, int V) {
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= 12 * V) return;
    const int c = e / V, s = e % V;
    dst[fidx(dst_r, c, s, V, dst_rb)] = src[fidx(src_r, c, s, V, src_rb)];
}

inline int st() { return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP; }

}  // namespace

int field_axpby_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const double *alpha, const void *x,
                     const double *beta, void *y, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t total = (size_t)sh.nrhs * 12 * V;
    const unsigned g = (unsigned)((total + 255) / 256);
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_axpby<double>, dim3(g), dim3(256), 0, (hipStream_t)stream, (const double2 *)alpha,
                           (const double2 *)x, (const double2 *)beta, (double2 *)y, V, sh.rb, sh.nrhs);
    else
        hipLaunchKernelGGL(k_axpby<float>, dim3(g), dim3(256), 0, (hipStream_t)stream, (const double2 *)alpha,
                           (const float2 *)x, (const double2 *)beta, (float2 *)y, V, sh.rb, sh.nrhs);
    return st();
}

size_t field_dot_ws_bytes(const int32_t dims[4], mpmc_shape sh) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const FieldTiling t = make_tiling(V, sh.nrhs, sh.rb);
    return align256((size_t)t.groups() * sh.rb * sizeof(double2));
}

int field_dot_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const void *x, const void *y, double *out,
                   void *ws, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const FieldTiling t = make_tiling(V, sh.nrhs, sh.rb);
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_dot_part<double>, dim3(t.groups()), dim3(kBlock), 0, (hipStream_t)stream,
                           (const double2 *)x, (const double2 *)y, V, sh.rb, t.spw, t.nblk, (double2 *)ws);
    else
        hipLaunchKernelGGL(k_dot_part<float>, dim3(t.groups()), dim3(kBlock), 0, (hipStream_t)stream,
                           (const float2 *)x, (const float2 *)y, V, sh.rb, t.spw, t.nblk, (double2 *)ws);
    if (hipGetLastError() != hipSuccess) return MPMC_EHIP;
    hipLaunchKernelGGL(k_dot_finish, dim3((sh.nrhs + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (const double2 *)ws, t.nblk, sh.rb, sh.nrhs, (double2 *)out);
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
