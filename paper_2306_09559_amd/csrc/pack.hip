// Layout conversion (canonical complex128 <-> library layouts) and Z4 noise
// materialisation.  Elementwise, one thread per complex number, coalesced on
// the library side.
#include "common.hpp"
#include "internal.hpp"

namespace mpmc {

namespace {

// canonical (N, V, 12) complex128 -> field layout ((nb*12 + c)*V + s)*rb + j
template <typename T>
__global__ void k_pack_fields(const double2 *canon, cplx_t<T> *field, int V, int rb, int nrhs) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;     // field-layout index
    const size_t total = (size_t)nrhs * 12 * (size_t)V;
    if (e >= total) return;
    const int j = (int)(e % (size_t)rb);
    size_t q = e / (size_t)rb;
    const int s = (int)(q % (size_t)V);
    q /= (size_t)V;
    const int c = (int)(q % 12);
    const int nbk = (int)(q / 12);
    const int r = nbk * rb + j;
    const double2 v = canon[((size_t)r * V + s) * 12 + c];
    field[e] = mk<T>((T)v.x, (T)v.y);
}

template <typename T>
__global__ void k_unpack_fields(const cplx_t<T> *field, double2 *canon, int V, int rb, int nrhs) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nrhs * 12 * (size_t)V;
    if (e >= total) return;
    const int j = (int)(e % (size_t)rb);
    size_t q = e / (size_t)rb;
    const int s = (int)(q % (size_t)V);
    q /= (size_t)V;
    const int c = (int)(q % 12);
    const int nbk = (int)(q / 12);
    const int r = nbk * rb + j;
    const cplx_t<T> v = field[e];
    double2 o;
    o.x = (double)v.x;
    o.y = (double)v.y;
    canon[((size_t)r * V + s) * 12 + c] = o;
}

// canonical (4, V, 3, 3) -> [mu][e][V]
template <typename T>
__global__ void k_pack_gauge(const double2 *canon, cplx_t<T> *gauge, int V) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)36 * V;
    if (e >= total) return;
    const int s = (int)(e % (size_t)V);
    const int me = (int)(e / (size_t)V);        // mu*9 + element
    const int mu = me / 9, el = me % 9;
    const double2 v = canon[((size_t)mu * V + s) * 9 + el];
    gauge[e] = mk<T>((T)v.x, (T)v.y);
}

template <typename T>
__global__ void k_probe_fill(cplx_t<T> *field, const int32_t *colour, int V, int rb, int nrhs, int64_t first) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nrhs * 12 * (size_t)V;
    if (e >= total) return;
    const int j = (int)(e % (size_t)rb);
    size_t q = e / (size_t)rb;
    const int s = (int)(q % (size_t)V);
    q /= (size_t)V;
    const int c = (int)(q % 12);
    const int nbk = (int)(q / 12);
    const int64_t p = first + (int64_t)(nbk * rb + j);
    const bool on = (c == (int)(p % 12)) && ((int64_t)colour[s] == p / 12);
    field[e] = mk<T>(on ? T(1) : T(0), T(0));
}

__global__ void k_counter_add(uint64_t *c, uint64_t inc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = c[0] + inc;
}

template <typename T>
__global__ void k_z4_fill(cplx_t<T> *field, int V, int rb, int nrhs, uint64_t key, uint64_t first,
                          const uint64_t *off) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nrhs * 12 * (size_t)V;
    if (e >= total) return;
    const int j = (int)(e % (size_t)rb);
    size_t q = e / (size_t)rb;
    const int s = (int)(q % (size_t)V);
    q /= (size_t)V;
    const int c = (int)(q % 12);
    const int nbk = (int)(q / 12);
    const uint64_t S = sample_state(key, sample_base(first, off) + (uint64_t)(nbk * rb + j));
    field[e] = z4_value<T>(z4_code(S, 12u * (unsigned)s + (unsigned)c));
}

template <typename T>
__global__ void k_copy(const cplx_t<T> *src, cplx_t<T> *dst, size_t total) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < total) dst[e] = src[e];
}

inline unsigned nblocks(size_t total, int thr) { return (unsigned)((total + thr - 1) / thr); }

inline int last_status() { return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP; }

}  // namespace

int pack_gauge_impl(const int32_t dims[4], int32_t prec, const double *canon, void *gauge, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t total = (size_t)36 * V;
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_pack_gauge<double>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)canon, (double2 *)gauge, V);
    else
        hipLaunchKernelGGL(k_pack_gauge<float>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)canon, (float2 *)gauge, V);
    return last_status();
}

int pack_fields_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const double *canon, void *field, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t total = (size_t)sh.nrhs * 12 * V;
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_pack_fields<double>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)canon, (double2 *)field, V, sh.rb, sh.nrhs);
    else
        hipLaunchKernelGGL(k_pack_fields<float>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)canon, (float2 *)field, V, sh.rb, sh.nrhs);
    return last_status();
}

int unpack_fields_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const void *field, double *canon,
                       void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t total = (size_t)sh.nrhs * 12 * V;
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_unpack_fields<double>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)field, (double2 *)canon, V, sh.rb, sh.nrhs);
    else
        hipLaunchKernelGGL(k_unpack_fields<float>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const float2 *)field, (double2 *)canon, V, sh.rb, sh.nrhs);
    return last_status();
}

// Deviation of the links from SU(3): one workgroup strides over all 4V
// links, each thread keeps its maxima, and a fixed-order tree combines them.
template <typename T>
__global__ void __launch_bounds__(1024) k_unitarity(const cplx_t<T> *g, int V, double *out) {
    __shared__ double red[2][1024];
    double du = 0.0, dd = 0.0;
    for (int l = (int)threadIdx.x; l < 4 * V; l += (int)blockDim.x) {
        const int mu = l / V, s = l % V;
        double ur[9], ui[9];
        for (int e = 0; e < 9; ++e) {
            const cplx_t<T> v = g[(size_t)(mu * 9 + e) * V + s];
            ur[e] = (double)v.x;
            ui[e] = (double)v.y;
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double re = 0.0, im = 0.0;          // (U U^H)_ab = sum_c U_ac conj(U_bc)
                for (int c = 0; c < 3; ++c) {
                    re += ur[3 * a + c] * ur[3 * b + c] + ui[3 * a + c] * ui[3 * b + c];
                    im += ui[3 * a + c] * ur[3 * b + c] - ur[3 * a + c] * ui[3 * b + c];
                }
                if (a == b) re -= 1.0;
                du = fmax(du, sqrt(re * re + im * im));
            }
        // det U by the first row's cofactors
        double dr = 0.0, di = 0.0;
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const double mr = ur[3 + c1] * ur[6 + c2] - ui[3 + c1] * ui[6 + c2] - (ur[3 + c2] * ur[6 + c1] - ui[3 + c2] * ui[6 + c1]);
            const double mi = ur[3 + c1] * ui[6 + c2] + ui[3 + c1] * ur[6 + c2] - (ur[3 + c2] * ui[6 + c1] + ui[3 + c2] * ur[6 + c1]);
            dr += ur[c] * mr - ui[c] * mi;
            di += ur[c] * mi + ui[c] * mr;
        }
        dd = fmax(dd, sqrt((dr - 1.0) * (dr - 1.0) + di * di));
    }
    red[0][threadIdx.x] = du;
    red[1][threadIdx.x] = dd;
    __syncthreads();
    for (int st = (int)blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + st]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

int gauge_unitarity_impl(const int32_t dims[4], int32_t prec, const void *gauge, double *out, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_unitarity<double>, dim3(1), dim3(1024), 0, (hipStream_t)stream, (const double2 *)gauge, V,
                           out);
    else
        hipLaunchKernelGGL(k_unitarity<float>, dim3(1), dim3(1024), 0, (hipStream_t)stream, (const float2 *)gauge, V,
                           out);
    return last_status();
}

int probe_fill_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const int32_t *colour, int64_t first,
                    void *field, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t total = (size_t)sh.nrhs * 12 * V;
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_probe_fill<double>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (double2 *)field, colour, V, sh.rb, sh.nrhs, first);
    else
        hipLaunchKernelGGL(k_probe_fill<float>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (float2 *)field, colour, V, sh.rb, sh.nrhs, first);
    return last_status();
}

int counter_add_impl(uint64_t *counter, uint64_t inc, void *stream) {
    hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(64), 0, (hipStream_t)stream, counter, inc);
    return last_status();
}

int z4_fill_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const mpmc_noise &nz, void *field, void *stream) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t total = (size_t)sh.nrhs * 12 * V;
    const uint64_t key = noise_key(nz);
    if (prec == MPMC_F64)
        hipLaunchKernelGGL(k_z4_fill<double>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (double2 *)field, V, sh.rb, sh.nrhs, key, nz.first_sample, nz.sample_offset);
    else
        hipLaunchKernelGGL(k_z4_fill<float>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (float2 *)field, V, sh.rb, sh.nrhs, key, nz.first_sample, nz.sample_offset);
    return last_status();
}

template <typename T>
int copy_or_noise_t(const mpmc_lattice &lat, mpmc_shape sh, const void *x, uint64_t key, uint64_t first,
                    const uint64_t *off, void *out,
                    void *stream) {
    const int V = lat.dims[0] * lat.dims[1] * lat.dims[2] * lat.dims[3];
    const size_t total = (size_t)sh.nrhs * 12 * V;
    if (x == nullptr)
        hipLaunchKernelGGL(k_z4_fill<T>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (cplx_t<T> *)out, V, sh.rb, sh.nrhs, key, first, off);
    else
        hipLaunchKernelGGL(k_copy<T>, dim3(nblocks(total, 256)), dim3(256), 0, (hipStream_t)stream,
                           (const cplx_t<T> *)x, (cplx_t<T> *)out, total);
    return last_status();
}

template int copy_or_noise_t<double>(const mpmc_lattice &, mpmc_shape, const void *, uint64_t, uint64_t,
                                     const uint64_t *, void *, void *);
template int copy_or_noise_t<float>(const mpmc_lattice &, mpmc_shape, const void *, uint64_t, uint64_t,
                                    const uint64_t *, void *, void *);

}  // namespace mpmc
