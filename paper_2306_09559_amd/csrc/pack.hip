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
