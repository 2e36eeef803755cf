// Host-side launchers shared between the libmpmc translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/mpmc.h"

namespace mpmc {

// carve of the caller's workspace for one polynomial application
struct PolyWs {
    void *f[5];     // field buffers (2 for a single polynomial, 5 for a composite)
    void *part;     // dot partials, one complex FP64 per (workgroup, vector)
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline size_t field_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs) {
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    return V * 12 * (size_t)nrhs * (prec == MPMC_F64 ? 16 : 8);
}

// FP64 complex partial sums the polynomial workspace holds: one per (site
// block of 256 / rb sites, vector) for the field kernels, and at least one per
// (64 sites, vector), which covers every (t-chunk, xyz-block) of a t-sweep
// (blocks of at least 64 sites, at most Lt chunks)
inline size_t poly_part_count(size_t V, int nrhs, int rb) {
    const size_t spw = 256 / (size_t)rb;
    const size_t a = (V + spw - 1) / spw, b = (V + 63) / 64;
    return (a > b ? a : b) * (size_t)nrhs;
}
size_t poly_ws_bytes(const int32_t dims[4], int32_t prec, const mpmc_poly &poly, mpmc_shape sh);
PolyWs carve_poly_ws(const int32_t dims[4], int32_t prec, const mpmc_poly &poly, mpmc_shape sh, void *ws);

template <typename T> int wilson_apply_t(const mpmc_lattice &, mpmc_shape, const void *x, void *y, void *stream);
// out = b - A x, b a field or (b == nullptr) the noise (key, first)
template <typename T>
int residual_apply_t(const mpmc_lattice &, mpmc_shape, const void *x, const void *b, uint64_t key, uint64_t first,
                     const uint64_t *off,
                     void *out, void *stream);
// t-sweep Newton steps (an xyz-block per workgroup); see sweep.hip
struct SweepPlan {
    bool ok = false;       // the sweep applies to this lattice and batch
    bool halo = false;     // blocks smaller than the plane, with a halo in LDS (FP32)
    int B[3] = {0, 0, 0};  // block extents in x, y, z
    int Pb = 0, Hb = 0;    // block sites (= workgroup size) and halo sites
    int nbp = 1;           // blocks per plane
    size_t lds = 0;        // dynamic LDS bytes
    bool fills = false;    // the batch gives every CU a full workgroup's worth of threads
    bool busy = false;     // the workgroups, in t-chunks, cover the CUs (the sweep beats streaming)
    int nranked = 1;       // blocked planes: candidate blocks ranked by the plan's cost (rank option)
    int nch = 1;           // t-chunks: each workgroup walks Lt / nch planes
};
SweepPlan sweep_plan(const mpmc_lattice &lat, mpmc_shape sh);
int sweep_prepare_kernels();
template <typename T>
int sweep_newton_t(const mpmc_lattice &lat, mpmc_shape sh, const SweepPlan &plan, int n, const double *troots,
                   const void *x, bool x_is_noise, const void *bvec, uint64_t key, uint64_t first, const uint64_t *off,
                   double2 *part, double2 *bhy, void *w0, void *w1, void *yacc, void *stream,
                   const int32_t *colour = nullptr);

// count plain Newton steps w <- w - t_j A w (j = 0 .. count-1, no dot) of
// nrhs vectors from `in` (block width rb_in); outputs alternate w0, w1 at
// block width 1.  *out is the last output (in itself when count is 0).
template <typename T>
int sweep_chain_t(const mpmc_lattice &lat, mpmc_shape sh, const SweepPlan &plan, int count, const double *troots,
                  const void *in, int rb_in, void *w0, void *w1, const void **out, void *stream);

// process-wide kernel-selection options (mpmc_set_option); the batch builder
// and the autotuner set them around each enqueue and restore them after
extern int g_opt_sweep;
extern int g_opt_sweep_rank;
extern int g_opt_sweep_chunks;
extern int g_opt_hop_slab;
extern int g_opt_link_buf;

template <typename T>
int poly_apply_t(const mpmc_lattice &, const mpmc_poly &, mpmc_shape, const void *x, const mpmc_noise *noise, void *y,
                 double *bhy, const PolyWs &ws, void *stream);

// layout / noise kernels
template <typename T>
int copy_or_noise_t(const mpmc_lattice &lat, mpmc_shape sh, const void *x, uint64_t key, uint64_t first,
                    const uint64_t *off, void *out,
                    void *stream);
int pack_gauge_impl(const int32_t dims[4], int32_t prec, const double *canon, void *gauge, void *stream);
int pack_fields_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const double *canon, void *field, void *stream);
int unpack_fields_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const void *field, double *canon,
                       void *stream);
int counter_add_impl(uint64_t *counter, uint64_t inc, void *stream);
int probe_fill_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const int32_t *colour, int64_t first,
                    void *field, void *stream);
int gauge_unitarity_impl(const int32_t dims[4], int32_t prec, const void *gauge, double *out, void *stream);
int z4_fill_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const mpmc_noise &nz, void *field, void *stream);

// field utilities (Krylov set-up)
int field_axpby_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const double *alpha, const void *x,
                     const double *beta, void *y, void *stream);
size_t field_dot_ws_bytes(const int32_t dims[4], mpmc_shape sh);
int field_dot_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, const void *x, const void *y, double *out,
                   void *ws, void *stream);
int field_relayout_impl(const int32_t dims[4], int32_t prec, int32_t nrhs, const void *src, int32_t src_rb, void *dst,
                        int32_t dst_rb, void *stream);
int field_copy_vector_impl(const int32_t dims[4], int32_t prec, mpmc_shape ssh, const void *src, int32_t si,
                           mpmc_shape dsh, void *dst, int32_t di, void *stream);
int field_copy_bytes_impl(const void *src, void *dst, size_t bytes, void *stream);
int field_axpby_mixed_impl(const int32_t dims[4], mpmc_shape sh, int32_t xp, const double *alpha, const void *x,
                           int32_t yp, const double *beta, void *y, void *stream);
size_t block_dot_ws_bytes(const int32_t dims[4], mpmc_shape sh, int k);
int field_block_dot_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, int k, const void *basis, const void *x,
                         double *out, void *ws, void *stream);
int field_block_axpy_impl(const int32_t dims[4], int32_t prec, mpmc_shape sh, int k, const void *basis,
                          const double *coeff, int accumulate, void *y, void *stream);

// deflation
size_t defl_ws_bytes(const mpmc_lattice &lat, const mpmc_defl &df, mpmc_shape sh);
int deflate_impl(const mpmc_lattice &lat, const mpmc_defl &df, int32_t mode, mpmc_shape sh, const void *b,
                 const mpmc_noise *noise, double *zeta, double *omega, double *d, void *X, void *ws, void *stream);

// level
size_t level_ws_bytes(const mpmc_lattice &lat, const mpmc_level &lv, mpmc_shape sh);
int level_impl(const mpmc_lattice &lat, const mpmc_level &lv, mpmc_shape sh, const mpmc_noise &nz, double *samples,
               double *acc, void *ws, void *stream);
int stop_check_impl(const double *samples, int nrhs, int first, int every, double *state, void *stream);

}  // namespace mpmc
