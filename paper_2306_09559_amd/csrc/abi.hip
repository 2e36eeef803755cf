// The extern "C" boundary of libmpmc: argument validation on the host,
// workspace sizing and dispatch to the precision-specific launchers.
#include <stdio.h>

#include "common.hpp"
#include "internal.hpp"

namespace mpmc {

int g_opt_sweep = 2;
int g_opt_sweep_rank = 0;
int g_opt_sweep_chunks = 0;
int g_opt_hop_slab = 1;
int g_opt_link_buf = 1;

size_t poly_ws_bytes(const int32_t dims[4], int32_t prec, const mpmc_poly &poly, mpmc_shape sh) {
    const size_t fb = align256(field_bytes(dims, prec, sh.nrhs));
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t part = align256(poly_part_count((size_t)V, sh.nrhs, sh.rb) * sizeof(double2));
    const int nf = poly.n_out > 0 ? 5 : (poly.n_in > 1 ? 2 : 0);
    return (size_t)nf * fb + part;
}

PolyWs carve_poly_ws(const int32_t dims[4], int32_t prec, const mpmc_poly &poly, mpmc_shape sh, void *ws) {
    PolyWs p{};
    const size_t fb = align256(field_bytes(dims, prec, sh.nrhs));
    const int nf = poly.n_out > 0 ? 5 : (poly.n_in > 1 ? 2 : 0);
    char *w = (char *)ws;
    for (int i = 0; i < nf; ++i) p.f[i] = w + (size_t)i * fb;
    p.part = w + (size_t)nf * fb;
    return p;
}

}  // namespace mpmc

using namespace mpmc;

namespace {

bool valid_dims(const int32_t *dims) {
    if (!dims) return false;
    long long V = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 1) return false;
        V *= dims[d];
    }
    return V * 12 < (1LL << 31);
}

bool valid_prec(int32_t p) { return p == MPMC_F64 || p == MPMC_F32; }

bool valid_shape(mpmc_shape s) {
    if (s.nrhs < 1 || s.rb < 1 || s.rb > 256) return false;
    if ((s.rb & (s.rb - 1)) != 0) return false;
    return s.nrhs % s.rb == 0;
}

// the field kernels address one component plane of an RHS block with 32-bit
// byte offsets: V * rb * sizeof(complex) must stay below 4 GiB
bool plane_fits(const int32_t *dims, int32_t prec, mpmc_shape s) {
    const unsigned long long V = (unsigned long long)dims[0] * dims[1] * dims[2] * dims[3];
    return V * (unsigned long long)s.rb * (prec == MPMC_F64 ? 16ull : 8ull) < (1ull << 32);
}

int check_lattice(const mpmc_lattice *lat) {
    if (!lat || !valid_dims(lat->dims) || !lat->gauge) return MPMC_EINVAL;
    if (!valid_prec(lat->prec)) return MPMC_EUNSUPPORTED;
    if (lat->antiperiodic_t != 0 && lat->antiperiodic_t != 1) return MPMC_EINVAL;
    if (lat->link_rows != 0 && lat->link_rows != 2 && lat->link_rows != 3) return MPMC_EINVAL;
    return MPMC_OK;
}

int check_poly(const mpmc_poly *p) {
    if (!p || p->n_in < 1 || !p->inv_roots_in || p->n_out < 0) return MPMC_EINVAL;
    if (p->n_out > 0 && !p->inv_roots_out) return MPMC_EINVAL;
    return MPMC_OK;
}

int check_defl(const mpmc_defl *d, bool need_hinv) {
    if (!d || d->k < 1 || d->kpad < d->k || d->kpad % 16 != 0 || d->kpad > 256) return MPMC_EINVAL;
    if (!d->V || !d->pair || !d->scale) return MPMC_EINVAL;
    if (need_hinv && !d->hinv) return MPMC_EINVAL;
    return MPMC_OK;
}

int check_ws(void *ws, size_t have, size_t need) {
    if (have < need) return MPMC_EWORKSPACE;
    if (need > 0 && !ws) return MPMC_EINVAL;
    return MPMC_OK;
}

#define MPMC_TRY(x)                       \
    do {                                  \
        const int _s = (x);               \
        if (_s != MPMC_OK) return _s;     \
    } while (0)

}  // namespace

extern "C" {

const char *mpmc_status_string(int status) {
    switch (status) {
    case MPMC_OK: return "ok";
    case MPMC_EINVAL: return "invalid argument (null pointer, size or layout out of range)";
    case MPMC_EUNSUPPORTED: return "unsupported precision, mode or operator kind";
    case MPMC_EWORKSPACE: return "workspace smaller than the required size";
    case MPMC_EHIP: return "HIP runtime or kernel launch failure";
    case MPMC_ESINGULAR: return "singular small dense system (zero pivot)";
    case MPMC_ENOTCONVERGED: return "iteration did not reach its tolerance";
    default: return "unknown status";
    }
}

const char *mpmc_build_info(void) { return "libmpmc 0.1 gfx950"; }

int mpmc_set_option(int32_t option, int32_t value) {
    switch (option) {
    case MPMC_OPT_PLANE_SWEEP:
        if (value < 0 || value > 2) return MPMC_EINVAL;
        g_opt_sweep = value;
        return MPMC_OK;
    case MPMC_OPT_SWEEP_RANK:
        if (value < 0 || value > 63) return MPMC_EINVAL;
        g_opt_sweep_rank = value;
        return MPMC_OK;
    case MPMC_OPT_HOP_SLAB:
        if (value != 0 && value != 1) return MPMC_EINVAL;
        g_opt_hop_slab = value;
        return MPMC_OK;
    case MPMC_OPT_LINK_BUF:
        if (value != 0 && value != 1) return MPMC_EINVAL;
        g_opt_link_buf = value;
        return MPMC_OK;
    case MPMC_OPT_SWEEP_CHUNKS:
        if (value < 0 || value > 1024) return MPMC_EINVAL;
        g_opt_sweep_chunks = value;
        return MPMC_OK;
    default: return MPMC_EUNSUPPORTED;
    }
}

int mpmc_counter_add(uint64_t *counter, uint64_t increment, void *stream) {
    if (!counter) return MPMC_EINVAL;
    return counter_add_impl(counter, increment, stream);
}

int mpmc_gauge_unitarity(const int32_t dims[4], int32_t prec, const void *gauge, double *out, void *stream) {
    if (!valid_dims(dims) || !gauge || !out) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return gauge_unitarity_impl(dims, prec, gauge, out, stream);
}

int mpmc_sweep_plan(const mpmc_lattice *lat, mpmc_shape shape, int32_t *out) {
    MPMC_TRY(check_lattice(lat));
    if (!valid_shape(shape) || !out) return MPMC_EINVAL;
    const SweepPlan p = sweep_plan(*lat, shape);
    const int32_t v[9] = {p.ok ? 1 : 0, p.halo ? 1 : 0, p.B[0], p.B[1], p.B[2], p.Pb, p.Hb, p.nbp, p.nch};
    for (int i = 0; i < 9; ++i) out[i] = v[i];
    return MPMC_OK;
}

int mpmc_probe_fill(const int32_t dims[4], int32_t prec, mpmc_shape shape, const int32_t *colour,
                    int64_t first_probe, void *field, void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !colour || !field || first_probe < 0) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return probe_fill_impl(dims, prec, shape, colour, first_probe, field, stream);
}

int mpmc_pack_gauge(const int32_t dims[4], int32_t prec, const double *canon, void *gauge, void *stream) {
    if (!valid_dims(dims) || !canon || !gauge) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return pack_gauge_impl(dims, prec, canon, gauge, stream);
}

int mpmc_pack_fields(const int32_t dims[4], int32_t prec, mpmc_shape shape, const double *canon, void *field,
                     void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !canon || !field) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return pack_fields_impl(dims, prec, shape, canon, field, stream);
}

int mpmc_unpack_fields(const int32_t dims[4], int32_t prec, mpmc_shape shape, const void *field, double *canon,
                       void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !canon || !field) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return unpack_fields_impl(dims, prec, shape, field, canon, stream);
}

int mpmc_z4_fill(const int32_t dims[4], int32_t prec, mpmc_shape shape, const mpmc_noise *noise, void *field,
                 void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !noise || !field) return MPMC_EINVAL;
    if (noise->probe_colour) return MPMC_EUNSUPPORTED;          // mpmc_probe_fill writes probe vectors
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return z4_fill_impl(dims, prec, shape, *noise, field, stream);
}

int mpmc_wilson_apply(const mpmc_lattice *lat, mpmc_shape shape, const void *x, void *y, void *stream) {
    MPMC_TRY(check_lattice(lat));
    if (!valid_shape(shape) || !plane_fits(lat->dims, lat->prec, shape) || !x || !y || x == y) return MPMC_EINVAL;
    return lat->prec == MPMC_F64 ? wilson_apply_t<double>(*lat, shape, x, y, stream)
                                 : wilson_apply_t<float>(*lat, shape, x, y, stream);
}

int mpmc_field_axpby(const int32_t dims[4], int32_t prec, mpmc_shape shape, const double *alpha, const void *x,
                     const double *beta, void *y, void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !alpha || !x || !y) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    return field_axpby_impl(dims, prec, shape, alpha, x, beta, y, stream);
}

size_t mpmc_field_dot_workspace_size(const int32_t dims[4], mpmc_shape shape) {
    if (!valid_dims(dims) || !valid_shape(shape)) return 0;
    return field_dot_ws_bytes(dims, shape);
}

int mpmc_field_dot(const int32_t dims[4], int32_t prec, mpmc_shape shape, const void *x, const void *y, double *out,
                   void *ws, size_t ws_bytes, void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !x || !y || !out) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    MPMC_TRY(check_ws(ws, ws_bytes, field_dot_ws_bytes(dims, shape)));
    return field_dot_impl(dims, prec, shape, x, y, out, ws, stream);
}

int mpmc_field_axpby_mixed(const int32_t dims[4], mpmc_shape shape, int32_t x_prec, const double *alpha,
                           const void *x, int32_t y_prec, const double *beta, void *y, void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || !alpha || !x || !y) return MPMC_EINVAL;
    if (!valid_prec(x_prec) || !valid_prec(y_prec)) return MPMC_EUNSUPPORTED;
    // x and y must not overlap (the sizes of the two precisions differ)
    const size_t xb = field_bytes(dims, x_prec, shape.nrhs), yb = field_bytes(dims, y_prec, shape.nrhs);
    const char *xc = (const char *)x, *yc = (const char *)y;
    if (xc < yc + yb && yc < xc + xb) return MPMC_EINVAL;
    return field_axpby_mixed_impl(dims, shape, x_prec, alpha, x, y_prec, beta, y, stream);
}

size_t mpmc_field_block_dot_workspace_size(const int32_t dims[4], mpmc_shape shape, int32_t k) {
    if (!valid_dims(dims) || !valid_shape(shape) || k < 1) return 0;
    return block_dot_ws_bytes(dims, shape, k);
}

int mpmc_field_block_dot(const int32_t dims[4], int32_t prec, mpmc_shape shape, int32_t k, const void *basis,
                         const void *x, double *out, void *ws, size_t ws_bytes, void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || k < 1 || !basis || !x || !out) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    MPMC_TRY(check_ws(ws, ws_bytes, block_dot_ws_bytes(dims, shape, k)));
    return field_block_dot_impl(dims, prec, shape, k, basis, x, out, ws, stream);
}

int mpmc_field_block_axpy(const int32_t dims[4], int32_t prec, mpmc_shape shape, int32_t k, const void *basis,
                          const double *coeff, int32_t accumulate, void *y, void *stream) {
    if (!valid_dims(dims) || !valid_shape(shape) || k < 1 || !basis || !coeff || !y) return MPMC_EINVAL;
    if (accumulate != 0 && accumulate != 1) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    const size_t fb = field_bytes(dims, prec, shape.nrhs);
    const char *bc = (const char *)basis, *yc = (const char *)y;
    if (yc < bc + (size_t)k * fb && bc < yc + fb) return MPMC_EINVAL;
    return field_block_axpy_impl(dims, prec, shape, k, basis, coeff, accumulate, y, stream);
}

int mpmc_field_copy_vector(const int32_t dims[4], int32_t prec, mpmc_shape src_shape, const void *src,
                           int32_t src_index, mpmc_shape dst_shape, void *dst, int32_t dst_index, void *stream) {
    if (!valid_dims(dims) || !valid_shape(src_shape) || !valid_shape(dst_shape) || !src || !dst) return MPMC_EINVAL;
    if (!valid_prec(prec)) return MPMC_EUNSUPPORTED;
    if (src_index < 0 || src_index >= src_shape.nrhs || dst_index < 0 || dst_index >= dst_shape.nrhs) return MPMC_EINVAL;
    if (src == dst) return MPMC_EINVAL;
    return field_copy_vector_impl(dims, prec, src_shape, src, src_index, dst_shape, dst, dst_index, stream);
}

int mpmc_field_copy_bytes(const void *src, void *dst, size_t bytes, void *stream) {
    if (bytes == 0) return MPMC_OK;
    if (!src || !dst || bytes % 16 != 0) return MPMC_EINVAL;
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return MPMC_EINVAL;
    const char *s = (const char *)src, *d = (const char *)dst;
    if (d < s + bytes && s < d + bytes) return MPMC_EINVAL;
    return field_copy_bytes_impl(src, dst, bytes, stream);
}

size_t mpmc_poly_workspace_size(const mpmc_lattice *lat, const mpmc_poly *poly, mpmc_shape shape) {
    if (check_lattice(lat) != MPMC_OK || check_poly(poly) != MPMC_OK || !valid_shape(shape)) return 0;
    return poly_ws_bytes(lat->dims, lat->prec, *poly, shape);
}

int mpmc_poly_apply(const mpmc_lattice *lat, const mpmc_poly *poly, mpmc_shape shape, const void *x,
                    const mpmc_noise *noise, void *y, double *bhy, void *ws, size_t ws_bytes, void *stream) {
    MPMC_TRY(check_lattice(lat));
    MPMC_TRY(check_poly(poly));
    if (!valid_shape(shape) || !plane_fits(lat->dims, lat->prec, shape)) return MPMC_EINVAL;
    if (!y && !bhy) return MPMC_EINVAL;
    if (!x && !noise) return MPMC_EINVAL;
    if (x && x == y) return MPMC_EINVAL;
    if (noise && noise->probe_colour && (x || y || !bhy || poly->n_out != 0 || poly->n_in < 2))
        return MPMC_EUNSUPPORTED;                                 // probes: the scalar t-sweep only
    MPMC_TRY(check_ws(ws, ws_bytes, poly_ws_bytes(lat->dims, lat->prec, *poly, shape)));
    const PolyWs p = carve_poly_ws(lat->dims, lat->prec, *poly, shape, ws);
    return lat->prec == MPMC_F64 ? poly_apply_t<double>(*lat, *poly, shape, x, noise, y, bhy, p, stream)
                                 : poly_apply_t<float>(*lat, *poly, shape, x, noise, y, bhy, p, stream);
}

size_t mpmc_deflate_workspace_size(const mpmc_lattice *lat, const mpmc_defl *defl, mpmc_shape shape) {
    if (check_lattice(lat) != MPMC_OK || check_defl(defl, false) != MPMC_OK || !valid_shape(shape)) return 0;
    return defl_ws_bytes(*lat, *defl, shape);
}

int mpmc_deflate_project(const mpmc_lattice *lat, const mpmc_defl *defl, int32_t mode, mpmc_shape shape,
                         const void *b, const mpmc_noise *noise, double *zeta, double *omega, double *d, void *X,
                         void *ws, size_t ws_bytes, void *stream) {
    MPMC_TRY(check_lattice(lat));
    if (mode != MPMC_DEFL_COEFF && mode != MPMC_DEFL_RECON && mode != MPMC_DEFL_PROJECT) return MPMC_EUNSUPPORTED;
    MPMC_TRY(check_defl(defl, mode == MPMC_DEFL_PROJECT));
    if (!valid_shape(shape) || !plane_fits(lat->dims, lat->prec, shape)) return MPMC_EINVAL;
    if (mode != MPMC_DEFL_RECON && !b && !noise) return MPMC_EINVAL;
    if (noise && noise->probe_colour) return MPMC_EUNSUPPORTED;
    if (mode == MPMC_DEFL_COEFF && !zeta && !omega) return MPMC_EINVAL;
    if (mode == MPMC_DEFL_RECON && (!d || !X)) return MPMC_EINVAL;
    if (mode == MPMC_DEFL_PROJECT && (!d || !X || (b && b == X))) return MPMC_EINVAL;
    MPMC_TRY(check_ws(ws, ws_bytes, defl_ws_bytes(*lat, *defl, shape)));
    return deflate_impl(*lat, *defl, mode, shape, b, noise, zeta, omega, d, X, ws, stream);
}

size_t mpmc_level_workspace_size(const mpmc_lattice *lat, const mpmc_level *level, mpmc_shape shape) {
    if (check_lattice(lat) != MPMC_OK || !level || !valid_shape(shape)) return 0;
    if (level->kind_hi != MPMC_OP_SOLVE && check_poly(&level->poly_hi) != MPMC_OK) return 0;
    if (level->kind_lo != MPMC_OP_NONE && check_poly(&level->poly_lo) != MPMC_OK) return 0;
    return level_ws_bytes(*lat, *level, shape);
}

int mpmc_level_stop_check(const double *samples, int32_t nrhs, int32_t first, int32_t every, double *state,
                          void *stream) {
    if (!samples || !state || nrhs < 1 || first < 2 || every < 1) return MPMC_EINVAL;
    return stop_check_impl(samples, nrhs, first, every, state, stream);
}

int mpmc_mlmc_level_estimate(const mpmc_lattice *lat, const mpmc_level *level, mpmc_shape shape,
                             const mpmc_noise *noise, double *samples, double *acc, void *ws, size_t ws_bytes,
                             void *stream) {
    MPMC_TRY(check_lattice(lat));
    if (!level || !noise || !samples || !acc || !valid_shape(shape)) return MPMC_EINVAL;
    if (noise->probe_colour) return MPMC_EUNSUPPORTED;
    if (!plane_fits(lat->dims, lat->prec, shape)) return MPMC_EINVAL;
    const int kh = level->kind_hi, kl = level->kind_lo;
    if (kh != MPMC_OP_POLY && kh != MPMC_OP_DEFLATED_POLY && kh != MPMC_OP_SOLVE) return MPMC_EUNSUPPORTED;
    if (kl != MPMC_OP_NONE && kl != MPMC_OP_POLY && kl != MPMC_OP_DEFLATED_POLY) return MPMC_EUNSUPPORTED;
    if (kh == MPMC_OP_SOLVE) {
        if (!level->solve_x) return MPMC_EINVAL;
    } else {
        MPMC_TRY(check_poly(&level->poly_hi));
    }
    if (kl != MPMC_OP_NONE) MPMC_TRY(check_poly(&level->poly_lo));
    const bool proj = kh == MPMC_OP_DEFLATED_POLY || kl == MPMC_OP_DEFLATED_POLY;
    if (proj || level->deflate_samples) MPMC_TRY(check_defl(level->defl, proj));
    if (level->deflate_samples && !level->c) return MPMC_EINVAL;
    if (level->deflate_samples != 0 && level->deflate_samples != 1) return MPMC_EINVAL;
    MPMC_TRY(check_ws(ws, ws_bytes, level_ws_bytes(*lat, *level, shape)));
    return level_impl(*lat, *level, shape, *noise, samples, acc, ws, stream);
}

}  // extern "C"
