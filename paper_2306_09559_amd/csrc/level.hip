// One Monte Carlo level of the multilevel formula (eq. multpolytr, Sec. 3.1)
// with Monte Carlo deflation (Sec. 4.1) and the deflated polynomial
// operator (Sec. 4.3): Hutchinson samples (Sec. 1)
//     s = b^H P_hi b - b^H P_lo b - sum_i c_i conj(zeta_i) omega_i
// and their FP64 accumulation.
#include "common.hpp"
#include "internal.hpp"

namespace mpmc {

namespace {

struct LevelWs {
    double *zeta, *omega, *d;     // k x N complex each
    double *hi, *lo;              // N complex each
    void *defl;                   // deflation scratch
    void *rfield;                 // projected residual b - A V d
    void *poly;                   // polynomial scratch (reused by hi and lo)
};

bool needs_defl(const mpmc_level &lv) {
    return lv.deflate_samples || lv.kind_hi == MPMC_OP_DEFLATED_POLY || lv.kind_lo == MPMC_OP_DEFLATED_POLY;
}
bool needs_project(const mpmc_level &lv) {
    return lv.kind_hi == MPMC_OP_DEFLATED_POLY || lv.kind_lo == MPMC_OP_DEFLATED_POLY;
}

// x = A^{-1} b is supplied (MPMC_OP_SOLVE): b^H x is the degree-0 polynomial
// p = 1 applied to x and dotted against the noise
__device__ double2 g_unit_root = {1.0, 0.0};

int unit_poly(mpmc_poly *p) {
    static const double *addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MPMC_EHIP;
    if (!addr[dev]) {
        void *a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(g_unit_root)) != hipSuccess || !a) return MPMC_EHIP;
        addr[dev] = (const double *)a;
    }
    p->n_in = 1;
    p->n_out = 0;
    p->inv_roots_in = addr[dev];
    p->inv_roots_out = nullptr;
    return MPMC_OK;
}

mpmc_poly hi_poly_shape(const mpmc_level &lv) {
    if (lv.kind_hi != MPMC_OP_SOLVE) return lv.poly_hi;
    mpmc_poly p{};
    p.n_in = 1;
    return p;
}

size_t carve(const mpmc_lattice &lat, const mpmc_level &lv, mpmc_shape sh, void *base, LevelWs *out) {
    char *w = (char *)base;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = w ? (void *)(w + off) : nullptr;
        off += align256(bytes);
        return p;
    };
    const int k = (lv.defl && needs_defl(lv)) ? lv.defl->k : 0;
    LevelWs ws{};
    ws.zeta = (double *)take((size_t)k * sh.nrhs * 16);
    ws.omega = (double *)take((size_t)k * sh.nrhs * 16);
    ws.d = (double *)take((size_t)k * sh.nrhs * 16);
    ws.hi = (double *)take((size_t)sh.nrhs * 16);
    ws.lo = (double *)take((size_t)sh.nrhs * 16);
    if (k) ws.defl = take(defl_ws_bytes(lat, *lv.defl, sh));
    if (needs_project(lv)) ws.rfield = take(field_bytes(lat.dims, lat.prec, sh.nrhs));
    size_t pb = poly_ws_bytes(lat.dims, lat.prec, hi_poly_shape(lv), sh);
    if (lv.kind_lo != MPMC_OP_NONE) {
        const size_t pl = poly_ws_bytes(lat.dims, lat.prec, lv.poly_lo, sh);
        pb = pl > pb ? pl : pb;
    }
    ws.poly = take(pb);
    if (out) *out = ws;
    return off;
}

__device__ __forceinline__ double2 z2(double x, double y) {
    double2 r;
    r.x = x;
    r.y = y;
    return r;
}

// single workgroup: samples, batch mean and M2 in a fixed order, Chan merge
__global__ void __launch_bounds__(256) k_assemble(int nrhs, int k, int hi_defl, int lo_defl, int has_lo,
                                                  int deflate_samples, const double2 *hi, const double2 *lo,
                                                  const double2 *zeta, const double2 *omega, const double2 *d,
                                                  const double2 *c, double *samples, double *acc) {
    __shared__ double sre[256], sim[256], sm2[256];
    __shared__ int snf[256];
    const int tid = (int)threadIdx.x;
    double are = 0.0, aim = 0.0;
    int nf = 0;
    for (int r = tid; r < nrhs; r += 256) {
        double2 h = hi[r];
        double2 l = has_lo ? lo[r] : z2(0.0, 0.0);
        double2 zd = z2(0.0, 0.0), dd = z2(0.0, 0.0);
        for (int i = 0; i < k; ++i) {
            const double2 zt = zeta[(size_t)i * nrhs + r];
            if (hi_defl || lo_defl) {   // zeta^H H^{-1} omega = sum conj(zeta_i) d_i
                const double2 di = d[(size_t)i * nrhs + r];
                zd.x += zt.x * di.x + zt.y * di.y;
                zd.y += zt.x * di.y - zt.y * di.x;
            }
            if (deflate_samples) {      // c_i conj(zeta_i) omega_i
                const double2 om = omega[(size_t)i * nrhs + r], ci = c[i];
                const double pr = zt.x * om.x + zt.y * om.y, pi = zt.x * om.y - zt.y * om.x;
                dd.x += ci.x * pr - ci.y * pi;
                dd.y += ci.x * pi + ci.y * pr;
            }
        }
        if (hi_defl) { h.x += zd.x; h.y += zd.y; }
        if (lo_defl) { l.x += zd.x; l.y += zd.y; }
        const double sr = h.x - l.x - dd.x, si = h.y - l.y - dd.y;
        double *o = samples + (size_t)r * 6;
        o[0] = sr; o[1] = si; o[2] = h.x; o[3] = h.y; o[4] = l.x; o[5] = l.y;
        if (!isfinite(sr) || !isfinite(si)) ++nf;
        are += sr;
        aim += si;
    }
    sre[tid] = are;
    sim[tid] = aim;
    snf[tid] = nf;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            sre[tid] += sre[tid + st];
            sim[tid] += sim[tid + st];
            snf[tid] += snf[tid + st];
        }
        __syncthreads();
    }
    const double mre = sre[0] / nrhs, mim = sim[0] / nrhs;
    __syncthreads();
    double m2 = 0.0;
    for (int r = tid; r < nrhs; r += 256) {
        const double dr = samples[(size_t)r * 6] - mre, di = samples[(size_t)r * 6 + 1] - mim;
        m2 += dr * dr + di * di;
    }
    sm2[tid] = m2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) sm2[tid] += sm2[tid + st];
        __syncthreads();
    }
    if (tid == 0) {
        // pairwise merge (Chan, Golub & LeVeque) of (n, mean, M2) into acc
        const double n0 = acc[0], nb = (double)nrhs, n1 = n0 + nb;
        const double dre = mre - acc[1], dim = mim - acc[2];
        acc[1] = acc[1] + dre * (nb / n1);
        acc[2] = acc[2] + dim * (nb / n1);
        acc[3] = acc[3] + sm2[0] + (dre * dre + dim * dim) * (n0 * nb / n1);
        acc[0] = n1;
        acc[4] = acc[4] + (double)snf[0];
    }
}

template <typename T>
int level_t(const mpmc_lattice &lat, const mpmc_level &lv, mpmc_shape sh, const mpmc_noise &nz, double *samples,
            double *acc, void *wsb, void *stream) {
    LevelWs ws;
    carve(lat, lv, sh, wsb, &ws);
    const bool defl = lv.defl && needs_defl(lv);
    const int k = defl ? lv.defl->k : 0;
    int st;
    if (defl) {
        if (needs_project(lv))
            st = deflate_impl(lat, *lv.defl, MPMC_DEFL_PROJECT, sh, nullptr, &nz, ws.zeta, ws.omega, ws.d, ws.rfield,
                              ws.defl, stream);
        else
            st = deflate_impl(lat, *lv.defl, MPMC_DEFL_COEFF, sh, nullptr, &nz, ws.zeta, ws.omega, nullptr, nullptr,
                              ws.defl, stream);
        if (st != MPMC_OK) return st;
    }
    mpmc_poly ph = lv.poly_hi;
    const void *xin_hi = lv.kind_hi == MPMC_OP_DEFLATED_POLY ? ws.rfield : nullptr;
    if (lv.kind_hi == MPMC_OP_SOLVE) {
        st = unit_poly(&ph);
        if (st != MPMC_OK) return st;
        xin_hi = lv.solve_x;
    }
    const PolyWs phi = carve_poly_ws(lat.dims, lat.prec, ph, sh, ws.poly);
    st = poly_apply_t<T>(lat, ph, sh, xin_hi, &nz, nullptr, ws.hi, phi, stream);
    if (st != MPMC_OK) return st;
    if (lv.kind_lo != MPMC_OP_NONE) {
        const PolyWs plo = carve_poly_ws(lat.dims, lat.prec, lv.poly_lo, sh, ws.poly);
        const void *xin_lo = lv.kind_lo == MPMC_OP_DEFLATED_POLY ? ws.rfield : nullptr;
        st = poly_apply_t<T>(lat, lv.poly_lo, sh, xin_lo, &nz, nullptr, ws.lo, plo, stream);
        if (st != MPMC_OK) return st;
    }
    hipLaunchKernelGGL(k_assemble, dim3(1), dim3(256), 0, (hipStream_t)stream, sh.nrhs, k,
                       (int)(lv.kind_hi == MPMC_OP_DEFLATED_POLY), (int)(lv.kind_lo == MPMC_OP_DEFLATED_POLY),
                       (int)(lv.kind_lo != MPMC_OP_NONE), (int)(defl && lv.deflate_samples), (const double2 *)ws.hi,
                       (const double2 *)ws.lo, (const double2 *)ws.zeta, (const double2 *)ws.omega,
                       (const double2 *)ws.d, (const double2 *)lv.c, samples, acc);
    return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

// The stopping rule of Sec. 5 step 3 applied one sample at a time, as the
// paper's loop draws them: state (FP64, see mpmc_level_stop_check) keeps the
// level's running (n, mean, M2) -- Welford's update over complex samples as
// pairs of reals -- and after every sample that lands on a check point
// (first, first + every, ...) compares the standard error
// sqrt(M2 / ((n - 1) n)) with the target.  The first success records the
// statistics of exactly the samples up to that point and freezes the state.
// One thread: a batch is at most a few hundred samples, in order.
__global__ void k_stop_scan(const double *samples, int nrhs, int first, int every, double *state) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (state[4] != 0.0) return;                   // stopped earlier
    double n = state[0], mr = state[1], mi = state[2], m2 = state[3];
    const double target = state[7];
    for (int r = 0; r < nrhs; ++r) {
        const double sr = samples[(size_t)r * 6], si = samples[(size_t)r * 6 + 1];
        n += 1.0;
        const double dr = sr - mr, di = si - mi;
        mr += dr / n;
        mi += di / n;
        m2 += dr * (sr - mr) + di * (si - mi);
        const long long nn = (long long)n;
        if (nn >= first && nn >= 2 && (nn - first) % every == 0 && sqrt(m2 / ((n - 1.0) * n)) <= target) {
            state[4] = 1.0;
            state[5] = n;
            state[8] = mr;
            state[9] = mi;
            state[10] = m2;
            break;
        }
    }
    state[0] = n;
    state[1] = mr;
    state[2] = mi;
    state[3] = m2;
}

}  // namespace

size_t level_ws_bytes(const mpmc_lattice &lat, const mpmc_level &lv, mpmc_shape sh) {
    return carve(lat, lv, sh, nullptr, nullptr);
}

int stop_check_impl(const double *samples, int nrhs, int first, int every, double *state, void *stream) {
    hipLaunchKernelGGL(k_stop_scan, dim3(1), dim3(64), 0, (hipStream_t)stream, samples, nrhs, first, every, state);
    return hipGetLastError() == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

int level_impl(const mpmc_lattice &lat, const mpmc_level &lv, mpmc_shape sh, const mpmc_noise &nz, double *samples,
               double *acc, void *ws, void *stream) {
    return lat.prec == MPMC_F64 ? level_t<double>(lat, lv, sh, nz, samples, acc, ws, stream)
                                : level_t<float>(lat, lv, sh, nz, samples, acc, ws, stream);
}

}  // namespace mpmc
