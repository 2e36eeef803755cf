// Batched steps of the multilevel estimate (Sec. 5 step 3: every level of
// eq. multpolytr draws its samples) recorded once as a HIP graph, the kernel
// shape autotuner, and the small dense inverse of the Left-right Projection
// (Sec. 2.1).  Host code around the level launchers of level.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

using namespace mpmc;

struct mpmc_handle_s {
    int device = -1;
    hipStream_t main = nullptr;                 // the stream a step is recorded on
    std::vector<hipStream_t> branch;            // one per branch of the recorded step
    std::vector<hipEvent_t> join;               // branch b done
    hipEvent_t fork = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::map<std::string, std::pair<mpmc_tune_choice, double>> tuned;
};

namespace {

// the kernel-selection options of one enqueue, restored on scope exit
struct OptionScope {
    int sweep, rank, chunks;
    OptionScope(int s, int r, int c) : sweep(g_opt_sweep), rank(g_opt_sweep_rank), chunks(g_opt_sweep_chunks) {
        g_opt_sweep = s;
        g_opt_sweep_rank = r;
        g_opt_sweep_chunks = c;
    }
    ~OptionScope() {
        g_opt_sweep = sweep;
        g_opt_sweep_rank = rank;
        g_opt_sweep_chunks = chunks;
    }
};

bool same_choice(const mpmc_tune_choice &a, const mpmc_tune_choice &b) {
    return a.rb == b.rb && a.plane_sweep == b.plane_sweep && a.sweep_rank == b.sweep_rank &&
           a.sweep_chunks == b.sweep_chunks;
}

void drop_graph(mpmc_handle h) {
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->exec = nullptr;
    h->graph = nullptr;
}

int ensure_streams(mpmc_handle h, int nbranch) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MPMC_EHIP;
    if (h->device >= 0 && h->device != dev) return MPMC_EINVAL;   // a handle serves one device
    h->device = dev;
    // default-priority, non-blocking streams owned by the handle
    if (!h->main && hipStreamCreateWithFlags(&h->main, hipStreamNonBlocking) != hipSuccess) return MPMC_EHIP;
    if (!h->fork && hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess) return MPMC_EHIP;
    while ((int)h->branch.size() < nbranch) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return MPMC_EHIP;
        h->branch.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MPMC_EHIP;
        h->join.push_back(e);
    }
    return MPMC_OK;
}

bool polynomial_level(const mpmc_level *lv) {
    return lv && (lv->kind_hi == MPMC_OP_POLY || lv->kind_hi == MPMC_OP_DEFLATED_POLY);
}

std::string tune_key(int dev, const mpmc_lattice &lat, const mpmc_level &lv, int nrhs) {
    char buf[512];
    const int k = lv.defl ? lv.defl->k : 0;
    snprintf(buf, sizeof buf, "%d|%d,%d,%d,%d|%d|%d|%d|%d:%d,%d|%d:%d,%d|%d,%d|%d", dev, lat.dims[0], lat.dims[1],
             lat.dims[2], lat.dims[3], lat.prec, lat.link_rows, lat.antiperiodic_t, lv.kind_hi, lv.poly_hi.n_in,
             lv.poly_hi.n_out, lv.kind_lo, lv.poly_lo.n_in, lv.poly_lo.n_out, k, lv.deflate_samples, nrhs);
    return std::string(buf);
}

}  // namespace

extern "C" {

int mpmc_handle_create(mpmc_handle *out) {
    if (!out) return MPMC_EINVAL;
    *out = new (std::nothrow) mpmc_handle_s();
    return *out ? MPMC_OK : MPMC_EINVAL;
}

int mpmc_handle_destroy(mpmc_handle h) {
    if (!h) return MPMC_OK;
    drop_graph(h);
    for (hipEvent_t e : h->join) (void)hipEventDestroy(e);
    for (hipStream_t s : h->branch) (void)hipStreamDestroy(s);
    if (h->fork) (void)hipEventDestroy(h->fork);
    if (h->main) (void)hipStreamDestroy(h->main);
    delete h;
    return MPMC_OK;
}

int mpmc_batch_build(mpmc_handle h, const mpmc_batch_item *items, int32_t n_items) {
    if (!h || !items || n_items < 1) return MPMC_EINVAL;
    int nbranch = 0;
    for (int i = 0; i < n_items; ++i) {
        const mpmc_batch_item &it = items[i];
        if (!it.lat || !it.counter || it.batches < 1 || it.branch < 0 || it.branch > 255) return MPMC_EINVAL;
        if (!polynomial_level(it.level)) return MPMC_EUNSUPPORTED;
        if (it.plane_sweep < 0 || it.plane_sweep > 2) return MPMC_EINVAL;
        if (it.sweep_rank < 0 || it.sweep_rank > 63) return MPMC_EINVAL;
        if (it.sweep_chunks < 0 || it.sweep_chunks > 1024) return MPMC_EINVAL;
        if (it.stop_state && (it.stop_first < 2 || it.stop_every < 1)) return MPMC_EINVAL;
        // descriptor, shape and workspace (the level call validates the rest while it is recorded,
        // and any failure there abandons the recording: nothing has run)
        const size_t need = mpmc_level_workspace_size(it.lat, it.level, it.shape);
        if (need == 0) return MPMC_EINVAL;
        if (it.ws_bytes < need) return MPMC_EWORKSPACE;
        if (!it.samples || !it.acc || !it.ws) return MPMC_EINVAL;
        if (it.branch + 1 > nbranch) nbranch = it.branch + 1;
    }
    int st = ensure_streams(h, nbranch);
    if (st != MPMC_OK) return st;
    st = sweep_prepare_kernels();          // no attribute calls while recording
    if (st != MPMC_OK) return st;
    drop_graph(h);
    if (hipStreamBeginCapture(h->main, hipStreamCaptureModeRelaxed) != hipSuccess) return MPMC_EHIP;
    // fork: every branch stream joins the recording through an event of the main stream
    st = hipEventRecord(h->fork, h->main) == hipSuccess ? MPMC_OK : MPMC_EHIP;
    std::vector<char> used(nbranch, 0);
    for (int b = 0; b < nbranch && st == MPMC_OK; ++b)
        for (int i = 0; i < n_items; ++i)
            if (items[i].branch == b) used[b] = 1;
    for (int b = 0; b < nbranch && st == MPMC_OK; ++b) {
        if (!used[b]) continue;
        hipStream_t s = h->branch[b];
        if (hipStreamWaitEvent(s, h->fork, 0) != hipSuccess) {
            st = MPMC_EHIP;
            break;
        }
        for (int i = 0; i < n_items && st == MPMC_OK; ++i) {
            const mpmc_batch_item &it = items[i];
            if (it.branch != b) continue;
            OptionScope opts(it.plane_sweep, it.sweep_rank, it.sweep_chunks);
            mpmc_noise nz = it.noise;
            nz.sample_offset = it.counter;
            for (int rep = 0; rep < it.batches && st == MPMC_OK; ++rep) {
                st = mpmc_mlmc_level_estimate(it.lat, it.level, it.shape, &nz, it.samples, it.acc, it.ws,
                                              it.ws_bytes, s);
                if (st == MPMC_OK && it.stop_state)
                    st = stop_check_impl(it.samples, it.shape.nrhs, it.stop_first, it.stop_every, it.stop_state, s);
                if (st == MPMC_OK) st = counter_add_impl(it.counter, (uint64_t)it.shape.nrhs, s);
            }
        }
        if (st == MPMC_OK && (hipEventRecord(h->join[b], s) != hipSuccess ||
                              hipStreamWaitEvent(h->main, h->join[b], 0) != hipSuccess))
            st = MPMC_EHIP;
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->main, &g);
    if (st == MPMC_OK && (ec != hipSuccess || !g)) st = MPMC_EHIP;
    if (st != MPMC_OK) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess || !ex) {
        (void)hipGraphDestroy(g);
        return MPMC_EHIP;
    }
    h->graph = g;
    h->exec = ex;
    return MPMC_OK;
}

int mpmc_batch_launch(mpmc_handle h, void *stream) {
    if (!h || !h->exec) return MPMC_EINVAL;
    return hipGraphLaunch(h->exec, (hipStream_t)stream) == hipSuccess ? MPMC_OK : MPMC_EHIP;
}

size_t mpmc_autotune_workspace_size(const mpmc_lattice *lat, const mpmc_level *level, int32_t nrhs) {
    if (!lat || !level || nrhs < 1) return 0;
    size_t most = 0;
    for (int rb = 1; rb <= 32 && rb <= nrhs; rb *= 2) {
        if (nrhs % rb) continue;
        const size_t b = mpmc_level_workspace_size(lat, level, mpmc_shape{nrhs, rb});
        if (b > most) most = b;
    }
    return align256(most) + align256((size_t)nrhs * 6 * sizeof(double)) + align256(8 * sizeof(double));
}

int mpmc_autotune(mpmc_handle h, const mpmc_lattice *lat, const mpmc_level *level, int32_t nrhs,
                  const mpmc_noise *noise, int32_t reps, double keep_within, void *ws, size_t ws_bytes,
                  mpmc_tune_choice *best, double *best_seconds, int32_t *cached, mpmc_tune_result *results,
                  int32_t max_results, int32_t *n_results, void *stream) {
    if (!h || !lat || !level || !noise || !best || nrhs < 1 || reps < 1 || keep_within < 0.0) return MPMC_EINVAL;
    if (best->plane_sweep < 0 || best->plane_sweep > 2 || best->sweep_rank < 0 || best->sweep_rank > 63 ||
        best->sweep_chunks < 0 || best->sweep_chunks > 1024)
        return MPMC_EINVAL;
    if (!polynomial_level(level)) return MPMC_EUNSUPPORTED;
    const size_t need = mpmc_autotune_workspace_size(lat, level, nrhs);
    if (need == 0) return MPMC_EINVAL;
    if (ws_bytes < need) return MPMC_EWORKSPACE;
    if (!ws) return MPMC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MPMC_EHIP;
    if (n_results) *n_results = 0;
    if (cached) *cached = 0;
    const std::string key = tune_key(dev, *lat, *level, nrhs);
    auto hit = h->tuned.find(key);
    if (hit != h->tuned.end()) {
        *best = hit->second.first;
        if (best_seconds) *best_seconds = hit->second.second;
        if (cached) *cached = 1;
        return MPMC_OK;
    }
    // scratch: the level workspace, then samples and accumulator
    char *w = (char *)ws;
    size_t lvl_bytes = 0;
    for (int rb = 1; rb <= 32 && rb <= nrhs; rb *= 2)
        if (nrhs % rb == 0) {
            const size_t b = mpmc_level_workspace_size(lat, level, mpmc_shape{nrhs, rb});
            if (b > lvl_bytes) lvl_bytes = b;
        }
    double *samples = (double *)(w + align256(lvl_bytes));
    double *acc = (double *)(w + align256(lvl_bytes) + align256((size_t)nrhs * 6 * sizeof(double)));
    mpmc_noise nz = *noise;
    nz.sample_offset = nullptr;
    // candidates
    std::vector<mpmc_tune_choice> cand;
    const int Lt = lat->dims[3];
    for (int rb = 1; rb <= 32 && rb <= nrhs; rb *= 2) {
        if (nrhs % rb) continue;
        cand.push_back(mpmc_tune_choice{rb, 0, 0, 0});
        if (rb < 8) continue;
        for (int r = 0; r < 3; ++r) {
            int k0 = 1;
            {
                OptionScope o(1, r, 0);
                const SweepPlan p = sweep_plan(*lat, mpmc_shape{nrhs, rb});
                if (!p.ok || r >= p.nranked) break;
                k0 = p.nch;
            }
            cand.push_back(mpmc_tune_choice{rb, 1, r, 0});
            // the divisors of Lt next to the plan's t-chunk count (chunks of at least 2 planes)
            int lower = 0, upper = 0;
            for (int k = 1; k < k0; ++k)
                if (Lt % k == 0) lower = k;
            for (int k = k0 + 1; k <= Lt / 2 && !upper; ++k)
                if (Lt % k == 0) upper = k;
            for (int k : {lower, upper}) {
                if (k < 1) continue;
                OptionScope o(1, r, k);
                const SweepPlan p = sweep_plan(*lat, mpmc_shape{nrhs, rb});
                if (p.ok && p.nch == k) cand.push_back(mpmc_tune_choice{rb, 1, r, k});
            }
        }
    }
    bool have_current = false;
    for (const auto &c : cand)
        if (same_choice(c, *best)) have_current = true;
    // the current shape is timed too when the workspace covers it (rb <= 32, like the candidates)
    if (!have_current && best->rb >= 1 && best->rb <= 32 && nrhs % best->rb == 0 && (best->rb & (best->rb - 1)) == 0)
        cand.push_back(*best);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MPMC_EHIP;
    std::vector<double> secs(cand.size(), 0.0);
    int st = MPMC_OK;
    for (size_t c = 0; c < cand.size() && st == MPMC_OK; ++c) {
        OptionScope opts(cand[c].plane_sweep, cand[c].sweep_rank, cand[c].sweep_chunks);
        const mpmc_shape sh{nrhs, cand[c].rb};
        if (hipMemsetAsync(acc, 0, 8 * sizeof(double), (hipStream_t)stream) != hipSuccess) st = MPMC_EHIP;
        if (st == MPMC_OK)
            st = mpmc_mlmc_level_estimate(lat, level, sh, &nz, samples, acc, w, lvl_bytes, stream);   // untimed
        if (st == MPMC_OK && hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) st = MPMC_EHIP;
        for (int r = 0; r < reps && st == MPMC_OK; ++r)
            st = mpmc_mlmc_level_estimate(lat, level, sh, &nz, samples, acc, w, lvl_bytes, stream);
        if (st == MPMC_OK && hipEventRecord(e1, (hipStream_t)stream) != hipSuccess) st = MPMC_EHIP;
        if (st == MPMC_OK && hipEventSynchronize(e1) != hipSuccess) st = MPMC_EHIP;
        float ms = 0.f;
        if (st == MPMC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = MPMC_EHIP;
        secs[c] = (double)ms * 1e-3 / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MPMC_OK) return st;
    size_t ib = 0, icur = cand.size();
    for (size_t c = 0; c < cand.size(); ++c) {
        if (secs[c] < secs[ib]) ib = c;
        if (same_choice(cand[c], *best)) icur = c;
    }
    // keep the current shape unless another is faster by more than keep_within
    if (icur < cand.size() && secs[icur] <= secs[ib] * (1.0 + keep_within)) ib = icur;
    *best = cand[ib];
    if (best_seconds) *best_seconds = secs[ib];
    if (results) {
        const int n = (int)cand.size() < max_results ? (int)cand.size() : max_results;
        for (int c = 0; c < n; ++c) results[c] = mpmc_tune_result{cand[c], secs[c]};
        if (n_results) *n_results = n;
    }
    h->tuned[key] = std::make_pair(*best, secs[ib]);
    return MPMC_OK;
}

int mpmc_small_inverse(int32_t k, const double *a, double tiny, double *out) {
    if (k < 1 || k > 4096 || !a || !out || !(tiny >= 0.0)) return MPMC_EINVAL;
    using cd = std::complex<double>;
    const size_t n = (size_t)k;
    std::vector<cd> m(n * n), inv(n * n, cd(0.0, 0.0));
    double amax = 0.0;
    for (size_t i = 0; i < n * n; ++i) {
        m[i] = cd(a[2 * i], a[2 * i + 1]);
        amax = std::max(amax, std::abs(m[i]));
    }
    for (size_t i = 0; i < n; ++i) inv[i * n + i] = cd(1.0, 0.0);
    for (size_t c = 0; c < n; ++c) {
        size_t piv = c;
        for (size_t r = c + 1; r < n; ++r)
            if (std::abs(m[r * n + c]) > std::abs(m[piv * n + c])) piv = r;
        const double pv = std::abs(m[piv * n + c]);
        if (!(pv > tiny * amax) || !std::isfinite(pv)) return MPMC_ESINGULAR;
        if (piv != c)
            for (size_t j = 0; j < n; ++j) {
                std::swap(m[c * n + j], m[piv * n + j]);
                std::swap(inv[c * n + j], inv[piv * n + j]);
            }
        const cd d = cd(1.0, 0.0) / m[c * n + c];
        for (size_t j = 0; j < n; ++j) {
            m[c * n + j] *= d;
            inv[c * n + j] *= d;
        }
        for (size_t r = 0; r < n; ++r) {
            if (r == c) continue;
            const cd f = m[r * n + c];
            if (f == cd(0.0, 0.0)) continue;
            for (size_t j = 0; j < n; ++j) {
                m[r * n + j] -= f * m[c * n + j];
                inv[r * n + j] -= f * inv[c * n + j];
            }
        }
    }
    for (size_t i = 0; i < n * n; ++i) {
        out[2 * i] = inv[i].real();
        out[2 * i + 1] = inv[i].imag();
    }
    return MPMC_OK;
}

}  // extern "C"
