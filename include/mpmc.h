/*
 * mpmc.h -- C ABI of libmpmc.so: the GPU hot path of Multipolynomial Monte
 * Carlo trace estimation (Lashomb, Morgan, Whyte, Wilcox, arXiv:2306.09559)
 * for gfx950 (AMD Instinct MI355X).
 *
 * The library estimates pieces of Tr(A^{-1}) for the Wilson-Dirac matrix A
 * with Hutchinson samples b^H M b over Z4 noise b (Sec. 1), where M is a
 * difference of GMRES polynomials in A (eq. multpolytr, Sec. 3.1), possibly
 * a composite polynomial (Sec. 2.4, Sec. 3.2), possibly deflated with right
 * and left eigenvectors (Sec. 4.1, Sec. 4.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice    dims = {Lx, Ly, Lz, Lt}; site s = x + Lx*(y + Ly*(z + Lz*t));
 *            V = Lx*Ly*Lz*Lt sites, n = 12*V unknowns per vector, unknown
 *            i = 12*s + 3*spin + colour.  x, y, z are periodic; t is
 *            periodic or antiperiodic (a hop across the t boundary carries -1).
 * Operator   (A psi)(x) = psi(x) - kappa sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                  + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
 *            with DeGrand-Rossi (chiral) gamma matrices, g5 = diag(1,1,-1,-1).
 *            The paper names the quenched Wilson-Dirac matrix (Sec. 5,
 *            Example 2); this hopping-parameter form is the reading used.
 * Precision  MPMC_F64: fields, links and eigenvectors are complex128.
 *            MPMC_F32: they are complex64.  Step coefficients (inverse
 *            roots, kappa t_j, axpby coefficients) stay FP64: the entries of
 *            a vector update are widened, combined in FP64 and rounded once,
 *            so the polynomial applied is the FP64 one.  Every dot product,
 *            sample value, deflation coefficient and accumulator is FP64.
 * Field      a batch of N vectors in "field layout" with RHS block width rb
 *            (a power of two, 1..256, dividing N): unknown (spin,colour) =
 *            c in 0..11 of site s of vector r = nb*rb + j is the complex
 *            number at index ((nb*12 + c)*V + s)*rb + j.  Complex numbers
 *            are (re, im) pairs of the field precision.
 * Gauge      library gauge layout (written by mpmc_pack_gauge): link
 *            element (row a, col b) of U_mu(s) at index (mu*9 + 3a + b)*V + s.
 * Noise      Z4 entries {1, i, -1, -i} (Sec. 1) from SplitMix64 (Steele,
 *            Lea & Flood 2014), out(x, k) = mix(x + k*0x9E3779B97F4A7C15):
 *              key  = out(out(out(seed,1) ^ lattice,1) ^ level,1)
 *              S_r  = out(key ^ r, 1)          r = global sample index
 *              q    = (out(S_r, i/32 + 1) >> 2*(i%32)) & 3,  b_r[i] = i^q.
 *            Noise is regenerated in registers wherever it is consumed.
 * Roots      a GMRES polynomial of degree d is given by the d+1 inverse
 *            roots t_j = 1/theta_j of its residual polynomial
 *            pi(a) = prod_j (1 - a/theta_j) = 1 - a p(a) (Sec. 3.1), as
 *            complex FP64 (re, im) pairs in device memory, in the order they
 *            are applied (Leja order).  p is applied in Newton form:
 *            w_0 = x, w_{j+1} = w_j - t_j A w_j, p(A) x = sum_j t_j w_j.
 *
 * Memory and streams
 * ------------------
 * Every pointer marked "device" is caller-owned device memory of the current
 * HIP device; the library only borrows it for the work it enqueues.  Calls
 * enqueue on `stream` (a hipStream_t, NULL = default stream), return without
 * synchronising, never allocate device memory, and never read device memory
 * on the host.  Scratch memory is the caller's `ws` of at least the size
 * the matching *_workspace_size function returns (256-byte aligned).
 *
 * Errors
 * ------
 * Every entry point returns MPMC_OK (0) or a negative status; arguments are
 * validated on the host before anything is enqueued, so an error leaves the
 * outputs untouched.  MPMC_EHIP reports a launch failure (hipGetLastError).
 * Non-finite sample values are counted in the level accumulator.  No C++
 * exception crosses this interface.  Calls are thread-compatible.
 */
#ifndef MPMC_H
#define MPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MPMC_OK = 0,
    MPMC_EINVAL = -1,       /* null pointer, size or layout out of range */
    MPMC_EUNSUPPORTED = -2, /* unknown precision, mode or operator kind */
    MPMC_EWORKSPACE = -3,   /* ws smaller than the *_workspace_size result */
    MPMC_EHIP = -4,         /* HIP runtime or launch failure */
    MPMC_ESINGULAR = -5,    /* a small dense system has a zero pivot (mpmc_small_inverse) */
    MPMC_ENOTCONVERGED = -6 /* an iteration missed its tolerance: no entry point of the library
                               iterates to a tolerance itself; the host-driven solver of the
                               binding (GMRES cycles around mpmc_* calls) reports it with this code */
};

enum { MPMC_F64 = 0, MPMC_F32 = 1 };

typedef struct {
    int32_t dims[4];        /* Lx, Ly, Lz, Lt, each >= 1, V*12 < 2^31 */
    int32_t antiperiodic_t; /* 0 or 1 */
    int32_t prec;           /* MPMC_F64 or MPMC_F32: precision of gauge and fields */
    double kappa;           /* hopping parameter */
    const void *gauge;      /* device, library gauge layout, 36*V complex */
    int32_t link_rows;      /* 3 (or 0): every entry of a link is read.  2: the links are special
                               unitary (SU(3), as the gauge links of the paper's quenched
                               ensembles) and the kernels read rows 0 and 1 only, rebuilding
                               row 2 = conj(row 0 x row 1): a third less link traffic.  Exact for
                               SU(3) links; check a gauge field with mpmc_gauge_unitarity. */
} mpmc_lattice;

typedef struct {
    int32_t nrhs;           /* N >= 1 */
    int32_t rb;             /* RHS block width: power of two in [1, 256], divides N */
} mpmc_shape;

typedef struct {
    uint64_t seed;
    uint64_t lattice;       /* lattice id */
    uint64_t level;         /* level id */
    uint64_t first_sample;  /* vector r of a batch is global sample first_sample + r (+ *sample_offset) */
    const uint64_t *sample_offset;  /* device counter added to first_sample when the kernels run, or
                                       NULL.  Lets a captured HIP graph draw new samples on every
                                       replay: advance it with mpmc_counter_add inside the graph. */
    const int32_t *probe_colour;    /* NULL: Z4 noise (seed, lattice, level).  Otherwise probe
                                       vectors of a distance colouring (Sec. 3.1, Sec. 5 step 3d):
                                       device int32[V], the colour of every site; vector r is
                                       b_{g/12, g%12}, g = first_sample + r (+ *sample_offset), with
                                       b_{c,k} = 1 at unknown k of every site of colour c, 0
                                       elsewhere.  Accepted only by mpmc_poly_apply in scalar mode
                                       for a single polynomial with x = NULL on a lattice and batch
                                       that take the t-sweep (mpmc_sweep_plan); every other use
                                       returns MPMC_EUNSUPPORTED.  Same vectors as mpmc_probe_fill. */
} mpmc_noise;

typedef struct {
    int32_t n_in;                /* roots of p (single) or of p_in (composite), >= 1 */
    int32_t n_out;               /* 0: single polynomial; >= 1: roots of p_out */
    const double *inv_roots_in;  /* device, n_in complex FP64 */
    const double *inv_roots_out; /* device, n_out complex FP64, or NULL when n_out = 0 */
} mpmc_poly;

/* Deflation data (Sec. 4): right eigenvectors z_i and left eigenvectors
 * u_i = scale_i * g5 z_{pair_i} (the g5 rule of Sec. 4 with the biorthonormal
 * scaling u_i^H z_i = 1), so U is never stored. */
typedef struct {
    int32_t k;                   /* triplets, 1 <= k <= kpad */
    int32_t kpad;                /* multiple of 16, <= 256 */
    const void *V;               /* device, z_1..z_kpad in field layout with nrhs = rb = kpad
                                    (entries i >= k must be zero), lattice precision */
    const int32_t *pair;         /* device, k indices in [0, k) */
    const double *scale;         /* device, k complex FP64 */
    const double *hinv;          /* device, k*k complex FP64 row-major H^{-1}, H = U^H A V
                                    (Sec. 2.1 step 2); needed by MPMC_DEFL_PROJECT only */
} mpmc_defl;

/* Status code as text (static storage). */
const char *mpmc_status_string(int status);

/* Library version and the gfx target it was built for. */
const char *mpmc_build_info(void);

/* Process-wide kernel-selection options (set them before enqueueing work;
 * not synchronised with concurrent calls).
 *   MPMC_OPT_PLANE_SWEEP  2 (default): scalar-mode single polynomials on a
 *     lattice whose xyz-plane (Lx*Ly*Lz a multiple of 64, at most 512 sites
 *     and 160 KiB of LDS at the field precision) run as a t-sweep with one
 *     workgroup per (vector, t-chunk) when those workgroups cover the GPU's
 *     CUs (below that the streaming kernel is faster: the sweep's launch time
 *     does not shrink with the batch); larger FP32 planes take the blocked
 *     t-sweep when its workgroups, in t-chunks of at least 4 planes, cover
 *     the CUs; vector mode at block width 1 takes the sweep when its threads
 *     fill the GPU; probe vectors always take the t-sweep.  1: the t-sweep
 *     whenever the lattice admits one (mpmc_sweep_plan ok), whatever the
 *     batch.  0: always the streaming site-parallel kernel (probe vectors:
 *     unsupported).
 *   MPMC_OPT_SWEEP_RANK   0 (default) .. 63: on FP32 planes too large for
 *     one workgroup, the t-sweep cuts the plane into xyz-blocks with a halo
 *     in LDS; the candidate blocks are ranked by the bytes each moves per
 *     site, and this option picks the rank-th (clamped to the last).
 *   MPMC_OPT_HOP_SLAB     1 (default): the streaming kernel hands each XCD a
 *     z-slab of the lattice swept along t (neighbours stay in its L2);
 *     0: each XCD takes a contiguous range of tiles in site order.
 *   MPMC_OPT_LINK_BUF     1 (default): the streaming kernel reads the links
 *     through buffer loads when the link array is below 4 GiB; 0: always
 *     through 64-bit flat addresses (the path of larger arrays).
 *   MPMC_OPT_SWEEP_CHUNKS 0 (default): the plan chooses how many t-chunks a
 *     t-sweep's planes are cut into (each workgroup walks Lt / k planes,
 *     starting from its chunk's previous plane, so that small batches still
 *     occupy the GPU); k = 1 .. 1024: k chunks when k divides Lt and the
 *     partial sums fit the polynomial workspace, else 1.
 * Every choice computes the same values up to the order of floating-point
 * sums (the work order changes no value at all). */
enum {
    MPMC_OPT_PLANE_SWEEP = 1,
    MPMC_OPT_SWEEP_RANK = 2,
    MPMC_OPT_HOP_SLAB = 3,
    MPMC_OPT_LINK_BUF = 4,
    MPMC_OPT_SWEEP_CHUNKS = 5
};
int mpmc_set_option(int32_t option, int32_t value);

/* Which t-sweep a scalar-mode polynomial on this lattice and batch would
 * use (host only, enqueues nothing).  out (host, 9 int32): [0] 1 if a sweep
 * applies, [1] 1 if the xyz-plane is cut into blocks with a halo in LDS (FP32
 * lattices whose plane exceeds one workgroup), [2..4] block extents in x, y,
 * z, [5] sites per block (= workgroup size), [6] halo sites, [7] blocks per
 * plane, [8] t-chunks (each workgroup walks Lt / [8] planes). */
int mpmc_sweep_plan(const mpmc_lattice *lat, mpmc_shape shape, int32_t *out);

/* *counter += increment, enqueued on `stream` as a one-thread kernel (plain
 * vector store; capturable in a HIP graph, unlike a memset or memcpy node).
 * counter: device, caller-owned. */
int mpmc_counter_add(uint64_t *counter, uint64_t increment, void *stream);

/* ---- layout conversion and noise ------------------------------------- */

/* canon: device complex128 (4, V, 3, 3) = U[mu][s][a][b] -> gauge (lattice
 * precision, library gauge layout).  Both device, caller-owned. */
int mpmc_pack_gauge(const int32_t dims[4], int32_t prec, const double *canon, void *gauge,
                    void *stream);

/* How far the packed links are from SU(3): out[0] = max over links of
 * max_ab |(U U^H - I)_ab|, out[1] = max |det U - 1| (device, 2 FP64, computed
 * by one workgroup in a fixed order).  Both are at the rounding level of the
 * precision for links that may use link_rows = 2. */
int mpmc_gauge_unitarity(const int32_t dims[4], int32_t prec, const void *gauge, double *out, void *stream);

/* Probe vectors for an exact trace by probing (Sec. 3.1, Sec. 5 step 3d):
 * vector r of the batch is probe p = first_probe + r, i.e. colour c = p / 12
 * and unknown k = p % 12 (k = 3 spin + colour index): entry (k, s) is 1 where
 * colour[s] == c, every other entry 0.  With a colouring in which sites of one
 * colour are further apart than the degree of p, the sum over all probes of
 * b^H p(A) b is Tr p(A).
 *   colour  device, V int32 (colour of each site, 0 .. ncolours-1)
 *   field   device field of `shape` (written) */
int mpmc_probe_fill(const int32_t dims[4], int32_t prec, mpmc_shape shape, const int32_t *colour,
                    int64_t first_probe, void *field, void *stream);

/* canon: device complex128 (N, V, 4, 3) <-> field (prec, field layout). */
int mpmc_pack_fields(const int32_t dims[4], int32_t prec, mpmc_shape shape, const double *canon,
                     void *field, void *stream);
int mpmc_unpack_fields(const int32_t dims[4], int32_t prec, mpmc_shape shape, const void *field,
                       double *canon, void *stream);

/* Write the Z4 vectors of `noise` (samples first_sample .. +N-1) into a field
 * (Sec. 1).  Bit-identical to the noise every other entry point regenerates. */
int mpmc_z4_fill(const int32_t dims[4], int32_t prec, mpmc_shape shape, const mpmc_noise *noise,
                 void *field, void *stream);

/* ---- vector utilities for the Krylov set-up (Sec. 5, setup step 2) ------ */

/* y_r = alpha_r x_r + beta_r y_r for every vector r of a batch.
 *   alpha  device, N complex FP64 (applied in FP64, result rounded once)
 *   beta   device, N complex FP64, or NULL: y_r = alpha_r x_r (y is not read)
 * x and y are device fields of the same shape; x == y is allowed. */
int mpmc_field_axpby(const int32_t dims[4], int32_t prec, mpmc_shape shape, const double *alpha, const void *x,
                     const double *beta, void *y, void *stream);

/* The same update with x and y in different precisions (x_prec, y_prec):
 * moves residuals and corrections between the FP64 outer and the FP32 inner
 * iteration of iterative refinement.  x and y must not overlap. */
int mpmc_field_axpby_mixed(const int32_t dims[4], mpmc_shape shape, int32_t x_prec, const double *alpha,
                           const void *x, int32_t y_prec, const double *beta, void *y, void *stream);

size_t mpmc_field_dot_workspace_size(const int32_t dims[4], mpmc_shape shape);

/* out_r = x_r^H y_r accumulated in FP64 in a fixed order (bitwise
 * reproducible).  out: device, N complex FP64. */
int mpmc_field_dot(const int32_t dims[4], int32_t prec, mpmc_shape shape, const void *x, const void *y, double *out,
                   void *ws, size_t ws_bytes, void *stream);

/* Copy vector src_index of batch src (shape src_shape) into vector
 * dst_index of batch dst (shape dst_shape): moves single vectors in and out
 * of an Arnoldi basis held as a batch with nrhs = rb.  src != dst. */
int mpmc_field_copy_vector(const int32_t dims[4], int32_t prec, mpmc_shape src_shape, const void *src,
                           int32_t src_index, mpmc_shape dst_shape, void *dst, int32_t dst_index, void *stream);

/* dst[0 .. bytes) = src[0 .. bytes): a plain streaming device copy (16-byte
 * nontemporal loads and stores).  Moves whole batches, and is the reference
 * copy against which the kernels' HBM rates are compared.  bytes a multiple
 * of 16, both pointers 16-byte aligned, the ranges disjoint; bytes == 0 is a
 * no-op.  Violations return MPMC_EINVAL before anything is enqueued. */
int mpmc_field_copy_bytes(const void *src, void *dst, size_t bytes, void *stream);

/* ---- Krylov bases of a batch (GMRES cycles, Sec. 2.1, Sec. 5 step 3a) --
 * A basis is k fields of one shape stored back to back: vector i of the
 * basis starts N*12*V complex numbers after vector i-1.  Every vector r of
 * the batch has its own basis (v_0)_r .. (v_{k-1})_r, as in k independent
 * GMRES runs. */

size_t mpmc_field_block_dot_workspace_size(const int32_t dims[4], mpmc_shape shape, int32_t k);

/* out[i*N + r] = (v_i)_r^H x_r for i < k, accumulated in FP64 in a fixed
 * order (bitwise reproducible); one pass over x for up to 8 basis vectors.
 *   basis  device, k fields;  x  device field;  out  device, k x N complex FP64 */
int mpmc_field_block_dot(const int32_t dims[4], int32_t prec, mpmc_shape shape, int32_t k, const void *basis,
                         const void *x, double *out, void *ws, size_t ws_bytes, void *stream);

/* y_r = sum_{i<k} coeff[i*N + r] (v_i)_r  (+ y_r when accumulate = 1; y is
 * not read when accumulate = 0), summed in FP64 and rounded once.
 *   coeff  device, k x N complex FP64.  y must not overlap the basis. */
int mpmc_field_block_axpy(const int32_t dims[4], int32_t prec, mpmc_shape shape, int32_t k, const void *basis,
                          const double *coeff, int32_t accumulate, void *y, void *stream);

/* ---- the operator ------------------------------------------------------ */

/* y = A x for N vectors (the matrix-vector product every cost in the paper
 * is counted in, Sec. 5).  x, y: device fields, distinct. */
int mpmc_wilson_apply(const mpmc_lattice *lat, mpmc_shape shape, const void *x, void *y,
                      void *stream);

/* ---- polynomials (Sec. 2.3, 2.4, 3.1, 3.2) ----------------------------- */

size_t mpmc_poly_workspace_size(const mpmc_lattice *lat, const mpmc_poly *poly, mpmc_shape shape);

/* Apply a GMRES polynomial p(A) (n_out = 0) or the composite polynomial
 * p_1(A) = p_in(A) p_out(A p_in(A)) (n_out >= 1, Sec. 3.2; cost
 * n_in*n_out - 1 operator applications) to N vectors.
 *   x      device field, or NULL: x = Z4 noise of `noise`
 *   noise  the Z4 batch b; when NULL, b = x
 *   y      device field receiving p(A) x, or NULL (scalar mode)
 *   bhy    device, 2*N FP64 receiving b_r^H (p(A) x)_r, or NULL
 * At least one of y, bhy must be non-NULL; x == NULL needs noise. */
int mpmc_poly_apply(const mpmc_lattice *lat, const mpmc_poly *poly, mpmc_shape shape,
                    const void *x, const mpmc_noise *noise, void *y, double *bhy, void *ws,
                    size_t ws_bytes, void *stream);

/* ---- deflation (Sec. 2.1, Sec. 4) -------------------------------------- */

enum {
    MPMC_DEFL_COEFF = 0,    /* zeta = V^H b, omega = U^H b                               */
    MPMC_DEFL_RECON = 1,    /* X = V d                                                   */
    MPMC_DEFL_PROJECT = 2   /* Left-right Projection of b with x0 = 0 (Sec. 2.1):        */
                            /* zeta, omega as COEFF, d = H^{-1} omega, X = b - A V d     */
};

size_t mpmc_deflate_workspace_size(const mpmc_lattice *lat, const mpmc_defl *defl, mpmc_shape shape);

/*   b      device field, or NULL: b = Z4 noise of `noise` (COEFF, PROJECT)
 *   zeta   device k x N complex FP64 (row i = eigenvector), or NULL (COEFF)
 *   omega  device k x N complex FP64, or NULL (COEFF); both written by PROJECT
 *   d      device k x N complex FP64: read by RECON, written by PROJECT
 *   X      device field: written by RECON and PROJECT
 * The V^H products run on FP64 (MPMC_F64) or FP32 (MPMC_F32) matrix cores
 * and are accumulated in FP64 across the lattice. */
int mpmc_deflate_project(const mpmc_lattice *lat, const mpmc_defl *defl, int32_t mode,
                         mpmc_shape shape, const void *b, const mpmc_noise *noise, double *zeta,
                         double *omega, double *d, void *X, void *ws, size_t ws_bytes,
                         void *stream);

/* ---- one Monte Carlo level (eq. multpolytr; Sec. 4.1; Sec. 5 step 3) --- */

enum {
    MPMC_OP_NONE = 0,            /* operator 0                                          */
    MPMC_OP_POLY = 1,            /* p(A): single or composite polynomial               */
    MPMC_OP_DEFLATED_POLY = 2,   /* Q = V H^{-1} U^H + p(A)(I - A V H^{-1} U^H) (Sec. 4.3) */
    MPMC_OP_SOLVE = 3            /* A^{-1}: b^H x with x = solve_x, a solution of A x = b
                                    computed beforehand (Sec. 5 step 3a); kind_hi only */
};

typedef struct {
    int32_t kind_hi, kind_lo;    /* MPMC_OP_* ; kind_hi must not be NONE */
    mpmc_poly poly_hi, poly_lo;
    const mpmc_defl *defl;       /* eigen-triplets, or NULL; required by DEFLATED_POLY */
    int32_t deflate_samples;     /* 1: subtract sum_i c_i conj(zeta_i) omega_i from each sample */
    const double *c;             /* device, k complex FP64 c_i = f_hi(l_i) - f_lo(l_i) (Sec. 4.1) */
    const void *solve_x;         /* device field of the batch shape (kind_hi = SOLVE): x_r with
                                    A x_r = b_r for the level's noise; NULL otherwise */
} mpmc_level;

size_t mpmc_level_workspace_size(const mpmc_lattice *lat, const mpmc_level *level, mpmc_shape shape);

/* Draw N Z4 samples b_r of `noise` and compute, in FP64,
 *   hi_r = b_r^H P_hi b_r,  lo_r = b_r^H P_lo b_r,
 *   s_r  = hi_r - lo_r - sum_i c_i conj(zeta_ir) omega_ir   (deflated levels)
 * with zeta = V^H b, omega = U^H b.
 *   samples  device, N x 6 FP64: (s, hi, lo) as complex pairs per sample
 *   acc      device, 8 FP64, updated in place (zero it before the first batch):
 *            [0] count, [1] mean re, [2] mean im, [3] sum |s - mean|^2,
 *            [4] non-finite samples seen, [5..7] reserved (0).
 * Batches merge into acc with the pairwise update of Chan, Golub & LeVeque,
 * in submission order, so results are reproducible bit for bit.  The level
 * estimate is acc mean + sum_i c_i (u_i^H z_i = 1 by the scaling). */
int mpmc_mlmc_level_estimate(const mpmc_lattice *lat, const mpmc_level *level, mpmc_shape shape,
                             const mpmc_noise *noise, double *samples, double *acc, void *ws,
                             size_t ws_bytes, void *stream);

/* The stopping rule of the adaptive multilevel estimate (Sec. 5 step 3) on
 * the device, one sample at a time in batch order, as the paper's loop
 * draws them: after every sample whose running count n is a check point
 * (first, first + every, first + 2 every, ...) the level stops when its
 * standard error sqrt(M2 / ((n - 1) n)) is at most the target.
 *   samples  device, nrhs x 6 FP64 (mpmc_mlmc_level_estimate's output; s is columns 0, 1)
 *   state    device, 16 FP64, caller-owned: zero it before the level's first
 *            batch and set [7] = target.  [0] n, [1..2] mean, [3] M2 =
 *            sum |s - mean|^2 of every sample scanned (Welford's update);
 *            [4] 1 once stopped, [5] n at the stop, [8..9] mean and [10] M2
 *            of exactly the samples up to the stop.  After the stop, further
 *            calls change nothing.
 * first >= 2, every >= 1.  One tiny kernel, capturable in a HIP graph. */
int mpmc_level_stop_check(const double *samples, int32_t nrhs, int32_t first, int32_t every, double *state,
                          void *stream);

/* ---- batched steps and the autotuner (Sec. 5 step 3: every level of the
 * multilevel estimate draws its samples; eq. multpolytr) -------------------
 *
 * A step of the multilevel method draws Z4 samples on every level of one or
 * several lattices.  The library records such a step once as a HIP graph
 * (every launch of every level, of uneven degree and sample count, in one
 * graph) and replays it with one launch.  Each item of a step takes its
 * sample index from a device counter that the graph itself advances, so
 * every replay draws new samples and the level accumulators keep merging
 * them on the device; nothing is read back between replays.
 *
 * The handle owns the graph, the streams it was recorded on and the tuner's
 * results; it owns no device memory.  One handle per thread. */
typedef struct mpmc_handle_s *mpmc_handle;

/* *out = a new handle (host memory only).  MPMC_EINVAL for out == NULL. */
int mpmc_handle_create(mpmc_handle *out);
/* Destroys the handle, its graph and its streams (waits for none of its
 * work: synchronise the launch stream first).  NULL is a no-op. */
int mpmc_handle_destroy(mpmc_handle h);

/* One level of one lattice in a batched step: `batches` batches of
 * shape.nrhs samples, each followed by *counter += shape.nrhs.  Batch b of a
 * replay draws samples noise.first_sample + *counter + (0 .. nrhs-1), where
 * *counter is read when that batch runs (noise.sample_offset is ignored).
 * Items with the same branch run in the given order on one stream; items of
 * different branches may run concurrently (give each lattice its own).  The
 * descriptors (lat, level, and what they point to on the host) are read
 * during mpmc_batch_build only; every device buffer they and the item name
 * must stay valid while the graph may run.  Two items must not share a
 * workspace, samples or acc buffer unless they are in the same branch. */
typedef struct {
    const mpmc_lattice *lat;
    const mpmc_level *level;     /* a polynomial level: kind_hi POLY or DEFLATED_POLY (SOLVE needs a
                                    host-driven solve per batch and is not batched) */
    mpmc_shape shape;
    mpmc_noise noise;            /* seed, lattice, level id, first_sample */
    uint64_t *counter;           /* device, caller-owned sample counter of this item */
    int32_t batches;             /* >= 1 */
    double *samples;             /* device, nrhs x 6 FP64 (holds the last batch) */
    double *acc;                 /* device, 8 FP64 level accumulator (as mpmc_mlmc_level_estimate) */
    void *ws;                    /* device, mpmc_level_workspace_size(lat, level, shape) bytes */
    size_t ws_bytes;
    int32_t branch;              /* >= 0 */
    int32_t plane_sweep;         /* kernel selection for this item: MPMC_OPT_PLANE_SWEEP value */
    int32_t sweep_rank;          /* MPMC_OPT_SWEEP_RANK value */
    int32_t sweep_chunks;        /* MPMC_OPT_SWEEP_CHUNKS value (0: the plan's choice) */
    double *stop_state;          /* device state of mpmc_level_stop_check, or NULL: when given, every
                                    batch is followed by the stopping check on its samples */
    int32_t stop_first, stop_every;  /* the level's check points (as mpmc_level_stop_check) */
} mpmc_batch_item;

/* Record the step made of items[0 .. n_items-1] as a HIP graph held by the
 * handle (replacing any previous one).  Enqueues nothing and runs nothing:
 * recording only captures the launches.  Arguments are validated first
 * (MPMC_EINVAL, MPMC_EUNSUPPORTED, MPMC_EWORKSPACE as the level call would
 * return); MPMC_EHIP if recording or instantiation fails. */
int mpmc_batch_build(mpmc_handle h, const mpmc_batch_item *items, int32_t n_items);

/* Launch the recorded step on `stream` (asynchronous).  MPMC_EINVAL if no
 * step was built. */
int mpmc_batch_launch(mpmc_handle h, void *stream);

/* A kernel shape for one level: RHS block width and the three t-sweep
 * options above. */
typedef struct {
    int32_t rb;
    int32_t plane_sweep;
    int32_t sweep_rank;
    int32_t sweep_chunks;
} mpmc_tune_choice;

typedef struct {
    mpmc_tune_choice choice;
    double seconds;              /* per call of mpmc_mlmc_level_estimate with this shape */
} mpmc_tune_result;

/* Workspace the tuner needs for this level and batch size (every candidate
 * shape fits in it, plus scratch samples and accumulator). */
size_t mpmc_autotune_workspace_size(const mpmc_lattice *lat, const mpmc_level *level, int32_t nrhs);

/* Time one level's batch of nrhs samples under every candidate shape and
 * pick the fastest: block widths rb = 1, 2, 4, .. 32 dividing nrhs on the
 * streaming kernel; rb >= 8 on the t-sweep where it applies; on FP32 planes
 * cut into blocks, the three best-ranked blocks; for each sweep, the plan's
 * number of t-chunks and the divisors of Lt next to it.  `best` is in/out:
 * on entry the current shape, timed with its own plane_sweep (2 leaves the
 * choice to the plan, as a call under the default options would) and kept
 * unless a candidate is faster by more than keep_within (a fraction, e.g.
 * 0.03); a current shape with rb > 32 (outside the workspace) is not timed,
 * and the fastest candidate is taken; on exit the choice.  Each candidate
 * runs once untimed, then `reps` times between HIP events on
 * `stream`; the call synchronises with `stream` and returns after timing
 * (it is not capturable).  The noise's first_sample is used for every run;
 * the level's samples and accumulator are not touched (scratch in ws).
 * Results are cached in the handle by (device, lattice shape, precision,
 * level kinds and degrees, deflation size, nrhs): a repeated call returns
 * the cached choice with *cached = 1 and times nothing.  results (nullable)
 * receives up to max_results timings, *n_results (nullable) their count. */
int mpmc_autotune(mpmc_handle h, const mpmc_lattice *lat, const mpmc_level *level, int32_t nrhs,
                  const mpmc_noise *noise, int32_t reps, double keep_within, void *ws, size_t ws_bytes,
                  mpmc_tune_choice *best, double *best_seconds, int32_t *cached, mpmc_tune_result *results,
                  int32_t max_results, int32_t *n_results, void *stream);

/* Host helper: inverse of a k x k complex FP64 matrix (row-major (re, im)
 * pairs, host memory) by Gaussian elimination with partial pivoting; used
 * for H^{-1}, H = U^H A V, of the Left-right Projection (Sec. 2.1).
 * MPMC_ESINGULAR when a pivot is below tiny * max |entry| (nothing is
 * written to out then); a and out may not overlap. */
int mpmc_small_inverse(int32_t k, const double *a, double tiny, double *out);

/* ---- a level entry point that allocates nothing -------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, semantics and results (bit for bit) as mpmc_mlmc_level_estimate
 * without ws/ws_bytes: the workspace is a static device array of
 * mpmc_noalloc_scratch_bytes() bytes (64 MiB) that the library holds on
 * every GPU it runs on until the process ends.  A level whose
 * mpmc_level_workspace_size exceeds it returns MPMC_EWORKSPACE before
 * anything is enqueued.  The call allocates nothing (no hipMalloc, no
 * allocating library routine).  Every call on one GPU shares that GPU's
 * array: calls that may overlap on one GPU (different streams or threads)
 * race on it; serialise them.  Nothing in the array has to start at zero. */
size_t mpmc_noalloc_scratch_bytes(void);
int mpmc_mlmc_level_estimate_noalloc(const mpmc_lattice *lat, const mpmc_level *level, mpmc_shape shape,
                                     const mpmc_noise *noise, double *samples, double *acc, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MPMC_H */
