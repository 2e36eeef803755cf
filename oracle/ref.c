/*
 * Oracle (test infrastructure only): plain, slow, obviously correct FP64
 * implementations of the operations on the trace-estimation hot path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library; the product path never does.
 *
 * Layouts are canonical:
 *   site   s = x + Lx*(y + Ly*(z + Lz*t))
 *   vector index i = 12*s + 3*spin + colour
 *   gauge  U[((mu*V + s)*3 + row)*3 + col], mu = 0..3 for x, y, z, t
 *   batch of N vectors: vector r occupies [r*12V, (r+1)*12V)
 *
 * Built with -O2 -ffp-contract=off and no fast-math, so every product and
 * sum is rounded exactly as written.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Dirac matrices, DeGrand-Rossi (chiral) basis, written out in full.  */
/* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).     */
/* ------------------------------------------------------------------ */
static const cplx GAMMA[4][4][4] = {
    /* gamma_1 */
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    /* gamma_2 */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_3 */
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    /* gamma_4 */
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

void ora_gamma(int mu, double *out /* 4x4 complex, row-major, re/im interleaved */)
{
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            out[2 * (4 * a + b)] = creal(GAMMA[mu][a][b]);
            out[2 * (4 * a + b) + 1] = cimag(GAMMA[mu][a][b]);
        }
}

/* neighbour of site s in direction mu, step +1 or -1; *sign gets -1 when the
 * hop wraps around the time boundary of an antiperiodic lattice */
static int64_t hop(const int *L, int64_t s, int mu, int step, int antiperiodic_t, double *sign)
{
    int c[4];
    int64_t r = s;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(r % L[d]);
        r /= L[d];
    }
    int v = c[mu] + step;
    *sign = 1.0;
    if (v == L[mu]) {
        v = 0;
        if (mu == 3 && antiperiodic_t) *sign = -1.0;
    } else if (v < 0) {
        v = L[mu] - 1;
        if (mu == 3 && antiperiodic_t) *sign = -1.0;
    }
    c[mu] = v;
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

/*
 * Wilson-Dirac matrix applied to one vector:
 *   (A psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                        + (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
 * with periodic x, y, z and (optionally) antiperiodic t.  The paper names the
 * operator (quenched Wilson-Dirac matrix, Sec. 5 Example 2); this is the
 * hopping-parameter form, with full 4x4 spin matrices and 3x3 colour products.
 */
static void wilson_one(const int *L, int antiperiodic_t, double kappa, const cplx *U,
                       const cplx *x, cplx *y)
{
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx acc[4][3];
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) acc[sp][a] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                double sign;
                const int64_t nb = hop(L, s, mu, dir == 0 ? +1 : -1, antiperiodic_t, &sign);
                /* colour product: forward uses U_mu(x), backward U_mu(x-mu)^H */
                cplx cu[4][3];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) {
                            cplx u;
                            if (dir == 0)
                                u = U[((mu * V + s) * 3 + a) * 3 + b];
                            else
                                u = conj(U[((mu * V + nb) * 3 + b) * 3 + a]);
                            t += u * x[12 * nb + 3 * sp + b];
                        }
                        cu[sp][a] = sign * t;
                    }
                /* spin product with (1 - gamma_mu) forward, (1 + gamma_mu) backward */
                const double pm = dir == 0 ? -1.0 : 1.0;
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int sq = 0; sq < 4; ++sq) {
                            cplx g = (sp == sq ? 1.0 : 0.0) + pm * GAMMA[mu][sp][sq];
                            t += g * cu[sq][a];
                        }
                        acc[sp][a] += t;
                    }
            }
        }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a)
                y[12 * s + 3 * sp + a] = x[12 * s + 3 * sp + a] - kappa * acc[sp][a];
    }
}

void ora_wilson_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U,
                      const cplx *x, cplx *y, int nrhs)
{
    const int64_t n = 12LL * L[0] * L[1] * L[2] * L[3];
    for (int r = 0; r < nrhs; ++r) wilson_one(L, antiperiodic_t, kappa, U, x + r * n, y + r * n);
}

/* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4, formed by matrix products */
static void gamma5_matrix(cplx g5[4][4])
{
    cplx t[4][4], u[4][4];
    memcpy(t, GAMMA[0], sizeof(t));
    for (int m = 1; m < 4; ++m) {
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx acc = 0;
                for (int c = 0; c < 4; ++c) acc += t[a][c] * GAMMA[m][c][b];
                u[a][b] = acc;
            }
        memcpy(t, u, sizeof(t));
    }
    memcpy(g5, t, sizeof(t));
}

void ora_gamma5_matrix(double *out /* 4x4 complex, re/im interleaved */)
{
    cplx g5[4][4];
    gamma5_matrix(g5);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            out[2 * (4 * a + b)] = creal(g5[a][b]);
            out[2 * (4 * a + b) + 1] = cimag(g5[a][b]);
        }
}

/* y = gamma_5 x for a batch of vectors (spin matrix applied at every site) */
void ora_gamma5(int64_t V, const cplx *x, cplx *y, int nrhs)
{
    cplx g5[4][4];
    gamma5_matrix(g5);
    for (int64_t r = 0; r < nrhs; ++r)
        for (int64_t s = 0; s < V; ++s)
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx acc = 0;
                    for (int sq = 0; sq < 4; ++sq) acc += g5[sp][sq] * x[r * 12 * V + 12 * s + 3 * sq + a];
                    y[r * 12 * V + 12 * s + 3 * sp + a] = acc;
                }
}

/* ------------------------------------------------------------------ */
/* Z4 noise: entries drawn uniformly from {1, i, -1, -i} (Sec. 1), from */
/* a counter-based generator so any entry can be recomputed anywhere.  */
/* The generator is SplitMix64 (Steele, Lea & Flood, OOPSLA 2014):     */
/* output k of a generator with state x is mix(x + k*gamma).           */
/* ------------------------------------------------------------------ */
static const uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ULL;

static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* k-th output (k >= 1) of SplitMix64 started from state x */
uint64_t ora_splitmix64(uint64_t x, uint64_t k) { return sm_mix(x + k * SM_GAMMA); }

/* stream key of (seed, lattice, level): three chained first outputs */
uint64_t ora_noise_key(uint64_t seed, uint64_t lattice, uint64_t level)
{
    uint64_t k = ora_splitmix64(seed, 1);
    k = ora_splitmix64(k ^ lattice, 1);
    k = ora_splitmix64(k ^ level, 1);
    return k;
}

/*
 * Fill nsamples Z4 vectors of length n = 12V.  Sample r (global index
 * first + j) uses the generator with state S = first output from (key ^ r);
 * entry i takes the 2-bit field (i mod 32) of output number floor(i/32)+1,
 * and q = 0,1,2,3 gives 1, i, -1, -i.
 */
void ora_z4_fill(uint64_t seed, uint64_t lattice, uint64_t level, uint64_t first,
                 int nsamples, int64_t n, cplx *out)
{
    const uint64_t key = ora_noise_key(seed, lattice, level);
    for (int j = 0; j < nsamples; ++j) {
        const uint64_t S = ora_splitmix64(key ^ (first + (uint64_t)j), 1);
        for (int64_t i = 0; i < n; ++i) {
            const uint64_t word = ora_splitmix64(S, (uint64_t)(i / 32) + 1);
            const unsigned q = (unsigned)((word >> (2 * (i % 32))) & 3u);
            cplx b;
            switch (q) {
            case 0: b = 1.0; break;
            case 1: b = I; break;
            case 2: b = -1.0; break;
            default: b = -I; break;
            }
            out[(int64_t)j * n + i] = b;
        }
    }
}

/* ------------------------------------------------------------------ */
/* GMRES polynomial applied to vectors (Sec. 2.3, Sec. 3.1).           */
/* With residual polynomial pi(a) = prod_j (1 - a/theta_j) = 1 - a p(a) */
/* over d+1 roots, p(a) = sum_j theta_j^{-1} prod_{i<j} (1 - a/theta_i): */
/* w_1 = b, y = sum_j theta_j^{-1} w_j, w_{j+1} = w_j - theta_j^{-1} A w_j. */
/* inv_roots holds theta_j^{-1} in the order the roots are to be taken. */
/* ------------------------------------------------------------------ */
typedef void (*ora_op)(void *ctx, const cplx *x, cplx *y); /* y = Op x for one vector */

typedef struct {
    const int *L;
    int antiperiodic_t;
    double kappa;
    const cplx *U;
} wilson_ctx;

static void wilson_op(void *c, const cplx *x, cplx *y)
{
    const wilson_ctx *w = (const wilson_ctx *)c;
    wilson_one(w->L, w->antiperiodic_t, w->kappa, w->U, x, y);
}

/* y = p(Op) b with p given by its nroots inverse roots (degree nroots-1) */
static void newton_poly(ora_op op, void *ctx, int64_t n, int nroots, const cplx *inv_roots,
                        const cplx *b, cplx *y)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * n);
    cplx *aw = (cplx *)malloc(sizeof(cplx) * n);
    memcpy(w, b, sizeof(cplx) * n);
    for (int64_t i = 0; i < n; ++i) y[i] = 0;
    for (int j = 0; j < nroots; ++j) {
        const cplx t = inv_roots[j];
        for (int64_t i = 0; i < n; ++i) y[i] += t * w[i];
        if (j + 1 < nroots) {
            op(ctx, w, aw);
            for (int64_t i = 0; i < n; ++i) w[i] = w[i] - t * aw[i];
        }
    }
    free(w);
    free(aw);
}

/* Y[r] = p(A) B[r]; if bhy != NULL also bhy[r] = B[r]^H p(A) B[r] */
void ora_poly_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U, int nroots,
                    const cplx *inv_roots, const cplx *B, cplx *Y, cplx *bhy, int nrhs)
{
    wilson_ctx ctx = {L, antiperiodic_t, kappa, U};
    const int64_t n = 12LL * L[0] * L[1] * L[2] * L[3];
    for (int r = 0; r < nrhs; ++r) {
        newton_poly(wilson_op, &ctx, n, nroots, inv_roots, B + r * n, Y + r * n);
        if (bhy) {
            cplx acc = 0;
            for (int64_t i = 0; i < n; ++i) acc += conj(B[r * n + i]) * Y[r * n + i];
            bhy[r] = acc;
        }
    }
}

/*
 * Composite ("double") polynomial of Sec. 2.4 / Sec. 3.2:
 *   p_1(A) = p_in(A) p_out(A p_in(A)),
 * applied as written: the operator Bop(v) = A (p_in(A) v), p_out(Bop) by its
 * own inverse roots, then p_in(A) once more.
 */
typedef struct {
    wilson_ctx *w;
    int64_t n;
    int n_in;
    const cplx *inv_in;
    cplx *tmp;
} pp_ctx;

static void pp_op(void *c, const cplx *x, cplx *y)
{
    pp_ctx *p = (pp_ctx *)c;
    newton_poly(wilson_op, p->w, p->n, p->n_in, p->inv_in, x, p->tmp);
    wilson_op(p->w, p->tmp, y);
}

void ora_composite_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U, int n_in,
                         const cplx *inv_in, int n_out, const cplx *inv_out, const cplx *B, cplx *Y,
                         cplx *bhy, int nrhs)
{
    wilson_ctx w = {L, antiperiodic_t, kappa, U};
    const int64_t n = 12LL * L[0] * L[1] * L[2] * L[3];
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * n);
    cplx *z = (cplx *)malloc(sizeof(cplx) * n);
    pp_ctx p = {&w, n, n_in, inv_in, tmp};
    for (int r = 0; r < nrhs; ++r) {
        newton_poly(pp_op, &p, n, n_out, inv_out, B + r * n, z);
        newton_poly(wilson_op, &w, n, n_in, inv_in, z, Y + r * n);
        if (bhy) {
            cplx acc = 0;
            for (int64_t i = 0; i < n; ++i) acc += conj(B[r * n + i]) * Y[r * n + i];
            bhy[r] = acc;
        }
    }
    free(tmp);
    free(z);
}

/* y_r = prod_j (1 - A/theta_j) b_r, the residual polynomial itself */
void ora_residual_poly_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U,
                             int nroots, const cplx *inv_roots, const cplx *B, cplx *Y, int nrhs)
{
    wilson_ctx ctx = {L, antiperiodic_t, kappa, U};
    const int64_t n = 12LL * L[0] * L[1] * L[2] * L[3];
    cplx *aw = (cplx *)malloc(sizeof(cplx) * n);
    for (int r = 0; r < nrhs; ++r) {
        cplx *w = Y + r * n;
        memcpy(w, B + r * n, sizeof(cplx) * n);
        for (int j = 0; j < nroots; ++j) {
            wilson_op(&ctx, w, aw);
            for (int64_t i = 0; i < n; ++i) w[i] = w[i] - inv_roots[j] * aw[i];
        }
    }
    free(aw);
}
