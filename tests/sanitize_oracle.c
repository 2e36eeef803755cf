/* Driver for the oracle's C reference under AddressSanitizer and UBSan
 * (built and run by tests/test_sanitizers.py).  Every entry point runs on
 * small lattices with odd and unit extents -- where the periodic index
 * arithmetic wraps -- with buffers of exactly the documented size, so any
 * out-of-bounds access or undefined operation aborts the run.  A few exact
 * identities are checked on the way: kappa = 0 gives A = I, gamma_5 is an
 * involution, the Newton polynomial of one root is that root times x. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;
void ora_gamma(int mu, double *out);
void ora_gamma5_matrix(double *out);
void ora_wilson_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U, const cplx *x, cplx *y,
                      int nrhs);
void ora_gamma5(int64_t V, const cplx *x, cplx *y, int nrhs);
uint64_t ora_splitmix64(uint64_t x, uint64_t k);
uint64_t ora_noise_key(uint64_t seed, uint64_t lattice, uint64_t level);
void ora_z4_fill(uint64_t seed, uint64_t lattice, uint64_t level, uint64_t first, int nsamples, int64_t n, cplx *out);
void ora_poly_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U, int nroots, const cplx *inv_roots,
                    const cplx *B, cplx *Y, cplx *bhy, int nrhs);
void ora_composite_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U, int n_in, const cplx *inv_in,
                         int n_out, const cplx *inv_out, const cplx *B, cplx *Y, cplx *bhy, int nrhs);
void ora_residual_poly_apply(const int *L, int antiperiodic_t, double kappa, const cplx *U, int nroots,
                             const cplx *inv_roots, const cplx *B, cplx *Y, int nrhs);

static uint64_t state = 12345;
static double rnd(void) {
    state = ora_splitmix64(state, 1);
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}
static cplx *filled(size_t n) {
    cplx *p = (cplx *)malloc(n * sizeof(cplx));
    for (size_t i = 0; i < n; ++i) p[i] = rnd() + I * rnd();
    return p;
}
static int fail(const char *what, const int *L) {
    printf("FAIL %s on %dx%dx%dx%d\n", what, L[0], L[1], L[2], L[3]);
    return 1;
}

int main(void) {
    const int lats[4][4] = {{1, 1, 1, 1}, {2, 3, 1, 5}, {3, 1, 2, 2}, {1, 4, 3, 1}};
    double g[32];
    for (int mu = 0; mu < 4; ++mu) ora_gamma(mu, g);
    ora_gamma5_matrix(g);
    for (int li = 0; li < 4; ++li) {
        const int *L = lats[li];
        const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3], n = 12 * V;
        const int nrhs = 2;
        cplx *U = filled((size_t)(36 * V)), *x = filled((size_t)(n * nrhs)), *y = filled((size_t)(n * nrhs));
        cplx *z = filled((size_t)(n * nrhs)), *bhy = filled(nrhs);
        for (int ap = 0; ap < 2; ++ap) {
            ora_wilson_apply(L, ap, 0.0, U, x, y, nrhs);
            for (int64_t i = 0; i < n * nrhs; ++i)
                if (y[i] != x[i]) return fail("kappa = 0 identity", L);
            ora_wilson_apply(L, ap, 0.13, U, x, y, nrhs);
        }
        ora_gamma5(V, x, y, nrhs);
        ora_gamma5(V, y, z, nrhs);
        for (int64_t i = 0; i < n * nrhs; ++i)
            if (z[i] != x[i]) return fail("gamma_5 involution", L);
        ora_z4_fill(7, 1, 2, 3, nrhs, n, z);
        const cplx t1[1] = {0.75 + 0.25 * I};
        ora_poly_apply(L, 1, 0.13, U, 1, t1, x, y, bhy, nrhs);
        for (int64_t i = 0; i < n * nrhs; ++i)
            if (cabs(y[i] - t1[0] * x[i]) > 1e-15 * cabs(x[i]) + 1e-300) return fail("degree-0 polynomial", L);
        cplx *tin = filled(3), *tout = filled(2);
        ora_poly_apply(L, 0, 0.13, U, 3, tin, x, y, bhy, nrhs);
        ora_composite_apply(L, 1, 0.13, U, 3, tin, 2, tout, x, y, bhy, nrhs);
        ora_composite_apply(L, 0, 0.13, U, 3, tin, 1, tout, x, y, NULL, nrhs);
        ora_residual_poly_apply(L, 1, 0.13, U, 3, tin, x, y, nrhs);
        free(tin); free(tout); free(U); free(x); free(y); free(z); free(bhy);
    }
    if (ora_noise_key(1, 2, 3) == ora_noise_key(1, 2, 4)) return 1;
    printf("ok\n");
    return 0;
}
