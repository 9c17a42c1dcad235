/*
 * oracle_driver.c -- runs every entry point of the CPU oracle (both the
 * double and the long-double build) at small bandwidths, for a build of the
 * oracle with AddressSanitizer and UndefinedBehaviorSanitizer: any
 * out-of-bounds access, use of freed memory, leak or undefined operation
 * aborts the run.  Also checks that forward(inverse(c)) returns c (the
 * sampling theorem of Sect. 2.3), so the instrumented code computes what the
 * plain build computes.  Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#define DECL(S)                                                                        \
    int so3o_weights_##S(int, double *);                                               \
    int so3o_wigner_d_##S(int, int, int, double, double *);                            \
    int so3o_wigner_d_grid_##S(int, int, int, int, double *);                          \
    int so3o_dft2_##S(int, int, double *);                                             \
    int so3o_forward_##S(int, const double *, double *);                               \
    int so3o_inverse_##S(int, const double *, double *);                               \
    int so3o_adjoint_##S(int, const double *, double *);                               \
    int so3o_adjoint_inverse_##S(int, const double *, double *);                       \
    int so3o_separation_forward_##S(int, const double *, double *);                    \
    int so3o_idwt_##S(int, const double *, double *);                                  \
    int so3o_inverse_slice_##S(int, const double *, int, double *);                    \
    int so3o_forward_pairs_##S(int, const double *, int, const int *, double *);       \
    int so3o_num_threads_##S(void);
DECL(f64)
DECL(f80)

static long ncoef(int B) { return (long)B * (4L * B * B - 1) / 3; }

static double frand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / (double)(1u << 24) - 0.5;
}

#define RUN(S)                                                                                   \
    static int run_##S(int B) {                                                                  \
        const int N = 2 * B, P = 2 * B - 1;                                                      \
        const long nc = ncoef(B), ng = (long)N * N * N;                                          \
        double *c = malloc(sizeof(double) * 2 * nc), *c2 = malloc(sizeof(double) * 2 * nc);      \
        double *g = malloc(sizeof(double) * 2 * ng), *g2 = malloc(sizeof(double) * 2 * ng);      \
        double *w = malloc(sizeof(double) * N), *d = malloc(sizeof(double) * B);                 \
        double *S = malloc(sizeof(double) * 2 * P * P * N), *sl = malloc(sizeof(double) * 2 * N * N); \
        double *a = malloc(sizeof(double) * 2 * N * N), *pr = malloc(sizeof(double) * 2 * 3 * B); \
        unsigned seed = 12345u + (unsigned)B;                                                    \
        int bad = 0;                                                                             \
        for (long i = 0; i < 2 * nc; ++i) c[i] = frand(&seed);                                   \
        for (long i = 0; i < 2 * N * N; ++i) a[i] = frand(&seed);                                \
        bad |= so3o_weights_##S(B, w) | so3o_wigner_d_##S(B, B - 1, 1 - B, 0.3, d);               \
        bad |= so3o_wigner_d_grid_##S(B, 0, 0, N - 1, d) | so3o_dft2_##S(N, 1, a);                \
        bad |= so3o_inverse_##S(B, c, g) | so3o_forward_##S(B, g, c2);                            \
        double err = 0, mx = 0;                                                                  \
        for (long i = 0; i < 2 * nc; ++i) {                                                      \
            err = fmax(err, fabs(c2[i] - c[i]));                                                 \
            mx = fmax(mx, fabs(c[i]));                                                           \
        }                                                                                        \
        if (!(err <= 1e-11 * mx)) {                                                              \
            fprintf(stderr, #S " B=%d round trip %g\n", B, err / mx);                             \
            bad = 1;                                                                             \
        }                                                                                        \
        bad |= so3o_adjoint_##S(B, c, g2) | so3o_adjoint_inverse_##S(B, g, c2);                   \
        bad |= so3o_separation_forward_##S(B, g, S) | so3o_idwt_##S(B, c, S);                     \
        bad |= so3o_inverse_slice_##S(B, c, N - 1, sl);                                          \
        const int pairs[6] = {0, 0, B - 1, 1 - B, 1 - B, B - 1};                                  \
        bad |= so3o_forward_pairs_##S(B, g, 3, pairs, pr);                                       \
        bad |= so3o_num_threads_##S() < 1;                                                       \
        /* invalid arguments are rejected, not read */                                           \
        if (so3o_inverse_slice_##S(B, c, N, sl) != -1 || so3o_weights_##S(0, w) != -1) bad = 1;   \
        free(c); free(c2); free(g); free(g2); free(w); free(d); free(S); free(sl); free(a); free(pr); \
        return bad;                                                                              \
    }
RUN(f64)
RUN(f80)

int main(void) {
    int bad = 0;
    for (int B = 1; B <= 6; ++B) bad |= run_f64(B) | run_f80(B);
    bad |= run_f64(8);
    printf("oracle under sanitizers: %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
