/*
 * so3_oracle.c -- plain, slow, CPU reference for the fast Fourier transform on
 * SO(3) (Kostelec-Rockmore FSOFT / iFSOFT as reviewed by Lux, Wuelker and
 * Chirikjian, "Parallelization of the FFT on SO(3)").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * The file is compiled twice: once with REAL = double (symbols *_f64) and
 * once with -DSO3O_LONG_DOUBLE, REAL = long double (x87 80-bit, symbols
 * *_f80).  Every public function takes and returns IEEE double arrays; the
 * long-double build only computes in extended precision and rounds once on
 * output.
 *
 * Conventions (all from Sect. 2 of the paper):
 *   grid    f[i][j][k] = f(alpha_i, beta_j, gamma_k), i, j, k in [0, 2B),
 *           row-major with k fastest, interleaved complex (re, im).
 *   angles  alpha_i = i pi / B, beta_j = (2j+1) pi / (4B), gamma_k = k pi / B
 *           (sampling theorem, eq. "quadrature").
 *   coeffs  f°(l,m,m') at flat index l(4l^2-1)/3 + (m+l)(2l+1) + (m'+l),
 *           0 <= l < B, m and m' ascending from -l to l (the B(4B^2-1)/3
 *           coefficients counted in Sect. 2.4), interleaved complex.
 *   d       d(l,m,m';beta) exactly as the paper's explicit Jacobi-polynomial
 *           definition in Sect. 2.2 (which is the transpose of the
 *           Wikipedia / Sakurai ordering d^l_{m m'}).
 *
 * Readings taken where the paper is silent:
 *   R1  the three-term recurrence (eq. "Wigner_d_recurrence") is stated for
 *       l >= 1.  For m = m' = 0 it is started at l = 0 with the 0/0 ratio
 *       m m'/(l(l+1)) and the d(l-1) term both taken as 0, so d(1,0,0) = cos b.
 *   R2  at the seed degree l0 = max(|m|,|m'|) the d(l0-1) term has the exact
 *       coefficient 0 (one of l0^2 - m^2, l0^2 - m'^2 vanishes) and is dropped.
 *   R3  when |m| = |m'| both seed formulas of Sect. 2.2 apply; the one with
 *       the first order index at +-l0 is used when |m| >= |m'|.
 *   R4  seeds are evaluated in log space (lgamma, log cos, log sin, exp); the
 *       factorial (2l0)! overflows a double for l0 >= 86.
 *   R5  the separation of variables (Sect. 2.4) keeps only |m|,|m'| <= B-1 of
 *       the 2B x 2B DFT; the forward transform ignores the +-B bin and the
 *       inverse transform writes 0 into it.
 *   R6  forward S carries the e^{+i(m alpha + m' gamma)} kernel unnormalised
 *       (Sect. 2.4); the inverse grid is the plain sum of eq.
 *       "fourier_representation", i.e. an unnormalised e^{-i} 2-D DFT of
 *       S'(j;m,m') = sum_l d(l,m,m';beta_j) f°(l,m,m').
 */
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef SO3O_LONG_DOUBLE
#define REAL long double
#define SUFFIX(name) name##_f80
#else
#define REAL double
#define SUFFIX(name) name##_f64
#endif

typedef REAL real;

#define API __attribute__((visibility("default")))

static real pi_r(void) { return acos((real)-1); }

/* ------------------------------------------------------------------------- */
/* Indexing                                                                  */
/* ------------------------------------------------------------------------- */

/* Flat coefficient index of (l, m, m'), the layout stated in the header. */
static long coeff_index(int l, int m, int mp)
{
    long L = l;
    return L * (4 * L * L - 1) / 3 + (long)(m + l) * (2 * l + 1) + (mp + l);
}

static int iabs_(int a) { return a < 0 ? -a : a; }

/* ------------------------------------------------------------------------- */
/* Quadrature weights, eq. "weights" (sampling theorem, Sect. 2.3)           */
/* ------------------------------------------------------------------------- */

static void weights_r(int B, real *w)
{
    const real PI = pi_r();
    for (int j = 0; j < 2 * B; ++j) {
        real beta = (real)(2 * j + 1) * PI / (real)(4 * B);
        real s = 0;
        for (int i = 0; i < B; ++i)
            s += sin((real)(2 * i + 1) * beta) / (real)(2 * i + 1);
        w[j] = (real)2 * PI * sin(beta) / ((real)B * (real)B) * s;
    }
}

/* ------------------------------------------------------------------------- */
/* Wigner-d: seeds of Sect. 2.2 + three-term recurrence in l                 */
/* ------------------------------------------------------------------------- */

/* Seed d(l0, m, m'; beta) at l0 = max(|m|, |m'|) (Sect. 2.2 "initial cases"),
 * evaluated in log space (reading R4).  The two families:
 *   d(l0, +-l0, m') = sqrt((2 l0)! / ((l0+m')!(l0-m')!)) cos^{l0+-m'}(b/2) (+-sin(b/2))^{l0-+m'}
 *   d(l0, m, +-l0)  = sqrt((2 l0)! / ((l0+m)!(l0-m)!))   cos^{l0+-m}(b/2)  (-+sin(b/2))^{l0-+m}
 */
static real seed_r(int m, int mp, real beta)
{
    int am = iabs_(m), amp = iabs_(mp);
    int l0 = am > amp ? am : amp;
    int k, p, q, neg;
    if (am >= amp) {            /* first order index is +-l0 (reading R3) */
        k = mp;
        if (m >= 0) { p = l0 + k; q = l0 - k; neg = 0; }
        else        { p = l0 - k; q = l0 + k; neg = q & 1; }
    } else {                    /* second order index is +-l0 */
        k = m;
        if (mp > 0) { p = l0 + k; q = l0 - k; neg = q & 1; }
        else        { p = l0 - k; q = l0 + k; neg = 0; }
    }
    real logbin = (lgamma((real)(2 * l0 + 1)) - lgamma((real)(l0 + k + 1))
                   - lgamma((real)(l0 - k + 1))) / (real)2;
    real e = logbin;
    if (p) e += (real)p * log(cos(beta / (real)2));
    if (q) e += (real)q * log(sin(beta / (real)2));
    real v = exp(e);
    return neg ? -v : v;
}

/* d(l, m, m'; beta) for l = 0 .. B-1 (zero for l < max(|m|,|m'|)), by the
 * three-term recurrence of eq. "Wigner_d_recurrence" from the seed. */
static void wigner_d_r(int B, int m, int mp, real beta, real *d)
{
    int l0 = iabs_(m) > iabs_(mp) ? iabs_(m) : iabs_(mp);
    for (int l = 0; l < B; ++l) d[l] = 0;
    if (l0 >= B) return;
    real x = cos(beta);
    real dprev = 0, dcur = seed_r(m, mp, beta);
    d[l0] = dcur;
    real M = (real)m, MP = (real)mp;
    for (int l = l0; l + 1 < B; ++l) {
        real L = (real)l, L1 = (real)(l + 1);
        real den = sqrt((L1 * L1 - M * M) * (L1 * L1 - MP * MP));
        real a = L1 * ((real)2 * L + 1) / den;
        real ratio = 0, b = 0;                        /* reading R1 at l = 0 */
        if (l > 0) {
            ratio = M * MP / (L * L1);
            if (l > l0)                               /* reading R2 at l = l0 */
                b = L1 * sqrt((L * L - M * M) * (L * L - MP * MP)) / (L * den);
        }
        real dn = a * (x - ratio) * dcur - b * dprev;
        d[l + 1] = dn;
        dprev = dcur;
        dcur = dn;
    }
}

/* ------------------------------------------------------------------------- */
/* Textbook 1-D / 2-D DFT: radix-2 for powers of two, direct sum otherwise   */
/* ------------------------------------------------------------------------- */

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

/* Unnormalised DFT of n complex values x[0], x[s], ..., x[(n-1)s] in place:
 * X[q] = sum_p x[p] exp(sign * 2 pi i p q / n). */
static void dft1_r(int n, int sign, real *x, long s, real *tmp)
{
    const real PI = pi_r();
    if (is_pow2(n)) {
        for (int p = 0; p < n; ++p) {               /* bit-reversed copy */
            int r = 0;
            for (int b = 1, t = p; b < n; b <<= 1, t >>= 1) r = (r << 1) | (t & 1);
            tmp[2 * r] = x[2 * p * s];
            tmp[2 * r + 1] = x[2 * p * s + 1];
        }
        for (int len = 2; len <= n; len <<= 1) {     /* iterative butterflies */
            for (int k = 0; k < len / 2; ++k) {
                real ang = (real)sign * (real)2 * PI * (real)k / (real)len;
                real c = cos(ang), sn = sin(ang);
                for (int st = 0; st < n; st += len) {
                    real *u = tmp + 2 * (st + k), *v = tmp + 2 * (st + k + len / 2);
                    real vr = v[0] * c - v[1] * sn, vi = v[0] * sn + v[1] * c;
                    v[0] = u[0] - vr; v[1] = u[1] - vi;
                    u[0] += vr;       u[1] += vi;
                }
            }
        }
    } else {
        for (int q = 0; q < n; ++q) {
            real ar = 0, ai = 0;
            for (int p = 0; p < n; ++p) {
                real ang = (real)sign * (real)2 * PI * (real)(((long)p * q) % n) / (real)n;
                real c = cos(ang), sn = sin(ang);
                real xr = x[2 * p * s], xi = x[2 * p * s + 1];
                ar += xr * c - xi * sn;
                ai += xr * sn + xi * c;
            }
            tmp[2 * q] = ar; tmp[2 * q + 1] = ai;
        }
    }
    for (int q = 0; q < n; ++q) {
        x[2 * q * s] = tmp[2 * q];
        x[2 * q * s + 1] = tmp[2 * q + 1];
    }
}

/* Unnormalised 2-D DFT of an n x n row-major complex array in place. */
static void dft2_r(int n, int sign, real *a, real *tmp)
{
    for (int r = 0; r < n; ++r) dft1_r(n, sign, a + 2L * r * n, 1, tmp);
    for (int c = 0; c < n; ++c) dft1_r(n, sign, a + 2L * c, n, tmp);
}

/* ------------------------------------------------------------------------- */
/* Transform steps (Sect. 2.4)                                               */
/* ------------------------------------------------------------------------- */

/* S(m,m';j) = sum_{i,k} f(alpha_i,beta_j,gamma_k) e^{+i(m alpha_i + m' gamma_k)}
 * for |m|,|m'| <= B-1, stored S[pair][j] with pair = (m+B-1)(2B-1) + (m'+B-1). */
static void separation_forward(int B, const double *grid, real *S)
{
    const int N = 2 * B, P = 2 * B - 1;
#pragma omp parallel
    {
        real *a = malloc(sizeof(real) * 2L * N * N);
        real *tmp = malloc(sizeof(real) * 2L * N);
#pragma omp for schedule(dynamic)
        for (int j = 0; j < N; ++j) {
            for (int i = 0; i < N; ++i)
                for (int k = 0; k < N; ++k) {
                    long g = (((long)i * N + j) * N + k) * 2;
                    a[2 * ((long)i * N + k)] = (real)grid[g];
                    a[2 * ((long)i * N + k) + 1] = (real)grid[g + 1];
                }
            dft2_r(N, +1, a, tmp);
            for (int m = 1 - B; m < B; ++m)
                for (int mp = 1 - B; mp < B; ++mp) {
                    int im = (m + N) % N, imp = (mp + N) % N;
                    long pair = (long)(m + B - 1) * P + (mp + B - 1);
                    S[2 * (pair * N + j)] = a[2 * ((long)im * N + imp)];
                    S[2 * (pair * N + j) + 1] = a[2 * ((long)im * N + imp) + 1];
                }
        }
        free(a); free(tmp);
    }
}

/* f_ijk = sum_{m,m'} S'(j;m,m') e^{-i(m alpha_i + m' gamma_k)}, the +-B bin 0. */
static void separation_inverse(int B, const real *S, double *grid)
{
    const int N = 2 * B, P = 2 * B - 1;
#pragma omp parallel
    {
        real *a = malloc(sizeof(real) * 2L * N * N);
        real *tmp = malloc(sizeof(real) * 2L * N);
#pragma omp for schedule(dynamic)
        for (int j = 0; j < N; ++j) {
            memset(a, 0, sizeof(real) * 2L * N * N);
            for (int m = 1 - B; m < B; ++m)
                for (int mp = 1 - B; mp < B; ++mp) {
                    int im = (m + N) % N, imp = (mp + N) % N;
                    long pair = (long)(m + B - 1) * P + (mp + B - 1);
                    a[2 * ((long)im * N + imp)] = S[2 * (pair * N + j)];
                    a[2 * ((long)im * N + imp) + 1] = S[2 * (pair * N + j) + 1];
                }
            dft2_r(N, -1, a, tmp);
            for (int i = 0; i < N; ++i)
                for (int k = 0; k < N; ++k) {
                    long g = (((long)i * N + j) * N + k) * 2;
                    grid[g] = (double)a[2 * ((long)i * N + k)];
                    grid[g + 1] = (double)a[2 * ((long)i * N + k) + 1];
                }
        }
        free(a); free(tmp);
    }
}

/* DWT of one order pair: out(l) = vscale(l) sum_j wj d(l,m,m';beta_j) S(j)
 * with vscale = (2l+1)/(8 pi B) when apply_v (Sect. 2.4 matrix form V T W). */
static void dwt_pair(int B, int m, int mp, const real *w, int apply_v,
                     const real *Sp, double *coeffs, real *d, real *acc)
{
    const int N = 2 * B;
    const real PI = pi_r();
    int l0 = iabs_(m) > iabs_(mp) ? iabs_(m) : iabs_(mp);
    for (int l = 0; l < B; ++l) { acc[2 * l] = 0; acc[2 * l + 1] = 0; }
    for (int j = 0; j < N; ++j) {
        real beta = (real)(2 * j + 1) * PI / (real)(4 * B);
        wigner_d_r(B, m, mp, beta, d);
        real sr = Sp[2 * j], si = Sp[2 * j + 1];
        real wj = w ? w[j] : (real)1;
        for (int l = l0; l < B; ++l) {
            acc[2 * l] += wj * d[l] * sr;
            acc[2 * l + 1] += wj * d[l] * si;
        }
    }
    for (int l = l0; l < B; ++l) {
        real v = apply_v ? (real)(2 * l + 1) / ((real)8 * PI * (real)B) : (real)1;
        long c = coeff_index(l, m, mp);
        coeffs[2 * c] = (double)(v * acc[2 * l]);
        coeffs[2 * c + 1] = (double)(v * acc[2 * l + 1]);
    }
}

/* iDWT of one order pair: S'(j) = sum_l d(l,m,m';beta_j) vscale(l) f°(l,m,m')
 * (Sect. 2.4, T^T), with vscale = (2l+1)/(8 pi B) only for the adjoint. */
static void idwt_pair(int B, int m, int mp, int apply_v, const double *coeffs,
                      real *Sp, real *d)
{
    const int N = 2 * B;
    const real PI = pi_r();
    int l0 = iabs_(m) > iabs_(mp) ? iabs_(m) : iabs_(mp);
    for (int j = 0; j < N; ++j) {
        real beta = (real)(2 * j + 1) * PI / (real)(4 * B);
        wigner_d_r(B, m, mp, beta, d);
        real sr = 0, si = 0;
        for (int l = l0; l < B; ++l) {
            long c = coeff_index(l, m, mp);
            real v = apply_v ? (real)(2 * l + 1) / ((real)8 * PI * (real)B) : (real)1;
            sr += d[l] * v * (real)coeffs[2 * c];
            si += d[l] * v * (real)coeffs[2 * c + 1];
        }
        Sp[2 * j] = sr;
        Sp[2 * j + 1] = si;
    }
}

/* Shared driver: forward (apply_w = apply_v = 1) and the adjoint of the
 * inverse (both 0). */
static int forward_common(int B, const double *grid, double *coeffs, int scaled)
{
    if (B < 1 || !grid || !coeffs) return -1;
    const int N = 2 * B, P = 2 * B - 1;
    real *S = malloc(sizeof(real) * 2L * P * P * N);
    real *w = malloc(sizeof(real) * N);
    if (!S || !w) { free(S); free(w); return -3; }
    separation_forward(B, grid, S);
    weights_r(B, w);
#pragma omp parallel
    {
        real *d = malloc(sizeof(real) * B);
        real *acc = malloc(sizeof(real) * 2L * B);
#pragma omp for schedule(dynamic)
        for (long pair = 0; pair < (long)P * P; ++pair) {
            int m = (int)(pair / P) - (B - 1), mp = (int)(pair % P) - (B - 1);
            dwt_pair(B, m, mp, scaled ? w : NULL, scaled, S + 2 * pair * N, coeffs, d, acc);
        }
        free(d); free(acc);
    }
    free(S); free(w);
    return 0;
}

/* Shared driver: inverse (scaled = 0) and the adjoint of the forward
 * (scaled = 1: coefficients scaled by V first, grid slices by W after). */
static int inverse_common(int B, const double *coeffs, double *grid, int scaled)
{
    if (B < 1 || !grid || !coeffs) return -1;
    const int N = 2 * B, P = 2 * B - 1;
    real *S = malloc(sizeof(real) * 2L * P * P * N);
    if (!S) return -3;
#pragma omp parallel
    {
        real *d = malloc(sizeof(real) * B);
#pragma omp for schedule(dynamic)
        for (long pair = 0; pair < (long)P * P; ++pair) {
            int m = (int)(pair / P) - (B - 1), mp = (int)(pair % P) - (B - 1);
            idwt_pair(B, m, mp, scaled, coeffs, S + 2 * pair * N, d);
        }
        free(d);
    }
    separation_inverse(B, S, grid);
    free(S);
    if (scaled) {
        real *w = malloc(sizeof(real) * N);
        weights_r(B, w);
        for (long i = 0; i < N; ++i)
            for (long j = 0; j < N; ++j)
                for (long k = 0; k < N; ++k) {
                    long g = ((i * N + j) * N + k) * 2;
                    grid[g] = (double)((real)grid[g] * w[j]);
                    grid[g + 1] = (double)((real)grid[g + 1] * w[j]);
                }
        free(w);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Public entry points                                                       */
/* ------------------------------------------------------------------------- */

/* Quadrature weights w_B(j), j < 2B (eq. "weights"). */
API int SUFFIX(so3o_weights)(int B, double *w)
{
    if (B < 1 || !w) return -1;
    real *t = malloc(sizeof(real) * 2 * B);
    weights_r(B, t);
    for (int j = 0; j < 2 * B; ++j) w[j] = (double)t[j];
    free(t);
    return 0;
}

/* d(l,m,m';beta) for l < B (Sect. 2.2 seeds + eq. "Wigner_d_recurrence"). */
API int SUFFIX(so3o_wigner_d)(int B, int m, int mp, double beta, double *d)
{
    if (B < 1 || !d) return -1;
    real *t = malloc(sizeof(real) * B);
    wigner_d_r(B, m, mp, (real)beta, t);
    for (int l = 0; l < B; ++l) d[l] = (double)t[l];
    free(t);
    return 0;
}

/* Same, with beta given as beta_j of the bandwidth-B grid (exact in REAL). */
API int SUFFIX(so3o_wigner_d_grid)(int B, int m, int mp, int j, double *d)
{
    if (B < 1 || !d || j < 0 || j >= 2 * B) return -1;
    real *t = malloc(sizeof(real) * B);
    real beta = (real)(2 * j + 1) * pi_r() / (real)(4 * B);
    wigner_d_r(B, m, mp, beta, t);
    for (int l = 0; l < B; ++l) d[l] = (double)t[l];
    free(t);
    return 0;
}

/* Unnormalised 2-D DFT of an n x n complex array, exp(sign 2 pi i (.)/n). */
API int SUFFIX(so3o_dft2)(int n, int sign, double *a)
{
    if (n < 1 || !a || (sign != 1 && sign != -1)) return -1;
    real *t = malloc(sizeof(real) * 2L * n * n), *tmp = malloc(sizeof(real) * 2L * n);
    for (long i = 0; i < 2L * n * n; ++i) t[i] = (real)a[i];
    dft2_r(n, sign, t, tmp);
    for (long i = 0; i < 2L * n * n; ++i) a[i] = (double)t[i];
    free(t); free(tmp);
    return 0;
}

/* FSOFT: coefficients f°(l,m,m') of a grid (eq. "quadrature" through the
 * separation of variables of Sect. 2.4). */
API int SUFFIX(so3o_forward)(int B, const double *grid, double *coeffs)
{
    return forward_common(B, grid, coeffs, 1);
}

/* iFSOFT: grid values of eq. "fourier_representation" on the sampling grid. */
API int SUFFIX(so3o_inverse)(int B, const double *coeffs, double *grid)
{
    return inverse_common(B, coeffs, grid, 0);
}

/* Adjoint of the forward transform, F^H = W I V (W scales beta-slice j by
 * w_B(j), V scales degree l by (2l+1)/(8 pi B)). */
API int SUFFIX(so3o_adjoint)(int B, const double *coeffs, double *grid)
{
    return inverse_common(B, coeffs, grid, 1);
}

/* Adjoint of the inverse transform, I^H = V^-1 F W^-1: the separation of
 * variables followed by the plain T-contraction with unit weights. */
API int SUFFIX(so3o_adjoint_inverse)(int B, const double *grid, double *coeffs)
{
    return forward_common(B, grid, coeffs, 0);
}

/* Intermediate of the forward transform: S(m,m';j) (unweighted), stored
 * [m+B-1][m'+B-1][j], complex.  Exposed for stage-wise checks. */
API int SUFFIX(so3o_separation_forward)(int B, const double *grid, double *S)
{
    if (B < 1 || !grid || !S) return -1;
    const int N = 2 * B, P = 2 * B - 1;
    real *t = malloc(sizeof(real) * 2L * P * P * N);
    separation_forward(B, grid, t);
    for (long i = 0; i < 2L * P * P * N; ++i) S[i] = (double)t[i];
    free(t);
    return 0;
}

/* Intermediate of the inverse transform: S'(j;m,m') = sum_l d f°, stored
 * [m+B-1][m'+B-1][j], complex. */
API int SUFFIX(so3o_idwt)(int B, const double *coeffs, double *S)
{
    if (B < 1 || !coeffs || !S) return -1;
    const int N = 2 * B, P = 2 * B - 1;
#pragma omp parallel
    {
        real *d = malloc(sizeof(real) * B);
        real *sp = malloc(sizeof(real) * 2L * N);
#pragma omp for schedule(dynamic)
        for (long pair = 0; pair < (long)P * P; ++pair) {
            int m = (int)(pair / P) - (B - 1), mp = (int)(pair % P) - (B - 1);
            idwt_pair(B, m, mp, 0, coeffs, sp, d);
            for (int q = 0; q < 2 * N; ++q) S[2 * pair * N + q] = (double)sp[q];
        }
        free(d); free(sp);
    }
    return 0;
}

/* One beta-slice of the inverse transform, f(alpha_i, beta_j, gamma_k) for
 * all (i, k), as an n x n array (n = 2B).  O(B^3) work; used to sample the
 * inverse at bandwidths where the full oracle is too slow. */
API int SUFFIX(so3o_inverse_slice)(int B, const double *coeffs, int j, double *slice)
{
    if (B < 1 || !coeffs || !slice || j < 0 || j >= 2 * B) return -1;
    const int N = 2 * B;
    const real PI = pi_r();
    real *a = calloc(2L * N * N, sizeof(real));
    real *tmp = malloc(sizeof(real) * 2L * N);
    real beta = (real)(2 * j + 1) * PI / (real)(4 * B);
#pragma omp parallel
    {
        real *d = malloc(sizeof(real) * B);
#pragma omp for schedule(dynamic)
        for (int m = 1 - B; m < B; ++m)
            for (int mp = 1 - B; mp < B; ++mp) {
                int l0 = iabs_(m) > iabs_(mp) ? iabs_(m) : iabs_(mp);
                wigner_d_r(B, m, mp, beta, d);
                real sr = 0, si = 0;
                for (int l = l0; l < B; ++l) {
                    long c = coeff_index(l, m, mp);
                    sr += d[l] * (real)coeffs[2 * c];
                    si += d[l] * (real)coeffs[2 * c + 1];
                }
                int im = (m + N) % N, imp = (mp + N) % N;
                a[2 * ((long)im * N + imp)] = sr;
                a[2 * ((long)im * N + imp) + 1] = si;
            }
        free(d);
    }
    dft2_r(N, -1, a, tmp);
    for (long q = 0; q < 2L * N * N; ++q) slice[q] = (double)a[q];
    free(a); free(tmp);
    return 0;
}

/* Forward coefficients f°(l,m,m') for l < B of a few listed order pairs
 * (pairs = [m0, m0', m1, m1', ...]), out[p][l] complex (0 for l below the
 * pair's lowest degree).  Streams the 2-D DFT slice by slice, so memory is
 * O(B^2); used to sample the forward at large bandwidths. */
API int SUFFIX(so3o_forward_pairs)(int B, const double *grid, int npairs,
                                   const int *pairs, double *out)
{
    if (B < 1 || !grid || !out || npairs < 0 || (npairs && !pairs)) return -1;
    const int N = 2 * B;
    const real PI = pi_r();
    for (int p = 0; p < npairs; ++p)
        if (iabs_(pairs[2 * p]) >= B || iabs_(pairs[2 * p + 1]) >= B) return -1;
    real *S = malloc(sizeof(real) * 2L * npairs * N);
#pragma omp parallel
    {
        real *a = malloc(sizeof(real) * 2L * N * N);
        real *tmp = malloc(sizeof(real) * 2L * N);
#pragma omp for schedule(dynamic)
        for (int j = 0; j < N; ++j) {
            for (int i = 0; i < N; ++i)
                for (int k = 0; k < N; ++k) {
                    long g = (((long)i * N + j) * N + k) * 2;
                    a[2 * ((long)i * N + k)] = (real)grid[g];
                    a[2 * ((long)i * N + k) + 1] = (real)grid[g + 1];
                }
            dft2_r(N, +1, a, tmp);
            for (int p = 0; p < npairs; ++p) {
                int im = (pairs[2 * p] + N) % N, imp = (pairs[2 * p + 1] + N) % N;
                S[2 * ((long)p * N + j)] = a[2 * ((long)im * N + imp)];
                S[2 * ((long)p * N + j) + 1] = a[2 * ((long)im * N + imp) + 1];
            }
        }
        free(a); free(tmp);
    }
    real *w = malloc(sizeof(real) * N);
    weights_r(B, w);
    real *d = malloc(sizeof(real) * B);
    for (int p = 0; p < npairs; ++p) {
        int m = pairs[2 * p], mp = pairs[2 * p + 1];
        int l0 = iabs_(m) > iabs_(mp) ? iabs_(m) : iabs_(mp);
        double *o = out + 2L * p * B;
        for (int l = 0; l < 2 * B; ++l) o[l] = 0;
        real *acc = calloc(2L * B, sizeof(real));
        for (int j = 0; j < N; ++j) {
            real beta = (real)(2 * j + 1) * PI / (real)(4 * B);
            wigner_d_r(B, m, mp, beta, d);
            for (int l = l0; l < B; ++l) {
                acc[2 * l] += w[j] * d[l] * S[2 * ((long)p * N + j)];
                acc[2 * l + 1] += w[j] * d[l] * S[2 * ((long)p * N + j) + 1];
            }
        }
        for (int l = l0; l < B; ++l) {
            real v = (real)(2 * l + 1) / ((real)8 * PI * (real)B);
            o[2 * l] = (double)(v * acc[2 * l]);
            o[2 * l + 1] = (double)(v * acc[2 * l + 1]);
        }
        free(acc);
    }
    free(d); free(w); free(S);
    return 0;
}

/* Number of OpenMP threads the oracle runs on. */
API int SUFFIX(so3o_num_threads)(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
