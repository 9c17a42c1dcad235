// sphere.hip -- the ends of the rotational-matching pipeline the paper names
// as an application (Sect. 1): the spherical-harmonic transform of functions
// sampled on the sphere, which gives the a(l, m), b(l, m) the correlation
// head takes, and the read-out of the best rotation from a correlation grid
// with a sub-grid refinement.
//
// Spherical-harmonic transform.  A function on the sphere is sampled at
// (theta_j, phi_k) = ((2j+1) pi/(4B), k pi/B), j, k < 2B (the beta and alpha
// samples of the sampling theorem, Sect. 2.3), stored f[j][k] with k fastest;
//   a(l, m) = sqrt((2l+1)/(4 pi)) sum_j w_B(j) d^l_{m0}(theta_j) F_m(j),
//   F_m(j)  = sum_k f[j][k] e^{-i m phi_k},
// where d^l_{m0} is d(l, 0, m) of Sect. 2.2, i.e. the orthonormal Y_l^m with
// the Condon-Shortley phase, and the quadrature is exact below degree B.
// With the representative d(l) = d(l, |m|, 0; theta) of the symmetry group
// of (|m|, 0) (eq. "Wigner_symmetries"): d(l, 0, |m|) = (-1)^m d(l) and
// d(l, 0, -|m|) = d(l).  One block per (function, |m|), one theta sample per
// lane: the lane forms F_{+|m|}(j) and F_{-|m|}(j) by a direct sum over its
// row with exact twiddles, seeds d(|m|) in log space, runs the three-term
// recurrence of eq. "Wigner_d_recurrence" (at m' = 0 its d(l-1) coefficient
// is sqrt(l^2 - m^2)/sqrt((l+1)^2 - m^2) and it has no constant term), and
// the sums over theta of each degree are reduced across the lanes (a
// butterfly within each wave, then the waves in LDS, 16 degrees at a time).
// Arithmetic is FP64 in every precision; only loads and stores take the
// plan's complex type.
#include <algorithm>

#include "soft_internal.h"

namespace soft {
namespace {

template <typename C>
__global__ __launch_bounds__(1024) void k_sh_forward(int B, const C *__restrict__ f, C *__restrict__ a) {
    using R = decltype(C{}.x);
    extern __shared__ double sh[];  // twiddles e^{-2 pi i t/N} (2N), then partials [wave][16][4]
    const int N = 2 * B;
    const int m = blockIdx.x, fn = blockIdx.y;
    const int NT = blockDim.x, NWV = NT >> 6;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = threadIdx.x;
    const bool jin = j < N;
    double *tw = sh;
    double *part = sh + 2 * N;
    for (int t = threadIdx.x; t < N; t += NT) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)N, &s, &c);
        tw[2 * t] = c;
        tw[2 * t + 1] = s;
    }
    __syncthreads();

    // F_{+m}(j) and F_{-m}(j): direct sums over the lane's row
    double fpr = 0.0, fpi = 0.0, fmr = 0.0, fmi = 0.0;
    if (jin) {
        const C *row = f + ((size_t)fn * N + j) * N;
        for (int k = 0; k < N; ++k) {
            const C v = row[k];
            const int t = (int)(((long long)m * k) % N);
            const double c = tw[2 * t], s = tw[2 * t + 1];  // e^{-i m phi_k} = c + i s
            const double vr = (double)v.x, vi = (double)v.y;
            fpr += vr * c - vi * s;
            fpi += vr * s + vi * c;
            fmr += vr * c + vi * s;  // times e^{+i m phi_k} = c - i s
            fmi += vi * c - vr * s;
        }
    }
    // quadrature weight w_B(j) (eq. "weights"), seed d(m, m, 0; theta_j) and cos theta_j
    const double theta = (2.0 * j + 1.0) * M_PI / (4.0 * B);
    double wj = 0.0, e = 0.0;
    if (jin) {
        double s = 0.0;
        for (int i = 0; i < B; ++i) s += sin((2.0 * i + 1.0) * theta) / (2.0 * i + 1.0);
        wj = 2.0 * M_PI * sin(theta) / ((double)B * B) * s;
        const double lg = 0.5 * (lgamma(2.0 * m + 1.0) - 2.0 * lgamma(m + 1.0)) +
                          (double)m * log(0.5 * sin(theta));
        e = exp(lg);
    }
    const double x = cos(theta);
    const double sgn = (m & 1) ? -1.0 : 1.0;  // d(l, 0, m) = (-1)^m d(l, m, 0)
    double ep = 0.0;
    const int L = B - m;
    C *out = a + (size_t)fn * B * B;
    for (int l0 = 0; l0 < L; l0 += 16) {
        for (int r = 0; r < 16 && l0 + r < L; ++r) {
            const int l = m + l0 + r;
            double v[4] = {wj * e * fpr, wj * e * fpi, wj * e * fmr, wj * e * fmi};
#pragma unroll
            for (int b = 32; b >= 1; b >>= 1)
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], b, 64);
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < 4; ++q) part[(wave * 16 + r) * 4 + q] = v[q];
            // d(l+1) = (2l+1)/sqrt((l+1)^2 - m^2) cos(theta) d(l) - sqrt(l^2 - m^2)/sqrt((l+1)^2 - m^2) d(l-1)
            const double L1 = l + 1.0, M2 = (double)m * m;
            const double den = sqrt(L1 * L1 - M2);
            const double en = ((2.0 * l + 1.0) * x * e - sqrt((double)l * l - M2) * ep) / den;
            ep = e;
            e = en;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < 16 * 2; t += NT) {
            const int r = t >> 1, neg = t & 1, l = m + l0 + r;
            if (l0 + r < L && (!neg || m > 0)) {
                double re = 0.0, im = 0.0;
                for (int w = 0; w < NWV; ++w) {
                    re += part[(w * 16 + r) * 4 + 2 * neg];
                    im += part[(w * 16 + r) * 4 + 2 * neg + 1];
                }
                const double nrm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * (neg ? 1.0 : sgn);
                C o;
                o.x = (R)(re * nrm);
                o.y = (R)(im * nrm);
                out[l * l + l + (neg ? -m : m)] = o;
            }
        }
        __syncthreads();
    }
}

// Read-out of the best rotation of pair p from its correlation grid and the
// grid maximum index[p]: along each axis a parabola through Re C at the
// maximum and its two neighbours (periodic in alpha and gamma; none at the
// first and last beta sample) moves the grid coordinate by
// (c- - c+) / (2 (c- - 2 c0 + c+)) when the three values bend down, clamped
// to [-1/2, 1/2].  The rotation g(w) = f(R^-1 w) of the pair (a = f, b = g)
// is R = Rz(alpha) Ry(beta) Rz(gamma) with (alpha, beta, gamma) = (gamma_k,
// beta_j, alpha_i) at the refined coordinates (the outer angles swap because
// d(l, m, m') of Sect. 2.2 is the transpose of the textbook d^l_{m m'}).
template <typename C>
__global__ __launch_bounds__(256) void k_match_refine(int B, int n, const C *__restrict__ grid,
                                                      const long long *__restrict__ index, double *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const long long N = 2 * B, idx = index[p];
    double *o = out + 3 * (size_t)p;
    if (idx < 0 || idx >= N * N * N) {
        o[0] = o[1] = o[2] = __builtin_nan("");
        return;
    }
    const C *g = grid + (size_t)p * N * N * N;
    const int i = (int)(idx / (N * N)), j = (int)((idx / N) % N), k = (int)(idx % N);
    auto at = [&](int ii, int jj, int kk) { return (double)g[((size_t)ii * N + jj) * N + kk].x; };
    const double c0 = at(i, j, k);
    auto step = [&](double cm, double cp) {
        const double den = cm - 2.0 * c0 + cp;
        if (!(den < 0.0)) return 0.0;
        return fmin(0.5, fmax(-0.5, (cm - cp) / (2.0 * den)));
    };
    const int Ni = (int)N;
    const double di = step(at((i + Ni - 1) % Ni, j, k), at((i + 1) % Ni, j, k));
    const double dk = step(at(i, j, (k + Ni - 1) % Ni), at(i, j, (k + 1) % Ni));
    const double dj = (j > 0 && j < Ni - 1) ? step(at(i, j - 1, k), at(i, j + 1, k)) : 0.0;
    o[0] = (k + dk) * M_PI / B;
    o[1] = (2.0 * (j + dj) + 1.0) * M_PI / (4.0 * B);
    o[2] = (i + di) * M_PI / B;
}

// ---------------------------------------------------------------------------
// Off-grid polishing of a correlation maximum: Newton steps on
// F(w) = Re C(Q0 exp([w]x)), w local rotation-vector coordinates around the
// current rotation Q0, with C the SO(3) function of the correlation
// coefficients fo evaluated at a rotation by the sum of eq.
// "fourier_representation" (C at grid index (i, j, k) is the inverse
// transform's grid value; the rotation Q = Rz(a) Ry(b) Rz(c) of angles
// (a, b, c) is C's point (alpha, beta, gamma) = (c, b, a)).  Each step:
//   * F at the ten points w = 0, +-h e_i, h (e_i + e_j) (i < j);
//   * g_i = (F(h e_i) - F(-h e_i)) / 2h, H_ii = (F(h e_i) - 2F(0) + F(-h e_i)) / h^2,
//     H_ij from F(h e_i + h e_j) (exact for a quadratic);
//   * step -H^-1 g when -H has a Cholesky factor, else -g_i / H_ii per axis
//     (h toward larger F where H_ii >= 0); each component clamped to [-h, h];
//   * Q0 = Q0 exp([step]x), h = min(h, max(1e-5, 2 max|step|)), h0 = pi/(4B).
// A pass samples the ten points: blocks (chunk, pair) split a pair's groups;
// lanes 10q + p (q < 6) of a wave take stencil point p of six groups, so the
// ten lanes of a group read the same coefficients (one transaction); each
// lane runs the group's rescaled recurrence (the plan's table) at beta_p and
// at pi - beta_p (members of slots 4-7), sums sign * d * fo over the degrees
// per member, and adds Re of the member's phase e^{-i (m alpha_p + m'
// gamma_p)} times that sum to its point's partial.  A second kernel adds the
// chunks' partials in a fixed order and takes the step.
namespace polish {

struct M3 {
    double a[3][3];
};

__device__ __forceinline__ M3 mul(const M3 &x, const M3 &y) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.a[i][j] = x.a[i][0] * y.a[0][j] + x.a[i][1] * y.a[1][j] + x.a[i][2] * y.a[2][j];
    return r;
}

__device__ __forceinline__ M3 rz(double t) {
    double s, c;
    sincos(t, &s, &c);
    return M3{{{c, -s, 0.0}, {s, c, 0.0}, {0.0, 0.0, 1.0}}};
}

__device__ __forceinline__ M3 ry(double t) {
    double s, c;
    sincos(t, &s, &c);
    return M3{{{c, 0.0, s}, {0.0, 1.0, 0.0}, {-s, 0.0, c}}};
}

// exp([w]x) by Rodrigues' formula, (1 - cos t)/t^2 written as 2 sin^2(t/2)/t^2.
__device__ __forceinline__ M3 expso3(double w0, double w1, double w2) {
    const double t = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    M3 r{{{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}}};
    if (t < 1e-300) return r;
    const double s1 = sin(t) / t, sh = sin(0.5 * t), s2 = 2.0 * sh * sh / (t * t);
    const double K[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double kk = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
            r.a[i][j] += s1 * K[i][j] + s2 * kk;
        }
    return r;
}

// Angles (a, b, c), b in [0, pi], of Q = Rz(a) Ry(b) Rz(c); on the axis c = 0.
__device__ __forceinline__ void zyz(const M3 &q, double &a, double &b, double &c) {
    const double sb = hypot(q.a[0][2], q.a[1][2]);
    b = atan2(sb, q.a[2][2]);
    if (sb > 0.0) {
        a = atan2(q.a[1][2], q.a[0][2]);
        c = atan2(q.a[2][1], -q.a[2][0]);
    } else if (q.a[2][2] > 0.0) {
        a = atan2(q.a[1][0], q.a[0][0]);
        c = 0.0;
    } else {
        a = atan2(-q.a[1][0], -q.a[0][0]);
        c = 0.0;
    }
}

// Stencil point p of spacing h: w = 0, +-h e_i (p = 1..6), h (e_i + e_j) (p = 7..9).
__device__ __forceinline__ void stencil(int p, double h, double &w0, double &w1, double &w2) {
    w0 = w1 = w2 = 0.0;
    switch (p) {
        case 1: w0 = h; break;
        case 2: w0 = -h; break;
        case 3: w1 = h; break;
        case 4: w1 = -h; break;
        case 5: w2 = h; break;
        case 6: w2 = -h; break;
        case 7: w0 = h; w1 = h; break;
        case 8: w0 = h; w2 = h; break;
        case 9: w1 = h; w2 = h; break;
        default: break;
    }
}

// The Newton step of the ten samples F (in stencil order).
__device__ __forceinline__ void newton(const double *F, double h, double &s0, double &s1, double &s2) {
    const double F0 = F[0];
    const double g[3] = {(F[1] - F[2]) / (2.0 * h), (F[3] - F[4]) / (2.0 * h), (F[5] - F[6]) / (2.0 * h)};
    double H[3][3];
    H[0][0] = (F[1] - 2.0 * F0 + F[2]) / (h * h);
    H[1][1] = (F[3] - 2.0 * F0 + F[4]) / (h * h);
    H[2][2] = (F[5] - 2.0 * F0 + F[6]) / (h * h);
    H[0][1] = H[1][0] = (F[7] - F0 - h * (g[0] + g[1]) - 0.5 * h * h * (H[0][0] + H[1][1])) / (h * h);
    H[0][2] = H[2][0] = (F[8] - F0 - h * (g[0] + g[2]) - 0.5 * h * h * (H[0][0] + H[2][2])) / (h * h);
    H[1][2] = H[2][1] = (F[9] - F0 - h * (g[1] + g[2]) - 0.5 * h * h * (H[1][1] + H[2][2])) / (h * h);
    // Cholesky of A = -H
    double st[3];
    bool ok = -H[0][0] > 0.0;
    double l00 = 0.0, l10 = 0.0, l20 = 0.0, l11 = 0.0, l21 = 0.0, l22 = 0.0, r11 = 0.0, r22 = 0.0;
    if (ok) {
        l00 = sqrt(-H[0][0]);
        l10 = -H[1][0] / l00;
        l20 = -H[2][0] / l00;
        r11 = -H[1][1] - l10 * l10;
        ok = r11 > 0.0;
    }
    if (ok) {
        l11 = sqrt(r11);
        l21 = (-H[2][1] - l20 * l10) / l11;
        r22 = -H[2][2] - l20 * l20 - l21 * l21;
        ok = r22 > 0.0;
    }
    if (ok) {
        l22 = sqrt(r22);
        const double y0 = g[0] / l00;
        const double y1 = (g[1] - l10 * y0) / l11;
        const double y2 = (g[2] - l20 * y0 - l21 * y1) / l22;
        st[2] = y2 / l22;
        st[1] = (y1 - l21 * st[2]) / l11;
        st[0] = (y0 - l10 * st[1] - l20 * st[2]) / l00;
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) st[i] = H[i][i] < 0.0 ? -g[i] / H[i][i] : (g[i] >= 0.0 ? h : -h);
    }
    s0 = fmin(h, fmax(-h, st[0]));
    s1 = fmin(h, fmax(-h, st[1]));
    s2 = fmin(h, fmax(-h, st[2]));
}

constexpr int kPoints = 10;
constexpr int kGroupsPerWave = 6;  // lanes 0..59: six groups of ten points
constexpr int kWaves = 4;
constexpr int kState = 10;  // per pair: Q0 (row-major 3 x 3), h

}  // namespace polish

// Pass kernel of the polish: block (chunk, pair) sums the ten stencil values
// over the groups g = chunk, chunk + nchunk, ... of its pair (interleaved,
// so every chunk gets long and short recurrences) and writes them to
// part[(pair * nchunk + chunk) * 10 + point].
template <typename C>
__global__ __launch_bounds__(polish::kWaves * 64) void k_corr_stencil(PlanView v, const double2 *__restrict__ rec,
                                                                      const double *__restrict__ rscale,
                                                                      const C *__restrict__ coeffs,
                                                                      const double *__restrict__ state, int nchunk,
                                                                      double *__restrict__ part) {
    using namespace polish;
    constexpr int NT = kWaves * 64;
    __shared__ double red[NT];
    const int B = v.B, G = v.G;
    const int chunk = blockIdx.x, pr = blockIdx.y;
    const C *fo = coeffs + (size_t)pr * (size_t)v.Nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool active = lane < kGroupsPerWave * kPoints;
    const int p = lane % kPoints;
    const double *st = state + (size_t)pr * kState;
    M3 Q;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Q.a[r][c] = st[3 * r + c];
    const double h = st[9];
    // this lane's stencil point, as C's coordinates (alpha, beta, gamma)
    double w0, w1, w2, qa, qb, qc;
    stencil(p, h, w0, w1, w2);
    zyz(mul(Q, expso3(w0, w1, w2)), qa, qb, qc);
    const double al = qc, be = qb, ga = qa;
    double sh2, ch2;
    sincos(0.5 * be, &sh2, &ch2);
    const double lc = log(ch2), ls = log(sh2), x = cos(be);
    double acc = 0.0;
    if (active) {
        const int g0 = (wave * kGroupsPerWave + lane / kPoints) * nchunk + chunk;
        for (int g = g0; g < G; g += kWaves * kGroupsPerWave * nchunk) {
            const GroupInfo gi = v.grp[g];
            const int m = gi.m, mp = gi.mp, mask = gi.mask, L = B - m;
            const long long row = v.goff[g];
            // seeds d(m, m, m') at beta and at pi - beta (cos and sin of beta/2 swap)
            const double lb = v.lbin[g].x;
            const int pa = m + mp, pb = m - mp;
            double e = exp(lb + (pa ? pa * lc : 0.0) + (pb ? pb * ls : 0.0)), ep = 0.0;
            double er = exp(lb + (pa ? pa * ls : 0.0) + (pb ? pb * lc : 0.0)), epr = 0.0;
            // members: (mm, mm') and sign at l = m; slots 4..7 flip sign with each degree
            int mm[8], mmp[8];
            double sg[8], ire[8], iim[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                group_member(s, m, mp, m, mm[s], mmp[s], sg[s]);
                if (!((mask >> s) & 1)) sg[s] = 0.0;
                ire[s] = iim[s] = 0.0;
            }
            for (int t = 0; t < L; ++t) {
                const int l = m + t;
                const double sl = rscale[row + t];
                const double d = sl * e, dr = sl * er;
                // index of f°(l, mm, mm') = l(4l^2-1)/3 + (mm+l)(2l+1) + (mm'+l)
                const long long c0 = (long long)l * (4LL * l * l - 1) / 3 + (long long)l * (2 * l + 1) + l;
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    if (!((mask >> s) & 1)) continue;
                    const C cf = fo[c0 + (long long)mm[s] * (2 * l + 1) + mmp[s]];
                    const double dv = sg[s] * (s < 4 ? d : dr);
                    ire[s] = fma(dv, (double)cf.x, ire[s]);
                    iim[s] = fma(dv, (double)cf.y, iim[s]);
                    if (s >= 4) sg[s] = -sg[s];
                }
                const double2 ab = rec[row + t];
                const double en = fma(fma(ab.x, x, -ab.y), e, -ep);
                const double enr = fma(fma(ab.x, -x, -ab.y), er, -epr);
                ep = e;
                e = en;
                epr = er;
                er = enr;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (!((mask >> s) & 1)) continue;
                double sn, cs;
                sincos(-((double)mm[s] * al + (double)mmp[s] * ga), &sn, &cs);
                acc += cs * ire[s] - sn * iim[s];  // Re(e^{-i(m alpha + m' gamma)} I)
            }
        }
    }
    red[threadIdx.x] = active ? acc : 0.0;
    __syncthreads();
    if (threadIdx.x < kPoints) {
        double f = 0.0;
        for (int w = 0; w < kWaves; ++w)
            for (int q = 0; q < kGroupsPerWave; ++q) f += red[w * 64 + q * kPoints + threadIdx.x];
        part[((size_t)pr * nchunk + chunk) * kPoints + threadIdx.x] = f;
    }
}

// Start state of the polish: Q0 = Rz(a) Ry(b) Rz(c) of the start angles, h = pi/(4B).
__global__ void k_corr_polish_init(int B, int n, const double *__restrict__ start, double *__restrict__ state) {
    using namespace polish;
    const int pr = blockIdx.x * blockDim.x + threadIdx.x;
    if (pr >= n) return;
    const M3 Q = mul(mul(rz(start[3 * pr]), ry(start[3 * pr + 1])), rz(start[3 * pr + 2]));
    double *st = state + (size_t)pr * kState;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) st[3 * r + c] = Q.a[r][c];
    st[9] = M_PI / (4.0 * B);
}

// Newton kernel of the polish, one thread per pair: the ten values are the
// chunk partials summed in chunk order; a step updates the state, the final
// pass writes the angles (a, b, c) of Q0 and Re C there.
__global__ void k_corr_newton(int n, int nchunk, const double *__restrict__ part, double *__restrict__ state,
                              int final_pass, double *__restrict__ angles, double *__restrict__ value) {
    using namespace polish;
    const int pr = blockIdx.x * blockDim.x + threadIdx.x;
    if (pr >= n) return;
    double F[kPoints];
#pragma unroll
    for (int q = 0; q < kPoints; ++q) F[q] = 0.0;
    for (int c = 0; c < nchunk; ++c)
#pragma unroll
        for (int q = 0; q < kPoints; ++q) F[q] += part[((size_t)pr * nchunk + c) * kPoints + q];
    double *st = state + (size_t)pr * kState;
    M3 Q;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Q.a[r][c] = st[3 * r + c];
    const double h = st[9];
    if (final_pass) {
        double a, b, c;
        zyz(Q, a, b, c);
        const double two_pi = 2.0 * M_PI;
        a = fmod(a, two_pi);
        c = fmod(c, two_pi);
        angles[3 * pr] = a < 0.0 ? a + two_pi : a;
        angles[3 * pr + 1] = b;
        angles[3 * pr + 2] = c < 0.0 ? c + two_pi : c;
        value[pr] = F[0];
        return;
    }
    double s0, s1, s2;
    newton(F, h, s0, s1, s2);
    Q = mul(Q, expso3(s0, s1, s2));
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) st[3 * r + c] = Q.a[r][c];
    st[9] = fmin(h, fmax(1e-5, 2.0 * fmax(fabs(s0), fmax(fabs(s1), fabs(s2)))));
}

}  // namespace

template <typename C>
hipError_t launch_sh_forward(int B, int n, const C *f, C *a, hipStream_t s) {
    if (B < 1 || B > 512 || n < 1 || n > 65535) return hipErrorInvalidValue;
    const int threads = (2 * B + 63) / 64 * 64;
    const size_t lds = (size_t)(2 * (2 * B) + (threads / 64) * 16 * 4) * sizeof(double);
    hipLaunchKernelGGL(k_sh_forward<C>, dim3(B, n), dim3(threads), lds, s, B, f, a);
    return hipGetLastError();
}

template <typename C>
hipError_t launch_match_refine(int B, int n, const C *grid, const long long *index, double *out, hipStream_t s) {
    if (n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_match_refine<C>, dim3((n + 255) / 256), dim3(256), 0, s, B, n, grid, index, out);
    return hipGetLastError();
}

// Chunks per pair for the pass kernel: about 2048 blocks in all, at most
// one per 24 groups.
int polish_chunks(int G, int n) {
    const int want = (2048 + n - 1) / n;
    const int most = (G + polish::kWaves * polish::kGroupsPerWave - 1) / (polish::kWaves * polish::kGroupsPerWave);
    return std::max(1, std::min(want, std::max(1, most)));
}

size_t polish_workspace_bytes(int G, int n) {
    return (size_t)n * (polish::kState + (size_t)polish_chunks(G, n) * polish::kPoints) * sizeof(double);
}

template <typename C>
hipError_t launch_corr_polish(const PlanView &v, const double2 *rec, const double *rscale, int n, const C *coeffs,
                              const double *start, int iters, double *angles, double *value, double *ws,
                              hipStream_t s) {
    if (n < 1 || n > 65535 || iters < 0 || iters > 64) return hipErrorInvalidValue;
    const int nchunk = polish_chunks(v.G, n);
    double *state = ws, *part = ws + (size_t)n * polish::kState;
    const dim3 pgrid(nchunk, n), one((n + 63) / 64);
    hipLaunchKernelGGL(k_corr_polish_init, one, dim3(64), 0, s, v.B, n, start, state);
    for (int it = 0; it <= iters; ++it) {
        hipLaunchKernelGGL(k_corr_stencil<C>, pgrid, dim3(polish::kWaves * 64), 0, s, v, rec, rscale, coeffs, state,
                           nchunk, part);
        hipLaunchKernelGGL(k_corr_newton, one, dim3(64), 0, s, n, nchunk, part, state, it == iters ? 1 : 0, angles,
                           value);
    }
    return hipGetLastError();
}

template hipError_t launch_corr_polish<double2>(const PlanView &, const double2 *, const double *, int,
                                                const double2 *, const double *, int, double *, double *, double *,
                                                hipStream_t);
template hipError_t launch_corr_polish<float2>(const PlanView &, const double2 *, const double *, int, const float2 *,
                                               const double *, int, double *, double *, double *, hipStream_t);
template hipError_t launch_sh_forward<double2>(int, int, const double2 *, double2 *, hipStream_t);
template hipError_t launch_sh_forward<float2>(int, int, const float2 *, float2 *, hipStream_t);
template hipError_t launch_match_refine<double2>(int, int, const double2 *, const long long *, double *, hipStream_t);
template hipError_t launch_match_refine<float2>(int, int, const float2 *, const long long *, double *, hipStream_t);

}  // namespace soft
