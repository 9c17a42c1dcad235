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

template hipError_t launch_sh_forward<double2>(int, int, const double2 *, double2 *, hipStream_t);
template hipError_t launch_sh_forward<float2>(int, int, const float2 *, float2 *, hipStream_t);
template hipError_t launch_match_refine<double2>(int, int, const double2 *, const long long *, double *, hipStream_t);
template hipError_t launch_match_refine<float2>(int, int, const float2 *, const long long *, double *, hipStream_t);

}  // namespace soft
