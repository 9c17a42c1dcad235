// fft.hip -- separation of variables of Sect. 2.4 on gfx950.
//
// Forward:  S(m, m'; j) = sum_{i,k} f(a_i, b_j, g_k) e^{+i(m a_i + m' g_k)}
// Inverse:  f(a_i, b_j, g_k) = sum_{m,m'} S'(j; m, m') e^{-i(m a_i + m' g_k)}
// with a_i = g_i = 2 pi i / N, N = 2B, |m|, |m'| <= B-1 (the +-B frequency is
// dropped on the way in and written as zero on the way out).
//
// Each direction is two HBM passes of batched 1-D FFTs over N points:
//   gamma pass:  rows along k (contiguous) <-> t1[q][j][i]   (q = m' mod N)
//   alpha pass:  rows along i (contiguous in t1) <-> S[group slot][j]
// A block holds T independent length-N sequences in LDS and transforms them
// with a Stockham autosort FFT (one radix-2 stage when log2 N is odd, then
// radix-4 stages).  The T sequences are neighbours along the axis that is
// contiguous in the *other* layout, so every global load and store moves
// runs of >= T * 16 bytes: the transposes cost no extra HBM pass.  The forward
// alpha pass also multiplies by the quadrature weight w_B(j) (the W_B factor
// of the DWT) and writes members at pi - beta in reversed j order, so the DWT
// sees every member of a symmetry group against the same d(l; b_j).
#include "soft_internal.h"

namespace soft {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// (SIGN i) * a
template <int SIGN>
__device__ __forceinline__ double2 cmul_si(double2 a) {
    return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Sequences per block for a length-N transform: enough work for the block's
// threads, at least 8 neighbours (128-byte runs) and never more than N.
constexpr int tile_for(int N, bool /*transposed_in*/) {
    return N < 8 ? N : (1024 / N > 8 ? (1024 / N < N ? 1024 / N : N) : 8);
}

// 512 threads for the 1024-point transform (its LDS tile allows one block per
// CU), 256 otherwise.
constexpr int threads_for(int N) { return N >= 1024 ? 512 : 256; }

// In-place Stockham FFT of T sequences of length N held in LDS (row stride
// N + 1 complex), X[q] = sum_p x[p] e^{SIGN 2 pi i p q / N}; tw[k] is
// e^{SIGN 2 pi i k / N}.  Starts and ends with all threads synchronised.
template <int N, int T, int NT, int SIGN>
__device__ __forceinline__ void fft_lds(double2 *buf, const double2 *__restrict__ tw) {
    constexpr int LOGN = ilog2(N);
    constexpr int S = N + 1;
    const int tid = threadIdx.x;
    int logNs = 0;
    if constexpr (LOGN & 1) {  // radix-2 stage with Ns = 1 (no twiddles)
        constexpr int NB = T * N / 2;
        constexpr int PER = (NB + NT - 1) / NT;
        double2 v[PER][2];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = tid + q * NT;
            if (NB % NT == 0 || b < NB) {
                const int t = b / (N / 2), jj = b % (N / 2);
                v[q][0] = buf[t * S + jj];
                v[q][1] = buf[t * S + jj + N / 2];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = tid + q * NT;
            if (NB % NT == 0 || b < NB) {
                const int t = b / (N / 2), jj = b % (N / 2);
                buf[t * S + 2 * jj] = cadd(v[q][0], v[q][1]);
                buf[t * S + 2 * jj + 1] = csub(v[q][0], v[q][1]);
            }
        }
        __syncthreads();
        logNs = 1;
    }
#pragma unroll
    for (int st = 0; st < LOGN / 2; ++st) {  // radix-4 stages
        constexpr int NB = T * N / 4;
        constexpr int PER = (NB + NT - 1) / NT;
        const int Ns = 1 << logNs;
        const int twstep = N >> (2 + logNs);  // N / (4 Ns)
        double2 v[PER][4];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = tid + q * NT;
            if (NB % NT == 0 || b < NB) {
                const int t = b / (N / 4), jj = b % (N / 4);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[q][r] = buf[t * S + jj + r * (N / 4)];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = tid + q * NT;
            if (NB % NT == 0 || b < NB) {
                const int t = b / (N / 4), jj = b % (N / 4);
                const int k = jj & (Ns - 1);
                if (logNs > 0) {
#pragma unroll
                    for (int r = 1; r < 4; ++r) v[q][r] = cmul(v[q][r], tw[k * r * twstep]);
                }
                const double2 a0 = cadd(v[q][0], v[q][2]);
                const double2 a1 = csub(v[q][0], v[q][2]);
                const double2 a2 = cadd(v[q][1], v[q][3]);
                const double2 a3 = cmul_si<SIGN>(csub(v[q][1], v[q][3]));
                const int base = (jj - k) * 4 + k;
                buf[t * S + base] = cadd(a0, a2);
                buf[t * S + base + Ns] = cadd(a1, a3);
                buf[t * S + base + 2 * Ns] = csub(a0, a2);
                buf[t * S + base + 3 * Ns] = csub(a1, a3);
            }
        }
        __syncthreads();
        logNs += 2;
    }
}

// gamma pass, forward: grid[i][j][k] -> t1[q][j][i], FFT along k, e^{+i}.
// Block (i-tile, j, batch); q = N/2 (the +-B bin) is not stored.
template <int N>
__global__ __launch_bounds__(threads_for(N)) void k_fft_gamma_fwd(PlanView p, const double2 *__restrict__ grid,
                                                           double2 *__restrict__ t1) {
    constexpr int T = tile_for(N, false);
    constexpr int NT = threads_for(N);
    constexpr int S = N + 1;
    __shared__ double2 buf[T * S];
    const int it = blockIdx.x, j = blockIdx.y;
    const size_t N3 = (size_t)N * N * N;
    const double2 *g = grid + blockIdx.z * N3;
    double2 *o = t1 + blockIdx.z * N3;
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e / N, n = e % N;
        buf[t * S + n] = g[((size_t)(it * T + t) * N + j) * N + n];
    }
    __syncthreads();
    fft_lds<N, T, NT, +1>(buf, p.twp);
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e % T, q = e / T;
        if (q != N / 2) o[((size_t)q * N + j) * N + it * T + t] = buf[t * S + q];
    }
}

// alpha pass, forward: t1[q][j][i] -> S[slot][j'], FFT along i, e^{+i},
// times w_B(j) when apply_w; j' = N-1-j for members at pi - beta.
// Block (j-tile, q != N/2, batch).
template <int N>
__global__ __launch_bounds__(threads_for(N)) void k_fft_alpha_fwd(PlanView p, const double2 *__restrict__ t1,
                                                           double2 *__restrict__ Sout, int apply_w) {
    constexpr int T = tile_for(N, false);
    constexpr int NT = threads_for(N);
    constexpr int S = N + 1;
    constexpr int B = N / 2;
    __shared__ double2 buf[T * S];
    const int jt = blockIdx.x;
    const int q = blockIdx.y < B ? blockIdx.y : blockIdx.y + 1;
    const size_t N3 = (size_t)N * N * N;
    const double2 *in = t1 + blockIdx.z * N3 + ((size_t)q * N + jt * T) * N;
    double2 *o = Sout + blockIdx.z * ((size_t)p.G * kSlots * N);
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e / N, n = e % N;
        buf[t * S + n] = in[e];
    }
    __syncthreads();
    fft_lds<N, T, NT, +1>(buf, p.twp);
    const int mp = q < B ? q : q - N;
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e % T, pi = e / T;
        if (pi == B) continue;
        const int m = pi < B ? pi : pi - N;
        const int sl = slot_code(m, mp);
        const int j = jt * T + t;
        const int jj = (sl & 1) ? N - 1 - j : j;
        double2 v = buf[t * S + pi];
        if (apply_w) {
            const double wj = p.w[j];
            v.x *= wj;
            v.y *= wj;
        }
        o[(size_t)(sl >> 1) * N + jj] = v;
    }
}

// alpha pass, inverse: S'[slot][j'] -> t1[q][j][i], FFT along m, e^{-i}.
template <int N>
__global__ __launch_bounds__(threads_for(N)) void k_fft_alpha_inv(PlanView p, const double2 *__restrict__ Sin,
                                                           double2 *__restrict__ t1) {
    constexpr int T = tile_for(N, true);
    constexpr int NT = threads_for(N);
    constexpr int S = N + 1;
    constexpr int B = N / 2;
    __shared__ double2 buf[T * S];
    const int jt = blockIdx.x;
    const int q = blockIdx.y < B ? blockIdx.y : blockIdx.y + 1;
    const size_t N3 = (size_t)N * N * N;
    const double2 *in = Sin + blockIdx.z * ((size_t)p.G * kSlots * N);
    double2 *o = t1 + blockIdx.z * N3 + ((size_t)q * N + jt * T) * N;
    const int mp = q < B ? q : q - N;
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e % T, pi = e / T;
        double2 v = make_double2(0.0, 0.0);
        if (pi != B) {
            const int m = pi < B ? pi : pi - N;
            const int sl = slot_code(m, mp);
            const int j = jt * T + t;
            const int jj = (sl & 1) ? N - 1 - j : j;
            v = in[(size_t)(sl >> 1) * N + jj];
        }
        buf[t * S + pi] = v;
    }
    __syncthreads();
    fft_lds<N, T, NT, -1>(buf, p.twm);
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e / N, n = e % N;
        o[e] = buf[t * S + n];
    }
}

// gamma pass, inverse: t1[q][j][i] -> grid[i][j][k], FFT along m', e^{-i},
// times w_B(j) when apply_w.  Block (i-tile, j, batch).
template <int N>
__global__ __launch_bounds__(threads_for(N)) void k_fft_gamma_inv(PlanView p, const double2 *__restrict__ t1,
                                                           double2 *__restrict__ grid, int apply_w) {
    constexpr int T = tile_for(N, true);
    constexpr int NT = threads_for(N);
    constexpr int S = N + 1;
    __shared__ double2 buf[T * S];
    const int it = blockIdx.x, j = blockIdx.y;
    const size_t N3 = (size_t)N * N * N;
    const double2 *in = t1 + blockIdx.z * N3;
    double2 *g = grid + blockIdx.z * N3;
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e % T, q = e / T;
        buf[t * S + q] = q == N / 2 ? make_double2(0.0, 0.0) : in[((size_t)q * N + j) * N + it * T + t];
    }
    __syncthreads();
    fft_lds<N, T, NT, -1>(buf, p.twm);
    const double wj = apply_w ? p.w[j] : 1.0;
#pragma unroll 4
    for (int e = threadIdx.x; e < T * N; e += NT) {
        const int t = e / N, n = e % N;
        double2 v = buf[t * S + n];
        v.x *= wj;
        v.y *= wj;
        g[((size_t)(it * T + t) * N + j) * N + n] = v;
    }
}

#define SOFT_FFT_DISPATCH(N_, CALL)           \
    switch (N_) {                             \
        case 2: { constexpr int NN = 2; CALL; } break;       \
        case 4: { constexpr int NN = 4; CALL; } break;       \
        case 8: { constexpr int NN = 8; CALL; } break;       \
        case 16: { constexpr int NN = 16; CALL; } break;     \
        case 32: { constexpr int NN = 32; CALL; } break;     \
        case 64: { constexpr int NN = 64; CALL; } break;     \
        case 128: { constexpr int NN = 128; CALL; } break;   \
        case 256: { constexpr int NN = 256; CALL; } break;   \
        case 512: { constexpr int NN = 512; CALL; } break;   \
        case 1024: { constexpr int NN = 1024; CALL; } break; \
        default: return hipErrorInvalidValue;               \
    }

}  // namespace

hipError_t launch_fft_gamma_fwd(const PlanView &p, int batch, const double2 *grid, double2 *t1, hipStream_t s) {
    SOFT_FFT_DISPATCH(p.N, {
        dim3 g(NN / tile_for(NN, false), NN, batch);
        hipLaunchKernelGGL(k_fft_gamma_fwd<NN>, g, dim3(threads_for(NN)), 0, s, p, grid, t1);
    });
    return hipGetLastError();
}

hipError_t launch_fft_alpha_fwd(const PlanView &p, int batch, const double2 *t1, double2 *S, bool apply_w,
                                hipStream_t s) {
    SOFT_FFT_DISPATCH(p.N, {
        dim3 g(NN / tile_for(NN, false), NN - 1, batch);
        hipLaunchKernelGGL(k_fft_alpha_fwd<NN>, g, dim3(threads_for(NN)), 0, s, p, t1, S, (int)apply_w);
    });
    return hipGetLastError();
}

hipError_t launch_fft_alpha_inv(const PlanView &p, int batch, const double2 *S, double2 *t1, hipStream_t s) {
    SOFT_FFT_DISPATCH(p.N, {
        dim3 g(NN / tile_for(NN, true), NN - 1, batch);
        hipLaunchKernelGGL(k_fft_alpha_inv<NN>, g, dim3(threads_for(NN)), 0, s, p, S, t1);
    });
    return hipGetLastError();
}

hipError_t launch_fft_gamma_inv(const PlanView &p, int batch, const double2 *t1, double2 *grid, bool apply_w,
                                hipStream_t s) {
    SOFT_FFT_DISPATCH(p.N, {
        dim3 g(NN / tile_for(NN, true), NN, batch);
        hipLaunchKernelGGL(k_fft_gamma_inv<NN>, g, dim3(threads_for(NN)), 0, s, p, t1, grid, (int)apply_w);
    });
    return hipGetLastError();
}

}  // namespace soft
