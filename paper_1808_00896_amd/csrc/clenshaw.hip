// clenshaw.hip -- the DWT pair of Sect. 2.4 evaluated by Clenshaw-type
// recurrences on the vector unit, the order of evaluation the paper names
// for the DWT and as the next step of its software:
//   inverse  S'(j; c) = sum_{l=l0}^{B-1} d(l; b_j) f_c(l)     (T_B^T)
//            by Clenshaw's backward summation over degrees;
//   forward  G_c(l) = sum_j d(l; b_j) X_c(j)                   (T_B W_B)
//            by the transposed (adjoint) evaluation: every lane runs the
//            forward three-term recurrence for its beta sample, and the sum
//            over beta of each degree is a reduction across the lanes.
//
// Inverse.  For a symmetry group with representative (m, m') and lowest
// degree l0 = m, every member column c (8 members x (re, im)) of the inverse
// is
//   S'(j; c) = sum_{l=l0}^{B-1} d(l; b_j) f_c(l) = sum_l e(l; b_j) c_l[c],
// with d(l) = s_l e(l) and c_l[c] = s_l x (member's sign at l) x f°(l, member)
// (x (2l+1)/(8 pi B) for the adjoint).  The rescaled recurrence of eq.
// "Wigner_d_recurrence", e(l+1) = A_l e(l) - e(l-1) with A_l = alpha_l x -
// gamma_l and e(l0-1) = 0, has the backward companion
//   b_l = c_l + A_l b_{l+1} - b_{l+2},   b_B = b_{B+1} = 0,
// and the sum is e(l0) b_{l0}: one FMA and one add per column and degree,
// no d values at all.
//
// One block per (function, group) work item, NB beta samples per lane, 16
// independent column chains per sample.  The group's c_l (L x 16 values, the
// same for every lane) are gathered once into LDS and read as broadcasts;
// the (alpha_l, gamma_l) pairs come through scalar loads.  The arithmetic is
// FP64 in every precision; only the loads and stores take the plan's type.
//
// Cost on gfx950: two FP64 vector operations per column and degree, where
// the matrix-core inverse spends one FMA slot of an FP64 MFMA (the two units
// share one FP64 rate) plus two recurrence FMAs per degree for all 16
// columns; measured 1.7x (2B = 256) to 2.2x (2B = 1024) the matrix-core time.
// NB = 2 (212 VGPRs, two waves per SIMD) is slower than NB = 1.
//
// Forward.  The transpose of that evaluation: with the beta samples of the
// group's columns X_c(j) (weights w_B(j) applied by the FFT pass, members at
// pi - beta stored j-reversed), G_c(l) = sum_j e(l; b_j) X_c(j) and
// f°(l, member) = (member's sign) s_l (2l+1)/(8 pi B) G_c(l).  Solving the
// transposed Clenshaw system is the forward recurrence e(l0), e(l0+1), ...
// itself, so each lane owns one beta sample and its 16 column values, and
// per degree forms the 16 products e(l; b_j) X_c(j); a wave sums them over
// its 64 samples by a butterfly that halves the columns a lane carries at
// each of its first four exchanges (lane ^ 32, 16, 8, 4), so after six
// exchanges (then ^ 2, ^ 1) lane 4c + q holds column c's wave sum; the
// waves' sums of 16 degrees meet in LDS and are added in order.
#include "soft_internal.h"

namespace soft {
namespace {

__device__ __forceinline__ long long coeff_flat(int l, int m, int mp) {
    return (long long)l * (4 * l * l - 1) / 3 + (m + l) * (2 * l + 1) + (mp + l);
}

template <int PR, int NB>
__global__ __launch_bounds__(1024 / NB) void k_idwt_clenshaw(DwtTables tab, const double2 *__restrict__ rec,
                                                       const WorkItem *__restrict__ items, int nitems,
                                                       const typename PrecT<PR>::C *__restrict__ coeffs,
                                                       typename PrecT<PR>::C *__restrict__ S, int flags) {
    using C = typename PrecT<PR>::C;
    using R = typename PrecT<PR>::R;
    const bool apply_v = flags & kFlagScale, stream = flags & kFlagStream;
    extern __shared__ double cl[];  // [L][16]
    const WorkItem it = items[item_of_block(blockIdx.x, nitems)];
    const int B = it.B, N = 2 * B;
    const int m = it.m, mp = it.mp, mask = it.mask;
    const int L = B - m;
    const int NT = blockDim.x;
    const R *__restrict__ cin = reinterpret_cast<const R *>(coeffs + it.coeff_off);
    const double v0 = apply_v ? 1.0 / (8.0 * M_PI * (double)B) : 0.0;

    // The inverse reorder: c_l of every member column, absent members zero.
    for (int e = threadIdx.x; e < L * 16; e += NT) {
        const int li = e >> 4, col = e & 15, slot = col >> 1;
        double val = 0.0;
        if ((mask >> slot) & 1) {
            const int l = m + li;
            int mm, mmp;
            double sign;
            group_member(slot, m, mp, l, mm, mmp, sign);
            const double f = sign * tab.rscale[it.goff + li] * (apply_v ? (2.0 * l + 1.0) * v0 : 1.0);
            val = (double)cin[2 * coeff_flat(l, mm, mmp) + (col & 1)] * f;
        }
        cl[e] = val;
    }
    double x[NB], seed[NB];
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const int j = threadIdx.x + h * NT;
        const bool jin = j < N;
        x[h] = tab.cosb[it.jbase + (jin ? j : 0)];
        seed[h] = tab.seed[it.seed_off + (jin ? j : 0)];  // 2B <= 1024: never an extended-range seed
    }
    __syncthreads();

    const double2 *__restrict__ Rr = rec + it.goff;
    double b1[NB][16], b2[NB][16];  // b_{l+1}, b_{l+2}
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int c = 0; c < 16; ++c) b1[h][c] = b2[h][c] = 0.0;
    for (int li = L - 1; li >= 0; --li) {
        const double2 ag = Rr[li];
        const double *cr = cl + li * 16;
        double cv[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) cv[c] = cr[c];
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            const double A = fma(ag.x, x[h], -ag.y);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const double t = fma(A, b1[h][c], cv[c] - b2[h][c]);
                b2[h][c] = b1[h][c];
                b1[h][c] = t;
            }
        }
    }
    C *Sg = S + it.s_off;
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const int j = threadIdx.x + h * NT;
        if (j >= N) continue;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            if (!((mask >> s) & 1)) continue;
            C o;
            o.x = (R)(seed[h] * b1[h][2 * s]);
            o.y = (R)(seed[h] * b1[h][2 * s + 1]);
            put_c(&Sg[(size_t)s * N + j], o, stream);
        }
    }
}

// Butterfly step of the forward reduction: a lane carrying n column values
// keeps the half selected by its lane bit `bit` and adds the partner's copy
// of that half (the partner keeps the other half).
template <int n>
__device__ __forceinline__ void reduce_half(double (&v)[16], int bit, bool hi) {
#pragma unroll
    for (int k = 0; k < n / 2; ++k) {
        const double keep = hi ? v[k + n / 2] : v[k];
        const double send = hi ? v[k] : v[k + n / 2];
        v[k] = keep + __shfl_xor(send, bit, 64);
    }
}

template <int PR>
__global__ __launch_bounds__(1024) void k_dwt_fwd_clenshaw(DwtTables tab, const double2 *__restrict__ rec,
                                                         const WorkItem *__restrict__ items, int nitems,
                                                         const typename PrecT<PR>::C *__restrict__ S,
                                                         typename PrecT<PR>::C *__restrict__ coeffs, int apply_v) {
    using C = typename PrecT<PR>::C;
    using R = typename PrecT<PR>::R;
    extern __shared__ double part[];  // [wave][16 degrees][16 columns]
    const WorkItem it = items[item_of_block(blockIdx.x, nitems)];
    const int B = it.B, N = 2 * B;
    const int m = it.m, mp = it.mp, mask = it.mask;
    const int L = B - m;
    const int NT = blockDim.x, NWV = NT >> 6;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = threadIdx.x;
    const bool jin = j < N;

    // this lane's beta sample of every member column (zero when absent)
    double X[16];
    const C *Sg = S + it.s_off;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        C v;
        v.x = v.y = (R)0;
        if (jin && ((mask >> s) & 1)) v = Sg[(size_t)s * N + j];
        X[2 * s] = (double)v.x;
        X[2 * s + 1] = (double)v.y;
    }
    const double x = tab.cosb[it.jbase + (jin ? j : 0)];
    double e = jin ? tab.seed[it.seed_off + (jin ? j : 0)] : 0.0, ep = 0.0;
    const double2 *__restrict__ Rr = rec + it.goff;
    const double *__restrict__ rs = tab.rscale + it.goff;
    R *out = reinterpret_cast<R *>(coeffs + it.coeff_off);
    const double v0 = apply_v ? 1.0 / (8.0 * M_PI * (double)B) : 0.0;

    for (int l0 = 0; l0 < L; l0 += 16) {
        for (int r = 0; r < 16 && l0 + r < L; ++r) {
            double v[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) v[c] = e * X[c];
            reduce_half<16>(v, 32, lane & 32);
            reduce_half<8>(v, 16, lane & 16);
            reduce_half<4>(v, 8, lane & 8);
            reduce_half<2>(v, 4, lane & 4);
            double q = v[0] + __shfl_xor(v[0], 2, 64);
            q += __shfl_xor(q, 1, 64);
            if ((lane & 3) == 0) part[(wave * 16 + r) * 16 + (lane >> 2)] = q;
            const double2 ag = Rr[l0 + r];
            const double A = fma(ag.x, x, -ag.y);
            const double en = fma(A, e, -ep);
            ep = e;
            e = en;
        }
        __syncthreads();
        // the waves' sums in order, with the member's sign, s_l and V_B
        for (int t = threadIdx.x; t < 256; t += NT) {
            const int li = l0 + (t >> 4), c = t & 15, slot = c >> 1;
            if (li < L && ((mask >> slot) & 1)) {
                double g = 0.0;
                for (int w = 0; w < NWV; ++w) g += part[(w * 16 + (t >> 4)) * 16 + c];
                const int l = m + li;
                int mm, mmp;
                double sign;
                group_member(slot, m, mp, l, mm, mmp, sign);
                const double f = sign * rs[li] * (apply_v ? (2.0 * l + 1.0) * v0 : 1.0);
                out[2 * coeff_flat(l, mm, mmp) + (c & 1)] = (R)(g * f);
            }
        }
        __syncthreads();
    }
}

}  // namespace

template <int PR>
hipError_t launch_idwt_clenshaw(const DwtTables &tab, const WorkItem *items, int nitems, int nmax,
                                const typename PrecT<PR>::C *coeffs, typename PrecT<PR>::C *S, bool apply_v,
                                bool stream, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (nmax < 2 || nmax > 1024) return hipErrorInvalidValue;
    constexpr int NB = 1;
    const int threads = (nmax + 64 * NB - 1) / (64 * NB) * 64;  // NB beta samples per lane
    const size_t lds = (size_t)(nmax / 2) * 16 * sizeof(double);  // L <= B = nmax / 2 degrees
    hipLaunchKernelGGL((k_idwt_clenshaw<PR, NB>), dim3(nitems), dim3(threads), lds, s, tab, tab.rec, items, nitems,
                       coeffs, S, (apply_v ? kFlagScale : 0) | (stream ? kFlagStream : 0));
    return hipGetLastError();
}

template <int PR>
hipError_t launch_dwt_fwd_clenshaw(const DwtTables &tab, const WorkItem *items, int nitems, int nmax,
                                   const typename PrecT<PR>::C *S, typename PrecT<PR>::C *coeffs, bool apply_v,
                                   hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (nmax < 2 || nmax > 1024) return hipErrorInvalidValue;
    const int threads = (nmax + 63) / 64 * 64;  // one beta sample per lane
    const size_t lds = (size_t)(threads / 64) * 256 * sizeof(double);
    hipLaunchKernelGGL((k_dwt_fwd_clenshaw<PR>), dim3(nitems), dim3(threads), lds, s, tab, tab.rec, items, nitems, S,
                       coeffs, apply_v ? 1 : 0);
    return hipGetLastError();
}

#define SOFT_CLENSHAW_INSTANTIATE(PR)                                                                          \
    template hipError_t launch_idwt_clenshaw<PR>(const DwtTables &, const WorkItem *, int, int,              \
                                                 const typename PrecT<PR>::C *, typename PrecT<PR>::C *, bool, \
                                                 bool, hipStream_t);                                    \
    template hipError_t launch_dwt_fwd_clenshaw<PR>(const DwtTables &, const WorkItem *, int, int,           \
                                                    const typename PrecT<PR>::C *, typename PrecT<PR>::C *,    \
                                                    bool, hipStream_t);
SOFT_CLENSHAW_INSTANTIATE(P64)
SOFT_CLENSHAW_INSTANTIATE(P32)
SOFT_CLENSHAW_INSTANTIATE(P32S)

}  // namespace soft
