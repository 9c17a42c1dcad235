// fft.hip -- separation of variables of Sect. 2.4 on gfx950.
//
// Forward:  S(m, m'; j) = sum_{i,k} f(a_i, b_j, g_k) e^{+i(m a_i + m' g_k)}
// Inverse:  f(a_i, b_j, g_k) = sum_{m,m'} S'(j; m, m') e^{-i(m a_i + m' g_k)}
// with a_i = g_i = 2 pi i / N, N = 2B, |m|, |m'| <= B-1 (the +-B frequency is
// dropped on the way in and written as zero on the way out).
//
// Each direction is two HBM passes of batched 1-D FFTs over N points:
//   gamma pass:  rows along k (contiguous) <-> u(j, q, i)   (q = m' mod N)
//   alpha pass:  rows along i (runs of T in u) <-> S[group slot][j]
// where u, the intermediate, is the plan's own tile-blocked t1 or, for plans
// that may use the grid buffer as scratch, a blocked layout inside the grid
// (see u_index).
// A block transforms T independent length-N sequences that are neighbours
// along the axis contiguous in the *other* layout, so every global access
// moves runs of T elements (128 bytes or more from N = 512 up) and the
// transposes cost no extra HBM pass.  The
// forward alpha pass multiplies by the quadrature weight w_B(j) (the W_B
// factor of the DWT) and writes members at pi - beta in reversed j order, so
// the DWT sees every member of a symmetry group against the same d(l; b_j).
//
// The FFT is a Stockham autosort decomposition N = R0 x 16 x 16 ... (R0 in
// {1, 2, 4, 8}); every thread keeps 16 points in registers and runs its
// radix-R butterflies there.  Stage 0 reads HBM directly and the last stage
// writes HBM directly, with the lane order (row index fastest, or tile index
// fastest) chosen per side so that both stay coalesced; only the exchanges
// between stages go through LDS (one for N <= 512, two for N = 1024).
#include "soft_internal.h"

namespace soft {
namespace {

// Complex helpers for double2 (FP64 plans) and float2 (FP32 plans).
template <typename C>
__device__ __forceinline__ C mk(double x, double y);
template <>
__device__ __forceinline__ double2 mk<double2>(double x, double y) { return make_double2(x, y); }
template <>
__device__ __forceinline__ float2 mk<float2>(double x, double y) { return make_float2((float)x, (float)y); }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
    C r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
    C r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename C>
__device__ __forceinline__ C cscale(C a, double w) {
    C r;
    r.x = a.x * (decltype(a.x))w;
    r.y = a.y * (decltype(a.y))w;
    return r;
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// cos and sin of 2 pi j / 16, j = 0..15, correctly rounded.
__device__ constexpr double kCos16[16] = {
    1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898,
    0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867,
    -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898,
    0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867};
__device__ constexpr double kSin16[16] = {
    0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867,
    1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898,
    0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867,
    -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};

// a * e^{SIGN 2 pi i j / R} for a compile-time j and R | 16.
template <int R, int J, int SIGN, typename C>
__device__ __forceinline__ C twc(C a) {
    using T = decltype(a.x);
    constexpr int jj = (J % R) * (16 / R);
    C r;
    if constexpr (jj == 0) {
        return a;
    } else if constexpr (jj == 4) {
        if (SIGN > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
        return r;
    } else if constexpr (jj == 8) {
        r.x = -a.x;
        r.y = -a.y;
        return r;
    } else if constexpr (jj == 12) {
        if (SIGN > 0) { r.x = a.y; r.y = -a.x; } else { r.x = -a.y; r.y = a.x; }
        return r;
    } else {
        const T c = (T)kCos16[jj], s = (T)(SIGN * kSin16[jj]);
        r.x = a.x * c - a.y * s;
        r.y = a.x * s + a.y * c;
        return r;
    }
}

// Load of one complex input.  The stage-0 loads of a pass read every element
// once; for 128 <= 2B <= 512 they are non-temporal, which measured faster for
// the pass and the kernels after it (B = 128 step 0.652 -> 0.630 ms, FP32-split
// 0.433 -> 0.403 ms; B = 256 5.58 -> 5.51 ms); at 2B = 1024 they slowed the
// passes down (B = 512: 62.0 -> 63.8 ms per step) and below 128 they gave
// nothing.
template <int N>
__device__ __forceinline__ double2 ld_in(const double2 *p) {
    if constexpr (N >= 128 && N <= 512) {
        typedef double r2 __attribute__((ext_vector_type(2)));
        const r2 v = __builtin_nontemporal_load(reinterpret_cast<const r2 *>(p));
        return make_double2(v[0], v[1]);
    } else {
        return *p;
    }
}
template <int N>
__device__ __forceinline__ float2 ld_in(const float2 *p) {
    if constexpr (N >= 128 && N <= 512) {
        typedef float r2 __attribute__((ext_vector_type(2)));
        const r2 v = __builtin_nontemporal_load(reinterpret_cast<const r2 *>(p));
        return make_float2(v[0], v[1]);
    } else {
        return *p;
    }
}

// In-register DFT of R points: X[k] = sum_n x[n] e^{SIGN 2 pi i n k / R}.
template <int R, int SIGN, typename C>
__device__ __forceinline__ void dft(C *v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const C a2 = cadd(v[1], v[3]), a3 = twc<4, 1, SIGN>(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[1] = cadd(a1, a3);
        v[2] = csub(a0, a2);
        v[3] = csub(a1, a3);
    } else {
        // R = 4 * Bq: n = Bq n1 + n2, k = k1 + 4 k2; inner DFT-4 over n1,
        // twiddle e^{SIGN 2 pi i n2 k1 / R}, outer DFT-Bq over n2.
        constexpr int A = 4, Bq = R / 4;
        C y[Bq][A];
#pragma unroll
        for (int n2 = 0; n2 < Bq; ++n2) {
            C a[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) a[n1] = v[Bq * n1 + n2];
            dft<A, SIGN, C>(a);
            y[n2][0] = a[0];
            if (n2 == 0) {
                y[0][1] = a[1];
                y[0][2] = a[2];
                y[0][3] = a[3];
            } else if (n2 == 1) {
                y[n2][1] = twc<R, 1, SIGN>(a[1]);
                y[n2][2] = twc<R, 2, SIGN>(a[2]);
                y[n2][3] = twc<R, 3, SIGN>(a[3]);
            } else if (n2 == 2) {
                y[n2][1] = twc<R, 2, SIGN>(a[1]);
                y[n2][2] = twc<R, 4, SIGN>(a[2]);
                y[n2][3] = twc<R, 6, SIGN>(a[3]);
            } else {
                y[n2][1] = twc<R, 3, SIGN>(a[1]);
                y[n2][2] = twc<R, 6, SIGN>(a[2]);
                y[n2][3] = twc<R, 9, SIGN>(a[3]);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            C b[Bq];
#pragma unroll
            for (int n2 = 0; n2 < Bq; ++n2) b[n2] = y[n2][k1];
            dft<Bq, SIGN, C>(b);
#pragma unroll
            for (int k2 = 0; k2 < Bq; ++k2) v[k1 + A * k2] = b[k2];
        }
    }
}

// Shape of the transform of length N: E points per thread, P threads per
// sequence, radix R0 of the first stage, NSTAGE stages.
template <int N>
struct Shape {
    static constexpr int E = N >= 16 ? 16 : N;
    static constexpr int P = N / E;
    static constexpr int LOG = ilog2(N);
    static constexpr int R0 = N >= 16 ? (1 << (LOG % 4)) : N;  // 1, 2, 4, 8 (or N when N < 16)
    static constexpr int NSTAGE = N >= 16 ? LOG / 4 + (LOG % 4 ? 1 : 0) : 1;
    static constexpr int RS = N + N / 16 + 1;  // LDS row stride (complex), padded
};

// The four passes: gamma (over k) and alpha (over i), forward and inverse.
enum Kind { GAMMA_FWD = 0, ALPHA_FWD = 1, ALPHA_INV = 2, GAMMA_INV = 3 };

// T neighbouring sequences per block: the transposed side of a pass moves
// runs of T elements, so T is chosen for runs of at least 128 bytes (T = 8
// complex128 or 16 complex64 from 2B = 512 up) within about 140 KB of LDS
// (one block of 512-1024 threads per CU at 2B = 1024); 32 for N <= 64, 16 up
// to 256; never more than N.  The inverse passes at 2B = 1024 through the
// plan's intermediate take half that (64-byte runs in FP64, two blocks per
// CU), which measured faster for both of them (FP64: 7.8 -> 7.5 and 8.0 ->
// 7.7 ms); the forward passes were slower with it, and so were the inverse
// passes staging in the grid (INGRID).  The intermediate of a direction is
// laid out by its gamma pass's T (TL); the complex64 forward alpha pass at
// 2B = 1024 reads it with half-height blocks (two blocks of 8 rows per
// 16-row layout tile, each still one contiguous run of 8N elements): 5.2 ->
// 4.8 ms at B = 512, where the gamma pass is faster with the full tile.
template <int N, typename C, int KIND, bool INGRID>
struct Tile {
    // At 2B = 2048 a tile of T sequences takes T * 34 KB (complex128) or
    // T * 17 KB (complex64) of LDS: T = 4 or 8 keeps it within a CU's 160 KB.
    static constexpr int TF = N <= 64 ? 32 : (N <= 256 ? 16 : (N <= 1024 ? (sizeof(C) == 16 ? 8 : 16)
                                                                          : (sizeof(C) == 16 ? 4 : 8)));
    static constexpr bool INV = KIND == ALPHA_INV || KIND == GAMMA_INV;
    static constexpr bool HALF = N == 1024 && !INGRID;
    static constexpr int TL0 = HALF && INV ? TF / 2 : TF;
    static constexpr int T0 = HALF && (INV || (KIND == ALPHA_FWD && sizeof(C) == 8)) ? TF / 2 : TF;
    static constexpr int T = T0 < N ? T0 : N;
    static constexpr int TL = TL0 < N ? TL0 : N;
    static constexpr int NT = T * Shape<N>::P;
    // Row halves: a tile whose exchange buffer would exceed 96 KB exchanges
    // through LDS one half of its rows at a time (RH = 2), so that two
    // blocks can share a CU without shortening the runs on the transposed
    // side.  That needs a kernel within 128 VGPRs at 512 threads: measured
    // (B = 512 / 1024 FP64, results bit-identical) it pays for the forward
    // gamma pass (7.8 -> 7.5 ms; in place 7.7 -> 6.9 ms; B = 1024 52.9 ->
    // 49.0 ms) and the in-grid inverse alpha pass at 2B = 1024 (8.5 -> 8.1 ms),
    // while the passes above 128 VGPRs only gain barriers (forward alpha 7.6
    // -> 8.7 ms; forcing 128 VGPRs made them spill and slower still).
    // At 2B = 256 the complex128 tile's whole buffer (70 KB) leaves two
    // blocks per CU; in halves (35 KB) three share a CU (the kernels use
    // 122-152 VGPRs).  Measured at B = 128 that pays for the passes through
    // the plan's intermediate except the forward gamma pass (alpha forward
    // 96 -> 92 us, the inverse passes 101 -> 99 us, the step 0.604 -> 0.599
    // ms; the forward gamma pass 88 -> 91 us, so it keeps the whole tile).
    static constexpr bool BIG = (size_t)T * Shape<N>::RS * sizeof(C) > 96 * 1024;
    static constexpr bool RH_PAYS = KIND == GAMMA_FWD || (KIND == ALPHA_INV && INGRID && N == 1024);
    static constexpr bool THREE = N == 256 && sizeof(C) == 16 && !INGRID && KIND != GAMMA_FWD;
    static constexpr int RH = Shape<N>::P > 1 && ((BIG && RH_PAYS) || THREE) && T % 2 == 0 && NT <= 512 ? 2 : 1;
    static constexpr int LDS = Shape<N>::P > 1 ? (T / RH) * Shape<N>::RS : 1;
};


// Radix of stage s: R0 first (when the decomposition needs it), then 16s.
template <int N, int S>
constexpr int radix_of() {
    if constexpr (N < 16) {
        return N;
    } else if constexpr (Shape<N>::R0 > 1) {
        return S == 0 ? Shape<N>::R0 : 16;
    } else {
        return 16;
    }
}
template <int N, int S>
constexpr int ns_of() {  // product of the radices before stage S
    if constexpr (S == 0) {
        return 1;
    } else {
        return ns_of<N, S - 1>() * radix_of<N, S - 1>();
    }
}

__device__ __forceinline__ int lds_pos(int t, int idx, int RS) { return t * RS + idx + (idx >> 4); }

// Twiddle and butterfly all of a thread's radix-R butterflies of stage S.
template <int N, int S, int SIGN, typename C>
__device__ __forceinline__ void run_stage(C (&v)[Shape<N>::E], int p, const C *__restrict__ tw) {
    constexpr int R = radix_of<N, S>(), NS = ns_of<N, S>();
    constexpr int P = Shape<N>::P, BPT = N / R / P;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        if constexpr (NS > 1) {
            const int b = p + k * P;
            const int kk = b % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) v[k * R + r] = cmul(v[k * R + r], tw[kk * r * (N / (R * NS))]);
        }
        dft<R, SIGN, C>(&v[k * R]);
    }
}

// Stage S outputs -> LDS (row t), element (b/NS)*NS*R + b%NS + r*NS.
template <int N, int S, typename C>
__device__ __forceinline__ void put_stage(const C (&v)[Shape<N>::E], C *lds, int t, int p) {
    constexpr int R = radix_of<N, S>(), NS = ns_of<N, S>();
    constexpr int P = Shape<N>::P, BPT = N / R / P, RS = Shape<N>::RS;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int b = p + k * P;
        const int base = (b / NS) * NS * R + b % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_pos(t, base + r * NS, RS)] = v[k * R + r];
    }
}

// Stage S inputs <- LDS (row t), element b + r*N/R.
template <int N, int S, typename C>
__device__ __forceinline__ void get_stage(C (&v)[Shape<N>::E], const C *lds, int t, int p) {
    constexpr int R = radix_of<N, S>();
    constexpr int P = Shape<N>::P, BPT = N / R / P, RS = Shape<N>::RS;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int b = p + k * P;
#pragma unroll
        for (int r = 0; r < R; ++r) v[k * R + r] = lds[lds_pos(t, b + r * (N / R), RS)];
    }
}

// One LDS exchange between stage SP (outputs in v, row tp, position pp_)
// and stage SG (inputs into v, row tg, position pg).  With row halves the
// buffer holds T/RH rows and the exchange runs in RH rounds; every thread's
// put row and get row lie in the same half (myh), so a thread puts before it
// gets and never overwrites values it has yet to store.
template <int N, int SP, int SG, typename C, int RH, int TH>
__device__ __forceinline__ void exchange(C (&v)[Shape<N>::E], C *lds, int tp, int pp_, int tg, int pg, int myh) {
    if constexpr (RH == 1) {
        put_stage<N, SP, C>(v, lds, tp, pp_);
        __syncthreads();
        get_stage<N, SG, C>(v, lds, tg, pg);
    } else {
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            if (myh == h) put_stage<N, SP, C>(v, lds, tp - h * TH, pp_);
            __syncthreads();
            if (myh == h) get_stage<N, SG, C>(v, lds, tg - h * TH, pg);
            if (h + 1 < RH) __syncthreads();
        }
    }
}

// Offset of the intermediate element u(j, q, i) (q = m' mod N after the
// gamma pass, i the alpha sample), in one of two layouts:
//   t1 (plan-owned, tile-blocked by T):  ((j/T * N + q) * T + j%T) * N + i
//   in-grid (SOFT_INPLACE_OK plans): inside the grid buffer, where the T
//     rows i0..i0+T-1 of beta sample j (the elements one gamma block reads)
//     hold that block's outputs in the order L = q * T + i%T:
//       ((i0 + L / N) * N + j) * N + L % N,   i0 = i - i%T.
// In both, an alpha block reads or writes runs of T elements (all of one
// contiguous T*N run for t1), and a gamma block only touches its own T rows
// in the in-grid layout, so that pass is safe in place.
template <int N, int T, bool INGRID>
__device__ __forceinline__ size_t u_index(int j, int q, int i) {
    if constexpr (INGRID) {
        const int L = q * T + i % T;
        return ((size_t)(i - i % T + L / N) * N + j) * N + L % N;
    } else {
        return ((size_t)((j / T) * N + q) * T + (j % T)) * N + i;
    }
}

// Pass kinds: where a block's T sequences come from and go to.

template <int KIND>
constexpr bool transposed_in() { return KIND == ALPHA_INV || KIND == GAMMA_INV; }
template <int KIND>
constexpr bool transposed_out() { return KIND == GAMMA_FWD || KIND == ALPHA_FWD; }

// Block -> (tile, line, batch).  Consecutive logical blocks are placed on the
// same XCD (the hardware deals blocks round-robin over the 8 XCDs), so the
// neighbouring runs touched by neighbouring tiles meet in one L2.
struct BlockPos {
    int tile, line, batch;
};
__device__ __forceinline__ BlockPos block_pos(int ntile, int nline) {
    const int per_batch = ntile * nline;
    int lin = blockIdx.x + gridDim.x * blockIdx.y;
    if (per_batch % 8 == 0) lin = (lin % 8) * (per_batch / 8) + lin / 8;
    return {lin % ntile, lin / ntile, (int)blockIdx.z};
}

// Beta rows of the alpha passes (PlanView::jn, a beta half of 2B = 2048 or
// all 2B): local row k is beta sample jrow(k), and S row position of beta
// sample j is jloc(j) (with stride jn).
__device__ __forceinline__ int jrow(const PlanView &p, int k) { return k + (k < p.jsplit ? p.joff0 : p.joff1); }
__device__ __forceinline__ int jloc(const PlanView &p, int j) {
    return j - (j < p.jsplit + p.joff0 ? p.joff0 : p.joff1);
}

// Twiddle table of a band for the complex type of the plan.
template <typename C>
__device__ __forceinline__ const C *twiddles(const PlanView &p, int sign);
template <>
__device__ __forceinline__ const double2 *twiddles<double2>(const PlanView &p, int sign) {
    return sign > 0 ? p.twp : p.twm;
}
template <>
__device__ __forceinline__ const float2 *twiddles<float2>(const PlanView &p, int sign) {
    return sign > 0 ? p.twpf : p.twmf;
}

// One pass over the functions of one band (blockIdx.z = index within the
// band; t1 holds one N^3 intermediate per such index).  Element addresses:
//   GAMMA_FWD: block (i-tile, j): in grid[(i*N + j)*N + k], out u(j, q, i)
//   ALPHA_FWD: block (j-tile, q): in u(j, q, i),               out S[slot*jn + jloc(j')]
//   ALPHA_INV: block (j-tile, q): in S[slot*jn + jloc(j')],    out u(j, q, i)
//   GAMMA_INV: block (i-tile, j): in u(j, q, i),               out grid[(i*N + j)*N + k]
// with u the intermediate in the t1 or the in-grid layout (u_index).  With
// t1, an alpha block then reads or writes one contiguous run of T*N
// elements, and a gamma block's runs of T elements for the N values of q
// stay within one window of T*N^2 elements (instead of striding over all
// N^3).  In the grid, every gamma block reads and writes only its own T
// rows, and all its loads are consumed before its first barrier (or, for
// N <= 16, by the one thread that owns the sequence), so in == out is safe.
//
// With ARGMAX (inverse gamma pass only) the pass stores nothing: each block
// reduces the values it would store to the best (Re, flat index) and writes
// that to part (see launch_fft_gamma_inv_argmax).
template <int N, int KIND, int SIGN, typename C, bool INGRID, bool ARGMAX = false>
__device__ __forceinline__ void fft_pass(const PlanView &p, const C *in, C *out, int flags,
                                         ArgBest *part = nullptr) {
    static_assert(!ARGMAX || (KIND == GAMMA_INV && !INGRID), "argmax is fused into the inverse gamma pass");
    // streaming stores are built for 2B <= 512 only (stream_stores never asks at 1024)
    const bool apply_w = flags & kFlagScale, stream = N <= 512 && (flags & kFlagStream);
    using Sh = Shape<N>;
    constexpr int T = Tile<N, C, KIND, INGRID>::T, P = Sh::P, E = Sh::E, NSTG = Sh::NSTAGE;
    constexpr int TL = Tile<N, C, KIND, INGRID>::TL;  // layout of the intermediate
    constexpr int B = N / 2;
    constexpr int LAST = NSTG - 1;
    constexpr bool ALPHA = KIND == ALPHA_FWD || KIND == ALPHA_INV;
    __shared__ C lds[Tile<N, C, KIND, INGRID>::LDS];
    const C *tw = twiddles<C>(p, SIGN);

    // lines: j for gamma passes (N of them), q != B for alpha passes (N - 1).
    const BlockPos bp = block_pos((ALPHA ? p.jn : N) / T, ALPHA ? N - 1 : N);
    const int tile = bp.tile;
    const int line = ALPHA ? (bp.line < B ? bp.line : bp.line + 1) : bp.line;
    const size_t N3 = (size_t)N * N * N;
    const FuncInfo fi = p.funcs[p.band_funcs[bp.batch]];
    const C *src;
    C *dst;
    const size_t u_off = INGRID ? (size_t)fi.grid_off : bp.batch * N3;  // the intermediate of this function
    if constexpr (KIND == GAMMA_FWD) {
        src = in + fi.grid_off;
        dst = out + u_off;
    } else if constexpr (KIND == ALPHA_FWD) {
        src = in + u_off;
        dst = out + fi.s_off;
    } else if constexpr (KIND == ALPHA_INV) {
        src = in + fi.s_off;
        dst = out + u_off;
    } else {
        src = in + u_off;
        dst = ARGMAX ? nullptr : out + fi.grid_off;
    }
    const int tid = threadIdx.x;
    const int mp_line = line < B ? line : line - N;  // m' of an alpha-pass block

    C v[E];
    // Thread -> (row, position).  On a transposed side the row index is
    // fastest (row tid % T), so T neighbouring lanes move one run of T
    // elements.  On a row side, position fastest; with row halves (RH = 2)
    // the rows are dealt so that a thread's row on every side lies in the
    // same half, (tid % T) / TH: lanes of one half take consecutive
    // positions of one row (runs of up to 32 elements per row and wave).
    constexpr int RH = Tile<N, C, KIND, INGRID>::RH, TH = T / RH;
    const int myh = RH == 1 ? 0 : (tid % T) / TH;
    int row_t, row_p;
    if constexpr (RH == 1) {
        row_t = tid / P;
        row_p = tid % P;
    } else {
        const int rank = (tid / T) * TH + tid % TH;
        row_t = myh * TH + rank / P;
        row_p = rank % P;
    }
    // ---- stage 0 inputs from HBM: element b + r*N/R ----
    const int t_in = transposed_in<KIND>() ? tid % T : row_t;
    const int p_in = transposed_in<KIND>() ? tid / T : row_p;
    {
        constexpr int R = radix_of<N, 0>(), BPT = N / R / P;
        const int row = ALPHA ? jrow(p, tile * T + t_in) : tile * T + t_in;  // i (gamma) or j (alpha)
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int n = p_in + k * P + r * (N / R);
                C x;
                if constexpr (KIND == GAMMA_FWD) {
                    x = ld_in<N>(&src[((size_t)row * N + line) * N + n]);
                } else if constexpr (KIND == ALPHA_FWD) {
                    x = ld_in<N>(&src[u_index<N, TL, INGRID>(row, line, n)]);
                } else if constexpr (KIND == ALPHA_INV) {
                    if (n == B) {
                        x = mk<C>(0.0, 0.0);
                    } else {
                        const int sl = slot_code(n < B ? n : n - N, mp_line);
                        const int jj = (sl & 1) ? N - 1 - row : row;
                        x = ld_in<N>(&src[(size_t)(sl >> 1) * p.jn + jloc(p, jj)]);
                    }
                } else {
                    x = n == B ? mk<C>(0.0, 0.0) : ld_in<N>(&src[u_index<N, TL, INGRID>(line, n, row)]);
                }
                v[k * R + r] = x;
            }
        }
    }
    run_stage<N, 0, SIGN, C>(v, p_in, tw);

    // ---- exchanges through LDS ----
    int t_out = t_in, p_out = p_in;
    if constexpr (NSTG > 1) {
        const int t = row_t, pp = row_p;
        t_out = transposed_out<KIND>() ? tid % T : t;
        p_out = transposed_out<KIND>() ? tid / T : pp;
        if constexpr (NSTG > 2) {
            exchange<N, 0, 1, C, RH, TH>(v, lds, t_in, p_in, t, pp, myh);
            run_stage<N, 1, SIGN, C>(v, pp, tw);
            __syncthreads();
            exchange<N, 1, LAST, C, RH, TH>(v, lds, t, pp, t_out, p_out, myh);
        } else {
            exchange<N, 0, LAST, C, RH, TH>(v, lds, t_in, p_in, t_out, p_out, myh);
        }
        run_stage<N, LAST, SIGN, C>(v, p_out, tw);
    }

    // ---- last stage outputs to HBM: element b + r*N/R ----
    {
        constexpr int R = radix_of<N, LAST>(), BPT = N / R / P;
        const int row = ALPHA ? jrow(p, tile * T + t_out) : tile * T + t_out;
        double wj = 1.0;
        if constexpr (KIND == ALPHA_FWD || KIND == GAMMA_INV) {
            if (apply_w) wj = p.w[KIND == ALPHA_FWD ? row : line];
        }
        ArgBest best{-__builtin_huge_val(), kNoIndex};
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int n = p_out + k * P + r * (N / R);
                const C x = v[k * R + r];
                if constexpr (KIND == GAMMA_FWD) {
                    if (n != B) put_c(&dst[u_index<N, TL, INGRID>(line, n, row)], x, stream);
                } else if constexpr (KIND == ALPHA_FWD) {
                    if (n != B) {
                        const int sl = slot_code(n < B ? n : n - N, mp_line);
                        const int jj = (sl & 1) ? N - 1 - row : row;
                        put_c(&dst[(size_t)(sl >> 1) * p.jn + jloc(p, jj)], cscale(x, wj), stream);
                    }
                } else if constexpr (KIND == ALPHA_INV) {
                    put_c(&dst[u_index<N, TL, INGRID>(row, line, n)], x, stream);
                } else if constexpr (ARGMAX) {
                    best = arg_better(best, ArgBest{(double)cscale(x, wj).x, ((long long)row * N + line) * N + n});
                } else {
                    put_c(&dst[((size_t)row * N + line) * N + n], cscale(x, wj), stream);
                }
            }
        }
        if constexpr (ARGMAX) {
            // Block reduction: across each wave by lane exchange, then over the
            // waves (or, in blocks of fewer than 64 threads, over the threads).
            constexpr int NT = Tile<N, C, KIND, INGRID>::NT, NR = NT >= 64 ? NT / 64 : NT;
            __shared__ double rv[NR];
            __shared__ long long ri[NR];
            if constexpr (NT >= 64) {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    ArgBest q;
                    q.v = __shfl_xor(best.v, o);
                    q.i = __shfl_xor(best.i, o);
                    best = arg_better(best, q);
                }
                if ((tid & 63) == 0) {
                    rv[tid >> 6] = best.v;
                    ri[tid >> 6] = best.i;
                }
            } else {
                rv[tid] = best.v;
                ri[tid] = best.i;
            }
            __syncthreads();
            if (tid == 0) {
                ArgBest r{rv[0], ri[0]};
                for (int w = 1; w < NR; ++w) r = arg_better(r, ArgBest{rv[w], ri[w]});
                part[(size_t)bp.batch * ((N / T) * N) + (size_t)line * (N / T) + tile] = r;
            }
        }
    }
}

// Intermediate in the plan's t1: input and output never alias.
template <int N, int KIND, int SIGN, typename C>
__global__ __launch_bounds__((Tile<N, C, KIND, false>::NT)) void k_fft(PlanView p, const C *__restrict__ in, C *__restrict__ out,
                                                     int flags) {
    fft_pass<N, KIND, SIGN, C, false>(p, in, out, flags);
}

// Intermediate in the grid buffer: the gamma passes run in place (in == out).
template <int N, int KIND, int SIGN, typename C>
__global__ __launch_bounds__((Tile<N, C, KIND, true>::NT)) void k_fft_ingrid(PlanView p, const C *in, C *out, int flags) {
    fft_pass<N, KIND, SIGN, C, true>(p, in, out, flags);
}

// The inverse gamma pass fused with the first argmax stage.
template <int N, typename C>
__global__ __launch_bounds__((Tile<N, C, GAMMA_INV, false>::NT)) void k_fft_gamma_inv_argmax(PlanView p, const C *__restrict__ in,
                                                                      ArgBest *__restrict__ part) {
    fft_pass<N, GAMMA_INV, -1, C, false, true>(p, in, nullptr, 0, part);
}

template <int N, typename C>
hipError_t launch_argmax_pass(const PlanView &p, const C *in, ArgBest *part, hipStream_t s) {
    using Ti = Tile<N, C, GAMMA_INV, false>;
    hipLaunchKernelGGL((k_fft_gamma_inv_argmax<N, C>), dim3(N / Ti::T, N, p.nfunc), dim3(Ti::NT), 0, s, p, in, part);
    return hipGetLastError();
}

template <int N, int KIND, int SIGN, typename C, bool INGRID>
hipError_t launch_kind(const PlanView &p, const C *in, C *out, int flags, hipStream_t s) {
    using Ti = Tile<N, C, KIND, INGRID>;
    constexpr bool ALPHA = KIND == ALPHA_FWD || KIND == ALPHA_INV;
    const int nline = ALPHA ? N - 1 : N;
    // Grid (tiles, lines, functions of the band); block_pos() re-deals (tile, line) across XCDs.
    // The alpha passes cover the view's beta rows (all, or one beta half).
    dim3 g((ALPHA ? p.jn : N) / Ti::T, nline, p.nfunc);
    if constexpr (INGRID)
        hipLaunchKernelGGL((k_fft_ingrid<N, KIND, SIGN, C>), g, dim3(Ti::NT), 0, s, p, in, out, flags);
    else
        hipLaunchKernelGGL((k_fft<N, KIND, SIGN, C>), g, dim3(Ti::NT), 0, s, p, in, out, flags);
    return hipGetLastError();
}

template <int KIND, int SIGN, typename C, bool INGRID>
hipError_t dispatch(const PlanView &p, const C *in, C *out, int flags, hipStream_t s) {
    switch (p.N) {
        case 2: return launch_kind<2, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 4: return launch_kind<4, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 8: return launch_kind<8, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 16: return launch_kind<16, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 32: return launch_kind<32, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 64: return launch_kind<64, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 128: return launch_kind<128, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 256: return launch_kind<256, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 512: return launch_kind<512, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 1024: return launch_kind<1024, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        case 2048: return launch_kind<2048, KIND, SIGN, C, INGRID>(p, in, out, flags, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// Entry points.  With t1 == nullptr the intermediate lives in the grid
// buffer: the forward gamma pass overwrites the input grid, the inverse
// alpha pass stages in the output grid.
template <typename C>
hipError_t launch_fft_gamma_fwd(const PlanView &p, const C *grid, C *t1, bool stream, hipStream_t s) {
    const int f = stream ? kFlagStream : 0;
    if (!t1) return dispatch<GAMMA_FWD, +1, C, true>(p, grid, const_cast<C *>(grid), f, s);
    return dispatch<GAMMA_FWD, +1, C, false>(p, grid, t1, f, s);
}
template <typename C>
hipError_t launch_fft_alpha_fwd(const PlanView &p, const C *t1, const C *grid, C *S, bool apply_w, bool stream,
                                hipStream_t s) {
    const int f = (apply_w ? kFlagScale : 0) | (stream ? kFlagStream : 0);
    if (!t1) return dispatch<ALPHA_FWD, +1, C, true>(p, grid, S, f, s);
    return dispatch<ALPHA_FWD, +1, C, false>(p, t1, S, f, s);
}
template <typename C>
hipError_t launch_fft_alpha_inv(const PlanView &p, const C *S, C *t1, C *grid, bool stream, hipStream_t s) {
    const int f = stream ? kFlagStream : 0;
    if (!t1) return dispatch<ALPHA_INV, -1, C, true>(p, S, grid, f, s);
    return dispatch<ALPHA_INV, -1, C, false>(p, S, t1, f, s);
}
template <typename C>
hipError_t launch_fft_gamma_inv(const PlanView &p, const C *t1, C *grid, bool apply_w, bool stream, hipStream_t s) {
    const int f = (apply_w ? kFlagScale : 0) | (stream ? kFlagStream : 0);
    if (!t1) return dispatch<GAMMA_INV, -1, C, true>(p, grid, grid, f, s);
    return dispatch<GAMMA_INV, -1, C, false>(p, t1, grid, f, s);
}

template <typename C>
hipError_t launch_fft_gamma_inv_argmax(const PlanView &p, const C *t1, ArgBest *part, hipStream_t s) {
    if (!t1 || !part) return hipErrorInvalidValue;
    switch (p.N) {
        case 2: return launch_argmax_pass<2, C>(p, t1, part, s);
        case 4: return launch_argmax_pass<4, C>(p, t1, part, s);
        case 8: return launch_argmax_pass<8, C>(p, t1, part, s);
        case 16: return launch_argmax_pass<16, C>(p, t1, part, s);
        case 32: return launch_argmax_pass<32, C>(p, t1, part, s);
        case 64: return launch_argmax_pass<64, C>(p, t1, part, s);
        case 128: return launch_argmax_pass<128, C>(p, t1, part, s);
        case 256: return launch_argmax_pass<256, C>(p, t1, part, s);
        case 512: return launch_argmax_pass<512, C>(p, t1, part, s);
        case 1024: return launch_argmax_pass<1024, C>(p, t1, part, s);
        case 2048: return launch_argmax_pass<2048, C>(p, t1, part, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {
template <typename C>
int argmax_blocks_of(int N) {
    switch (N) {
        case 2: return 2 / Tile<2, C, GAMMA_INV, false>::T * 2;
        case 4: return 4 / Tile<4, C, GAMMA_INV, false>::T * 4;
        case 8: return 8 / Tile<8, C, GAMMA_INV, false>::T * 8;
        case 16: return 16 / Tile<16, C, GAMMA_INV, false>::T * 16;
        case 32: return 32 / Tile<32, C, GAMMA_INV, false>::T * 32;
        case 64: return 64 / Tile<64, C, GAMMA_INV, false>::T * 64;
        case 128: return 128 / Tile<128, C, GAMMA_INV, false>::T * 128;
        case 256: return 256 / Tile<256, C, GAMMA_INV, false>::T * 256;
        case 512: return 512 / Tile<512, C, GAMMA_INV, false>::T * 512;
        case 1024: return 1024 / Tile<1024, C, GAMMA_INV, false>::T * 1024;
        case 2048: return 2048 / Tile<2048, C, GAMMA_INV, false>::T * 2048;
        default: return 0;
    }
}
}  // namespace

int gamma_argmax_blocks(int N, int csize) { return csize == 16 ? argmax_blocks_of<double2>(N) : argmax_blocks_of<float2>(N); }

#define SOFT_FFT_INSTANTIATE(C)                                                                               \
    template hipError_t launch_fft_gamma_fwd<C>(const PlanView &, const C *, C *, bool, hipStream_t);            \
    template hipError_t launch_fft_alpha_fwd<C>(const PlanView &, const C *, const C *, C *, bool, bool,         \
                                                hipStream_t);                                                  \
    template hipError_t launch_fft_alpha_inv<C>(const PlanView &, const C *, C *, C *, bool, hipStream_t);       \
    template hipError_t launch_fft_gamma_inv<C>(const PlanView &, const C *, C *, bool, bool, hipStream_t);      \
    template hipError_t launch_fft_gamma_inv_argmax<C>(const PlanView &, const C *, ArgBest *, hipStream_t);
SOFT_FFT_INSTANTIATE(double2)
SOFT_FFT_INSTANTIATE(float2)

}  // namespace soft
