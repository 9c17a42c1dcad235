// soft_internal.h -- plan structure and kernel launchers shared by the
// library's translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/soft.h"

namespace soft {

// Symmetry group of order pairs (Sect. 3, "Communication"/"Agglomeration"):
// one representative (m, m') with m >= m' >= 0 stands for up to eight pairs
// whose Wigner-d values coincide up to sign, at beta or at pi - beta (eq.
// "Wigner_symmetries").  Member slots, with d_rep(l;b) = d(l,m,m';b):
//   slot 0 ( m,  m') at b      sign 1
//   slot 1 (-m, -m') at b      sign (-1)^(m-m')
//   slot 2 ( m', m ) at b      sign (-1)^(m-m')
//   slot 3 (-m', -m) at b      sign 1
//   slot 4 (-m,  m') at pi-b   sign (-1)^(l-m')
//   slot 5 ( m, -m') at pi-b   sign (-1)^(l+m)
//   slot 6 (-m', m ) at pi-b   sign (-1)^(l-m')
//   slot 7 ( m', -m) at pi-b   sign (-1)^(l+m)
// Present slots: all 8 for m > m' > 0; {0,1,4,5} for m = m' > 0;
// {0,1,2,3} for m > 0 = m'; {0} for m = m' = 0.  Every (m, m') with
// |m|, |m'| < B belongs to exactly one (group, slot).
constexpr int kSlots = 8;

// Rows of padding after the last group in the per-row tables: the DWT kernels
// prefetch up to 32 rows past a group's end (the values are never used).
constexpr int kPadRows = 32;

// Kernel flag bits (the int flag argument of the FFT and inverse-DWT kernels).
constexpr int kFlagScale = 1;   // apply w_B(j) (FFT) or V_B (inverse DWT)
constexpr int kFlagStream = 2;  // write the main output with streaming stores
constexpr int kFlagAccum = 4;   // forward DWT: add to the coefficients instead of writing them

// Beta halves.  The band of 2B = 2048 keeps S for half of its beta samples
// at a time (half the workspace: FP64 at B = 1024 then fits one GPU), in two
// chunks closed under j -> 2B-1-j (the members at pi - beta are stored
// j-reversed, so a chunk holds both ends of every pair): chunk 0 is
// j < 2B/4 and j >= 3(2B)/4, chunk 1 the middle half.  A chunk's S rows are
// indexed by the chunk-local k in [0, n); its beta sample is
//   j = k + (k < split ? off0 : off1),
// and back, k = j - (j < split + off0 ? off0 : off1).  n = 0 means the whole
// range with k = j (every band below 2B = 2048).
struct JMap {
    int n = 0, split = 0, off0 = 0, off1 = 0;
};
constexpr int kBetaChunkN = 2048;  // bands of this 2B run in two beta halves
inline JMap beta_chunk(int N, int c) {
    JMap m;
    m.n = N / 2;
    if (c == 0) {
        m.split = N / 4;
        m.off0 = 0;
        m.off1 = N / 2;
    } else {
        m.split = N / 2;
        m.off0 = N / 4;
        m.off1 = N / 4;
    }
    return m;
}

// Whether a launch writes its main output with streaming (non-temporal)
// stores: bytes written by the launch, nmax its largest 2B, above the
// launch kind's threshold.  Measured on MI355X: they speed up the next kernel
// when the array written is well beyond the 256 MB last-level cache (B = 128
// with 4 to 64 functions, B = 256: 2-4 % per step); below that, plain stores
// leave much of the array cached for the next kernel.  Near the cache size
// the passes differ: at one B = 128 FP64 function (268 MB arrays) plain
// stores in the alpha passes and the inverse gamma pass, and streaming ones
// in the forward gamma pass and the iDWT, gave the fastest step of all 32
// choices (616 -> 588 us), and two functions or four FP32 ones (536 MB)
// were no slower or 2-3 % faster; so the former stream from 600 MB, the
// latter from 192 MB.  At 2B = 1024 streaming slowed the FFT passes down
// (B = 512: 3 % per step), so those launches keep plain stores.
constexpr double kStreamFrom = 192.0 * (1 << 20);      // forward gamma pass, iDWT
constexpr double kStreamFromLate = 600.0 * (1 << 20);  // alpha passes, inverse gamma pass
inline bool stream_stores(double bytes, int nmax, double from) { return nmax < 1024 && bytes > from; }

// Running argmax of Re over a grid: the larger value wins, on equal values
// the smaller flat index; NaN never wins (comparisons with NaN are false), so
// a scan that sees only NaN keeps kNoIndex.
struct ArgBest {
    double v;
    long long i;
};
constexpr long long kNoIndex = 0x7fffffffffffffffLL;
__device__ __forceinline__ ArgBest arg_better(ArgBest p, ArgBest q) {
    return (q.v > p.v || (q.v == p.v && q.i < p.i)) ? q : p;
}

// Store of one complex value, streaming (non-temporal) when asked.
__device__ __forceinline__ void put_c(double2 *p, double2 x, bool stream) {
    typedef double r2 __attribute__((ext_vector_type(2)));
    if (stream) __builtin_nontemporal_store((r2){x.x, x.y}, reinterpret_cast<r2 *>(p));
    else *p = x;
}
__device__ __forceinline__ void put_c(float2 *p, float2 x, bool stream) {
    typedef float r2 __attribute__((ext_vector_type(2)));
    if (stream) __builtin_nontemporal_store((r2){x.x, x.y}, reinterpret_cast<r2 *>(p));
    else *p = x;
}

// Group slot code of order pair (m, m'), |m|, |m'| < B: (g*8 + s)*2 + (s >= 4)
// with g = a(a+1)/2 + b for the representative a = max(|m|,|m'|),
// b = min(|m|,|m'|) (groups ordered by a, then b) and s the member slot above.
__host__ __device__ inline int slot_code(int m, int mp) {
    const int am = m < 0 ? -m : m, amp = mp < 0 ? -mp : mp;
    int a, b, s;
    if (am >= amp) {
        a = am;
        b = amp;
        s = m >= 0 ? (mp >= 0 ? 0 : 5) : (mp > 0 ? 4 : 1);
    } else {
        a = amp;
        b = am;
        s = mp > 0 ? (m >= 0 ? 2 : 6) : (m <= 0 ? 3 : 7);
    }
    const int g = a * (a + 1) / 2 + b;
    return (g * kSlots + s) * 2 + (s >= 4 ? 1 : 0);
}

// Block index -> symmetry group.  Groups are numbered largest first (cost
// ~ (B - m) * members), and the hardware deals blocks round-robin to the 8
// XCDs.  Each run of 64 blocks is re-dealt so that one XCD gets 8 consecutive
// groups: neighbouring groups touch neighbouring coefficients (f°(l,m,m') and
// f°(l,m,m'+-1) are adjacent), so their scattered 16-byte accesses meet in one
// L2, while the largest-first order holds at a granularity of 64 groups.
__device__ __forceinline__ int group_of_block(int b, int G) {
    if (b >= (G & ~63)) return b;
    return (b & ~63) + ((b & 7) << 3) + ((b >> 3) & 7);
}

// Flat l-major index of f°(l, m, m').
__host__ __device__ __forceinline__ long long coeff_index(int l, int m, int mp) {
    const long long L = l;
    return L * (4 * L * L - 1) / 3 + (long long)(m + l) * (2 * l + 1) + (mp + l);
}

// Member (m, m') of slot s of the representative (m0, m0') and its sign at
// degree l (table in the comment above kSlots).
__host__ __device__ __forceinline__ void group_member(int s, int m0, int mp0, int l, int &mm, int &mmp,
                                                      double &sign) {
    const bool odd_mmp = (m0 - mp0) & 1;  // (-1)^(m-m')
    const bool odd_lmp = (l - mp0) & 1;   // (-1)^(l-m')
    const bool odd_lm = (l + m0) & 1;     // (-1)^(l+m)
    bool neg = false;
    switch (s) {
        case 0: mm = m0;   mmp = mp0;  break;
        case 1: mm = -m0;  mmp = -mp0; neg = odd_mmp; break;
        case 2: mm = mp0;  mmp = m0;   neg = odd_mmp; break;
        case 3: mm = -mp0; mmp = -m0;  break;
        case 4: mm = -m0;  mmp = mp0;  neg = odd_lmp; break;
        case 5: mm = m0;   mmp = -mp0; neg = odd_lm; break;
        case 6: mm = -mp0; mmp = m0;   neg = odd_lmp; break;
        default: mm = mp0; mmp = -m0;  neg = odd_lm; break;
    }
    sign = neg ? -1.0 : 1.0;
}

struct GroupInfo {
    int m, mp;     // representative, m >= mp >= 0; lowest degree l0 = m
    int mask;      // bit s set when slot s is present
    int pad;
};

// Arithmetic of a plan.  P64: complex128 data, FP64 throughout.  P32:
// complex64 data, FP32 FFTs and FP32 MFMA contractions with d rounded to
// FP32.  P32S: as P32 but d is split into hi + lo FP32 parts: hi contracted
// on FP32 matrix cores, the tail lo (about 2^-24 of d) on bf16 matrix cores.
// In both FP32 modes the partial sums (at most 32 beta samples or 16
// degrees) are combined in FP64.  In every mode the seeds, the recurrence,
// s_l, V_B and w_B(j) stay in FP64.
enum Prec { P64 = 0, P32 = 1, P32S = 2 };
template <int PR>
struct PrecT {
    using R = float;
    using C = float2;
};
template <>
struct PrecT<P64> {
    using R = double;
    using C = double2;
};

// One function of a plan: element offsets (complex) of its grid, its
// coefficients and its beta-sample workspace, and its band.
struct FuncInfo {
    long long grid_off, coeff_off, s_off;
    int band, pad;
};

// One DWT work item: one symmetry group of one function, carrying every
// value a block indexes uniformly (so none of them comes through a pointer
// loaded from memory, which the compiler would treat as divergent).
struct WorkItem {
    long long goff;       // first row of the group in the plan-wide recurrence tables
    long long s_off;      // the group's beta-sample block in S (complex elements)
    long long coeff_off;  // the function's coefficient vector (complex elements)
    long long seed_off;   // the group's 2B seeds d(l0, l0, m'; b_j) in the seed table
    int B;                // bandwidth of the function
    int jbase;            // the band's first entry in the plan-wide beta tables
    int m, mp;            // representative, m >= mp >= 0
    int mask;             // bit s set when slot s is present
    int pad;
};

// Plan-wide tables of the DWT kernels (kernel arguments).
// Work item of DWT block b of n: runs of 64 items are re-dealt so that one XCD
// gets 8 consecutive items (8 neighbouring groups of one function, whose
// scattered 16-byte coefficient accesses then meet in one L2); the list
// itself is largest-cost first.  Everything a block indexes uniformly comes
// from its item and from the kernel arguments, so it stays in scalar
// registers.
__device__ __forceinline__ int item_of_block(int b, int n) {
    if (b >= (n & ~63)) return b;
    return (b & ~63) + ((b & 7) << 3) + ((b >> 3) & 7);
}

struct DwtTables {
    const double *cosb;   // cos(beta_j), band by band
    const double *seed;   // d(l0, l0, m'; b_j) per group and beta sample, band by band
    const double *rscale; // s_l per row (d(l) = s_l e(l))
    const double2 *rec;   // (alpha_l, gamma_l) per row (the kernels take it as a separate
                          // restrict argument, so its loads can use the scalar cache)
};

// The low parts of a SOFT_DD_RECURRENCE plan's tables (the DWT kernels'
// double-double recurrence): cos(beta_j) - cosb[j] band by band, and
// (alpha_l, gamma_l) - rec per row.
struct DdTables {
    const double *cosb_lo;
    const double2 *rec_lo;
};

// Device-side view of one band (all functions of one bandwidth).
struct PlanView {
    int B, N, G;
    int nfunc;             // functions in this band
    long long Nc;          // coefficients per function
    long long rows;        // group rows (one per group and degree) per function
    const double *w;       // [N]   quadrature weights w_B(j)
    const double *cosb;    // [N]   cos(beta_j) (slice of the plan-wide table)
    const double4 *lcs;    // [N]   (log cos(b_j/2) hi, lo, log sin(b_j/2) hi, lo) (slice)
    const double2 *lbin;   // [G]   0.5 log((2m)!/((m+m')!(m-m')!)) as (hi, lo) (slice)
    const GroupInfo *grp;  // [G]
    const long long *goff; // [G]   first row of group g in the plan's per-row tables
    const double2 *twp;    // [N]   e^{+2 pi i k/N}
    const double2 *twm;    // [N]   e^{-2 pi i k/N}
    const float2 *twpf;    // [N]   e^{+2 pi i k/N}, FP32
    const float2 *twmf;    // [N]   e^{-2 pi i k/N}, FP32
    const double *rscale;  // plan-wide per-row s_l (d(l) = s_l e(l)), indexed by goff
    const FuncInfo *funcs; // plan-wide function table
    const int *band_funcs; // [nfunc] function indices of this band
    // Beta rows of the alpha passes and of S (JMap with n = 0 as the whole
    // range): jn rows, S row stride jn, beta sample j = k + (k < jsplit ?
    // joff0 : joff1) of local row k.
    int jn, jsplit, joff0, joff1;
};

// FFT stage (separation of variables, Sect. 2.4), one launch per band; t1 is
// the band's tile-blocked intermediate, [nfunc][N^3].  With t1 == nullptr the
// passes keep the intermediate in grid order inside the grid buffer: the
// forward gamma pass overwrites the input grid in place and the inverse alpha
// pass stages in the output grid.  With stream the pass writes its output
// with streaming stores (stream_stores).
template <typename C>
hipError_t launch_fft_gamma_fwd(const PlanView &p, const C *grid, C *t1, bool stream, hipStream_t s);
template <typename C>
hipError_t launch_fft_alpha_fwd(const PlanView &p, const C *t1, const C *grid, C *S, bool apply_w, bool stream,
                                hipStream_t s);
template <typename C>
hipError_t launch_fft_alpha_inv(const PlanView &p, const C *S, C *t1, C *grid, bool stream, hipStream_t s);
template <typename C>
hipError_t launch_fft_gamma_inv(const PlanView &p, const C *t1, C *grid, bool apply_w, bool stream, hipStream_t s);

// The inverse gamma pass of a one-band plan fused with the first stage of
// the argmax of Re (rotational matching without materialising the grids):
// block (tile, line) of function f writes the best (Re, flat index
// (i*2B + j)*2B + k) of the values the pass would store to
// part[f * gamma_argmax_blocks(N, c) + line * (N / T) + tile], T the pass's
// tile height, c the complex size in bytes.  launch_argmax_final then
// reduces the gamma_argmax_blocks partials of each function.
template <typename C>
hipError_t launch_fft_gamma_inv_argmax(const PlanView &p, const C *t1, ArgBest *part, hipStream_t s);
int gamma_argmax_blocks(int N, int csize);

// Plan-time fill of the rescaled recurrence table of one band (rows from
// goff[g]; rec and rscale are the plan-wide tables).
hipError_t launch_fill_recurrence(const PlanView &p, double2 *rec, double *rscale, hipStream_t s);
// The same in double-double (rec + reclo; rscale rounded from a double-double product).
hipError_t launch_fill_recurrence_dd(const PlanView &p, double2 *rec, double2 *reclo, double *rscale,
                                     hipStream_t s);

// Plan-time fill of one band's seed table: seed[g*N + j] = d(l0, l0, m'; b_j)
// for every group g of the band (N = 2B entries per group).
hipError_t launch_fill_seeds(const PlanView &p, double *seed, hipStream_t s);

// DWT and iDWT over a device work list (one block per item), all items
// sharing one launch shape: nw waves, nsub subsets of 64 beta samples per
// wave (nw * nsub * 64 >= the beta rows of every item: its 2B, or jm.n).
// The forward writes the l-major coefficients (symmetry signs, s_l and, when
// apply_v, V_B applied), or adds to them with accum; the inverse reads them
// and writes S, with streaming stores when stream.  jm selects a beta half
// (JMap); xr runs the extended-range seeds of the 2B = 2048 band (the shapes
// 8x2, 16x1, 4x4 and 8x4 only); a non-null dd runs the recurrence in
// double-double with its tables (FP64; shapes 1x1, 2x1, 4x1, 8x1, 2x2, 4x2,
// 8x2, 16x1, 4x4; xr: 4x4, 8x2, 16x1).
template <int PR>
hipError_t launch_dwt_fwd(const DwtTables &tab, const WorkItem *items, int nitems, int nw, int nsub,
                          const typename PrecT<PR>::C *S, typename PrecT<PR>::C *coeffs, bool apply_v,
                          bool accum, const JMap &jm, bool xr, const DdTables *dd, hipStream_t s);
template <int PR>
hipError_t launch_dwt_inv(const DwtTables &tab, const WorkItem *items, int nitems, int nw, int nsub,
                          const typename PrecT<PR>::C *coeffs, typename PrecT<PR>::C *S, bool apply_v,
                          bool stream, const JMap &jm, bool xr, const DdTables *dd, hipStream_t s);

// The same inverse DWT by Clenshaw's backward summation (clenshaw.hip): one
// block of nmax rounded up to 64 lanes per work item, nmax/2 x 128 bytes of
// LDS; nmax is the largest 2B of the items (2 .. 1024).
template <int PR>
hipError_t launch_idwt_clenshaw(const DwtTables &tab, const WorkItem *items, int nitems, int nmax,
                                const typename PrecT<PR>::C *coeffs, typename PrecT<PR>::C *S, bool apply_v,
                                bool stream, hipStream_t s);

// The forward DWT by the transposed (adjoint) Clenshaw evaluation
// (clenshaw.hip): one block of nmax rounded up to 64 lanes per work item, one
// beta sample per lane, the sums over beta reduced across lanes; nmax is the
// largest 2B of the items (2 .. 1024).
template <int PR>
hipError_t launch_dwt_fwd_clenshaw(const DwtTables &tab, const WorkItem *items, int nitems, int nmax,
                                   const typename PrecT<PR>::C *S, typename PrecT<PR>::C *coeffs, bool apply_v,
                                   hipStream_t s);

// Rotational-matching head (match.hip).  n pairs of functions on the sphere
// (B^2 coefficients each): correlation coefficients a(l,M) conj(b(l,M')), the
// vector-Jacobian product of that map, and the per-grid argmax of Re over n
// grids of count elements (workspace of argmax_workspace_bytes(count, n)).
template <typename C>
hipError_t launch_corr_coeffs(int B, int n, const C *a, const C *b, C *coeffs, hipStream_t s);
template <typename C>
hipError_t launch_corr_vjp(int B, int n, const C *a, const C *b, const C *g, C *ga, C *gb, hipStream_t s);
size_t argmax_workspace_bytes(long long count, int n);
hipError_t launch_argmax_final(const ArgBest *part, int nblk, int n, long long *index, hipStream_t s);
template <typename C>
hipError_t launch_argmax_real(const C *x, long long count, int n, void *workspace, long long *index, hipStream_t s);

// Functions on the sphere (sphere.hip): the spherical-harmonic transform of
// n functions sampled on the (2B)^2 grid (theta_j, phi_k) into B^2
// coefficients each, and the refined rotation read-out of n correlation
// grids at their maxima (3 doubles per pair).
template <typename C>
hipError_t launch_sh_forward(int B, int n, const C *f, C *a, hipStream_t s);
template <typename C>
hipError_t launch_match_refine(int B, int n, const C *grid, const long long *index, double *out, hipStream_t s);
// Off-grid Newton polishing of n correlation maxima (sphere.hip): coeffs are
// the n correlation coefficient vectors of the one-band view v (B <= 512),
// rec / rscale the plan's recurrence table, start and angles n x 3 rotation
// angles (a, b, c) of Rz(a) Ry(b) Rz(c), value n values Re C at the result;
// ws a device workspace of polish_workspace_bytes(v.G, n) (state and chunk
// partials).
size_t polish_workspace_bytes(int G, int n);
template <typename C>
hipError_t launch_corr_polish(const PlanView &v, const double2 *rec, const double *rscale, int n, const C *coeffs,
                              const double *start, int iters, double *angles, double *value, double *ws,
                              hipStream_t s);

// Device ceilings (probe.hip): a streaming copy of `words` 16-byte words,
// and dependent-chain loops (kind 0: FP64 vector FMA, 1: FP64 MFMA 16x16x4,
// 2: FP32 MFMA 16x16x4) over `blocks` blocks of 4 waves; probe_flop_count is
// the flops one such launch performs.  sink: blocks * 256 doubles, never
// written in practice.
hipError_t launch_probe_copy(const void *src, void *dst, long long words, hipStream_t s);
hipError_t launch_probe_flops(int kind, int blocks, int iters, double *sink, hipStream_t s);
double probe_flop_count(int kind, int blocks, int iters);

}  // namespace soft
