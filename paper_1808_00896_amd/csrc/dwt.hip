// dwt.hip -- discrete Wigner transform (DWT) and its transpose (iDWT) on
// gfx950 for every symmetry group of order pairs: FP64 (v_mfma_f64_16x16x4)
// or, for complex64 plans, FP32 MFMA (v_mfma_f32_16x16x4) with d rounded to
// FP32 or split into hi + lo FP32 parts.
//
// Matrix form of Sect. 2.4: for each (m, m'),
//   forward  f°(l) = (2l+1)/(8 pi B) sum_j d(l,m,m';b_j) w_B(j) S(m,m';j)   (V T W)
//   inverse  S'(j) = sum_l d(l,m,m';b_j) f°(l)                              (T^T)
// The weights are applied by the FFT pass; the core of both kernels works on
// the representative d_rep(l; b_j) of a symmetry group and its <= 8 member
// columns c,
//   forward  G[l][c]  = sum_j d_rep(l; b_j) X[j][c]
//   inverse  Y[j][c]  = sum_l d_rep(l; b_j) F[l][c]
// (members at pi - beta were stored in reversed j order, eq. "Wigner_symmetries"),
// and the move between the l-major coefficient layout and the group columns,
// with each member's symmetry sign and the (2l+1)/(8 pi B) factor of V_B, is
// fused into the forward epilogue and the inverse staging.
//
// d_rep is never stored: each lane owns one beta_j, seeds d(l0,l0,m';b_j)
// (Sect. 2.2, evaluated in log space with double-double exponents) and runs
// the three-term recurrence of eq. "Wigner_d_recurrence" in FP64 registers.
// One block handles one (function, group) work item, so one recurrence feeds
// all members.  Every 16 degrees the lanes park the recurrence values in an
// LDS panel, which becomes the A operand of the MFMA contraction:
//   forward: 16 degrees x 4 beta samples (A) times 4 samples x 16 member
//            columns (B, the FFT output) reduce over beta; waves own disjoint
//            beta ranges and are summed in FP64 once per panel;
//   inverse: 16 samples x 4 degrees (A) times 4 degrees x 16 columns (B, the
//            coefficients) reduce over degrees inside each wave.
// In the FP32 modes the partial sums over one k-slot (16 beta samples) or one
// panel (16 degrees) are FP32 and are combined in FP64.  The split mode's
// tail products (d - hi(d), about 2^-24 of d) run on bf16 matrix cores, four
// FP32 k steps per v_mfma_f32_16x16x16_bf16.  FP64 plans made with
// SOFT_DD_RECURRENCE run the recurrence in double-double (the DD_ forms of
// the kernels) and round each value once into the same FP64 contraction.
#include "soft_internal.h"

namespace soft {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

// Four values as the bf16 operand of v_mfma_f32_16x16x16_bf16 (round to
// nearest even).  The split mode contracts the tail of d, about 2^-24 of d,
// on bf16 matrix cores: rounding tail and data to bf16 changes the tail's
// product by about 2^-8 of itself, about 2^-32 of the total.
__device__ __forceinline__ v4bf bf4(float a, float b, float c, float d) {
    v4bf r;
    r[0] = (__bf16)a;
    r[1] = (__bf16)b;
    r[2] = (__bf16)c;
    r[3] = (__bf16)d;
    return r;
}


struct DD {
    double hi, lo;
};

// The error-free sums and products below hold only if every operation
// rounds as written: hipcc contracts a product and a later sum into one FMA
// by default, which would drop the rounding that the error terms recover.
// Each of these functions turns that off for its own operations.
__device__ __forceinline__ DD two_prod(double a, double b) {
#pragma clang fp contract(off)
    const double h = a * b;
    return {h, fma(a, b, -h)};
}
__device__ __forceinline__ DD two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
// s + err = a + b exactly, for |a| >= |b| (or a = 0)
__device__ __forceinline__ DD quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return {s, b - (s - a)};
}

// Double-double arithmetic (Dekker's and Knuth's error-free sums and
// products, with the product's error by FMA): a value is hi + lo with
// |lo| <= ulp(hi)/2, about 106 significant bits.  The sums drop the rounding
// of lo + lo, so their relative error is about 2^-104 of |a| + |b|.
__device__ __forceinline__ DD dd_add(DD a, DD b) {
#pragma clang fp contract(off)
    const DD s = two_sum(a.hi, b.hi);
    return quick_two_sum(s.hi, s.lo + (a.lo + b.lo));
}
__device__ __forceinline__ DD dd_mul(DD a, DD b) {
#pragma clang fp contract(off)
    DD p = two_prod(a.hi, b.hi);
    p.lo = fma(a.hi, b.lo, fma(a.lo, b.hi, p.lo));
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ DD dd_mul(DD a, double b) {
#pragma clang fp contract(off)
    DD p = two_prod(a.hi, b);
    p.lo = fma(a.lo, b, p.lo);
    return quick_two_sum(p.hi, p.lo);
}
// a / b by long division: three quotient digits, each from the remainder so far.
__device__ __forceinline__ DD dd_div(DD a, DD b) {
#pragma clang fp contract(off)
    const double q1 = a.hi / b.hi;
    DD r = dd_add(a, dd_mul(b, -q1));
    const double q2 = r.hi / b.hi;
    r = dd_add(r, dd_mul(b, -q2));
    const double q3 = r.hi / b.hi;
    return dd_add(quick_two_sum(q1, q2), DD{q3, 0.0});
}
// sqrt(v) for a double v >= 0: the rounded root plus one Newton correction
// from its exact residual v - h^2 (one FMA).
__device__ __forceinline__ DD dd_sqrt(double v) {
#pragma clang fp contract(off)
    if (v <= 0.0) return {0.0, 0.0};
    const double h = sqrt(v);
    return quick_two_sum(h, fma(-h, h, v) / (2.0 * h));
}

// Seed d(l0, l0, m'; b_j) = sqrt((2 l0)!/((l0+m')!(l0-m')!)) cos^{l0+m'}(b/2)
// sin^{l0-m'}(b/2) for the representative (l0 = m >= m' >= 0), Sect. 2.2.
// The exponent is summed in double-double so only the final exp rounds.
//
// Extended range (xr, the bands of 2B = 2048).  Up to B = 512 every seed
// whose recurrence reaches 1e-20 before degree B is above 2^-700, but at
// B = 1024 such seeds go down to about 2^-1240 (for instance m = m' = 375
// near b = 2.39, whose d(l) reach 0.04 by l = 1023): below double
// precision's range.  There a seed under e^-700 is stored as -(seed * 2^1000)
// (seeds are never negative otherwise) and the kernels run that lane's
// recurrence scaled (panel_fill); seeds under 2^-2000 are 0.
constexpr double kXrScale = 0x1p1000, kXrUnscale = 0x1p-1000;
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;  // ln 2 = hi + lo

__device__ __forceinline__ double seed_d(double2 lb, double4 t, int m, int mp, bool xr) {
#pragma clang fp contract(off)
    const double P = (double)(m + mp), Q = (double)(m - mp);
    DD a = two_prod(P, t.x);
    a.lo = fma(P, t.y, a.lo);
    DD c = two_prod(Q, t.z);
    c.lo = fma(Q, t.w, c.lo);
    const DD s1 = two_sum(lb.x, a.hi);
    const DD s2 = two_sum(s1.hi, c.hi);
    const double lo = lb.y + a.lo + c.lo + s1.lo + s2.lo;
    if (!xr || s2.hi >= -700.0) {
        if (s2.hi < -745.0) return 0.0;
        return exp(s2.hi) * (1.0 + lo);  // exp(hi + lo) to O(lo^2), |lo| < 1e-12
    }
    // exp(hi + lo) 2^1000 = exp(r) 2^(q + 1000) with r = hi + lo - q ln 2 in double-double
    const double q = rint(s2.hi * M_LOG2E);
    if (q < -2000.0) return 0.0;
    const DD qa = two_prod(q, kLn2Hi);
    const DD r = two_sum(s2.hi, -qa.hi);
    const double rlo = ((r.lo - qa.lo) - q * kLn2Lo) + lo;
    return -ldexp(exp(r.hi) * (1.0 + rlo), (int)q + 1000);
}

// Rescaled three-term recurrence.  Eq. "Wigner_d_recurrence" reads, for the
// representative (m, m') and l >= l0,
//   d(l+1) = (A_l x - C_l) d(l) - Bc_l d(l-1),
//   A_l = (l+1)(2l+1)/sqrt(((l+1)^2-m^2)((l+1)^2-m'^2)),  C_l = A_l m m'/(l(l+1)),
//   Bc_l = (l+1) sqrt((l^2-m^2)(l^2-m'^2)) / (l sqrt(((l+1)^2-m^2)((l+1)^2-m'^2))),
// with C_0 = 0 and Bc_{l0} = 0 (the d(l0-1) term vanishes).  Writing
// d(l) = s_l e(l) with s_{l0} = s_{l0+1} = 1 and s_{l+1} = Bc_l s_{l-1} turns it
// into e(l+1) = (alpha_l x - gamma_l) e(l) - e(l-1), alpha_l = A_l s_l/s_{l+1},
// gamma_l = C_l s_l/s_{l+1}: two FMAs per step and two coefficients.  The
// kernels run e; s_l is applied where coefficients enter or leave.  Row goff[g] + (l - l0) of the
// table holds (alpha_l, gamma_l) and s_l; one thread per group fills it
// (s is a running product).
__global__ __launch_bounds__(256) void k_fill_recurrence(PlanView p, double2 *__restrict__ rec,
                                                        double *__restrict__ rscale) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= p.G) return;
    const GroupInfo gi = p.grp[g];
    const int m = gi.m, mp = gi.mp, l0 = m;
    const double M2 = (double)m * m, MP2 = (double)mp * mp, MMP = (double)m * mp;
    double2 *row = rec + p.goff[g];
    double *srow = rscale + p.goff[g];
    double s_prev = 0.0, s_cur = 1.0;  // s_{l-1}, s_l
    for (int t = 0; t < p.B - l0; ++t) {
        const int l = l0 + t;
        const double L = l, L1 = l + 1;
        const double den = sqrt((L1 * L1 - M2) * (L1 * L1 - MP2));
        const double A = L1 * (2.0 * L + 1.0) / den;
        const double C = l > 0 ? A * (MMP / (L * L1)) : 0.0;
        const double Bc = l > l0 ? L1 * sqrt((L * L - M2) * (L * L - MP2)) / (L * den) : 0.0;
        const double s_next = t == 0 ? 1.0 : Bc * s_prev;
        const double r = s_cur / s_next;
        row[t] = make_double2(A * r, C * r);
        srow[t] = s_cur;
        s_prev = s_cur;
        s_cur = s_next;
    }
}

// The same table in double-double (plans with SOFT_DD_RECURRENCE): rec gets
// the rounded (alpha_l, gamma_l), reclo what they lose in that rounding, and
// rscale the rounded s_l of a double-double running product.  The integer
// products under the square roots stay below 2^53 (l <= 2048), so they are
// exact, and every other step carries about 106 bits.
__global__ __launch_bounds__(256) void k_fill_recurrence_dd(PlanView p, double2 *__restrict__ rec,
                                                           double2 *__restrict__ reclo,
                                                           double *__restrict__ rscale) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= p.G) return;
    const GroupInfo gi = p.grp[g];
    const int m = gi.m, mp = gi.mp, l0 = m;
    const double M2 = (double)m * m, MP2 = (double)mp * mp, MMP = (double)m * mp;
    double2 *row = rec + p.goff[g];
    double2 *rlo = reclo + p.goff[g];
    double *srow = rscale + p.goff[g];
    DD s_prev = {0.0, 0.0}, s_cur = {1.0, 0.0};  // s_{l-1}, s_l
    for (int t = 0; t < p.B - l0; ++t) {
        const int l = l0 + t;
        const double L = l, L1 = l + 1;
        const DD den = dd_sqrt((L1 * L1 - M2) * (L1 * L1 - MP2));
        const DD A = dd_div(DD{L1 * (2.0 * L + 1.0), 0.0}, den);
        const DD C = l > 0 ? dd_div(dd_mul(A, MMP), DD{L * L1, 0.0}) : DD{0.0, 0.0};
        const DD Bc = l > l0 ? dd_div(dd_mul(dd_sqrt((L * L - M2) * (L * L - MP2)), L1), dd_mul(den, L))
                             : DD{0.0, 0.0};
        const DD s_next = t == 0 ? DD{1.0, 0.0} : dd_mul(Bc, s_prev);
        const DD r = dd_div(s_cur, s_next);
        const DD a = dd_mul(A, r), c = dd_mul(C, r);
        row[t] = make_double2(a.hi, c.hi);
        rlo[t] = make_double2(a.lo, c.lo);
        srow[t] = s_cur.hi;
        s_prev = s_cur;
        s_cur = s_next;
    }
}

// Seeds of every group of a band at every beta sample, once per plan (the
// DWT kernels load them instead of evaluating exp per work item).
__global__ __launch_bounds__(256) void k_fill_seeds(PlanView p, double *__restrict__ seed) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)p.G * p.N) return;
    const int g = (int)(e / p.N), j = (int)(e - (long long)g * p.N);
    const GroupInfo gi = p.grp[g];
    seed[e] = seed_d(p.lbin[g], p.lcs[j], gi.m, gi.mp, p.N >= 2048);
}

// ---------------------------------------------------------------------------
// Shared pieces
// ---------------------------------------------------------------------------
// Wave panels hold row r (degree l0 + lp + r) of 64 beta samples at
// pan[r * RS + jl].  The LDS has 64 four-byte banks and serves 8-byte reads 32
// lanes at a time, so the row stride is padded per access pattern:
//   writes (jl = lane, fixed r): contiguous, any stride;
//   forward A reads (r = lane%16, jl = 4s + lane/16): RS = 66 puts the 32
//     lanes of a pass on banks 4(lane%16) + 2(lane/16) + {0,1}, all distinct;
//   inverse A reads (jl = 16t + lane%16, r = s + 4(lane/16), the k slot's
//     degrees taken four apart): RS = 68 puts them on 32(lane/16) + 2(lane%16)
//     + {0,1}.
// Every address is then one per-lane base register plus an immediate offset.
constexpr int kRowFwd = 66;
constexpr int kRowInv = 68;

// Flat index of f°(l, m, m') (64-bit: at B = 1024 twice the index of the
// real part passes 2^31).
__device__ __forceinline__ long long coeff_index64(int l, int m, int mp) {
    return (long long)l * (4 * l * l - 1) / 3 + (m + l) * (2 * l + 1) + (mp + l);
}

// s_waitcnt lgkmcnt(0) (vmcnt and expcnt left at their maxima), fenced so the
// scheduler keeps later loads behind it.
__device__ __forceinline__ void lds_wait_all() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_sched_barrier(0);
}

// Block barrier that orders LDS only: each wave's LDS operations complete
// (lgkmcnt(0)) before it arrives, while its global loads, stores and LDS DMA
// stay in flight.  A __syncthreads (or a fence on LDS alone, which must also
// cover the LDS DMA) would wait for all of those with vmcnt(0).  The barrier
// is an asm statement with a memory clobber, so the compiler keeps every
// memory access on its side.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    asm volatile("s_barrier" ::: "memory");
}

// Value of the neighbouring lane (lane ^ 1): DPP quad_perm [1, 0, 3, 2].
__device__ __forceinline__ int swap_pair_lanes(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float swap_pair_lanes(float v) { return __int_as_float(swap_pair_lanes(__float_as_int(v))); }
__device__ __forceinline__ double swap_pair_lanes(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = swap_pair_lanes((int)b), hi = swap_pair_lanes((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Panel entry for the precision: FP64 stores e; FP32 stores (hi, lo) floats
// in the same 8 bytes (lo = e - hi, used by the split mode).
template <int PR>
__device__ __forceinline__ void panel_put(double *slotp, double e) {
    if constexpr (PR == P64) {
        *slotp = e;
    } else {
        const float hi = (float)e;
        const float lo = PR == P32S ? (float)(e - (double)hi) : 0.0f;
        *reinterpret_cast<float2 *>(slotp) = make_float2(hi, lo);
    }
}

// A lane's seed as stored (seed_d): e(l0) and its scale xs (1, or 2^-1000
// for an extended-range seed).
__device__ __forceinline__ void seed_load(double sd, bool in, double &e, double &xs) {
    e = in ? fabs(sd) : 0.0;
    xs = sd < 0.0 ? kXrUnscale : 1.0;
}

// One panel of a lane's recurrence: rows r = 0..15 (pan[r * RS], pan offset
// by the lane) get e(l0 + lp + r), and (ecur, eprev) advance 16 degrees with
// the panel's coefficients c.  With XR (the launch shapes that cover
// 2B = 2048), a lane whose seed was stored scaled runs e = d 2^1000 / s_l
// and writes e * xs; once |e| passes 2^800 the scale is folded back (d grows
// by at most about 2^116 over 16 degrees, so e stays far below the double
// range in between).  A wave without a scaled lane takes the plain loop.
// With DD (SOFT_DD_RECURRENCE) the step runs in double-double: alpha, gamma
// (c + cl), x (x + xl) and e (ecur + ecl, eprev + epl), and the panel gets e
// rounded to double.
template <int PR, int RS, bool XR, bool DD_>
__device__ __forceinline__ void panel_fill(double *pan, const double2 (&c)[16], const double2 (&cl)[16], double x,
                                           double xl, double &ecur, double &eprev, double &ecl, double &epl,
                                           double &xs) {
    if constexpr (DD_) {
#pragma clang fp contract(off)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            panel_put<PR>(&pan[r * RS], XR ? ecur * xs : ecur);
            // u = alpha x - gamma
            DD pr = two_prod(c[r].x, x);
            pr.lo = fma(c[r].x, xl, fma(cl[r].x, x, pr.lo));
            DD u = two_sum(pr.hi, -c[r].y);
            u = quick_two_sum(u.hi, u.lo + (pr.lo - cl[r].y));
            // e(l + 1) = u e(l) - e(l - 1)
            DD q = two_prod(u.hi, ecur);
            q.lo = fma(u.hi, ecl, fma(u.lo, ecur, q.lo));
            DD en = two_sum(q.hi, -eprev);
            en = quick_two_sum(en.hi, en.lo + (q.lo - epl));
            eprev = ecur;
            epl = ecl;
            ecur = en.hi;
            ecl = en.lo;
        }
        if (XR && xs != 1.0 && fabs(ecur) >= 0x1p800) {
            ecur *= kXrUnscale;
            ecl *= kXrUnscale;
            eprev *= kXrUnscale;
            epl *= kXrUnscale;
            xs = 1.0;
        }
        return;
    }
    if constexpr (XR) {
        if (__builtin_amdgcn_ballot_w64(xs != 1.0) != 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                panel_put<PR>(&pan[r * RS], ecur * xs);
                const double u = fma(c[r].x, x, -c[r].y);
                const double en = fma(u, ecur, -eprev);
                eprev = ecur;
                ecur = en;
            }
            if (xs != 1.0 && fabs(ecur) >= 0x1p800) {
                ecur *= kXrUnscale;
                eprev *= kXrUnscale;
                xs = 1.0;
            }
            return;
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        panel_put<PR>(&pan[r * RS], ecur);
        const double u = fma(c[r].x, x, -c[r].y);
        const double en = fma(u, ecur, -eprev);
        eprev = ecur;
        ecur = en;
    }
}

// MFMA output rows: FP64 16x16x4 puts C[lane/16 + 4 r] in register r, FP32
// 16x16x4 puts C[4 (lane/16) + r].
template <int PR>
__device__ __forceinline__ int out_row(int krow, int r) {
    return PR == P64 ? krow + 4 * r : 4 * krow + r;
}

// ---------------------------------------------------------------------------
// Forward DWT: panel x X on MFMA.
// ---------------------------------------------------------------------------
// Beta sample of chunk-local row k (JMap; n = 0: the whole range, k = j).
__device__ __forceinline__ int beta_of(const JMap &jm, int k) {
    return jm.n ? k + (k < jm.split ? jm.off0 : jm.off1) : k;
}

// The panel loop of one forward work item: recurrence, panels, MFMA
// contraction and the fused reorder epilogue.  On entry x, ecur, eprev and
// xs hold each lane's cos b_j, first two recurrence values and seed scale,
// xb the B operand, c the first panel's recurrence coefficients, and srow
// the item's s_l (visible after the first barrier).  flags: kFlagScale
// applies V_B, kFlagAccum adds to the coefficients (the second beta half).
template <int NW, int NSUB, int PR, bool XR, bool DD_>
__device__ __forceinline__ void fwd_item_panels(double (&panel)[NW][16 * kRowFwd], const double *srow,
                                                const WorkItem &it, const double2 *__restrict__ Rr,
                                                const double2 *__restrict__ Rl, double2 (&c)[16],
                                                double2 (&cl)[16], typename PrecT<PR>::R (&xb)[NSUB][16],
                                                double (&x)[NSUB], double (&xl)[NSUB], double (&ecur)[NSUB],
                                                double (&eprev)[NSUB], double (&ecl)[NSUB], double (&epl)[NSUB],
                                                double (&xs)[NSUB], typename PrecT<PR>::C *__restrict__ coeffs,
                                                int flags) {
    using R = typename PrecT<PR>::R;
    const int B = it.B;
    const int m = it.m, mp = it.mp, mask = it.mask;
    const int L = B - m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, krow = lane >> 4;
    double *pan = panel[wave];
    R *out = reinterpret_cast<R *>(coeffs + it.coeff_off);
    const bool apply_v = flags & kFlagScale, accum = flags & kFlagAccum;
    const double v0 = apply_v ? 1.0 / (8.0 * M_PI * (double)B) : 0.0;
    // Epilogue constants: thread slot q writes column t = threadIdx.x + q*NT of
    // every panel; its member, sign and part never change, because the
    // degrees of a panel row advance by 16 (the parity-dependent signs stay).
    constexpr int NT = NW * 64, EPI = (256 + NT - 1) / NT;
    int e_mm[EPI], e_mmp[EPI];
    double e_sign[EPI];
    bool e_on[EPI];
#pragma unroll
    for (int q = 0; q < EPI; ++q) {
        const int t = threadIdx.x + q * NT;
        const int slot = (t & 15) >> 1;
        e_on[q] = t < 256 && ((mask >> slot) & 1);
        group_member(slot, m, mp, m + (t >> 4), e_mm[q], e_mmp[q], e_sign[q]);
    }
    for (int lp = 0; lp < L; lp += 16) {
        double tot[4];
        if constexpr (PR == P64) {
            v4d acc[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int h = 0; h < NSUB; ++h) {
                panel_fill<PR, kRowFwd, XR, DD_>(pan + lane, c, cl, x[h], xl[h], ecur[h], eprev[h], ecl[h], epl[h], xs[h]);
                double a[16];
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    a[s] = pan[col * kRowFwd + 4 * s + krow];
                    // With one subset the compiler pairs these reads into
                    // ds_read2_b64 (offsets 32 bytes apart), whose two halves
                    // meet on the same banks: 2.9 conflict cycles per LDS
                    // instruction (rocprofv3 SQ_LDS_BANK_CONFLICT) and a forward
                    // 5-7 % slower at B = 64 ... 256.  An empty asm with a memory
                    // clobber between them keeps them single ds_read_b64.
                    if constexpr (NSUB == 1) asm volatile("" ::: "memory");
                }
                if (h == NSUB - 1) {
                    lds_wait_all();
#pragma unroll
                    for (int r = 0; r < 16; ++r) c[r] = Rr[lp + 16 + r];
                    if constexpr (DD_) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) cl[r] = Rl[lp + 16 + r];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int s = 0; s < 16; ++s)
                    acc[s & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], xb[h][s], acc[s & 3], 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[r] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
        } else {
            // FP32 head chains of at most two subsets (32 samples), added in FP64
            v4f acc[4], acl[1];  // acl: the split mode's tail products
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[r] = 0.0;
            acl[0] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int h = 0; h < NSUB; ++h) {
                panel_fill<PR, kRowFwd, XR, DD_>(pan + lane, c, cl, x[h], xl[h], ecur[h], eprev[h], ecl[h], epl[h], xs[h]);
                float2 a[16];
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    a[s] = *reinterpret_cast<const float2 *>(&pan[col * kRowFwd + 4 * s + krow]);
                    // single ds_read_b64s with one subset, as in FP64 (split mode:
                    // 4-6 % faster; plain FP32 reads 4 bytes and gains nothing)
                    if constexpr (PR == P32S && NSUB == 1) asm volatile("" ::: "memory");
                }
                if (h == NSUB - 1) {
                    lds_wait_all();
#pragma unroll
                    for (int r = 0; r < 16; ++r) c[r] = Rr[lp + 16 + r];
                    if constexpr (DD_) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) cl[r] = Rl[lp + 16 + r];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int s = 0; s < 16; ++s)
                    acc[s & 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s].x, xb[h][s], acc[s & 3], 0, 0, 0);
                // The tail: four k steps per bf16 MFMA (bf16 element e of the
                // lane is step 4t + e, the sample it feeds at that FP32 step),
                // all into one accumulator.
                if constexpr (PR == P32S) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acl[0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                            bf4(a[4 * t].y, a[4 * t + 1].y, a[4 * t + 2].y, a[4 * t + 3].y),
                            bf4(xb[h][4 * t], xb[h][4 * t + 1], xb[h][4 * t + 2], xb[h][4 * t + 3]), acl[0], 0, 0, 0);
                }
                // the head's chains go to FP64 every two subsets; the tail
                // (about 2^-24 of the value) keeps one chain and joins last
                if (h % 2 == 1 || h == NSUB - 1) {
                    if (h != NSUB - 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double t = PR == P32S && h == NSUB - 1 ? (double)acl[0][r] : 0.0;
#pragma unroll
                        for (int a = 0; a < 4; ++a) t += (double)acc[a][r];
                        tot[r] += t;
                    }
#pragma unroll
                    for (int a = 0; a < 4; ++a) acc[a] = (v4f){0.f, 0.f, 0.f, 0.f};
                    if (h != NSUB - 1) __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        // The wave's panel is free once its A operands are in registers: park
        // the wave's 16 x 16 partial sums there for the cross-wave sum.
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[out_row<PR>(krow, r) * 16 + col] = tot[r];
        lds_sync();
        // Epilogue (the reorder): column c = 2 slot + part of row lp + r is
        // f°(l, member of slot) up to the slot's symmetry sign, s_l and V_B.
#pragma unroll
        for (int q = 0; q < EPI; ++q) {
            const int t = threadIdx.x + q * NT;
            const int li = lp + (t >> 4);
            if (e_on[q] && li < L) {
                double sum = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) sum += panel[w][t];
                const int l = m + li;
                const double f = e_sign[q] * srow[li] * (apply_v ? (2.0 * l + 1.0) * v0 : 1.0);
                R *o = &out[2 * coeff_index64(l, e_mm[q], e_mmp[q]) + (t & 1)];
                *o = accum ? (R)((double)*o + sum * f) : (R)(sum * f);
            }
        }
        // every wave has read the partial sums before any panel is refilled
        lds_sync();
    }
}

// Block = NW waves; wave w owns the j-range [w*NSUB*64, (w+1)*NSUB*64), split
// into NSUB subsets of 64 (one j per lane each).  Panel slot (jl, r) holds the
// recurrence value at degree l0 + lp + r for j-local jl in the wave's own LDS
// region.  Panel rows past the group's last degree hold values of the
// continued recurrence; they only reach output rows that are never written.
// A wave's LDS operations complete in order, so filling and reading its own
// panel needs no block barrier.  Once its A operands are in registers, each
// wave parks its 16 x 16 partial sums in its own panel; one barrier before
// and one after the cross-wave FP64 sum (no separate reduction buffer, which
// keeps four 4-wave blocks within a CU's LDS).  The recurrence
// coefficients of a panel (16 x (alpha, gamma)) sit in scalar registers; the
// next panel's are loaded after this panel's LDS reads, behind the MFMAs.
// Four accumulators keep four MFMA chains in flight (in the FP32 modes each
// covers 16 beta samples; the split mode keeps the lo products apart).
// Lane row k of the launch's beta rows (all 2B, or one beta half of jm) is
// beta sample beta_of(jm, k); XR: extended-range seeds (2B = 2048); DD_: the
// double-double recurrence with the low parts in ddt.
template <int NW, int NSUB, int PR, bool XR, bool DD_>
__global__ __launch_bounds__(NW * 64) void k_dwt_fwd(DwtTables tab, const double2 *__restrict__ rec,
                                                    const WorkItem *__restrict__ items, int nitems,
                                                    const typename PrecT<PR>::C *__restrict__ S,
                                                    typename PrecT<PR>::C *__restrict__ coeffs, int flags, JMap jm,
                                                    DdTables ddt) {
    using C = typename PrecT<PR>::C;
    using R = typename PrecT<PR>::R;
    // s_l of the group's degrees: at most B <= NW*NSUB*64 (a launch in beta
    // halves covers B rows).
    constexpr int SROW = NW * NSUB * 64;
    __shared__ double panel[NW][16 * kRowFwd];
    __shared__ double srow[SROW];
    const WorkItem it = items[item_of_block(blockIdx.x, nitems)];
    const int B = it.B;
    const int N = jm.n ? jm.n : 2 * B;  // beta rows of S (samples past N are zeroed)
    const int m = it.m, mp = it.mp, mask = it.mask;
    const int L = B - m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long goff = it.goff;
    const double2 *__restrict__ Rr = rec + goff;
    const double2 *__restrict__ Rl = DD_ ? ddt.rec_lo + goff : nullptr;

    const C *Sg = S + it.s_off;
    // B operand: X[j][c] with c = 2*slot + (re, im); lane holds row k = lane/16, column lane%16.
    const int col = lane & 15, krow = lane >> 4;
    const bool col_present = (mask >> (col >> 1)) & 1;
    const bool odd = col & 1;

    // Every load of the prologue goes out before any is used, so they are
    // all in flight at once: the recurrence coefficients of the first panel
    // (scalar), the S block (read once: non-temporal loads, about 1 % off the
    // B = 128 step), cos b_j and seeds, and s_l of the lane's row.
    double2 c[16], cl[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = Rr[r];  // the table is padded past the last group
    if constexpr (DD_) {
#pragma unroll
        for (int r = 0; r < 16; ++r) cl[r] = Rl[r];
    }
    // Lanes load whole complex samples: the even lane of a pair (re) that of
    // step s, the odd lane (im) that of step s + 1; one swap of a half between
    // the two lanes later leaves each with its part of both steps.  A load
    // then reads 4 x 2 neighbouring samples, 128 contiguous bytes in FP64, per
    // slot row.  Samples past N load sample 0 and, like absent slots, are
    // zeroed: no branches.
    C raw[NSUB][8];
    double xv[NSUB], xlv[NSUB], sv[NSUB];
#pragma unroll
    for (int h = 0; h < NSUB; ++h) {
        const int jbase = (wave * NSUB + h) * 64;
#pragma unroll
        for (int s = 0; s < 16; s += 2) {
            const int jl = jbase + 4 * s + krow + (odd ? 4 : 0);
            typedef R r2 __attribute__((ext_vector_type(2)));
            const r2 v = __builtin_nontemporal_load(
                reinterpret_cast<const r2 *>(Sg + (size_t)(col >> 1) * N + (jl < N ? jl : 0)));
            raw[h][s / 2].x = v[0];
            raw[h][s / 2].y = v[1];
        }
        const int j = beta_of(jm, jbase + lane < N ? jbase + lane : 0);
        xv[h] = tab.cosb[it.jbase + j];
        if constexpr (DD_) xlv[h] = ddt.cosb_lo[it.jbase + j];
        sv[h] = tab.seed[it.seed_off + j];
    }
    // s_l of the group's rows (L <= B <= SROW, so at most RSN per thread),
    // read in the panel epilogues (visible after the first panel's barrier)
    constexpr int RSN = (SROW + NW * 64 - 1) / (NW * 64);
    double rs[RSN];
#pragma unroll
    for (int q = 0; q < RSN; ++q) rs[q] = tab.rscale[goff + min((int)threadIdx.x + q * NW * 64, L - 1)];
    __builtin_amdgcn_sched_barrier(0);

    R xb[NSUB][16];
    double x[NSUB], ecur[NSUB], eprev[NSUB], xs[NSUB], xl[NSUB], ecl[NSUB], epl[NSUB];
#pragma unroll
    for (int h = 0; h < NSUB; ++h) {
        const int jbase = (wave * NSUB + h) * 64;
#pragma unroll
        for (int s = 0; s < 16; s += 2) {
            const int j0 = jbase + 4 * s + krow, j1 = j0 + 4;
            const C v = raw[h][s / 2];
            const R recv = swap_pair_lanes(odd ? v.x : v.y);
            xb[h][s] = col_present && j0 < N ? (odd ? recv : v.x) : (R)0;
            xb[h][s + 1] = col_present && j1 < N ? (odd ? v.y : recv) : (R)0;
        }
        const bool jin = jbase + lane < N;
        x[h] = jin ? xv[h] : 0.0;
        seed_load(sv[h], jin, ecur[h], xs[h]);
        eprev[h] = 0.0;
        if constexpr (DD_) {
            xl[h] = jin ? xlv[h] : 0.0;
            ecl[h] = 0.0;
            epl[h] = 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < RSN; ++q)
        if ((int)threadIdx.x + q * NW * 64 < L) srow[threadIdx.x + q * NW * 64] = rs[q];
    fwd_item_panels<NW, NSUB, PR, XR, DD_>(panel, srow, it, Rr, Rl, c, cl, xb, x, xl, ecur, eprev, ecl, epl, xs,
                                           coeffs, flags);
}

// ---------------------------------------------------------------------------
// Inverse DWT on MFMA: Y[j][c] = sum_l e(l; b_j) F[l][c].
// ---------------------------------------------------------------------------
// Wave w owns the j-range [w*NSUB*64, (w+1)*NSUB*64) outright, so waves only
// share the staged coefficients.  Every 16 degrees each lane parks its
// recurrence values in the wave's LDS panel; the MFMA A operand is 16 beta
// samples x 4 degrees of it and the B operand 4 degrees x 16 member columns of
// the group's coefficients.  Those are gathered by the whole block straight
// from the l-major layout (the inverse reorder: symmetry sign, s_l and
// optionally V_B applied on the way) into double-buffered LDS chunks of KC
// degrees, issued one chunk ahead; rows past the group's end are zero, so
// panel rows past it (the continued recurrence) contribute nothing.  The
// recurrence coefficients arrive through scalar loads issued after the
// panel's LDS reads.  FP32 modes sum each panel in FP32 and the panels in FP64.
// Degrees per staged chunk: 16 for blocks of up to four waves (a smaller
// stage buffer lets a fourth block share the CU), 32 above.
template <int NW>
constexpr int chunk_of() { return NW <= 4 ? 16 : 32; }

// Thread k-slot q of a block gathers element e = threadIdx.x + q*NT = row*16
// + col of every chunk (degree c*KC + row, column col = 2 slot + part).  Its
// member, sign and part are the same in every chunk (chunks advance the
// degree by KC, an even number, so parity-dependent signs stay), so they are
// set once.  A gather only issues the loads (the coefficient part and s_l, as
// stored); the scaling waits for the staging a chunk later, so the loads of
// chunk c + 1 are in flight while chunk c is contracted.
template <int NT, int KC, typename R>
struct InvGather {
    static constexpr int PER = (KC * 16 + NT - 1) / NT;  // values per thread
    R raw[PER];
    double rs[PER];
    int mm[PER], mmp[PER];
    double sign[PER];
    bool on[PER];
};

template <int NT, int KC, typename R>
__device__ __forceinline__ void inv_gather_init(InvGather<NT, KC, R> &st, const WorkItem &it) {
#pragma unroll
    for (int k = 0; k < InvGather<NT, KC, R>::PER; ++k) {
        const int e = threadIdx.x + k * NT;
        const int slot = (e & 15) >> 1;
        st.on[k] = e < KC * 16 && ((it.mask >> slot) & 1);
        group_member(slot, it.m, it.mp, it.m + (e >> 4), st.mm[k], st.mmp[k], st.sign[k]);
    }
}

// Issue the loads of chunk c (degrees c*KC .. c*KC+KC-1).  Rows past the
// group's last degree load that degree instead (every member has |mm|, |mmp|
// <= m <= l, so each index stays inside the function's coefficients); their
// values are dropped at staging.
template <int NT, int KC, typename R>
__device__ __forceinline__ void inv_gather(InvGather<NT, KC, R> &st, const double *__restrict__ rscale,
                                           const R *__restrict__ cin, const WorkItem &it, int L, int c) {
#pragma unroll
    for (int k = 0; k < InvGather<NT, KC, R>::PER; ++k) {
        const int e = threadIdx.x + k * NT;
        if (e < KC * 16) {
            const int li = min(c * KC + (e >> 4), L - 1);
            st.raw[k] = cin[2 * coeff_index64(it.m + li, st.mm[k], st.mmp[k]) + (e & 1)];
            st.rs[k] = rscale[it.goff + li];
        }
    }
}

// Stage chunk c: the inverse reorder, with the member's sign, s_l and
// optionally V_B applied; absent members and rows past L are zero.  Within
// each 16-degree block, degree d goes to row 4(d%4) + d/4, so the MFMA k slot
// (s, lane/16) that takes degree s + 4(lane/16) reads the contiguous rows
// 4s + lane/16.
template <int NT, int KC, typename R>
__device__ __forceinline__ void inv_put(const InvGather<NT, KC, R> &st, R *buf, const WorkItem &it, int L, int c,
                                        double v0) {
#pragma unroll
    for (int k = 0; k < InvGather<NT, KC, R>::PER; ++k) {
        const int e = threadIdx.x + k * NT;
        const int row = e >> 4;
        const int li = c * KC + row;
        const int prow = (row & ~15) | ((row & 3) << 2) | ((row >> 2) & 3);
        if (e < KC * 16) {
            double val = 0.0;
            if (st.on[k] && li < L) {
                const int l = it.m + li;
                val = (double)st.raw[k] * (st.sign[k] * st.rs[k] * (v0 != 0.0 ? (2.0 * l + 1.0) * v0 : 1.0));
            }
            buf[prow * 16 + (e & 15)] = (R)val;
        }
    }
}

// One 16-degree panel of an inverse work item (degrees lp .. lp+15): the
// recurrence fills the wave's panel and advances, and the panel (A) times
// bop (B, this lane's four coefficient values of the panel) accumulates into
// acc on matrix cores.  Loads the next panel's recurrence coefficients into c.
template <int NW, int NSUB, int PR, bool XR, bool DD_>
__device__ __forceinline__ void inv_panel(double (&panel)[NW][16 * kRowInv], const typename PrecT<PR>::R (&bop)[4],
                                          double2 (&c)[16], double2 (&cl)[16], const double2 *__restrict__ Rr,
                                          const double2 *__restrict__ Rl, int lp, const double (&x)[NSUB],
                                          const double (&xl)[NSUB], double (&ecur)[NSUB], double (&eprev)[NSUB],
                                          double (&ecl)[NSUB], double (&epl)[NSUB], double (&xs)[NSUB],
                                          v4d (&acc)[NSUB][4]) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, krow = lane >> 4;
    double *pan = panel[threadIdx.x >> 6];
    v4bf bopb;
    if constexpr (PR == P32S) bopb = bf4((float)bop[0], (float)bop[1], (float)bop[2], (float)bop[3]);
#pragma unroll
    for (int h = 0; h < NSUB; ++h) {
        panel_fill<PR, kRowInv, XR, DD_>(pan + lane, c, cl, x[h], xl[h], ecur[h], eprev[h], ecl[h], epl[h], xs[h]);
        if constexpr (PR == P64) {
            double a[4][4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    a[t][s] = pan[(s + 4 * krow) * kRowInv + 16 * t + col];
                    // single ds_read_b64s, as in the forward (1-4 % faster with one subset)
                    if constexpr (NSUB == 1) asm volatile("" ::: "memory");
                }
            if (h == NSUB - 1) {
                lds_wait_all();
#pragma unroll
                for (int r = 0; r < 16; ++r) c[r] = Rr[lp + 16 + r];
                if constexpr (DD_) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) cl[r] = Rl[lp + 16 + r];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t][s], bop[s], acc[h][t], 0, 0, 0);
        } else {
            float2 a[4][4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    a[t][s] = *reinterpret_cast<const float2 *>(&pan[(s + 4 * krow) * kRowInv + 16 * t + col]);
                    if constexpr (PR == P32S && NSUB == 1) asm volatile("" ::: "memory");
                }
            if (h == NSUB - 1) {
                lds_wait_all();
#pragma unroll
                for (int r = 0; r < 16; ++r) c[r] = Rr[lp + 16 + r];
                if constexpr (DD_) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) cl[r] = Rl[lp + 16 + r];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                v4f ap = {0.f, 0.f, 0.f, 0.f}, al = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    ap = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][s].x, bop[s], ap, 0, 0, 0);
                // the tail: the panel's four k steps in one bf16 MFMA
                // (element s of the lane is step s, as above)
                if constexpr (PR == P32S)
                    al = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                        bf4(a[t][0].y, a[t][1].y, a[t][2].y, a[t][3].y), bopb, al, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[h][t][r] += (double)ap[r] + (PR == P32S ? (double)al[r] : 0.0);
            }
        }
    }
}

// The end of an inverse work item: acc (Y[j][c] for this wave's beta samples)
// goes through the wave's panel to each slot's row of S, beta contiguous.
template <int NSUB, int PR>
__device__ __forceinline__ void inv_store(double *pan, const v4d (&acc)[NSUB][4], const WorkItem &it,
                                          typename PrecT<PR>::C *__restrict__ S, bool stream, int N) {
    using C = typename PrecT<PR>::C;
    using R = typename PrecT<PR>::R;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, krow = lane >> 4;
    // Register r of lane holds Y[j = 16 t + out_row(krow, r)][c = col] of tile t.
    // Transpose through the wave's panel (pairs (re, im) swizzled by j) and
    // store each slot's beta samples contiguously.
    C *Sg = S + it.s_off;
    const int slot = col >> 1, part = col & 1;
#pragma unroll
    for (int h = 0; h < NSUB; ++h) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jl = 16 * t + out_row<PR>(krow, r);
                pan[jl * 16 + 2 * (slot ^ (jl & 7)) + part] = acc[h][t][r];
            }
        const int j = (wave * NSUB + h) * 64 + lane;
#pragma unroll
        for (int s2 = 0; s2 < kSlots; ++s2) {
            const double2 v = *reinterpret_cast<const double2 *>(pan + lane * 16 + 2 * (s2 ^ (lane & 7)));
            C o;
            o.x = (R)v.x;
            o.y = (R)v.y;
            if (j < N && ((it.mask >> s2) & 1)) put_c(&Sg[(size_t)s2 * N + j], o, stream);
        }
    }
}

template <int NW, int NSUB, int PR, bool XR, bool DD_>
__global__ __launch_bounds__(NW * 64) void k_dwt_inv(DwtTables tab, const double2 *__restrict__ rec,
                                                    const WorkItem *__restrict__ items, int nitems,
                                                    const typename PrecT<PR>::C *__restrict__ coeffs,
                                                    typename PrecT<PR>::C *__restrict__ S, int flags, JMap jm,
                                                    DdTables ddt) {
    using C = typename PrecT<PR>::C;
    using R = typename PrecT<PR>::R;
    constexpr int NT = NW * 64;
    const bool apply_v = flags & kFlagScale, stream = flags & kFlagStream;
    __shared__ double panel[NW][16 * kRowInv];
    constexpr int KC = chunk_of<NW>();
    __shared__ R stage[2][KC * 16];
    const WorkItem it = items[item_of_block(blockIdx.x, nitems)];
    const int B = it.B;
    const int N = jm.n ? jm.n : 2 * B;  // beta rows of S this launch writes
    const int m = it.m, mp = it.mp;
    const int L = B - m;
    const int nchunk = (L + KC - 1) / KC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, krow = lane >> 4;
    const double2 *__restrict__ Rr = rec + it.goff;
    const double2 *__restrict__ Rl = DD_ ? ddt.rec_lo + it.goff : nullptr;
    const R *__restrict__ cin = reinterpret_cast<const R *>(coeffs + it.coeff_off);
    const double v0 = apply_v ? 1.0 / (8.0 * M_PI * (double)B) : 0.0;

    InvGather<NT, KC, R> st;
    inv_gather_init<NT, KC, R>(st, it);
    inv_gather<NT, KC, R>(st, tab.rscale, cin, it, L, 0);

    double x[NSUB], ecur[NSUB], eprev[NSUB], xs[NSUB], xl[NSUB], ecl[NSUB], epl[NSUB];
#pragma unroll
    for (int h = 0; h < NSUB; ++h) {
        const int k = (wave * NSUB + h) * 64 + lane;
        const bool jin = k < N;
        const int j = beta_of(jm, jin ? k : 0);
        const double xv = tab.cosb[it.jbase + j];
        const double sv = tab.seed[it.seed_off + j];
        x[h] = jin ? xv : 0.0;
        seed_load(sv, jin, ecur[h], xs[h]);
        eprev[h] = 0.0;
        if constexpr (DD_) {
            const double xlv = ddt.cosb_lo[it.jbase + j];
            xl[h] = jin ? xlv : 0.0;
            ecl[h] = 0.0;
            epl[h] = 0.0;
        }
    }
    v4d acc[NSUB][4];
#pragma unroll
    for (int h = 0; h < NSUB; ++h)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[h][t] = (v4d){0.0, 0.0, 0.0, 0.0};

    double2 c[16], cl[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = Rr[r];  // the table is padded past the last group
    if constexpr (DD_) {
#pragma unroll
        for (int r = 0; r < 16; ++r) cl[r] = Rl[r];
    }

    inv_put<NT, KC, R>(st, stage[0], it, L, 0, v0);
    if (nchunk > 1) inv_gather<NT, KC, R>(st, tab.rscale, cin, it, L, 1);
    __syncthreads();

    double *pan = panel[wave];
    for (int lp = 0; lp < L; lp += 16) {
        const int ch = lp / KC;
        const R *fb = stage[ch & 1] + (lp - ch * KC) * 16;
        R bop[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) bop[s] = fb[(4 * s + krow) * 16 + col];
        inv_panel<NW, NSUB, PR, XR, DD_>(panel, bop, c, cl, Rr, Rl, lp, x, xl, ecur, eprev, ecl, epl, xs, acc);
        // Chunk boundary: stage the next chunk (its loads were issued a chunk ago).
        if (lp + 16 - ch * KC == KC || lp + 16 >= L) {
            if (ch + 1 < nchunk) {
                inv_put<NT, KC, R>(st, stage[(ch + 1) & 1], it, L, ch + 1, v0);
                if (ch + 2 < nchunk) inv_gather<NT, KC, R>(st, tab.rscale, cin, it, L, ch + 2);
            }
            __syncthreads();
        }
    }

    inv_store<NSUB, PR>(pan, acc, it, S, stream, N);
}

}  // namespace

hipError_t launch_fill_seeds(const PlanView &p, double *seed, hipStream_t s) {
    const long long n = (long long)p.G * p.N;
    hipLaunchKernelGGL(k_fill_seeds, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, seed);
    return hipGetLastError();
}

hipError_t launch_fill_recurrence(const PlanView &p, double2 *rec, double *rscale, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_recurrence, dim3((p.G + 255) / 256), dim3(256), 0, s, p, rec, rscale);
    return hipGetLastError();
}

hipError_t launch_fill_recurrence_dd(const PlanView &p, double2 *rec, double2 *reclo, double *rscale,
                                     hipStream_t s) {
    hipLaunchKernelGGL(k_fill_recurrence_dd, dim3((p.G + 255) / 256), dim3(256), 0, s, p, rec, reclo, rscale);
    return hipGetLastError();
}

// Launch shapes (waves x subsets of 64 beta samples per wave): 1x1, 2x1, 4x1,
// 8x1, 1x2, 2x2, 4x2, 8x2, 16x1, 4x4, 8x4; a shape covers items with beta
// rows (2B, or jm.n) <= waves*subsets*64.  The extended-range (xr) forms
// exist for the shapes that cover a beta half of 2B = 2048 or all of it.
// The double-double recurrence (dd, FP64 only) is built for the shapes
// 1x1, 2x1, 4x1, 8x1, 2x2, 4x2, 8x2, 16x1 and 4x4 (and 4x4, 8x2, 16x1 xr).
template <int PR>
hipError_t launch_dwt_fwd(const DwtTables &tab, const WorkItem *items, int nitems, int nw, int nsub,
                          const typename PrecT<PR>::C *S, typename PrecT<PR>::C *coeffs, bool apply_v,
                          bool accum, const JMap &jm, bool xr, const DdTables *dd, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const int fl = (apply_v ? kFlagScale : 0) | (accum ? kFlagAccum : 0);
    const dim3 grid(nitems);
    const DdTables ddt = dd ? *dd : DdTables{nullptr, nullptr};
#define SOFT_DWT_FWD(NW_, NS_, XR_, DD_)                                                                     \
    if (nw == NW_ && nsub == NS_ && xr == XR_ && (dd != nullptr) == DD_) {                                    \
        hipLaunchKernelGGL((k_dwt_fwd<NW_, NS_, PR, XR_, DD_>), grid, dim3(NW_ * 64), 0, s, tab, tab.rec, items,    \
                           nitems, S, coeffs, fl, jm, ddt);                                                     \
        return hipGetLastError();                                                                             \
    }
    SOFT_DWT_FWD(1, 1, false, false)
    SOFT_DWT_FWD(2, 1, false, false)
    SOFT_DWT_FWD(4, 1, false, false)
    SOFT_DWT_FWD(8, 1, false, false)
    SOFT_DWT_FWD(1, 2, false, false)
    SOFT_DWT_FWD(2, 2, false, false)
    SOFT_DWT_FWD(4, 2, false, false)
    SOFT_DWT_FWD(8, 2, false, false)
    SOFT_DWT_FWD(4, 4, false, false)
    SOFT_DWT_FWD(8, 4, false, false)
    SOFT_DWT_FWD(16, 1, false, false)
    SOFT_DWT_FWD(8, 2, true, false)
    SOFT_DWT_FWD(16, 1, true, false)
    SOFT_DWT_FWD(4, 4, true, false)
    SOFT_DWT_FWD(8, 4, true, false)
    if constexpr (PR == P64) {
        SOFT_DWT_FWD(1, 1, false, true)
        SOFT_DWT_FWD(2, 1, false, true)
        SOFT_DWT_FWD(4, 1, false, true)
        SOFT_DWT_FWD(2, 2, false, true)
        SOFT_DWT_FWD(4, 2, false, true)
        SOFT_DWT_FWD(4, 4, false, true)
        SOFT_DWT_FWD(8, 1, false, true)
        SOFT_DWT_FWD(8, 2, false, true)
        SOFT_DWT_FWD(16, 1, false, true)
        SOFT_DWT_FWD(4, 4, true, true)
        SOFT_DWT_FWD(8, 2, true, true)
        SOFT_DWT_FWD(16, 1, true, true)
    }
#undef SOFT_DWT_FWD
    return hipErrorInvalidValue;
}

template <int PR>
hipError_t launch_dwt_inv(const DwtTables &tab, const WorkItem *items, int nitems, int nw, int nsub,
                          const typename PrecT<PR>::C *coeffs, typename PrecT<PR>::C *S, bool apply_v,
                          bool stream, const JMap &jm, bool xr, const DdTables *dd, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const int fl = (apply_v ? kFlagScale : 0) | (stream ? kFlagStream : 0);
    const dim3 grid(nitems);
    const DdTables ddt = dd ? *dd : DdTables{nullptr, nullptr};
#define SOFT_DWT_INV(NW_, NS_, XR_, DD_)                                                                     \
    if (nw == NW_ && nsub == NS_ && xr == XR_ && (dd != nullptr) == DD_) {                                    \
        hipLaunchKernelGGL((k_dwt_inv<NW_, NS_, PR, XR_, DD_>), grid, dim3(NW_ * 64), 0, s, tab, tab.rec, items,    \
                           nitems, coeffs, S, fl, jm, ddt);                                                     \
        return hipGetLastError();                                                                             \
    }
    SOFT_DWT_INV(1, 1, false, false)
    SOFT_DWT_INV(2, 1, false, false)
    SOFT_DWT_INV(4, 1, false, false)
    SOFT_DWT_INV(8, 1, false, false)
    SOFT_DWT_INV(1, 2, false, false)
    SOFT_DWT_INV(2, 2, false, false)
    SOFT_DWT_INV(4, 2, false, false)
    SOFT_DWT_INV(8, 2, false, false)
    SOFT_DWT_INV(4, 4, false, false)
    SOFT_DWT_INV(8, 4, false, false)
    SOFT_DWT_INV(16, 1, false, false)
    SOFT_DWT_INV(8, 2, true, false)
    SOFT_DWT_INV(16, 1, true, false)
    SOFT_DWT_INV(4, 4, true, false)
    SOFT_DWT_INV(8, 4, true, false)
    if constexpr (PR == P64) {
        SOFT_DWT_INV(1, 1, false, true)
        SOFT_DWT_INV(2, 1, false, true)
        SOFT_DWT_INV(4, 1, false, true)
        SOFT_DWT_INV(2, 2, false, true)
        SOFT_DWT_INV(4, 2, false, true)
        SOFT_DWT_INV(4, 4, false, true)
        SOFT_DWT_INV(8, 1, false, true)
        SOFT_DWT_INV(8, 2, false, true)
        SOFT_DWT_INV(16, 1, false, true)
        SOFT_DWT_INV(4, 4, true, true)
        SOFT_DWT_INV(8, 2, true, true)
        SOFT_DWT_INV(16, 1, true, true)
    }
#undef SOFT_DWT_INV
    return hipErrorInvalidValue;
}

#define SOFT_DWT_INSTANTIATE(PR)                                                                          \
    template hipError_t launch_dwt_fwd<PR>(const DwtTables &, const WorkItem *, int, int, int,               \
                                           const PrecT<PR>::C *, PrecT<PR>::C *, bool, bool, const JMap &,  \
                                           bool, const DdTables *, hipStream_t);                            \
    template hipError_t launch_dwt_inv<PR>(const DwtTables &, const WorkItem *, int, int, int,               \
                                           const PrecT<PR>::C *, PrecT<PR>::C *, bool, bool, const JMap &,  \
                                           bool, const DdTables *, hipStream_t);
SOFT_DWT_INSTANTIATE(P64)
SOFT_DWT_INSTANTIATE(P32)
SOFT_DWT_INSTANTIATE(P32S)

}  // namespace soft
