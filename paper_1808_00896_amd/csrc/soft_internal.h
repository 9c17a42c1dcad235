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

// Device-side view of a plan, passed by value to kernels.
struct PlanView {
    int B, N, G;
    long long Nc;          // coefficients per function
    long long rows;        // group rows (one per group and degree) per function
    const double *w;       // [N]   quadrature weights w_B(j)
    const double *cosb;    // [N]   cos(beta_j)
    const double4 *lcs;    // [N]   (log cos(b_j/2) hi, lo, log sin(b_j/2) hi, lo)
    const double2 *lbin;   // [G]   0.5 log((2m)!/((m+m')!(m-m')!)) as (hi, lo)
    const GroupInfo *grp;  // [G]
    const long long *goff; // [G]   first row of group g in the per-row tables
    const int *slot;       // [(2B-1)^2] (g*8 + s)*2 + (s >= 4), indexed (m+B-1)(2B-1) + (m'+B-1)
    const double2 *rec;    // [rows + kPadRows] rescaled recurrence coefficients (alpha_l, gamma_l)
    const double *rscale;  // [rows + kPadRows] s_l, with d(l) = s_l e(l)
    const double2 *twp;    // [N]   e^{+2 pi i k/N}
    const double2 *twm;    // [N]   e^{-2 pi i k/N}
};

// FFT stage (separation of variables, Sect. 2.4).
hipError_t launch_fft_gamma_fwd(const PlanView &p, int batch, const double2 *grid, double2 *t1, hipStream_t s);
hipError_t launch_fft_alpha_fwd(const PlanView &p, int batch, const double2 *t1, double2 *S, bool apply_w, hipStream_t s);
hipError_t launch_fft_alpha_inv(const PlanView &p, int batch, const double2 *S, double2 *t1, hipStream_t s);
hipError_t launch_fft_gamma_inv(const PlanView &p, int batch, const double2 *t1, double2 *grid, bool apply_w, hipStream_t s);

// Discrete Wigner transform and its transpose (Sect. 2.4 matrix form).
hipError_t launch_fill_recurrence(const PlanView &p, double2 *rec, double *rscale, hipStream_t s);
// Forward DWT with the reorder fused into its epilogue: writes the l-major
// coefficients directly (symmetry signs, s_l and, when apply_v, V_B applied).
hipError_t launch_dwt_fwd(const PlanView &p, int batch, const double2 *S, double2 *coeffs, bool apply_v,
                          hipStream_t s);
// Inverse DWT reading the l-major coefficients directly (the inverse reorder
// is fused into its staging: symmetry signs, s_l and, when apply_v, V_B).
hipError_t launch_dwt_inv(const PlanView &p, int batch, const double2 *coeffs, double2 *S, bool apply_v,
                          hipStream_t s);

}  // namespace soft
