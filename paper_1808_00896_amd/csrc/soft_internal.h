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

// Rows of padding after the last group in the per-row tables and the
// group-major coefficient buffer: the DWT kernels prefetch up to 32 rows past
// a group's end (the values are never used).
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

struct GroupInfo {
    int m, mp;     // representative, m >= mp >= 0; lowest degree l0 = m
    int mask;      // bit s set when slot s is present
    int pad;
};

// Device-side view of a plan, passed by value to kernels.
struct PlanView {
    int B, N, G;
    long long Nc;          // coefficients per function
    long long rows;        // group-major coefficient rows per function (8 complex each)
    const double *w;       // [N]   quadrature weights w_B(j)
    const double *cosb;    // [N]   cos(beta_j)
    const double4 *lcs;    // [N]   (log cos(b_j/2) hi, lo, log sin(b_j/2) hi, lo)
    const double2 *lbin;   // [G]   0.5 log((2m)!/((m+m')!(m-m')!)) as (hi, lo)
    const GroupInfo *grp;  // [G]
    const long long *goff; // [G]   first row of group g in the group-major coefficients
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
hipError_t launch_dwt_fwd(const PlanView &p, int batch, const double2 *S, double2 *Cg, hipStream_t s);
hipError_t launch_dwt_inv(const PlanView &p, int batch, const double2 *Cg, double2 *S, hipStream_t s);

// Group-major <-> l-major coefficient layout, with the symmetry signs and,
// when asked, the (2l+1)/(8 pi B) factor of V_B.
hipError_t launch_reorder_fwd(const PlanView &p, int batch, const double2 *Cg, double2 *coeffs, bool apply_v, hipStream_t s);
hipError_t launch_reorder_inv(const PlanView &p, int batch, const double2 *coeffs, double2 *Cg, bool apply_v, hipStream_t s);

}  // namespace soft
