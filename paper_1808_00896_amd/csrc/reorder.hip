// reorder.hip -- group-major <-> l-major coefficients.
//
// The DWT kernels work on group-major rows: row (goff[g] + l - l0) holds the
// eight member columns of symmetry group g at degree l.  The public layout is
// l-major, f°(l,m,m') at l(4l^2-1)/3 + (m+l)(2l+1) + (m'+l).  This pass maps
// between them and applies what the DWT left out:
//   * the symmetry sign of each member (eq. "Wigner_symmetries"),
//   * the scale s_l of the rescaled recurrence (the DWT kernels run
//     e(l) = d(l)/s_l),
//   * the factor (2l+1)/(8 pi B) of V_B (Sect. 2.4) when asked.
// One block per group: reads of the group's rows are contiguous; each
// coefficient is one 16-byte store (forward) or load (inverse).
#include "soft_internal.h"

namespace soft {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ long long coeff_index(int l, int m, int mp) {
    const long long L = l;
    return L * (4 * L * L - 1) / 3 + (long long)(m + l) * (2 * l + 1) + (mp + l);
}

// Member (m, m') of slot s of representative (m0, m0') and its sign at degree l.
__device__ __forceinline__ void member(int s, int m0, int mp0, int l, int &mm, int &mmp, double &sign) {
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

__global__ __launch_bounds__(kThreads) void k_reorder_fwd(PlanView p, const double2 *__restrict__ Cg,
                                                         double2 *__restrict__ coeffs, int apply_v) {
    const int g = blockIdx.x;
    const GroupInfo gi = p.grp[g];
    const int L = p.B - gi.m;
    const double2 *rows = Cg + (size_t)blockIdx.y * p.rows * kSlots + (size_t)p.goff[g] * kSlots;
    double2 *out = coeffs + (size_t)blockIdx.y * p.Nc;
    const double *sl = p.rscale + p.goff[g];
    const double v0 = 1.0 / (8.0 * M_PI * (double)p.B);
    for (int e = threadIdx.x; e < L * kSlots; e += kThreads) {
        const int s = e & (kSlots - 1), li = e >> 3;
        if (!((gi.mask >> s) & 1)) continue;
        const int l = gi.m + li;
        int mm, mmp;
        double sign;
        member(s, gi.m, gi.mp, l, mm, mmp, sign);
        const double f = (apply_v ? sign * (2.0 * l + 1.0) * v0 : sign) * sl[li];
        const double2 v = rows[e];
        out[coeff_index(l, mm, mmp)] = make_double2(v.x * f, v.y * f);
    }
}

__global__ __launch_bounds__(kThreads) void k_reorder_inv(PlanView p, const double2 *__restrict__ coeffs,
                                                         double2 *__restrict__ Cg, int apply_v) {
    const int g = blockIdx.x;
    const GroupInfo gi = p.grp[g];
    const int L = p.B - gi.m;
    double2 *rows = Cg + (size_t)blockIdx.y * p.rows * kSlots + (size_t)p.goff[g] * kSlots;
    const double2 *in = coeffs + (size_t)blockIdx.y * p.Nc;
    const double *sl = p.rscale + p.goff[g];
    const double v0 = 1.0 / (8.0 * M_PI * (double)p.B);
    for (int e = threadIdx.x; e < L * kSlots; e += kThreads) {
        const int s = e & (kSlots - 1), li = e >> 3;
        double2 v = make_double2(0.0, 0.0);
        if ((gi.mask >> s) & 1) {
            const int l = gi.m + li;
            int mm, mmp;
            double sign;
            member(s, gi.m, gi.mp, l, mm, mmp, sign);
            const double f = (apply_v ? sign * (2.0 * l + 1.0) * v0 : sign) * sl[li];
            const double2 c = in[coeff_index(l, mm, mmp)];
            v = make_double2(c.x * f, c.y * f);
        }
        rows[e] = v;
    }
}

}  // namespace

hipError_t launch_reorder_fwd(const PlanView &p, int batch, const double2 *Cg, double2 *coeffs, bool apply_v,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_reorder_fwd, dim3(p.G, batch), dim3(kThreads), 0, s, p, Cg, coeffs, (int)apply_v);
    return hipGetLastError();
}

hipError_t launch_reorder_inv(const PlanView &p, int batch, const double2 *coeffs, double2 *Cg, bool apply_v,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_reorder_inv, dim3(p.G, batch), dim3(kThreads), 0, s, p, coeffs, Cg, (int)apply_v);
    return hipGetLastError();
}

}  // namespace soft
