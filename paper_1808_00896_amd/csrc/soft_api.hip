// soft_api.hip -- plan creation and the C-ABI entry points of include/soft.h.
//
// Plan-time tables are computed on the host in x87 long double and rounded
// once to double (or split into double-double hi/lo pairs where the device
// sums them):
//   w_B(j)                 quadrature weights, eq. "weights"
//   cos(b_j)               recurrence argument, eq. "Wigner_d_recurrence"
//   log cos(b_j/2), log sin(b_j/2), 0.5 log((2m)!/((m+m')!(m-m')!))
//                          seed exponents, Sect. 2.2 "initial cases"
//   e^{+-2 pi i k/2B}      FFT twiddles
//   group / slot tables    symmetry groups of order pairs (Sect. 3)
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "soft_internal.h"

struct soft_plan_s {
    int B = 0, N = 0, batch = 0, G = 0, device = 0;
    long long Nc = 0, rows = 0;
    soft::PlanView view{};
    // device allocations
    void *tables = nullptr;
    double2 *S = nullptr, *t1 = nullptr;
    double2 *rec = nullptr;
    double *rscale = nullptr;
    size_t ws_bytes = 0;
    // stage timing
    struct Pending {
        int stage;
        hipEvent_t start, end;
    };
    bool timing = false;
    std::vector<hipEvent_t> free_events, used_events;
    std::vector<Pending> pending;
    double stage_ms[SOFT_NUM_STAGES] = {};
    long long stage_n[SOFT_NUM_STAGES] = {};
};

namespace {

using soft::GroupInfo;
using soft::kSlots;

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

void free_plan(soft_plan_s *p) {
    if (!p) return;
    for (hipEvent_t e : p->free_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->used_events) (void)hipEventDestroy(e);
    if (p->tables) (void)hipFree(p->tables);
    if (p->S) (void)hipFree(p->S);
    if (p->t1) (void)hipFree(p->t1);
    if (p->rec) (void)hipFree(p->rec);
    if (p->rscale) (void)hipFree(p->rscale);
    delete p;
}

// Byte offsets of the table block, each 256-byte aligned.
struct TableLayout {
    size_t w, cosb, lcs, lbin, grp, goff, slot, twp, twm, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

TableLayout layout_tables(int B, int G) {
    const int N = 2 * B, P = 2 * B - 1;
    TableLayout t{};
    size_t o = 0;
    t.w = o;    o = align256(o + sizeof(double) * N);
    t.cosb = o; o = align256(o + sizeof(double) * N);
    t.lcs = o;  o = align256(o + sizeof(double4) * N);
    t.lbin = o; o = align256(o + sizeof(double2) * G);
    t.grp = o;  o = align256(o + sizeof(GroupInfo) * G);
    t.goff = o; o = align256(o + sizeof(long long) * G);
    t.slot = o; o = align256(o + sizeof(int) * (size_t)P * P);
    t.twp = o;  o = align256(o + sizeof(double2) * N);
    t.twm = o;  o = align256(o + sizeof(double2) * N);
    t.total = o;
    return t;
}

void split_dd(long double x, double &hi, double &lo) {
    hi = (double)x;
    lo = (double)(x - (long double)hi);
}

int build_tables(soft_plan_s *p, std::vector<unsigned char> &host, TableLayout &lay) {
    const int B = p->B, N = p->N, P = 2 * B - 1, G = p->G;
    lay = layout_tables(B, G);
    host.assign(lay.total, 0);
    double *w = reinterpret_cast<double *>(host.data() + lay.w);
    double *cosb = reinterpret_cast<double *>(host.data() + lay.cosb);
    double4 *lcs = reinterpret_cast<double4 *>(host.data() + lay.lcs);
    double2 *lbin = reinterpret_cast<double2 *>(host.data() + lay.lbin);
    GroupInfo *grp = reinterpret_cast<GroupInfo *>(host.data() + lay.grp);
    long long *goff = reinterpret_cast<long long *>(host.data() + lay.goff);
    int *slot = reinterpret_cast<int *>(host.data() + lay.slot);
    double2 *twp = reinterpret_cast<double2 *>(host.data() + lay.twp);
    double2 *twm = reinterpret_cast<double2 *>(host.data() + lay.twm);

    const long double PI = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < N; ++j) {
        const long double beta = (long double)(2 * j + 1) * PI / (long double)(4 * B);
        long double s = 0;
        for (int i = 0; i < B; ++i) s += sinl((long double)(2 * i + 1) * beta) / (long double)(2 * i + 1);
        w[j] = (double)(2.0L * PI * sinl(beta) / ((long double)B * (long double)B) * s);
        cosb[j] = (double)cosl(beta);
        double a, b, c, d;
        split_dd(logl(cosl(beta / 2)), a, b);
        split_dd(logl(sinl(beta / 2)), c, d);
        lcs[j] = make_double4(a, b, c, d);
    }
    for (int k = 0; k < N; ++k) {
        const long double ang = 2.0L * PI * (long double)k / (long double)N;
        const double cr = (double)cosl(ang), si = (double)sinl(ang);
        twp[k] = make_double2(cr, si);
        twm[k] = make_double2(cr, -si);
    }
    for (int i = 0; i < P * P; ++i) slot[i] = -1;
    long long row = 0;
    int g = 0;
    for (int m = 0; m < B; ++m) {
        for (int mp = 0; mp <= m; ++mp, ++g) {
            int mask;
            if (m == 0) mask = 0x01;
            else if (mp == 0) mask = 0x0f;
            else if (mp == m) mask = 0x33;
            else mask = 0xff;
            grp[g] = GroupInfo{m, mp, mask, 0};
            goff[g] = row;
            row += B - m;
            double hi, lo;
            split_dd((lgammal(2.0L * m + 1) - lgammal((long double)(m + mp) + 1) -
                      lgammal((long double)(m - mp) + 1)) / 2,
                     hi, lo);
            lbin[g] = make_double2(hi, lo);
            const int mem[8][2] = {{m, mp}, {-m, -mp}, {mp, m}, {-mp, -m},
                                   {-m, mp}, {m, -mp}, {-mp, m}, {mp, -m}};
            for (int s = 0; s < kSlots; ++s) {
                if (!((mask >> s) & 1)) continue;
                const int idx = (mem[s][0] + B - 1) * P + (mem[s][1] + B - 1);
                if (slot[idx] != -1) return SOFT_ERR_INVALID;  // pair claimed twice
                slot[idx] = (g * kSlots + s) * 2 + (s >= 4 ? 1 : 0);
            }
        }
    }
    for (int i = 0; i < P * P; ++i)  // every pair covered, and by the kernels' slot_code
        if (slot[i] < 0 || slot[i] != soft::slot_code(i / P - (B - 1), i % P - (B - 1))) return SOFT_ERR_INVALID;
    p->rows = row;
    return SOFT_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SOFT_OK : SOFT_ERR_HIP; }

int check_call(soft_plan_t plan, const void *a, const void *b) {
    if (!plan || !a || !b) return SOFT_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SOFT_ERR_HIP;
    if (dev != plan->device) return SOFT_ERR_INVALID;
    return SOFT_OK;
}

// Records one HIP event between consecutive kernels of a call when the plan
// has timing enabled; stage s spans the events around its kernel.
class StageClock {
  public:
    StageClock(soft_plan_s *p, hipStream_t s) : p_(p), s_(s) {}
    hipError_t start() { return p_->timing ? record(&prev_) : hipSuccess; }
    hipError_t lap(int stage) {
        if (!p_->timing) return hipSuccess;
        hipEvent_t e;
        const hipError_t r = record(&e);
        if (r == hipSuccess) p_->pending.push_back({stage, prev_, e});
        prev_ = e;
        return r;
    }

  private:
    hipError_t record(hipEvent_t *out) {
        hipEvent_t e;
        if (!p_->free_events.empty()) {
            e = p_->free_events.back();
            p_->free_events.pop_back();
        } else {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        p_->used_events.push_back(e);
        *out = e;
        return hipEventRecord(e, s_);
    }
    soft_plan_s *p_;
    hipStream_t s_;
    hipEvent_t prev_ = nullptr;
};

// Forward-type transform: FFT (gamma, then alpha with optional W), DWT with
// the reorder (optional V) in its epilogue.  soft_forward uses W and V; soft_adjoint_inverse
// uses neither.
int run_forward(soft_plan_t p, const void *grid, void *coeffs, hipStream_t s, bool scaled) {
    const int rc = check_call(p, grid, coeffs);
    if (rc != SOFT_OK) return rc;
    StageClock clk(p, s);
    hipError_t e = clk.start();
    if (e == hipSuccess) e = soft::launch_fft_gamma_fwd(p->view, p->batch, static_cast<const double2 *>(grid), p->t1, s);
    if (e == hipSuccess) e = clk.lap(SOFT_STAGE_FFT_GAMMA_FWD);
    if (e == hipSuccess) e = soft::launch_fft_alpha_fwd(p->view, p->batch, p->t1, p->S, scaled, s);
    if (e == hipSuccess) e = clk.lap(SOFT_STAGE_FFT_ALPHA_FWD);
    if (e == hipSuccess)
        e = soft::launch_dwt_fwd(p->view, p->batch, p->S, static_cast<double2 *>(coeffs), scaled, s);
    if (e == hipSuccess) e = clk.lap(SOFT_STAGE_DWT_FWD);
    return hip_status(e);
}

// Inverse-type transform: iDWT (gathering the l-major coefficients, optional
// V), FFT (alpha, then gamma with optional W).  soft_inverse uses neither
// factor; soft_adjoint uses both.
int run_inverse(soft_plan_t p, const void *coeffs, void *grid, hipStream_t s, bool scaled) {
    const int rc = check_call(p, coeffs, grid);
    if (rc != SOFT_OK) return rc;
    StageClock clk(p, s);
    hipError_t e = clk.start();
    if (e == hipSuccess)
        e = soft::launch_dwt_inv(p->view, p->batch, static_cast<const double2 *>(coeffs), p->S, scaled, s);
    if (e == hipSuccess) e = clk.lap(SOFT_STAGE_DWT_INV);
    if (e == hipSuccess) e = soft::launch_fft_alpha_inv(p->view, p->batch, p->S, p->t1, s);
    if (e == hipSuccess) e = clk.lap(SOFT_STAGE_FFT_ALPHA_INV);
    if (e == hipSuccess)
        e = soft::launch_fft_gamma_inv(p->view, p->batch, p->t1, static_cast<double2 *>(grid), scaled, s);
    if (e == hipSuccess) e = clk.lap(SOFT_STAGE_FFT_GAMMA_INV);
    return hip_status(e);
}

}  // namespace

extern "C" {

int soft_plan(int B, int batch, int precision, unsigned flags, soft_plan_t *out) {
    if (!out || B < 1 || batch < 1 || flags != 0) return SOFT_ERR_INVALID;
    if (precision != SOFT_FP64) return SOFT_ERR_INVALID;
    if (!is_pow2(B) || B > 512) return SOFT_ERR_UNSUPPORTED;
    soft_plan_s *p = new (std::nothrow) soft_plan_s;
    if (!p) return SOFT_ERR_OOM;
    p->B = B;
    p->N = 2 * B;
    p->batch = batch;
    p->G = B * (B + 1) / 2;
    p->Nc = (long long)B * (4LL * B * B - 1) / 3;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return SOFT_ERR_HIP;
    }
    std::vector<unsigned char> host;
    TableLayout lay;
    int rc = build_tables(p, host, lay);
    if (rc != SOFT_OK) {
        delete p;
        return rc;
    }
    const size_t N = p->N;
    const size_t s_elems = (size_t)batch * p->G * kSlots * N;
    const size_t t1_elems = (size_t)batch * N * N * N;
    const size_t rec_rows = (size_t)p->rows + soft::kPadRows;
    if (hipMalloc(&p->tables, lay.total) != hipSuccess || hipMalloc(&p->S, s_elems * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->t1, t1_elems * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->rec, rec_rows * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->rscale, rec_rows * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        return SOFT_ERR_OOM;
    }
    p->ws_bytes = lay.total + (s_elems + t1_elems) * sizeof(double2) +
                  rec_rows * (sizeof(double2) + sizeof(double));
    if (hipMemcpy(p->tables, host.data(), lay.total, hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p);
        return SOFT_ERR_HIP;
    }
    const unsigned char *base = static_cast<const unsigned char *>(p->tables);
    soft::PlanView &v = p->view;
    v.B = B;
    v.N = p->N;
    v.G = p->G;
    v.Nc = p->Nc;
    v.rows = p->rows;
    v.w = reinterpret_cast<const double *>(base + lay.w);
    v.cosb = reinterpret_cast<const double *>(base + lay.cosb);
    v.lcs = reinterpret_cast<const double4 *>(base + lay.lcs);
    v.lbin = reinterpret_cast<const double2 *>(base + lay.lbin);
    v.grp = reinterpret_cast<const GroupInfo *>(base + lay.grp);
    v.goff = reinterpret_cast<const long long *>(base + lay.goff);
    v.slot = reinterpret_cast<const int *>(base + lay.slot);
    v.twp = reinterpret_cast<const double2 *>(base + lay.twp);
    v.twm = reinterpret_cast<const double2 *>(base + lay.twm);
    v.rec = p->rec;
    v.rscale = p->rscale;
    // Padding rows are read (never used) by prefetches; give them defined values.
    if (hipMemset(p->rec, 0, rec_rows * sizeof(double2)) != hipSuccess ||
        hipMemset(p->rscale, 0, rec_rows * sizeof(double)) != hipSuccess ||
        soft::launch_fill_recurrence(v, p->rec, p->rscale, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        free_plan(p);
        return SOFT_ERR_HIP;
    }
    *out = p;
    return SOFT_OK;
}

int soft_plan_sizes(soft_plan_t p, size_t *grid_elems, size_t *coeff_elems, size_t *workspace_bytes) {
    if (!p) return SOFT_ERR_INVALID;
    if (grid_elems) *grid_elems = (size_t)p->batch * p->N * p->N * p->N;
    if (coeff_elems) *coeff_elems = (size_t)p->batch * p->Nc;
    if (workspace_bytes) *workspace_bytes = p->ws_bytes;
    return SOFT_OK;
}

int soft_forward(soft_plan_t p, const void *grid, void *coeffs, hipStream_t s) {
    return run_forward(p, grid, coeffs, s, true);
}

int soft_adjoint_inverse(soft_plan_t p, const void *grid, void *coeffs, hipStream_t s) {
    return run_forward(p, grid, coeffs, s, false);
}

int soft_inverse(soft_plan_t p, const void *coeffs, void *grid, hipStream_t s) {
    return run_inverse(p, coeffs, grid, s, false);
}

int soft_adjoint(soft_plan_t p, const void *coeffs, void *grid, hipStream_t s) {
    return run_inverse(p, coeffs, grid, s, true);
}

int soft_plan_set_timing(soft_plan_t p, int enable) {
    if (!p) return SOFT_ERR_INVALID;
    p->timing = enable != 0;
    return SOFT_OK;
}

int soft_plan_stage_times(soft_plan_t p, double *ms, long long *launches, int reset) {
    if (!p) return SOFT_ERR_INVALID;
    hipError_t err = hipSuccess;
    for (const auto &r : p->pending) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.end);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.end);
        if (e != hipSuccess) {
            err = e;
            continue;
        }
        p->stage_ms[r.stage] += t;
        p->stage_n[r.stage] += 1;
    }
    p->pending.clear();
    p->free_events.insert(p->free_events.end(), p->used_events.begin(), p->used_events.end());
    p->used_events.clear();
    for (int i = 0; i < SOFT_NUM_STAGES; ++i) {
        if (ms) ms[i] = p->stage_ms[i];
        if (launches) launches[i] = p->stage_n[i];
        if (reset) {
            p->stage_ms[i] = 0.0;
            p->stage_n[i] = 0;
        }
    }
    return hip_status(err);
}

int soft_plan_destroy(soft_plan_t p) {
    if (!p) return SOFT_OK;
    const hipError_t e = hipDeviceSynchronize();
    free_plan(p);
    return hip_status(e);
}

const char *soft_status_string(int status) {
    switch (status) {
        case SOFT_OK: return "ok";
        case SOFT_ERR_INVALID: return "invalid argument";
        case SOFT_ERR_UNSUPPORTED: return "unsupported configuration";
        case SOFT_ERR_OOM: return "out of memory";
        case SOFT_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

}  // extern "C"
