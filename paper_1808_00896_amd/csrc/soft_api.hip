// soft_api.hip -- plan creation and the C-ABI entry points of include/soft.h.
//
// A plan holds n functions; the functions of one bandwidth form a band.  Per
// band the host computes, in x87 long double rounded once to double (or split
// into double-double hi/lo pairs where the device sums them):
//   w_B(j)                 quadrature weights, eq. "weights"
//   cos(b_j)               recurrence argument, eq. "Wigner_d_recurrence"
//   log cos(b_j/2), log sin(b_j/2), 0.5 log((2m)!/((m+m')!(m-m')!))
//                          seed exponents, Sect. 2.2 "initial cases"
//   e^{+-2 pi i k/2B}      FFT twiddles (FP64 and FP32)
//   group tables           symmetry groups of order pairs (Sect. 3)
// and a plan-time kernel fills the rescaled recurrence table of every band.
// A transform runs the FFT passes band by band, and the DWT as one launch per
// launch shape over a cost-sorted work list of (function, group) items, so
// all bands with 2B <= 256 share a single DWT launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include <unistd.h>

#include "soft_internal.h"

namespace {

using soft::FuncInfo;
using soft::GroupInfo;
using soft::kSlots;
using soft::PlanView;
using soft::WorkItem;

struct Band {
    int B = 0, N = 0, G = 0;
    int chunks = 1;            // beta halves of S (2 at 2B = 2048: soft::JMap)
    int jbase = 0, gbase = 0;  // first entry in the plan-wide beta and group tables
    long long seed_base = 0;   // first entry of the band's G x 2B seeds in the seed table
    long long Nc = 0, rows = 0, row_base = 0;
    std::vector<int> funcs;  // plan function indices, increasing
    size_t tab_off = 0;      // byte offset of the band's tables in the table block
    PlanView view{};         // host copy holding device pointers
};

struct LaunchGroup {
    int nw_f = 1, nsub_f = 1;  // forward DWT launch shape (waves, subsets of 64 beta samples)
    int nw_i = 1, nsub_i = 1;  // inverse DWT launch shape
    int nmax = 0;              // largest 2B among the group's items
    int chunks = 1;            // beta halves its band runs in (soft::JMap)
    int rows = 0;              // beta rows per launch: nmax / chunks (what a shape must cover)
    int nitems = 0;
    bool tuned = false;
    size_t items_off = 0;  // byte offset of the work items in the table block
    std::vector<int> bands;
};

}  // namespace

struct soft_plan_s {
    int precision = 0, n = 0, device = 0;
    unsigned flags = 0;
    bool tune_cached = false;  // SOFT_PLAN_TUNE shapes came from the SOFT_TUNE_CACHE file
    std::vector<Band> bands;
    std::vector<FuncInfo> funcs;
    std::vector<LaunchGroup> groups;
    size_t grid_total = 0, coeff_total = 0, s_total = 0, t1_elems = 0, csize = 16;
    long long rows_total = 0;
    // device allocations
    unsigned char *tables = nullptr;
    void *S = nullptr, *t1 = nullptr;
    double2 *rec = nullptr;
    double2 *rec_lo = nullptr;  // SOFT_DD_RECURRENCE: the recurrence table's low parts
    double *rscale = nullptr;
    double *seed = nullptr;
    long long seed_total = 0;
    soft::DwtTables dtab{};
    soft::DdTables ddtab{};  // read by the DWT launches of SOFT_DD_RECURRENCE plans
    size_t ws_bytes = 0;
    // stage timing
    struct Pending {
        int stage;
        hipEvent_t start, end;
    };
    unsigned timing_mask = 0;  // bit s: time the kernels of stage s
    std::vector<hipEvent_t> free_events, used_events;
    std::vector<Pending> pending;
    double stage_ms[SOFT_NUM_STAGES] = {};
    long long stage_n[SOFT_NUM_STAGES] = {};
    // End of the last call's work, recorded on its stream: destroy waits for
    // it instead of for the whole device.
    hipEvent_t done = nullptr;
    bool done_recorded = false;
    // SOFT_PLAN_GRAPH: per call kind (forward, inverse, adjoint, adjoint
    // inverse) the executable graph of its kernels and the pointers it was
    // captured with; capture runs on a plan-owned stream.
    struct GraphSlot {
        hipGraphExec_t exec = nullptr;
        const void *in = nullptr;
        void *out = nullptr;
    };
    GraphSlot graphs[4];
    hipStream_t capture = nullptr;
};

// Rotational-matching head: n pairs of functions on the sphere at bandwidth
// B, their correlation coefficients, the inverse transform of those (a plan
// of n functions) and the argmax of each correlation grid.
struct soft_match_s {
    int B = 0, n = 0;
    soft_plan_t plan = nullptr;  // owned
    void *coeffs = nullptr;      // n coefficient vectors
    void *part = nullptr;        // argmax partial results
    double *polish = nullptr;    // soft_match_polish: per-pair state and chunk partials
};

namespace {

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Functions per plan: launch grids index the functions of a band (FFT) or
// the pairs (matching head) in a 16-bit grid dimension.
constexpr int kMaxFunctions = 65535;

constexpr unsigned kKnownFlags =
    SOFT_PLAN_TUNE | SOFT_INPLACE_OK | SOFT_PLAN_GRAPH | SOFT_BETA_HALVES | SOFT_DD_RECURRENCE;

bool plan_dd(const soft_plan_s *p) { return (p->flags & SOFT_DD_RECURRENCE) != 0; }
// The DWT launches' double-double tables: null unless the plan runs the recurrence in double-double.
const soft::DdTables *dd_tables(const soft_plan_s *p) { return plan_dd(p) ? &p->ddtab : nullptr; }

void free_plan(soft_plan_s *p) {
    if (!p) return;
    for (hipEvent_t e : p->free_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->used_events) (void)hipEventDestroy(e);
    if (p->done) (void)hipEventDestroy(p->done);
    for (auto &g : p->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (p->capture) (void)hipStreamDestroy(p->capture);
    if (p->tables) (void)hipFree(p->tables);
    if (p->S) (void)hipFree(p->S);
    if (p->t1) (void)hipFree(p->t1);
    if (p->rec) (void)hipFree(p->rec);
    if (p->rec_lo) (void)hipFree(p->rec_lo);
    if (p->rscale) (void)hipFree(p->rscale);
    if (p->seed) (void)hipFree(p->seed);
    delete p;
}

void free_match(soft_match_s *m) {
    if (!m) return;
    if (m->coeffs) (void)hipFree(m->coeffs);
    if (m->part) (void)hipFree(m->part);
    if (m->polish) (void)hipFree(m->polish);
    free_plan(m->plan);
    delete m;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void split_dd(long double x, double &hi, double &lo) {
    hi = (double)x;
    lo = (double)(x - (long double)hi);
}

// Byte offsets of one band's own tables, each 256-byte aligned (its beta
// and log-binomial tables are slices of plan-wide arrays).
struct BandLayout {
    size_t w, grp, goff, twp, twm, twpf, twmf, bfuncs, total;
};

BandLayout band_layout(const Band &b) {
    const size_t N = b.N, G = b.G;
    BandLayout t{};
    size_t o = 0;
    t.w = o;      o = align256(o + sizeof(double) * N);
    t.grp = o;    o = align256(o + sizeof(GroupInfo) * G);
    t.goff = o;   o = align256(o + sizeof(long long) * G);
    t.twp = o;    o = align256(o + sizeof(double2) * N);
    t.twm = o;    o = align256(o + sizeof(double2) * N);
    t.twpf = o;   o = align256(o + sizeof(float2) * N);
    t.twmf = o;   o = align256(o + sizeof(float2) * N);
    t.bfuncs = o; o = align256(o + sizeof(int) * b.funcs.size());
    t.total = o;
    return t;
}

// Symmetry-group mask of representative (m, m'): slots (m,m'), (-m,-m'),
// (m',m), (-m',-m) at beta and (-m,m'), (m,-m'), (-m',m), (m',-m) at pi - beta,
// keeping one slot per distinct pair.
int group_mask(int m, int mp) {
    if (m == 0) return 0x01;
    if (mp == 0) return 0x0f;
    if (mp == m) return 0x33;
    return 0xff;
}

// Fills one band's tables at host address base (laid out by band_layout) and
// its slices cosb[N], cosb_lo[N], lcs[N], lbin[G] of the plan-wide arrays.
int fill_band(const Band &b, const BandLayout &lay, unsigned char *base, double *cosb, double *cosb_lo,
              double4 *lcs, double2 *lbin) {
    const int B = b.B, N = b.N, P = 2 * B - 1;
    double *w = reinterpret_cast<double *>(base + lay.w);
    GroupInfo *grp = reinterpret_cast<GroupInfo *>(base + lay.grp);
    long long *goff = reinterpret_cast<long long *>(base + lay.goff);
    double2 *twp = reinterpret_cast<double2 *>(base + lay.twp);
    double2 *twm = reinterpret_cast<double2 *>(base + lay.twm);
    float2 *twpf = reinterpret_cast<float2 *>(base + lay.twpf);
    float2 *twmf = reinterpret_cast<float2 *>(base + lay.twmf);
    int *bfuncs = reinterpret_cast<int *>(base + lay.bfuncs);

    const long double PI = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < N; ++j) {
        const long double beta = (long double)(2 * j + 1) * PI / (long double)(4 * B);
        long double s = 0;
        for (int i = 0; i < B; ++i) s += sinl((long double)(2 * i + 1) * beta) / (long double)(2 * i + 1);
        w[j] = (double)(2.0L * PI * sinl(beta) / ((long double)B * (long double)B) * s);
        cosb[j] = (double)cosl(beta);
        cosb_lo[j] = (double)(cosl(beta) - (long double)cosb[j]);
        double a, c, d, e;
        split_dd(logl(cosl(beta / 2)), a, c);
        split_dd(logl(sinl(beta / 2)), d, e);
        lcs[j] = make_double4(a, c, d, e);
    }
    for (int k = 0; k < N; ++k) {
        const long double ang = 2.0L * PI * (long double)k / (long double)N;
        const long double cr = cosl(ang), si = sinl(ang);
        twp[k] = make_double2((double)cr, (double)si);
        twm[k] = make_double2((double)cr, (double)-si);
        twpf[k] = make_float2((float)cr, (float)si);
        twmf[k] = make_float2((float)cr, (float)-si);
    }
    std::vector<int> slot((size_t)P * P, -1);
    long long row = b.row_base;
    int g = 0;
    for (int m = 0; m < B; ++m) {
        for (int mp = 0; mp <= m; ++mp, ++g) {
            const int mask = group_mask(m, mp);
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
                const size_t idx = (size_t)(mem[s][0] + B - 1) * P + (mem[s][1] + B - 1);
                if (slot[idx] != -1) return SOFT_ERR_INVALID;  // pair claimed twice
                slot[idx] = (g * kSlots + s) * 2 + (s >= 4 ? 1 : 0);
            }
        }
    }
    // Every pair is covered, and exactly as the kernels' slot_code() says.
    for (size_t i = 0; i < slot.size(); ++i)
        if (slot[i] < 0 || slot[i] != soft::slot_code((int)(i / P) - (B - 1), (int)(i % P) - (B - 1)))
            return SOFT_ERR_INVALID;
    if (row != b.row_base + b.rows) return SOFT_ERR_INVALID;
    for (size_t f = 0; f < b.funcs.size(); ++f) bfuncs[f] = b.funcs[f];
    return SOFT_OK;
}

// Default DWT launch shape (waves per block, subsets of 64 beta samples per
// wave) for N beta rows (2B, or a beta half of 2B = 2048), forward and
// inverse: the fastest shape measured per length on MI355X (SOFT_PLAN_TUNE
// re-measures on the plan itself).
std::pair<int, int> shape_for(int N, bool forward, int precision, bool dd) {
    // the double-double recurrence (more registers per lane): fewer subsets per wave
    if (dd && N == 256) return {2, 2};
    if (dd && N == 1024) return {8, 2};
    if (N <= 32) return {1, 1};
    if (N == 64) return forward ? std::make_pair(1, 1) : std::make_pair(2, 1);
    if (N == 128) return {2, 1};
    if (N == 256) return forward ? std::make_pair(2, 2) : std::make_pair(4, 1);
    if (N == 512) return {4, 2};
    // 2B = 1024: four waves of four subsets, two blocks per CU, except for the
    // FP32 inverses (FP32: 8x2; FP32-split, whose four-subset inverse needs
    // more registers than two blocks leave: 16x1)
    if (forward || precision == SOFT_FP64) return {4, 4};
    return precision == SOFT_FP32 ? std::make_pair(8, 2) : std::make_pair(16, 1);
}

int hip_status(hipError_t e) { return e == hipSuccess ? SOFT_OK : SOFT_ERR_HIP; }

// Marks the end of a call's work on its stream (what soft_plan_destroy waits for).
hipError_t mark_done(soft_plan_s *p, hipStream_t s) {
    const hipError_t e = hipEventRecord(p->done, s);
    p->done_recorded = p->done_recorded || e == hipSuccess;
    return e;
}

// Waits for the last call's work on the plan (a no-op before the first call).
hipError_t wait_done(soft_plan_s *p) { return p->done_recorded ? hipEventSynchronize(p->done) : hipSuccess; }

int check_call(soft_plan_t plan, const void *a, const void *b) {
    if (!plan || !a || !b) return SOFT_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SOFT_ERR_HIP;
    if (dev != plan->device) return SOFT_ERR_INVALID;
    return SOFT_OK;
}

// Records one HIP event between consecutive kernels of a call when the plan
// has timing enabled; each lap is charged to the stage of the kernel before it.
// Stage timer of one call: HIP events on the call's stream around the
// kernels of the stages in the plan's timing mask.  Adjacent timed kernels
// share an event (the end of one is the start of the next).
class StageClock {
  public:
    StageClock(soft_plan_s *p, hipStream_t s) : p_(p), s_(s) {}
    // Before launching a kernel of `stage`: an event marks its start.
    hipError_t before(int stage) {
        if (!on(stage) || have_) return hipSuccess;
        const hipError_t r = record(&prev_);
        have_ = r == hipSuccess;
        return r;
    }
    // After launching it: its end, which also starts a kernel launched next.
    hipError_t after(int stage) {
        if (!on(stage)) {
            have_ = false;
            return hipSuccess;
        }
        hipEvent_t e;
        const hipError_t r = record(&e);
        if (r == hipSuccess) p_->pending.push_back({stage, prev_, e});
        prev_ = e;
        have_ = r == hipSuccess;
        return r;
    }
    // Other work was enqueued since the last event.
    void lose_mark() { have_ = false; }

  private:
    bool on(int stage) const { return (p_->timing_mask >> stage) & 1u; }
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
    bool have_ = false;
};

const WorkItem *items_of(const soft_plan_s *p, const LaunchGroup &lg) {
    return reinterpret_cast<const WorkItem *>(p->tables + lg.items_off);
}

// Forward-type transform: per band the gamma then alpha FFT pass (optional W),
// then the DWT launches, which write the l-major coefficients (optional V).
// soft_forward uses W and V; soft_adjoint_inverse uses neither.  A band in
// beta halves (2B = 2048) runs, after its gamma pass, the alpha pass and the
// DWT once per half; the second half's DWT adds to the first's coefficients.
// Streaming stores (soft::stream_stores) by the bytes a launch writes: a
// band's FFT pass writes nfunc N^3 elements, an inverse-DWT launch 8 slot rows
// of up to 2B samples per item.
template <typename C>
bool band_streams(const Band &b, double from) {
    const double n = b.view.N;
    return soft::stream_stores((double)b.view.nfunc * n * n * n * sizeof(C), b.view.N, from);
}
template <typename C>
bool group_streams(const LaunchGroup &lg) {
    return soft::stream_stores((double)lg.nitems * soft::kSlots * lg.nmax * sizeof(C), lg.nmax, soft::kStreamFrom);
}

// The view of beta half c of a band (its alpha passes read or write S rows of
// that half only), and the DWT row map of a launch group's half c.
PlanView half_view(const Band &b, int c) {
    PlanView v = b.view;
    const soft::JMap m = soft::beta_chunk(b.N, c);
    v.jn = m.n;
    v.jsplit = m.split;
    v.joff0 = m.off0;
    v.joff1 = m.off1;
    return v;
}
soft::JMap group_rows(const LaunchGroup &lg, int c) { return lg.chunks > 1 ? soft::beta_chunk(lg.nmax, c) : soft::JMap{}; }
bool group_xr(const LaunchGroup &lg) { return lg.nmax >= soft::kBetaChunkN; }

template <int PR>
hipError_t run_forward(soft_plan_t p, const void *grid, void *coeffs, hipStream_t s, bool scaled) {
    using C = typename soft::PrecT<PR>::C;
    const C *gin = static_cast<const C *>(grid);
    C *cout_ = static_cast<C *>(coeffs);
    C *t1 = static_cast<C *>(p->t1);
    C *S = static_cast<C *>(p->S);
    StageClock clk(p, s);
    hipError_t e = hipSuccess;
    for (const Band &b : p->bands) {
        if (e == hipSuccess) e = clk.before(SOFT_STAGE_FFT_GAMMA_FWD);
        if (e == hipSuccess) e = soft::launch_fft_gamma_fwd<C>(b.view, gin, t1, band_streams<C>(b, soft::kStreamFrom), s);
        if (e == hipSuccess) e = clk.after(SOFT_STAGE_FFT_GAMMA_FWD);
        if (b.chunks > 1) continue;  // its alpha passes run per beta half below
        if (e == hipSuccess) e = clk.before(SOFT_STAGE_FFT_ALPHA_FWD);
        if (e == hipSuccess) e = soft::launch_fft_alpha_fwd<C>(b.view, t1, gin, S, scaled, band_streams<C>(b, soft::kStreamFromLate), s);
        if (e == hipSuccess) e = clk.after(SOFT_STAGE_FFT_ALPHA_FWD);
    }
    for (const LaunchGroup &lg : p->groups) {
        for (int c = 0; c < lg.chunks; ++c) {
            if (lg.chunks > 1) {
                const Band &b = p->bands[lg.bands[0]];
                if (e == hipSuccess) e = clk.before(SOFT_STAGE_FFT_ALPHA_FWD);
                if (e == hipSuccess)
                    e = soft::launch_fft_alpha_fwd<C>(half_view(b, c), t1, gin, S, scaled,
                                                      band_streams<C>(b, soft::kStreamFromLate), s);
                if (e == hipSuccess) e = clk.after(SOFT_STAGE_FFT_ALPHA_FWD);
            }
            if (e == hipSuccess) e = clk.before(SOFT_STAGE_DWT_FWD);
            if (e == hipSuccess)
                e = lg.nw_f == 0 ? soft::launch_dwt_fwd_clenshaw<PR>(p->dtab, items_of(p, lg), lg.nitems, lg.nmax, S,
                                                                     cout_, scaled, s)
                                 : soft::launch_dwt_fwd<PR>(p->dtab, items_of(p, lg), lg.nitems, lg.nw_f, lg.nsub_f, S,
                                                            cout_, scaled, c > 0, group_rows(lg, c), group_xr(lg),
                                                            dd_tables(p), s);
            if (e == hipSuccess) e = clk.after(SOFT_STAGE_DWT_FWD);
        }
    }
    return e;
}

// Inverse-type transform: the iDWT launches (reading the l-major coefficients,
// optional V), then per band the alpha then gamma FFT pass (optional W).
// soft_inverse uses neither factor; soft_adjoint uses both.  A band in beta
// halves runs the iDWT and its alpha pass once per half, then its gamma pass.
//
// With part (a one-band plan with its own FFT intermediate) the grid is not
// written: the last pass reduces each block's values to argmax partials
// instead (soft::launch_fft_gamma_inv_argmax), and grid may be null.
template <int PR>
hipError_t run_inverse(soft_plan_t p, const void *coeffs, void *grid, hipStream_t s, bool scaled,
                       soft::ArgBest *part = nullptr) {
    using C = typename soft::PrecT<PR>::C;
    const C *cin = static_cast<const C *>(coeffs);
    C *gout = static_cast<C *>(grid);
    C *t1 = static_cast<C *>(p->t1);
    C *S = static_cast<C *>(p->S);
    StageClock clk(p, s);
    hipError_t e = hipSuccess;
    for (const LaunchGroup &lg : p->groups) {
        for (int c = 0; c < lg.chunks; ++c) {
            if (e == hipSuccess) e = clk.before(SOFT_STAGE_DWT_INV);
            if (e == hipSuccess)
                e = lg.nw_i == 0 ? soft::launch_idwt_clenshaw<PR>(p->dtab, items_of(p, lg), lg.nitems, lg.nmax, cin,
                                                                   S, scaled, group_streams<C>(lg), s)
                                 : soft::launch_dwt_inv<PR>(p->dtab, items_of(p, lg), lg.nitems, lg.nw_i, lg.nsub_i,
                                                            cin, S, scaled, group_streams<C>(lg), group_rows(lg, c),
                                                            group_xr(lg), dd_tables(p), s);
            if (e == hipSuccess) e = clk.after(SOFT_STAGE_DWT_INV);
            if (lg.chunks > 1) {
                const Band &b = p->bands[lg.bands[0]];
                if (e == hipSuccess) e = clk.before(SOFT_STAGE_FFT_ALPHA_INV);
                if (e == hipSuccess)
                    e = soft::launch_fft_alpha_inv<C>(half_view(b, c), S, t1, gout,
                                                      band_streams<C>(b, soft::kStreamFromLate), s);
                if (e == hipSuccess) e = clk.after(SOFT_STAGE_FFT_ALPHA_INV);
            }
        }
    }
    for (const Band &b : p->bands) {
        if (b.chunks == 1) {
            if (e == hipSuccess) e = clk.before(SOFT_STAGE_FFT_ALPHA_INV);
            if (e == hipSuccess) e = soft::launch_fft_alpha_inv<C>(b.view, S, t1, gout, band_streams<C>(b, soft::kStreamFromLate), s);
            if (e == hipSuccess) e = clk.after(SOFT_STAGE_FFT_ALPHA_INV);
        }
        if (e == hipSuccess) e = clk.before(SOFT_STAGE_FFT_GAMMA_INV);
        if (e == hipSuccess)
            e = part ? soft::launch_fft_gamma_inv_argmax<C>(b.view, t1, part, s)
                     : soft::launch_fft_gamma_inv<C>(b.view, t1, gout, scaled, band_streams<C>(b, soft::kStreamFromLate), s);
        if (e == hipSuccess) e = clk.after(SOFT_STAGE_FFT_GAMMA_INV);
    }
    return e;
}

// Enqueues the kernels of one call on stream s.
hipError_t enqueue_call(soft_plan_t p, const void *in, void *out, hipStream_t s, bool forward, bool scaled) {
    switch (p->precision) {
        case SOFT_FP64:
            return forward ? run_forward<soft::P64>(p, in, out, s, scaled)
                           : run_inverse<soft::P64>(p, in, out, s, scaled);
        case SOFT_FP32:
            return forward ? run_forward<soft::P32>(p, in, out, s, scaled)
                           : run_inverse<soft::P32>(p, in, out, s, scaled);
        default:
            return forward ? run_forward<soft::P32S>(p, in, out, s, scaled)
                           : run_inverse<soft::P32S>(p, in, out, s, scaled);
    }
}

// SOFT_PLAN_GRAPH: launches the call's graph on s, capturing its kernels on
// the plan's own stream first when the call kind has no graph yet or its
// pointers changed (then the executable graph is updated in place, or made
// anew when the update is refused).  The kernels take their buffers as
// arguments, so a graph is valid only for the pointers it was captured with.
hipError_t graph_call(soft_plan_t p, const void *in, void *out, hipStream_t s, bool forward, bool scaled) {
    soft_plan_s::GraphSlot &g = p->graphs[(forward ? 0 : 1) + (scaled ? 2 : 0)];
    hipError_t e = hipSuccess;
    if (!g.exec || g.in != in || g.out != out) {
        if (!p->capture) e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
        hipGraph_t graph = nullptr;
        if (e == hipSuccess) e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t ek = enqueue_call(p, in, out, p->capture, forward, scaled);
            e = hipStreamEndCapture(p->capture, &graph);
            if (ek != hipSuccess) e = ek;
        }
        if (e == hipSuccess && g.exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult how;
            if (hipGraphExecUpdate(g.exec, graph, &bad, &how) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(g.exec);
                g.exec = nullptr;
            }
        }
        if (e == hipSuccess && !g.exec) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.in = nullptr;
            g.out = nullptr;
            return e;
        }
        g.in = in;
        g.out = out;
    }
    return hipGraphLaunch(g.exec, s);
}

int dispatch(soft_plan_t p, const void *in, void *out, hipStream_t s, bool forward, bool scaled) {
    const int rc = check_call(p, in, out);
    if (rc != SOFT_OK) return rc;
    // stage timing records events between the kernels: such calls run eagerly
    const hipError_t e0 = (p->flags & SOFT_PLAN_GRAPH) && !p->timing_mask
                              ? graph_call(p, in, out, s, forward, scaled)
                              : enqueue_call(p, in, out, s, forward, scaled);
    const hipError_t e = e0 == hipSuccess ? mark_done(p, s) : e0;
    return hip_status(e);
}

template <int PR>
hipError_t run_match(soft_match_s *m, const void *a, const void *b, void *grid, long long *index, hipStream_t s) {
    using C = typename soft::PrecT<PR>::C;
    soft_plan_s *p = m->plan;
    StageClock clk(p, s);
    hipError_t e = clk.before(SOFT_STAGE_MATCH_COEFFS);
    if (e == hipSuccess)
        e = soft::launch_corr_coeffs<C>(m->B, m->n, static_cast<const C *>(a), static_cast<const C *>(b),
                                        static_cast<C *>(m->coeffs), s);
    if (e == hipSuccess) e = clk.after(SOFT_STAGE_MATCH_COEFFS);
    // Without a grid the inverse gamma pass reduces straight to argmax partials.
    soft::ArgBest *fused = grid ? nullptr : static_cast<soft::ArgBest *>(m->part);
    if (e == hipSuccess) e = run_inverse<PR>(p, m->coeffs, grid, s, false, fused);
    clk.lose_mark();
    if (e == hipSuccess) e = clk.before(SOFT_STAGE_ARGMAX);
    if (e == hipSuccess)
        e = fused ? soft::launch_argmax_final(fused, soft::gamma_argmax_blocks(2 * m->B, (int)p->csize), m->n, index, s)
                  : soft::launch_argmax_real<C>(static_cast<const C *>(grid), 8LL * m->B * m->B * m->B, m->n, m->part,
                                                index, s);
    if (e == hipSuccess) e = clk.after(SOFT_STAGE_ARGMAX);
    return e;
}

// DWT launch shapes the library instantiates (waves, subsets of 64 beta
// samples per wave).
constexpr int kDwtShapes[][2] = {{1, 1}, {2, 1}, {4, 1}, {8, 1}, {1, 2}, {2, 2}, {4, 2}, {8, 2}, {16, 1}, {4, 4},
                                 {8, 4}};

// Largest bandwidth of a plan (2B = 2048 beta samples), and of the Clenshaw
// DWT forms (one beta sample per lane, at most 1024 lanes a block).
constexpr int kMaxB = 1024;
constexpr int kMaxClenshawN = 1024;

// The shapes built with the double-double recurrence.
constexpr int kDdShapes[][2] = {{1, 1}, {2, 1}, {4, 1}, {8, 1}, {2, 2}, {4, 2}, {8, 2}, {16, 1}, {4, 4}};

bool known_shape(int waves, int subsets, bool dd) {
    if (dd) {
        for (const auto &sh : kDdShapes)
            if (sh[0] == waves && sh[1] == subsets) return true;
        return false;
    }
    for (const auto &sh : kDwtShapes)
        if (sh[0] == waves && sh[1] == subsets) return true;
    return false;
}

// Autotuner: for every DWT launch group and direction, time each shape that
// covers the group's largest 2B (and is at most twice that), and also the
// Clenshaw kernel of the direction, on the plan's own work list and
// workspace, with zeroed data, and keep the fastest.  Every
// candidate runs once untimed (which also brings the clocks up), then
// kTuneRounds rounds launch each candidate once in turn, each launch between
// two HIP events on the null stream; a candidate's time is its fastest
// launch, so a slow outlier or a clock ramp inside one round decides nothing.
constexpr int kTuneRounds = 5;

template <int PR>
hipError_t tune_dwt_prec(soft_plan_s *p, void *coeffs) {
    using C = typename soft::PrecT<PR>::C;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    C *S = static_cast<C *>(p->S), *cf = static_cast<C *>(coeffs);
    for (LaunchGroup &lg : p->groups) {
        for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
            // candidates (waves, subsets): the matrix-core shapes that cover
            // the launch's beta rows, and the Clenshaw form (0, 0); a band in
            // beta halves is timed on its first half
            std::vector<std::pair<int, int>> cand;
            for (const auto &sh : kDwtShapes) {
                const int cover = sh[0] * sh[1] * 64;
                if (cover >= lg.rows && cover <= 2 * lg.rows && known_shape(sh[0], sh[1], plan_dd(p)))
                    cand.emplace_back(sh[0], sh[1]);
            }
            if (lg.chunks == 1 && lg.nmax <= kMaxClenshawN && !plan_dd(p)) cand.emplace_back(0, 0);
            auto launch = [&](std::pair<int, int> c) {
                if (c.first == 0)
                    return dir == 0 ? soft::launch_dwt_fwd_clenshaw<PR>(p->dtab, items_of(p, lg), lg.nitems, lg.nmax,
                                                                        S, cf, true, 0)
                                    : soft::launch_idwt_clenshaw<PR>(p->dtab, items_of(p, lg), lg.nitems, lg.nmax,
                                                                     cf, S, false, group_streams<C>(lg), 0);
                const int nw = c.first, ns = c.second;
                return dir == 0 ? soft::launch_dwt_fwd<PR>(p->dtab, items_of(p, lg), lg.nitems, nw, ns, S, cf, true,
                                                           false, group_rows(lg, 0), group_xr(lg), dd_tables(p), 0)
                                : soft::launch_dwt_inv<PR>(p->dtab, items_of(p, lg), lg.nitems, nw, ns, cf, S, false,
                                                           group_streams<C>(lg), group_rows(lg, 0), group_xr(lg),
                                                           dd_tables(p), 0);
            };
            std::vector<float> best(cand.size(), 0.f);
            for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) e = launch(cand[i]);
            for (int r = 0; r < kTuneRounds && e == hipSuccess; ++r) {
                for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
                    e = hipEventRecord(t0, 0);
                    if (e == hipSuccess) e = launch(cand[i]);
                    if (e == hipSuccess) e = hipEventRecord(t1, 0);
                    if (e == hipSuccess) e = hipEventSynchronize(t1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                    if (e == hipSuccess && (r == 0 || ms < best[i])) best[i] = ms;
                }
            }
            if (e != hipSuccess || cand.empty()) continue;
            size_t bi = 0;
            for (size_t i = 1; i < cand.size(); ++i)
                if (best[i] < best[bi]) bi = i;
            (dir == 0 ? lg.nw_f : lg.nw_i) = cand[bi].first;
            (dir == 0 ? lg.nsub_f : lg.nsub_i) = cand[bi].second;
        }
        lg.tuned = e == hipSuccess;
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    return e;
}

// Autotune cache (SOFT_TUNE_CACHE names a file): the launch shapes a tuned
// plan chose, keyed by the device architecture, the precision (with "_dd"
// for the double-double recurrence), whether the plan runs beta halves, and
// its bandwidths with their function counts.  The file is a JSON object with
// one entry per line,
//   "gfx950|fp64|whole|128x1": [[4, 1, 4, 1]],
// one [forward waves, subsets, inverse waves, subsets] per DWT launch in
// plan order.  A plan whose key is present, with one valid shape per launch,
// takes those shapes instead of timing; otherwise it tunes and writes its
// entry (the file is rewritten whole: through a temporary file and a
// rename, so readers never see a partial one).  Lines that do not parse are
// dropped on that rewrite.  Plans made at the same time in several
// processes may each tune and the last rename wins; every entry stays valid.
std::mutex g_tune_cache_mu;

std::string tune_cache_key(const soft_plan_s *p) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    static const char *const prec[] = {"fp64", "fp32", "fp32_split"};
    std::string k = arch + "|" + prec[p->precision] + (plan_dd(p) ? "_dd" : "") + "|" +
                    ((p->flags & SOFT_BETA_HALVES) ? "halves" : "whole") + "|";
    for (size_t bi = 0; bi < p->bands.size(); ++bi)
        k += (bi ? "," : "") + std::to_string(p->bands[bi].B) + "x" + std::to_string(p->bands[bi].funcs.size());
    return k;
}

// Entries of a cache file: key -> flat list of shape numbers (4 per launch).
std::map<std::string, std::vector<int>> read_tune_cache(const char *path) {
    std::map<std::string, std::vector<int>> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"'), q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        const size_t colon = line.find(':', q1);
        if (colon == std::string::npos) continue;
        std::vector<int> nums;
        bool ok = true;
        for (size_t i = colon + 1; i < line.size() && ok;) {
            const char ch = line[i];
            if (ch >= '0' && ch <= '9') {
                long v = 0;
                while (i < line.size() && line[i] >= '0' && line[i] <= '9' && v < 100000) v = v * 10 + (line[i++] - '0');
                nums.push_back((int)v);
            } else {
                ok = ch == '[' || ch == ']' || ch == ',' || ch == ' ';
                ++i;
            }
        }
        if (ok && !nums.empty() && nums.size() % 4 == 0) out[line.substr(q0 + 1, q1 - q0 - 1)] = nums;
    }
    return out;
}

bool write_tune_cache(const char *path, const std::map<std::string, std::vector<int>> &entries) {
    static int serial = 0;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid()) + "." + std::to_string(++serial);
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : entries) {
            f << "\"" << kv.first << "\": [";
            for (size_t s = 0; s < kv.second.size(); s += 4)
                f << (s ? ", " : "") << "[" << kv.second[s] << ", " << kv.second[s + 1] << ", " << kv.second[s + 2]
                  << ", " << kv.second[s + 3] << "]";
            f << "]" << (++i < entries.size() ? "," : "") << "\n";
        }
        f << "}\n";
        if (!f) return false;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

// A launch shape from the cache is usable for a launch group when it is
// built and covers the group (or is a Clenshaw form the group allows).
bool cached_shape_ok(const LaunchGroup &lg, int waves, int subsets, bool dd) {
    if (waves == 0 && subsets == 0) return !dd && lg.chunks == 1 && lg.nmax <= 1024;
    return known_shape(waves, subsets, dd) && waves * subsets * 64 >= lg.rows;
}

// Applies the cached shapes of p, if its key is in the file; true on a hit.
bool tune_from_cache(soft_plan_s *p, const char *path) {
    std::lock_guard<std::mutex> lock(g_tune_cache_mu);
    const auto entries = read_tune_cache(path);
    const auto it = entries.find(tune_cache_key(p));
    if (it == entries.end() || it->second.size() != 4 * p->groups.size()) return false;
    const std::vector<int> &v = it->second;
    for (size_t gi = 0; gi < p->groups.size(); ++gi)
        if (!cached_shape_ok(p->groups[gi], v[4 * gi], v[4 * gi + 1], plan_dd(p)) ||
            !cached_shape_ok(p->groups[gi], v[4 * gi + 2], v[4 * gi + 3], plan_dd(p)))
            return false;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        LaunchGroup &lg = p->groups[gi];
        lg.nw_f = v[4 * gi];
        lg.nsub_f = v[4 * gi + 1];
        lg.nw_i = v[4 * gi + 2];
        lg.nsub_i = v[4 * gi + 3];
        lg.tuned = true;
    }
    return true;
}

void tune_to_cache(const soft_plan_s *p, const char *path) {
    std::lock_guard<std::mutex> lock(g_tune_cache_mu);
    auto entries = read_tune_cache(path);
    std::vector<int> &v = entries[tune_cache_key(p)];
    v.clear();
    for (const LaunchGroup &lg : p->groups) {
        v.push_back(lg.nw_f);
        v.push_back(lg.nsub_f);
        v.push_back(lg.nw_i);
        v.push_back(lg.nsub_i);
    }
    (void)write_tune_cache(path, entries);  // a cache that cannot be written only costs the next plan a tuning
}

int tune_dwt(soft_plan_s *p) {
    void *coeffs = nullptr;
    if (hipMalloc(&coeffs, p->coeff_total * p->csize) != hipSuccess) {
        (void)hipGetLastError();
        return SOFT_ERR_OOM;
    }
    hipError_t e = hipMemset(coeffs, 0, p->coeff_total * p->csize);
    if (e == hipSuccess) e = hipMemset(p->S, 0, p->s_total * p->csize);
    if (e == hipSuccess) {
        switch (p->precision) {
            case SOFT_FP64: e = tune_dwt_prec<soft::P64>(p, coeffs); break;
            case SOFT_FP32: e = tune_dwt_prec<soft::P32>(p, coeffs); break;
            default: e = tune_dwt_prec<soft::P32S>(p, coeffs); break;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    (void)hipFree(coeffs);
    return hip_status(e);
}

bool valid_precision(int precision) {
    return precision == SOFT_FP64 || precision == SOFT_FP32 || precision == SOFT_FP32_SPLIT;
}

// Known flags, and SOFT_DD_RECURRENCE only with FP64.
bool valid_flags(unsigned flags, int precision) {
    return !(flags & ~kKnownFlags) && (!(flags & SOFT_DD_RECURRENCE) || precision == SOFT_FP64);
}

// Host side of a plan: its tables, function table and DWT work lists in
// one block laid out as on the device, plus the offsets of its parts.
struct HostTables {
    std::vector<unsigned char> host;
    size_t funcs_off = 0, cosb_off = 0, cosb_lo_off = 0, lcs_off = 0, lbin_off = 0, total = 0;
    std::vector<BandLayout> lays;
    std::vector<std::vector<WorkItem>> lists;
};

// Builds bands, the function table and the DWT work lists of a plan for the
// bandwidths Bs[0..n) (validated by the caller) into p and ht, without
// touching a device.
int build_host(soft_plan_s *p, const int *Bs, int n, int precision, unsigned flags, HostTables &ht) {
    // Bands in increasing B; functions keep the caller's order.
    std::vector<int> distinct(Bs, Bs + n);
    std::sort(distinct.begin(), distinct.end());
    distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
    int jtot = 0, gtot = 0;
    for (int B : distinct) {
        Band b;
        b.B = B;
        b.N = 2 * B;
        b.G = B * (B + 1) / 2;
        // Beta halves: always at 2B = 2048; on request from 2B = 128 (a half's
        // quarter-range segments then hold whole FFT tiles).
        b.chunks = b.N == soft::kBetaChunkN || ((flags & SOFT_BETA_HALVES) && b.N >= 128) ? 2 : 1;
        b.jbase = jtot;
        b.gbase = gtot;
        b.seed_base = p->seed_total;
        p->seed_total += (long long)b.G * b.N;
        jtot += b.N;
        gtot += b.G;
        b.Nc = (long long)B * (4LL * B * B - 1) / 3;
        for (int m = 0; m < B; ++m) b.rows += (long long)(m + 1) * (B - m);
        b.row_base = p->rows_total;
        p->rows_total += b.rows;
        p->bands.push_back(b);
    }
    p->funcs.resize(n);
    for (int f = 0; f < n; ++f) {
        const int bi = (int)(std::lower_bound(distinct.begin(), distinct.end(), Bs[f]) - distinct.begin());
        Band &b = p->bands[bi];
        FuncInfo &fi = p->funcs[f];
        fi.band = bi;
        fi.pad = 0;
        fi.grid_off = (long long)p->grid_total;
        fi.coeff_off = (long long)p->coeff_total;
        fi.s_off = (long long)p->s_total;
        p->grid_total += (size_t)b.N * b.N * b.N;
        p->coeff_total += (size_t)b.Nc;
        p->s_total += (size_t)b.G * kSlots * (b.N / b.chunks);
        b.funcs.push_back(f);
    }
    // The tile-blocked FFT intermediate; a SOFT_INPLACE_OK plan has none
    // and stages the intermediate in the grid buffer instead.
    if (!(flags & SOFT_INPLACE_OK))
        for (const Band &b : p->bands)
            p->t1_elems = std::max(p->t1_elems, b.funcs.size() * (size_t)b.N * b.N * b.N);

    // DWT launch groups: in a plan of several bands, the bands with
    // 2B <= 64 share one launch (with the 2B = 64 shapes); every other
    // length has its own (sharing one launch down from 2B = 256 left the
    // lanes of the shorter bands idle: 2-3 % slower on the 256-function
    // batch of B = 16 ... 128).
    const bool merged = p->bands.size() > 1;
    std::vector<int> keys;  // 0 for the shared launch, else 2B
    std::vector<std::vector<int>> group_bands;
    for (size_t bi = 0; bi < p->bands.size(); ++bi) {
        const int key = merged && p->bands[bi].N <= 64 ? 0 : p->bands[bi].N;
        size_t gi = std::find(keys.begin(), keys.end(), key) - keys.begin();
        if (gi == keys.size()) {
            keys.push_back(key);
            group_bands.emplace_back();
        }
        group_bands[gi].push_back((int)bi);
    }
    // Per band and group g (ordered by m, then m'): m and the first row.
    std::vector<std::vector<int>> gm(p->bands.size());
    std::vector<std::vector<long long>> grow(p->bands.size());
    for (size_t bi = 0; bi < p->bands.size(); ++bi) {
        const Band &b = p->bands[bi];
        long long row = b.row_base;
        for (int m = 0; m < b.B; ++m)
            for (int mp = 0; mp <= m; ++mp) {
                gm[bi].push_back(m);
                grow[bi].push_back(row);
                row += b.B - m;
            }
    }
    // Work lists: runs of 8 consecutive groups of one function (the XCD
    // remap hands each run to one XCD), ordered by the cost (B - m) 2B of
    // their first group, largest first, so the long recurrences start
    // early and the short ones fill the tail.
    std::vector<std::vector<WorkItem>> &lists = ht.lists;
    lists.assign(keys.size(), {});
    for (size_t gi = 0; gi < keys.size(); ++gi) {
        struct Run {
            long long cost;
            int band, func, g0, g1;
        };
        std::vector<Run> runs;
        for (int bi : group_bands[gi]) {
            const Band &b = p->bands[bi];
            for (int f : b.funcs)
                for (int g0 = 0; g0 < b.G; g0 += 8)
                    runs.push_back({(long long)(b.B - gm[bi][g0]) * b.N, bi, f, g0, std::min(b.G, g0 + 8)});
        }
        std::stable_sort(runs.begin(), runs.end(), [](const Run &a, const Run &c) { return a.cost > c.cost; });
        for (const Run &r : runs) {
            const Band &b = p->bands[r.band];
            const FuncInfo &fi = p->funcs[r.func];
            for (int g = r.g0; g < r.g1; ++g) {
                const int m = gm[r.band][g], mp = g - m * (m + 1) / 2;
                WorkItem w{};
                w.goff = grow[r.band][g];
                w.s_off = fi.s_off + (long long)g * kSlots * (b.N / b.chunks);
                w.coeff_off = fi.coeff_off;
                w.B = b.B;
                w.jbase = b.jbase;
                w.seed_off = b.seed_base + (long long)g * b.N;
                w.m = m;
                w.mp = mp;
                w.mask = group_mask(m, mp);
                lists[gi].push_back(w);
            }
        }
        if (lists[gi].size() > (size_t)0x7fffffff) return SOFT_ERR_UNSUPPORTED;
        LaunchGroup lg;
        lg.bands = group_bands[gi];
        for (int bi : group_bands[gi]) {
            lg.nmax = std::max(lg.nmax, p->bands[bi].N);
            lg.chunks = std::max(lg.chunks, p->bands[bi].chunks);  // a band in halves has its own launch
        }
        lg.rows = lg.nmax / lg.chunks;
        const int len = keys[gi] ? lg.rows : 64;
        std::tie(lg.nw_f, lg.nsub_f) = shape_for(len, true, precision, plan_dd(p));
        std::tie(lg.nw_i, lg.nsub_i) = shape_for(len, false, precision, plan_dd(p));
        lg.nitems = (int)lists[gi].size();
        p->groups.push_back(lg);
    }

    // Table block: band tables, function table, band views, work lists.
    size_t off = 0;
    std::vector<BandLayout> &lays = ht.lays;
    for (Band &b : p->bands) {
        b.tab_off = off;
        lays.push_back(band_layout(b));
        off = align256(off + lays.back().total);
    }
    const size_t funcs_off = ht.funcs_off = off;
    off = align256(off + sizeof(FuncInfo) * n);
    const size_t cosb_off = ht.cosb_off = off;
    off = align256(off + sizeof(double) * jtot);
    const size_t cosb_lo_off = ht.cosb_lo_off = off;
    off = align256(off + sizeof(double) * jtot);
    const size_t lcs_off = ht.lcs_off = off;
    off = align256(off + sizeof(double4) * jtot);
    const size_t lbin_off = ht.lbin_off = off;
    off = align256(off + sizeof(double2) * gtot);
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        p->groups[gi].items_off = off;
        off = align256(off + sizeof(WorkItem) * lists[gi].size());
    }
    const size_t total = ht.total = off;
    std::vector<unsigned char> &host = ht.host;
    host.assign(total, 0);
    double *cosb_h = reinterpret_cast<double *>(host.data() + cosb_off);
    double *cosb_lo_h = reinterpret_cast<double *>(host.data() + cosb_lo_off);
    double4 *lcs_h = reinterpret_cast<double4 *>(host.data() + lcs_off);
    double2 *lbin_h = reinterpret_cast<double2 *>(host.data() + lbin_off);
    for (size_t bi = 0; bi < p->bands.size(); ++bi) {
        const Band &b = p->bands[bi];
        const int rc = fill_band(b, lays[bi], host.data() + b.tab_off, cosb_h + b.jbase, cosb_lo_h + b.jbase,
                                 lcs_h + b.jbase, lbin_h + b.gbase);
        if (rc != SOFT_OK) return rc;
    }
    std::memcpy(host.data() + funcs_off, p->funcs.data(), sizeof(FuncInfo) * n);
    for (size_t gi = 0; gi < p->groups.size(); ++gi)
        std::memcpy(host.data() + p->groups[gi].items_off, lists[gi].data(), sizeof(WorkItem) * lists[gi].size());
    return SOFT_OK;
}

// Checks a plan's host tables: every (function, symmetry group) appears in
// exactly one work item, each item's offsets lie inside its function's S
// block, coefficient vector, seed and recurrence rows, and every launch
// shape covers its launch.  (fill_band has checked that the groups' member
// slots cover every order pair exactly once.)
int check_host(const soft_plan_s *p, const HostTables &ht) {
    std::vector<std::vector<unsigned char>> seen(p->n);
    for (int f = 0; f < p->n; ++f) seen[f].assign(p->bands[p->funcs[f].band].G, 0);
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const LaunchGroup &lg = p->groups[gi];
        if ((size_t)lg.nitems != ht.lists[gi].size()) return SOFT_ERR_INVALID;
        if ((lg.nw_f && lg.nw_f * lg.nsub_f * 64 < lg.rows) || (lg.nw_i && lg.nw_i * lg.nsub_i * 64 < lg.rows))
            return SOFT_ERR_INVALID;
        if (!known_shape(lg.nw_f, lg.nsub_f, plan_dd(p)) || !known_shape(lg.nw_i, lg.nsub_i, plan_dd(p)))
            return SOFT_ERR_INVALID;  // every default shape is a built one
        if (lg.chunks > 1 && (lg.bands.size() != 1 || p->bands[lg.bands[0]].chunks != lg.chunks))
            return SOFT_ERR_INVALID;
        for (const WorkItem &w : ht.lists[gi]) {
            int f = -1;
            for (int q = 0; q < p->n && f < 0; ++q)
                if (p->funcs[q].coeff_off == w.coeff_off) f = q;
            if (f < 0) return SOFT_ERR_INVALID;
            const Band &b = p->bands[p->funcs[f].band];
            const long long N = b.N;
            if (w.B != b.B || w.jbase != b.jbase || w.m < 0 || w.m >= b.B || w.mp < 0 || w.mp > w.m)
                return SOFT_ERR_INVALID;
            const int g = w.m * (w.m + 1) / 2 + w.mp;
            if (seen[f][g]++) return SOFT_ERR_INVALID;
            if (w.mask != group_mask(w.m, w.mp) || b.N > lg.nmax) return SOFT_ERR_INVALID;
            const long long NS = N / b.chunks;  // S rows per slot
            if (w.s_off != p->funcs[f].s_off + (long long)g * kSlots * NS || w.s_off + kSlots * NS > (long long)p->s_total)
                return SOFT_ERR_INVALID;
            if (w.seed_off != b.seed_base + (long long)g * N || w.seed_off + N > p->seed_total) return SOFT_ERR_INVALID;
            if (w.goff < b.row_base || w.goff + (b.B - w.m) > b.row_base + b.rows) return SOFT_ERR_INVALID;
            if (w.coeff_off + b.Nc > (long long)p->coeff_total) return SOFT_ERR_INVALID;
        }
    }
    for (int f = 0; f < p->n; ++f)
        for (unsigned char c : seen[f])
            if (c != 1) return SOFT_ERR_INVALID;
    if (ht.host.size() != ht.total) return SOFT_ERR_INVALID;
    return SOFT_OK;
}

int make_plan(const int *Bs, int n, int precision, unsigned flags, soft_plan_t *out) {
    soft_plan_s *p = new (std::nothrow) soft_plan_s;
    if (!p) return SOFT_ERR_OOM;
    try {
        p->precision = precision;
        p->n = n;
        p->flags = flags;
        p->csize = precision == SOFT_FP64 ? sizeof(double2) : sizeof(float2);
        if (hipGetDevice(&p->device) != hipSuccess) {
            delete p;
            return SOFT_ERR_HIP;
        }
        HostTables ht;
        const int rc = build_host(p, Bs, n, precision, flags, ht);
        if (rc != SOFT_OK) {
            delete p;
            return rc;
        }
        const size_t total = ht.total;
        const std::vector<unsigned char> &host = ht.host;
        const size_t funcs_off = ht.funcs_off, cosb_off = ht.cosb_off, cosb_lo_off = ht.cosb_lo_off,
                     lcs_off = ht.lcs_off, lbin_off = ht.lbin_off;
        const std::vector<BandLayout> &lays = ht.lays;

        const size_t rec_rows = (size_t)p->rows_total + soft::kPadRows;
        if (hipMalloc(&p->tables, total) != hipSuccess || hipMalloc(&p->S, p->s_total * p->csize) != hipSuccess ||
            (p->t1_elems && hipMalloc(&p->t1, p->t1_elems * p->csize) != hipSuccess) ||
            hipMalloc(&p->rec, rec_rows * sizeof(double2)) != hipSuccess ||
            (plan_dd(p) && hipMalloc(&p->rec_lo, rec_rows * sizeof(double2)) != hipSuccess) ||
            hipMalloc(&p->rscale, rec_rows * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->seed, p->seed_total * sizeof(double)) != hipSuccess ||
            hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            free_plan(p);
            return SOFT_ERR_OOM;
        }
        p->ws_bytes = total + (p->s_total + p->t1_elems) * p->csize +
                      rec_rows * ((plan_dd(p) ? 2 : 1) * sizeof(double2) + sizeof(double)) +
                      p->seed_total * sizeof(double);

        // Band views with device pointers (kernel arguments of the FFT passes
        // and of the recurrence fill), and the DWT kernels' plan-wide tables.
        const double *cosb_d = reinterpret_cast<const double *>(p->tables + cosb_off);
        const double4 *lcs_d = reinterpret_cast<const double4 *>(p->tables + lcs_off);
        const double2 *lbin_d = reinterpret_cast<const double2 *>(p->tables + lbin_off);
        const double *cosb_lo_d = reinterpret_cast<const double *>(p->tables + cosb_lo_off);
        p->dtab = soft::DwtTables{cosb_d, p->seed, p->rscale, p->rec};
        p->ddtab = soft::DdTables{cosb_lo_d, p->rec_lo};
        for (size_t bi = 0; bi < p->bands.size(); ++bi) {
            Band &b = p->bands[bi];
            const BandLayout &lay = lays[bi];
            const unsigned char *base = p->tables + b.tab_off;
            PlanView &v = b.view;
            v.B = b.B;
            v.N = b.N;
            v.G = b.G;
            v.nfunc = (int)b.funcs.size();
            v.Nc = b.Nc;
            v.rows = b.rows;
            v.w = reinterpret_cast<const double *>(base + lay.w);
            v.cosb = cosb_d + b.jbase;
            v.lcs = lcs_d + b.jbase;
            v.lbin = lbin_d + b.gbase;
            v.grp = reinterpret_cast<const GroupInfo *>(base + lay.grp);
            v.goff = reinterpret_cast<const long long *>(base + lay.goff);
            v.twp = reinterpret_cast<const double2 *>(base + lay.twp);
            v.twm = reinterpret_cast<const double2 *>(base + lay.twm);
            v.twpf = reinterpret_cast<const float2 *>(base + lay.twpf);
            v.twmf = reinterpret_cast<const float2 *>(base + lay.twmf);
            v.rscale = p->rscale;
            v.funcs = reinterpret_cast<const FuncInfo *>(p->tables + funcs_off);
            v.band_funcs = reinterpret_cast<const int *>(base + lay.bfuncs);
            v.jn = b.N;  // all beta rows (half_view() narrows a band in halves)
            v.jsplit = b.N;
            v.joff0 = 0;
            v.joff1 = 0;
        }

        hipError_t e = hipMemcpy(p->tables, host.data(), total, hipMemcpyHostToDevice);
        // Padding rows are read (never used) by prefetches; give them defined values.
        if (e == hipSuccess) e = hipMemset(p->rec, 0, rec_rows * sizeof(double2));
        if (e == hipSuccess && p->rec_lo) e = hipMemset(p->rec_lo, 0, rec_rows * sizeof(double2));
        if (e == hipSuccess) e = hipMemset(p->rscale, 0, rec_rows * sizeof(double));
        for (const Band &b : p->bands) {
            if (e == hipSuccess)
                e = plan_dd(p) ? soft::launch_fill_recurrence_dd(b.view, p->rec, p->rec_lo, p->rscale, 0)
                               : soft::launch_fill_recurrence(b.view, p->rec, p->rscale, 0);
            if (e == hipSuccess) e = soft::launch_fill_seeds(b.view, p->seed + b.seed_base, 0);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e == hipSuccess && (flags & SOFT_PLAN_TUNE)) {
            const char *cache = std::getenv("SOFT_TUNE_CACHE");
            if (cache && *cache && tune_from_cache(p, cache)) {
                p->tune_cached = true;
            } else {
                const int rc = tune_dwt(p);
                if (rc != SOFT_OK) {
                    free_plan(p);
                    return rc;
                }
                if (cache && *cache) tune_to_cache(p, cache);
            }
        }
        if (e != hipSuccess) {
            free_plan(p);
            return SOFT_ERR_HIP;
        }
    } catch (const std::bad_alloc &) {
        free_plan(p);
        return SOFT_ERR_OOM;
    }
    *out = p;
    return SOFT_OK;
}

// Allocation-free argmax: its partial results live in this file-scope device
// array (1 MiB on every GPU the library runs on, held until the process ends)
// instead of a plan's buffer.  argmax_blocks() deals about 4096 blocks over all
// grids and at least one per grid, so n <= kArgmaxScratchEntries grids always
// fit.  In host code `scratch` only names the symbol: kernels get its device
// address, looked up once per device with that device current.
constexpr int kArgmaxScratchEntries = 65536;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) soft::ArgBest scratch[kArgmaxScratchEntries];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device).
int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SOFT_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return SOFT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return SOFT_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SOFT_OK;
}

}  // namespace

extern "C" {

int soft_plan(int B, int batch, int precision, unsigned flags, soft_plan_t *out) {
    if (!out || B < 1 || batch < 1 || !valid_precision(precision) || !valid_flags(flags, precision)) return SOFT_ERR_INVALID;
    if (!is_pow2(B) || B > kMaxB || batch > kMaxFunctions) return SOFT_ERR_UNSUPPORTED;
    std::vector<int> Bs;
    try {
        Bs.assign(batch, B);
    } catch (const std::bad_alloc &) {
        return SOFT_ERR_OOM;
    }
    return make_plan(Bs.data(), batch, precision, flags, out);
}

int soft_plan_uneven(const int *B_list, int n, int precision, unsigned flags, soft_plan_t *out) {
    if (!out || !B_list || n < 1 || !valid_precision(precision) || !valid_flags(flags, precision)) return SOFT_ERR_INVALID;
    for (int i = 0; i < n; ++i)
        if (B_list[i] < 1) return SOFT_ERR_INVALID;
    if (n > kMaxFunctions) return SOFT_ERR_UNSUPPORTED;
    for (int i = 0; i < n; ++i)
        if (!is_pow2(B_list[i]) || B_list[i] > kMaxB) return SOFT_ERR_UNSUPPORTED;
    return make_plan(B_list, n, precision, flags, out);
}

int soft_plan_check(const int *B_list, int n, int precision, unsigned flags) {
    if (!B_list || n < 1 || !valid_precision(precision) || !valid_flags(flags, precision)) return SOFT_ERR_INVALID;
    for (int i = 0; i < n; ++i)
        if (B_list[i] < 1) return SOFT_ERR_INVALID;
    if (n > kMaxFunctions) return SOFT_ERR_UNSUPPORTED;
    for (int i = 0; i < n; ++i)
        if (!is_pow2(B_list[i]) || B_list[i] > kMaxB) return SOFT_ERR_UNSUPPORTED;
    soft_plan_s *p = new (std::nothrow) soft_plan_s;
    if (!p) return SOFT_ERR_OOM;
    int rc;
    try {
        p->precision = precision;
        p->n = n;
        p->flags = flags;
        p->csize = precision == SOFT_FP64 ? sizeof(double2) : sizeof(float2);
        HostTables ht;
        rc = build_host(p, B_list, n, precision, flags, ht);
        if (rc == SOFT_OK) rc = check_host(p, ht);
    } catch (const std::bad_alloc &) {
        rc = SOFT_ERR_OOM;
    }
    delete p;
    return rc;
}

int soft_plan_sizes(soft_plan_t p, size_t *grid_elems, size_t *coeff_elems, size_t *workspace_bytes) {
    if (!p) return SOFT_ERR_INVALID;
    if (grid_elems) *grid_elems = p->grid_total;
    if (coeff_elems) *coeff_elems = p->coeff_total;
    if (workspace_bytes) *workspace_bytes = p->ws_bytes;
    return SOFT_OK;
}

int soft_plan_describe(soft_plan_t p, char *buf, size_t len) {
    if (!p || !buf || len == 0) return SOFT_ERR_INVALID;
    std::string d = "{\"precision\": " + std::to_string(p->precision) + ", \"functions\": " + std::to_string(p->n) +
                    ", \"workspace_bytes\": " + std::to_string(p->ws_bytes) +
                    ", \"inplace_ok\": " + ((p->flags & SOFT_INPLACE_OK) ? "true" : "false") +
                    ", \"dd_recurrence\": " + (plan_dd(p) ? "true" : "false") +
                    ", \"tuned_from_cache\": " + (p->tune_cached ? "true" : "false") + ", \"bands\": [";
    for (size_t bi = 0; bi < p->bands.size(); ++bi)
        d += std::string(bi ? ", " : "") + "{\"B\": " + std::to_string(p->bands[bi].B) +
             ", \"functions\": " + std::to_string(p->bands[bi].funcs.size()) + "}";
    d += "], \"dwt_launches\": [";
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const LaunchGroup &lg = p->groups[gi];
        d += std::string(gi ? ", " : "") + "{\"max_2B\": " + std::to_string(lg.nmax) +
             ", \"beta_halves\": " + std::to_string(lg.chunks) + ", \"items\": " + std::to_string(lg.nitems) +
             ", \"forward\": [" + std::to_string(lg.nw_f) + ", " +
             std::to_string(lg.nsub_f) + "], \"inverse\": [" + std::to_string(lg.nw_i) + ", " +
             std::to_string(lg.nsub_i) + "], \"tuned\": " + (lg.tuned ? "true" : "false") + "}";
    }
    d += "]}";
    const size_t k = std::min(len - 1, d.size());
    std::memcpy(buf, d.data(), k);
    buf[k] = '\0';
    return SOFT_OK;
}

int soft_plan_set_dwt_shape(soft_plan_t p, int launch, int direction, int waves, int subsets) {
    if (!p || launch < 0 || launch >= (int)p->groups.size() || (direction != 0 && direction != 1))
        return SOFT_ERR_INVALID;
    LaunchGroup &lg = p->groups[launch];
    if (waves == 0 && subsets == 0) {  // the Clenshaw forms
        if (lg.nmax > kMaxClenshawN || plan_dd(p)) return SOFT_ERR_INVALID;
        (direction == 0 ? lg.nw_f : lg.nw_i) = 0;
        (direction == 0 ? lg.nsub_f : lg.nsub_i) = 0;
        return SOFT_OK;
    }
    if (!known_shape(waves, subsets, plan_dd(p)) || waves * subsets * 64 < lg.rows) return SOFT_ERR_INVALID;
    (direction == 0 ? lg.nw_f : lg.nw_i) = waves;
    (direction == 0 ? lg.nsub_f : lg.nsub_i) = subsets;
    return SOFT_OK;
}

int soft_plan_offsets(soft_plan_t p, size_t *grid_offsets, size_t *coeff_offsets) {
    if (!p) return SOFT_ERR_INVALID;
    for (int f = 0; f < p->n; ++f) {
        if (grid_offsets) grid_offsets[f] = (size_t)p->funcs[f].grid_off;
        if (coeff_offsets) coeff_offsets[f] = (size_t)p->funcs[f].coeff_off;
    }
    if (grid_offsets) grid_offsets[p->n] = p->grid_total;
    if (coeff_offsets) coeff_offsets[p->n] = p->coeff_total;
    return SOFT_OK;
}

int soft_forward(soft_plan_t p, const void *grid, void *coeffs, hipStream_t s) {
    return dispatch(p, grid, coeffs, s, true, true);
}

int soft_adjoint_inverse(soft_plan_t p, const void *grid, void *coeffs, hipStream_t s) {
    return dispatch(p, grid, coeffs, s, true, false);
}

int soft_inverse(soft_plan_t p, const void *coeffs, void *grid, hipStream_t s) {
    return dispatch(p, coeffs, grid, s, false, false);
}

int soft_adjoint(soft_plan_t p, const void *coeffs, void *grid, hipStream_t s) {
    return dispatch(p, coeffs, grid, s, false, true);
}

int soft_plan_set_timing(soft_plan_t p, int enable) {
    if (!p) return SOFT_ERR_INVALID;
    p->timing_mask = enable ? (1u << SOFT_NUM_STAGES) - 1u : 0u;
    return SOFT_OK;
}

int soft_plan_set_timing_stages(soft_plan_t p, unsigned mask) {
    if (!p || (mask >> SOFT_NUM_STAGES)) return SOFT_ERR_INVALID;
    p->timing_mask = mask;
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
    const hipError_t e = wait_done(p);
    free_plan(p);
    return hip_status(e);
}

int soft_match_plan(int B, int n, int precision, unsigned flags, soft_match_t *out) {
    if (!out || B < 1 || n < 1 || !valid_precision(precision) || !valid_flags(flags, precision)) return SOFT_ERR_INVALID;
    if (!is_pow2(B) || B > 512 || n > kMaxFunctions) return SOFT_ERR_UNSUPPORTED;
    soft_match_s *m = new (std::nothrow) soft_match_s;
    if (!m) return SOFT_ERR_OOM;
    m->B = B;
    m->n = n;
    int rc = soft_plan(B, n, precision, flags, &m->plan);
    if (rc != SOFT_OK) {
        delete m;
        return rc;
    }
    const long long N3 = 8LL * B * B * B;
    // argmax partials: of the grid scan, or of the inverse gamma pass fused with it
    const size_t part_bytes = std::max(soft::argmax_workspace_bytes(N3, n),
                                       sizeof(soft::ArgBest) * (size_t)n *
                                           (size_t)soft::gamma_argmax_blocks(2 * B, (int)m->plan->csize));
    if (hipMalloc(&m->coeffs, m->plan->coeff_total * m->plan->csize) != hipSuccess ||
        hipMalloc(&m->part, part_bytes) != hipSuccess ||
        hipMalloc(&m->polish, soft::polish_workspace_bytes(B * (B + 1) / 2, n)) != hipSuccess) {
        (void)hipGetLastError();
        free_match(m);
        return SOFT_ERR_OOM;
    }
    *out = m;
    return SOFT_OK;
}

int soft_match_sizes(soft_match_t m, size_t *sh_elems, size_t *coeff_elems, size_t *grid_elems) {
    if (!m) return SOFT_ERR_INVALID;
    if (sh_elems) *sh_elems = (size_t)m->n * m->B * m->B;
    return soft_plan_sizes(m->plan, grid_elems, coeff_elems, nullptr);
}

int soft_match_plan_soft(soft_match_t m, soft_plan_t *plan) {
    if (!m || !plan) return SOFT_ERR_INVALID;
    *plan = m->plan;
    return SOFT_OK;
}

int soft_match_coeffs(soft_match_t m, const void *a, const void *b, void *coeffs, hipStream_t s) {
    if (!m || !b) return SOFT_ERR_INVALID;
    const int rc = check_call(m->plan, a, coeffs);
    if (rc != SOFT_OK) return rc;
    hipError_t e;
    if (m->plan->precision == SOFT_FP64)
        e = soft::launch_corr_coeffs<double2>(m->B, m->n, static_cast<const double2 *>(a),
                                              static_cast<const double2 *>(b), static_cast<double2 *>(coeffs), s);
    else
        e = soft::launch_corr_coeffs<float2>(m->B, m->n, static_cast<const float2 *>(a),
                                             static_cast<const float2 *>(b), static_cast<float2 *>(coeffs), s);
    return hip_status(e);
}

int soft_match_coeffs_vjp(soft_match_t m, const void *a, const void *b, const void *gcoeffs, void *ga, void *gb,
                          hipStream_t s) {
    if (!m || !b || !gcoeffs || !gb) return SOFT_ERR_INVALID;
    const int rc = check_call(m->plan, a, ga);
    if (rc != SOFT_OK) return rc;
    hipError_t e;
    if (m->plan->precision == SOFT_FP64)
        e = soft::launch_corr_vjp<double2>(m->B, m->n, static_cast<const double2 *>(a),
                                           static_cast<const double2 *>(b), static_cast<const double2 *>(gcoeffs),
                                           static_cast<double2 *>(ga), static_cast<double2 *>(gb), s);
    else
        e = soft::launch_corr_vjp<float2>(m->B, m->n, static_cast<const float2 *>(a), static_cast<const float2 *>(b),
                                          static_cast<const float2 *>(gcoeffs), static_cast<float2 *>(ga),
                                          static_cast<float2 *>(gb), s);
    return hip_status(e);
}

int soft_match_argmax(soft_match_t m, const void *grid, long long *index, hipStream_t s) {
    if (!m) return SOFT_ERR_INVALID;
    const int rc = check_call(m->plan, grid, index);
    if (rc != SOFT_OK) return rc;
    const long long N3 = 8LL * m->B * m->B * m->B;
    hipError_t e;
    if (m->plan->precision == SOFT_FP64)
        e = soft::launch_argmax_real<double2>(static_cast<const double2 *>(grid), N3, m->n, m->part, index, s);
    else
        e = soft::launch_argmax_real<float2>(static_cast<const float2 *>(grid), N3, m->n, m->part, index, s);
    if (e == hipSuccess) e = mark_done(m->plan, s);
    return hip_status(e);
}

int soft_match_argmax_noalloc(int B, int n, int precision, const void *grid, long long *index, hipStream_t s) {
    if (B < 1 || n < 1 || !grid || !index || !valid_precision(precision)) return SOFT_ERR_INVALID;
    if (!is_pow2(B) || B > 512 || n > kMaxFunctions) return SOFT_ERR_UNSUPPORTED;
    const long long N3 = 8LL * B * B * B;
    if (soft::argmax_workspace_bytes(N3, n) > sizeof(soft::ArgBest) * (size_t)kArgmaxScratchEntries)
        return SOFT_ERR_UNSUPPORTED;
    void *part = nullptr;
    const int rc = scratch_address(&part);
    if (rc != SOFT_OK) return rc;
    hipError_t e;
    if (precision == SOFT_FP64)
        e = soft::launch_argmax_real<double2>(static_cast<const double2 *>(grid), N3, n, part, index, s);
    else
        e = soft::launch_argmax_real<float2>(static_cast<const float2 *>(grid), N3, n, part, index, s);
    return hip_status(e);
}

int soft_match(soft_match_t m, const void *a, const void *b, void *grid, long long *index, hipStream_t s) {
    if (!m || !a || !b) return SOFT_ERR_INVALID;
    // no grid: the argmax is fused into the last FFT pass, which needs the
    // plan's own FFT intermediate
    if (!grid && !m->plan->t1) return SOFT_ERR_INVALID;
    const int rc = check_call(m->plan, grid ? grid : index, index);
    if (rc != SOFT_OK) return rc;
    hipError_t e;
    switch (m->plan->precision) {
        case SOFT_FP64: e = run_match<soft::P64>(m, a, b, grid, index, s); break;
        case SOFT_FP32: e = run_match<soft::P32>(m, a, b, grid, index, s); break;
        default: e = run_match<soft::P32S>(m, a, b, grid, index, s); break;
    }
    if (e == hipSuccess) e = mark_done(m->plan, s);
    return hip_status(e);
}

int soft_sh_forward(int B, int n, int precision, const void *f, void *a, hipStream_t s) {
    if (B < 1 || n < 1 || !f || !a || !valid_precision(precision)) return SOFT_ERR_INVALID;
    if (!is_pow2(B) || B > 512 || n > kMaxFunctions) return SOFT_ERR_UNSUPPORTED;
    const hipError_t e =
        precision == SOFT_FP64
            ? soft::launch_sh_forward<double2>(B, n, static_cast<const double2 *>(f), static_cast<double2 *>(a), s)
            : soft::launch_sh_forward<float2>(B, n, static_cast<const float2 *>(f), static_cast<float2 *>(a), s);
    return hip_status(e);
}

int soft_match_polish(soft_match_t m, const void *coeffs, const double *start, int iters, double *angles,
                      double *value, hipStream_t s) {
    if (!m || !coeffs || !start || !angles || !value || iters < 0 || iters > 64) return SOFT_ERR_INVALID;
    const int rc = check_call(m->plan, coeffs, angles);
    if (rc != SOFT_OK) return rc;
    const soft_plan_s *p = m->plan;
    const PlanView &v = p->bands[0].view;
    const hipError_t e =
        p->precision == SOFT_FP64
            ? soft::launch_corr_polish<double2>(v, p->rec, p->rscale, m->n, static_cast<const double2 *>(coeffs),
                                                start, iters, angles, value, m->polish, s)
            : soft::launch_corr_polish<float2>(v, p->rec, p->rscale, m->n, static_cast<const float2 *>(coeffs),
                                               start, iters, angles, value, m->polish, s);
    return hip_status(e);
}

int soft_match_refine(soft_match_t m, const void *grid, const long long *index, double *angles, hipStream_t s) {
    if (!m || !grid || !index || !angles) return SOFT_ERR_INVALID;
    const int rc = check_call(m->plan, grid, angles);
    if (rc != SOFT_OK) return rc;
    const hipError_t e =
        m->plan->precision == SOFT_FP64
            ? soft::launch_match_refine<double2>(m->B, m->n, static_cast<const double2 *>(grid), index, angles, s)
            : soft::launch_match_refine<float2>(m->B, m->n, static_cast<const float2 *>(grid), index, angles, s);
    return hip_status(e);
}

int soft_match_destroy(soft_match_t m) {
    if (!m) return SOFT_OK;
    const hipError_t e = wait_done(m->plan);
    free_match(m);
    return hip_status(e);
}

int soft_probe_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    if (!src || !dst || bytes == 0 || bytes % 16 != 0) return SOFT_ERR_INVALID;
    return hip_status(soft::launch_probe_copy(src, dst, (long long)(bytes / 16), s));
}

int soft_probe_flops(int kind, int blocks, int iters, double *sink, hipStream_t s) {
    if (kind < 0 || kind > 2 || blocks < 1 || iters < 1 || !sink) return SOFT_ERR_INVALID;
    return hip_status(soft::launch_probe_flops(kind, blocks, iters, sink, s));
}

double soft_probe_flop_count(int kind, int blocks, int iters) {
    if (kind < 0 || kind > 2 || blocks < 1 || iters < 1) return 0.0;
    return soft::probe_flop_count(kind, blocks, iters);
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
