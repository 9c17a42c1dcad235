/*
 * soft.h -- C-ABI of the MI355X (gfx950) fast Fourier transform on SO(3).
 *
 * The transform pair is Kostelec and Rockmore's FSOFT / iFSOFT as reviewed in
 * Sect. 2 of Lux, Wuelker, Chirikjian, "Parallelization of the FFT on SO(3)":
 *
 *   forward (FSOFT, eq. "quadrature"):
 *     f°(l,m,m') = (2l+1)/(8 pi B) sum_{i,j,k<2B} w_B(j) f(a_i,b_j,g_k)
 *                  * conj(D(l,m,m'; a_i,b_j,g_k))
 *   inverse (iFSOFT, eq. "fourier_representation" on the grid):
 *     f(a_i,b_j,g_k) = sum_{l<B} sum_{|m|,|m'|<=l} f°(l,m,m') D(l,m,m'; a_i,b_j,g_k)
 *
 * with D(l,m,m';a,b,g) = e^{-i m a} d(l,m,m';b) e^{-i m' g} (eq. "Wigner_D"),
 * d as defined by the explicit Jacobi form of Sect. 2.2, sampling angles
 * a_i = i pi/B, b_j = (2j+1) pi/(4B), g_k = k pi/B and weights w_B(j) of eq.
 * "weights".  Both directions run as the separation of variables of Sect.
 * 2.4: a 2-D FFT per beta sample plus the discrete Wigner transform (DWT,
 * V_B T_B W_B) or its transpose (iDWT, T_B^T) per order pair (m, m').
 *
 * Data layout (device memory, owned by the caller):
 *   grid    complex, [2B][2B][2B] row-major, index ((i*2B + j)*2B + k) for
 *           f(a_i, b_j, g_k)  (k fastest).
 *   coeffs  complex, B(4B^2-1)/3 entries (the count of Sect. 2.4), f°(l,m,m')
 *           at index l(4l^2-1)/3 + (m+l)(2l+1) + (m'+l), 0 <= l < B,
 *           -l <= m, m' <= l.
 *   complex numbers are interleaved (re, im): double2 for SOFT_FP64,
 *   float2 for SOFT_FP32 and SOFT_FP32_SPLIT.
 *   A plan for n functions (one bandwidth with soft_plan, mixed bandwidths
 *   with soft_plan_uneven) expects the n grids back to back, and the n
 *   coefficient vectors back to back, in the order the functions were given;
 *   soft_plan_offsets() returns where each one starts.
 *
 * Streams: every transform call is stream-ordered and asynchronous; it
 * enqueues kernels on `stream` and returns.  No call synchronises the device
 * or copies to the host after plan creation.  A plan owns device workspace,
 * so calls that use the same plan must not overlap in time (two streams, or
 * two host threads): serialise them on one stream.  Distinct plans are
 * independent.
 *
 * Errors: functions return SOFT_OK (0) or a negative soft_status.  Argument
 * errors are detected before anything is enqueued and leave the outputs
 * untouched.  SOFT_ERR_HIP reports a failed HIP call or kernel launch; a
 * fault inside a running kernel surfaces at the caller's next
 * synchronisation, as with any HIP work.
 */
#ifndef SOFT_H
#define SOFT_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct soft_plan_s *soft_plan_t;

/*
 * Arithmetic of a plan.  The recurrence for d (eq. "Wigner_d_recurrence"),
 * its seeds and the quadrature weights are FP64 in every mode; the modes
 * differ in the storage of grids, coefficients and intermediates and in the
 * arithmetic of the FFT and of the DWT contraction (the matrix products of
 * Sect. 2.4).
 *   SOFT_FP64        complex128 data; FP64 FFT and FP64 matrix-core DWT.
 *   SOFT_FP32        complex64 data; FP32 FFT; the DWT contracts FP32 data
 *                    with d rounded to FP32 on FP32 matrix cores and adds
 *                    the FP32 partial sums (at most 32 beta samples in the
 *                    forward, 16 degrees in the inverse) in FP64.
 *   SOFT_FP32_SPLIT  as SOFT_FP32, but d is split into an FP32 head and an
 *                    FP32 tail (d = hi + lo to about 2^-48 relative); the
 *                    head is contracted on FP32 matrix cores and the tail
 *                    (about 2^-24 of d) on bf16 matrix cores, which keeps d
 *                    to about 2^-32 relative, so the DWT error is that of
 *                    FP32 data rather than of FP32 d; relative error about
 *                    1e-6 or below at B <= 1024 for data of unit scale.
 */
typedef enum {
    SOFT_FP64 = 0,
    SOFT_FP32 = 1,
    SOFT_FP32_SPLIT = 2
} soft_precision;

/*
 * Plan flags (bitwise or).
 *   SOFT_PLAN_TUNE  at plan time, time every DWT launch shape (waves per
 *                   block, beta samples per lane) that fits each DWT launch,
 *                   forward and inverse separately, and also the Clenshaw
 *                   form of each direction (see soft_plan_set_dwt_shape), on the
 *                   plan's own work list with zeroed data, and keep the
 *                   fastest.  Costs a few
 *                   DWT launches per candidate at plan creation; without it
 *                   a fixed shape per 2B, direction and precision is used.
 *                   When the environment variable SOFT_TUNE_CACHE names a
 *                   file, a plan whose key (device architecture, precision
 *                   and recurrence, beta halves or not, bandwidths with their function
 *                   counts) is in it takes the stored shapes instead of
 *                   timing, and a plan that times writes its entry there
 *                   (a JSON object, one entry per line, rewritten whole
 *                   through a temporary file and a rename).
 *   SOFT_INPLACE_OK the plan may use the grid buffers as scratch, and holds
 *                   no FFT intermediate of its own (that saves (2B)^3 complex
 *                   elements per function of the largest band: 16 GiB at
 *                   B = 512 in FP64).  soft_forward and soft_adjoint_inverse
 *                   then overwrite their input grid (its contents are
 *                   unspecified after the call); soft_inverse and
 *                   soft_adjoint stage in their output grid.  Results are
 *                   bit-identical to a plan without the flag; the FFT passes
 *                   move shorter runs and are somewhat slower.
 *   SOFT_PLAN_GRAPH each transform call (soft_forward, soft_inverse,
 *                   soft_adjoint, soft_adjoint_inverse) launches a HIP graph
 *                   of its kernels, captured on a plan-owned stream at the
 *                   first call of that kind and captured again (the
 *                   executable graph updated) when the call's input or output
 *                   pointer differs from the last capture; a replay with the
 *                   same pointers costs one graph launch instead of one
 *                   launch per kernel.  Results are bit-identical to calls
 *                   without the flag.  Calls made while stage timing is
 *                   enabled run without the graph.
 *   SOFT_BETA_HALVES every band with 2B >= 128 holds its per-order-pair beta
 *                   samples (the S workspace) for half of the beta samples
 *                   at a time: the two halves j < 2B/4 or j >= 3(2B)/4 and
 *                   the middle half (each closed under j -> 2B-1-j, so the
 *                   members at pi - beta stay with their pair), each running
 *                   its own alpha FFT pass and DWT launch; the forward adds
 *                   the second half's sums to the first's.  Halves that
 *                   workspace (FP64, B = 512: 17.2 -> 8.6 GB) for two more
 *                   launches per direction.  Inverse results are
 *                   bit-identical to a plan without the flag; forward
 *                   results differ by the rounding of that one addition.
 *                   Bands with 2B = 2048 always run this way.
 *   SOFT_DD_RECURRENCE  (FP64 plans only; SOFT_ERR_INVALID with the other
 *                   precisions) the DWT runs the three-term recurrence of
 *                   eq. "Wigner_d_recurrence" in double-double: its
 *                   coefficients (filled in double-double at plan time, 16
 *                   more bytes per recurrence row), cos(beta_j) and the
 *                   recurrence values carry about 106 bits, and each value
 *                   enters the FP64 matrix contraction rounded once.  The
 *                   FP64 recurrence loses accuracy with the degree (near
 *                   beta = 0 most: there alpha_l x - gamma_l cancels, and the
 *                   rounding of the coefficients and of cos(beta_j) is
 *                   amplified); this mode leaves the FP64 rounding of the FFT
 *                   and of the contraction (Sect. 5 names B = 512 as the size
 *                   where double precision alone falls short on its CPU
 *                   design, which used extended precision).  Costs about
 *                   fifteen times the recurrence's arithmetic (1.7 times the
 *                   FP64 transform time at B = 512); the DWT launch shapes
 *                   are those of soft_plan_set_dwt_shape's list for it, and
 *                   the Clenshaw forms are not available.
 */
enum {
    SOFT_PLAN_TUNE = 1u,
    SOFT_INPLACE_OK = 2u,
    SOFT_PLAN_GRAPH = 4u,
    SOFT_BETA_HALVES = 8u,
    SOFT_DD_RECURRENCE = 16u
};

typedef enum {
    SOFT_OK = 0,
    SOFT_ERR_INVALID = -1,     /* null pointer, B < 1, batch < 1, unknown precision or flag, wrong device */
    SOFT_ERR_UNSUPPORTED = -2, /* valid for the paper but not built here: B not a power of two, B > 1024
                                  (B > 512 for the matching entry points), more than 65535 functions in
                                  one plan */
    SOFT_ERR_OOM = -3,         /* device or host allocation failed at plan time */
    SOFT_ERR_HIP = -4          /* a HIP runtime call or kernel launch failed */
} soft_status;

/*
 * soft_plan -- plan `batch` transforms of bandwidth B (Sect. 2.3: a function
 * of bandwidth B lives in H_B, degrees l < B).
 *   B          bandwidth, a power of two with 1 <= B <= 1024.  At B = 1024
 *              (2B = 2048) the seeds d(l0, l0, m'; b_j) that the recurrence
 *              needs reach about 2^-1240, below double precision's range:
 *              that band keeps such seeds scaled by 2^1000 and the DWT runs
 *              those recurrences scaled until they pass 2^-200 (Sect. 5
 *              names B = 512 as the size where double precision alone falls
 *              short on its CPU design).  That band also runs in two beta
 *              halves (the per-order-pair samples are held for half of the
 *              beta samples at a time): with SOFT_INPLACE_OK an FP64 plan
 *              at B = 1024 holds about 82 GB (242 GB with the caller's grid
 *              and coefficients), an FP32 or FP32-split plan about 47 GB;
 *              without the flag the FFT intermediate adds one grid's size.
 *   batch      number of functions per call, 1 <= batch <= 65535.
 *   precision  a soft_precision.
 *   flags      any of SOFT_PLAN_TUNE, SOFT_INPLACE_OK, SOFT_PLAN_GRAPH,
 *              SOFT_BETA_HALVES and (FP64) SOFT_DD_RECURRENCE; other bits
 *              are SOFT_ERR_INVALID.
 *   out        receives the plan handle; unchanged on error.
 * Allocates the plan's device workspace (per function, about 2 (2B)^3
 * complex elements for the FFT intermediate and the per-order-pair beta
 * samples, or about (2B)^3 with SOFT_INPLACE_OK, half of that for the
 * samples at 2B = 2048; per distinct bandwidth, 24 bytes per recurrence
 * row (40 with SOFT_DD_RECURRENCE), about B^3/6 rows, and the 8-byte seeds
 * d(l0, l0, m'; b_j) of every symmetry group at every beta sample,
 * B(B+1)/2 x 2B of them) and its tables (quadrature weights, Wigner-d seed
 * constants, FFT twiddles, symmetry groups, work lists) on the current HIP
 * device; later calls must run with the same device current.  Synchronous.
 * Returns SOFT_OK, SOFT_ERR_INVALID, SOFT_ERR_UNSUPPORTED, SOFT_ERR_OOM or
 * SOFT_ERR_HIP.
 */
int soft_plan(int B, int batch, int precision, unsigned flags, soft_plan_t *out);

/*
 * soft_plan_uneven -- plan one call over n functions of mixed bandwidths
 * (the batched transform over uneven bandwidths: each function keeps its own
 * B, grid and coefficient count).
 *   B_list     host array of n bandwidths, each a power of two <= 1024, in
 *              the order the functions are stored; read during the call only.
 *   n          number of functions, 1 <= n <= 65535.
 *   precision, flags, out   as for soft_plan.
 * Functions of equal B share one set of tables.  The FFT passes run once
 * per distinct B; the DWT runs as one launch over all functions with
 * 2B <= 256 (largest recurrence first) plus one per larger bandwidth.
 * Returns as soft_plan.
 */
int soft_plan_uneven(const int *B_list, int n, int precision, unsigned flags, soft_plan_t *out);

/*
 * soft_plan_check -- build the host side of a plan for the bandwidths
 * B_list[0..n) (its tables of Sect. 2.2-2.4 and its DWT work lists) without
 * touching a device, check it, and release it: every (function, symmetry
 * group) in exactly one work item, every order pair of every function in
 * exactly one group slot (eq. "Wigner_symmetries"), every offset inside its
 * buffer, every launch shape covering its launch.  For testing the plan logic
 * on hosts without a GPU.  Arguments as for soft_plan_uneven.  Returns
 * SOFT_OK, SOFT_ERR_INVALID (bad arguments, or a check failed),
 * SOFT_ERR_UNSUPPORTED or SOFT_ERR_OOM.
 */
int soft_plan_check(const int *B_list, int n, int precision, unsigned flags);

/*
 * soft_plan_sizes -- element counts of one call's buffers.
 *   grid_elems   complex elements of all grids of the plan (sum of (2B)^3).
 *   coeff_elems  complex elements of all coefficient vectors (sum of B(4B^2-1)/3).
 *   workspace_bytes  device bytes the plan holds.
 * Any output pointer may be NULL.  Returns SOFT_OK or SOFT_ERR_INVALID.
 */
int soft_plan_sizes(soft_plan_t plan, size_t *grid_elems, size_t *coeff_elems,
                    size_t *workspace_bytes);

/*
 * soft_plan_describe -- a one-line JSON description of the plan (bands,
 * functions, workspace bytes, whether it was made with SOFT_INPLACE_OK,
 * whether it runs the double-double recurrence (SOFT_DD_RECURRENCE),
 * whether its tuned shapes came from the SOFT_TUNE_CACHE file, and
 * per DWT launch its largest 2B, the number of beta halves it runs in (2 for
 * 2B = 2048, see soft_plan), work items, forward and inverse launch shapes
 * and whether they were tuned), written to
 * buf as a NUL-terminated string truncated to len - 1 characters.
 * Returns SOFT_OK or SOFT_ERR_INVALID (NULL plan or buf, len == 0).
 */
int soft_plan_describe(soft_plan_t plan, char *buf, size_t len);

/*
 * soft_plan_set_dwt_shape -- pin the launch shape of one DWT launch of the
 * plan (as listed by soft_plan_describe, in order).
 *   launch     index of the DWT launch (0 <= launch < number of launches).
 *   direction  0 = forward DWT, 1 = inverse DWT.
 *   waves, subsets  one of the built shapes (waves x subsets of 64 beta
 *              samples per wave): 1x1, 2x1, 4x1, 8x1, 1x2, 2x2, 4x2, 8x2, 16x1, 4x4,
 *              8x4, covering the launch: waves * subsets * 64 >= its beta
 *              rows (its largest 2B, or 2B/2 for a launch in beta halves);
 *              or 0x0 (launches with 2B <= 1024): the DWT by Clenshaw-type recurrences on the FP64
 *              vector unit instead of the matrix contraction (Sect. 2.4),
 *              one beta sample per lane: the inverse by Clenshaw's backward
 *              summation over degrees, the forward by its transpose (the
 *              adjoint-Clenshaw evaluation: each lane runs the three-term
 *              recurrence forward and the sums over beta are reduced across
 *              lanes).  soft_plan_describe reports it as [0, 0].
 *              A SOFT_DD_RECURRENCE plan takes 1x1, 2x1, 4x1, 8x1, 2x2, 4x2,
 *              8x2, 16x1 and 4x4 only (no Clenshaw form).
 * Takes effect for later calls.  Returns SOFT_OK or SOFT_ERR_INVALID.
 */
int soft_plan_set_dwt_shape(soft_plan_t plan, int launch, int direction, int waves, int subsets);

/*
 * soft_plan_offsets -- start of each function's grid and coefficients.
 *   grid_offsets   host array of n+1 entries (or NULL): element offset of
 *                  function f's grid in the grid buffer; entry n = total.
 *   coeff_offsets  host array of n+1 entries (or NULL): the same for the
 *                  coefficient buffer.
 * Offsets count complex elements of the plan's precision.
 * Returns SOFT_OK or SOFT_ERR_INVALID.
 */
int soft_plan_offsets(soft_plan_t plan, size_t *grid_offsets, size_t *coeff_offsets);

/*
 * soft_forward -- FSOFT (eq. "quadrature" via Sect. 2.4): coefficients of
 * the sampled functions.
 *   grid    device pointer, the plan's grids (read only; overwritten with
 *           scratch by a SOFT_INPLACE_OK plan).
 *   coeffs  device pointer, the plan's coefficient vectors (written).
 *   stream  HIP stream the work is enqueued on (0 = null stream).
 * The input grid need not be band-limited; the result is the quadrature sum.
 */
int soft_forward(soft_plan_t plan, const void *grid, void *coeffs, hipStream_t stream);

/*
 * soft_inverse -- iFSOFT (eq. "fourier_representation" sampled on the grid,
 * computed as T_B^T per order pair then a 2-D FFT per beta sample).
 *   coeffs  device pointer, the plan's coefficient vectors (read only).
 *   grid    device pointer, the plan's grids (written).
 */
int soft_inverse(soft_plan_t plan, const void *coeffs, void *grid, hipStream_t stream);

/*
 * soft_adjoint -- F^H, the adjoint (conjugate transpose under the plain
 * Euclidean inner products of grid and coefficient vectors) of soft_forward:
 * F^H = W I V, i.e. scale degree l by (2l+1)/(8 pi B), run the inverse, scale
 * beta-slice j by w_B(j) (the factors of the matrix form in Sect. 2.4).
 * Same arguments as soft_inverse.
 */
int soft_adjoint(soft_plan_t plan, const void *coeffs, void *grid, hipStream_t stream);

/*
 * soft_adjoint_inverse -- I^H, the adjoint of soft_inverse: I^H = V^-1 F W^-1,
 * i.e. the separation of variables followed by the plain contraction with
 * T_B (no weights, no (2l+1)/(8 pi B)).  Same arguments as soft_forward.
 */
int soft_adjoint_inverse(soft_plan_t plan, const void *grid, void *coeffs, hipStream_t stream);

/*
 * Stage timing (measurement support).  When enabled, every transform call
 * records a HIP event on its stream before and after each kernel of a timed
 * stage it enqueues (adjacent timed kernels share one);
 * soft_plan_stage_times() waits for the recorded events and returns, per
 * stage, the summed elapsed milliseconds and the number of launches timed.
 * A plan of several bandwidths launches the FFT stages once per distinct B
 * and the DWT stages once per launch shape; each launch counts once.
 * Stages (SOFT_STAGE_*):
 *   0 gamma FFT (forward)      1 alpha FFT + weights (forward)
 *   2 DWT, writing f° (fwd)    3 iDWT, reading f° (inverse)
 *   4 alpha FFT (inverse)      5 gamma FFT (inverse)
 *   6 correlation coefficients and 7 argmax, recorded by soft_match on the
 *     plan returned by soft_match_plan_soft.
 */
enum {
    SOFT_STAGE_FFT_GAMMA_FWD = 0,
    SOFT_STAGE_FFT_ALPHA_FWD = 1,
    SOFT_STAGE_DWT_FWD = 2,
    SOFT_STAGE_DWT_INV = 3,
    SOFT_STAGE_FFT_ALPHA_INV = 4,
    SOFT_STAGE_FFT_GAMMA_INV = 5,
    SOFT_STAGE_MATCH_COEFFS = 6,
    SOFT_STAGE_ARGMAX = 7,
    SOFT_NUM_STAGES = 8
};

/*
 * soft_plan_set_timing -- enable (1) or disable (0) stage timing of every
 * stage for later calls on this plan.  Returns SOFT_OK or SOFT_ERR_INVALID.
 */
int soft_plan_set_timing(soft_plan_t plan, int enable);

/*
 * soft_plan_set_timing_stages -- time only the stages whose bit is set in
 * mask (bit s = stage s, s < SOFT_NUM_STAGES; 0 disables timing), for later
 * calls on this plan.  Each timed kernel costs about two event records on
 * its stream, so timing one stage perturbs a call less than timing all.
 * Returns SOFT_OK or SOFT_ERR_INVALID (unknown bits).
 */
int soft_plan_set_timing_stages(soft_plan_t plan, unsigned mask);

/*
 * soft_plan_stage_times -- wait for all recorded stage events of this plan,
 * add their durations to the plan's totals and copy the totals out:
 * ms[s] = summed milliseconds, launches[s] = number of timed launches, for
 * s < SOFT_NUM_STAGES (either pointer may be NULL).  reset != 0 clears the
 * totals afterwards.  Blocks the host until the recorded work has run.
 * Returns SOFT_OK, SOFT_ERR_INVALID or SOFT_ERR_HIP.
 */
int soft_plan_stage_times(soft_plan_t plan, double *ms, long long *launches, int reset);

/*
 * soft_plan_destroy -- release the plan's device memory.  Waits first for
 * the work of the plan's last transform call (an event recorded on that
 * call's stream), so no enqueued work still uses the workspace; other streams
 * and other work on the device are not waited for.  NULL is accepted and
 * ignored.  Returns SOFT_OK or SOFT_ERR_HIP.
 */
int soft_plan_destroy(soft_plan_t plan);

/*
 * Rotational-matching head.  Matching two functions on the sphere over
 * rotations (the application of Sect. 1) correlates them: with a(l, m) and
 * b(l, m) their spherical-harmonic coefficients, the SO(3) coefficients
 *   f°(l, M, M') = a(l, M) conj(b(l, M'))
 * define a function on SO(3) whose inverse transform (soft_inverse) is the
 * correlation grid, and the grid point of largest real part is the best
 * rotation on the grid.
 *
 * Layouts: a function on the sphere is B^2 complex coefficients, (l, m) at
 * l^2 + m + l (0 <= l < B, -l <= m <= l); n of them back to back.  SO(3)
 * coefficients and grids as above, n of each back to back.  Complex type as
 * the precision says (complex128 for SOFT_FP64, complex64 otherwise).
 */
typedef struct soft_match_s *soft_match_t;

/*
 * soft_match_plan -- plan the head for n pairs at bandwidth B.
 *   B, precision, flags as for soft_plan; n >= 1 pairs.
 *   out  receives the handle; unchanged on error.
 * Owns a soft_plan of n functions of bandwidth B (made with the same flags:
 * with SOFT_INPLACE_OK it holds no FFT intermediate, and soft_adjoint_inverse
 * on it overwrites its input grid), one set of n coefficient vectors, the
 * argmax partial results (16 bytes per pair and scanned block), and the
 * workspace of soft_match_polish (80 bytes per pair plus at most 160 KB).
 * Synchronous.  Returns as soft_plan.
 */
int soft_match_plan(int B, int n, int precision, unsigned flags, soft_match_t *out);

/*
 * soft_match_sizes -- per-call element counts: sh_elems of each of a and b
 * (n B^2), coeff_elems of the coefficients (n B(4B^2-1)/3) and grid_elems of
 * the grids (n (2B)^3).  Any pointer may be NULL.
 */
int soft_match_sizes(soft_match_t match, size_t *sh_elems, size_t *coeff_elems, size_t *grid_elems);

/*
 * soft_match_plan_soft -- the soft_plan the head owns (for soft_adjoint_inverse
 * in a backward pass, or stage timing).  Valid until soft_match_destroy; do
 * not destroy it.
 */
int soft_match_plan_soft(soft_match_t match, soft_plan_t *plan);

/*
 * soft_match_coeffs -- coeffs = f°(l, M, M') = a(l, M) conj(b(l, M')) for
 * every pair.  a, b: device, n B^2 each (read only); coeffs: device, written.
 */
int soft_match_coeffs(soft_match_t match, const void *a, const void *b, void *coeffs, hipStream_t stream);

/*
 * soft_match_coeffs_vjp -- vector-Jacobian product of soft_match_coeffs
 * (gradients as conjugate Wirtinger derivatives, the convention of complex
 * automatic differentiation): given g = dL/d conj(f°),
 *   ga(l, M)  = sum_M' g(l, M, M') b(l, M'),
 *   gb(l, M') = sum_M conj(g(l, M, M')) a(l, M).
 * a, b, g: device (read only); ga, gb: device, n B^2 each (written).  Sums
 * run in FP64 in every precision.
 */
int soft_match_coeffs_vjp(soft_match_t match, const void *a, const void *b, const void *g, void *ga, void *gb,
                          hipStream_t stream);

/*
 * soft_match_argmax -- for each of the n grids, the flat index
 * (i*2B + j)*2B + k of the largest real part, the smallest such index on
 * exact ties; NaN entries never win (-1 when every entry is NaN).
 *   grid   device, n grids (read only).
 *   index  device, n int64 (written).
 */
int soft_match_argmax(soft_match_t match, const void *grid, long long *index, hipStream_t stream);

/*
 * soft_match -- the whole head: correlation coefficients of every pair (in
 * the head's own buffer), soft_inverse of them into grid, argmax of each
 * grid into index.  a, b: device (read only); grid: device, n grids
 * (written), or NULL; index: device, n int64 (written).
 * With grid NULL no grid is written: the last FFT pass of the inverse
 * reduces its values to argmax partial results in the head's buffer, and
 * index is the same as with a grid (the same values are compared, with the
 * same tie rule).  That needs the soft_plan's own FFT intermediate:
 * SOFT_ERR_INVALID for a head made with SOFT_INPLACE_OK.
 */
int soft_match(soft_match_t match, const void *a, const void *b, void *grid, long long *index, hipStream_t stream);

/*
 * soft_match_argmax_noalloc -- soft_match_argmax without a head, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops that forbid hipMalloc): the same result for n grids of bandwidth B,
 * with the partial results in a 1 MiB array that the library holds in static
 * device memory on every GPU it runs on until the process ends.  Calls no
 * allocating routine; its first call on a device looks up that device's copy
 * of the array.
 *   B          bandwidth of the grids, a power of two <= 512.
 *   n          number of grids, 1 <= n <= 65535 (every such n fits the array).
 *   precision  a soft_precision: complex128 grids for SOFT_FP64, complex64
 *              otherwise.
 *   grid       device, n grids of (2B)^3 elements back to back (read only).
 *   index      device, n int64 (written), as soft_match_argmax.
 * Every call on one GPU shares that GPU's array, so calls that overlap in
 * time on one GPU (two streams, two host threads) race: serialise them.
 * Returns SOFT_OK, SOFT_ERR_INVALID (NULL pointer, B < 1, n < 1, unknown
 * precision), SOFT_ERR_UNSUPPORTED (B not a power of two or > 512, n > 65535)
 * or SOFT_ERR_HIP.
 */
int soft_match_argmax_noalloc(int B, int n, int precision, const void *grid, long long *index, hipStream_t stream);

/*
 * soft_sh_forward -- spherical-harmonic coefficients of n functions on the
 * sphere (the inputs of rotational matching, Sect. 1), by the sampling
 * theorem of Sect. 2.3 at m' = 0:
 *   a(l, m) = sum_{j,k} w_B(j) f(theta_j, phi_k) conj(Y_l^m(theta_j, phi_k)),
 *   Y_l^m(theta, phi) = sqrt((2l+1)/(4 pi)) e^{i m phi} d(l, 0, m; theta),
 * the orthonormal spherical harmonics with the Condon-Shortley phase (d(l, 0, m)
 * of Sect. 2.2 is the textbook d^l_{m0}); exact for functions of degree < B.
 *   B          bandwidth, a power of two <= 512; n >= 1 functions (<= 65535).
 *   precision  a soft_precision (complex128 data for SOFT_FP64, complex64
 *              otherwise; the arithmetic is FP64 in every precision).
 *   f          device, n sample grids [2B][2B], f(theta_j, phi_k) at
 *              j * 2B + k with theta_j = (2j+1) pi/(4B), phi_k = k pi/B (read only).
 *   a          device, n x B^2 coefficients, (l, m) at l^2 + m + l (written).
 * Allocates nothing.  Returns SOFT_OK, SOFT_ERR_INVALID, SOFT_ERR_UNSUPPORTED
 * or SOFT_ERR_HIP.
 */
int soft_sh_forward(int B, int n, int precision, const void *f, void *a, hipStream_t stream);

/*
 * soft_match_refine -- the rotation of each pair read off its correlation
 * grid (as written by soft_match) at its maximum index (from soft_match or
 * soft_match_argmax), refined below the grid spacing: along each axis a
 * parabola through Re C at the maximum and its two neighbours (periodic in
 * alpha and gamma; none at the first and last beta sample) moves the grid
 * coordinate by (c- - c+) / (2 (c- - 2 c0 + c+)) when the three values bend
 * down, clamped to half a step.  With a = coefficients of f and b of g
 * (f°(l, M, M') = a(l, M) conj(b(l, M'))), the result is the rotation R with
 * g(w) = f(R^-1 w), R = Rz(alpha) Ry(beta) Rz(gamma): (alpha, beta, gamma)
 * = (gamma_k, beta_j, alpha_i) at the refined grid coordinates (i, j, k)
 * (the outer angles swap because d(l, m, m') of Sect. 2.2 is the transpose of
 * the textbook d^l_{m m'}).
 *   grid    device, the head's n grids (read only).
 *   index   device, n int64 grid maxima; an index of -1 gives NaN angles.
 *   angles  device, n x 3 doubles (alpha, beta, gamma) (written).
 * Returns SOFT_OK, SOFT_ERR_INVALID or SOFT_ERR_HIP.
 */
int soft_match_refine(soft_match_t match, const void *grid, const long long *index, double *angles,
                      hipStream_t stream);

/*
 * soft_match_polish -- the maximum of each pair's correlation function off
 * the grid: Newton steps on Re C(Q), C the SO(3) function with the pair's
 * correlation coefficients evaluated at a rotation Q by the sum of eq.
 * "fourier_representation" (at the rotation that grid index (i, j, k) names,
 * soft_match_refine's read-out, C equals the grid value).  The steps run in
 * local rotation-vector coordinates w around the current rotation Q0 (no
 * Euler-angle pole on the way): F(w) = Re C(Q0 exp([w]x)) at the ten points
 * w = 0, +-h e_i, h (e_i + e_j) gives the gradient and Hessian of a quadratic
 * model; the step is -H^-1 g when -H is positive definite, else a per-axis
 * step, each component clamped to [-h, h]; then Q0 = Q0 exp([step]x) and h =
 * min(h, max(1e-5, 2 max|step|)), from h = pi/(4B).  For band-limited
 * functions the correlation's maximum is the rotation itself, which the
 * steps reach to about 1e-9 from soft_match_refine's start.
 *   match   a match plan (B <= 512): its bandwidth, n and precision.
 *   coeffs  device, n correlation coefficient vectors (soft_match_coeffs
 *           layout and complex type; read only).
 *   start   device, n x 3 double rotation angles (a, b, c) of Rz(a) Ry(b) Rz(c)
 *           (soft_match_refine's output; read only).
 *   iters   Newton steps, 0 .. 64 (each costs ten evaluations of C, each a
 *           pass over the coefficients; about 6 converge).
 *   angles  device, n x 3 double (written): the polished (a, b, c), b in
 *           [0, pi], a and c in [0, 2 pi).
 *   value   device, n double (written): Re C at the polished rotation.
 * Each step is one launch that evaluates the ten points over chunks of the
 * symmetry groups (blocks of (chunk, pair), about 2048 in all) and one that
 * sums the chunks and takes the step (a thread per pair).  The per-pair state
 * and chunk sums live in the head's workspace (made by soft_match_plan), so
 * calls on one head must not overlap; allocates nothing.  Returns SOFT_OK,
 * SOFT_ERR_INVALID or SOFT_ERR_HIP.
 */
int soft_match_polish(soft_match_t match, const void *coeffs, const double *start, int iters, double *angles,
                      double *value, hipStream_t stream);

/* soft_match_destroy -- release the head and its soft_plan, after waiting for the
 * work of its last call as soft_plan_destroy does (NULL ignored). */
int soft_match_destroy(soft_match_t match);

/*
 * Device ceilings (measurement support, not part of the transform): kernels
 * of this library that measure what the GPU sustains, so that the roofline
 * fractions of the transform kernels can be read against measured rates as
 * well as the published peaks.
 *
 * soft_probe_copy -- copy `bytes` (a multiple of 16) from src to dst, both
 *   device pointers, with non-temporal loads and stores (every byte read
 *   once and written once: 2 * bytes of HBM traffic).  Returns SOFT_OK,
 *   SOFT_ERR_INVALID (NULL pointer, bytes 0 or not a multiple of 16) or
 *   SOFT_ERR_HIP.
 * soft_probe_flops -- run a dependent-chain arithmetic loop on `blocks`
 *   blocks of four waves for `iters` iterations: kind 0 FP64 vector FMA,
 *   1 FP64 matrix core (16x16x4 MFMA), 2 FP32 matrix core (16x16x4 MFMA).
 *   sink: device, blocks * 256 doubles (kept as an output so the loop is not
 *   removed; not written in practice).  Returns SOFT_OK, SOFT_ERR_INVALID or
 *   SOFT_ERR_HIP.
 * soft_probe_flop_count -- the flops one soft_probe_flops launch performs
 *   (FMA = 2 flops); 0 for invalid arguments.
 */
int soft_probe_copy(const void *src, void *dst, size_t bytes, hipStream_t stream);
int soft_probe_flops(int kind, int blocks, int iters, double *sink, hipStream_t stream);
double soft_probe_flop_count(int kind, int blocks, int iters);

/* soft_status_string -- static text for a status code (never NULL). */
const char *soft_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SOFT_H */
