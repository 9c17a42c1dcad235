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
 *   complex numbers are interleaved (re, im): double2 for SOFT_FP64.
 *   A plan for `batch` functions of one bandwidth expects `batch` grids and
 *   `batch` coefficient vectors stored back to back.
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

typedef enum {
    SOFT_FP64 = 0 /* complex128 grids/coefficients, FP64 arithmetic throughout */
} soft_precision;

typedef enum {
    SOFT_OK = 0,
    SOFT_ERR_INVALID = -1,     /* null pointer, B < 1, batch < 1, unknown flag */
    SOFT_ERR_UNSUPPORTED = -2, /* valid for the paper but not built here: B not a power of two or B > 512 */
    SOFT_ERR_OOM = -3,         /* device or host allocation failed at plan time */
    SOFT_ERR_HIP = -4          /* a HIP runtime call or kernel launch failed */
} soft_status;

/*
 * soft_plan -- plan `batch` transforms of bandwidth B (Sect. 2.3: a function
 * of bandwidth B lives in H_B, degrees l < B).
 *   B          bandwidth, a power of two with 1 <= B <= 512.
 *   batch      number of functions per call (>= 1).
 *   precision  SOFT_FP64.
 *   flags      must be 0.
 *   out        receives the plan handle; unchanged on error.
 * Allocates the plan's device workspace (about 16 (2B)^3 bytes for the FFT
 * intermediate plus 16 (2B)^3 for the per-order-pair beta samples, per
 * function, and 4 B^3 bytes of recurrence tables) and its FP64 tables (quadrature weights, Wigner-d seed
 * constants, FFT twiddles), on the current HIP device; later calls must run
 * with the same device current.  Synchronous.
 * Returns SOFT_OK, SOFT_ERR_INVALID, SOFT_ERR_UNSUPPORTED, SOFT_ERR_OOM or
 * SOFT_ERR_HIP.
 */
int soft_plan(int B, int batch, int precision, unsigned flags, soft_plan_t *out);

/*
 * soft_plan_sizes -- element counts of one call's buffers.
 *   grid_elems   complex elements of all grids of the batch (batch * (2B)^3).
 *   coeff_elems  complex elements of all coefficient vectors (batch * B(4B^2-1)/3).
 *   workspace_bytes  device bytes the plan holds.
 * Any output pointer may be NULL.  Returns SOFT_OK or SOFT_ERR_INVALID.
 */
int soft_plan_sizes(soft_plan_t plan, size_t *grid_elems, size_t *coeff_elems,
                    size_t *workspace_bytes);

/*
 * soft_forward -- FSOFT (eq. "quadrature" via Sect. 2.4): coefficients of
 * the sampled functions.
 *   grid    device pointer, batch grids (read only).
 *   coeffs  device pointer, batch coefficient vectors (written).
 *   stream  HIP stream the work is enqueued on (0 = null stream).
 * The input grid need not be band-limited; the result is the quadrature sum.
 */
int soft_forward(soft_plan_t plan, const void *grid, void *coeffs, hipStream_t stream);

/*
 * soft_inverse -- iFSOFT (eq. "fourier_representation" sampled on the grid,
 * computed as T_B^T per order pair then a 2-D FFT per beta sample).
 *   coeffs  device pointer, batch coefficient vectors (read only).
 *   grid    device pointer, batch grids (written).
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
 * records a HIP event on its stream before and after each kernel it enqueues;
 * soft_plan_stage_times() waits for the recorded events and returns, per
 * stage, the summed elapsed milliseconds and the number of launches timed.
 * Stages (SOFT_STAGE_*), each one kernel:
 *   0 gamma FFT (forward)      1 alpha FFT + weights (forward)
 *   2 DWT, writing f° (fwd)    3 iDWT, reading f° (inverse)
 *   4 alpha FFT (inverse)      5 gamma FFT (inverse)
 */
enum {
    SOFT_STAGE_FFT_GAMMA_FWD = 0,
    SOFT_STAGE_FFT_ALPHA_FWD = 1,
    SOFT_STAGE_DWT_FWD = 2,
    SOFT_STAGE_DWT_INV = 3,
    SOFT_STAGE_FFT_ALPHA_INV = 4,
    SOFT_STAGE_FFT_GAMMA_INV = 5,
    SOFT_NUM_STAGES = 6
};

/*
 * soft_plan_set_timing -- enable (1) or disable (0) stage timing for later
 * calls on this plan.  Returns SOFT_OK or SOFT_ERR_INVALID.
 */
int soft_plan_set_timing(soft_plan_t plan, int enable);

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
 * soft_plan_destroy -- release the plan's device memory.  Synchronises the
 * device first so no enqueued work still uses the workspace.  NULL is
 * accepted and ignored.  Returns SOFT_OK or SOFT_ERR_HIP.
 */
int soft_plan_destroy(soft_plan_t plan);

/* soft_status_string -- static text for a status code (never NULL). */
const char *soft_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SOFT_H */
