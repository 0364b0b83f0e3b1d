/*
 * sg.h — C ABI of the MI355X (gfx950) library for the in-plane
 * self-gravitational forces of infinitesimally thin disks with order-k
 * B-spline density interpolation (Wang, Shiue, Wu & Yen, arXiv 1904.07400).
 *
 * The problem (Sec. 1, Eq. (Fx_convolution); Sec. 2, Eqs. (eqnSigma)-(eqnw)):
 * a surface density sigma confined to the rectangle [x0,x1] x [y0,y1], cut
 * into nx x ny equal cells, is interpolated with order-k tensor B-splines
 * (k = 1, 2, 3: piecewise constant, linear, quadratic; Sec. 2, Eqs.
 * (Bspline1)-(Bspline3); k = 4, 5: cubic and quartic, the extension to
 * higher orders that Case 3 of Sec. 2.2 and the end of Sec. 2.3 state); the forces at the cell centres are the discrete
 * convolutions  F^x_ij = sum_{i'j'} C_{i'j'} w^x_{i-i',j-j'}  (Eq. (eqnF)) with
 * the kernel weights of Eq. (eqnwB), G = 1, attractive sign (the integrand
 * is (x'-x)/r^3, Sec. 2.2 Case 1).  The convolutions are evaluated with
 * zero-padded 2nx x 2ny FFTs, so mass confined to the domain needs no
 * boundary values.
 *
 * Conventions shared by every call:
 *  - All array arguments are caller-owned DEVICE pointers (hipMalloc'd or
 *    torch CUDA tensors), except where a parameter says HOST.
 *  - Grid arrays are row-major [ny][nx], x fastest: cell (i, j) of the paper
 *    (1-based) is element (j-1)*nx + (i-1).  A plan with several grids uses
 *    packed buffers: grid g occupies elements [offset_g, offset_{g+1}) (see
 *    sg_plan_layout).
 *  - Element type: double for SG_FP64 plans; float for SG_FP32_SPLIT plans
 *    (sigma, forces and gradients), except sg_weights, always double.
 *  - Per-step calls (sg_bspline_coeffs, sg_forces, sg_forces_adjoint) are
 *    asynchronous on the plan's HIP stream, allocate no device memory and do
 *    not synchronise (except sg_forces on a plan created with
 *    SG_FLAG_CHECK_FINITE, which waits for the check's result); buffers must
 *    stay alive until the stream has passed the call.  Two calls on one
 *    plan must not overlap in time (they share the plan's workspace): issue
 *    them on the plan's stream.
 *  - Every call returns an sg_status; a non-OK status leaves a thread-local
 *    message for sg_last_error_message().  After a device error
 *    (SG_ERR_DEVICE) the plan is sticky: every later call on it returns
 *    SG_ERR_STATE until it is destroyed.
 *  - Diagnostics from the environment: SG_LOG=1 prints every plan's launch
 *    choices and every error message to stderr; SG_ROCTX=1 marks the entry
 *    points and the passes of an eager step with roctx ranges (rocprofv3
 *    --marker-trace), from libroctx64 loaded at first use.
 */
#ifndef SG_H
#define SG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_plan_s* sg_plan;

typedef enum {
  SG_OK = 0,
  SG_ERR_ARG = 1,         /* null pointer, bad size, empty or non-finite domain, bad index */
  SG_ERR_UNSUPPORTED = 2, /* order outside 1..5, grid size without a kernel instantiation */
  SG_ERR_NOMEM = 3,       /* device or host allocation failed */
  SG_ERR_DEVICE = 4,      /* a HIP call or kernel launch failed (message holds the HIP error) */
  SG_ERR_STATE = 5        /* plan is in the sticky error state, or a non-finite input was found */
} sg_status;

typedef enum {
  SG_FP64 = 0,       /* every per-step array double; FFT and products in FP64 */
  SG_FP32_SPLIT = 1  /* float arrays; coefficient solve in FP64, FFT in FP32 with
                        FP64-derived twiddles; kernel spectra as hi+lo float pairs (as single floats
                        for ny = 2048, 4096, 8192 unless SG_FLAG_SPECTRA_SPLIT) */
} sg_precision;

/* One grid.  Cell sizes are dx = (x1-x0)/nx, dy = (y1-y0)/ny (Sec. 2, grid
 * points x_{i+1/2} = x0 + i dx).  nx, ny: each 2^a from 4 to 8192 or
 * 3 * 2^a from 12 to 1536 (other sizes: SG_ERR_UNSUPPORTED). */
typedef struct {
  int32_t nx, ny;
  double x0, x1, y0, y1;
  int32_t order; /* k in {1, 2, 3, 4, 5} */
} sg_grid;

/* plan flags */
#define SG_FLAG_CHECK_FINITE 0x1u /* sg_forces rejects non-finite sigma (SG_ERR_STATE); costs one extra read */
#define SG_FLAG_GRAPH 0x2u        /* sg_forces replays a captured HIP graph of the whole step (see sg_forces) */
#define SG_FLAG_AUTOTUNE 0x4u     /* sg_plan_create times the launch variants and tiles of every class not
                                     in the tuning store and keeps the best (see sg_plan_tuning) */
#define SG_FLAG_SPECTRA_SPLIT 0x8u /* SG_FP32_SPLIT: keep the kernel spectra of grids with ny = 2048, 4096 or 8192
                                      as hi + lo float pairs (8 B per bin).  Without it those grids' spectra are
                                      single floats (4 B per bin; the lo part moves the error by about 10 %, well
                                      inside 1e-6, and costs 8 B per cell of column-pass traffic); smaller grids
                                      always keep hi + lo.  Ignored by SG_FP64 plans. */

/* Create a plan for ngrids grids (all of one precision) on the given HIP
 * stream (hipStream_t; NULL = the null stream).  Plan time does what the
 * paper does "once at the beginning of simulations" (end of Sec. 2.2): it
 * evaluates the weight tables of Eq. (eqnwB) on the GPU in FP64 (closed form
 * of Appendix A on the piece holding the singularity, Gauss-Legendre
 * elsewhere), transforms them (FP64 FFT) and keeps their spectra.  Allocates
 * all workspace.  Synchronises the stream before returning. */
sg_status sg_plan_create(sg_plan* out, const sg_grid* grids /* HOST, ngrids */, int32_t ngrids,
                         sg_precision prec, void* hip_stream, uint32_t flags);

/* Release everything the plan owns; synchronises its stream first.
 * NULL is accepted (no-op). */
sg_status sg_plan_destroy(sg_plan p);

/* Packed-buffer layout: offsets[g] = first element of grid g, offsets[ngrids]
 * = total element count.  offsets: HOST array of ngrids+1. */
sg_status sg_plan_layout(sg_plan p, int64_t* offsets);

/* Number of grids, precision and device bytes held by the plan (any may be NULL; HOST). */
sg_status sg_plan_info(sg_plan p, int32_t* ngrids, int32_t* prec, int64_t* device_bytes);

/* Where sigma of grid g must be sampled (HOST outputs): point (i, j), 0-based,
 * is (xs0 + i*dx, ys0 + j*dy).  Odd k: the cell centres (interpolation
 * condition Eq. (eqnSigmaB)); even k: the vertices x0 + (i+1) dx, i.e. the
 * centres of the order-2 splines of Case 2 (Sec. 2.2), where C = sigma, and
 * of the cubic splines. */
sg_status sg_sample_points(sg_plan p, int32_t g, double* xs0, double* ys0, double* dx, double* dy);

/* Export the weights of grid g (Eq. (eqnwB)), FP64 DEVICE arrays of
 * (2ny-1) x (2nx-1): w(m, n), m = i-i' in [-(nx-1), nx-1], n = j-j' in
 * [-(ny-1), ny-1], at (n+ny-1)*(2nx-1) + (m+nx-1).  wx or wy may be NULL.
 * Recomputed on the plan's stream; asynchronous. */
sg_status sg_weights(sg_plan p, int32_t g, double* wx, double* wy);

/* sigma -> spline coefficients C for every grid of the plan (Sec. 2.3): the
 * identity for k = 1, 2; for k = 3 the tridiagonal systems of Eqs.
 * (z_system) and (C_system), C = 0 outside the grid; for k = 4, 5 the
 * systems of the same construction with the cubic spline's values
 * (1, 4, 1) / 6 and the quartic's (1, 76, 230, 76, 1) / 384 per axis.  Packed buffers;
 * sigma and coeffs may alias. */
sg_status sg_bspline_coeffs(sg_plan p, const void* sigma, void* coeffs);

/* sigma -> (Fx, Fy) at the cell centres for every grid of the plan:
 * coefficient solve, then one forward and two inverse zero-padded FFT
 * convolutions (Sec. 4.2).  Packed buffers; fx and fy must not alias sigma
 * or each other.
 *
 * Batching: the plan groups its grids into classes of equal (nx, ny, order);
 * each of the three passes is one launch for all grids of a class.  With
 * SG_FLAG_GRAPH the whole step (every class and pass, classes spread over
 * up to four plan-owned streams so that they overlap) is captured as a HIP
 * graph on the first call with a given (sigma, fx, fy) and replayed on
 * later calls with the same pointers (the four most recent are kept); the
 * replay is ordered after earlier work on the plan's stream and before
 * later work on it.  Per-pass timing is not recorded for graph plans. */
sg_status sg_forces(sg_plan p, const void* sigma, void* fx, void* fy);

/* sg_forces for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same launches,
 * results and arguments as sg_forces, with the per-step workspace (row
 * spectra X and combined spectra V of every grid) in a fixed 64 MiB device
 * array of the library instead of the plan's own.  Nothing is allocated,
 * freed, cleared or synchronised; the launches are eager (no graph) and
 * SG_FLAG_CHECK_FINITE is not applied.  The array is set up once per device
 * at plan creation and held until the process ends.  Limit: the workspace of
 * the plan's grids, 24 B per cell in FP32-split and 48 B per cell in FP64
 * plus 256-byte alignment per array (e.g. one 1024^2 grid), must fit in 64
 * MiB, else SG_ERR_ARG.  Every call on a GPU shares that GPU's array: calls
 * that overlap in time on one GPU (other streams, other plans, other host
 * threads) race and give wrong forces; the array keeps the last call's
 * contents, which the next call overwrites before reading. */
sg_status sg_forces_noalloc(sg_plan p, const void* sigma, void* fx, void* fy);

/* The plan's grid classes: *nclasses (HOST) and, for the first cap classes,
 * 8 HOST int32 each in info: nx, ny, order, number of grids, then the rows
 * per workgroup of the row passes and the columns per workgroup of the
 * column pass in use (A, B, C; chosen by the autotuner with
 * SG_FLAG_AUTOTUNE), then how they were chosen (as sg_plan_tuning).  info
 * may be NULL. */
sg_status sg_plan_classes(sg_plan p, int32_t* nclasses, int32_t* info, int32_t cap);

/* Launch choices of class cls (0-based, as sg_plan_classes), 8 HOST int32
 * in out: the launch variant of passes A, B, C (kernels of the same
 * transforms with other buffering or elements per thread; variant
 * choices that change the elements per thread change rounding, within the
 * precision of the plan), the tile of each pass (0 = compiled maximum), how
 * they were chosen (0 defaults, 1 timed at this plan's creation, 2 taken
 * from the tuning store), then 0.
 *
 * Tuning (plan time only): the choices live in a process-wide store; every
 * plan takes the variants recorded for its device, precision, size and
 * order (so that plans of one process compute identical results), and the
 * tiles recorded for its class size.  Missing entries are timed on zero
 * input when the plan has SG_FLAG_AUTOTUNE (variants, then tiles) and
 * recorded.  Environment: SG_TUNE=off (defaults only, the store ignored),
 * quick (time tiles only, for every plan), full (time variants and tiles,
 * for every plan); SG_TUNE_CACHE=path keeps the store in a JSON file, read
 * on first use and rewritten (merged, via a temporary file and a rename)
 * after new timings.  Entries carry the library build, so a rebuilt library
 * ignores older ones. */
sg_status sg_plan_tuning(sg_plan p, int32_t cls, int32_t* out);

/* Adjoint of sg_forces: gsigma = d<gfx,Fx> + <gfy,Fy> / d sigma, i.e. the
 * transposed convolutions (correlation with the weights) followed by the
 * transposed coefficient solve (the matrices of Eqs. (z_system) and
 * (C_system) are symmetric).  Packed buffers; gsigma must not alias the
 * inputs. */
sg_status sg_forces_adjoint(sg_plan p, const void* gfx, const void* gfy, void* gsigma);

/* Per-pass timing, a profiling aid.  While enabled, sg_forces records HIP
 * events on the plan's stream around each of its three kernel passes (row
 * transform, column transform with the spectral products, inverse row
 * transform).  sg_plan_pass_times synchronises the stream, returns the
 * milliseconds spent in each pass summed over all grids and calls since
 * timing was enabled (ms: HOST array of 3) and the number of calls, and
 * starts a new accumulation.  Enabling or disabling also resets it. */
sg_status sg_plan_set_timing(sg_plan p, int32_t enable);
sg_status sg_plan_pass_times(sg_plan p, double* ms, int64_t* calls);

/* Static string for a status code. */
const char* sg_status_string(sg_status s);

/* Detail for the last non-OK status returned on the calling thread ("" if none). */
const char* sg_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
