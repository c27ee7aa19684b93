/*
 * vgx.h -- C ABI of the MI355X VEGAS hot path (libvgx.so).
 *
 * The operations follow the thesis's statement of the problem:
 *   - Monte Carlo integration with importance sampling and the VEGAS
 *     adaptive separable grid (thesis Sec. "Monte Carlo integration",
 *     "Importance sampling", "Adaptive Monte Carlo: VEGAS algorithm",
 *     "Inverse transform method");
 *   - PDF access in LHAPDF style, xf(x, Q^2) on a grid of knots with
 *     subgrids, log-bicubic interpolation with a bilinear fallback (thesis
 *     Sec. on LHAPDF and PDFFlow's design);
 *   - the hadronic master formula sigma = sum_ab int dPhi L |M|^2 with the
 *     pp -> t tbar sub-processes (thesis MadFlow chapter);
 *   - a learned importance-sampling proposal trained with Adam (thesis
 *     optimiser section); the coupling flow itself is not in the thesis
 *     (Mueller et al. 2019, piecewise-linear couplings).
 *
 * General conventions
 *   - Every pointer argument is named *_dev (device memory, caller-owned,
 *     e.g. a torch tensor's storage) or *_host (host memory, caller-owned).
 *     Contexts (vgx_vegas, vgx_pdf, vgx_flow) are library-owned and freed by
 *     the matching *_destroy.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *     "async" only enqueue work on it; calls marked "sync" wait for it.
 *   - Device arrays are structure-of-arrays: a [d][n] array holds dimension
 *     j of sample i at j*n + i.
 *   - Errors: a non-zero vgx_status; nothing is launched on VGX_EINVAL.
 *     vgx_last_error() returns a thread-local message of the last failure.
 *     No C++ exception crosses the ABI.
 *   - The library runs on the device current at the call (hipSetDevice);
 *     a context must be used on the device it was created on.
 *   - Calls on one context are not thread-safe; distinct contexts are.
 *
 * Environment
 *   - VGX_TRACE=<file> ("-": standard error): every estimate a synchronous
 *     call reads back (vegas_iterate, vegas_iterate_points,
 *     flow_vegas_iterate) is appended as one JSON line: the record, the
 *     combination after it, chi^2/dof, and an FNV-1a hash of the grid it was
 *     sampled on.
 *   - VGX_FAIL_ALLOC=k: the k-th device or pinned-host allocation counted
 *     from the variable's last change fails with VGX_ENOMEM (for tests of
 *     the error paths; stream-ordered scratch allocations are not counted).
 *
 * Checkpoint and resume: an iteration depends only on its grid and its
 * Philox counters, so saving the grid (vegas_get_grid) and the records
 * (vegas_results), and continuing with the same iteration indices on a
 * context given that grid (vegas_set_grid), reproduces an uninterrupted
 * run's records bit for bit.
 */
#ifndef VGX_H
#define VGX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; everything declared here is
 * exported. */
#pragma GCC visibility push(default)

typedef enum {
  VGX_OK = 0,
  VGX_EINVAL = 1,     /* invalid argument (sizes, pointers, kinds)          */
  VGX_ENOMEM = 2,     /* device or pinned-host allocation failed            */
  VGX_EDEVICE = 3,    /* a HIP runtime call failed                          */
  VGX_ERANGE = 4,     /* PDF query outside the grid (outputs set to NaN)    */
  VGX_ENUMERIC = 5,   /* non-finite iteration estimate (excluded)           */
  VGX_EFALLBACK = 6,  /* proposal worse than plain VEGAS, or non-finite
                         training loss: fall back to plain VEGAS             */
  VGX_ESTATE = 7      /* call not valid in the context's current state      */
} vgx_status;

/* Thread-local, NUL-terminated message describing the last error. */
const char* vgx_last_error(void);

/* Library version string (static storage). */
const char* vgx_version(void);

/* ------------------------------------------------------------------------ */
/* Integrands                                                                */
/* ------------------------------------------------------------------------ */
enum {
  VGX_GAUSS = 0,      /* prod_j N(x_j; c_j, s_j), normalised on R.
                         params = [c_0..c_{d-1}, s_0..s_{d-1}]               */
  VGX_GENZ_OSC = 1,   /* cos(2 pi w_1 + sum c_j x_j).  params = [w_1, c_0..] */
  VGX_GENZ_PEAK = 2,  /* prod (c_j^-2 + (x_j - w_j)^2)^-1.
                         params = [w_0..w_{d-1}, c_0..c_{d-1}]               */
  VGX_TTBAR = 3,      /* LO pp -> t tbar, d = 3, (tau, y, cos theta*) map.
                         params = [sqrt_s, m_top, alpha_s, gev2_to_pb(, mode)];
                         needs a PDF context, evaluated at mu^2 = m_top^2.
                         mode 0 (default): the full log-bicubic stencil in
                         (ln x, ln Q^2) per event; mode 1: the Q^2 direction,
                         identical for every event at the fixed scale, is
                         contracted once per workgroup and each event does
                         the ln x direction only (same interpolant, FP32
                         rounding differs); mode 2: the scale set per event,
                         mu^2 = s_hat/4, PDFs at (x, mu^2) and alpha_s(mu)
                         from the PDF's alpha_s table (pdf_set_alphas;
                         params[2] unused); the scales [m_top^2, s/4] must
                         lie in one PDF subgrid and one alpha_s subgrid      */
  VGX_DRELLYAN = 4,   /* LO pp -> photon or Z -> l+ l- (massless leptons), d = 3,
                         (tau, y, cos theta*) map over the dilepton-mass
                         window m_lo < m_ll < m_hi.
                         params = [sqrt_s, m_lo, m_hi, m_z, gamma_z, sin2w,
                         alpha, gev2_to_pb(, mode)]; needs a PDF context,
                         evaluated at mu^2 = m_z^2; mode as for VGX_TTBAR.
                         Thesis: master formula (MadFlow chapter) and
                         factorisation (PDF chapter); the gamma + Z helicity
                         amplitudes are textbook electroweak theory         */
  VGX_SINGLETOP = 5   /* LO s-channel single top, u dbar and c sbar -> W ->
                         t bbar (the thesis's LO single-top example), d = 3,
                         (tau, y, cos theta*) map from threshold m_top^2.
                         params = [sqrt_s, m_top, m_w, gamma_w, sin2w, alpha,
                         gev2_to_pb(, mode)]; needs a PDF context, evaluated
                         at mu^2 = m_top^2; diagonal CKM matrix; mode as for
                         VGX_TTBAR                                          */
};
enum { VGX_F64 = 0, VGX_F32 = 1 };   /* integrand / output precision          */
/* PDF / alpha_s behaviour outside the grid (pdf_set_extrapolation) */
enum { VGX_EXTRAP_ERROR = 0, VGX_EXTRAP_FREEZE = 1, VGX_EXTRAP_CONTINUE = 2 };
enum { VGX_OPERANDS_BF16 = 0, VGX_OPERANDS_F32 = 1 };  /* flow matrix-product operands */

#define VGX_MAX_DIM 12
#define VGX_MAX_BINS 256
#define VGX_MAX_PART 10

/* ------------------------------------------------------------------------ */
/* PDF grids (LHAPDF-style, thesis PDF chapter)                              */
/* ------------------------------------------------------------------------ */
typedef struct vgx_pdf vgx_pdf;

typedef struct {
  int32_t n_x;              /* x knots, shared by all subgrids, >= 2        */
  int32_t n_sub;            /* number of Q^2 subgrids, >= 1                  */
  int32_t n_flav;           /* flavours, 1 .. 16                             */
  const double* x_knots;    /* host [n_x], strictly ascending, > 0           */
  const int32_t* nq_per_sub;/* host [n_sub], each >= 2                       */
  const double* q2_knots;   /* host, subgrids concatenated, each strictly
                               ascending; last knot of subgrid s equals the
                               first knot of subgrid s+1                     */
  const double* xf;         /* host, x*f node values, per subgrid the block
                               [n_flav][n_q(s)][n_x], blocks concatenated    */
} vgx_pdf_desc;

/* Copy a grid to the device (sync).  Thesis: LHAPDF section (a set's
 * members are grids of xf on knots in x and Q^2, split into subgrids at the
 * flavour thresholds) and PDFFlow's design (the grid is loaded once into
 * device memory).  The descriptor's host arrays may be
 * freed after the call.  VGX_EINVAL on malformed knots, on a value that is
 * not finite or beyond the FP32 range (the FP32-output path reads an FP32
 * copy), and when 16 (n_x + total Q^2 knots) + 2048 s bytes exceed 64 KiB,
 * s = max(9, n_flav) rounded up to odd (the knots and per-query slots the
 * interpolation kernel keeps in LDS: up to 2688 knots in all for 11
 * flavours, 2944 for one). */
vgx_status pdf_create(const vgx_pdf_desc* desc, void* stream, vgx_pdf** out);

/* A PDF set: n_members grids sharing the descriptor's knots (thesis PDF
 * chapter, multi-member evaluation: all members of a set loaded at once).
 * desc->xf holds n_members consecutive member blocks, each laid out as for
 * pdf_create.  pdf_interp, pdf_alphas and the fused integrands use member 0;
 * pdf_interp_members evaluates every member.  1 <= n_members <= 65535. */
vgx_status pdf_create_set(const vgx_pdf_desc* desc, int32_t n_members, void* stream, vgx_pdf** out);

/* xf for every flavour at n points (async).  Thesis: LHAPDF section,
 * interpolation paragraphs (log-bicubic: cubic Hermite splines in ln x and
 * ln Q^2 on the four knots around the point, bilinear where that stencil
 * is incomplete; the subgrid figure) and PDFFlow's design (the xfxQ2 call
 * over a batch of points; accuracy measured by eq. pdfflow-diff).  The
 * Hermite slopes (not printed in the thesis) are the average of the two
 * adjacent secants, as in LHAPDF 6.
 *   x_dev, q2_dev : device [n] FP64 query points.
 *   out_dtype     : VGX_F64 or VGX_F32.
 *   out_dev       : device [n_flav][n] of that type.
 * Log-bicubic where the 4x4 stencil exists in both axes, bilinear
 * otherwise; subgrid chosen with the upper one winning at a threshold.
 * Queries outside the grid follow the context's extrapolation mode
 * (pdf_set_extrapolation); those it gives no value (every such query in
 * VGX_EXTRAP_ERROR; x > x_max, x <= 0, Q^2 <= 0 or non-finite points in the
 * others) produce NaN in all flavours and are counted (pdf_out_of_range).
 * n = 0 is a no-op. */
vgx_status pdf_interp(const vgx_pdf* pdf, int64_t n, const double* x_dev, const double* q2_dev,
                      int32_t out_dtype, void* out_dev, void* stream);

/* Every flavour of every member of a PDF set at n points (async).  Thesis:
 * PDFFlow section, "Multi-PDF members evaluation" (all members at the x
 * points of a FastKernel table; the table tab:fktable).
 *   out_dev : device [n_members][n_flav][n] of out_dtype.
 * Same interpolation as pdf_interp; points outside the grid give NaN in all
 * members and are counted once (pdf_out_of_range) whatever the extrapolation
 * mode.  n = 0 is a no-op. */
vgx_status pdf_interp_members(const vgx_pdf* pdf, int64_t n, const double* x_dev, const double* q2_dev,
                              int32_t out_dtype, void* out_dev, void* stream);

/* Flavours per member and members of a PDF context (either may be NULL). */
vgx_status pdf_shape(const vgx_pdf* pdf, int32_t* n_flav, int32_t* n_members);

/* Number of out-of-grid queries seen by pdf_interp since the last call of
 * this function (sync on `stream`); resets the counter.  Returns VGX_ERANGE
 * if the count is non-zero. */
vgx_status pdf_out_of_range(vgx_pdf* pdf, void* stream, int64_t* count_host);

/* Behaviour outside the grid for pdf_interp and pdf_alphas (thesis PDF
 * chapter, LHAPDF extrapolation paragraphs and the alpha_s paragraph):
 *   VGX_EXTRAP_ERROR    (default) no value: NaN, counted.
 *   VGX_EXTRAP_FREEZE   the value at the nearest grid point (x, Q^2 clamped
 *                       to the grid's ranges); alpha_s: its lowest-knot value.
 *   VGX_EXTRAP_CONTINUE the legacy continuation: below x_min a straight line
 *                       in ln x through the values at the two lowest x knots
 *                       (through ln xf when both exceed 1e-3, else through xf);
 *                       above Q^2_max the same in ln Q^2 through the top two
 *                       knots; below Q^2_min xf = G0 r^((gamma-1) r + 1),
 *                       r = Q^2/Q^2_min, G0 = xf(x, Q^2_min), gamma =
 *                       d ln xf/d ln Q^2 at Q^2_min from the grid just above
 *                       it; x rule first where both are outside; no value
 *                       above x_max.  alpha_s below its lowest knot: the
 *                       straight-line rule in ln Q^2 through the two lowest
 *                       knots.
 * alpha_s above its top knot is the top value in every mode.  The fused
 * integrands never query outside the grid (their ranges are checked when a
 * context is created), so the mode does not affect them.  VGX_EINVAL on an
 * unknown mode, or for CONTINUE on a grid with fewer than two x knots or two
 * Q^2 knots in its lowest subgrid. */
vgx_status pdf_set_extrapolation(vgx_pdf* pdf, int32_t mode);

/* Grid limits in x and Q^2. */
vgx_status pdf_bounds(const vgx_pdf* pdf, double* xmin, double* xmax, double* q2min, double* q2max);

/* Attach an alpha_s(Q) table to a PDF context (sync; replaces any previous
 * one).  Thesis, PDF chapter (alpha_s paragraphs): sets carry alpha_s at knots
 * on the Q line, interpolated log-cubically with subgrids at the flavour
 * thresholds.
 *   n        : number of knots, >= 2.
 *   q2_knots : host [n], ascending; a knot equal to its predecessor starts a
 *              new subgrid (the threshold knot duplicated); each subgrid >= 2.
 *   alphas   : host [n] values.
 * Host arrays may be freed after the call.  VGX_EINVAL on malformed knots. */
vgx_status pdf_set_alphas(vgx_pdf* pdf, int32_t n, const double* q2_knots, const double* alphas, void* stream);

/* alpha_s at n scales (async).  Thesis: LHAPDF section, the alpha_s
 * paragraph (log-cubic interpolation on the set's Q knots); PDFFlow's alpha_s
 * accuracy figure.  Cubic Hermite in ln Q^2 with secant-average
 * slopes on interior cells of the subgrid holding Q^2 (the upper subgrid at a
 * threshold), linear on a subgrid's first and last cells, the top value
 * above the last knot; below the first knot as the context's extrapolation
 * mode says (NaN by default; the thesis's rule there is garbled and read as
 * the straight-line continuation); NaN for Q^2 <= 0 or non-finite.
 *   q2_dev  : device [n] FP64;  out_dev : device [n] FP64.
 * VGX_EINVAL if no table is attached.  n = 0 is a no-op. */
vgx_status pdf_alphas(const vgx_pdf* pdf, int64_t n, const double* q2_dev, double* out_dev, void* stream);

void pdf_destroy(vgx_pdf* pdf);

/* ------------------------------------------------------------------------ */
/* VEGAS integration (thesis MC chapter)                                     */
/* ------------------------------------------------------------------------ */
typedef struct vgx_vegas vgx_vegas;

typedef struct {
  int32_t kind;             /* VGX_GAUSS, VGX_GENZ_OSC, VGX_GENZ_PEAK, VGX_TTBAR,
                               VGX_DRELLYAN, VGX_SINGLETOP                      */
  int32_t dim;              /* 1 .. VGX_MAX_DIM (3 for the hadronic kinds)      */
  int32_t n_bins;           /* bins per dimension, 2 .. VGX_MAX_BINS            */
  double alpha;             /* refinement damping exponent (e.g. 1.5)           */
  uint64_t seed;            /* Philox key                                       */
  uint32_t stream_id;       /* Philox stream (< 2^23)                           */
  int32_t prec;             /* VGX_F64 or VGX_F32 integrand arithmetic          */
  const double* params;     /* host, integrand parameters (see the kinds)       */
  int32_t n_params;
  const vgx_pdf* pdf;       /* hadronic kinds only; must outlive the context.
                               The LDS tables the integrand reads (PDF rows,
                               knots, alpha_s) are taken from it once, at
                               creation: a later pdf_set_alphas leaves an
                               existing context as it was.                      */
} vgx_vegas_cfg;

typedef struct {
  double mean;              /* E = S1/n                                          */
  double var;               /* (S2/n - E^2)/(n-1), clamped at 0                  */
  double s1, s2;            /* compensated sums of w = f J and w^2               */
  int64_t n;
} vgx_iter_result;

/* Create a context with a uniform grid e[j][k] = k/N (sync).  Thesis: MC
 * chapter, "Adaptive Monte Carlo: VEGAS algorithm" (a separable grid with a
 * fixed number of bins per dimension, starting from equal widths). */
vgx_status vegas_create(const vgx_vegas_cfg* cfg, void* stream, vgx_vegas** out);

/* One iteration (sync).  Thesis: MC chapter, the importance-sampling
 * estimator (eq. mc_est_is, with p the grid's piecewise-constant density,
 * sampled by the inverse transform method, eq. inverse-method) and its
 * variance (eq. var-en-est, read as the variance of the mean); the VEGAS
 * section's per-bin accumulation that drives the refinement.  Samples
 * i = 0..n-1, uniforms from Philox with
 * counter (i, iteration, stream_id, block) and key seed, mapped through the
 * grid, w = f(x) J(u); accumulates the compensated sums and the per-bin
 * histogram of w^2, appends (E, var) to the context's list of estimates
 * (used by vegas_result) and stores the histogram for vegas_refine.
 * VGX_ENUMERIC if the estimate is not finite (it is then excluded). */
vgx_status vegas_iterate(vgx_vegas* v, int64_t n, int32_t iteration, vgx_iter_result* out_host);

/* Same as vegas_iterate but async: the result stays on the device (read it
 * with vegas_results).  Lets a caller queue many iterations back to back.
 * The estimate and the combination are completed later on the context's
 * stream: by the next vegas_refine (beside the refinement, in the same
 * launch), or else first thing in the next call that reads or adds
 * estimates (vegas_result(s), any iterate, batch_iterate); the values are
 * bit-identical to vegas_iterate's.  vegas_reset_results discards it. */
vgx_status vegas_iterate_async(vgx_vegas* v, int64_t n, int32_t iteration);

/* Refine the grid from the last iteration's histogram (async).  Thesis:
 * VEGAS section (bin widths adjusted so that each bin carries an equal share
 * of the integrand; the formula is Lepage's, which the thesis cites): Lepage's
 * 3-point smoothing, damping r = ((1-p)/ln(1/p))^alpha, re-binning to equal
 * shares of sum r.  A dimension whose histogram is all zero or not finite
 * (a non-finite iteration) is unchanged. */
vgx_status vegas_refine(vgx_vegas* v);

/* Inverse-variance combination of the stored estimates and chi^2/dof
 * (sync).  Thesis: VEGAS section, the weighted average of the iterations'
 * estimates and the consistency check eq. vegas-check.  Non-finite estimates are skipped; a zero variance returns that
 * estimate with sigma 0. */
vgx_status vegas_result(vgx_vegas* v, double* mean, double* sigma, double* chi2_dof, int32_t* n_used);

/* Copy up to cap stored per-iteration results to the host (sync). */
vgx_status vegas_results(vgx_vegas* v, vgx_iter_result* out_host, int32_t cap, int32_t* count);

/* Drop all stored estimates (the grid is kept). */
vgx_status vegas_reset_results(vgx_vegas* v);

/* Grid edges [dim][n_bins+1] and histogram [dim][n_bins] (sync copies). */
vgx_status vegas_get_grid(vgx_vegas* v, double* edges_host);
vgx_status vegas_set_grid(vgx_vegas* v, const double* edges_host);
vgx_status vegas_get_hist(vgx_vegas* v, double* hist_host);

/* Materialise samples first .. first+n-1 of an iteration (async), e.g. the
 * training data of a learned proposal (the VEGAS samples and their weights):
 * u_dev [dim][n] the Philox uniforms (the VEGAS unit-cube coordinates) and
 * g_dev [n] = f(G(u)) J_G(u).  Either output may be NULL. */
vgx_status vegas_sample(vgx_vegas* v, int64_t first, int64_t n, int32_t iteration,
                        double* u_dev, double* g_dev);

/* Estimate from given unit-cube points y with proposal density q (sync).
 * Thesis: MC chapter, importance sampling (eq. mc_est_is with p = q times
 * the grid's density, whatever q is, so the estimate stays unbiased):
 * w = f(G(y)) J_G(y) exp(-logq).  y_dev [dim][n], logq_dev [n] (NULL means
 * q = 1).  Appends the estimate like vegas_iterate; no histogram (a later
 * vegas_refine still uses the last plain iteration's).  Plain VEGAS judges
 * the proposal: when logq_dev is given and the estimate's variance per sample
 * n var(E) exceeds that of the context's latest plain iteration read back by
 * vegas_iterate, the call returns VGX_EFALLBACK (the estimate, which is
 * unbiased, is still recorded and combined, and *out_host is filled): the
 * caller should fall back to plain VEGAS.  VGX_ENUMERIC if not finite. */
vgx_status vegas_iterate_points(vgx_vegas* v, int64_t n, const double* y_dev, const double* logq_dev,
                                vgx_iter_result* out_host);

/* Stream the context enqueues on. */
void* vegas_stream(vgx_vegas* v);

/* Dimension and bins per dimension of a context (either may be NULL). */
vgx_status vegas_shape(const vgx_vegas* v, int32_t* dim, int32_t* n_bins);

/* Kernel timing (for measurement): every = 0 turns it off; every = k >= 1
 * brackets one fused sampling kernel in k (the first after the call, then
 * every k-th) with HIP events on the context's stream (recording does not
 * synchronise; the events carry no system-scope fence, so they add no cache
 * write-back, but each record still delays the next launch by a few
 * microseconds, which k > 1 spreads over k launches); vegas_kernel_time
 * (sync) returns the summed milliseconds and the number of launches timed
 * since timing was enabled. */
vgx_status vegas_set_timing(vgx_vegas* v, int32_t every);
vgx_status vegas_kernel_time(vgx_vegas* v, double* ms_host, int64_t* launches_host);

void vegas_destroy(vgx_vegas* v);

/* ------------------------------------------------------------------------ */
/* Event generation (thesis MC chapter: RAMBO, acceptance-rejection; MadFlow  */
/* chapter: phase-space generator, unweighted event exporter)                */
/* ------------------------------------------------------------------------ */

/* RAMBO phase-space points for a total momentum P = (sqrt_s, 0, 0, 0) (async).
 * Thesis: MC chapter, RAMBO subsection (the recipe, eq. rambo-transform,
 * the weight eq. rambo-w0 and the massive variant); MadFlow chapter, phase
 * space generation.
 *   n_part     : final-state particles, 2 .. VGX_MAX_PART.
 *   masses     : host [n_part], >= 0, sum < sqrt_s; all zero: massless RAMBO
 *                (flat weight w0), else the massive variant (weight w0 w_m,
 *                3-momenta rescaled by the xi that restores energy
 *                conservation).
 *   seed, stream_id (< 2^24), iteration : Philox-4x32-10 key and counter
 *                fields; event e draws the uniforms of sample `first + e` of
 *                the VEGAS kernels' convention (block i for particle i).
 *   mom_dev    : device [4][n_part][n_events] FP64 (E, px, py, pz) in GeV,
 *                structure of arrays: component c of particle i of event e at
 *                (c * n_part + i) * n_events + e.
 *   w_dev      : device [n_events] FP64 phase-space weights, GeV^(2 n_part - 4)
 *                with the measure (2 pi)^4 delta^4(P - sum p) prod d^3p/((2 pi)^3 2E).
 * n_events = 0 is a no-op.  VGX_EINVAL on bad sizes, masses or sqrt_s. */
vgx_status rambo_generate(int32_t n_part, const double* masses, double sqrt_s, uint64_t seed, uint32_t stream_id,
                          uint32_t iteration, int64_t first, int64_t n_events, double* mom_dev, double* w_dev,
                          void* stream);

/* Acceptance-rejection unweighting (sync: returns the count).  Thesis: MC
 * chapter, acceptance-rejection paragraph; MadFlow chapter, unweighted event
 * exporter (keep an event when its weight exceeds a uniform number times the
 * largest weight).  Event e is kept when w_e > r_e w_max, r_e the first
 * word of Philox block 0xFF of sample e for (seed, stream_id, iteration),
 * as a uniform.  No sampler of this library uses block 0xFF (VEGAS and the
 * flow use blocks 0..2, RAMBO blocks 0..n_part-1), so r_e is never one of the
 * numbers that made event e, even with the weights' own seed, stream and
 * iteration.
 *   w_dev      : device [n] FP64 weights; NaN and w <= 0 are never kept.
 *   w_max      : > 0: the bound to use (efficiency w/w_max); 0: the largest
 *                weight of the sample, found on the device.
 *   idx_dev    : device [n] int64; the kept indices in ascending order fill
 *                its first *n_kept entries.
 *   w_max_used : host, may be NULL: the bound used.
 * Allocates a stream-ordered scratch of about n/8 + n/512 bytes (one keep
 * bit and one 8-byte count per 4096 events) plus 8 bytes per workgroup of
 * the max search (at most 8 per CU), freed before the call returns.
 * n = 0 is a no-op. */
vgx_status unweight(int64_t n, const double* w_dev, double w_max, uint64_t seed, uint32_t stream_id,
                    uint32_t iteration, int64_t* idx_dev, int64_t* n_kept, double* w_max_used, void* stream);

/* Allocation-free unweighting, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the operation, arguments, results and errors of
 * unweight(), with its scratch (block maxima, block counts, keep masks) in
 * a fixed device array of VGX_UNWEIGHT_STATIC_BYTES that the library holds
 * on every GPU it runs on until the process ends; no allocation, no free.
 * n is limited to VGX_UNWEIGHT_NOALLOC_MAX events (one keep bit per event
 * and 8 bytes per 4096 events must fit): VGX_EINVAL beyond, nothing
 * launched.  All calls on one GPU share its array and leave their contents
 * in it: calls that overlap in time on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  Sync (a 16-byte read-back). */
#define VGX_UNWEIGHT_STATIC_BYTES (8 << 20)
#define VGX_UNWEIGHT_NOALLOC_MAX 65945600LL
vgx_status unweight_noalloc(int64_t n, const double* w_dev, double w_max, uint64_t seed, uint32_t stream_id,
                            uint32_t iteration, int64_t* idx_dev, int64_t* n_kept, double* w_max_used,
                            void* stream);

/* Asynchronous LHE 3.0 export (thesis MadFlow chapter, unweighted event
 * exporter: events written as Les Houches Event records by a CPU thread
 * separate from the device work).  A writer owns a file and one thread;
 * batches are queued and written in the order they were queued. */
typedef struct vgx_lhe vgx_lhe;

typedef struct {            /* the <init> block (Les Houches accord)          */
  int32_t beam_id[2];       /* IDBMUP: PDG codes of the beams                 */
  double beam_energy[2];    /* EBMUP (GeV)                                    */
  int32_t pdf_group[2];     /* PDFGUP                                         */
  int32_t pdf_set[2];       /* PDFSUP                                         */
  int32_t weight_mode;      /* IDWTUP (3: unweighted events, weight +XWGTUP)  */
  double xsec, xsec_err;    /* XSECUP, XERRUP (pb)                            */
  double xmax;              /* XMAXUP                                         */
  int32_t proc_id;          /* LPRUP                                          */
} vgx_lhe_init;

typedef struct {            /* per-batch event-line fields                    */
  double sqrt_s;            /* partonic centre-of-mass energy (GeV): the two
                               incoming partons are massless along +z and -z
                               with energy sqrt_s/2 each                      */
  double weight;            /* XWGTUP                                         */
  double scale;             /* SCALUP (GeV)                                   */
  double aqed, aqcd;        /* AQEDUP, AQCDUP                                 */
  int32_t proc_id;          /* IDPRUP                                         */
} vgx_lhe_event_info;

/* Open `path` for writing and write the header and <init> block (sync).
 * VGX_EINVAL if the file cannot be written. */
vgx_status lhe_open(const char* path, const vgx_lhe_init* init, vgx_lhe** out);

/* Queue the kept events of a batch (async on `stream`; never synchronises
 * it).  mom_dev is a rambo_generate output [4][n_part][n_total]; idx_dev
 * (device [n_kept] int64, e.g. from unweight; NULL: events 0..n_kept-1) lists
 * the events to write.  The events are gathered on the device into a stream-
 * ordered scratch, copied to a pooled pinned host buffer, and formatted by
 * the writer thread once the copy has completed; device buffers may be reused
 * as soon as later work on `stream` is ordered after this call.
 *   pdg_in  : host [2] PDG codes of the incoming partons.
 *   pdg_out : host [n_part] PDG codes; masses: host [n_part] (PUP5, GeV).
 * Particle lines carry colour 0 0 (not computed) and helicity 9 (unknown).
 * Momenta are written with 17 significant digits (exact round trip). */
vgx_status lhe_write_events(vgx_lhe* w, int32_t n_part, const int32_t* pdg_in, const int32_t* pdg_out,
                            const double* masses, const vgx_lhe_event_info* info, int64_t n_total,
                            const double* mom_dev, const int64_t* idx_dev, int64_t n_kept, void* stream);

/* Queue n events from host memory: mom_host [n][n_part][4] (E, px, py, pz),
 * copied before the call returns. */
vgx_status lhe_write_events_host(vgx_lhe* w, int32_t n_part, const int32_t* pdg_in, const int32_t* pdg_out,
                                 const double* masses, const vgx_lhe_event_info* info, int64_t n,
                                 const double* mom_host);

/* Wait until every queued event is written (sync); *written = events written
 * so far (may be NULL). */
vgx_status lhe_flush(vgx_lhe* w, int64_t* written);

/* Write the queue out, close the document and the file, free the writer. */
vgx_status lhe_close(vgx_lhe* w);

/* ------------------------------------------------------------------------ */
/* Batched integration: many contexts, one persistent launch per iteration    */
/* ------------------------------------------------------------------------ */
typedef struct vgx_batch vgx_batch;

/* Bundle contexts (all on one device, no hadronic kinds) into a batch.  Each
 * integral is plain VEGAS as above (MC chapter, VEGAS section); the batch is
 * a scheduling object the thesis does not have (its tools run one integral
 * per graph).  The batch
 * captures one iteration (persistent kernel + reductions + refinement) in
 * a HIP graph on first use.  tile = samples per work item (0: autotuned),
 * block = threads per workgroup (0: autotuned). */
vgx_status batch_create(vgx_vegas* const* ctxs, int32_t count, const int64_t* n_samples_host,
                        int32_t tile, int32_t block, void* stream, vgx_batch** out);

/* One iteration of every integral (sync), refining every grid afterwards.
 * out_host may be NULL; else [count] results. */
vgx_status batch_iterate(vgx_batch* b, int32_t iteration, vgx_iter_result* out_host);

/* Chosen tile / block after autotuning. */
vgx_status batch_config(vgx_batch* b, int32_t* tile, int32_t* block);

void batch_destroy(vgx_batch* b);

/* ------------------------------------------------------------------------ */
/* Coupling-flow proposal (neural importance sampling)                       */
/* ------------------------------------------------------------------------ */
typedef struct vgx_flow vgx_flow;

/* Number of FP32 parameters of a flow.  Masks: layer l transforms the dims
 * B_l = { j : bit k of j == (l even) }, k = (l/2) mod ceil(log2 dim),
 * conditioned on the others A_l.  Per layer, in this order: W1 [H][|A|],
 * b1 [H], W2 [H][H], b2 [H], W3 [|B| K][H], b3 [|B| K] (row-major).
 * Supported: dim 2..VGX_MAX_DIM, n_bins = 32, hidden = 64, n_layers 1..8. */
int64_t flow_num_params(int32_t dim, int32_t n_layers, int32_t n_bins, int32_t hidden);

/* Dimension and parameter count of a flow (either may be NULL). */
vgx_status flow_shape(const vgx_flow* f, int32_t* dim, int64_t* n_params);

/* Parameter segments of a flow, in the flat order (host-only, no device
 * work): for each segment its kind (0 = hidden weight matrix, 1 = hidden
 * bias, 2 = output-layer weight or bias, which an identity initialisation
 * sets to zero), its fan-in and its size.  At most cap segments are
 * written; *n_seg receives the total (6 per layer). */
vgx_status flow_param_layout(int32_t dim, int32_t n_layers, int32_t n_bins, int32_t hidden, int32_t* kind_host,
                             int32_t* fan_in_host, int64_t* size_host, int32_t cap, int32_t* n_seg);

/* Create a flow with the given FP32 initial parameters (sync copy).  The
 * caller supplies the initial weights (e.g. He-normal hidden layers and a
 * zero output layer, the identity map); the thesis's dense layer
 * y = phi(W x + b) and activation table (deep-learning chapter, "Neural
 * networks") define the networks. */
vgx_status flow_create(int32_t dim, int32_t n_layers, int32_t n_bins, int32_t hidden,
                       const float* params_host, int64_t n_params, void* stream, vgx_flow** out);

/* Operand precision of the flow's matrix products (sync).  VGX_OPERANDS_BF16
 * (the default) is the product path: BF16 weights and activations on
 * v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  VGX_OPERANDS_F32 is a
 * validation mode running the same kernels and tile structure with FP32
 * operands (v_mfma_f32_32x32x2_f32), so that densities and every gradient
 * element can be compared with the FP64 oracle at FP32 rounding.  The
 * network definition is the thesis's dense layer y = phi(W x + b)
 * (deep-learning chapter, "Neural networks").  The FP32 mode keeps all
 * layers' weights in LDS like the BF16 one, at twice the bytes: VGX_EINVAL
 * if they do not fit (dimensions above 4 with four layers); the mode is
 * then unchanged.  Training scratch is reallocated on the next training
 * call; the master weights and Adam moments are kept. */
vgx_status flow_set_operands(vgx_flow* f, int32_t operands);

/* Draw n points from the flow (async).  Thesis: MC chapter, importance
 * sampling (points from the proposal q together with ln q, so that
 * w = f/q keeps eq. mc_est_is unbiased) and the inverse transform method
 * (each coupling inverts a piecewise-linear CDF).  u from Philox (counter (i,
 * iteration, stream_id | 2^23, block), key seed), sampling direction
 * (inverse piecewise-linear CDFs, layers L-1..0) -> y_dev [dim][n] and
 * logq_dev [n] = ln q(y). */
vgx_status flow_sample(vgx_flow* f, int64_t n, uint64_t seed, uint32_t stream_id, int32_t iteration,
                       double* y_dev, double* logq_dev, void* stream);

/* Draw n points from the flow and add their importance-sampling estimate to
 * the VEGAS context, in one pass with no points in memory (sync).  Thesis:
 * MC chapter, eq. mc_est_is with the proposal p = q times the grid's density
 * (as vegas_iterate_points): w = f(G(y)) J_G(y) / q(y).  The points are
 * those flow_sample(f, n, seed, stream_id, iteration) draws, so the estimate
 * equals vegas_iterate_points on them up to the order of the sums.  Needs
 * the flow's dimension equal to the context's (2..8), BF16 operands, and the
 * flow's weights and the integrand's tables together within the LDS of a CU
 * (VGX_EINVAL otherwise).  Runs on the context's stream after the work
 * enqueued on the flow's stream; records and judges the estimate as
 * vegas_iterate_points does with logq (VGX_EFALLBACK, VGX_ENUMERIC); out_host
 * may be NULL. */
vgx_status flow_vegas_iterate(vgx_flow* f, vgx_vegas* v, int64_t n, uint64_t seed, uint32_t stream_id,
                              int32_t iteration, vgx_iter_result* out_host);

/* Density direction (async): y_dev [dim][n] -> u_dev [dim][n] (may be NULL),
 * logq_dev [n]. */
vgx_status flow_density(vgx_flow* f, int64_t n, const double* y_dev, double* u_dev, double* logq_dev,
                        void* stream);

/* Loss and gradient.  Thesis: MC chapter, eq. var_is (the variance of the
 * importance-sampling estimate is the second moment of f/p less I^2, so
 * minimising mean(g^2/q) minimises it); deep-learning chapter, learning by
 * gradient descent on a loss (eq. sgd).  Loss L = mean(g^2/q)/mean(g^2) over the batch (y_dev [dim][n] uniform
 * points of the unit cube, g_dev [n]) and its gradient (sync).  grad_host
 * [n_params] may be NULL. */
vgx_status flow_loss_grad(vgx_flow* f, int64_t n, const double* y_dev, const double* g_dev,
                          double* loss_host, float* grad_host);

/* One training step.  Thesis: "Optimization methods" (the Adam update
 * equations and their default constants).  Loss and gradient as above, then Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, learning rate lr) on the FP32 master weights.
 * loss_host may be NULL (then async).  VGX_EFALLBACK if the loss is not
 * finite (the weights are then left unchanged). */
vgx_status flow_train_step(vgx_flow* f, int64_t n, const double* y_dev, const double* g_dev,
                           float lr, double* loss_host);

/* Adam alone on a given gradient (async; for tests): grad_dev [n_params].
 * Thesis: "Optimization methods", the Adam equations. */
vgx_status flow_adam(vgx_flow* f, const float* grad_dev, float lr);

vgx_status flow_get_params(vgx_flow* f, float* params_host, int64_t cap, int64_t* n_params);
vgx_status flow_set_params(vgx_flow* f, const float* params_host, int64_t n_params);
void flow_destroy(vgx_flow* f);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif
#endif /* VGX_H */
