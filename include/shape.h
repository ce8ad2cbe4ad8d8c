/*
 * libshape: batched shape measurement of galaxies and stars on AMD MI355X
 * (gfx950), after Li, Xin & Cui (2012), "Fast Shape Estimation for Galaxies
 * and Stars" (arXiv:1203.0571).
 *
 * Three stages, each one call over a batch of square postage stamps:
 *   shape_centroid    starting estimates and the Gaussian-weighted centroid
 *                     (Sec. 2; starting point of Sec. 4.1)
 *   shape_moments     joint centroid + ellipticity with an elliptical weight
 *                     (Sec. 3, App. A, App. B)
 *   shape_fit_sersic  chi^2 fit of the remaining profile parameters with the
 *                     amplitudes solved analytically (Sec. 4.1, eqs. ser,
 *                     chi2 and the dchi2/dI0 = 0 normalisation)
 * plus the chi^2 of a given parameter set and its gradient (for automatic
 * differentiation and for driving the fit from outside).
 *
 * Conventions
 *   - Stamps are square, side W in [4, 128], row-major; pixel (row i, col j)
 *     has centre (x, y) = (j, i).
 *   - Parameters p = (x0, y0, e1, e2, Re, n, I0, sky).  The model is
 *       u = (x - x0, y - y0),  v = S(e) u,  S(e) = [[1-e1, -e2], [-e2, 1+e1]],
 *       R^2 = max(|v|^2 / (1 - |e|^2), 1e-8),
 *       Sersic: m = I0 exp(-b(n) (R/Re)^(1/n)) + sky, b(n) the half-light
 *               constant (P(2n, b) = 1/2);
 *       Moffat (stars, model = 1): m = I0 (1 + R^2/rd^2)^(-beta) + sky with
 *               rd in slot 4 and beta in slot 5 (held fixed).
 *     (e1, e2) is the reduced-shear ellipticity g of the paper:
 *     |e| = (a - b)/(a + b); e1 > 0 is elongated along x, e2 > 0 along y = x.
 *     Re is the circularised half-light radius.
 *   - All arrays passed to the stage calls are DEVICE pointers owned by the
 *     caller; the library allocates nothing.  Calls are asynchronous on
 *     `stream` (a hipStream_t; NULL = the default stream): SHAPE_OK means the
 *     work was enqueued, outputs are valid after the stream is synchronised.
 *   - Host-checkable argument errors return SHAPE_EINVAL before any launch;
 *     HIP launch errors return SHAPE_EDEVICE.  Problems with one stamp (side
 *     out of range, sigma <= 0, offset outside the pixel buffer, NaN/Inf
 *     pixels) never fail the call: they set that stamp's status bits and its
 *     outputs to NaN.  n = 0 is a no-op returning SHAPE_OK.
 *   - Reentrant; no global mutable state except the static workspace of
 *     shape_fit_queue_static (see there).
 */
#ifndef SHAPE_H
#define SHAPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHAPE_ABI_VERSION 2

typedef enum {
  SHAPE_OK = 0,
  SHAPE_EINVAL = -1,       /* bad argument (checked on the host) */
  SHAPE_EDEVICE = -2,      /* HIP API or launch failure */
  SHAPE_ENOMEM = -3,       /* workspace too small */
  SHAPE_EUNSUPPORTED = -4  /* valid but not implemented (e.g. a free mask) */
} shape_status;

typedef enum { SHAPE_F32 = 0, SHAPE_F16_SCALED = 1 } shape_dtype;
typedef enum { SHAPE_SERSIC = 0, SHAPE_MOFFAT = 1 } shape_model;

/* Per-stamp status bits (uint32 per stamp and stage). */
#define SHAPE_ST_CONVERGED        0x001u /* stopping rule met */
#define SHAPE_ST_MAX_ITER         0x002u /* iteration cap reached */
#define SHAPE_ST_STALLED          0x004u /* LM damping exceeded 1e10 */
#define SHAPE_ST_SINGULAR         0x008u /* a 2x2 or normal-equation solve failed */
#define SHAPE_ST_NONFINITE_INPUT  0x010u /* NaN/Inf pixel */
#define SHAPE_ST_NONPOSITIVE_FLUX 0x020u /* total or weighted flux <= 0, or I0 <= 0 */
#define SHAPE_ST_AT_BOUND         0x040u /* the fit ended on the edge of the parameter
                                            box (see shape_fit_sersic) */
#define SHAPE_ST_G_CLAMPED        0x080u /* an ellipticity step was halved */
#define SHAPE_ST_BAD_INPUT        0x100u /* side, sigma, model or offset invalid */
#define SHAPE_ST_LOST             0x200u /* the centre left the stamp */

/* Per-stamp record written by shape_centroid and shape_moments (9 floats). */
enum {
  SHAPE_REC_X0 = 0, SHAPE_REC_Y0 = 1, SHAPE_REC_E1 = 2, SHAPE_REC_E2 = 3,
  SHAPE_REC_SIGW = 4, SHAPE_REC_R50 = 5, SHAPE_REC_SKY0 = 6, SHAPE_REC_FLUX = 7,
  SHAPE_REC_SIZE = 8,
  SHAPE_REC_LEN = 9
};

typedef struct {
  const void*    pixels;   /* device: packed stamps (float, or _Float16 x scale) */
  const int64_t* offset;   /* device [n]: element offset of each stamp; NULL =>
                              stamp i starts at i * side0 * side0 */
  const int32_t* side;     /* device [n]: side of each stamp; NULL => side0 */
  const float*   scale;    /* device [n]: dequantisation scale (F16 only) */
  const float*   sigma;    /* device [n]: i.i.d. pixel noise sigma, > 0 */
  const uint8_t* model;    /* device [n]: shape_model; NULL => all Sersic */
  int64_t        n;        /* number of stamps, >= 0 */
  int64_t        n_pixels; /* elements in `pixels` (every stamp must lie inside) */
  int32_t        side0;    /* uniform side when `side` is NULL */
  int32_t        dtype;    /* shape_dtype */
} shape_batch;

typedef struct {
  int32_t  max_iter_centroid; /* centroid steps (Sec. 4.1: 20) */
  int32_t  max_iter_moments;  /* joint centroid + ellipticity steps (20) */
  int32_t  max_iter_lm;       /* LM trials, every trial counts (30) */
  uint32_t free_mask;         /* bit k => p[k] fitted; 0xFF all eight, 0xF0 =
                                 (Re, n, I0, sky) with centre and e held */
  double   k_gain;            /* centroid gain k (Sec. 2: 0.75) */
  double   tol_x;             /* centroid stop: max |step| in px (1e-4) */
  double   tol_g;             /* ellipticity stop: max |dg_i| (1e-5) */
  double   gmax;              /* bound on |g_w| and |e| (0.95) */
  double   tol_lm;            /* LM stop: a step with max_k |d_k|/s_k < tol_lm (1e-5),
                                 s = (1, 1, 1, 1, Re, n); at damping lambda <= 1e-3 the
                                 fit ends where the step begins (no sweep for it), at
                                 larger damping once the step is accepted */
  double   lambda0;           /* initial Marquardt damping (1e-3) */
  double   chi2_rtol;         /* accept a trial if chi2' <= chi2 (1 + rtol) (1e-6) */
  double   n0;                /* starting Sersic index (1) */
  double   moffat_beta;       /* fixed Moffat index (3) */
  int32_t  linear_init;       /* 1: profile the free (I0, sky) at every evaluated shape
                                 (the paper's split, Sec. 4.1; default); 0: search them
                                 with the shape by the same LM from their linear optimum
                                 at the start (shape_fit_sersic with free_mask 0xF0 and
                                 no model array only, else SHAPE_EUNSUPPORTED) */
  int32_t  reserved;
  double   tol_sigma;         /* LM stop, also: a step at damping lambda <= 1e-3 with
                                 d^T (A / sigma^2) d < tol_sigma^2, A the (profiled,
                                 damped) normal matrix, i.e. every fitted parameter would
                                 move by less than tol_sigma times its standard error;
                                 the fit ends where the step begins, with no sweep for
                                 it (1e-4; 0 turns this rule off) */
} shape_opts;

/* Fill `opts` with the defaults above.  Returns SHAPE_EINVAL if opts is NULL. */
int shape_default_opts(shape_opts* opts);

/* Static description of a status code (never NULL). */
const char* shape_status_string(int code);

/* ABI version of the loaded library (SHAPE_ABI_VERSION). */
int shape_abi_version(void);

/*
 * Starting estimates and circular-weight centroid (Sec. 2; Sec. 4.1 starting
 * point).  Per stamp: sky0 = mean of the border pixels; the brightest pixel
 * (lowest index on ties); r50 = first crossing of half the total sky-subtracted
 * flux by the growth curve over integer-radius rings about that pixel, linearly
 * interpolated; sigma_w = clamp(r50 / sqrt(2 ln 2), 1, W/4); then from the
 * brightest pixel, steps centre += (sum f W theta) / (k sum f W) with
 * W = exp(-|theta|^2 / 2 sigma_w^2), f = I - sky0, until both steps are below
 * tol_x or max_iter_centroid steps.
 *   rec    [n][9] out: x0, y0, 0, 0, sigma_w, r50, sky0, total flux, NaN
 *   iters  [n] out, status [n] out (SHAPE_ST_*)
 */
int shape_centroid(const shape_batch* batch, const shape_opts* opts, float* rec,
                   int32_t* iters, uint32_t* status, void* stream);

/*
 * Joint centroid + ellipticity (Sec. 3, App. A, App. B).  From g_w = 0 and
 * the centroid in rec_in, each step forms the elliptical-weight moments
 * (weight W(R^2) with R^2 = |S(g_w) theta|^2, App. A), the polarisability
 * P = X^SH + dX^SH - e_obs (x) (e^SH + de^SH), and updates
 * g_w += (1 - |g_w|^2) P^-1 (e_obs - 2 g_w / (1 + |g_w|^2)) (eq. newg),
 * halving the step while |g_w| > gmax, and centre += (sum f W theta)/(k sum f W).
 * Stops when the centre moves less than tol_x and g_w less than tol_g in a
 * step that was not halved.
 *   rec_in  [n][9] in (from shape_centroid), rec_out [n][9] out:
 *           x0, y0, e1, e2, sigma_w, r50, sky0, flux, size
 *   iters, status [n] out.  rec_in == rec_out is allowed.  A record with a
 *   non-finite field other than size gives SHAPE_ST_BAD_INPUT.
 * size (the profile fit's starting Re; not from the paper): with the last
 * step's weight, q = sum f W R^2 / sum f W is the weighted second moment of a
 * Gaussian source exp(-R^2 / 2 s^2) when s^2 = q sigma_w^2 / (2 sigma_w^2 - q);
 * size = s sqrt(2 ln 2) / sqrt(1 - |g_w|^2), that source's half-light radius
 * along the model's elliptical radius; NaN unless sum f W > 0 and
 * 0 < q < 1.96 sigma_w^2.
 */
int shape_moments(const shape_batch* batch, const shape_opts* opts, const float* rec_in,
                  float* rec_out, int32_t* iters, uint32_t* status, void* stream);

/*
 * Profile fit (Sec. 4.1).  Minimises chi^2 = sum ((m - I)/sigma)^2 over the
 * parameters in free_mask by Levenberg-Marquardt; free amplitudes (I0, sky)
 * are set to their linear optimum at every evaluated point (the dchi2/dI0 = 0
 * condition), the step solves (M + lambda diag M) d = J_N^T r with M the Schur
 * complement of the amplitude block of J^T J, in FP64 on the device.  Moffat
 * stamps (model = 1) are fitted with beta fixed at opts->moffat_beta.
 *   p_init [n][8] in, or NULL: start from rec (x0, y0, e1, e2 of the moments,
 *          Re = the record's size, or r50 where it is NaN (Moffat: the
 *          rd of half-light radius r50, r50 / sqrt(2^(1/(beta-1)) - 1)), n = n0)
 *   rec    [n][9] in (from shape_moments), used when p_init is NULL
 *   p_out  [n][8] out; chi2 [n] out; perr [n][8] out or NULL (sqrt of the
 *          diagonal of (J^T J / sigma^2)^-1 over the fitted parameters)
 *   iters, status [n] out; iters counts LM trials (every trial counts).
 *   sweeps [n] out or NULL: pixel sweeps done (the starting point's plus one
 *          per trial that passed the box check; the amplitude-only start
 *          sweep is not counted) -- the unit of work for throughput figures.
 * Returns SHAPE_EUNSUPPORTED for free masks other than 0xFF and 0xF0.
 */
int shape_fit_sersic(const shape_batch* batch, const shape_opts* opts, const float* p_init,
                     const float* rec, float* p_out, float* chi2, float* perr,
                     int32_t* iters, uint32_t* status, int32_t* sweeps, void* stream);

/*
 * chi^2 of given parameters (Sec. 4.1, eq. chi2): chi2[i] = sum over the
 * pixels of stamp i of ((d - m(p_i)) / sigma_i)^2, m the model above (Moffat
 * stamps read beta from slot 5).
 *   params [n][8] in (device), chi2 [n] out.
 * Non-finite parameters give NaN for that stamp.
 */
int shape_chi2_fwd(const shape_batch* batch, const float* params, float* chi2, void* stream);

/*
 * Gradient of chi^2 by the adjoint of the render: with r = (d - m)/sigma the
 * adjoint of a pixel is -(2/sigma) r dL/dchi2 and grad_p[i][k] =
 * sum over pixels of that adjoint times dm/dp_k (all eight parameters).
 *   params    [n][8] in
 *   grad_chi2 [n] in, the upstream dL/dchi2 per stamp, or NULL for 1
 *   chi2      [n] out or NULL
 *   grad_p    [n][8] out
 *   jtj       [n][36] out or NULL: J^T J / sigma^2, upper triangle row by row
 *   jtr       [n][8] out or NULL: J^T (d - m) / sigma^2 (the LM right-hand side)
 */
int shape_chi2_bwd(const shape_batch* batch, const float* params, const float* grad_chi2,
                   float* chi2, float* grad_p, float* jtj, float* jtr, void* stream);

/*
 * The chain rule after the adjoint: the gradient above is linear in the
 * upstream dL/dchi2 (Sec. 4.1, eq. chi2: chi^2 is the only function of the
 * pixels it scales), so a caller that took grad_unit from shape_chi2_bwd with
 * grad_chi2 = NULL (dL/dchi2 = 1; a forward pass that also takes the
 * gradient) forms grad_p[i][k] = grad_chi2[i] * grad_unit[i][k] later
 * without another sweep.
 *   grad_unit [n][8] in (device), grad_chi2 [n] in or NULL (a copy),
 *   grad_p [n][8] out; grad_p may equal grad_unit (in place).
 * Returns SHAPE_EINVAL for n < 0 or a missing array (n > 0).
 */
int shape_chi2_grad_scale(const float* grad_unit, const float* grad_chi2, int64_t n,
                          float* grad_p, void* stream);

/*
 * Star sizes from weighted moments (Sec. 4.2).  About the centre and
 * ellipticity in rec (from shape_moments), with R the elliptical radius of
 * the model and f = I - sky0, each step forms r0 = sum f W, r2 = sum f W R^2,
 * r4 = sum f W R^4 for the current weight width w and then
 *   profile 0, Gaussian star, W = exp(-R^2/2w^2): sigma = sqrt(r2/r0),
 *            I0 = r0/(pi sigma^2)  (Sec. 4.2.1);
 *   profile 1, Moffat star, W = (1 + R^2/w^2)^-3: beta = 1/(r4 r0/(2 r2^2) - 1),
 *            rd = sqrt(r2/r0 (beta + 1)), I0 = r0 (beta + 2)/(pi rd^2)  (Sec. 4.2.2);
 * sets w to the new size and repeats until the fractional change of the size
 * is below tol (the paper: 1e-4) or after max_iter steps (the paper: 20).
 * The weight starts at sigma_w of rec (Gaussian) or r50/sqrt(sqrt(2) - 1), the
 * beta = 3 Moffat whose half-light radius is the record's r50 (Moffat).
 * Precision: for tol >= 1e-5 the sums and the step run in FP32 (their
 * rounding, ~1e-7 relative, is far below such a tol); a smaller tol takes an
 * FP64 instance of the sums and the step (slower), since FP32 rounding would
 * keep the fractional change from falling below it.
 *   out [n][4] out: sigma or rd, beta (0 for Gaussian), I0, r0 of the last step
 *   iters, status [n] out.
 */
int shape_star_moments(const shape_batch* batch, int32_t profile, const float* rec, double tol,
                       int32_t max_iter, float* out, int32_t* iters, uint32_t* status,
                       void* stream);

/*
 * Moffat star sizes with beta fixed (Sec. 4.2.2: the paper's way out of the
 * rd-beta degeneracy and of the pixelation bias of faint stars is to measure
 * beta on bright stars and fix it for the others).  The same weight
 * W = (1 + R^2/w^2)^-3 and iteration as profile 1 of shape_star_moments, with
 * rd = sqrt(r2/r0 (beta + 1)) and I0 = r0 (beta + 2)/(pi rd^2) for the given
 * beta (r4 is not used, so the step cannot become singular).  The weight
 * starts at the rd whose half-light radius is the record's r50,
 * r50 / sqrt(2^(1/(beta-1)) - 1).
 *   beta in (1, 1e6]; out [n][4]: rd, beta, I0, r0; iters, status [n] out.
 * Same arguments, ownership and errors as shape_star_moments otherwise.
 */
int shape_star_moments_beta(const shape_batch* batch, double beta, const float* rec, double tol,
                            int32_t max_iter, float* out, int32_t* iters, uint32_t* status,
                            void* stream);

/* ------------------------------------------------------------------------
 * Work-queue form of shape_fit_sersic for large batches, uneven stamps (any
 * mix of sides and of Sersic / Moffat stamps) and callers that drive the LM
 * iteration themselves.  The same LM trials as the fused fit, with the same
 * results bit for bit, split into batched passes:
 *   shape_queue_start   orders the stamps largest side first (on the device),
 *                       forms every stamp's starting point and runs the
 *                       start sweeps (amplitudes, then the first full sweep);
 *   shape_queue_step    one LM trial of every still-active stamp: a persistent
 *                       sweep pass (waves pop stamps from atomic cursors and
 *                       render model, Jacobian, chi^2, J^T r, J^T J) and a
 *                       decide pass with one lane per stamp (amplitudes,
 *                       accept / reject, damped FP64 solve, next trial);
 *                       only the active stamps are visited;
 *   shape_queue_finish  writes the same outputs as shape_fit_sersic.
 * A step can be captured once into a hipGraph and replayed
 * (shape_queue_graph_*).  The caller owns the workspace (device memory of
 * shape_queue_workspace_bytes(n) bytes); the uint32 at byte offset 8,
 * `active`, counts the stamps still iterating after the last step and is
 * valid once the stream has synchronised.  max_iter_lm steps finish every
 * stamp.  Steps on one workspace must not overlap.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t team;           /* waves per stamp for stamps with side >= team_min_side: 1, 2, 4 */
  int32_t team_min_side;  /* threshold side for team processing (team > 1) */
  int32_t grid;           /* persistent workgroups of the sweep kernels; 0 = as many
                             as fit on the device (any count >= 1 drains every stamp:
                             a workgroup moves on to the next cursor when its own is
                             drained) */
  int32_t chunk;          /* stamps a wave (or team) takes from a cursor at most per
                             pop, 1 .. 64; 0 = 8.  Pops shrink towards one stamp as a
                             cursor's share runs out */
} shape_queue_cfg;

/* Defaults: team 1 (one wave per stamp), grid 0, chunk 0. */
int shape_queue_default_cfg(shape_queue_cfg* cfg);
/* Workspace bytes for n stamps (about 1.05 KB per stamp). */
int shape_queue_workspace_bytes(int64_t n, size_t* bytes);
/* Starting points (p_init [n][8] or, if NULL, the moments records rec [n][9]). */
int shape_queue_start(const shape_batch* batch, const shape_opts* opts, const shape_queue_cfg* cfg,
                      const float* p_init, const float* rec, void* ws, size_t ws_bytes,
                      void* stream);
/* One LM trial for every still-active stamp. */
int shape_queue_step(const shape_batch* batch, const shape_opts* opts, const shape_queue_cfg* cfg,
                     void* ws, size_t ws_bytes, void* stream);
/* Every still-active stamp finished in one persistent launch per model, one
 * wave per stamp: its pending trial, then LM trials until it converges,
 * stalls or reaches max_iter_lm (the results equal those of further steps).
 * For the end of a fit, when few stamps remain and a step would cost more
 * in launch and straggler time than in work.  Afterwards active = 0. */
int shape_queue_drain(const shape_batch* batch, const shape_opts* opts, const shape_queue_cfg* cfg,
                      void* ws, size_t ws_bytes, void* stream);
/* Outputs, as shape_fit_sersic (stamps still active are flagged MAX_ITER). */
int shape_queue_finish(const shape_batch* batch, const shape_opts* opts, void* ws,
                       size_t ws_bytes, float* p_out, float* chi2, float* perr, int32_t* iters,
                       uint32_t* status, int32_t* sweeps, void* stream);

/* A captured step: the batch, options, configuration and workspace are bound
 * at creation.  The handle is host memory owned by the library until
 * shape_queue_graph_destroy. */
typedef struct shape_queue_graph shape_queue_graph;
int shape_queue_graph_create(const shape_batch* batch, const shape_opts* opts,
                             const shape_queue_cfg* cfg, void* ws, size_t ws_bytes,
                             shape_queue_graph** graph);
int shape_queue_graph_launch(shape_queue_graph* graph, void* stream);
int shape_queue_graph_destroy(shape_queue_graph* graph);

/*
 * The work-queue fit in one call, with no allocation: for callers that cannot
 * allocate device memory (code under hipGraph/stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same inputs and outputs as
 * shape_fit_sersic plus the queue configuration; it runs shape_queue_start,
 * max_iter_lm steps (a step finds no work once every stamp is done) and
 * shape_queue_finish, with the workspace in a static device array of the
 * library (queue workspace of SHAPE_STATIC_MAX_STAMPS stamps, about 67 MB,
 * held on every device the library runs on until the process ends).  The
 * results equal those of the three calls with a caller's workspace.
 *   n > SHAPE_STATIC_MAX_STAMPS returns SHAPE_ENOMEM before any work.
 * The array is shared by every call on a device: calls that overlap on one
 * device (several streams or host threads) race and must be serialised by
 * the caller.  Its device address is looked up on the first call on each
 * device (hipGetSymbolAddress); make a first call outside stream capture.
 */
#define SHAPE_STATIC_MAX_STAMPS 65536
int shape_fit_queue_static(const shape_batch* batch, const shape_opts* opts,
                           const shape_queue_cfg* cfg, const float* p_init, const float* rec,
                           float* p_out, float* chi2, float* perr, int32_t* iters,
                           uint32_t* status, int32_t* sweeps, void* stream);

/* ------------------------------------------------------------------------
 * Front end on whole frames (Sec. 4.1, the paragraph on the starting point):
 * find the brightest pixel of each frame, estimate r50 by summing the pixels
 * outward from it until half the total flux, and cut the square of side
 * 6 r50 around it into a packed stamp batch for the calls above.
 * ------------------------------------------------------------------------ */
typedef struct {
  const void*  pixels;   /* [n][height][width] row-major frames (device); F32, or F16 with scale */
  const float* scale;    /* [n] F16 dequantisation scale; NULL for F32 */
  int64_t      n;        /* frames (>= 0) */
  int32_t      height;   /* 4 .. 4096 */
  int32_t      width;    /* 4 .. 4096 */
  int32_t      dtype;    /* shape_dtype */
  int32_t      reserved;
} shape_frames;

/*
 * Per frame: sky = mean of the border pixels; the brightest pixel (first
 * row-major index among equals); F = sum of (I - sky) over the frame; the
 * growth curve C(r) = sum of (I - sky) over pixels at distance <= r from the
 * brightest pixel, r = 1, 2, ..., with C(0) = 0, and r50 its first crossing
 * of F/2, linearly interpolated (min(H, W)/8 if F <= 0, status
 * SHAPE_ST_NONPOSITIVE_FLUX); then the square of side round(6 r50), clamped
 * to [4, min(max_side, H, W)], starting at the peak minus side/2 (integer
 * division) and shifted to lie inside the frame.  A frame with a NaN or Inf
 * pixel gets status SHAPE_ST_NONFINITE_INPUT, NaN info, peak (-1, -1) and an
 * empty box (side 0).
 *   max_side  in: 4 .. 128
 *   info  [n][3] out: sky, r50, F       peak [n][2] out: x, y of the brightest pixel
 *   box   [n][3] out: x0, y0, side      status [n] out
 * Errors: SHAPE_EINVAL for a NULL or out-of-range argument.
 */
int shape_frame_detect(const shape_frames* frames, int32_t max_side, float* info, int32_t* peak,
                       int32_t* box, uint32_t* status, void* stream);

/* Exclusive prefix sums of side^2 over box [n][3] (device): offset [n] of each
 * cut-out in the packed stamps, and total [1] = their sum (pixels to
 * allocate).  n = 0 writes total = 0. */
int shape_frame_offsets(const int32_t* box, int64_t n, int64_t* offset, int64_t* total,
                        void* stream);

/* Copy every box of every frame into stamps (FP32, F16 frames dequantised)
 * at offset[i]; stamps holds capacity floats (device).  sides [n] (optional,
 * may be NULL) receives each side, so (stamps, offset, sides) form a
 * shape_batch.  A box that does not lie inside its frame, or whose cut-out
 * would pass the capacity, copies nothing and gets side 0 (such a stamp is
 * then flagged BAD_INPUT by the stamp calls). */
int shape_frame_cut(const shape_frames* frames, const int32_t* box, const int64_t* offset,
                    float* stamps, int64_t capacity, int32_t* sides, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SHAPE_H */
