/*
 * FP64 CPU oracle for the per-object shape pipeline of Li, Xin & Cui (2012),
 * "Fast Shape Estimation for Galaxies and Stars".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, includes or calls
 * this code; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no source with the HIP path.
 *
 * Conventions: pixel (row i, col j) has centre (x, y) = (j, i); a stamp is a
 * side x side row-major array of doubles; parameters are
 * p = (x0, y0, e1, e2, Re, n, I0, sky) (Moffat: slots 4, 5 = rd, beta).
 */
#ifndef SHAPE_ORACLE_H
#define SHAPE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status bits (same meaning as the library's, defined independently) */
#define ORC_CONVERGED        0x001u
#define ORC_MAX_ITER         0x002u
#define ORC_STALLED          0x004u
#define ORC_SINGULAR         0x008u
#define ORC_NONFINITE_INPUT  0x010u
#define ORC_NONPOSITIVE_FLUX 0x020u
#define ORC_AT_BOUND         0x040u  /* the fit ended on the edge of the parameter box */
#define ORC_G_CLAMPED        0x080u
#define ORC_BAD_INPUT        0x100u
#define ORC_LOST             0x200u

#define ORC_SERSIC 0
#define ORC_MOFFAT 1
#define ORC_MOFFAT_BETA 2   /* star estimator only: Moffat with beta fixed */

typedef struct {
  int      max_iter_centroid;  /* cap on centroid steps (Sec. 4.1: 20) */
  int      max_iter_moments;   /* cap on joint centroid+ellipticity steps (20) */
  int      max_iter_lm;        /* cap on LM trials */
  double   k_gain;             /* centroid gain k (Sec. 2: 0.75) */
  double   tol_x;              /* centroid stop: max |dx|,|dy| in px */
  double   tol_g;              /* ellipticity stop: max |dg_i| */
  double   gmax;               /* step-halving bound on |g_w| */
  double   tol_lm;             /* LM stop: max_k |delta_k| / s_k of an accepted step */
  double   lambda0;            /* initial Marquardt damping */
  double   chi2_rtol;          /* accept a trial if chi2' <= chi2 (1 + chi2_rtol) */
  double   n0;                 /* initial Sersic index */
  double   moffat_beta;        /* fixed Moffat index for stars */
  uint32_t free_mask;          /* bit k set => p[k] is fitted */
  int      linear_init;        /* 1: profile free (I0, sky) out linearly at every point;
                                  0: search them with the shape by LM (linear start) */
} orc_opts;

void orc_default_opts(orc_opts* o);

/* Sersic b(n): root of P(2n, b) = 1/2 (regularised lower incomplete gamma). */
double orc_sersic_b(double n);
/* db/dn by Richardson-extrapolated central differences of orc_sersic_b. */
double orc_sersic_db(double n);
/* Regularised lower incomplete gamma P(a, x). */
double orc_gamma_p(double a, double x);

/* Model m and Jacobian dm/dp (J may be NULL), point-sampled on a side^2 grid. */
void orc_model(int side, const double* p, int kind, double* m, double* J);

/* Border-mean sky, brightest pixel, growth-curve r50, total flux. */
void orc_init(const double* img, int side, double* sky0, int* imax, double* r50,
              double* flux, double* sigw, uint32_t* status);

/* Circular-weight centroid from (x, y) (Sec. 2). */
void orc_centroid(const double* img, int side, double sky0, double sigw,
                  const orc_opts* o, double* x, double* y, int* iters, uint32_t* status);

/* One evaluation of the elliptical-weight KSB quantities (Sec. 3, App. A, B)
 * at centre (xc, yc) and weight ellipticity gw.  out (20 doubles):
 *  [0]  N = sum f W        [1..2] sum f W theta_i      [3] T = Q11 + Q22
 *  [4..5] e_obs            [6..9] X^SH (row-major)     [10..11] e^SH
 *  [12..15] Delta X^SH     [16..17] Delta e^SH         [18..19] unused (0) */
void orc_ksb_terms(const double* img, int side, double sky0, double sigw,
                   double xc, double yc, const double* gw, double* out);

/* Starting size for the profile fit from the weighted second moment at the
 * given centre and weight ellipticity (a reading: see oracle.c); NaN when
 * undefined. */
double orc_size(const double* img, int side, double sky0, double sigw, double xc, double yc,
                const double* gw);

/* Joint centroid + ellipticity iteration (Sec. 2, 3).  out: x0, y0, e1, e2, sigw, r50, and
 * orc_size at the centre and g_w of the last evaluated step. */
void orc_moments(const double* img, int side, double sky0, double sigw, double r50,
                 double x_in, double y_in, const orc_opts* o, double* out,
                 int* iters, uint32_t* status);

/* Linear (I0, sky) at fixed shape (eq. for I0 in Sec. 4.1, with a sky column). */
void orc_linear(const double* img, int side, const double* p, int kind,
                double* i0, double* sky);
/* Same for a subset of the amplitudes: bit 6 = I0, bit 7 = sky. */
void orc_linear_subset(const double* img, int side, const double* p, int kind,
                       uint32_t which, double* i0, double* sky);

/* chi^2 (eq. chi2), gradient d chi^2/dp and J^T J / sigma^2 (36 packed upper). */
double orc_chi2(const double* img, int side, double sigma, const double* p, int kind,
                double* grad, double* jtj);

/* Levenberg-Marquardt fit of the free parameters from p_init. */
void orc_fit(const double* img, int side, double sigma, int kind, const double* p_init,
             const orc_opts* o, double* p_out, double* chi2, int* iters,
             uint32_t* status, double* perr);

/* Star size from weighted moments (Sec. 4.2): kind ORC_SERSIC = Gaussian star,
 * ORC_MOFFAT = Moffat star, ORC_MOFFAT_BETA = Moffat star with beta fixed at
 * beta_fixed (ignored otherwise); w0 = starting weight width; out[6] =
 * (sigma or rd, beta, I0, r0, r2, r4). */
void orc_star_moments(const double* img, int side, double sky, double xc, double yc,
                      const double* g, int kind, double beta_fixed, double w0, double tol,
                      int max_iter, double* out, int* iters, uint32_t* status);

/* Whole pipeline over a batch, OpenMP over stamps.  Returns threads used.
 * pixels: FP64 packed stamps; offsets/sides/sigma/model per stamp.
 * Outputs per stamp: xy[2] (centroid), mom[7], p[8], chi2, perr[8] (may be NULL:
 * sqrt(diag((J^T J / sigma^2)^-1)) over the fitted parameters at the result),
 * iters[3], status[3]; the fit of a Sersic stamp starts at Re = mom[6] when it
 * is finite, else r50. */
int orc_pipeline(int64_t n, const double* pixels, const int64_t* offsets,
                 const int32_t* sides, const float* sigma, const uint8_t* model,
                 const orc_opts* o, double* xy, double* mom, double* p,
                 double* chi2, double* perr, int32_t* iters, uint32_t* status, int threads);

/* Front end on a whole H x W frame (Sec. 4.1, starting point): border-mean
 * sky, brightest pixel, growth-curve r50 about it, and the cut-out square
 * box = (x origin, y origin, side) with side = round(6 r50) clamped to
 * [4, min(max_side, H, W)], placed around the peak inside the frame. */
void orc_frame_detect(const double* img, int H, int W, int max_side, double* sky0,
                      double* r50, double* flux, int* peak_x, int* peak_y, int* box,
                      uint32_t* status);

/* Star sizes over a batch (Sec. 4.2), OpenMP over stamps; returns threads
 * used.  Per stamp: starting estimates, centroid, joint centre + ellipticity,
 * then orc_star_moments of the given kind (beta_fixed for ORC_MOFFAT_BETA);
 * out[6] as there, iters, status. */
int orc_star_pipeline(int64_t n, const double* pixels, const int64_t* offsets,
                      const int32_t* sides, const orc_opts* o, int kind, double beta_fixed,
                      double tol, int max_iter, double* out, int32_t* iters, uint32_t* status,
                      int threads);

#ifdef __cplusplus
}
#endif
#endif
