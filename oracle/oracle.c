/*
 * FP64 CPU oracle for the per-object shape pipeline of Li, Xin & Cui (2012),
 * "Fast Shape Estimation for Galaxies and Stars" (arXiv:1203.0571).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, step-by-step statement of what the
 * pipeline computes, used to check the HIP library.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or constant generator with the library.
 *
 * Every function below follows the passage cited in its comment.  Where the
 * paper is silent, the reading taken is stated at the function.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define R2_MIN 1e-8   /* floor on R^2 (px^2): keeps the Sersic cusp finite */
#define ORC_PI 3.14159265358979323846

void orc_default_opts(orc_opts* o) {
  o->max_iter_centroid = 20;   /* Sec. 4.1: at most 20 iterations */
  o->max_iter_moments = 20;
  o->max_iter_lm = 200;
  o->k_gain = 0.75;            /* Sec. 2: fixed gain k = 0.75 */
  o->tol_x = 1e-4;
  o->tol_g = 1e-5;
  o->gmax = 0.95;
  o->tol_lm = 1e-9;
  o->lambda0 = 1e-3;
  o->chi2_rtol = 1e-6;
  o->n0 = 1.0;
  o->moffat_beta = 3.0;
  o->free_mask = 0xFFu;
  o->linear_init = 1;
}

/* ------------------------------------------------------------------------ */
/* Incomplete gamma and the Sersic b(n) (Sec. 4.1, eq. ser: b is chosen so   */
/* that r_e is the half-light radius).  For I = I0 exp(-b (r/re)^(1/n)) the  */
/* flux inside r is proportional to P(2n, b (r/re)^(1/n)), so the half-light */
/* condition is P(2n, b) = 1/2.                                              */
/* ------------------------------------------------------------------------ */

/* P(a, x) from its power series (x < a + 1) or from the continued fraction
 * of Q(a, x) = 1 - P(a, x) (otherwise), the standard pair for the regularised
 * incomplete gamma function (e.g. Press et al., Numerical Recipes, 3rd ed.,
 * Sec. 6.2).  The continued fraction is evaluated by the modified Lentz
 * method (W. J. Lentz, Appl. Opt. 15, 668 (1976); I. J. Thompson and
 * A. R. Barnett, J. Comput. Phys. 64, 490 (1986)), whose steps and names
 * (a_n, b_n, C, D, the product h and its factor del) this follows. */
double orc_gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  double lpre = a * log(x) - x - lgamma(a);
  if (x < a + 1.0) {
    /* P = x^a e^-x / Gamma(a+1) * sum_k x^k / ((a+1)...(a+k)) */
    double term = 1.0 / a, sum = term, ap = a;
    for (int k = 0; k < 100000; ++k) {
      ap += 1.0;
      term *= x / ap;
      sum += term;
      if (fabs(term) < fabs(sum) * 1e-17) break;
    }
    return sum * exp(lpre);
  }
  /* Q = x^a e^-x / Gamma(a) * 1/(x+1-a- 1(1-a)/(x+3-a- 2(2-a)/(x+5-a- ...))) */
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 100000; ++i) {
    double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-17) break;
  }
  return 1.0 - exp(lpre) * h;
}

/* Newton on P(2n, b) - 1/2 with a bisection safeguard. */
double orc_sersic_b(double n) {
  double a = 2.0 * n;
  double lo = 0.0, hi = a + 20.0;
  double b = a - 1.0 / 3.0 + 4.0 / (405.0 * n);
  if (!(b > lo && b < hi)) b = 0.5 * a;
  for (int it = 0; it < 200; ++it) {
    double f = orc_gamma_p(a, b) - 0.5;
    if (f > 0.0) hi = b; else lo = b;
    double dfdx = exp((a - 1.0) * log(b) - b - lgamma(a));
    double nb = b - f / dfdx;
    if (!(nb > lo && nb < hi)) nb = 0.5 * (lo + hi);
    if (fabs(nb - b) <= 1e-16 * fabs(b)) { b = nb; break; }
    b = nb;
  }
  return b;
}

/* db/dn: central differences at h and h/2, combined by Richardson. */
double orc_sersic_db(double n) {
  double h = 1e-3 * n;
  double d1 = (orc_sersic_b(n + h) - orc_sersic_b(n - h)) / (2.0 * h);
  double d2 = (orc_sersic_b(n + 0.5 * h) - orc_sersic_b(n - 0.5 * h)) / h;
  return (4.0 * d2 - d1) / 3.0;
}

/* ------------------------------------------------------------------------ */
/* Model (Sec. 4.1 eq. ser for galaxies; Sec. 4.2.2 eq. mof for stars).     */
/* Reading: the elliptical radius is the area-preserving R^2 = |S(e)u|^2/D,  */
/* S(e) = [[1-e1,-e2],[-e2,1+e1]], D = 1-|e|^2 (the shear convention of the  */
/* weight in App. A, normalised so Re stays the circularised half-light      */
/* radius); the model is point-sampled at pixel centres.                    */
/* ------------------------------------------------------------------------ */
void orc_model(int side, const double* p, int kind, double* m, double* J) {
  double x0 = p[0], y0 = p[1], e1 = p[2], e2 = p[3];
  double D = 1.0 - e1 * e1 - e2 * e2;
  double b = 0.0, db = 0.0;
  if (kind == ORC_SERSIC) {
    b = orc_sersic_b(p[5]);
    if (J) db = orc_sersic_db(p[5]);
  }
  for (int i = 0; i < side; ++i) {
    for (int j = 0; j < side; ++j) {
      int k = i * side + j;
      double u1 = j - x0, u2 = i - y0;
      double v1 = (1.0 - e1) * u1 - e2 * u2;
      double v2 = -e2 * u1 + (1.0 + e1) * u2;
      double q = v1 * v1 + v2 * v2;
      double R2 = q / D;
      int floored = 0;
      if (R2 < R2_MIN) { R2 = R2_MIN; floored = 1; }
      double m0, dm_dR2, dm_d4, dm_d5;
      if (kind == ORC_SERSIC) {
        double Re = p[4], n = p[5], I0 = p[6];
        double s = sqrt(R2) / Re;
        double t = pow(s, 1.0 / n);
        m0 = exp(-b * t);
        double c = I0 * m0 * b * t;
        dm_dR2 = -c / (2.0 * n * R2);
        dm_d4 = c / (n * Re);                                   /* d/dRe */
        dm_d5 = -I0 * m0 * db * t + c * log(s) / (n * n);       /* d/dn  */
      } else {
        double rd = p[4], beta = p[5], I0 = p[6];
        double base = 1.0 + R2 / (rd * rd);
        m0 = pow(base, -beta);
        double g = I0 * beta * pow(base, -beta - 1.0);
        dm_dR2 = -g / (rd * rd);
        dm_d4 = 2.0 * g * R2 / (rd * rd * rd);                  /* d/drd */
        dm_d5 = -I0 * m0 * log(base);                           /* d/dbeta */
      }
      m[k] = p[6] * m0 + p[7];
      if (J) {
        double* Jk = J + 8 * (size_t)k;
        if (floored) dm_dR2 = 0.0;
        /* chain rule through R^2 = |S u|^2 / D */
        double w1 = (1.0 - e1) * v1 - e2 * v2;   /* (S^T v)_1 */
        double w2 = -e2 * v1 + (1.0 + e1) * v2;  /* (S^T v)_2 */
        double dR2_dx0 = -2.0 * w1 / D;
        double dR2_dy0 = -2.0 * w2 / D;
        double dR2_de1 = 2.0 * (-v1 * u1 + v2 * u2) / D + 2.0 * e1 * q / (D * D);
        double dR2_de2 = 2.0 * (-v1 * u2 - v2 * u1) / D + 2.0 * e2 * q / (D * D);
        Jk[0] = dm_dR2 * dR2_dx0;
        Jk[1] = dm_dR2 * dR2_dy0;
        Jk[2] = dm_dR2 * dR2_de1;
        Jk[3] = dm_dR2 * dR2_de2;
        Jk[4] = dm_d4;
        Jk[5] = dm_d5;
        Jk[6] = m0;
        Jk[7] = 1.0;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Starting estimates (Sec. 4.1, the paragraph on the starting point): the   */
/* brightest pixel, and r50 from summing pixels outward from it until half  */
/* the total flux.  Readings: sky is the mean of the stamp border (the       */
/* paper's simulations have none); "outward" means circular rings of        */
/* integer radius r (pixel in ring r if r-1 < d <= r), with the growth curve */
/* starting at 0 flux at radius 0 and linearly interpolated at its first     */
/* crossing of F/2; the weight scale is sigma_w = r50 / sqrt(2 ln 2) (the    */
/* Gaussian whose half-light radius is r50), clamped to [1, side/4], and     */
/* held fixed in the later iterations.                                       */
/* ------------------------------------------------------------------------ */
void orc_init(const double* img, int side, double* sky0, int* imax, double* r50,
              double* flux, double* sigw, uint32_t* status) {
  int W = side;
  double bsum = 0.0;
  for (int i = 0; i < W; ++i)
    for (int j = 0; j < W; ++j)
      if (i == 0 || j == 0 || i == W - 1 || j == W - 1) bsum += img[i * W + j];
  double sky = bsum / (4.0 * W - 4.0);
  int best = 0;
  for (int k = 1; k < W * W; ++k)
    if (img[k] > img[best]) best = k;
  int i0 = best / W, j0 = best % W;
  int nbins = 2 * W + 2;
  double* ring = (double*)calloc((size_t)nbins, sizeof(double));
  double F = 0.0;
  for (int i = 0; i < W; ++i) {
    for (int j = 0; j < W; ++j) {
      int d2 = (i - i0) * (i - i0) + (j - j0) * (j - j0);
      int r = 0;
      while (r * r < d2) ++r;           /* smallest r with r >= distance */
      double f = img[i * W + j] - sky;
      ring[r] += f;
      F += f;
    }
  }
  double half = 0.5 * F, rr = 0.125 * W;
  if (F > 0.0) {
    double prev = 0.0, cum = ring[0];
    for (int r = 1; r < nbins; ++r) {
      cum += ring[r];
      if (cum >= half) {
        rr = (r - 1) + (half - prev) / (cum - prev);
        break;
      }
      prev = cum;
    }
  } else {
    *status |= ORC_NONPOSITIVE_FLUX;
  }
  free(ring);
  double sw = rr / sqrt(2.0 * log(2.0));
  if (sw < 1.0) sw = 1.0;
  if (sw > 0.25 * W) sw = 0.25 * W;
  *sky0 = sky;
  *imax = best;
  *r50 = rr;
  *flux = F;
  *sigw = sw;
}

/* ------------------------------------------------------------------------ */
/* Centroid (Sec. 2): Gaussian-weighted first moments about the current      */
/* centre, N = sum I W, <x> = sum I W x; the offset is <x>/N = k dx, so the  */
/* centre moves by (<x>/N)/k with the fixed k.  Stop when both moves are     */
/* below tol_x or after max_iter_centroid steps (Sec. 4.1).                  */
/* ------------------------------------------------------------------------ */
void orc_centroid(const double* img, int side, double sky0, double sigw,
                  const orc_opts* o, double* x, double* y, int* iters, uint32_t* status) {
  double xc = *x, yc = *y;
  int it = 0;
  double inv2s2 = 1.0 / (2.0 * sigw * sigw);
  while (it < o->max_iter_centroid) {
    double N = 0.0, Sx = 0.0, Sy = 0.0;
    for (int i = 0; i < side; ++i) {
      for (int j = 0; j < side; ++j) {
        double t1 = j - xc, t2 = i - yc;
        double Wt = exp(-(t1 * t1 + t2 * t2) * inv2s2);
        double f = img[i * side + j] - sky0;
        N += f * Wt;
        Sx += f * Wt * t1;
        Sy += f * Wt * t2;
      }
    }
    ++it;
    if (!(N > 0.0)) { *status |= ORC_NONPOSITIVE_FLUX; break; }
    double dx = Sx / (o->k_gain * N), dy = Sy / (o->k_gain * N);
    xc += dx;
    yc += dy;
    if (xc < 0.0 || yc < 0.0 || xc > side - 1 || yc > side - 1) { *status |= ORC_LOST; break; }
    if (fabs(dx) < o->tol_x && fabs(dy) < o->tol_x) { *status |= ORC_CONVERGED; break; }
  }
  if (!(*status & (ORC_CONVERGED | ORC_NONPOSITIVE_FLUX | ORC_LOST))) *status |= ORC_MAX_ITER;
  *x = xc;
  *y = yc;
  *iters = it;
}

/* ------------------------------------------------------------------------ */
/* Elliptical-weight KSB quantities (Sec. 3; App. A eqs xshew, eshew; App. B */
/* eqs dxsh, desh and P1..P6).  Readings: f is the sky-subtracted image; the */
/* weight is W = exp(-R^2 / 2 sigma_w^2) with R^2 of App. A as printed (not  */
/* area-normalised), so W' = dW/dR^2 = -W / (2 sigma_w^2); T = Q11 + Q22     */
/* (the trace normalising e and X^SH in KSB); e_obs = (Q11 - Q22, 2 Q12)/T;  */
/* the subscript s of g in the last entry of X^SH and the unsubscripted g_1, */
/* g_2 of App. B are the weight's g_w.                                       */
/* ------------------------------------------------------------------------ */
void orc_ksb_terms(const double* img, int side, double sky0, double sigw,
                   double xc, double yc, const double* gw, double* out) {
  double g1 = gw[0], g2 = gw[1], gg = g1 * g1 + g2 * g2;
  double A = 1.0 + gg - 2.0 * g1, B = 1.0 + gg + 2.0 * g1;
  double inv2s2 = 1.0 / (2.0 * sigw * sigw);
  double N = 0, S1 = 0, S2 = 0, Q11 = 0, Q22 = 0, Q12 = 0;
  double X11 = 0, X12 = 0, X21 = 0, X22 = 0, E1 = 0, E2 = 0;
  double dX11 = 0, dX12 = 0, dX21 = 0, dX22 = 0, dE1 = 0, dE2 = 0;
  for (int i = 0; i < side; ++i) {
    for (int j = 0; j < side; ++j) {
      double t1 = j - xc, t2 = i - yc;
      double th2 = t1 * t1 + t2 * t2;
      double R2 = ((1 - g1) * (1 - g1) + g2 * g2) * t1 * t1 +
                  ((1 + g1) * (1 + g1) + g2 * g2) * t2 * t2 - 4.0 * g2 * t1 * t2;
      double W = exp(-R2 * inv2s2);
      double Wp = -W * inv2s2;
      double f = img[i * side + j] - sky0;
      N += f * W;
      S1 += f * W * t1;
      S2 += f * W * t2;
      Q11 += f * W * t1 * t1;
      Q22 += f * W * t2 * t2;
      Q12 += f * W * t1 * t2;
      double d = t1 * t1 - t2 * t2, pq = t1 * t2;
      /* App. A */
      double a1 = A * t1 * t1 - B * t2 * t2;
      double a2 = (A + B) * pq - 2.0 * g2 * th2;
      X11 += f * (2.0 * W * th2 + 2.0 * Wp * d * a1);
      X12 += f * (2.0 * Wp * d * a2);
      X21 += f * (4.0 * Wp * pq * a1);
      X22 += f * (2.0 * W * th2 + 4.0 * Wp * pq * a2);
      E1 += f * Wp * th2 * a1;
      E2 += f * Wp * th2 * a2;
      /* App. B */
      double c1 = A * t1 * t1 + B * t2 * t2 - 4.0 * g2 * pq;
      double c2 = (A - B) * pq + 2.0 * g2 * d;
      double P1 = 4.0 * W * d + 2.0 * Wp * d * c1;
      double P2 = 4.0 * W * pq + 2.0 * Wp * d * c2;
      double P3 = 8.0 * W * pq + 4.0 * Wp * pq * c1;
      double P4 = -2.0 * W * d + 4.0 * Wp * pq * c2;
      double P5 = 4.0 * W * th2 + 2.0 * Wp * th2 * c1;
      double P6 = 2.0 * Wp * th2 * c2;
      dX11 += f * (-g1 * P1 - g2 * P2);
      dX12 += f * (g1 * P2 - g2 * P1);
      dX21 += f * (-g1 * P3 - g2 * P4);
      dX22 += f * (g1 * P4 - g2 * P3);
      dE1 += f * (-g1 * P5 - g2 * P6);
      dE2 += f * (g1 * P6 - g2 * P5);
    }
  }
  double T = Q11 + Q22;
  double e1 = (Q11 - Q22) / T, e2 = 2.0 * Q12 / T;
  out[0] = N;
  out[1] = S1;
  out[2] = S2;
  out[3] = T;
  out[4] = e1;
  out[5] = e2;
  out[6] = X11 / T;
  out[7] = X12 / T;
  out[8] = X21 / T;
  out[9] = X22 / T;
  out[10] = 2.0 * e1 + 2.0 * E1 / T;
  out[11] = 2.0 * e2 + 2.0 * E2 / T;
  out[12] = dX11 / T;
  out[13] = dX12 / T;
  out[14] = dX21 / T;
  out[15] = dX22 / T;
  out[16] = dE1 / T;
  out[17] = dE2 / T;
  out[18] = 0.0;
  out[19] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Starting size for the profile fit (reading, not in the paper): the        */
/* half-light radius, along the model's elliptical radius, of the Gaussian   */
/* source that gives the weighted second moment measured with the moments   */
/* stage's weight.  With W = exp(-R^2 / 2 sigw^2), R^2 = |S(g_w) theta|^2,   */
/* a source exp(-R^2 / 2 s^2) has <R^2>_fW = 2 s^2 sigw^2 / (s^2 + sigw^2),  */
/* so s^2 = q sigw^2 / (2 sigw^2 - q) with q = sum f W R^2 / sum f W; the   */
/* model's radius is R / sqrt(1 - |g|^2) and a Gaussian's half-light radius */
/* is s sqrt(2 ln 2).  NaN unless sum f W > 0 and 0 < q < 1.96 sigw^2.       */
/* ------------------------------------------------------------------------ */
double orc_size(const double* img, int side, double sky0, double sigw, double xc, double yc,
                const double* gw) {
  double g1 = gw[0], g2 = gw[1];
  double inv2s2 = 1.0 / (2.0 * sigw * sigw);
  double N = 0.0, M = 0.0;
  for (int i = 0; i < side; ++i) {
    for (int j = 0; j < side; ++j) {
      double t1 = j - xc, t2 = i - yc;
      double u1 = (1.0 - g1) * t1 - g2 * t2, u2 = -g2 * t1 + (1.0 + g1) * t2;
      double R2 = u1 * u1 + u2 * u2;
      double fW = (img[i * side + j] - sky0) * exp(-R2 * inv2s2);
      N += fW;
      M += fW * R2;
    }
  }
  if (!(N > 0.0)) return NAN;
  double q = M / N, s2w = sigw * sigw;
  if (!(q > 0.0 && q < 1.96 * s2w)) return NAN;
  double s2 = q * s2w / (2.0 * s2w - q);
  return sqrt(2.0 * log(2.0) * s2 / (1.0 - (g1 * g1 + g2 * g2)));
}

/* ------------------------------------------------------------------------ */
/* Joint centroid + ellipticity iteration (Sec. 2 last paragraph; Sec. 3;    */
/* Sec. 4.1 starting point).  From g_w = 0 (the first step is the original   */
/* KSB estimate) each step evaluates the App. A/B sums at the current centre */
/* and g_w, then                                                             */
/*   P^SH = X^SH + dX^SH - e_obs (x) (e^SH + de^SH)      (eq. psh + App. B)  */
/*   dg   = (1 - |g_w|^2) (P^SH)^-1 (e_obs - e_w)         (eq. newg)          */
/* with e_w = 2 g_w / (1 + |g_w|^2), the distortion of an ellipse whose      */
/* reduced shear is g_w, and moves the centre by (S1, S2)/(k N) with the     */
/* same elliptical weight.  Reading: a step that would take |g_w| past gmax  */
/* is halved until it does not (the undamped iteration can leave the unit    */
/* disk for |g| near 0.7).  Stop when the centre moves less than tol_x and   */
/* g_w less than tol_g in a step that was not halved, or after              */
/* max_iter_moments steps.                                                  */
/* ------------------------------------------------------------------------ */
void orc_moments(const double* img, int side, double sky0, double sigw, double r50,
                 double x_in, double y_in, const orc_opts* o, double* out,
                 int* iters, uint32_t* status) {
  double xc = x_in, yc = y_in, g[2] = {0.0, 0.0};
  double t[20];
  int it = 0;
  double last[4] = {NAN, NAN, NAN, NAN};  /* centre and g_w of the last evaluated step */
  while (it < o->max_iter_moments) {
    orc_ksb_terms(img, side, sky0, sigw, xc, yc, g, t);
    last[0] = xc;
    last[1] = yc;
    last[2] = g[0];
    last[3] = g[1];
    ++it;
    double N = t[0], T = t[3];
    if (!(N > 0.0) || !(T > 0.0)) { *status |= ORC_NONPOSITIVE_FLUX; break; }
    double e1 = t[4], e2 = t[5];
    double gg = g[0] * g[0] + g[1] * g[1];
    double P11 = t[6] + t[12] - e1 * (t[10] + t[16]);
    double P12 = t[7] + t[13] - e1 * (t[11] + t[17]);
    double P21 = t[8] + t[14] - e2 * (t[10] + t[16]);
    double P22 = t[9] + t[15] - e2 * (t[11] + t[17]);
    double det = P11 * P22 - P12 * P21;
    if (!(fabs(det) > 1e-300) || !isfinite(det)) { *status |= ORC_SINGULAR; break; }
    double ew1 = 2.0 * g[0] / (1.0 + gg), ew2 = 2.0 * g[1] / (1.0 + gg);
    double r1 = e1 - ew1, r2 = e2 - ew2;
    double dg1 = (1.0 - gg) * (P22 * r1 - P12 * r2) / det;
    double dg2 = (1.0 - gg) * (-P21 * r1 + P11 * r2) / det;
    double h = 1.0;
    int halved = 0;
    for (int k = 0; k < 60; ++k) {
      double a = g[0] + h * dg1, b = g[1] + h * dg2;
      if (a * a + b * b <= o->gmax * o->gmax) break;
      h *= 0.5;
      halved = 1;
      *status |= ORC_G_CLAMPED;
    }
    dg1 *= h;
    dg2 *= h;
    double dx = t[1] / (o->k_gain * N), dy = t[2] / (o->k_gain * N);
    g[0] += dg1;
    g[1] += dg2;
    xc += dx;
    yc += dy;
    if (xc < 0.0 || yc < 0.0 || xc > side - 1 || yc > side - 1) { *status |= ORC_LOST; break; }
    /* a halved step says nothing about convergence (it is small because it
     * was cut at the |g_w| bound), so it never ends the iteration */
    if (!halved && fabs(dx) < o->tol_x && fabs(dy) < o->tol_x && fabs(dg1) < o->tol_g &&
        fabs(dg2) < o->tol_g) {
      *status |= ORC_CONVERGED;
      break;
    }
  }
  if (!(*status & (ORC_CONVERGED | ORC_NONPOSITIVE_FLUX | ORC_SINGULAR | ORC_LOST))) *status |= ORC_MAX_ITER;
  out[0] = xc;
  out[1] = yc;
  out[2] = g[0];
  out[3] = g[1];
  out[4] = sigw;
  out[5] = r50;
  out[6] = it > 0 ? orc_size(img, side, sky0, sigw, last[0], last[1], last + 2) : NAN;
  *iters = it;
}

/* ------------------------------------------------------------------------ */
/* Normalisation (Sec. 4.1, the dchi2/dI0 = 0 condition): with the shape     */
/* fixed the model is linear in its amplitudes, so their chi^2 optimum is    */
/* the solution of the normal equations.  Reading: the model carries a sky   */
/* level, so the amplitudes are (I0, sky) with columns (f, 1), f the unit-   */
/* amplitude profile; sigma is the same for every pixel of a stamp and       */
/* cancels.  `which` selects the amplitudes solved for (bit 6 = I0, bit 7 =  */
/* sky); the others keep their values from p.                                */
/* ------------------------------------------------------------------------ */
void orc_linear(const double* img, int side, const double* p, int kind,
                double* i0, double* sky) {
  orc_linear_subset(img, side, p, kind, 0xC0u, i0, sky);
}

void orc_linear_subset(const double* img, int side, const double* p, int kind,
                       uint32_t which, double* i0, double* sky) {
  int np = side * side;
  double q[8];
  memcpy(q, p, sizeof q);
  q[6] = 1.0;
  q[7] = 0.0;
  double* f = (double*)malloc(sizeof(double) * (size_t)np);
  orc_model(side, q, kind, f, NULL);
  double sff = 0, sf = 0, sfd = 0, sd = 0;
  for (int k = 0; k < np; ++k) {
    sff += f[k] * f[k];
    sf += f[k];
    sfd += f[k] * img[k];
    sd += img[k];
  }
  free(f);
  double a = p[6], c = p[7];
  if ((which & 0xC0u) == 0xC0u) {
    double det = sff * np - sf * sf;
    a = (sfd * np - sf * sd) / det;
    c = (sff * sd - sf * sfd) / det;
  } else if (which & 0x40u) {
    a = (sfd - c * sf) / sff;          /* sum f (d - sky) / sum f^2 */
  } else if (which & 0x80u) {
    c = (sd - a * sf) / np;            /* sum (d - I0 f) / N */
  }
  *i0 = a;
  *sky = c;
}

/* chi^2 (eq. chi2) with sigma_i = sigma; gradient 2 sum (m-d) J / sigma^2;
 * jtj = sum J J^T / sigma^2, upper triangle packed row by row (36 values). */
double orc_chi2(const double* img, int side, double sigma, const double* p, int kind,
                double* grad, double* jtj) {
  int np = side * side;
  double* m = (double*)malloc(sizeof(double) * (size_t)np);
  double* J = (grad || jtj) ? (double*)malloc(sizeof(double) * 8 * (size_t)np) : NULL;
  orc_model(side, p, kind, m, J);
  double inv2 = 1.0 / (sigma * sigma);
  double chi2 = 0.0;
  if (grad) for (int a = 0; a < 8; ++a) grad[a] = 0.0;
  if (jtj) for (int a = 0; a < 36; ++a) jtj[a] = 0.0;
  for (int k = 0; k < np; ++k) {
    double res = m[k] - img[k];
    chi2 += res * res * inv2;
    if (grad) for (int a = 0; a < 8; ++a) grad[a] += 2.0 * res * J[8 * (size_t)k + a] * inv2;
    if (jtj) {
      int idx = 0;
      for (int a = 0; a < 8; ++a)
        for (int b = a; b < 8; ++b) jtj[idx++] += J[8 * (size_t)k + a] * J[8 * (size_t)k + b] * inv2;
    }
  }
  free(m);
  free(J);
  return chi2;
}

/* In-place Cholesky solve of the k x k SPD system M x = rhs (row-major). */
static int chol_solve(int k, double* M, double* rhs) {
  for (int j = 0; j < k; ++j) {
    double s = M[j * k + j];
    for (int l = 0; l < j; ++l) s -= M[j * k + l] * M[j * k + l];
    if (!(s > 0.0)) return 0;
    double d = sqrt(s);
    M[j * k + j] = d;
    for (int i = j + 1; i < k; ++i) {
      double v = M[i * k + j];
      for (int l = 0; l < j; ++l) v -= M[i * k + l] * M[j * k + l];
      M[i * k + j] = v / d;
    }
  }
  for (int i = 0; i < k; ++i) {
    double v = rhs[i];
    for (int l = 0; l < i; ++l) v -= M[i * k + l] * rhs[l];
    rhs[i] = v / M[i * k + i];
  }
  for (int i = k - 1; i >= 0; --i) {
    double v = rhs[i];
    for (int l = i + 1; l < k; ++l) v -= M[l * k + i] * rhs[l];
    rhs[i] = v / M[i * k + i];
  }
  return 1;
}

static double jtj_at(const double* jtj, int a, int b) {
  if (a > b) { int t = a; a = b; b = t; }
  return jtj[a * 8 - a * (a - 1) / 2 + (b - a)];
}

/* The end point lies on the edge of the box (fitted parameters only). */
static int at_box_edge(const double* p, int kind, int side, double gmax, uint32_t mask) {
  const double m = 1e-3;
  if ((mask & 0x0Cu) && hypot(p[2], p[3]) >= gmax - m) return 1;
  if ((mask & 0x10u) && (p[4] <= 0.1 * (1.0 + m) || p[4] >= side * (1.0 - m))) return 1;
  if (kind == ORC_SERSIC && (mask & 0x20u) && (p[5] <= 0.2 * (1.0 + m) || p[5] >= 10.0 * (1.0 - m)))
    return 1;
  return 0;
}

static int in_bounds(const double* p, int kind, int side, double gmax) {
  if (!(p[2] * p[2] + p[3] * p[3] < gmax * gmax)) return 0;
  if (!(p[4] >= 0.1 && p[4] <= side)) return 0;
  if (kind == ORC_SERSIC) {
    if (!(p[5] >= 0.2 && p[5] <= 10.0)) return 0;
  } else {
    if (!(p[5] >= 1.01 && p[5] <= 20.0)) return 0;
  }
  if (!(p[6] > 0.0)) return 0;
  return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[7]);
}

/* Schur complement of the amplitude block: the Gauss-Newton matrix of the
 * residual with the amplitudes profiled out (M = A_NN - A_NL A_LL^-1 A_LN). */
static int schur_nl(const double* jtj, const int* nidx, int nn, const int* lidx, int nl,
                    double* M) {
  double L[4] = {0, 0, 0, 0}, Li[4];
  for (int a = 0; a < nn; ++a)
    for (int b = 0; b < nn; ++b) M[a * nn + b] = jtj_at(jtj, nidx[a], nidx[b]);
  if (nl == 0) return 1;
  for (int a = 0; a < nl; ++a)
    for (int b = 0; b < nl; ++b) L[a * nl + b] = jtj_at(jtj, lidx[a], lidx[b]);
  if (nl == 1) {
    if (!(L[0] > 0.0)) return 0;
    Li[0] = 1.0 / L[0];
  } else {
    double det = L[0] * L[3] - L[1] * L[2];
    if (!(det > 0.0)) return 0;
    Li[0] = L[3] / det;
    Li[1] = -L[1] / det;
    Li[2] = -L[2] / det;
    Li[3] = L[0] / det;
  }
  for (int a = 0; a < nn; ++a) {
    for (int b = 0; b < nn; ++b) {
      double s = 0.0;
      for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j)
          s += jtj_at(jtj, nidx[a], lidx[i]) * Li[i * nl + j] * jtj_at(jtj, lidx[j], nidx[b]);
      M[a * nn + b] -= s;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Profile fit (Sec. 4.1: the amplitude follows from dchi2/dI0 = 0 and only  */
/* the remaining shape parameters are searched; the paper searched (n, Re)   */
/* with MINUIT, here Levenberg-Marquardt does the search).                  */
/* At every evaluated point the free amplitudes (I0, sky) are first set to    */
/* their linear optimum (orc_linear_subset), then chi^2, its gradient and     */
/* J^T J are taken there; the step in the free shape parameters solves        */
/*   (M + lambda diag M) delta = J_N^T r / sigma^2                            */
/* with M the Schur complement above (Gauss-Newton for the profiled          */
/* residual), by Cholesky.  Readings (the paper gives no minimiser           */
/* constants): lambda starts at lambda0; every trial counts as one           */
/* iteration; a trial outside the box (|e| < gmax, Re or rd in [0.1, side],  */
/* n in [0.2, 10] or beta in [1.01, 20], I0 > 0) or with chi^2 above         */
/* chi^2 (1 + chi2_rtol) is rejected (lambda x 10), otherwise accepted       */
/* (lambda / 10, floor 1e-9).  Converged when an accepted step has           */
/* max_k |delta_k| / s_k < tol_lm, s = (1, 1, 1, 1, Re, n); stalled when      */
/* lambda exceeds 1e10.  A fit that ends with a fitted parameter within a    */
/* relative 1e-3 of the box (|e| >= gmax - 1e-3; Re <= 0.1 (1 + 1e-3) or      */
/* >= side (1 - 1e-3); Sersic n <= 0.2 (1 + 1e-3) or >= 10 (1 - 1e-3)) is     */
/* flagged AT_BOUND: its minimum lies on the box, not at a stationary point   */
/* of chi^2.                                                                 */
/* With linear_init = 0 the free amplitudes are not profiled: they start at  */
/* their linear optimum at the starting shape and are then searched by the   */
/* same LM together with the shape parameters (the plain form the           */
/* paper's split is compared with), with s_6 = |I0| and s_7 = sigma in the   */
/* stopping rule.                                                            */
/* ------------------------------------------------------------------------ */
void orc_fit(const double* img, int side, double sigma, int kind, const double* p_init,
             const orc_opts* o, double* p_out, double* chi2_out, int* iters,
             uint32_t* status, double* perr) {
  double p[8], pt[8], grad[8], jtj[36], gradt[8], jtjt[36];
  memcpy(p, p_init, sizeof p);
  uint32_t mask = o->free_mask;
  if (kind == ORC_MOFFAT) mask &= ~(1u << 5);
  uint32_t lin = o->linear_init ? (mask & 0xC0u) : 0u;
  int nidx[8], lidx[2], nn = 0, nl = 0;
  for (int k = 0; k < 8; ++k) {
    if (!(mask & (1u << k))) continue;
    if (lin & (1u << k)) lidx[nl++] = k;
    else nidx[nn++] = k;
  }
  if (mask & 0xC0u) orc_linear_subset(img, side, p, kind, mask & 0xC0u, &p[6], &p[7]);
  if (!(p[6] > 0.0)) *status |= ORC_NONPOSITIVE_FLUX;
  double chi2 = orc_chi2(img, side, sigma, p, kind, grad, jtj);
  double lambda = o->lambda0;
  int it = 0;
  while (it < o->max_iter_lm && nn > 0) {
    double M[64], rhs[8];
    ++it;
    int ok = schur_nl(jtj, nidx, nn, lidx, nl, M);
    for (int a = 0; a < nn; ++a) {
      M[a * nn + a] *= 1.0 + lambda;
      rhs[a] = -0.5 * grad[nidx[a]];
    }
    if (!ok || !chol_solve(nn, M, rhs)) {
      *status |= ORC_SINGULAR;
      lambda *= 10.0;
      if (lambda > 1e10) { *status |= ORC_STALLED; break; }
      continue;
    }
    memcpy(pt, p, sizeof pt);
    double smax = 0.0;
    double scl[8] = {1.0, 1.0, 1.0, 1.0, p[4], p[5], fabs(p[6]), sigma};
    for (int a = 0; a < nn; ++a) {
      pt[nidx[a]] += rhs[a];
      double r = fabs(rhs[a]) / scl[nidx[a]];
      if (r > smax) smax = r;
    }
    int inside = in_bounds(pt, kind, side, o->gmax);
    if (inside && lin) {
      orc_linear_subset(img, side, pt, kind, lin, &pt[6], &pt[7]);
      inside = in_bounds(pt, kind, side, o->gmax);
    }
    if (!inside) {
      lambda *= 10.0;
      if (lambda > 1e10) { *status |= ORC_STALLED; break; }
      continue;
    }
    double c2 = orc_chi2(img, side, sigma, pt, kind, gradt, jtjt);
    if (isfinite(c2) && c2 <= chi2 * (1.0 + o->chi2_rtol)) {
      memcpy(p, pt, sizeof p);
      memcpy(grad, gradt, sizeof grad);
      memcpy(jtj, jtjt, sizeof jtj);
      chi2 = c2;
      lambda = fmax(lambda * 0.1, 1e-9);
      if (smax < o->tol_lm) { *status |= ORC_CONVERGED; break; }
    } else {
      lambda *= 10.0;
      if (lambda > 1e10) { *status |= ORC_STALLED; break; }
    }
  }
  if (!(*status & (ORC_CONVERGED | ORC_STALLED))) *status |= ORC_MAX_ITER;
  if (at_box_edge(p, kind, side, o->gmax, mask)) *status |= ORC_AT_BOUND;
  if (perr) {
    int idx[8], nf = 0;
    for (int k = 0; k < 8; ++k)
      if (mask & (1u << k)) idx[nf++] = k;
    for (int k = 0; k < 8; ++k) perr[k] = 0.0;
    /* sigma_p = sqrt(diag(A^-1)) over all fitted parameters, column by column */
    for (int c = 0; c < nf; ++c) {
      double M[64], e[8];
      for (int a = 0; a < nf; ++a) {
        for (int b = 0; b < nf; ++b) M[a * nf + b] = jtj_at(jtj, idx[a], idx[b]);
        e[a] = (a == c) ? 1.0 : 0.0;
      }
      if (chol_solve(nf, M, e)) perr[idx[c]] = sqrt(e[c]);
      else perr[idx[c]] = NAN;
    }
  }
  memcpy(p_out, p, sizeof p);
  *chi2_out = chi2;
  *iters = it;
}

/* ------------------------------------------------------------------------ */
/* Star shapes from weighted moments (Sec. 4.2).  About the centre (xc, yc)  */
/* and with the ellipticity g from Secs. 2-3, r is the elliptical radius of */
/* the model (R^2 = |S(g) theta|^2 / (1 - |g|^2)), f = I - sky, and the      */
/* radial integrals become pixel sums:                                     */
/*   r0 = sum f W,  r2 = sum f W R^2,  r4 = sum f W R^4.                   */
/* Gaussian (Sec. 4.2.1, eqs. gaur0, gaur2): W = exp(-R^2 / 2 sigma_w^2);   */
/* with sigma_w = sigma, r0 = pi sigma^2 I0 and r2 = pi sigma^4 I0, so      */
/* sigma = sqrt(r2 / r0) and I0 = r0 / (pi sigma^2) (eqs. gausigiter,       */
/* gauI0iter); sigma_w is then set to sigma and the moments recomputed      */
/* until the fractional change of sigma is below tol or after max_iter.     */
/* Moffat (Sec. 4.2.2): W = (1 + R^2 / rdw^2)^-3; with rdw = rd the moments */
/* give beta = 1 / (r4 r0 / (2 r2^2) - 1), rd = sqrt(r2 / r0 (beta + 1)),   */
/* I0 = r0 (beta + 2) / (pi rd^2) (eqs. mofbetaiter, mofrditer, mofI0iter); */
/* rdw is iterated to rd the same way.                                       */
/* Moffat with beta fixed (the paper's remedy for the rd-beta degeneracy:   */
/* beta measured on bright stars and fixed for fainter ones): the same      */
/* weight, rd = sqrt(r2 / r0 (beta + 1)) and I0 = r0 (beta + 2) / (pi rd^2)  */
/* with the given beta; r4 is not used.                                      */
/* out: [0] sigma or rd, [1] beta (Moffat; 0 for Gaussian), [2] I0,          */
/*      [3] r0, [4] r2, [5] r4 of the last evaluation.                       */
/* ------------------------------------------------------------------------ */
static void star_sums(const double* img, int side, double sky, double xc, double yc,
                      const double* g, int kind, double w, double* r0, double* r2, double* r4) {
  double g1 = g[0], g2 = g[1], D = 1.0 - g1 * g1 - g2 * g2;
  double s0 = 0, s2 = 0, s4 = 0;
  for (int i = 0; i < side; ++i) {
    for (int j = 0; j < side; ++j) {
      double t1 = j - xc, t2 = i - yc;
      double v1 = (1.0 - g1) * t1 - g2 * t2, v2 = -g2 * t1 + (1.0 + g1) * t2;
      double R2 = (v1 * v1 + v2 * v2) / D;
      double W = kind == ORC_SERSIC ? exp(-R2 / (2.0 * w * w)) : pow(1.0 + R2 / (w * w), -3.0);
      double f = img[i * side + j] - sky;
      s0 += f * W;
      s2 += f * W * R2;
      s4 += f * W * R2 * R2;
    }
  }
  *r0 = s0;
  *r2 = s2;
  *r4 = s4;
}

void orc_star_moments(const double* img, int side, double sky, double xc, double yc,
                      const double* g, int kind, double beta_fixed, double w0, double tol,
                      int max_iter, double* out, int* iters, uint32_t* status) {
  /* kind: ORC_SERSIC selects the Gaussian star (n = 0.5), ORC_MOFFAT the     */
  /* Moffat, ORC_MOFFAT_BETA the Moffat with beta = beta_fixed                */
  double w = w0, r0 = 0, r2 = 0, r4 = 0, size = w0, beta = 0.0, I0 = 0.0;
  if (kind == ORC_MOFFAT_BETA) beta = beta_fixed;
  int it = 0;
  *status = 0;
  while (it < max_iter) {
    star_sums(img, side, sky, xc, yc, g, kind == ORC_SERSIC ? ORC_SERSIC : ORC_MOFFAT, w, &r0,
              &r2, &r4);
    ++it;
    if (!(r0 > 0.0) || !(r2 > 0.0)) { *status |= ORC_NONPOSITIVE_FLUX; break; }
    double nsize;
    if (kind == ORC_SERSIC) {
      nsize = sqrt(r2 / r0);
      I0 = r0 / (ORC_PI * nsize * nsize);
    } else if (kind == ORC_MOFFAT_BETA) {
      nsize = sqrt(r2 / r0 * (beta + 1.0));
      I0 = r0 * (beta + 2.0) / (ORC_PI * nsize * nsize);
    } else {
      double q = r4 * r0 / (2.0 * r2 * r2) - 1.0;
      if (!(q > 0.0)) { *status |= ORC_SINGULAR; break; }
      beta = 1.0 / q;
      nsize = sqrt(r2 / r0 * (beta + 1.0));
      I0 = r0 * (beta + 2.0) / (ORC_PI * nsize * nsize);
    }
    double change = fabs(nsize - w) / nsize;
    size = nsize;
    w = nsize;
    if (change < tol) { *status |= ORC_CONVERGED; break; }
  }
  if (!(*status & (ORC_CONVERGED | ORC_NONPOSITIVE_FLUX | ORC_SINGULAR))) *status |= ORC_MAX_ITER;
  out[0] = size;
  out[1] = beta;
  out[2] = I0;
  out[3] = r0;
  out[4] = r2;
  out[5] = r4;
  *iters = it;
}

/* ------------------------------------------------------------------------ */
/* Whole per-object procedure over a batch (Sec. 4.1, the paragraph on the   */
/* starting point): starting estimates, centroid from the brightest pixel,   */
/* joint centroid + ellipticity, then the profile fit from                   */
/* (x0, y0, g) of the moments, Re = the moments' size or r50 (Moffat: the    */
/* rd whose half-light radius is r50: the flux of (1 + R^2/rd^2)^-beta       */
/* inside R is 1 - (1 + R^2/rd^2)^(1-beta) of the total, so                  */
/* rd = r50 / sqrt(2^(1/(beta-1)) - 1)), n = n0 (Moffat: beta fixed), and    */
/* (I0, sky) solved linearly.                                                 */
/* ------------------------------------------------------------------------ */
int orc_pipeline(int64_t n, const double* pixels, const int64_t* offsets,
                 const int32_t* sides, const float* sigma, const uint8_t* model,
                 const orc_opts* o, double* xy, double* mom, double* p,
                 double* chi2, double* perr, int32_t* iters, uint32_t* status, int threads) {
  int used = 1;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  used = omp_get_max_threads();
#endif
#pragma omp parallel for schedule(dynamic, 2)
  for (int64_t s = 0; s < n; ++s) {
    int side = sides[s];
    double sg = sigma[s];
    int kind = model ? model[s] : ORC_SERSIC;
    uint32_t* st = status + 3 * s;
    int32_t* itr = iters + 3 * s;
    st[0] = st[1] = st[2] = 0;
    itr[0] = itr[1] = itr[2] = 0;
    for (int k = 0; k < 2; ++k) xy[2 * s + k] = NAN;
    for (int k = 0; k < 7; ++k) mom[7 * s + k] = NAN;
    for (int k = 0; k < 8; ++k) p[8 * s + k] = NAN;
    if (perr)
      for (int k = 0; k < 8; ++k) perr[8 * s + k] = NAN;
    chi2[s] = NAN;
    if (side < 4 || side > 128 || !(sg > 0.0) || (kind != ORC_SERSIC && kind != ORC_MOFFAT)) {
      st[0] = st[1] = st[2] = ORC_BAD_INPUT;
      continue;
    }
    const double* img = pixels + offsets[s];
    int finite = 1;
    for (int k = 0; k < side * side; ++k)
      if (!isfinite(img[k])) { finite = 0; break; }
    if (!finite) {
      st[0] = st[1] = st[2] = ORC_NONFINITE_INPUT;
      continue;
    }
    double sky0, r50, flux, sigw;
    int imax;
    orc_init(img, side, &sky0, &imax, &r50, &flux, &sigw, &st[0]);
    double x = imax % side, y = imax / side;
    int it;
    orc_centroid(img, side, sky0, sigw, o, &x, &y, &it, &st[0]);
    itr[0] = it;
    xy[2 * s] = x;
    xy[2 * s + 1] = y;
    double* mo = mom + 7 * s;
    orc_moments(img, side, sky0, sigw, r50, x, y, o, mo, &it, &st[1]);
    itr[1] = it;
    double pi[8];
    pi[0] = mo[0];
    pi[1] = mo[1];
    pi[2] = mo[2];
    pi[3] = mo[3];
    if (kind == ORC_SERSIC) {
      pi[4] = isfinite(mo[6]) ? mo[6] : r50;
      pi[5] = o->n0;
    } else {
      pi[4] = r50 / sqrt(pow(2.0, 1.0 / (o->moffat_beta - 1.0)) - 1.0);
      pi[5] = o->moffat_beta;
    }
    if (pi[4] < 0.1) pi[4] = 0.1;
    if (pi[4] > side) pi[4] = side;
    pi[6] = 1.0;
    pi[7] = sky0;
    double c2;
    orc_fit(img, side, sg, kind, pi, o, p + 8 * s, &c2, &it, &st[2], perr ? perr + 8 * s : NULL);
    itr[2] = it;
    chi2[s] = c2;
  }
  return used;
}

/* ------------------------------------------------------------------------ */
/* Star sizes over a batch (Sec. 4.2): starting estimates, centroid from the */
/* brightest pixel, joint centroid + ellipticity, then the star estimator of */
/* the given kind about that centre, starting from sigma_w (Gaussian) or     */
/* the Moffat of half-light radius r50, r50 / sqrt(2^(1/(beta-1)) - 1), with */
/* beta = 3 (free beta) or the fixed beta.                                   */
/* ------------------------------------------------------------------------ */
int orc_star_pipeline(int64_t n, const double* pixels, const int64_t* offsets,
                      const int32_t* sides, const orc_opts* o, int kind, double beta_fixed,
                      double tol, int max_iter, double* out, int32_t* iters, uint32_t* status,
                      int threads) {
  int used = 1;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  used = omp_get_max_threads();
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < n; ++s) {
    int side = sides[s];
    double* os = out + 6 * s;
    for (int k = 0; k < 6; ++k) os[k] = NAN;
    iters[s] = 0;
    status[s] = 0;
    if (side < 4 || side > 128) {
      status[s] = ORC_BAD_INPUT;
      continue;
    }
    const double* img = pixels + offsets[s];
    double sky0, r50, flux, sigw, mo[7];
    int imax, it;
    uint32_t st = 0;
    orc_init(img, side, &sky0, &imax, &r50, &flux, &sigw, &st);
    double x = imax % side, y = imax / side;
    orc_centroid(img, side, sky0, sigw, o, &x, &y, &it, &st);
    st = 0;
    orc_moments(img, side, sky0, sigw, r50, x, y, o, mo, &it, &st);
    double bw = kind == ORC_MOFFAT_BETA ? beta_fixed : 3.0;
    double w0 = kind == ORC_SERSIC ? sigw : r50 / sqrt(pow(2.0, 1.0 / (bw - 1.0)) - 1.0);
    int its;
    uint32_t sst;
    orc_star_moments(img, side, sky0, mo[0], mo[1], mo + 2, kind, beta_fixed, w0, tol, max_iter,
                     os, &its, &sst);
    iters[s] = its;
    status[s] = sst;
  }
  return used;
}

/* ------------------------------------------------------------------------ */
/* Front end on whole frames (Sec. 4.1, the paragraph on the starting        */
/* point): the brightest pixel of the frame, r50 from summing the pixels     */
/* outward from it until half the total flux, and a square of side 6 r50     */
/* cut out around it.  Same readings as the stamp estimates (border-mean     */
/* sky, integer-radius rings, interpolated first crossing).  Further         */
/* readings: the side is 6 r50 rounded to the nearest integer (halves away   */
/* from zero), clamped to [4, min(max_side, H, W)]; the square starts at     */
/* the peak minus side/2 (integer division) in each axis, shifted to lie     */
/* inside the frame; with no positive total flux r50 = min(H, W) / 8.        */
/* ------------------------------------------------------------------------ */
void orc_frame_detect(const double* img, int H, int W, int max_side, double* sky0,
                      double* r50, double* flux, int* peak_x, int* peak_y, int* box,
                      uint32_t* status) {
  for (size_t k = 0; k < (size_t)H * W; ++k) {
    if (!isfinite(img[k])) {
      /* a frame with a NaN or Inf pixel yields no cut-out (side 0) */
      *status = ORC_NONFINITE_INPUT;
      *sky0 = *r50 = *flux = NAN;
      *peak_x = *peak_y = -1;
      box[0] = box[1] = box[2] = 0;
      return;
    }
  }
  double bsum = 0.0;
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j)
      if (i == 0 || j == 0 || i == H - 1 || j == W - 1) bsum += img[(size_t)i * W + j];
  double sky = bsum / (2.0 * W + 2.0 * H - 4.0);
  size_t best = 0;
  for (size_t k = 1; k < (size_t)H * W; ++k)
    if (img[k] > img[best]) best = k;
  int i0 = (int)(best / W), j0 = (int)(best % W);
  int nbins = (int)ceil(sqrt((double)H * H + (double)W * W)) + 2;
  double* ring = (double*)calloc((size_t)nbins, sizeof(double));
  double F = 0.0;
  for (int i = 0; i < H; ++i) {
    for (int j = 0; j < W; ++j) {
      long d2 = (long)(i - i0) * (i - i0) + (long)(j - j0) * (j - j0);
      /* smallest integer r with r^2 >= d2 */
      int r = (int)ceil(sqrt((double)d2));
      while ((long)r * r < d2) ++r;
      while (r > 0 && (long)(r - 1) * (r - 1) >= d2) --r;
      double f = img[(size_t)i * W + j] - sky;
      ring[r] += f;
      F += f;
    }
  }
  int mind = H < W ? H : W;
  double half = 0.5 * F, rr = 0.125 * mind;
  *status = 0;
  if (F > 0.0) {
    double prev = 0.0, cum = ring[0];
    for (int r = 1; r < nbins; ++r) {
      cum += ring[r];
      if (cum >= half) {
        rr = (r - 1) + (half - prev) / (cum - prev);
        break;
      }
      prev = cum;
    }
  } else {
    *status |= ORC_NONPOSITIVE_FLUX;
  }
  free(ring);
  int smax = max_side;
  if (smax > mind) smax = mind;
  long side = lround(6.0 * rr);
  if (side < 4) side = 4;
  if (side > smax) side = smax;
  int ox = j0 - (int)side / 2, oy = i0 - (int)side / 2;
  if (ox > W - side) ox = W - (int)side;
  if (oy > H - side) oy = H - (int)side;
  if (ox < 0) ox = 0;
  if (oy < 0) oy = 0;
  *sky0 = sky;
  *r50 = rr;
  *flux = F;
  *peak_x = j0;
  *peak_y = i0;
  box[0] = ox;
  box[1] = oy;
  box[2] = (int)side;
}
