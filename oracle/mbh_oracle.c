/*
 * mbh_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Slow, obviously correct FP64 implementation of what the GPU library
 * computes, written from the paper (Katz 2021, arXiv:2111.01064) and from the
 * frozen model definitions that stand in for the external waveform/response
 * references the paper cites.  Nothing here is blocked, fused or reordered
 * beyond the definitions; every sum is Neumaier-compensated; the only
 * parallelism is OpenMP over independent walkers.  The GPU library never calls
 * this file and shares no code with it.
 *
 * Sections followed:
 *   Sec. 2 eq. (like)          log-likelihood  -1/2 <d-h|d-h>
 *   Sec. 2 eq. (inner)         4 Re sum_{A,E,T} int conj(a) b / S df, discretised on the grid
 *   Sec. 2.1 (TDI transform)   A=(Z-X)/sqrt2, E=(X-2Y+Z)/sqrt6, T=(X+Y+Z)/sqrt3
 *   Sec. 2.1 eq. (amp_and_phase), eq. (tf), eq. (response)
 *   Sec. 2.2 eqs. (discretized)-(h_h_rel_bin)  heterodyne / relative binning
 *   Sec. 3.2                   band where h0 != 0, log-spaced bin edges
 * Waveform ("IMR-lite") and response (cartwheel orbit, single-link transfer,
 * first-generation TDI) are the project's own frozen substitutes for PhenomD /
 * PhenomHM and the FD LISA transfer function, which the paper only cites.
 */
#include "mbh_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---- constants (the oracle's own copy) ---------------------------------- */
static const double PI = 3.14159265358979323846;
static const double MSUN_S = 4.925490947641267e-6;   /* G Msun / c^3 [s]   */
static const double C_SI = 299792458.0;               /* [m/s]              */
static const double GPC_M = 3.0856775814913673e25;    /* [m]                */
static const double AU_M = 1.495978707e11;            /* [m]                */
static const double YEAR_S = 31557600.0;              /* Julian year [s]    */
static const double ARM_M = 2.5e9;                    /* LISA arm [m]       */
static const double KAPPA = -1.0;                     /* merger-ringdown phase weight */

/* ---- Neumaier-compensated sum ------------------------------------------ */
typedef struct { double s, c; } nsum;
static void ns_add(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double ns_val(const nsum *a) { return a->s + a->c; }

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the walker loops (timing only; results do not depend on it) */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_n_chan(int model) { return model == OR_MODEL_TF2 ? 1 : 3; }

/* ---- spin-weighted spherical harmonics ----------------------------------
 * -2Y_lm(theta, phi) = sqrt((2l+1)/(4 pi)) d^l_{m,2}(theta) e^{i m phi},
 * Wigner small-d from its explicit sum over s. */
static double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
static double wigner_d(int l, int mp, int m, double theta) {
  double c = cos(0.5 * theta), s = sin(0.5 * theta);
  double pre = sqrt(fact(l + mp) * fact(l - mp) * fact(l + m) * fact(l - m));
  double sum = 0.0;
  for (int k = 0; k <= 2 * l; ++k) {
    int a = l + m - k, b = mp - m + k, d = l - mp - k;
    if (a < 0 || b < 0 || d < 0) continue;
    double sign = ((mp - m + k) % 2 == 0) ? 1.0 : -1.0;
    double term = sign * pre / (fact(a) * fact(k) * fact(b) * fact(d));
    term *= pow(c, 2 * l + m - mp - 2 * k) * pow(s, mp - m + 2 * k);
    sum += term;
  }
  return sum;
}
void oracle_sylm(int l, int m, double theta, double phi, double *re, double *im) {
  double amp = sqrt((2.0 * l + 1.0) / (4.0 * PI)) * wigner_d(l, m, 2, theta);
  *re = amp * cos(m * phi);
  *im = amp * sin(m * phi);
}
static cplx sylm(int l, int m, double theta, double phi) {
  double re, im;
  oracle_sylm(l, m, theta, phi, &re, &im);
  return re + I * im;
}

/* ---- IMR-lite waveform --------------------------------------------------- */
typedef struct {
  double M, eta, delta, DL;        /* M, D_L in seconds */
  double psi2, psi3;               /* 1PN, 1.5PN phase coefficients */
  double f1, fRD, fD, fcut, fmax;  /* transition, ringdown, damping, cutoff, f_ref */
  double P1, dP1, L1, at1;         /* inspiral phase & slope at f1, Lorentzian & atan at f1 */
  double ph_max, dph_max;          /* raw phase & slope at fmax */
  double AN;                       /* amplitude prefactor */
  double tref;
} wf_t;

static const int MODE_L[6] = {2, 3, 4, 2, 3, 4};
static const int MODE_M[6] = {2, 3, 4, 1, 2, 3};

static int imr_valid(const double *th) {
  for (int i = 0; i < OR_NPARAM; ++i)
    if (!isfinite(th[i])) return 0;
  if (!(th[0] > 0.0)) return 0;
  if (!(th[1] >= 0.05 && th[1] <= 1.0)) return 0;
  if (!(fabs(th[2]) <= 0.99 && fabs(th[3]) <= 0.99)) return 0;
  if (!(th[4] > 0.0)) return 0;
  return 1;
}

static void inspiral_phase(const wf_t *w, double f, double *ph, double *dph) {
  double v = cbrt(PI * w->M * f);
  double v2 = v * v, v3 = v2 * v, v5 = v3 * v2;
  *ph = -(3.0 / (128.0 * w->eta)) * (1.0 / v5 + w->psi2 / v3 + w->psi3 / v2);
  *dph = (1.0 / (128.0 * w->eta * f)) * (5.0 / v5 + 3.0 * w->psi2 / v3 + 2.0 * w->psi3 / v2);
}
static double lorentz(const wf_t *w, double f) {
  double x = f - w->fRD;
  return w->fD / (x * x + w->fD * w->fD);
}
static void raw_phase(const wf_t *w, double f, double *ph, double *dph) {
  if (f <= w->f1) {
    inspiral_phase(w, f, ph, dph);
    return;
  }
  double x = f - w->f1;
  *ph = w->P1 + w->dP1 * x + KAPPA * (atan((f - w->fRD) / w->fD) - w->at1 - w->L1 * x);
  *dph = w->dP1 + KAPPA * (lorentz(w, f) - w->L1);
}

static void wf_setup(const double *th, wf_t *w) {
  double q = th[1], a1 = th[2], a2 = th[3];
  w->M = th[0] * MSUN_S;
  double m1 = 1.0 / (1.0 + q), m2 = q / (1.0 + q);
  w->eta = m1 * m2;
  w->delta = m1 - m2;
  w->DL = th[4] * GPC_M / C_SI;
  w->psi2 = 3715.0 / 756.0 + 55.0 * w->eta / 9.0;
  double bso = ((113.0 * m1 * m1 + 75.0 * w->eta) * a1 + (113.0 * m2 * m2 + 75.0 * w->eta) * a2) / 12.0;
  w->psi3 = -16.0 * PI + 4.0 * bso;
  w->f1 = 0.018 / w->M;
  double Mf = w->M * (1.0 - 0.19 * w->eta);
  w->fRD = 0.0595 / Mf;
  w->fD = 0.0142 / Mf;
  w->fcut = 0.2 / w->M;
  inspiral_phase(w, w->f1, &w->P1, &w->dP1);
  w->L1 = lorentz(w, w->f1);
  w->at1 = atan((w->f1 - w->fRD) / w->fD);
  w->fmax = -2.0 * w->fRD + sqrt(9.0 * w->fRD * w->fRD + 5.0 * w->fD * w->fD);
  raw_phase(w, w->fmax, &w->ph_max, &w->dph_max);
  w->AN = PI * sqrt(2.0 * w->eta / 3.0) * w->M * w->M / w->DL;
  w->tref = th[10];
}

/* (2,2): amplitude, phase aligned at fmax, and its slope */
static void wf22(const wf_t *w, double f, double *amp, double *ph, double *dph) {
  double v = cbrt(PI * w->M * f);
  double lam = 1.0;
  if (f > w->f1) {
    double a = w->f1 - w->fRD, b = f - w->fRD, g2 = w->fD * w->fD;
    lam = sqrt((a * a + g2) / (b * b + g2));
  }
  *amp = w->AN * pow(v, -3.5) * lam;
  double p, dp;
  raw_phase(w, f, &p, &dp);
  *ph = p - w->ph_max - w->dph_max * (f - w->fmax);
  *dph = dp - w->dph_max;
}

/* Relative amplitude of mode index mi at (2,2)-equivalent frequency fp, i.e.
 * A_lm(f) / A_22(fp) with fp = 2 f / m (both at the same orbital frequency,
 * v = (pi M fp)^(1/3)).  It is the product of
 *  - the leading-order magnitude |H_lm| of the post-Newtonian mode amplitude
 *    relative to H_22 = 1 (Blanchet, Living Rev. Relativ. 17 (2014) 2,
 *    Sec. 9.5), with delta = (m1 - m2) / M:
 *      |H33| = (3/4) sqrt(15/14) delta v,  |H44| = (8/9) sqrt(5/7) (1 - 3 eta) v^2,
 *      |H21| = (1/3) delta v,               |H32| = (1/3) sqrt(5/7) (1 - 3 eta) v^2,
 *      |H43| = 9 / (4 sqrt 70) delta (1 - 2 eta) v^3;
 *  - the ratio sqrt(2/m) of the stationary-phase factors sqrt(2 pi / (m Phi''))
 *    of mode m and of mode 2 at the same orbital frequency (the Fourier
 *    amplitude of a mode is its time-domain amplitude times that factor). */
static double mode_rel_amp(const wf_t *w, int mi, double fp) {
  double v = cbrt(PI * w->M * fp);
  double H = 0.0;
  switch (mi) {
    case 0: H = 1.0; break;
    case 1: H = 0.75 * sqrt(15.0 / 14.0) * w->delta * v; break;
    case 2: H = (8.0 / 9.0) * sqrt(5.0 / 7.0) * (1.0 - 3.0 * w->eta) * v * v; break;
    case 3: H = (1.0 / 3.0) * w->delta * v; break;
    case 4: H = (1.0 / 3.0) * sqrt(5.0 / 7.0) * (1.0 - 3.0 * w->eta) * v * v; break;
    case 5: H = 9.0 / (4.0 * sqrt(70.0)) * w->delta * (1.0 - 2.0 * w->eta) * v * v * v; break;
  }
  return H * sqrt(2.0 / MODE_M[mi]);
}

/* mode mi at frequency f: amplitude, phase phi_lm (no t_ref term), t_lm */
static int wf_mode(const wf_t *w, int mi, double f, double t_obs, double *amp, double *ph,
                   double *tf) {
  int m = MODE_M[mi];
  double fp = 2.0 * f / m;
  double a22, p22, dp22;
  wf22(w, fp, &a22, &p22, &dp22);
  *amp = mode_rel_amp(w, mi, fp) * a22;
  *ph = 0.5 * m * p22;
  *tf = w->tref - dp22 / (2.0 * PI);  /* eq. (tf) */
  return (fp <= w->fcut) && (*tf >= 0.0) && (*tf <= t_obs);
}

static int mode_index(int l, int m) {
  for (int i = 0; i < 6; ++i)
    if (MODE_L[i] == l && MODE_M[i] == m) return i;
  return -1;
}

int oracle_mode(const double *theta, int l, int m, int n, const double *f, double *amp,
                double *phase, double *tf, int *on) {
  int mi = mode_index(l, m);
  if (mi < 0 || !imr_valid(theta)) return OR_EINVAL;
  wf_t w;
  wf_setup(theta, &w);
  for (int i = 0; i < n; ++i) on[i] = wf_mode(&w, mi, f[i], INFINITY, &amp[i], &phase[i], &tf[i]);
  return OR_OK;
}

double oracle_fmax(const double *theta) {
  wf_t w;
  wf_setup(theta, &w);
  return w.fmax;
}

/* ---- LISA orbit and response -------------------------------------------- */
void oracle_orbit(double t, double *p) {
  double R = AU_M / C_SI, L = ARM_M / C_SI;
  double e = L / (2.0 * sqrt(3.0) * R);
  double a = 2.0 * PI * t / YEAR_S;
  for (int k = 0; k < 3; ++k) {
    double b = 2.0 * PI * k / 3.0;
    p[3 * k + 0] = R * cos(a) + 0.5 * e * R * (cos(2.0 * a - b) - 3.0 * cos(b));
    p[3 * k + 1] = R * sin(a) + 0.5 * e * R * (sin(2.0 * a - b) - 3.0 * sin(b));
    p[3 * k + 2] = -sqrt(3.0) * e * R * cos(a - b);
  }
}

typedef struct {
  double khat[3], pv[3], qv[3];
} sky_t;

static void sky_setup(double lam, double beta, double psi, sky_t *s) {
  s->khat[0] = -cos(beta) * cos(lam);
  s->khat[1] = -cos(beta) * sin(lam);
  s->khat[2] = -sin(beta);
  double u[3] = {sin(lam), -cos(lam), 0.0};
  double v[3] = {-sin(beta) * cos(lam), -sin(beta) * sin(lam), cos(beta)};
  for (int i = 0; i < 3; ++i) {
    s->pv[i] = cos(psi) * u[i] + sin(psi) * v[i];
    s->qv[i] = -sin(psi) * u[i] + cos(psi) * v[i];
  }
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* y_{i->j}: emitted at spacecraft i, received at j */
static cplx link_y(int i, int j, double f, const double *p, const sky_t *s, cplx Kp, cplx Kc) {
  double L = ARM_M / C_SI;
  double n[3], sum[3];
  for (int x = 0; x < 3; ++x) {
    n[x] = p[3 * j + x] - p[3 * i + x];
    sum[x] = p[3 * j + x] + p[3 * i + x];
  }
  double nn = sqrt(dot3(n, n));
  for (int x = 0; x < 3; ++x) n[x] /= nn;
  double np = dot3(n, s->pv), nq = dot3(n, s->qv);
  cplx proj = Kp * (np * np - nq * nq) + Kc * (2.0 * np * nq);
  double kn = dot3(s->khat, n);
  double x = PI * f * L * (1.0 - kn);
  double sinc = (x == 0.0) ? 1.0 : sin(x) / x;
  double ph = PI * f * (L + dot3(s->khat, sum));
  return I * PI * f * L * sinc * cexp(I * ph) * proj;
}

void oracle_link(int i, int j, double f, const double *p, double lam, double beta, double psi,
                 const double *Kp, const double *Kc, double *y) {
  sky_t s;
  sky_setup(lam, beta, psi, &s);
  cplx r = link_y(i, j, f, p, &s, Kp[0] + I * Kp[1], Kc[0] + I * Kc[1]);
  y[0] = creal(r);
  y[1] = cimag(r);
}

/* first-generation TDI X, Y, Z then A, E, T; out[0..5] */
static void tdi(double f, double t, const sky_t *s, cplx Kp, cplx Kc, cplx *out) {
  double p[9];
  oracle_orbit(t, p);
  cplx y[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (i != j) y[i][j] = link_y(i, j, f, p, s, Kp, Kc);
  double L = ARM_M / C_SI;
  cplx z = cexp(2.0 * I * PI * f * L);
  cplx w = 1.0 - z * z;
  cplx X = w * ((y[2][0] + z * y[0][2]) - (y[1][0] + z * y[0][1]));
  cplx Y = w * ((y[0][1] + z * y[1][0]) - (y[2][1] + z * y[1][2]));
  cplx Z = w * ((y[1][2] + z * y[2][1]) - (y[0][2] + z * y[2][0]));
  out[0] = X;
  out[1] = Y;
  out[2] = Z;
  out[3] = (Z - X) / sqrt(2.0);
  out[4] = (X - 2.0 * Y + Z) / sqrt(6.0);
  out[5] = (X + Y + Z) / sqrt(3.0);
}

void oracle_tdi(double f, double t, double lam, double beta, double psi, const double *Kp,
                const double *Kc, double *out) {
  sky_t s;
  sky_setup(lam, beta, psi, &s);
  cplx o[6];
  tdi(f, t, &s, Kp[0] + I * Kp[1], Kc[0] + I * Kc[1], o);
  for (int i = 0; i < 6; ++i) {
    out[2 * i] = creal(o[i]);
    out[2 * i + 1] = cimag(o[i]);
  }
}

/* ---- template at one frequency ------------------------------------------ */
typedef struct {
  int model, valid;
  uint32_t modes;
  wf_t w;
  sky_t sky;
  cplx Kp[6], Kc[6];
  double tf2[4]; /* TF2: Mc [s], amp, t_c, phi_c */
} src_t;

static void src_setup(int model, uint32_t modes, const double *th, src_t *s) {
  memset(s, 0, sizeof(*s));
  s->model = model;
  s->modes = modes;
  if (model == OR_MODEL_TF2) {
    s->valid = isfinite(th[0]) && isfinite(th[1]) && isfinite(th[2]) && isfinite(th[3]) && th[0] > 0.0;
    s->tf2[0] = th[0] * MSUN_S;
    s->tf2[1] = th[1];
    s->tf2[2] = th[2];
    s->tf2[3] = th[3];
    return;
  }
  s->valid = imr_valid(th);
  if (!s->valid) return;
  wf_setup(th, &s->w);
  sky_setup(th[7], th[8], th[9], &s->sky);
  double phiref = th[5], iota = th[6];
  for (int mi = 0; mi < 6; ++mi) {
    int l = MODE_L[mi], m = MODE_M[mi];
    cplx Y = sylm(l, m, iota, phiref);
    cplx Ym = conj(sylm(l, -m, iota, phiref));
    double sg = (l % 2 == 0) ? 1.0 : -1.0;
    s->Kp[mi] = 0.5 * (Y + sg * Ym);
    s->Kc[mi] = 0.5 * I * (Y - sg * Ym);
  }
}

/* h[c] at frequency f (eq. (response)); returns the number of channels */
static int tmpl_point(const src_t *s, double f, double t_obs, cplx *h) {
  if (s->model == OR_MODEL_TF2) {
    double Mc = s->tf2[0];
    double phase = s->tf2[3] - 2.0 * PI * f * s->tf2[2] - (3.0 / 128.0) * pow(PI * Mc * f, -5.0 / 3.0);
    h[0] = s->tf2[1] * pow(f, -7.0 / 6.0) * cexp(-I * phase);
    return 1;
  }
  h[0] = h[1] = h[2] = 0.0;
  for (int mi = 0; mi < 6; ++mi) {
    if (!(s->modes & (1u << mi))) continue;
    double amp, ph, tf;
    if (!wf_mode(&s->w, mi, f, t_obs, &amp, &ph, &tf)) continue;
    cplx hlm = amp * cexp(-I * (ph - 2.0 * PI * f * s->w.tref)); /* eq. (amp_and_phase) with t_ref shift */
    cplx o[6];
    tdi(f, tf, &s->sky, s->Kp[mi], s->Kc[mi], o);
    for (int c = 0; c < 3; ++c) h[c] += o[3 + c] * hlm;
  }
  return 3;
}

int oracle_template(int model, uint32_t modes, const double *theta, int64_t n, const double *f,
                    double t_obs, double *h) {
  src_t s;
  src_setup(model, modes, theta, &s);
  if (!s.valid) return OR_EINVAL;
  int nc = oracle_n_chan(model);
  for (int64_t k = 0; k < n; ++k) {
    cplx hp[3];
    tmpl_point(&s, f[k], t_obs, hp);
    for (int c = 0; c < nc; ++c) {
      h[(c * n + k) * 2] = creal(hp[c]);
      h[(c * n + k) * 2 + 1] = cimag(hp[c]);
    }
  }
  return OR_OK;
}

/* ---- inner product and full-grid likelihood ------------------------------ */
double oracle_inner(int n_chan, int64_t n_f, const double *a, const double *b, const double *psd,
                    double df) {
  nsum acc = {0, 0};
  for (int c = 0; c < n_chan; ++c)
    for (int64_t k = 0; k < n_f; ++k) {
      int64_t i = c * n_f + k;
      /* Re(conj(a) b) */
      double re = a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1];
      ns_add(&acc, 4.0 * re / psd[i] * df);
    }
  return ns_val(&acc);
}

double oracle_loglike_of(int n_chan, int64_t n_f, const double *d, const double *h,
                         const double *psd, double df, double *dh, double *hh) {
  nsum r = {0, 0}, sdh = {0, 0}, shh = {0, 0};
  for (int c = 0; c < n_chan; ++c)
    for (int64_t k = 0; k < n_f; ++k) {
      int64_t i = c * n_f + k;
      double w = 4.0 * df / psd[i];
      double xr = d[2 * i] - h[2 * i], xi = d[2 * i + 1] - h[2 * i + 1];
      ns_add(&r, (xr * xr + xi * xi) * w);
      ns_add(&sdh, (d[2 * i] * h[2 * i] + d[2 * i + 1] * h[2 * i + 1]) * w);
      ns_add(&shh, (h[2 * i] * h[2 * i] + h[2 * i + 1] * h[2 * i + 1]) * w);
    }
  if (dh) *dh = ns_val(&sdh);
  if (hh) *hh = ns_val(&shh);
  return -0.5 * ns_val(&r);
}

int oracle_loglike_full(int model, uint32_t modes, int64_t W, const double *theta, int n_chan,
                        int64_t n_f, double f0, double df, double t_obs, const double *d,
                        const double *psd, double *lnL, double *dh, double *hh) {
  if (n_chan != oracle_n_chan(model)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t w = 0; w < W; ++w) {
    src_t s;
    src_setup(model, modes, theta + w * OR_NPARAM, &s);
    if (!s.valid) {
      lnL[w] = -INFINITY;
      if (dh) dh[w] = 0.0;
      if (hh) hh[w] = 0.0;
      continue;
    }
    nsum r = {0, 0}, sdh = {0, 0}, shh = {0, 0};
    for (int64_t k = 0; k < n_f; ++k) {
      double f = f0 + k * df;
      cplx h[3];
      tmpl_point(&s, f, t_obs, h);
      for (int c = 0; c < n_chan; ++c) {
        int64_t i = c * n_f + k;
        cplx dk = d[2 * i] + I * d[2 * i + 1];
        double wgt = 4.0 * df / psd[i];
        cplx x = dk - h[c];
        ns_add(&r, (creal(x) * creal(x) + cimag(x) * cimag(x)) * wgt);
        ns_add(&sdh, creal(conj(dk) * h[c]) * wgt);
        ns_add(&shh, (creal(h[c]) * creal(h[c]) + cimag(h[c]) * cimag(h[c])) * wgt);
      }
    }
    lnL[w] = -0.5 * ns_val(&r); /* eq. (like) */
    if (dh) dh[w] = ns_val(&sdh);
    if (hh) hh[w] = ns_val(&shh);
  }
  return OR_OK;
}

/* ---- heterodyne: per-bin sums for given edges ---------------------------
 * Grid points k_lo..k_hi are assigned to bins [F_b, F_b+1) (the last bin
 * closed); A0, A1, B0, B1 of eqs. (d_h_rel_bin), (h_h_rel_bin) and the dropped
 * B2 = sum |h0|^2/S (f-f_b)^2 df, with f_b the arithmetic bin centre. */
void oracle_bin_sums(int n_chan, int64_t n_f, double f0, double df, const double *d,
                     const double *psd, const double *h0r, int n_bins, const double *edges,
                     int64_t lo, int64_t hi, int64_t *kb, double *A0, double *A1, double *B0,
                     double *B1, double *B2) {
  const cplx *h0 = (const cplx *)h0r;
  for (int j = 0; j <= n_bins; ++j) kb[j] = hi + 1;
  kb[0] = lo;
  int b = 0;
  for (int64_t k = lo; k <= hi; ++k) {
    double f = f0 + k * df;
    while (b < n_bins - 1 && f >= edges[b + 1]) {
      ++b;
      kb[b] = k;
    }
  }
  for (int j = n_bins - 1; j >= 1; --j)
    if (kb[j] > kb[j + 1]) kb[j] = kb[j + 1];

  for (int c = 0; c < n_chan; ++c)
    for (int bb = 0; bb < n_bins; ++bb) {
      double fb = 0.5 * (edges[bb] + edges[bb + 1]);
      nsum a0r = {0, 0}, a0i = {0, 0}, a1r = {0, 0}, a1i = {0, 0};
      nsum b0 = {0, 0}, b1 = {0, 0}, b2 = {0, 0};
      for (int64_t k = kb[bb]; k < kb[bb + 1]; ++k) {
        int64_t i = c * n_f + k;
        double f = f0 + k * df;
        cplx dk = d[2 * i] + I * d[2 * i + 1];
        cplx t = dk * conj(h0[i]) / psd[i] * df;
        double h2 = (creal(h0[i]) * creal(h0[i]) + cimag(h0[i]) * cimag(h0[i])) / psd[i] * df;
        ns_add(&a0r, creal(t));
        ns_add(&a0i, cimag(t));
        ns_add(&a1r, creal(t) * (f - fb));
        ns_add(&a1i, cimag(t) * (f - fb));
        ns_add(&b0, h2);
        ns_add(&b1, h2 * (f - fb));
        ns_add(&b2, h2 * (f - fb) * (f - fb));
      }
      int64_t o = (int64_t)c * n_bins + bb;
      A0[2 * o] = ns_val(&a0r);
      A0[2 * o + 1] = ns_val(&a0i);
      A1[2 * o] = ns_val(&a1r);
      A1[2 * o + 1] = ns_val(&a1i);
      B0[o] = ns_val(&b0);
      B1[o] = ns_val(&b1);
      if (B2) B2[o] = ns_val(&b2);
    }
}

/* ---- heterodyne: reference preparation ---------------------------------- */
int oracle_reference(int model, uint32_t modes, const double *theta0, int n_chan, int64_t n_f,
                     double f0, double df, double t_obs, const double *d, const double *psd,
                     int n_bins, int64_t *k_lo, int64_t *k_hi, double *edges, int64_t *kb,
                     double *A0, double *A1, double *B0, double *B1, double *B2, double *dd,
                     double *h0_edges) {
  if (n_bins < 1 || n_chan != oracle_n_chan(model)) return OR_EINVAL;
  src_t s;
  src_setup(model, modes, theta0, &s);
  if (!s.valid) return OR_EINVAL;

  /* <d|d> over the whole grid */
  nsum sdd = {0, 0};
  for (int c = 0; c < n_chan; ++c)
    for (int64_t k = 0; k < n_f; ++k) {
      int64_t i = c * n_f + k;
      ns_add(&sdd, (d[2 * i] * d[2 * i] + d[2 * i + 1] * d[2 * i + 1]) * 4.0 * df / psd[i]);
    }
  *dd = ns_val(&sdd);

  /* h0 on the full grid; band = first/last grid frequency where h0 != 0 */
  cplx *h0 = (cplx *)malloc(sizeof(cplx) * n_chan * n_f);
  int64_t lo = -1, hi = -1;
  for (int64_t k = 0; k < n_f; ++k) {
    cplx hp[3];
    tmpl_point(&s, f0 + k * df, t_obs, hp);
    int nz = 0;
    for (int c = 0; c < n_chan; ++c) {
      h0[c * n_f + k] = hp[c];
      if (hp[c] != 0.0) nz = 1;
    }
    if (nz) {
      if (lo < 0) lo = k;
      hi = k;
    }
  }
  if (lo < 0 || hi <= lo) {
    free(h0);
    return OR_EBAND;
  }
  *k_lo = lo;
  *k_hi = hi;

  /* log-spaced edges between the band ends (ends exact) */
  double F0 = f0 + lo * df, FN = f0 + hi * df;
  edges[0] = F0;
  edges[n_bins] = FN;
  for (int j = 1; j < n_bins; ++j) edges[j] = exp(log(F0) + j * (log(FN) - log(F0)) / n_bins);

  oracle_bin_sums(n_chan, n_f, f0, df, d, psd, (const double *)h0, n_bins, edges, lo, hi, kb,
                  A0, A1, B0, B1, B2);
  free(h0);

  /* h0 at the edges; the ratio h/h0 must exist there */
  int rc = OR_OK;
  for (int j = 0; j <= n_bins; ++j) {
    cplx hp[3];
    tmpl_point(&s, edges[j], t_obs, hp);
    for (int c = 0; c < n_chan; ++c) {
      int64_t o = (int64_t)c * (n_bins + 1) + j;
      h0_edges[2 * o] = creal(hp[c]);
      h0_edges[2 * o + 1] = cimag(hp[c]);
    }
  }
  /* the ratio h/h0 must exist at every edge: an edge where h0 vanishes (a
   * gap in the support inside the band) cannot be heterodyned */
  for (int c = 0; c < n_chan; ++c)
    for (int j = 0; j <= n_bins; ++j) {
      int64_t o = (int64_t)c * (n_bins + 1) + j;
      double a = hypot(h0_edges[2 * o], h0_edges[2 * o + 1]);
      if (!(a > 0.0) || !isfinite(a)) rc = OR_EBAND;
    }
  return rc;
}

/* ---- heterodyne: online evaluation -------------------------------------- */
static cplx ratio_at(const double *h, const double *h0, int64_t o) {
  cplx a = h[2 * o] + I * h[2 * o + 1];
  cplx b = h0[2 * o] + I * h0[2 * o + 1];
  return a / b;
}

void oracle_het_core(int n_chan, int n_bins, const double *edges, const double *A0,
                     const double *A1, const double *B0, const double *B1, double dd,
                     const double *h0_edges, const double *h_edges, double *lnL, double *dh,
                     double *hh) {
  nsum zdh = {0, 0}, zhh = {0, 0};
  for (int c = 0; c < n_chan; ++c)
    for (int b = 0; b < n_bins; ++b) {
      int64_t e0 = (int64_t)c * (n_bins + 1) + b;
      cplx ra = ratio_at(h_edges, h0_edges, e0);     /* r = h / h0 at F_b   */
      cplx rb = ratio_at(h_edges, h0_edges, e0 + 1); /* r at F_{b+1}        */
      cplx r0 = 0.5 * (ra + rb);                     /* line at the bin centre */
      cplx r1 = (rb - ra) / (edges[b + 1] - edges[b]); /* slope              */
      int64_t o = (int64_t)c * n_bins + b;
      cplx a0 = A0[2 * o] + I * A0[2 * o + 1];
      cplx a1 = A1[2 * o] + I * A1[2 * o + 1];
      ns_add(&zdh, creal(a0 * conj(r0) + a1 * conj(r1)));                   /* eq. (d_h_rel_bin) */
      ns_add(&zhh, B0[o] * creal(r0 * conj(r0)) + 2.0 * B1[o] * creal(r0 * conj(r1))); /* eq. (h_h_rel_bin) */
    }
  double Zdh = 4.0 * ns_val(&zdh), Zhh = 4.0 * ns_val(&zhh);
  *lnL = -0.5 * (dd + Zhh - 2.0 * Zdh); /* eq. (like) */
  if (dh) *dh = Zdh;
  if (hh) *hh = Zhh;
}

void oracle_het_core_residual(int n_chan, int n_bins, const double *edges, const double *A0,
                              const double *A1, const double *B0, const double *B1, double dd,
                              const double *h0_edges, const double *h_edges, double *lnL) {
  nsum sa0 = {0, 0}, sb0 = {0, 0}, acc = {0, 0};
  for (int c = 0; c < n_chan; ++c)
    for (int b = 0; b < n_bins; ++b) {
      int64_t o = (int64_t)c * n_bins + b;
      ns_add(&sa0, A0[2 * o]);
      ns_add(&sb0, B0[o]);
      int64_t e0 = (int64_t)c * (n_bins + 1) + b;
      cplx da = ratio_at(h_edges, h0_edges, e0) - 1.0;
      cplx db = ratio_at(h_edges, h0_edges, e0 + 1) - 1.0;
      cplx d0 = 0.5 * (da + db);
      cplx d1 = (db - da) / (edges[b + 1] - edges[b]);
      cplx a0 = A0[2 * o] + I * A0[2 * o + 1] - B0[o];
      cplx a1 = A1[2 * o] + I * A1[2 * o + 1] - B1[o];
      ns_add(&acc, 4.0 * creal(a0 * conj(d0) + a1 * conj(d1)));
      ns_add(&acc, -2.0 * (B0[o] * creal(d0 * conj(d0)) + 2.0 * B1[o] * creal(d0 * conj(d1))));
    }
  double lnL0 = -0.5 * dd + 4.0 * ns_val(&sa0) - 2.0 * ns_val(&sb0);
  *lnL = lnL0 + ns_val(&acc);
}

int oracle_loglike_het(int model, uint32_t modes, int64_t W, const double *theta, int n_chan,
                       int n_bins, const double *edges, const double *A0, const double *A1,
                       const double *B0, const double *B1, double dd, const double *h0_edges,
                       double t_obs, double *lnL, double *dh, double *hh) {
  if (n_chan != oracle_n_chan(model)) return OR_EINVAL;
  int E = n_bins + 1;
#pragma omp parallel
  {
    double *he = (double *)malloc(sizeof(double) * 2 * n_chan * E);
#pragma omp for schedule(dynamic, 4)
    for (int64_t w = 0; w < W; ++w) {
      src_t s;
      src_setup(model, modes, theta + w * OR_NPARAM, &s);
      if (!s.valid) {
        lnL[w] = -INFINITY;
        if (dh) dh[w] = 0.0;
        if (hh) hh[w] = 0.0;
        continue;
      }
      for (int j = 0; j < E; ++j) {
        cplx hp[3];
        tmpl_point(&s, edges[j], t_obs, hp);
        for (int c = 0; c < n_chan; ++c) {
          he[2 * (c * E + j)] = creal(hp[c]);
          he[2 * (c * E + j) + 1] = cimag(hp[c]);
        }
      }
      double a, b, cc;
      oracle_het_core(n_chan, n_bins, edges, A0, A1, B0, B1, dd, h0_edges, he, &a, &b, &cc);
      lnL[w] = a;
      if (dh) dh[w] = b;
      if (hh) hh[w] = cc;
    }
    free(he);
  }
  return OR_OK;
}
