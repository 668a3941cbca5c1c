/*
 * mbh_oracle.h -- plain FP64 CPU oracle for the heterodyned (relative-binning)
 * and full-grid likelihoods of Katz (2021), arXiv:2111.01064.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, constant or helper with the GPU library, and the GPU library never
 * calls it.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.
 *
 * Conventions (all host pointers, all FP64, row-major):
 *   theta        [W][11]  {M_T [Msun], q=m2/m1, a1, a2, D_L [Gpc], phi_ref,
 *                          iota, lambda, beta, psi, t_ref [s]}   (Sec. 2.1)
 *                model OR_MODEL_TF2 uses slots {Mc [Msun], amp, t_c, phi_c}.
 *   complex data [n_chan][n][2]  (re, im)
 *   psd          [n_chan][n]
 *   Fourier grid f_k = f0 + k*df, k = 0..n_f-1.
 */
#ifndef MBH_ORACLE_H
#define MBH_ORACLE_H
#include <stdint.h>

#define OR_NPARAM 11
#define OR_MODEL_IMR 0   /* IMR-lite modes + LISA A/E/T response, 3 channels */
#define OR_MODEL_TF2 1   /* 0PN chirp, one channel, no response            */

/* harmonic-mode bits, order fixed: (2,2) (3,3) (4,4) (2,1) (3,2) (4,3) */
#define OR_MODE_22 (1u << 0)
#define OR_MODE_33 (1u << 1)
#define OR_MODE_44 (1u << 2)
#define OR_MODE_21 (1u << 3)
#define OR_MODE_32 (1u << 4)
#define OR_MODE_43 (1u << 5)

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EBAND (-3)

int oracle_n_chan(int model);

/* spin-weight -2 spherical harmonic */
void oracle_sylm(int l, int m, double theta, double phi, double *re, double *im);

/* (l,m) mode amplitude, phase phi_lm (without the t_ref shift) and t_lm(f);
 * on[i] = 1 if (f, lm) is inside the template support. */
int oracle_mode(const double *theta, int l, int m, int n, const double *f,
                double *amp, double *phase, double *tf, int *on);

/* f_max, the frequency of the maximum of f^2 A_22 */
double oracle_fmax(const double *theta);

/* spacecraft positions p[k][xyz] in seconds at SSB time t */
void oracle_orbit(double t, double *p);

/* one-link transfer y_{i->j} (complex) for a plane wave with polarisation
 * content H = Kp e+ + Kc ex, spacecraft positions p[3][3] (seconds). */
void oracle_link(int i, int j, double f, const double *p, double lam, double beta,
                 double psi, const double *Kp, const double *Kc, double *y);

/* TDI X,Y,Z and A,E,T transfer for one mode at (f, t): out[6][2] = X,Y,Z,A,E,T */
void oracle_tdi(double f, double t, double lam, double beta, double psi,
                const double *Kp, const double *Kc, double *out);

/* template on arbitrary frequencies: h[n_chan][n][2] */
int oracle_template(int model, uint32_t modes, const double *theta, int64_t n,
                    const double *f, double t_obs, double *h);

/* eq. (inner): 4 Re sum_c sum_k conj(a) b / S df */
double oracle_inner(int n_chan, int64_t n_f, const double *a, const double *b,
                    const double *psd, double df);

/* eq. (like) on the full grid, W walkers (OpenMP over walkers) */
int oracle_loglike_full(int model, uint32_t modes, int64_t W, const double *theta,
                        int n_chan, int64_t n_f, double f0, double df, double t_obs,
                        const double *d, const double *psd,
                        double *lnL, double *dh, double *hh);

/* full-grid likelihood of a given template array (no waveform) */
double oracle_loglike_of(int n_chan, int64_t n_f, const double *d, const double *h,
                         const double *psd, double df, double *dh, double *hh);

/* reference preparation: band, log-spaced edges, bin assignment and the
 * per-bin sums A0, A1, B0, B1 (and the dropped B2) per channel. */
int oracle_reference(int model, uint32_t modes, const double *theta0,
                     int n_chan, int64_t n_f, double f0, double df, double t_obs,
                     const double *d, const double *psd, int n_bins,
                     int64_t *k_lo, int64_t *k_hi,
                     double *edges,      /* [n_bins+1]              */
                     int64_t *kb,        /* [n_bins+1] first k of bin b; kb[n_bins] = k_hi+1 */
                     double *A0, double *A1,   /* [n_chan][n_bins][2] */
                     double *B0, double *B1, double *B2, /* [n_chan][n_bins] */
                     double *dd,         /* <d|d> */
                     double *h0_edges);  /* [n_chan][n_bins+1][2] */

/* per-bin sums for explicit edges and an explicit reference template
 * h0[n_chan][n_f][2] on the grid; grid points lo..hi are binned. */
void oracle_bin_sums(int n_chan, int64_t n_f, double f0, double df, const double *d,
                     const double *psd, const double *h0, int n_bins, const double *edges,
                     int64_t lo, int64_t hi, int64_t *kb, double *A0, double *A1, double *B0,
                     double *B1, double *B2);

/* binned likelihood from a reference and the template at the edges, in the
 * form printed in the paper; also returns Z[d,h] and Z[h,h]. */
void oracle_het_core(int n_chan, int n_bins, const double *edges,
                     const double *A0, const double *A1, const double *B0,
                     const double *B1, double dd, const double *h0_edges,
                     const double *h_edges, double *lnL, double *dh, double *hh);

/* the same quantity in residual form (algebraically identical) */
void oracle_het_core_residual(int n_chan, int n_bins, const double *edges,
                              const double *A0, const double *A1, const double *B0,
                              const double *B1, double dd, const double *h0_edges,
                              const double *h_edges, double *lnL);

/* heterodyned likelihood of W walkers (OpenMP over walkers) */
int oracle_loglike_het(int model, uint32_t modes, int64_t W, const double *theta,
                       int n_chan, int n_bins, const double *edges,
                       const double *A0, const double *A1, const double *B0,
                       const double *B1, double dd, const double *h0_edges,
                       double t_obs, double *lnL, double *dh, double *hh);

int oracle_max_threads(void);
#endif
