/*
 * mbh.h -- C ABI of libmbh, the MI355X (gfx950) library for the batched
 * heterodyned ("relative binning") and full-grid log-likelihoods of massive
 * black hole binaries with the LISA A/E/T response (Katz 2021,
 * arXiv:2111.01064).
 *
 * Conventions for every entry point:
 *  - Return value: mbh_status, MBH_OK (0) on success, a negative code on
 *    failure.  No entry point aborts, throws or exits; mbh_last_error()
 *    gives a human-readable message for the calling thread's last failure.
 *  - Pointers marked _dev are device (HBM) pointers owned by the caller,
 *    e.g. torch.cuda tensors' data_ptr(); pointers marked _host are host
 *    memory owned by the caller.  Everything behind an opaque handle is
 *    owned by the library and freed by the matching *_release / destroy.
 *  - Layouts are row-major.  Complex arrays are interleaved (re, im) FP64.
 *  - Work is enqueued on the given stream and is asynchronous unless stated;
 *    outputs are valid after the stream is synchronised.  Handles are
 *    immutable after creation, so concurrent calls on different streams may
 *    share them.
 *  - Walker parameters theta[W][11] follow Sec. 2.1 of the paper:
 *      {M_T [Msun], q = m2/m1, a1, a2, D_L [Gpc], phi_ref, iota,
 *       lambda, beta, psi, t_ref [s]}  (SSB frame).
 *    For MBH_MODEL_TF2 (single-channel 0PN chirp) the slots are
 *      {Mc [Msun], amplitude, t_c [s], phi_c, unused...}.
 *    A walker outside the model domain (non-finite entries, M_T <= 0,
 *    q outside [0.05, 1], |a_i| > 0.99, D_L <= 0; Mc <= 0 for TF2) gets
 *    lnL = -inf (never NaN) and <d|h> = <h|h> = 0; the call still succeeds.
 */
#ifndef MBH_H
#define MBH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mbh_status;
#define MBH_OK 0
#define MBH_EINVAL (-1)   /* bad argument, shape or null pointer           */
#define MBH_ENOMEM (-2)   /* device allocation failed or HBM budget exceeded */
#define MBH_EBAND (-3)    /* reference template empty or zero at a bin edge  */
#define MBH_EDEVICE (-4)  /* a HIP runtime call failed                       */
#define MBH_EAGAIN (-5)   /* serving: request not finished / queue full      */
#define MBH_ENOTFOUND (-6)/* serving: unknown request id                     */

/* waveform models */
#define MBH_MODEL_IMR 0   /* IMR-lite harmonics + LISA TDI A/E/T, 3 channels */
#define MBH_MODEL_TF2 1   /* 0PN chirp, 1 channel, no response             */

/* harmonic modes (bit mask, MBH_MODEL_IMR only); (2,2) is Sec. 2.1's dominant mode */
#define MBH_MODE_22 (1u << 0)
#define MBH_MODE_33 (1u << 1)
#define MBH_MODE_44 (1u << 2)
#define MBH_MODE_21 (1u << 3)
#define MBH_MODE_32 (1u << 4)
#define MBH_MODE_43 (1u << 5)
#define MBH_MODES_ALL 0x3Fu

typedef enum { MBH_FP64 = 0, MBH_MIXED = 1 } mbh_precision;

typedef struct mbh_ctx mbh_ctx;
typedef struct mbh_data mbh_data;
typedef struct mbh_ref mbh_ref;
typedef struct mbh_batch mbh_batch;
typedef struct mbh_server mbh_server;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context's handles and scratch may hold (0 = no cap).
 * Errors: MBH_EINVAL (bad device / null out), MBH_EDEVICE. */
mbh_status mbh_create(int device, size_t hbm_budget_bytes, mbh_ctx **out);
/* Release the caller's context handle.  Data, references, batches and servers
 * created from the context keep it alive: it is freed when the last of them
 * is released, so handles may be released in any order. */
mbh_status mbh_destroy(mbh_ctx *ctx);

/* Message of the calling thread's last failed call ("" if none). */
const char *mbh_last_error(void);
const char *mbh_strerror(mbh_status s);

/* Device memory currently held by the context's handles and scratch. */
mbh_status mbh_memory_in_use(const mbh_ctx *ctx, size_t *bytes_out);

/* ------------------------------------------------------------------- data */

/* Frequency-domain data d(f) and noise PSD S_n(f) of n_chan channels on the
 * uniform grid f_k = f0 + k*df, k = 0..n_freq-1 (eq. inner of Sec. 2: the
 * PSDs are known analytic inputs).
 *   d_reim_dev [n_chan][n_freq][2] FP64, psd_dev [n_chan][n_freq] FP64 > 0.
 * n_chan is 3 (A, E, T) for MBH_MODEL_IMR and 1 for MBH_MODEL_TF2.
 * t_obs is the observation time bounding the template support.
 * The library copies (whitened) data; the caller may free its inputs once
 * the stream is synchronised.  Also computes <d|d>.
 * Errors: MBH_EINVAL, MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_data_create(mbh_ctx *ctx, int n_chan, int64_t n_freq, double f0, double df,
                           double t_obs, const double *d_reim_dev, const double *psd_dev,
                           hipStream_t stream, mbh_data **out);
mbh_status mbh_data_release(mbh_data *data);
/* <d|d> (synchronises the creation stream on first use). */
mbh_status mbh_data_inner_dd(mbh_data *data, double *dd_out);

/* TDI ingest (Sec. 2.1): the A, E, T frequency series of X, Y, Z time
 * series.  A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3
 * (the combination the paper gives), each multiplied by a Tukey window
 * (cosine tapers of alpha (N - 1) / 2 samples at either end; alpha = 0: no
 * window) and Fourier transformed in the templates' convention:
 *   out_c(f_k) = dt sum_n w_n c(t0 + n dt) e^{-2 pi i f_k (t0 + n dt)},
 *   f_k = k / (N dt),  k = k_first .. k_first + n_freq - 1.
 *   xyz_dev [3][N] FP64 on the device (X, then Y, then Z; sample n at time
 *   t0 + n dt), caller-owned; aet_dev [3][n_freq][2] FP64 (re, im), the
 *   layout mbh_data_create takes.
 * Requires 4 <= N < 2^31, dt > 0, finite t0, 0 <= alpha <= 1, k_first >= 1,
 * n_freq >= 2 and k_first + n_freq - 1 <= N / 2.  Allocates device scratch
 * (~72 N bytes plus the transform's work area, released in stream order) and,
 * on the first call with a given N, an FFT plan that the context keeps until
 * it is destroyed.  Does not synchronise: xyz_dev must stay valid, and
 * aet_dev is written, in stream order.
 * Errors: MBH_EINVAL, MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_tdi_to_aet_fd(mbh_ctx *ctx, int64_t n_samples, double dt, double t0,
                             const double *xyz_dev, double tukey_alpha, int64_t k_first,
                             int64_t n_freq, double *aet_dev, hipStream_t stream);
/* Data handle straight from X, Y, Z time series: mbh_tdi_to_aet_fd on the
 * band, then mbh_data_create on the grid f0 = k_first / (N dt),
 * df = 1 / (N dt) with psd_dev [3][n_freq] (A, E, T PSDs on that grid).
 * Synchronises `stream`; the caller may free its inputs on return.
 * Errors: as mbh_tdi_to_aet_fd and mbh_data_create. */
mbh_status mbh_data_create_tdi(mbh_ctx *ctx, int64_t n_samples, double dt, double t0,
                               const double *xyz_dev, double tukey_alpha, int64_t k_first,
                               int64_t n_freq, const double *psd_dev, double t_obs,
                               hipStream_t stream, mbh_data **out);

/* Template h^c(f_k) of one parameter vector on the data grid (eq. response
 * of Sec. 2.1), FP64, written to h_dev [n_chan][n_freq][2].  For synthetic
 * signal injection and tests.  Errors: MBH_EINVAL (incl. invalid theta). */
mbh_status mbh_template_full(mbh_ctx *ctx, const mbh_data *data, int model, uint32_t modes,
                             const double *theta_host, double *h_dev, hipStream_t stream);

/* ------------------------------------------------------- reference (a9) */

/* Heterodyne precompute of Sec. 2.2 / Sec. 3.2: the band [F_0, F_Nb] is the
 * first and last grid frequency where the reference h0 = h(theta0) is non
 * zero; n_bins log-spaced bins (half-open, the last closed); per bin and
 * channel the sums A0, A1, B0, B1 of eqs. (d_h_rel_bin) and (h_h_rel_bin)
 * over the grid, lnL(h0) = -1/2 <d-h0|d-h0>, and h0 at the bin edges.
 * Synchronises `stream` (the band must be known on the host).
 * Errors: MBH_EINVAL (bad args, invalid theta0, n_bins outside [1, 4096]),
 * MBH_EBAND (h0 empty on the grid or exactly zero at an edge), MBH_ENOMEM. */
mbh_status mbh_build_reference_coeffs(mbh_ctx *ctx, const mbh_data *data, int model,
                                      uint32_t modes, const double *theta0_host, int n_bins,
                                      hipStream_t stream, mbh_ref **out);
mbh_status mbh_ref_release(mbh_ref *ref);

typedef struct {
  int32_t model, n_chan, n_bins;
  uint32_t modes;
  int64_t k_lo, k_hi;  /* band in grid indices                           */
  double lnL0;         /* lnL(h0) = -1/2 <d-h0|d-h0>                      */
  double dd, dh0, hh0; /* <d|d>, <d|h0>, <h0|h0>                          */
} mbh_ref_info;
mbh_status mbh_ref_get_info(const mbh_ref *ref, mbh_ref_info *out);

/* Copy the reference out to host buffers, in the paper's form:
 *   edges [n_bins+1], kb [n_bins+1] (first grid index of bin b;
 *   kb[n_bins] = k_hi + 1), A0, A1 [n_chan][n_bins][2], B0, B1
 *   [n_chan][n_bins], h0_edges [n_chan][n_bins+1][2].  Any pointer may be
 *   NULL.  Synchronous. */
mbh_status mbh_ref_export(const mbh_ref *ref, double *edges, int64_t *kb, double *A0, double *A1,
                          double *B0, double *B1, double *h0_edges);

/* Per-mode relative binning for higher modes: Sec. 2.2's relative binning
 * applied to every harmonic mode of the reference on its own.  Mode L of
 * h0 = h(theta0) gets its own band (first and last grid frequency where
 * h0_L != 0 in any channel; a mode with no band takes no part), n_bins_mode[L]
 * log-spaced bins over it (half-open, the last closed) and its own ratio
 * r_L = h_L / h0_L, fitted by a complex line across each of its bins.
 * <d|h> and the diagonal <h_L|h_L> terms are eqs. (d_h_rel_bin) and
 * (h_h_rel_bin) per mode; the cross terms <h_L|h_L'> are summed on the merged
 * edge grid of the two modes (the union of their edges over the overlap of
 * their bands), with both lines evaluated at each merged bin's centre and
 * their product linearised about it.  IMR model only; the likelihood calls
 * (mbh_loglike_heterodyned, batches) evaluate such a reference in MBH_FP64
 * only and return MBH_EINVAL for MBH_MIXED.  Not for the server, the
 * device reference update, mbh_loglike_heterodyned_noalloc, the autotuner or
 * mbh_ref_export (MBH_EINVAL); mbh_ref_get_info reports the total bin count
 * and the union of the bands.  A likelihood call over such a reference runs
 * an edge pass (every mode edge of every walker) and a cross pass (every
 * merged bin); the cross pass takes one workgroup per walker, or per two
 * walkers while their values stay within 64 KB, with the edge values staged
 * in LDS (48 B per mode edge and walker) when they fit the LDS of one
 * workgroup, else a chunked form; the environment variable
 * MBH_PM_CROSS_LDS_MAX (bytes), read by mbh_create, lowers that limit for
 * the context (0: always the chunked form).  Both forms give results within
 * the FP64 rounding of each other.
 *   n_bins_mode [6] (host): bins of each mode in the mask, in the order of
 *   the MBH_MODE_* bits, each in [1, 4096].
 * Synchronises `stream`.  Device memory during the build: 16 B per grid
 * point, channel and mode, plus one more such array.
 * Errors: MBH_EINVAL, MBH_EBAND (no mode has a band, or a mode's reference
 * is exactly zero at one of its edges), MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_build_reference_coeffs_pm(mbh_ctx *ctx, const mbh_data *data, int model,
                                         uint32_t modes, const double *theta0_host,
                                         const int32_t *n_bins_mode, hipStream_t stream,
                                         mbh_ref **out);
/* Modes of a per-mode reference that have bins (bit mask) and the number of
 * mode pairs with overlapping bands.  MBH_EINVAL for other references. */
mbh_status mbh_ref_pm_info(const mbh_ref *ref, uint32_t *modes_with_bins, int32_t *n_pairs);
/* One mode of a per-mode reference, to host buffers (any may be NULL; call
 * with NULL buffers to learn n_bins first): band k_lo..k_hi, edges
 * [n_bins+1], kb [n_bins+1] (first grid index of each bin, kb[n_bins] =
 * k_hi + 1), the residual-form sums Ares0, Ares1 [3][n_bins][2]
 * (sum (d - h0) conj(h0_L) / S df and the same times (f - f_b)), B0, B1
 * [3][n_bins] (|h0_L|^2 / S df and times (f - f_b)), h0_edges
 * [3][n_bins+1][2] (h0_L at its edges).  mode_index is the bit position of
 * the mode (0 = (2,2)); MBH_EINVAL if the mode has no bins. */
mbh_status mbh_ref_pm_mode(const mbh_ref *ref, int mode_index, int64_t *k_lo, int64_t *k_hi,
                           int32_t *n_bins, double *edges, int64_t *kb, double *Ares0,
                           double *Ares1, double *B0, double *B1, double *h0_edges);
/* One mode pair of a per-mode reference (pairs ordered by mode index):
 * the two modes, the merged edges [n_merged+1], kb [n_merged+1], each mode's
 * own bin holding each merged bin (bin_a, bin_b [n_merged]), and the sums
 * C0 = sum h0_a conj(h0_b) / S df and C1 = the same times (f - f_m)
 * [3][n_merged][2].  Any pointer may be NULL. */
mbh_status mbh_ref_pm_pair(const mbh_ref *ref, int pair, int32_t *mode_a, int32_t *mode_b,
                           int32_t *n_merged, double *edges, int64_t *kb, int32_t *bin_a,
                           int32_t *bin_b, double *C0, double *C1);

/* Reference update of Sec. 3.2 (the reference is replaced, every few
 * thousand sampler iterations, by the highest-likelihood point of the
 * population), done on the device with no host round trip.  Picks the
 * walker with the largest finite lnL_dev[w] (the lowest index among equal
 * values; NaN and +-inf are skipped) and rebuilds `ref` in place from
 * theta_dev[w] exactly as mbh_build_reference_coeffs would: same model,
 * modes and n_bins, new band, edges, bin assignment, coefficients, lnL(h0).
 *   theta_dev [W][11] FP64 and lnL_dev [W] FP64 on the device, caller-owned
 *   (typically the walkers and the heterodyned lnL the sampler holds);
 *   `data` must be the data the reference was built on.
 * Asynchronous on `stream`; nothing is synchronised.  Work issued later on
 * `stream` (likelihood calls, batch launches, also batches created before
 * the refresh: they read the reference's device arrays) sees the new
 * reference; work on other streams must be ordered by the caller, and must
 * not run on `ref` while the refresh does.  For a reference resident in a
 * server, use mbh_server_refresh, which orders the update with the
 * server's own streams.  The outcome is known on the
 * device only: if no walker has a finite lnL, the picked walker lies outside
 * the model domain (MBH_EINVAL) or its template is empty on the grid or zero
 * at an edge (MBH_EBAND), the reference is left unchanged; read the outcome
 * with mbh_ref_refresh_result.  mbh_ref_get_info and mbh_ref_export wait for
 * the last refresh and report the live reference.
 * The first refresh of a reference allocates its staging and work buffers
 * (about 16 B per grid point and channel, plus a few times the reference's
 * size; freed with the reference) and synchronises `stream` once; later
 * refreshes allocate nothing and only enqueue kernels.  The work buffers are
 * the reference's own: refreshes of one reference must be ordered (issue
 * them on one stream).
 * Errors returned at once: MBH_EINVAL (null pointers, W < 1, another
 * context, a data grid other than the reference's), MBH_ENOMEM,
 * MBH_EDEVICE. */
mbh_status mbh_ref_refresh(mbh_ctx *ctx, const mbh_data *data, mbh_ref *ref,
                           const double *theta_dev, const double *lnL_dev, int64_t W,
                           hipStream_t stream);
/* Allocate the update buffers of `ref` now (what its first mbh_ref_refresh
 * would do: device memory and one synchronisation of `stream`), so that no
 * update allocates.  Idempotent.  Errors: MBH_EINVAL, MBH_ENOMEM,
 * MBH_EDEVICE. */
mbh_status mbh_ref_refresh_prepare(mbh_ref *ref, hipStream_t stream);
/* Outcome of the last mbh_ref_refresh of `ref` (waits for it): its status
 * (MBH_OK, or the reason the reference was left unchanged), the walker it
 * picked (-1 if none) and the number of refreshes committed so far.  Before
 * any refresh: MBH_OK, -1, 0.  Any out pointer may be NULL. */
mbh_status mbh_ref_refresh_result(mbh_ref *ref, int32_t *status, int64_t *pick,
                                  int32_t *generation);

/* ---------------------------------------------------- likelihoods (a1-a8) */

/* Heterodyned log-likelihood of W walkers against a reference (Sec. 2.2):
 * the template at the N_b+1 bin edges, r = h/h0, the complex line across
 * each bin (r0 at the bin centre, slope r1) and the contraction with the
 * per-bin coefficients, evaluated in the algebraically identical residual
 * form lnL(h0) + sum_b {...} so that FP32 terms stay small.
 *   theta_dev [W][11] FP64; lnL_dev [W] FP64; dh_hh_dev [W][2] (Z[d,h],
 *   Z[h,h]) or NULL.  MBH_FP64 runs every step in FP64.  MBH_MIXED runs the
 *   sinc series of the six link transfers, the link phase factors and the
 *   sine and cosine of the (FP64-reduced) carrier difference to h0 in FP32,
 *   and everything else (phases, times, Doppler, geometry, per-walker
 *   amplitude and polarisation factors, the ratio and the contraction) in
 *   FP64.  The FP32 error of lnL is estimated per segment of a walker's
 *   bins (the bins one wavefront handles); segments whose share could take
 *   the walker's estimate above the tolerance (9e-4 by default, see
 *   mbh_set_mixed_tolerance) are recomputed in FP64 by the same wavefront,
 *   so mixed results stay within 1e-3 of FP64.
 * Errors: MBH_EINVAL, MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_loglike_heterodyned(mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev,
                                   int64_t W, mbh_precision prec, double *lnL_dev,
                                   double *dh_hh_dev, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work
 * and results of mbh_loglike_heterodyned, with its scratch (walker constants
 * and partial sums) taken from a fixed device array of
 * MBH_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends (its address is resolved once per device by mbh_create).
 * The call allocates nothing, neither device nor host memory.  A call of W
 * walkers at N_b bins needs W * 568 bytes (rounded up to 256) plus
 * W * 32 * ((N_b - 1) / 63 + 2) bytes; larger calls are refused with
 * MBH_EINVAL and a message (at 128 bins about 36 000 walkers fit).  Every
 * call on one GPU shares that GPU's array: calls that overlap on the device
 * (on different streams, or from several contexts on one GPU) race and give
 * wrong results, so the caller must order them, e.g. issue them on one
 * stream.  The array keeps the last call's contents; nothing in it needs to
 * start at zero.  Arguments, outputs and errors as mbh_loglike_heterodyned. */
#define MBH_NOALLOC_SCRATCH_BYTES ((size_t)24 << 20)
mbh_status mbh_loglike_heterodyned_noalloc(mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev,
                                           int64_t W, mbh_precision prec, double *lnL_dev,
                                           double *dh_hh_dev, hipStream_t stream);

/* Full-grid log-likelihood -1/2 <d-h|d-h> (eqs. like and inner, Sec. 2) of W
 * walkers: the template is generated on every grid frequency on the fly and
 * never stored; lnL is formed as -1/2 (<d|d> + sum (|h|^2 - 2 Re d* h)), so
 * grid points outside the template's support add nothing.  Same argument
 * conventions as above.  Every step runs in FP64 for either precision:
 * MBH_MIXED is accepted and gives the FP64 results (on this hardware FP32
 * arithmetic issues at the FP64 rate; an FP32 response loses accuracy where
 * the TDI combinations cancel, and an FP32 carrier with the error control it
 * then needs is slower than FP64).  The grid tile is the context's
 * (mbh_set_full_shape, mbh_autotune_full); results do not depend on its
 * walkers per workgroup and differ between frequencies-per-thread settings
 * only by rounding.
 * Errors: MBH_EINVAL, MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_loglike_full(mbh_ctx *ctx, const mbh_data *data, int model, uint32_t modes,
                            const double *theta_dev, int64_t W, mbh_precision prec,
                            double *lnL_dev, double *dh_hh_dev, hipStream_t stream);

/* ------------------------------------------------------ batching (a10) */

/* One launch over many (reference, walker batch) items with ragged modes,
 * bin counts and walker counts.  Items are packed into a device work list of
 * tiles, grouped by mapping and longest first within a group (one grid of
 * one workgroup per tile per group, between the setup and totals grids);
 * the whole pass is captured once into a HIP graph and replayed by
 * mbh_batch_launch.  The mapping of
 * each item (see mbh_set_lanes) comes from the autotuner table (per bin count
 * and mode count), so a walker's result depends only on its inputs, its
 * reference and its index within its item, never on the rest of the batch.
 *   refs[n], theta_dev[n] ([W_i][11]), W[n], lnL_dev[n] ([W_i]),
 *   dh_hh_dev[n] (each [W_i][2] or NULL; the array itself may be NULL).
 * Caller buffers must stay valid while the batch exists.  Items may hold
 * no walkers (W[i] = 0), but not all of them.
 * Errors: MBH_EINVAL (also for a batch with no walkers at all), MBH_ENOMEM,
 * MBH_EDEVICE. */
mbh_status mbh_batch_create(mbh_ctx *ctx, int n, const mbh_ref *const *refs,
                            const double *const *theta_dev, const int64_t *W,
                            double *const *lnL_dev, double *const *dh_hh_dev,
                            mbh_precision prec, mbh_batch **out);
/* The same with a precision per item (precs[n], MBH_FP64 or MBH_MIXED):
 * the tiles are grouped by precision as well, each item's results are those
 * of the uniform batch (or the single call) in its own precision.  For
 * populations whose hot part gains nothing from the mixed path (walkers far
 * from the reference mostly exceed the FP32 error budget and are computed
 * twice), e.g. a tempered ensemble with its cold rungs mixed and the rest in
 * FP64.  Per-mode references must be MBH_FP64.  Errors: as mbh_batch_create. */
mbh_status mbh_batch_create_prec(mbh_ctx *ctx, int n, const mbh_ref *const *refs,
                                 const double *const *theta_dev, const int64_t *W,
                                 double *const *lnL_dev, double *const *dh_hh_dev,
                                 const mbh_precision *precs, mbh_batch **out);
mbh_status mbh_batch_launch(mbh_batch *batch, hipStream_t stream);
/* The same work as mbh_batch_launch, issued as the batch's kernel launches on
 * the stream (setup, one main-pass grid per mapping group, totals) instead of
 * one graph replay; results are bit-identical.  On ROCm a graph replay costs
 * several microseconds more per launch than the equivalent stream launches,
 * which matters for steps of a few tens of microseconds.  The launches can
 * themselves be captured into a caller's graph.
 * Errors: MBH_EINVAL, MBH_EDEVICE. */
mbh_status mbh_batch_launch_direct(mbh_batch *batch, hipStream_t stream);
/* One stage of the same work launched on its own (stream launches), for
 * measuring stages separately: MBH_STAGE_SETUP (walker constants, a1),
 * MBH_STAGE_MAIN (the heterodyned main pass, a2-a7, with the mixed path's
 * FP64 recomputation: the dominant kernel), MBH_STAGE_FINISH (per-walker
 * totals).  Launching the three in this order on one stream is the work of
 * mbh_batch_launch.
 * Errors: MBH_EINVAL, MBH_EDEVICE. */
enum { MBH_STAGE_SETUP = 1, MBH_STAGE_MAIN = 2, MBH_STAGE_FINISH = 3 };
mbh_status mbh_batch_launch_stage(mbh_batch *batch, int stage, hipStream_t stream);
/* Walker segments of this batch that the mixed path recomputed in FP64 (see
 * mbh_loglike_heterodyned; a segment is a walker's bins within one
 * 63-bin chunk of the flattened mapping, or the whole walker in a lane-group
 * mapping), summed over all launches so far.  Synchronous. */
mbh_status mbh_batch_fp64_segments(const mbh_batch *batch, uint64_t *count_out);
mbh_status mbh_batch_release(mbh_batch *batch);

/* --------------------------------------------------------- autotuner */

/* Time the heterodyned kernel for each mapping (flattened, and lane groups
 * of 16, 32 and 64 lanes per walker) at this reference's shape and record the
 * fastest in the context's table (saved and restored by
 * mbh_autotune_save/load).  theta_dev [W][11] (device) are representative
 * walkers, e.g. the sampler's current ensemble; if NULL, W copies of a fixed
 * valid parameter point are used.  Synchronous.  lanes_out may be NULL. */
mbh_status mbh_autotune_heterodyned(mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev,
                                    int64_t W, mbh_precision prec, int *lanes_out);
/* Mapping the library uses for this shape (table, else 0). */
mbh_status mbh_lanes_for(const mbh_ctx *ctx, int n_bins, int n_modes, mbh_precision prec,
                         int *lanes_out);
/* Set the mapping of the heterodyned pass for a shape: 0 = flattened (one
 * lane per walker and bin edge, 63 bins per wavefront; the default), or
 * 1..64 (power of two) lanes per walker.  Results differ between mappings
 * only by rounding. */
mbh_status mbh_set_lanes(mbh_ctx *ctx, int n_bins, int n_modes, mbh_precision prec, int lanes);
/* Tolerance of the mixed path on the estimated FP32 error of each walker's
 * lnL (default 9e-4): work whose share of the estimate could exceed it is
 * recomputed in FP64.  0 recomputes everything (mixed results then equal the
 * FP64 path's bit for bit); +inf recomputes nothing (the plain FP32 error,
 * for measurement).  Applies to calls, batches and server batches created
 * afterwards.  Errors: MBH_EINVAL for a negative or NaN tolerance. */
mbh_status mbh_set_mixed_tolerance(mbh_ctx *ctx, double tol);
mbh_status mbh_get_mixed_tolerance(const mbh_ctx *ctx, double *tol_out);
/* Tile of the full-grid pass for a mode class (higher_modes 0: the (2,2)
 * mode alone or the chirp model; 1: any other mode mask): kf grid
 * frequencies per thread (1 or 2) and at most wpb_cap walkers per workgroup
 * (8, 16, 32, 64 or 128).  Default (1, 32).  Applies to later calls.
 * Errors: MBH_EINVAL for another value. */
mbh_status mbh_set_full_shape(mbh_ctx *ctx, int higher_modes, int kf, int wpb_cap);
mbh_status mbh_full_shape(const mbh_ctx *ctx, int higher_modes, int *kf_out, int *wpb_cap_out);
/* Time mbh_loglike_full over every supported tile with these walkers
 * (theta_dev [W][11] on the device, e.g. the sampler's ensemble) and record
 * the fastest for this mode class; synchronous.  Outputs may be NULL.
 * Errors: as mbh_loglike_full. */
mbh_status mbh_autotune_full(mbh_ctx *ctx, const mbh_data *data, int model, uint32_t modes,
                             const double *theta_dev, int64_t W, int *kf_out, int *wpb_cap_out);
/* Save or load the tuned mappings and full-grid tiles (a text file, one
 * entry per line; entries of another architecture are ignored). */
mbh_status mbh_autotune_save(const mbh_ctx *ctx, const char *path);
mbh_status mbh_autotune_load(mbh_ctx *ctx, const char *path);

/* --------------------------------------------------------- serving (a11) */

typedef struct {
  int32_t max_inflight;      /* batches in flight on the device (>= 1)           */
  int32_t max_batch_walkers; /* walkers packed into one launch                    */
  size_t hbm_budget_bytes;   /* device memory for in-flight request buffers       */
  mbh_precision prec;
} mbh_server_config;

/* Continuous-batching request server over resident references.  A
 * scheduler thread packs queued requests into batches as walker slots and
 * HBM budget free up, launches them on its own streams (several in flight),
 * and completes each request when its batch's event fires.
 * Errors: MBH_EINVAL, MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_server_create(mbh_ctx *ctx, int n_refs, const mbh_ref *const *refs,
                             const mbh_server_config *cfg, mbh_server **out);
/* Enqueue W walkers (host memory, copied) for reference ref_index.
 * Returns MBH_EAGAIN if the request alone exceeds the batch or budget caps. */
mbh_status mbh_server_submit(mbh_server *srv, int ref_index, const double *theta_host,
                             int64_t W, uint64_t *request_id);
/* Queue the reference update of Sec. 3.2 (see mbh_ref_refresh) for resident
 * reference ref_index, in submission order: requests submitted before it are
 * evaluated against the old reference, requests submitted after it against
 * the new one.  The population (theta_host [W][11], lnL_host [W], host
 * memory, copied) is the one the update picks its best walker from; `data`
 * must be the data the reference was built on and stay alive until the
 * update has completed.  The update runs on the device, ordered after the
 * batches in flight by their events and before later batches by an event of
 * its own (no host synchronisation).  mbh_server_wait on *request_id
 * returns when it has completed (no results are copied);
 * mbh_ref_refresh_result on the reference gives its outcome.
 * Errors: MBH_EINVAL (bad arguments, another data grid), MBH_EAGAIN (W above
 * the per-batch capacity). */
mbh_status mbh_server_refresh(mbh_server *srv, int ref_index, const mbh_data *data,
                              const double *theta_host, const double *lnL_host, int64_t W,
                              uint64_t *request_id);
/* Copy results of a finished request to host buffers (lnL [W], dh_hh [W][2];
 * either may be NULL) and forget it.  capacity is the number of walkers the
 * caller's buffers hold: MBH_EINVAL (nothing copied, the request kept) if a
 * buffer is given and capacity is below the request's W (0 for a reference
 * update).  timeout_ms < 0 waits forever, 0 polls.  MBH_EAGAIN if not
 * finished in time; MBH_ENOTFOUND for an unknown id; MBH_EDEVICE (and the
 * request forgotten) if its batch or update could not be issued.
 * latency_s_out (may be NULL) = completion time - submit time. */
mbh_status mbh_server_wait(mbh_server *srv, uint64_t request_id, int timeout_ms,
                           double *lnL_host, double *dh_hh_host, int64_t capacity,
                           double *latency_s_out);
/* One request of a trace for mbh_server_replay. */
typedef struct {
  double t_arrival_s; /* seconds after the replay starts; finite, >= 0, non-decreasing */
  int32_t ref_index;  /* resident reference                                          */
  int32_t reserved;   /* 0                                                           */
  int64_t W;          /* walkers, 1 .. the server's per-batch capacity               */
  int64_t theta_row;  /* the request's walkers are theta_host[theta_row .. + W)      */
} mbh_request_spec;
/* Replay a request trace through the server from native code, so that the
 * measured latencies and rates are the server's own (no interpreter in the
 * loop).  The calling thread submits request i (as mbh_server_submit) when
 * the steady clock reaches t_arrival_s after the start, at once if it is
 * behind; a second thread collects the results in request order.  Returns
 * when every request has finished.
 *   theta_host [theta_rows][11] (host, caller-owned; rows may be shared by
 *   requests); latency_s [n]: result available on the host minus the
 *   scheduled arrival (NaN for a request whose batch could not be issued);
 *   submit_lag_s [n] or NULL: submission minus scheduled arrival (how far
 *   the submitting thread fell behind); lnL_host [sum W] or NULL: results
 *   in request order; wall_s or NULL: start to the last result.
 * Requests submitted by other threads meanwhile are served alongside.
 * Errors: MBH_EINVAL (bad trace; nothing submitted), MBH_EAGAIN, MBH_EDEVICE. */
mbh_status mbh_server_replay(mbh_server *srv, const mbh_request_spec *reqs, int64_t n,
                             const double *theta_host, int64_t theta_rows, double *latency_s,
                             double *submit_lag_s, double *lnL_host, double *wall_s);
typedef struct {
  uint64_t submitted, completed, batches, walkers;
  uint64_t max_walkers_in_flight;
  uint64_t max_bytes_in_flight;
  uint64_t admission_waits; /* times the scheduler held work back for budget/slots */
  double host_build_s;      /* scheduler thread: building work lists and issuing launches */
  double host_complete_s;   /* scheduler thread: copying results out */
} mbh_server_stats;
mbh_status mbh_server_get_stats(const mbh_server *srv, mbh_server_stats *out);
mbh_status mbh_server_destroy(mbh_server *srv);

/* ---------------------------------------------------------- sampler (Sec. 3) */

/* Tempered ensemble sampler on the device, as described in Sec. 3 of the
 * paper: an affine-invariant ensemble with parallel tempering, the stretch
 * proposal for most moves and sky-mode hops for the rest, the extracted-SNR
 * stopping rule of the first (full-grid) search, the maximum-likelihood
 * convergence rule of the heterodyned search, and the reference moved to the
 * best walker every few thousand iterations.
 * Sampling coordinates x (11, per walker): (ln M_T, q, a1, a2, D_L, phi_ref,
 * cos iota, lambda, sin beta, psi, t_ref), with a uniform prior on a box
 * (the paper's prior table); the likelihood takes theta (M_T, q, a1, a2, D_L,
 * phi_ref, iota, lambda, beta, psi, t_ref).  Rung k samples
 * L(x)^betas[k] p(x).  Each rung's walkers move in two halves (the first with
 * the second as complement, then the reverse); each walker draws its move:
 * a stretch (partner from the other half, z from g(z) ~ 1/sqrt(z) on
 * [1/a, a], acceptance factor z^10) or, with the shares p_sky_*, a hop to one
 * of the eight sky modes at random (lambda and psi turned by k pi/2, times the
 * reflection beta -> -beta, cos iota -> -cos iota, psi -> pi - psi), a
 * longitudinal turn alone or the reflection alone.  After both halves,
 * adjacent rungs exchange walkers (walker i of rung k with walker (i + s) mod W
 * of rung k + 1, s uniform per iteration and pair).  Every random number is a
 * Philox4x32-10 draw keyed by `seed` with counter (iteration, index, stream,
 * half), so a run is reproducible and independent of launch shapes. */
typedef struct mbh_sampler mbh_sampler;
typedef struct {
  int32_t n_temps;          /* rungs, 1..64                                   */
  int32_t walkers_per_temp; /* even, 4..65536                                 */
  double stretch_a;         /* stretch scale a > 1 (2 is usual)               */
  double p_sky_all, p_sky_lon, p_sky_lat; /* hop shares (the paper: 0.04, 0.03, 0.08) */
  uint64_t seed;
  mbh_precision prec;       /* of the heterodyned / full-grid likelihood      */
  int32_t mixed_rungs;      /* with prec MBH_MIXED and a heterodyned
                               likelihood: only the mixed_rungs coldest rungs
                               run mixed, the rest FP64 (0: every rung mixed) */
} mbh_sampler_config;
/* The likelihood a sampler evaluates: heterodyned against `ref` (IMR; a
 * per-mode reference runs in FP64), or, with ref NULL, the full grid of
 * `data` with `modes` (IMR). */
typedef struct {
  const mbh_ref *ref;
  const mbh_data *data;
  uint32_t modes;
} mbh_likelihood;
/* betas_host [n_temps]: inverse temperatures, betas[0] = 1, strictly
 * decreasing, >= 0.  prior_lo_host, prior_hi_host [11]: the box in x.
 * Errors: MBH_EINVAL, MBH_ENOMEM, MBH_EDEVICE. */
mbh_status mbh_sampler_create(mbh_ctx *ctx, const mbh_sampler_config *cfg, const double *betas_host,
                              const double *prior_lo_host, const double *prior_hi_host,
                              mbh_sampler **out);
mbh_status mbh_sampler_destroy(mbh_sampler *s);
/* Walkers x_host [n_temps * walkers_per_temp][11] (rung-major, host,
 * copied) and their lnL: lnL_host [n_temps * walkers_per_temp] if given
 * (their <d|h>, <h|h> set to 0; `like` may then be NULL), else evaluated
 * under `like` on `stream`. */
mbh_status mbh_sampler_set_walkers(mbh_sampler *s, const double *x_host, const double *lnL_host,
                                   const mbh_likelihood *like, hipStream_t stream);
/* n_iter iterations on `stream` (asynchronous).  With the heterodyned
 * likelihood a half step is three launches: the proposals fused with the
 * walker setup of the sampler's batch, the batch's main pass, its per-walker
 * totals fused with the decisions; the results equal those of the separate
 * calls below bit for bit. */
mbh_status mbh_sampler_step(mbh_sampler *s, const mbh_likelihood *like, int64_t n_iter, hipStream_t stream);
/* n_iter iterations with the heterodyned likelihood of a request server's
 * resident reference ref_index (Sec. 3's search as one of the server's
 * clients): the proposal kernel writes each half step's proposals into the
 * sampler's pinned host staging, they are submitted as one request of
 * n_temps * walkers_per_temp / 2 walkers, and when it completes the decision
 * kernel reads its lnL and <d|h>, <h|h> from the staging (no runtime copies).
 * Synchronous (the stream is synchronised at every half step; the staging is
 * allocated on first use).  The states equal those of mbh_sampler_step under
 * the same reference with the server's precision and mixed_rungs 0, bit for
 * bit.  latency_s [2 n_iter] or NULL: each request's latency (completion
 * minus submission).  Several samplers may be driven this way from separate
 * threads, each on its own stream.
 * Errors: MBH_EINVAL, MBH_EDEVICE and those of mbh_server_submit and
 * mbh_server_wait. */
mbh_status mbh_sampler_step_served(mbh_sampler *s, mbh_server *srv, int ref_index, int64_t n_iter,
                                   hipStream_t stream, double *latency_s);
/* The parts of one iteration, for callers that evaluate the likelihood
 * themselves: mbh_sampler_propose writes the proposals of half 0 or 1 of
 * every rung (mbh_sampler_proposals copies them out: x and theta
 * [n_temps * walkers_per_temp / 2][11], theta[0] NaN outside the prior box,
 * and the move kind 0 stretch, 1 all sky modes, 2 longitudinal,
 * 3 latitudinal); mbh_sampler_accept takes their lnL (device,
 * [n_temps * walkers_per_temp / 2], rung-major; -inf outside the prior) and
 * optionally their <d|h>, <h|h> ([..][2] or NULL); mbh_sampler_swap makes the
 * exchanges and ends the iteration.  propose(0), accept(0), propose(1),
 * accept(1), swap is one iteration. */
mbh_status mbh_sampler_propose(mbh_sampler *s, int half, hipStream_t stream);
mbh_status mbh_sampler_proposals(mbh_sampler *s, double *x_host, double *theta_host, int32_t *kind_host);
mbh_status mbh_sampler_accept(mbh_sampler *s, int half, const double *lnL_prop_dev,
                              const double *dh_hh_prop_dev, hipStream_t stream);
mbh_status mbh_sampler_swap(mbh_sampler *s, hipStream_t stream);
/* Current walkers (x [n][11], lnL [n], <d|h> <h|h> [n][2]; any may be NULL)
 * and the iterations done.  Synchronous. */
mbh_status mbh_sampler_get(mbh_sampler *s, double *x_host, double *lnL_host, double *dh_hh_host,
                           int64_t *iteration);
/* Accepted and proposed moves per rung and move kind ([n_temps][4]) and
 * accepted exchanges per pair of rungs ([n_temps - 1]); any may be NULL. */
mbh_status mbh_sampler_stats(mbh_sampler *s, uint64_t *accepted, uint64_t *proposed, uint64_t *swaps);
/* Stopping rules of Sec. 3 (checked every check_every iterations on the
 * best walker of the first rung): snr_stop > 0 stops when its extracted SNR
 * <d|h> / sqrt(<h|h>) reaches snr_stop (the first search); lnl_checks > 0
 * stops when the maximum lnL has moved by less than lnl_tol over lnl_checks
 * consecutive checks (the heterodyned search: 1 and 30).  refresh_every > 0
 * moves the reference to the best walker of the population every
 * refresh_every iterations (mbh_ref_refresh, on the device) and re-evaluates
 * every walker against it (heterodyned likelihood only; refresh_data is the
 * data the reference was built on). */
enum { MBH_STOP_MAX_ITER = 0, MBH_STOP_SNR = 1, MBH_STOP_CONVERGED = 2 };
typedef struct {
  int32_t check_every;
  double snr_stop;
  double lnl_tol;
  int32_t lnl_checks;
  int32_t refresh_every;
  const mbh_data *refresh_data;
  int64_t max_iter;
} mbh_sampler_stop;
typedef struct {
  int64_t iterations;  /* done in this call                       */
  int32_t reason;      /* MBH_STOP_*                              */
  int32_t checks, refreshes;
  double max_lnL;      /* best lnL of the first rung at the last check */
  double best_snr;     /* its extracted SNR                       */
  double seconds;      /* wall time of the call                   */
} mbh_sampler_report;
/* Iterate until a stopping rule holds or max_iter iterations are done.
 * Synchronises `stream` at every check.  Errors: MBH_EINVAL, MBH_EDEVICE and
 * those of the likelihood calls. */
mbh_status mbh_sampler_run(mbh_sampler *s, const mbh_likelihood *like, const mbh_sampler_stop *stop,
                           hipStream_t stream, mbh_sampler_report *report);

#ifdef __cplusplus
}
#endif
#endif /* MBH_H */
