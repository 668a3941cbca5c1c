// mbh_internal.hpp -- handle layouts shared by the translation units of libmbh.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mbh.h"
#include "mbh_kernels.hpp"

struct mbh_ctx {
  int device = 0;
  size_t budget = 0;
  std::atomic<size_t> in_use{0};
  int n_cu = 256;
  // LDS one workgroup may take: a per-mode item's cross pass runs one
  // workgroup per walker when the walker's deltas fit (else the chunked pass);
  // MBH_PM_CROSS_LDS_MAX (bytes) lowers it, 0 forcing the chunked pass
  size_t lds_max = 65536;
  std::string arch;
  mutable std::mutex mu;
  // lanes per walker of the heterodyned kernel, keyed by (n_bins, n_modes, precision)
  std::map<std::tuple<int, int, int>, int> lanes;
  // mixed path: estimated lnL error above which work is recomputed in FP64
  // (set from kMixedRouteTol at creation)
  double mixed_tol = 0.0;
  // full-grid tile: (frequencies per thread, most walkers per workgroup),
  // keyed by mode class (1: higher modes); absent = (1, 32)
  std::map<int, std::pair<int, int>> full_shape;
  // ingest: batched real-to-complex transform plans keyed by series length,
  // made on first use (their work areas come with each call) and destroyed
  // with the context through fft_plan_destroy
  std::map<int64_t, void *> fft_plans;
  void (*fft_plan_destroy)(void *) = nullptr;
  // the caller's reference plus one per live object created from the context
  std::atomic<int> refs{1};
};

void ctx_retain(mbh_ctx *ctx);
void ctx_release(mbh_ctx *ctx);

// Member of every object created from a context: keeps the context alive
// until the object is deleted, so objects and context may be released in any
// order.
struct CtxHold {
  mbh_ctx *c = nullptr;
  CtxHold() = default;
  CtxHold(const CtxHold &) = delete;
  CtxHold &operator=(const CtxHold &) = delete;
  void set(mbh_ctx *x) {
    ctx_retain(x);
    c = x;
  }
  ~CtxHold() {
    if (c) ctx_release(c);
  }
};

struct mbh_data {
  mbh_ctx *ctx = nullptr;
  CtxHold hold;
  int n_chan = 0;
  int64_t n_f = 0;
  double f0 = 0, df = 0, t_obs = 0;
  double2 *dw64 = nullptr;  // whitened data d sqrt(4 df / S)         [C][N]
  double *sw64 = nullptr;   // sqrt(4 df / S) / amplitude scale        [C][N]
  double *dd_dev = nullptr;
  double dd_host = 0;
  bool dd_ready = false;
  hipEvent_t ready = nullptr;
  size_t bytes = 0;
  std::mutex mu;
};

struct mbh_ref {
  mbh_ctx *ctx = nullptr;
  CtxHold hold;
  int model = 0;
  uint32_t modes = 0;
  int n_chan = 0, n_bins = 0;
  int64_t k_lo = 0, k_hi = 0;
  double t_obs = 0, lnL0 = 0, dd = 0, dh0 = 0, hh0 = 0;
  // <h0|h0> at build time (never changed afterwards: read without a lock by
  // the server's tile ordering)
  double hh0_build = 0;
  // device: edges [E], response factors [E][kFq], carrier phase of h0 [E],
  // 1/s0 [C][E][2], residual-form coefficients [C][Nb][6], scalars
  double *F = nullptr, *fq = nullptr, *psi0 = nullptr, *is064 = nullptr, *coef = nullptr;
  mbh::RefMeta *meta = nullptr;
  // host copies for mbh_ref_get_info / mbh_ref_export (refreshed from the
  // device after a refresh on the device)
  std::vector<double> edges, A0, A1, B0, B1, h0_edges;
  std::vector<int64_t> kb;
  // the data grid the reference was built on
  int64_t n_f = 0;
  double f0 = 0, df = 0;
  // refresh on the device (allocated at the first refresh): staging copies
  // of the arrays above, and the export arrays (kb [E], paper-form
  // coefficients [C][Nb][6], h0 at the edges [C][E][2]) live and staged
  struct Refresh {
    double *F = nullptr, *fq = nullptr, *psi0 = nullptr, *is064 = nullptr, *coef = nullptr;
    mbh::RefMeta *meta = nullptr;
    int64_t *kb = nullptr, *kb_live = nullptr;
    double *paper = nullptr, *paper_live = nullptr, *h0e = nullptr, *h0e_live = nullptr;
    // work buffers of the rebuild (kept, so that a refresh allocates nothing)
    mbh::WalkerC *wc = nullptr;
    unsigned long long *band = nullptr;
    double2 *h0w = nullptr, *s0 = nullptr;
    double *part1 = nullptr, *sums1 = nullptr, *part2 = nullptr, *sums2 = nullptr;
    int nb1 = 0, n_sub = 0;
    int64_t max_len = 0;
    hipEvent_t done = nullptr;  // recorded after the last refresh's commit
    int64_t issued = 0, mirrored = 0;
  } rf;
  bool rf_ready = false;
  std::mutex mu;
  // edges held by F, fq, psi0 and is064: n_bins + 1, or T1 for a per-mode
  // reference
  int32_t n_edges = 0;
  // per-mode relative binning (mbh_build_reference_coeffs_pm): every mode
  // with its own band, bins and ratio; F, fq, psi0, is064 hold the edges of
  // all modes one mode after the other (T1), coef their bins (n_bins in all)
  bool pm = false;
  struct PmMode {
    int mode;
    int64_t k_lo, k_hi;
    int32_t e_off, b_off;  // first edge and first bin of the mode in the concatenated arrays
    std::vector<double> edges, Ares0, Ares1, B0, B1, h0_edges;
    std::vector<int64_t> kb;
  };
  struct PmPair {
    int mode_a, mode_b;
    std::vector<double> edges, C0, C1;
    std::vector<int64_t> kb;
    std::vector<int32_t> bin_a, bin_b;
  };
  std::vector<PmMode> pm_modes;
  std::vector<PmPair> pm_pairs;
  int32_t pm_T1 = 0, pm_T2 = 0;
  int32_t *pm_mode_of = nullptr, *pm_bin_of = nullptr;
  mbh::PmCross *pm_cross = nullptr;
  double *pm_ccoef = nullptr;
};

mbh_status mbh_fail(mbh_status s, const char *fmt, ...);
mbh_status ctx_alloc(mbh_ctx *ctx, void **p, size_t bytes);
void ctx_free(mbh_ctx *ctx, void *p, size_t bytes);
mbh_status ctx_alloc_async(mbh_ctx *ctx, void **p, size_t bytes, hipStream_t st);
void ctx_free_async(mbh_ctx *ctx, void *p, size_t bytes, hipStream_t st);
// The device copy of a batch's items (for kernels that run a batch's setup
// or totals fused with their own work).
const mbh::WorkItem *batch_device_items(const mbh_batch *b);
