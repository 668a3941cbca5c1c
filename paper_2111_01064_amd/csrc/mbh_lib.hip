// mbh_lib.hip -- host runtime and C ABI of libmbh (see include/mbh.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mbh.h"
#include "mbh_internal.hpp"
#include "mbh_kernels.hpp"
#include "mbh_work.hpp"

using namespace mbh;

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

mbh_status mbh_fail(mbh_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

extern "C" const char *mbh_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *mbh_strerror(mbh_status s) {
  switch (s) {
    case MBH_OK: return "ok";
    case MBH_EINVAL: return "invalid argument";
    case MBH_ENOMEM: return "out of device memory or over the HBM budget";
    case MBH_EBAND: return "reference template empty or zero at a bin edge";
    case MBH_EDEVICE: return "HIP runtime error";
    case MBH_EAGAIN: return "not ready";
    case MBH_ENOTFOUND: return "unknown request";
  }
  return "unknown status";
}

// ---------------------------------------------------------------- memory
mbh_status ctx_alloc(mbh_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return MBH_OK;
  size_t cur = ctx->in_use.fetch_add(bytes);
  if (ctx->budget && cur + bytes > ctx->budget) {
    ctx->in_use.fetch_sub(bytes);
    return mbh_fail(MBH_ENOMEM, "HBM budget exceeded: %zu + %zu > %zu bytes", cur, bytes, ctx->budget);
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    ctx->in_use.fetch_sub(bytes);
    *p = nullptr;
    return mbh_fail(MBH_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  return MBH_OK;
}

void ctx_free(mbh_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->in_use.fetch_sub(bytes);
}

mbh_status ctx_alloc_async(mbh_ctx *ctx, void **p, size_t bytes, hipStream_t st) {
  *p = nullptr;
  if (bytes == 0) return MBH_OK;
  size_t cur = ctx->in_use.fetch_add(bytes);
  if (ctx->budget && cur + bytes > ctx->budget) {
    ctx->in_use.fetch_sub(bytes);
    return mbh_fail(MBH_ENOMEM, "HBM budget exceeded: %zu + %zu > %zu bytes", cur, bytes, ctx->budget);
  }
  hipError_t e = hipMallocAsync(p, bytes, st);
  if (e != hipSuccess) {
    ctx->in_use.fetch_sub(bytes);
    *p = nullptr;
    return mbh_fail(MBH_ENOMEM, "hipMallocAsync(%zu): %s", bytes, hipGetErrorString(e));
  }
  return MBH_OK;
}

void ctx_free_async(mbh_ctx *ctx, void *p, size_t bytes, hipStream_t st) {
  if (!p) return;
  (void)hipFreeAsync(p, st);
  ctx->in_use.fetch_sub(bytes);
}

// RAII scratch for one call
struct Scratch {
  mbh_ctx *ctx;
  hipStream_t st;
  std::vector<std::pair<void *, size_t>> bufs;
  explicit Scratch(mbh_ctx *c, hipStream_t s) : ctx(c), st(s) {}
  ~Scratch() {
    for (auto &b : bufs) ctx_free_async(ctx, b.first, b.second, st);
  }
  template <typename T>
  mbh_status get(T **p, size_t n) {
    void *v = nullptr;
    mbh_status s = ctx_alloc_async(ctx, &v, n * sizeof(T), st);
    if (s != MBH_OK) return s;
    bufs.emplace_back(v, n * sizeof(T));
    *p = (T *)v;
    return MBH_OK;
  }
};

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return mbh_fail(MBH_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

#define MBH_TRY(x)                  \
  do {                              \
    mbh_status s_ = (x);            \
    if (s_ != MBH_OK) return s_;    \
  } while (0)

// ---------------------------------------------------------------- no-allocation scratch
// Scratch of mbh_loglike_heterodyned_noalloc (walker constants and partial
// sums) in a file-scope device array: every GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device memory: the device address is resolved once per
// device (hipGetSymbolAddress, with that device current) by mbh_create and
// kept in g_scratch_dev, which is what host code passes to kernels.
static __device__ __align__(256) unsigned char scratch[MBH_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

// with `device` current
static mbh_status noalloc_scratch_init(int device) {
  if (device >= kMaxDevices) return MBH_OK;  // the no-allocation entry point refuses such devices
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_dev[device]) return MBH_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return mbh_fail(MBH_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_scratch_dev[device] = p;
  return MBH_OK;
}

static void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_dev[device];
}

// ---------------------------------------------------------------- context
extern "C" mbh_status mbh_create(int device, size_t hbm_budget_bytes, mbh_ctx **out) {
  if (!out) return mbh_fail(MBH_EINVAL, "null out");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return mbh_fail(MBH_EINVAL, "device %d of %d", device, n);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  MBH_TRY(noalloc_scratch_init(device));
  mbh_ctx *c = new mbh_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  c->n_cu = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  c->lds_max = prop.sharedMemPerBlock;
  if (const char *e = std::getenv("MBH_PM_CROSS_LDS_MAX")) c->lds_max = std::min(c->lds_max, (size_t)std::strtoull(e, nullptr, 10));
  c->mixed_tol = kMixedRouteTol;
  *out = c;
  return MBH_OK;
}

void ctx_retain(mbh_ctx *ctx) { ctx->refs.fetch_add(1); }

void ctx_release(mbh_ctx *ctx) {
  if (ctx->refs.fetch_sub(1) != 1) return;
  if (ctx->fft_plan_destroy && !ctx->fft_plans.empty()) {
    (void)hipSetDevice(ctx->device);
    for (auto &p : ctx->fft_plans) ctx->fft_plan_destroy(p.second);
  }
  delete ctx;
}

extern "C" mbh_status mbh_destroy(mbh_ctx *ctx) {
  if (!ctx) return MBH_OK;
  ctx_release(ctx);
  return MBH_OK;
}

extern "C" mbh_status mbh_memory_in_use(const mbh_ctx *ctx, size_t *bytes_out) {
  if (!ctx || !bytes_out) return mbh_fail(MBH_EINVAL, "null argument");
  *bytes_out = ctx->in_use.load();
  return MBH_OK;
}

// The kernels that generate templates are compiled twice: for the (2,2)
// mode alone (the chirp model included) and for any mode mask.
static bool modes_hm(int model, uint32_t modes) { return model != MBH_MODEL_TF2 && modes != MBH_MODE_22; }

// workgroups of `block` threads of kernel k resident on the whole device at once
static int resident_blocks(const mbh_ctx *ctx, const void *k, int block) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu * ctx->n_cu;
}

// the reference grid pass for this mode set and its grid: one round of
// resident workgroups (more workgroups run in several rounds and were
// measured slower)
static const void *ref_grid_kernel(bool hm) {
  return hm ? reinterpret_cast<const void *>(&k_ref_grid<true>) : reinterpret_cast<const void *>(&k_ref_grid<false>);
}

// ---------------------------------------------------------------- data
static int grid_blocks(int64_t n, int cap) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

extern "C" mbh_status mbh_data_create(mbh_ctx *ctx, int n_chan, int64_t n_freq, double f0, double df,
                                      double t_obs, const double *d_reim_dev, const double *psd_dev,
                                      hipStream_t st, mbh_data **out) {
  if (!ctx || !out || !d_reim_dev || !psd_dev) return mbh_fail(MBH_EINVAL, "null argument");
  *out = nullptr;
  if (n_chan != 1 && n_chan != 3) return mbh_fail(MBH_EINVAL, "n_chan must be 1 or 3 (got %d)", n_chan);
  if (n_freq < 2) return mbh_fail(MBH_EINVAL, "n_freq must be >= 2");
  if (!(df > 0.0) || !(f0 > 0.0) || !std::isfinite(f0) || !std::isfinite(df))
    return mbh_fail(MBH_EINVAL, "grid needs f0 > 0 and df > 0");
  if (!(t_obs > 0.0)) return mbh_fail(MBH_EINVAL, "t_obs must be > 0");
  HIP_TRY(hipSetDevice(ctx->device));
  mbh_data *d = new mbh_data();
  d->ctx = ctx;
  d->hold.set(ctx);
  d->n_chan = n_chan;
  d->n_f = n_freq;
  d->f0 = f0;
  d->df = df;
  d->t_obs = t_obs;
  const int64_t n = (int64_t)n_chan * n_freq;
  auto fail_free = [&](mbh_status s) {
    mbh_data_release(d);
    return s;
  };
  mbh_status s;
  if ((s = ctx_alloc(ctx, (void **)&d->dw64, n * sizeof(double2))) != MBH_OK) return fail_free(s);
  d->bytes += n * sizeof(double2);
  if ((s = ctx_alloc(ctx, (void **)&d->sw64, n * sizeof(double))) != MBH_OK) return fail_free(s);
  d->bytes += n * sizeof(double);
  if ((s = ctx_alloc(ctx, (void **)&d->dd_dev, sizeof(double))) != MBH_OK) return fail_free(s);
  d->bytes += sizeof(double);
  const int nb = grid_blocks(n, 2048);
  double *part = nullptr;
  if ((s = ctx_alloc_async(ctx, (void **)&part, nb * sizeof(double), st)) != MBH_OK) return fail_free(s);
  hipLaunchKernelGGL(k_whiten, dim3(nb), dim3(kBlock), 0, st, d_reim_dev, psd_dev, n, df, d->dw64, d->sw64, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, part, nb, 1, 1, d->dd_dev);
  ctx_free_async(ctx, part, nb * sizeof(double), st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_free(mbh_fail(MBH_EDEVICE, "whitening launch: %s", hipGetErrorString(e)));
  if (hipEventCreateWithFlags(&d->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(d->ready, st) != hipSuccess)
    return fail_free(mbh_fail(MBH_EDEVICE, "event"));
  *out = d;
  return MBH_OK;
}

extern "C" mbh_status mbh_data_release(mbh_data *d) {
  if (!d) return MBH_OK;
  (void)hipSetDevice(d->ctx->device);
  (void)hipDeviceSynchronize();
  ctx_free(d->ctx, d->dw64, d->n_chan * d->n_f * sizeof(double2));
  ctx_free(d->ctx, d->sw64, d->n_chan * d->n_f * sizeof(double));
  ctx_free(d->ctx, d->dd_dev, sizeof(double));
  if (d->ready) (void)hipEventDestroy(d->ready);
  delete d;
  (void)hipGetLastError();  // teardown errors are not left for the next call to find
  return MBH_OK;
}

static mbh_status data_dd(mbh_data *d, double *out) {
  std::lock_guard<std::mutex> g(d->mu);
  if (!d->dd_ready) {
    HIP_TRY(hipSetDevice(d->ctx->device));
    HIP_TRY(hipEventSynchronize(d->ready));
    HIP_TRY(hipMemcpy(&d->dd_host, d->dd_dev, sizeof(double), hipMemcpyDeviceToHost));
    d->dd_ready = true;
  }
  *out = d->dd_host;
  return MBH_OK;
}

extern "C" mbh_status mbh_data_inner_dd(mbh_data *d, double *dd_out) {
  if (!d || !dd_out) return mbh_fail(MBH_EINVAL, "null argument");
  return data_dd(d, dd_out);
}

static mbh_status check_model(const mbh_data *d, int model, uint32_t modes) {
  if (model == MBH_MODEL_IMR) {
    if (d->n_chan != 3) return mbh_fail(MBH_EINVAL, "IMR model needs 3 channels");
    if (modes == 0 || (modes & ~MBH_MODES_ALL)) return mbh_fail(MBH_EINVAL, "bad mode mask 0x%x", modes);
    double fmax = d->f0 + (double)(d->n_f - 1) * d->df;
    if (fmax > kMaxFreq * (1.0 + 1e-12))
      return mbh_fail(MBH_EINVAL, "grid reaches %.4g Hz; the response series covers f <= %.3g Hz", fmax, kMaxFreq);
  } else if (model == MBH_MODEL_TF2) {
    if (d->n_chan != 1) return mbh_fail(MBH_EINVAL, "chirp model needs 1 channel");
  } else {
    return mbh_fail(MBH_EINVAL, "unknown model %d", model);
  }
  return MBH_OK;
}

// walker constants of one host parameter vector, on the device
static mbh_status setup_one(Scratch &sc, const double *theta_host, int model, uint32_t modes, WalkerC **wc_out,
                            bool *valid) {
  double *th = nullptr;
  MBH_TRY(sc.get(&th, 11));
  WalkerC *wc = nullptr;
  MBH_TRY(sc.get(&wc, 1));
  HIP_TRY(hipMemcpyAsync(th, theta_host, 11 * sizeof(double), hipMemcpyHostToDevice, sc.st));
  hipLaunchKernelGGL(k_walker_setup, dim3(1), dim3(128), 0, sc.st, th, (int64_t)1, model, modes, wc);
  int32_t v = 0;
  HIP_TRY(hipMemcpyAsync(&v, &wc->valid, sizeof(int32_t), hipMemcpyDeviceToHost, sc.st));
  HIP_TRY(hipStreamSynchronize(sc.st));
  *valid = v != 0;
  *wc_out = wc;
  return MBH_OK;
}

extern "C" mbh_status mbh_template_full(mbh_ctx *ctx, const mbh_data *data, int model, uint32_t modes,
                                        const double *theta_host, double *h_dev, hipStream_t st) {
  if (!ctx || !data || !theta_host || !h_dev) return mbh_fail(MBH_EINVAL, "null argument");
  MBH_TRY(check_model(data, model, modes));
  HIP_TRY(hipSetDevice(ctx->device));
  Scratch sc(ctx, st);
  WalkerC *wc = nullptr;
  bool valid = false;
  MBH_TRY(setup_one(sc, theta_host, model, modes, &wc, &valid));
  if (!valid) return mbh_fail(MBH_EINVAL, "theta outside the model domain");
  hipLaunchKernelGGL(k_template_grid, dim3((unsigned)((data->n_f + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     wc, modes, data->n_chan, data->n_f, data->f0, data->df, data->t_obs, (double2 *)h_dev);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

// ---------------------------------------------------------------- reference
static void release_ref_dev(mbh_ref *r) {
  mbh_ctx *c = r->ctx;
  const int E = r->n_edges;
  ctx_free(c, r->pm_mode_of, (size_t)r->pm_T1 * sizeof(int32_t));
  ctx_free(c, r->pm_bin_of, (size_t)r->pm_T1 * sizeof(int32_t));
  ctx_free(c, r->pm_cross, (size_t)r->pm_T2 * sizeof(PmCross));
  ctx_free(c, r->pm_ccoef, (size_t)r->n_chan * r->pm_T2 * 4 * sizeof(double));
  r->pm_mode_of = r->pm_bin_of = nullptr;
  r->pm_cross = nullptr;
  r->pm_ccoef = nullptr;
  ctx_free(c, r->F, E * sizeof(double));
  ctx_free(c, r->psi0, E * sizeof(double));
  ctx_free(c, r->fq, (size_t)E * kFq * sizeof(double));
  ctx_free(c, r->is064, (size_t)r->n_chan * E * 2 * sizeof(double));
  const size_t nce = (size_t)r->n_chan * E, ncb = (size_t)r->n_chan * r->n_bins;
  ctx_free(c, r->coef, ncb * 6 * sizeof(double));
  ctx_free(c, r->meta, sizeof(RefMeta));
  r->F = r->psi0 = r->fq = r->is064 = r->coef = nullptr;
  r->meta = nullptr;
  if (r->rf_ready) {
    auto &f = r->rf;
    ctx_free(c, f.F, E * sizeof(double));
    ctx_free(c, f.psi0, E * sizeof(double));
    ctx_free(c, f.fq, (size_t)E * kFq * sizeof(double));
    ctx_free(c, f.is064, nce * 2 * sizeof(double));
    ctx_free(c, f.coef, ncb * 6 * sizeof(double));
    ctx_free(c, f.meta, sizeof(RefMeta));
    ctx_free(c, f.kb, E * sizeof(int64_t));
    ctx_free(c, f.kb_live, E * sizeof(int64_t));
    ctx_free(c, f.paper, ncb * 6 * sizeof(double));
    ctx_free(c, f.paper_live, ncb * 6 * sizeof(double));
    ctx_free(c, f.h0e, nce * 2 * sizeof(double));
    ctx_free(c, f.h0e_live, nce * 2 * sizeof(double));
    ctx_free(c, f.wc, sizeof(WalkerC));
    ctx_free(c, f.band, 2 * sizeof(unsigned long long));
    ctx_free(c, f.h0w, (size_t)r->n_f * r->n_chan * sizeof(double2));
    ctx_free(c, f.s0, nce * sizeof(double2));
    ctx_free(c, f.part1, (size_t)f.nb1 * 3 * sizeof(double));
    ctx_free(c, f.sums1, 3 * sizeof(double));
    ctx_free(c, f.part2, (size_t)r->n_bins * f.n_sub * 18 * sizeof(double));
    ctx_free(c, f.sums2, (size_t)r->n_bins * 18 * sizeof(double));
    if (f.done) (void)hipEventDestroy(f.done);
    f = mbh_ref::Refresh{};
    r->rf_ready = false;
  }
}

extern "C" mbh_status mbh_ref_release(mbh_ref *r) {
  if (!r) return MBH_OK;
  (void)hipSetDevice(r->ctx->device);
  (void)hipDeviceSynchronize();
  release_ref_dev(r);
  delete r;
  (void)hipGetLastError();  // teardown errors are not left for the next call to find
  return MBH_OK;
}

// grid frequency on the host with the same two roundings as the device
#pragma clang fp contract(off)
static double host_grid_freq(double f0, double df, int64_t k) {
  volatile double t = (double)k * df;
  return f0 + t;
}
static void host_edges(double F0, double FN, int n_bins, std::vector<double> &edges) {
  edges.assign(n_bins + 1, 0.0);
  edges[0] = F0;
  edges[n_bins] = FN;
  for (int j = 1; j < n_bins; ++j) edges[j] = std::exp(std::log(F0) + j * (std::log(FN) - std::log(F0)) / n_bins);
}
#pragma clang fp contract(on)

// Byte offsets of several device arrays inside one scratch allocation
// (each aligned to 256 bytes), so that a call makes one allocation.
struct Carve {
  size_t bytes = 0;
  template <typename T>
  size_t add(size_t n) {
    bytes = (bytes + 255) & ~(size_t)255;
    const size_t o = bytes;
    bytes += std::max<size_t>(1, n) * sizeof(T);
    return o;
  }
};

// the walker's domain check as the gate of the grid pass: an invalid theta0
// leaves the pass idle and is reported with the band
static __global__ void k_valid_gate(const WalkerC *wc, RefMeta *gate) {
  RefMeta m{};
  m.status = wc[0].valid ? 0 : MBH_EINVAL;
  m.pick = -1;
  *gate = m;
}

// Host build: two synchronisations of `st`, one after the grid pass (the
// band sets the edges, computed on the host in FP64 as the oracle does) and
// one after the bin sums and coefficients (computed on the device by the
// same kernel as a reference update), which also brings back the host
// mirrors used by mbh_ref_export.
extern "C" mbh_status mbh_build_reference_coeffs(mbh_ctx *ctx, const mbh_data *data_c, int model,
                                                 uint32_t modes, const double *theta0_host, int n_bins,
                                                 hipStream_t st, mbh_ref **out) {
  mbh_data *data = const_cast<mbh_data *>(data_c);
  if (!ctx || !data || !theta0_host || !out) return mbh_fail(MBH_EINVAL, "null argument");
  *out = nullptr;
  if (n_bins < 1 || n_bins > 4096) return mbh_fail(MBH_EINVAL, "n_bins %d outside [1, 4096]", n_bins);
  MBH_TRY(check_model(data, model, modes));
  HIP_TRY(hipSetDevice(ctx->device));
  const int C = data->n_chan, E = n_bins + 1;
  const int64_t N = data->n_f;
  const uint32_t m_modes = model == MBH_MODEL_IMR ? modes : 0u;
  const bool hm = modes_hm(model, m_modes);
  const int nb1 = grid_blocks(N, resident_blocks(ctx, ref_grid_kernel(hm), kBlock));
  Scratch sc(ctx, st);

  // pass 1: walker constants, h0 on the grid, band, lnL(h0) pieces
  Carve c1;
  const size_t o_th = c1.add<double>(11), o_wc = c1.add<WalkerC>(1), o_gate = c1.add<RefMeta>(1),
               o_band = c1.add<unsigned long long>(2), o_sums1 = c1.add<double>(3),
               o_part1 = c1.add<double>((size_t)nb1 * 3), o_h0w = c1.add<double2>((size_t)C * N);
  char *b1 = nullptr;
  MBH_TRY(sc.get(&b1, c1.bytes));
  double *th = (double *)(b1 + o_th), *sums1 = (double *)(b1 + o_sums1), *part1 = (double *)(b1 + o_part1);
  WalkerC *wc = (WalkerC *)(b1 + o_wc);
  RefMeta *gate = (RefMeta *)(b1 + o_gate);
  unsigned long long *band = (unsigned long long *)(b1 + o_band);
  double2 *h0w = (double2 *)(b1 + o_h0w);
  HIP_TRY(hipMemcpyAsync(th, theta0_host, 11 * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_walker_setup, dim3(1), dim3(128), 0, st, th, (int64_t)1, model, m_modes, wc);
  hipLaunchKernelGGL(k_valid_gate, dim3(1), dim3(1), 0, st, wc, gate);
  hipLaunchKernelGGL(k_init_band, dim3(1), dim3(1), 0, st, band);
  if (hm)
    hipLaunchKernelGGL(k_ref_grid<true>, dim3(nb1), dim3(kBlock), 0, st, wc, m_modes, C, N, data->f0, data->df,
                       data->t_obs, data->dw64, data->sw64, h0w, band, part1, gate);
  else
    hipLaunchKernelGGL(k_ref_grid<false>, dim3(nb1), dim3(kBlock), 0, st, wc, m_modes, C, N, data->f0, data->df,
                       data->t_obs, data->dw64, data->sw64, h0w, band, part1, gate);
  hipLaunchKernelGGL(k_sum_partials, dim3(3), dim3(64), 0, st, part1, nb1, 3, 3, sums1);
  HIP_TRY(hipGetLastError());
  unsigned long long hb[2];
  RefMeta g{};
  HIP_TRY(hipMemcpyAsync(&g, gate, sizeof(g), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hb, band, sizeof(hb), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (g.status != 0) return mbh_fail(MBH_EINVAL, "theta0 outside the model domain");
  if (hb[0] == ~0ull || hb[1] <= hb[0]) return mbh_fail(MBH_EBAND, "reference template is empty on the grid");
  const int64_t k_lo = (int64_t)hb[0], k_hi = (int64_t)hb[1];

  // band, log-spaced edges and the first grid index of each bin (host, FP64)
  std::vector<double> edges;
  host_edges(host_grid_freq(data->f0, data->df, k_lo), host_grid_freq(data->f0, data->df, k_hi), n_bins, edges);
  std::vector<int64_t> kb(E);
  kb[0] = k_lo;
  kb[n_bins] = k_hi + 1;
  for (int b = 1; b < n_bins; ++b) {
    int64_t lo = k_lo, hi = k_hi;  // smallest k with f_k >= edges[b]
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (host_grid_freq(data->f0, data->df, mid) >= edges[b]) hi = mid;
      else lo = mid + 1;
    }
    kb[b] = lo;
  }
  int64_t max_len = 0;
  for (int b = 0; b < n_bins; ++b) max_len = std::max(max_len, kb[b + 1] - kb[b]);
  const int n_sub = (int)std::max<int64_t>(1, (max_len + kRefChunk - 1) / kRefChunk);

  mbh_ref *r = new mbh_ref();
  r->ctx = ctx;
  r->hold.set(ctx);
  r->model = model;
  r->modes = m_modes;
  r->n_chan = C;
  r->n_bins = n_bins;
  r->n_edges = E;
  r->k_lo = k_lo;
  r->k_hi = k_hi;
  r->t_obs = data->t_obs;
  r->n_f = N;
  r->f0 = data->f0;
  r->df = data->df;
  r->edges = edges;
  r->kb = kb;
  auto fail_free = [&](mbh_status s) {
    release_ref_dev(r);
    delete r;
    return s;
  };
  mbh_status s;
  if ((s = ctx_alloc(ctx, (void **)&r->F, E * sizeof(double))) != MBH_OK) return fail_free(s);
  if ((s = ctx_alloc(ctx, (void **)&r->psi0, E * sizeof(double))) != MBH_OK) return fail_free(s);
  if ((s = ctx_alloc(ctx, (void **)&r->fq, (size_t)E * kFq * sizeof(double))) != MBH_OK) return fail_free(s);
  if ((s = ctx_alloc(ctx, (void **)&r->is064, (size_t)C * E * 2 * sizeof(double))) != MBH_OK) return fail_free(s);
  if ((s = ctx_alloc(ctx, (void **)&r->coef, (size_t)C * n_bins * 6 * sizeof(double))) != MBH_OK)
    return fail_free(s);
  if ((s = ctx_alloc(ctx, (void **)&r->meta, sizeof(RefMeta))) != MBH_OK) return fail_free(s);

  // pass 2: bin sums, h0 at the edges, coefficients and scalars
  Carve c2;
  const size_t o_kb = c2.add<int64_t>(E), o_part2 = c2.add<double>((size_t)n_bins * n_sub * 18),
               o_sums2 = c2.add<double>((size_t)n_bins * 18), o_s0 = c2.add<double2>((size_t)C * E),
               o_paper = c2.add<double>((size_t)C * n_bins * 6), o_h0e = c2.add<double>((size_t)C * E * 2);
  char *b2 = nullptr;
  if ((s = sc.get(&b2, c2.bytes)) != MBH_OK) return fail_free(s);
  int64_t *kb_dev = (int64_t *)(b2 + o_kb);
  double *part2 = (double *)(b2 + o_part2), *sums2 = (double *)(b2 + o_sums2);
  double *paper = (double *)(b2 + o_paper), *h0e = (double *)(b2 + o_h0e);
  double2 *s0 = (double2 *)(b2 + o_s0);
  RefMeta m{};
  m.k_lo = k_lo;
  m.k_hi = k_hi;
  m.pick = -1;
  if (hipMemcpyAsync(r->F, edges.data(), E * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(kb_dev, kb.data(), E * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(r->meta, &m, sizeof(m), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail_free(mbh_fail(MBH_EDEVICE, "upload edges"));
  hipLaunchKernelGGL(k_ref_bins, dim3(n_bins, n_sub), dim3(kBlock), 0, st, kb_dev, r->F, n_bins, n_sub, C, N,
                     data->f0, data->df, data->dw64, h0w, part2, nullptr);
  // sum the n_sub chunks of each bin in order: part2 is [Nb][n_sub][18]
  hipLaunchKernelGGL(k_sum_bins, dim3((n_bins * 18 + 255) / 256), dim3(256), 0, st, part2, n_bins, n_sub, sums2);
  hipLaunchKernelGGL(k_ref_edges, dim3((E + 63) / 64), dim3(64), 0, st, wc, r->modes, C, E, r->F, data->t_obs,
                     r->fq, r->psi0, s0, nullptr);
  // paper-form and residual-form coefficients, 1/s0, h0 at the edges, lnL(h0)
  // and the sinc term counts; status MBH_EBAND if h0 vanishes at an edge
  hipLaunchKernelGGL(k_refresh_finish, dim3(1), dim3(256), 0, st, sums1, sums2, s0, r->F, r->psi0, C, n_bins, r->coef,
                     r->is064, paper, h0e, r->meta);
  if (hipGetLastError() != hipSuccess) return fail_free(mbh_fail(MBH_EDEVICE, "reference kernels"));
  std::vector<double> hp((size_t)C * n_bins * 6);
  r->h0_edges.assign((size_t)C * E * 2, 0.0);
  if (hipMemcpyAsync(&m, r->meta, sizeof(m), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hp.data(), paper, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(r->h0_edges.data(), h0e, r->h0_edges.size() * sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_free(mbh_fail(MBH_EDEVICE, "download reference"));
  if (m.status != 0) return fail_free(mbh_fail(MBH_EBAND, "reference is zero or not finite at a bin edge"));
  double dd = 0.0;
  if ((s = data_dd(data, &dd)) != MBH_OK) return fail_free(s);
  r->dd = dd;
  r->lnL0 = m.lnL0;
  r->dh0 = m.dh0;
  r->hh0 = m.hh0;
  r->hh0_build = m.hh0;
  r->A0.assign((size_t)C * n_bins * 2, 0.0);
  r->A1.assign((size_t)C * n_bins * 2, 0.0);
  r->B0.assign((size_t)C * n_bins, 0.0);
  r->B1.assign((size_t)C * n_bins, 0.0);
  for (size_t o = 0; o < (size_t)C * n_bins; ++o) {
    r->A0[2 * o] = hp[6 * o + 0];
    r->A0[2 * o + 1] = hp[6 * o + 1];
    r->A1[2 * o] = hp[6 * o + 2];
    r->A1[2 * o + 1] = hp[6 * o + 3];
    r->B0[o] = hp[6 * o + 4];
    r->B1[o] = hp[6 * o + 5];
  }
  *out = r;
  return MBH_OK;
}

// ---------------------------------------------------------------- per-mode reference
// first grid index of each bin: kb[b] = smallest k in [k_lo, k_hi] with
// f_k >= edges[b] (b >= 1), kb[0] = k_lo, kb[n] = k_hi + 1 (FP64 on the host)
static std::vector<int64_t> host_kb(double f0, double df, int64_t k_lo, int64_t k_hi, const std::vector<double> &edges) {
  const int n = (int)edges.size() - 1;
  std::vector<int64_t> kb(n + 1);
  kb[0] = k_lo;
  kb[n] = k_hi + 1;
  for (int b = 1; b < n; ++b) {
    int64_t lo = k_lo, hi = k_hi + 1;
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (host_grid_freq(f0, df, mid) >= edges[b]) hi = mid;
      else lo = mid + 1;
    }
    kb[b] = lo;
  }
  for (int b = n - 1; b >= 1; --b) kb[b] = std::min(kb[b], kb[b + 1]);
  return kb;
}

// the bin [F_b, F_b+1) (the last closed) of a mode's edges that holds f
static int host_bin_of(const std::vector<double> &edges, double f) {
  const int n = (int)edges.size() - 1;
  int b = (int)(std::upper_bound(edges.begin(), edges.end(), f) - edges.begin()) - 1;
  return std::min(std::max(b, 0), n - 1);
}

extern "C" mbh_status mbh_build_reference_coeffs_pm(mbh_ctx *ctx, const mbh_data *data_c, int model, uint32_t modes,
                                                    const double *theta0_host, const int32_t *n_bins_mode,
                                                    hipStream_t st, mbh_ref **out) {
  mbh_data *data = const_cast<mbh_data *>(data_c);
  if (!ctx || !data || !theta0_host || !n_bins_mode || !out) return mbh_fail(MBH_EINVAL, "null argument");
  *out = nullptr;
  if (model != MBH_MODEL_IMR) return mbh_fail(MBH_EINVAL, "per-mode binning needs the IMR model");
  MBH_TRY(check_model(data, model, modes));
  std::vector<int> mode_list;
  for (int mi = 0; mi < kNumModes; ++mi)
    if (modes & (1u << mi)) {
      if (n_bins_mode[mi] < 1 || n_bins_mode[mi] > 4096)
        return mbh_fail(MBH_EINVAL, "mode %d: n_bins %d outside [1, 4096]", mi, n_bins_mode[mi]);
      mode_list.push_back(mi);
    }
  HIP_TRY(hipSetDevice(ctx->device));
  const int C = 3, nm = (int)mode_list.size();
  const int64_t N = data->n_f;
  const double f0 = data->f0, df = data->df;
  Scratch sc(ctx, st);
  WalkerC *wc = nullptr;
  bool valid = false;
  MBH_TRY(setup_one(sc, theta0_host, model, modes, &wc, &valid));
  if (!valid) return mbh_fail(MBH_EINVAL, "theta0 outside the model domain");

  // grid pass: each mode's whitened h0, their sum, bands, lnL(h0) pieces
  double2 *h0w = nullptr, *htot = nullptr;
  MBH_TRY(sc.get(&h0w, (size_t)nm * C * N));
  MBH_TRY(sc.get(&htot, (size_t)C * N));
  unsigned long long *band = nullptr;
  MBH_TRY(sc.get(&band, 2 * kNumModes));
  const int nb1 = grid_blocks(N, resident_blocks(ctx, reinterpret_cast<const void *>(&k_pm_ref_grid), kBlock));
  double *part1 = nullptr, *sums1 = nullptr;
  MBH_TRY(sc.get(&part1, (size_t)nb1 * 3));
  MBH_TRY(sc.get(&sums1, 3));
  unsigned long long band0[2 * kNumModes];
  for (int i = 0; i < kNumModes; ++i) {
    band0[2 * i] = ~0ull;
    band0[2 * i + 1] = 0ull;
  }
  HIP_TRY(hipMemcpyAsync(band, band0, sizeof(band0), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_pm_ref_grid, dim3(nb1), dim3(kBlock), 0, st, wc, modes, N, f0, df, data->t_obs, data->dw64,
                     data->sw64, h0w, htot, band, part1);
  hipLaunchKernelGGL(k_sum_partials, dim3(3), dim3(64), 0, st, part1, nb1, 3, 3, sums1);
  HIP_TRY(hipGetLastError());
  unsigned long long hb[2 * kNumModes];
  double s1[3];
  HIP_TRY(hipMemcpyAsync(hb, band, sizeof(hb), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(s1, sums1, sizeof(s1), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));

  mbh_ref *r = new mbh_ref();
  r->ctx = ctx;
  r->hold.set(ctx);
  r->model = model;
  r->modes = modes;
  r->n_chan = C;
  r->t_obs = data->t_obs;
  r->n_f = N;
  r->f0 = f0;
  r->df = df;
  r->pm = true;
  auto fail_free = [&](mbh_status e) {
    release_ref_dev(r);
    delete r;
    return e;
  };
  // modes with a band on the grid (a mode without one takes no part), their
  // edges and bins, one mode after the other
  std::vector<int> rank_of(kNumModes, -1);
  int32_t T1 = 0, NB = 0;
  for (int rk = 0; rk < nm; ++rk) {
    const int mi = mode_list[rk];
    rank_of[mi] = rk;
    if (hb[2 * rk] == ~0ull || hb[2 * rk + 1] <= hb[2 * rk]) continue;
    mbh_ref::PmMode pmm;
    pmm.mode = mi;
    pmm.k_lo = (int64_t)hb[2 * rk];
    pmm.k_hi = (int64_t)hb[2 * rk + 1];
    host_edges(host_grid_freq(f0, df, pmm.k_lo), host_grid_freq(f0, df, pmm.k_hi), n_bins_mode[mi], pmm.edges);
    pmm.kb = host_kb(f0, df, pmm.k_lo, pmm.k_hi, pmm.edges);
    pmm.e_off = T1;
    pmm.b_off = NB;
    T1 += n_bins_mode[mi] + 1;
    NB += n_bins_mode[mi];
    r->pm_modes.push_back(std::move(pmm));
  }
  if (r->pm_modes.empty()) return fail_free(mbh_fail(MBH_EBAND, "reference template empty on the grid in every mode"));
  r->n_bins = NB;
  r->n_edges = T1;
  r->pm_T1 = T1;
  r->k_lo = INT64_MAX;
  r->k_hi = 0;
  for (auto &m : r->pm_modes) {
    r->k_lo = std::min(r->k_lo, m.k_lo);
    r->k_hi = std::max(r->k_hi, m.k_hi);
  }
  // mode pairs with overlapping bands: merged edges, bins, each mode's bin
  std::vector<PmCross> cross;
  std::vector<int64_t> mkbeg, mkend;
  std::vector<double> mfc;
  std::vector<int32_t> mra, mrb;
  for (size_t a = 0; a < r->pm_modes.size(); ++a)
    for (size_t b = a + 1; b < r->pm_modes.size(); ++b) {
      const auto &A = r->pm_modes[a], &B = r->pm_modes[b];
      const int64_t lo = std::max(A.k_lo, B.k_lo), hi = std::min(A.k_hi, B.k_hi);
      if (hi < lo) continue;
      const double Flo = host_grid_freq(f0, df, lo), Fhi = host_grid_freq(f0, df, hi);
      mbh_ref::PmPair pp;
      pp.mode_a = A.mode;
      pp.mode_b = B.mode;
      for (double e : A.edges)
        if (e >= Flo && e <= Fhi) pp.edges.push_back(e);
      for (double e : B.edges)
        if (e >= Flo && e <= Fhi) pp.edges.push_back(e);
      std::sort(pp.edges.begin(), pp.edges.end());
      pp.edges.erase(std::unique(pp.edges.begin(), pp.edges.end()), pp.edges.end());
      if (pp.edges.size() < 2) pp.edges = {Flo, Fhi};  // an overlap of one grid point
      pp.kb = host_kb(f0, df, lo, hi, pp.edges);
      const int nmb = (int)pp.edges.size() - 1;
      for (int m = 0; m < nmb; ++m) {
        const double fm = 0.5 * (pp.edges[m] + pp.edges[m + 1]);
        const int ba = host_bin_of(A.edges, pp.edges[m]), bb = host_bin_of(B.edges, pp.edges[m]);
        pp.bin_a.push_back(ba);
        pp.bin_b.push_back(bb);
        PmCross x;
        x.ea = A.e_off + ba;
        x.eb = B.e_off + bb;
        x.xa = fm - 0.5 * (A.edges[ba] + A.edges[ba + 1]);
        x.xb = fm - 0.5 * (B.edges[bb] + B.edges[bb + 1]);
        x.ia = 1.0 / (A.edges[ba + 1] - A.edges[ba]);
        x.ib = 1.0 / (B.edges[bb + 1] - B.edges[bb]);
        cross.push_back(x);
        mkbeg.push_back(pp.kb[m]);
        mkend.push_back(pp.kb[m + 1]);
        mfc.push_back(fm);
        mra.push_back(rank_of[A.mode]);
        mrb.push_back(rank_of[B.mode]);
      }
      r->pm_pairs.push_back(std::move(pp));
    }
  const int32_t T2 = (int32_t)cross.size();
  r->pm_T2 = T2;

  // concatenated edge arrays and the edge -> mode / bin maps
  std::vector<double> Fcat(T1);
  std::vector<int32_t> mode_of(T1), bin_of(T1);
  for (auto &m : r->pm_modes) {
    const int n = (int)m.edges.size() - 1;
    for (int j = 0; j <= n; ++j) {
      Fcat[m.e_off + j] = m.edges[j];
      mode_of[m.e_off + j] = m.mode;
      bin_of[m.e_off + j] = j < n ? m.b_off + j : -1;
    }
  }
  mbh_status e;
  if ((e = ctx_alloc(ctx, (void **)&r->F, T1 * sizeof(double))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->psi0, T1 * sizeof(double))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->fq, (size_t)T1 * kFq * sizeof(double))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->is064, (size_t)C * T1 * 2 * sizeof(double))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->coef, (size_t)C * NB * 6 * sizeof(double))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->meta, sizeof(RefMeta))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->pm_mode_of, T1 * sizeof(int32_t))) != MBH_OK) return fail_free(e);
  if ((e = ctx_alloc(ctx, (void **)&r->pm_bin_of, T1 * sizeof(int32_t))) != MBH_OK) return fail_free(e);
  if (T2 > 0) {
    if ((e = ctx_alloc(ctx, (void **)&r->pm_cross, (size_t)T2 * sizeof(PmCross))) != MBH_OK) return fail_free(e);
    if ((e = ctx_alloc(ctx, (void **)&r->pm_ccoef, (size_t)C * T2 * 4 * sizeof(double))) != MBH_OK)
      return fail_free(e);
  }
  // per-mode bin sums (one mode after the other through one part buffer)
  int64_t max_part = 0;
  std::vector<int> n_sub_of;
  for (auto &m : r->pm_modes) {
    int64_t ml = 0;
    for (size_t b = 0; b + 1 < m.kb.size(); ++b) ml = std::max(ml, m.kb[b + 1] - m.kb[b]);
    const int ns = (int)std::max<int64_t>(1, (ml + kRefChunk - 1) / kRefChunk);
    n_sub_of.push_back(ns);
    max_part = std::max<int64_t>(max_part, (int64_t)(m.edges.size() - 1) * ns * 18);
  }
  int64_t *kb_dev = nullptr;
  double *part2 = nullptr, *sums2 = nullptr;
  double2 *s0 = nullptr;
  int32_t *mode_of_dev = r->pm_mode_of;
  if ((e = sc.get(&kb_dev, (size_t)T1)) != MBH_OK) return fail_free(e);
  if ((e = sc.get(&part2, (size_t)max_part)) != MBH_OK) return fail_free(e);
  if ((e = sc.get(&sums2, (size_t)NB * 18)) != MBH_OK) return fail_free(e);
  if ((e = sc.get(&s0, (size_t)C * T1)) != MBH_OK) return fail_free(e);
  std::vector<int64_t> kbcat(T1);
  for (auto &m : r->pm_modes)
    for (size_t j = 0; j < m.kb.size(); ++j) kbcat[m.e_off + j] = m.kb[j];
  if (hipMemcpyAsync(r->F, Fcat.data(), T1 * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(kb_dev, kbcat.data(), T1 * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(mode_of_dev, mode_of.data(), T1 * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(r->pm_bin_of, bin_of.data(), T1 * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail_free(mbh_fail(MBH_EDEVICE, "upload edges"));
  for (size_t i = 0; i < r->pm_modes.size(); ++i) {
    const auto &m = r->pm_modes[i];
    const int n = (int)m.edges.size() - 1, ns = n_sub_of[i];
    hipLaunchKernelGGL(k_pm_mode_bins, dim3(n, ns), dim3(kBlock), 0, st, kb_dev + m.e_off, r->F + m.e_off, ns, N, f0,
                       df, data->dw64, htot, h0w + (int64_t)rank_of[m.mode] * C * N, part2);
    hipLaunchKernelGGL(k_pm_sum, dim3((n * 18 + 255) / 256), dim3(256), 0, st, part2, n, ns, 18,
                       sums2 + (int64_t)m.b_off * 18);
  }
  // merged bins of the mode pairs
  double *csum = nullptr;
  if (T2 > 0) {
    int64_t ml = 0;
    for (int32_t m = 0; m < T2; ++m) ml = std::max(ml, mkend[m] - mkbeg[m]);
    const int ns = (int)std::max<int64_t>(1, (ml + kRefChunk - 1) / kRefChunk);
    int64_t *kbeg_d = nullptr, *kend_d = nullptr;
    double *fm_d = nullptr, *part3 = nullptr;
    int32_t *ra_d = nullptr, *rb_d = nullptr;
    if ((e = sc.get(&kbeg_d, T2)) != MBH_OK || (e = sc.get(&kend_d, T2)) != MBH_OK ||
        (e = sc.get(&fm_d, T2)) != MBH_OK || (e = sc.get(&ra_d, T2)) != MBH_OK || (e = sc.get(&rb_d, T2)) != MBH_OK ||
        (e = sc.get(&part3, (size_t)T2 * ns * 12)) != MBH_OK || (e = sc.get(&csum, (size_t)T2 * 12)) != MBH_OK)
      return fail_free(e);
    if (hipMemcpyAsync(kbeg_d, mkbeg.data(), T2 * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(kend_d, mkend.data(), T2 * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(fm_d, mfc.data(), T2 * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(ra_d, mra.data(), T2 * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(rb_d, mrb.data(), T2 * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(r->pm_cross, cross.data(), T2 * sizeof(PmCross), hipMemcpyHostToDevice, st) != hipSuccess)
      return fail_free(mbh_fail(MBH_EDEVICE, "upload merged bins"));
    hipLaunchKernelGGL(k_pm_pair_bins, dim3(T2, ns), dim3(kBlock), 0, st, kbeg_d, kend_d, fm_d, ra_d, rb_d, ns, N, f0,
                       df, h0w, part3);
    hipLaunchKernelGGL(k_pm_sum, dim3((T2 * 12 + 255) / 256), dim3(256), 0, st, part3, T2, ns, 12, csum);
  }
  double fmax_e = 0.0;
  for (double f : Fcat) fmax_e = std::max(fmax_e, f);
  const int ns64 = sinc_terms_for<double>(fmax_e);
  hipLaunchKernelGGL(k_pm_ref_edges, dim3((T1 + 63) / 64), dim3(64), 0, st, wc, mode_of_dev, T1, r->F, ns64,
                     data->t_obs, r->fq, r->psi0, s0);
  if (hipGetLastError() != hipSuccess) return fail_free(mbh_fail(MBH_EDEVICE, "per-mode reference kernels"));
  std::vector<double> hs2((size_t)NB * 18), hs0((size_t)C * T1 * 2), hcs((size_t)T2 * 12), psi(T1);
  if (hipMemcpyAsync(hs2.data(), sums2, hs2.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hs0.data(), s0, hs0.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      (T2 > 0 &&
       hipMemcpyAsync(hcs.data(), csum, hcs.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) ||
      hipMemcpyAsync(psi.data(), r->psi0, T1 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_free(mbh_fail(MBH_EDEVICE, "download per-mode sums"));
  // each mode's ratio must exist at each of its edges
  for (auto &m : r->pm_modes)
    for (int c = 0; c < C; ++c)
      for (size_t j = 0; j < m.edges.size(); ++j) {
        const size_t i = (size_t)c * T1 + m.e_off + j;
        const double re = hs0[2 * i], im = hs0[2 * i + 1];
        if (!(re != 0.0 || im != 0.0) || !std::isfinite(re) || !std::isfinite(im))
          return fail_free(mbh_fail(MBH_EBAND, "mode %d of the reference is zero at its edge %zu (f = %.6g Hz), channel %d",
                                    m.mode, j, m.edges[j], c));
      }
  double dd = 0.0;
  if ((e = data_dd(data, &dd)) != MBH_OK) return fail_free(e);
  r->dd = dd;
  r->lnL0 = -0.5 * s1[0];
  r->dh0 = s1[1];
  r->hh0 = s1[2];
  r->hh0_build = s1[2];
  // coefficients: residual form for the kernels ([C][NB][6], slopes scaled
  // by 1 / dF_b), sums in df / S units for export (the grid sums carry
  // w = 4 df / S)
  std::vector<double> coef((size_t)C * NB * 6);
  for (auto &m : r->pm_modes) {
    const int n = (int)m.edges.size() - 1;
    m.Ares0.assign((size_t)C * n * 2, 0.0);
    m.Ares1.assign((size_t)C * n * 2, 0.0);
    m.B0.assign((size_t)C * n, 0.0);
    m.B1.assign((size_t)C * n, 0.0);
    m.h0_edges.assign((size_t)C * (n + 1) * 2, 0.0);
    for (int c = 0; c < C; ++c)
      for (int b = 0; b < n; ++b) {
        const double *q = &hs2[(size_t)(m.b_off + b) * 18 + c * 6];
        const size_t o = (size_t)c * n + b;
        m.Ares0[2 * o] = 0.25 * q[0];
        m.Ares0[2 * o + 1] = 0.25 * q[1];
        m.Ares1[2 * o] = 0.25 * q[2];
        m.Ares1[2 * o + 1] = 0.25 * q[3];
        m.B0[o] = 0.25 * q[4];
        m.B1[o] = 0.25 * q[5];
        const double idf = 1.0 / (m.edges[b + 1] - m.edges[b]);
        double *k = &coef[6 * ((size_t)c * NB + m.b_off + b)];
        k[0] = 0.25 * q[0];
        k[1] = 0.25 * q[1];
        k[2] = 0.25 * q[2] * idf;
        k[3] = 0.25 * q[3] * idf;
        k[4] = 0.25 * q[4];
        k[5] = 0.25 * q[5] * idf;
      }
    for (int c = 0; c < C; ++c)
      for (int j = 0; j <= n; ++j) {
        const size_t i = (size_t)c * T1 + m.e_off + j;
        const double re = hs0[2 * i], im = hs0[2 * i + 1];
        const double p = std::remainder(psi[m.e_off + j], 2.0 * M_PI);
        const double cp = std::cos(p), sp = std::sin(p);
        m.h0_edges[2 * ((size_t)c * (n + 1) + j)] = (re * cp + im * sp) / kAmpScale;
        m.h0_edges[2 * ((size_t)c * (n + 1) + j) + 1] = (im * cp - re * sp) / kAmpScale;
      }
  }
  std::vector<double> is64((size_t)C * T1 * 2);
  for (size_t i = 0; i < (size_t)C * T1; ++i) {
    const double re = hs0[2 * i], im = hs0[2 * i + 1], den = re * re + im * im;
    is64[2 * i] = re / den;
    is64[2 * i + 1] = -im / den;
  }
  std::vector<double> ccoef((size_t)C * T2 * 4);
  {
    int32_t mu = 0;
    for (auto &pp : r->pm_pairs) {
      const int n = (int)pp.edges.size() - 1;
      pp.C0.assign((size_t)C * n * 2, 0.0);
      pp.C1.assign((size_t)C * n * 2, 0.0);
      for (int m = 0; m < n; ++m, ++mu)
        for (int c = 0; c < C; ++c) {
          const double *q = &hcs[(size_t)mu * 12 + c * 4];
          const size_t o = (size_t)c * n + m;
          pp.C0[2 * o] = 0.25 * q[0];
          pp.C0[2 * o + 1] = 0.25 * q[1];
          pp.C1[2 * o] = 0.25 * q[2];
          pp.C1[2 * o + 1] = 0.25 * q[3];
          double *k = &ccoef[4 * ((size_t)c * T2 + mu)];
          for (int i = 0; i < 4; ++i) k[i] = 0.25 * q[i];
        }
    }
  }
  RefMeta mt{};
  mt.lnL0 = r->lnL0;
  mt.dh0 = r->dh0;
  mt.hh0 = r->hh0;
  mt.ns64 = ns64;
  mt.ns32 = sinc_terms_for<float>(fmax_e);
  mt.k_lo = r->k_lo;
  mt.k_hi = r->k_hi;
  mt.pick = -1;
  if (hipMemcpyAsync(r->coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(r->is064, is64.data(), is64.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(r->meta, &mt, sizeof(mt), hipMemcpyHostToDevice, st) != hipSuccess ||
      (T2 > 0 && hipMemcpyAsync(r->pm_ccoef, ccoef.data(), ccoef.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
                     hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_free(mbh_fail(MBH_EDEVICE, "upload per-mode coefficients"));
  *out = r;
  return MBH_OK;
}

extern "C" mbh_status mbh_ref_pm_info(const mbh_ref *r, uint32_t *modes_with_bins, int32_t *n_pairs) {
  if (!r) return mbh_fail(MBH_EINVAL, "null reference");
  if (!r->pm) return mbh_fail(MBH_EINVAL, "not a per-mode reference");
  uint32_t m = 0;
  for (auto &x : r->pm_modes) m |= 1u << x.mode;
  if (modes_with_bins) *modes_with_bins = m;
  if (n_pairs) *n_pairs = (int32_t)r->pm_pairs.size();
  return MBH_OK;
}

extern "C" mbh_status mbh_ref_pm_mode(const mbh_ref *r, int mode_index, int64_t *k_lo, int64_t *k_hi,
                                      int32_t *n_bins, double *edges, int64_t *kb, double *Ares0, double *Ares1,
                                      double *B0, double *B1, double *h0_edges) {
  if (!r) return mbh_fail(MBH_EINVAL, "null reference");
  if (!r->pm) return mbh_fail(MBH_EINVAL, "not a per-mode reference");
  for (auto &m : r->pm_modes) {
    if (m.mode != mode_index) continue;
    if (k_lo) *k_lo = m.k_lo;
    if (k_hi) *k_hi = m.k_hi;
    if (n_bins) *n_bins = (int32_t)m.edges.size() - 1;
    auto cp = [](void *dst, const auto &v) {
      if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(edges, m.edges);
    cp(kb, m.kb);
    cp(Ares0, m.Ares0);
    cp(Ares1, m.Ares1);
    cp(B0, m.B0);
    cp(B1, m.B1);
    cp(h0_edges, m.h0_edges);
    return MBH_OK;
  }
  return mbh_fail(MBH_EINVAL, "mode %d has no bins in this reference", mode_index);
}

extern "C" mbh_status mbh_ref_pm_pair(const mbh_ref *r, int pair, int32_t *mode_a, int32_t *mode_b,
                                      int32_t *n_merged, double *edges, int64_t *kb, int32_t *bin_a, int32_t *bin_b,
                                      double *C0, double *C1) {
  if (!r) return mbh_fail(MBH_EINVAL, "null reference");
  if (!r->pm) return mbh_fail(MBH_EINVAL, "not a per-mode reference");
  if (pair < 0 || pair >= (int)r->pm_pairs.size()) return mbh_fail(MBH_EINVAL, "pair %d", pair);
  const auto &p = r->pm_pairs[pair];
  if (mode_a) *mode_a = p.mode_a;
  if (mode_b) *mode_b = p.mode_b;
  if (n_merged) *n_merged = (int32_t)p.edges.size() - 1;
  auto cp = [](void *dst, const auto &v) {
    if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(edges, p.edges);
  cp(kb, p.kb);
  cp(bin_a, p.bin_a);
  cp(bin_b, p.bin_b);
  cp(C0, p.C0);
  cp(C1, p.C1);
  return MBH_OK;
}

// After a refresh on the device, bring the host copies of the reference up
// to date (waits for the last refresh).
static mbh_status sync_mirror(const mbh_ref *rc) {
  mbh_ref *r = const_cast<mbh_ref *>(rc);
  std::lock_guard<std::mutex> g(r->mu);
  if (!r->rf_ready || r->rf.mirrored == r->rf.issued) return MBH_OK;
  HIP_TRY(hipSetDevice(r->ctx->device));
  HIP_TRY(hipEventSynchronize(r->rf.done));
  const int C = r->n_chan, Nb = r->n_bins, E = Nb + 1;
  RefMeta m;
  std::vector<double> paper((size_t)C * Nb * 6), h0e((size_t)C * E * 2), F(E);
  std::vector<int64_t> kb(E);
  HIP_TRY(hipMemcpy(&m, r->meta, sizeof(m), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(F.data(), r->F, E * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(kb.data(), r->rf.kb_live, E * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(paper.data(), r->rf.paper_live, paper.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(h0e.data(), r->rf.h0e_live, h0e.size() * sizeof(double), hipMemcpyDeviceToHost));
  r->lnL0 = m.lnL0;
  r->dh0 = m.dh0;
  r->hh0 = m.hh0;
  r->k_lo = m.k_lo;
  r->k_hi = m.k_hi;
  r->edges = F;
  r->kb = kb;
  r->h0_edges = h0e;
  for (size_t o = 0; o < (size_t)C * Nb; ++o) {
    r->A0[2 * o] = paper[6 * o + 0];
    r->A0[2 * o + 1] = paper[6 * o + 1];
    r->A1[2 * o] = paper[6 * o + 2];
    r->A1[2 * o + 1] = paper[6 * o + 3];
    r->B0[o] = paper[6 * o + 4];
    r->B1[o] = paper[6 * o + 5];
  }
  r->rf.mirrored = r->rf.issued;
  return MBH_OK;
}

extern "C" mbh_status mbh_ref_get_info(const mbh_ref *r, mbh_ref_info *o) {
  if (!r || !o) return mbh_fail(MBH_EINVAL, "null argument");
  MBH_TRY(sync_mirror(r));
  o->model = r->model;
  o->n_chan = r->n_chan;
  o->n_bins = r->n_bins;
  o->modes = r->modes;
  o->k_lo = r->k_lo;
  o->k_hi = r->k_hi;
  o->lnL0 = r->lnL0;
  o->dd = r->dd;
  o->dh0 = r->dh0;
  o->hh0 = r->hh0;
  return MBH_OK;
}

extern "C" mbh_status mbh_ref_export(const mbh_ref *r, double *edges, int64_t *kb, double *A0, double *A1,
                                     double *B0, double *B1, double *h0_edges) {
  if (!r) return mbh_fail(MBH_EINVAL, "null reference");
  if (r->pm) return mbh_fail(MBH_EINVAL, "per-mode reference: export with mbh_ref_pm_mode and mbh_ref_pm_pair");
  MBH_TRY(sync_mirror(r));
  if (edges) std::memcpy(edges, r->edges.data(), r->edges.size() * sizeof(double));
  if (kb) std::memcpy(kb, r->kb.data(), r->kb.size() * sizeof(int64_t));
  if (A0) std::memcpy(A0, r->A0.data(), r->A0.size() * sizeof(double));
  if (A1) std::memcpy(A1, r->A1.data(), r->A1.size() * sizeof(double));
  if (B0) std::memcpy(B0, r->B0.data(), r->B0.size() * sizeof(double));
  if (B1) std::memcpy(B1, r->B1.data(), r->B1.size() * sizeof(double));
  if (h0_edges) std::memcpy(h0_edges, r->h0_edges.data(), r->h0_edges.size() * sizeof(double));
  return MBH_OK;
}

// staging and export buffers of the refresh, allocated once per reference;
// the live export arrays start as the host build's values
static mbh_status refresh_alloc(mbh_ref *r, hipStream_t st) {
  if (r->rf_ready) return MBH_OK;
  mbh_ctx *ctx = r->ctx;
  const int C = r->n_chan, Nb = r->n_bins, E = Nb + 1;
  const size_t nce = (size_t)C * E, ncb = (size_t)C * Nb;
  mbh_ref::Refresh f;
  // grid points of the widest bin: the last (log spacing), at most
  // f_max (1 - (f_min / f_max)^(1 / Nb)) / df + 1, plus slack for rounding
  const int64_t N = r->n_f;
  const double fmax = r->f0 + (double)(N - 1) * r->df;
  f.max_len = N;
  if (r->f0 > 0.0 && fmax > r->f0) {
    const double len = -fmax * std::expm1(-std::log(fmax / r->f0) / Nb) / r->df;
    f.max_len = std::min<int64_t>(N, (int64_t)std::ceil(len) + 3);
  }
  f.n_sub = (int)std::max<int64_t>(1, (f.max_len + kRefChunk - 1) / kRefChunk);
  f.nb1 = grid_blocks(N, resident_blocks(ctx, ref_grid_kernel(modes_hm(r->model, r->modes)), kBlock));  // as in the build
  std::vector<std::pair<void **, size_t>> want = {
      {(void **)&f.wc, sizeof(WalkerC)},
      {(void **)&f.band, 2 * sizeof(unsigned long long)},
      {(void **)&f.h0w, (size_t)N * C * sizeof(double2)},
      {(void **)&f.s0, nce * sizeof(double2)},
      {(void **)&f.part1, (size_t)f.nb1 * 3 * sizeof(double)},
      {(void **)&f.sums1, 3 * sizeof(double)},
      {(void **)&f.part2, (size_t)Nb * f.n_sub * 18 * sizeof(double)},
      {(void **)&f.sums2, (size_t)Nb * 18 * sizeof(double)},
      {(void **)&f.F, E * sizeof(double)},          {(void **)&f.psi0, E * sizeof(double)},
      {(void **)&f.fq, (size_t)E * kFq * sizeof(double)}, {(void **)&f.is064, nce * 2 * sizeof(double)},
      {(void **)&f.coef, ncb * 6 * sizeof(double)},  {(void **)&f.meta, sizeof(RefMeta)},
      {(void **)&f.kb, E * sizeof(int64_t)},         {(void **)&f.kb_live, E * sizeof(int64_t)},
      {(void **)&f.paper, ncb * 6 * sizeof(double)}, {(void **)&f.paper_live, ncb * 6 * sizeof(double)},
      {(void **)&f.h0e, nce * 2 * sizeof(double)},   {(void **)&f.h0e_live, nce * 2 * sizeof(double)}};
  size_t done = 0;
  mbh_status s = MBH_OK;
  for (; done < want.size(); ++done)
    if ((s = ctx_alloc(ctx, want[done].first, want[done].second)) != MBH_OK) break;
  if (s == MBH_OK && hipEventCreateWithFlags(&f.done, hipEventDisableTiming) != hipSuccess)
    s = mbh_fail(MBH_EDEVICE, "refresh event");
  std::vector<double> paper(ncb * 6);
  for (size_t o = 0; o < ncb && s == MBH_OK; ++o) {
    paper[6 * o + 0] = r->A0[2 * o];
    paper[6 * o + 1] = r->A0[2 * o + 1];
    paper[6 * o + 2] = r->A1[2 * o];
    paper[6 * o + 3] = r->A1[2 * o + 1];
    paper[6 * o + 4] = r->B0[o];
    paper[6 * o + 5] = r->B1[o];
  }
  if (s == MBH_OK &&
      (hipMemcpyAsync(f.kb_live, r->kb.data(), E * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(f.paper_live, paper.data(), paper.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
           hipSuccess ||
       hipMemcpyAsync(f.h0e_live, r->h0_edges.data(), nce * 2 * sizeof(double), hipMemcpyHostToDevice, st) !=
           hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    s = mbh_fail(MBH_EDEVICE, "refresh set-up");
  if (s != MBH_OK) {
    for (size_t i = 0; i < done; ++i) ctx_free(ctx, *want[i].first, want[i].second);
    if (f.done) (void)hipEventDestroy(f.done);
    return s;
  }
  r->rf = f;
  r->rf_ready = true;
  return MBH_OK;
}

extern "C" mbh_status mbh_ref_refresh_prepare(mbh_ref *r, hipStream_t st) {
  if (!r) return mbh_fail(MBH_EINVAL, "null reference");
  if (r->pm) return mbh_fail(MBH_EINVAL, "per-mode references are not updated on the device");
  HIP_TRY(hipSetDevice(r->ctx->device));
  std::lock_guard<std::mutex> g(r->mu);
  return refresh_alloc(r, st);
}

extern "C" mbh_status mbh_ref_refresh(mbh_ctx *ctx, const mbh_data *data, mbh_ref *r, const double *theta_dev,
                                      const double *lnL_dev, int64_t W, hipStream_t st) {
  if (!ctx || !data || !r || !theta_dev || !lnL_dev) return mbh_fail(MBH_EINVAL, "null argument");
  if (W < 1) return mbh_fail(MBH_EINVAL, "W = %lld", (long long)W);
  if (r->pm) return mbh_fail(MBH_EINVAL, "per-mode references are not updated on the device");
  if (r->ctx != ctx || data->ctx != ctx) return mbh_fail(MBH_EINVAL, "reference or data from another context");
  if (data->n_chan != r->n_chan || data->n_f != r->n_f || data->f0 != r->f0 || data->df != r->df ||
      data->t_obs != r->t_obs)
    return mbh_fail(MBH_EINVAL, "data grid differs from the one the reference was built on");
  HIP_TRY(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> g(r->mu);
  MBH_TRY(refresh_alloc(r, st));
  const int C = r->n_chan, Nb = r->n_bins, E = Nb + 1;
  const int64_t N = data->n_f;
  const double f0 = data->f0, df = data->df;
  auto &f = r->rf;
  WalkerC *wc = f.wc;
  unsigned long long *band = f.band;
  double2 *h0w = f.h0w, *s0 = f.s0;
  double *part1 = f.part1, *sums1 = f.sums1, *part2 = f.part2, *sums2 = f.sums2;
  const int nb1 = f.nb1, n_sub = f.n_sub;
  const int64_t max_len = f.max_len;
  hipLaunchKernelGGL(k_refresh_pick, dim3(1), dim3(256), 0, st, theta_dev, lnL_dev, W, r->model, r->modes, wc, band,
                     f.meta);
  if (modes_hm(r->model, r->modes))
    hipLaunchKernelGGL(k_ref_grid<true>, dim3(nb1), dim3(kBlock), 0, st, wc, r->modes, C, N, f0, df, data->t_obs,
                       data->dw64, data->sw64, h0w, band, part1, f.meta);
  else
    hipLaunchKernelGGL(k_ref_grid<false>, dim3(nb1), dim3(kBlock), 0, st, wc, r->modes, C, N, f0, df, data->t_obs,
                       data->dw64, data->sw64, h0w, band, part1, f.meta);
  hipLaunchKernelGGL(k_sum_partials, dim3(3), dim3(64), 0, st, part1, nb1, 3, 3, sums1);
  hipLaunchKernelGGL(k_refresh_edges, dim3(1), dim3(256), 0, st, band, f0, df, Nb, max_len, f.F, f.kb, f.meta);
  hipLaunchKernelGGL(k_ref_bins, dim3(Nb, n_sub), dim3(kBlock), 0, st, f.kb, f.F, Nb, n_sub, C, N, f0, df,
                     data->dw64, h0w, part2, f.meta);
  hipLaunchKernelGGL(k_sum_bins, dim3((Nb * 18 + 255) / 256), dim3(256), 0, st, part2, Nb, n_sub, sums2);
  hipLaunchKernelGGL(k_ref_edges, dim3((E + 63) / 64), dim3(64), 0, st, wc, r->modes, C, E, f.F, data->t_obs, f.fq,
                     f.psi0, s0, f.meta);
  hipLaunchKernelGGL(k_refresh_finish, dim3(1), dim3(256), 0, st, sums1, sums2, s0, f.F, f.psi0, C, Nb, f.coef,
                     f.is064, f.paper, f.h0e, f.meta);
  RefreshCopy cp{};
  auto add = [&](const void *src, void *dst, int64_t n) {
    cp.src[cp.count] = (const uint64_t *)src;
    cp.dst[cp.count] = (uint64_t *)dst;
    cp.n[cp.count] = n;
    ++cp.count;
  };
  add(f.F, r->F, E);
  add(f.fq, r->fq, (int64_t)E * kFq);
  add(f.psi0, r->psi0, E);
  add(f.is064, r->is064, (int64_t)C * E * 2);
  add(f.coef, r->coef, (int64_t)C * Nb * 6);
  add(f.kb, f.kb_live, E);
  add(f.paper, f.paper_live, (int64_t)C * Nb * 6);
  add(f.h0e, f.h0e_live, (int64_t)C * E * 2);
  hipLaunchKernelGGL(k_refresh_commit, dim3(8), dim3(256), 0, st, cp, (const RefMeta *)f.meta, r->meta);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(f.done, st));
  ++f.issued;
  return MBH_OK;
}

extern "C" mbh_status mbh_ref_refresh_result(mbh_ref *r, int32_t *status, int64_t *pick, int32_t *generation) {
  if (!r) return mbh_fail(MBH_EINVAL, "null reference");
  RefMeta m{};
  m.pick = -1;
  {
    std::lock_guard<std::mutex> g(r->mu);
    if (r->rf_ready && r->rf.issued > 0) {
      HIP_TRY(hipSetDevice(r->ctx->device));
      HIP_TRY(hipEventSynchronize(r->rf.done));
      HIP_TRY(hipMemcpy(&m, r->meta, sizeof(m), hipMemcpyDeviceToHost));
    }
  }
  if (status) *status = m.status;
  if (pick) *pick = m.pick;
  if (generation) *generation = m.generation;
  return MBH_OK;
}

HetRef ref_view(const mbh_ref *r) {
  HetRef h;
  h.F = r->F;
  h.psi0 = r->psi0;
  h.fq = r->fq;
  h.is064 = r->is064;
  h.coef = r->coef;
  h.meta = r->meta;
  h.t_obs = r->t_obs;
  h.n_bins = r->n_bins;
  h.n_chan = r->n_chan;
  h.modes = r->modes;
  h.ns64 = h.ns32 = 0;  // set from meta on the device
  return h;
}

// ---------------------------------------------------------------- heterodyned launches
int popcount_modes(uint32_t m) { return __builtin_popcount(m); }

// mapping of the heterodyned pass: 0 = flattened (one lane per walker and
// edge), else lanes per walker of the lane-group mapping
int default_lanes(int n_bins, int n_modes) {
  (void)n_bins;
  (void)n_modes;
  return 0;
}

int lanes_lookup(const mbh_ctx *ctx, int n_bins, int n_modes, int prec) {
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->lanes.find(std::make_tuple(n_bins, n_modes, prec));
  if (it != ctx->lanes.end()) return it->second;
  return default_lanes(n_bins, n_modes);
}

// FP64-recomputation threshold of the mixed path for a tolerance tol on the
// estimated error of a walker's lnL: the walker's error sum may reach
// tol^2 / (8 kMixedErrScale^2), shared among its segments by bin count
void set_error_limits(WorkItem &it, double tol) { it.est_lim = tol * tol / (8.0 * kMixedErrScale * kMixedErrScale); }

// dynamic LDS of the per-walker cross pass of per-mode reference r, per
// walker: its deltas, T1 x C complex values; the kernel's static block-sum
// array takes at most kPmCrossStaticLds beside them
size_t pm_cross_lds(const mbh_ref *r) { return (size_t)r->pm_T1 * 3 * sizeof(double2); }
constexpr size_t kPmCrossStaticLds = 256;

// a work item for reference r with mapping G; buffers are set by the caller
WorkItem make_item(const mbh_ctx *ctx, const mbh_ref *r, int G) {
  WorkItem it;
  std::memset(&it, 0, sizeof(it));
  it.ref = ref_view(r);
  it.E = r->n_bins + 1;
  it.K = flat_slots(it.E);
  it.G = G;
  it.model = r->model;
  it.hm = modes_hm(r->model, r->modes) ? 1 : 0;
  if (r->pm) {  // per-mode reference: edge pass over T1 tasks, cross pass over T2 + 1, flattened
    it.G = 0;
    it.E = r->pm_T1;
    it.K1 = flat_slots(r->pm_T1);
    it.E2 = r->pm_T2 + 1;
    // two walkers per workgroup while their deltas stay within 64 KB of LDS
    // (the merged-bin constants then load once for both), else one if it fits
    if (r->pm_T2 > 0 && pm_cross_lds(r) + kPmCrossStaticLds <= ctx->lds_max)
      it.pm.cross_wg = 2 * pm_cross_lds(r) + kPmCrossStaticLds <= std::min(ctx->lds_max, (size_t)65536) ? 2 : 1;
    it.K = it.K1 + (it.pm.cross_wg ? 1 : flat_slots(it.E2));
    it.pm.mode_of = r->pm_mode_of;
    it.pm.bin_of = r->pm_bin_of;
    it.pm.cross = r->pm_cross;
    it.pm.ccoef = r->pm_ccoef;
    it.pm.T1 = r->pm_T1;
    it.pm.T2 = r->pm_T2;
  }
  double tol;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    tol = ctx->mixed_tol;
  }
  set_error_limits(it, tol);
  return it;
}

template <typename R, bool DH, bool HM>
static void launch_main_t(const WorkItem &it, hipStream_t st) {
  if (it.G == 0) {
    const int64_t nc = flat_chunks(it.W, it.E);
    hipLaunchKernelGGL((k_het_flat<R, DH, HM>), dim3((unsigned)((nc + kWaves - 1) / kWaves)), dim3(kBlock), 0, st,
                       it, nc);
    return;
  }
  const int wpb = kBlock / it.G;
  const dim3 grid((unsigned)((it.W + wpb - 1) / wpb)), blk(kBlock);
  switch (it.G) {
    case 1: hipLaunchKernelGGL((k_het_lane<R, 1, DH, HM>), grid, blk, 0, st, it); break;
    case 2: hipLaunchKernelGGL((k_het_lane<R, 2, DH, HM>), grid, blk, 0, st, it); break;
    case 4: hipLaunchKernelGGL((k_het_lane<R, 4, DH, HM>), grid, blk, 0, st, it); break;
    case 8: hipLaunchKernelGGL((k_het_lane<R, 8, DH, HM>), grid, blk, 0, st, it); break;
    case 16: hipLaunchKernelGGL((k_het_lane<R, 16, DH, HM>), grid, blk, 0, st, it); break;
    case 32: hipLaunchKernelGGL((k_het_lane<R, 32, DH, HM>), grid, blk, 0, st, it); break;
    default: hipLaunchKernelGGL((k_het_lane<R, 64, DH, HM>), grid, blk, 0, st, it); break;
  }
}

template <typename R, bool DH>
static void launch_main_m(const WorkItem &it, hipStream_t st) {
  if (it.hm) launch_main_t<R, DH, true>(it, st);
  else launch_main_t<R, DH, false>(it, st);
}

// main heterodyned pass of one item (partial sums only)
static void launch_main(int prec, bool dh, const WorkItem &it, hipStream_t st) {
  if (prec == MBH_FP64) {
    if (dh) launch_main_m<double, true>(it, st);
    else launch_main_m<double, false>(it, st);
  } else {
    if (dh) launch_main_m<float, true>(it, st);
    else launch_main_m<float, false>(it, st);
  }
}

// Per-walker totals of the main pass.  Batches pass their walker tiles
// (n_wtiles of them); a single item passes it by value with items == nullptr.
void launch_finish(const WorkItem *items, const WorkItem &one, const WalkerTile *wtiles, int64_t n_wtiles,
                   hipStream_t st) {
  const dim3 fb((unsigned)std::max<int64_t>(1, items ? n_wtiles : (one.W + kWalkerTile - 1) / kWalkerTile));
  hipLaunchKernelGGL(k_het_final, fb, dim3(kWalkerTile), 0, st, items, one, wtiles);
}

static mbh_status het_check(const mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev, int64_t W,
                            mbh_precision prec, const double *lnL_dev) {
  if (!ctx || !ref || (W > 0 && (!theta_dev || !lnL_dev))) return mbh_fail(MBH_EINVAL, "null argument");
  if (W < 0 || W > (int64_t)1 << 30) return mbh_fail(MBH_EINVAL, "W = %lld out of range", (long long)W);
  if (prec != MBH_FP64 && prec != MBH_MIXED) return mbh_fail(MBH_EINVAL, "bad precision");
  return MBH_OK;
}

// the single-call work item of W walkers (its scratch pointers set by the caller)
static WorkItem het_item(const mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev, int64_t W,
                         mbh_precision prec, double *lnL_dev, double *dh_hh_dev) {
  const int G = lanes_lookup(ctx, ref->n_bins, popcount_modes(ref->modes ? ref->modes : 1u), prec);
  WorkItem it = make_item(ctx, ref, G);
  it.prec = prec;
  it.theta = theta_dev;
  it.lnL = lnL_dev;
  it.dhhh = dh_hh_dev;
  it.W = W;
  it.offset = 0;
  return it;
}

// setup, main pass and totals of one item on `st`
static mbh_status het_launch(const WorkItem &it, mbh_precision prec, hipStream_t st) {
  hipLaunchKernelGGL(k_setup_one, dim3((unsigned)((it.W + 63) / 64)), dim3(128), 0, st, it);
  launch_main(prec, it.dhhh != nullptr, it, st);
  launch_finish(nullptr, it, nullptr, 0, st);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

// setup, edge pass, cross pass and totals of one per-mode item on `st` (FP64)
static mbh_status pm_launch(const WorkItem &it, hipStream_t st) {
  hipLaunchKernelGGL(k_setup_one, dim3((unsigned)((it.W + 63) / 64)), dim3(128), 0, st, it);
  const int64_t n1 = flat_chunks(it.W, it.E), n2 = flat_chunks(it.W, it.E2);
  const dim3 g1((unsigned)((n1 + kWaves - 1) / kWaves)), g2((unsigned)((n2 + kWaves - 1) / kWaves));
  const int nw = std::max(it.pm.cross_wg, 1);
  const dim3 gw((unsigned)((it.W + nw - 1) / nw));
  const size_t lds = (size_t)nw * it.pm.T1 * 3 * sizeof(double2);
  if (it.dhhh) {
    hipLaunchKernelGGL(k_pm_edges<true>, g1, dim3(kBlock), 0, st, it, n1);
    if (it.pm.cross_wg) hipLaunchKernelGGL(k_pm_cross_wg<true>, gw, dim3(kBlock), lds, st, it);
    else if (it.pm.T2 > 0) hipLaunchKernelGGL(k_pm_cross<true>, g2, dim3(kBlock), 0, st, it, n2);
  } else {
    hipLaunchKernelGGL(k_pm_edges<false>, g1, dim3(kBlock), 0, st, it, n1);
    if (it.pm.cross_wg) hipLaunchKernelGGL(k_pm_cross_wg<false>, gw, dim3(kBlock), lds, st, it);
    else if (it.pm.T2 > 0) hipLaunchKernelGGL(k_pm_cross<false>, g2, dim3(kBlock), 0, st, it, n2);
  }
  launch_finish(nullptr, it, nullptr, 0, st);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

extern "C" mbh_status mbh_loglike_heterodyned(mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev,
                                              int64_t W, mbh_precision prec, double *lnL_dev,
                                              double *dh_hh_dev, hipStream_t st) {
  MBH_TRY(het_check(ctx, ref, theta_dev, W, prec, lnL_dev));
  if (ref->pm && prec != MBH_FP64) return mbh_fail(MBH_EINVAL, "per-mode references are evaluated in MBH_FP64");
  if (W == 0) return MBH_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  Scratch sc(ctx, st);
  WorkItem it = het_item(ctx, ref, theta_dev, W, prec, lnL_dev, dh_hh_dev);
  MBH_TRY(sc.get(&it.wc, (size_t)W));
  MBH_TRY(sc.get(&it.part, (size_t)W * it.K * 4));
  if (ref->pm) {
    MBH_TRY(sc.get(&it.pm.dsc, (size_t)W * it.pm.T1 * 3));
    return pm_launch(it, st);
  }
  return het_launch(it, prec, st);
}

// Bytes of scratch a single call of W walkers needs: walker constants, then
// (from the next 256-byte boundary) the partial sums [W][K][4].
static size_t het_scratch_bytes(int64_t W, int K, size_t *part_off) {
  const size_t wc = ((size_t)W * sizeof(WalkerC) + 255) & ~(size_t)255;
  *part_off = wc;
  return wc + (size_t)W * K * 4 * sizeof(double);
}

extern "C" mbh_status mbh_loglike_heterodyned_noalloc(mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev,
                                                      int64_t W, mbh_precision prec, double *lnL_dev,
                                                      double *dh_hh_dev, hipStream_t st) {
  MBH_TRY(het_check(ctx, ref, theta_dev, W, prec, lnL_dev));
  if (ref->pm) return mbh_fail(MBH_EINVAL, "per-mode references are evaluated with mbh_loglike_heterodyned");
  if (W == 0) return MBH_OK;
  size_t part_off = 0;
  const size_t need = het_scratch_bytes(W, flat_slots(ref->n_bins + 1), &part_off);
  if (need > (size_t)MBH_NOALLOC_SCRATCH_BYTES)
    return mbh_fail(MBH_EINVAL, "W = %lld walkers at %d bins need %zu bytes of scratch, above the %zu-byte maximum",
                    (long long)W, ref->n_bins, need, (size_t)MBH_NOALLOC_SCRATCH_BYTES);
  unsigned char *base = (unsigned char *)noalloc_scratch(ctx->device);
  if (!base) return mbh_fail(MBH_EINVAL, "no scratch on device %d", ctx->device);
  HIP_TRY(hipSetDevice(ctx->device));
  WorkItem it = het_item(ctx, ref, theta_dev, W, prec, lnL_dev, dh_hh_dev);
  // every slot the totals read is written by the main pass of the same call,
  // so nothing needs clearing between calls
  it.wc = (WalkerC *)base;
  it.part = (double *)(base + part_off);
  return het_launch(it, prec, st);
}

// ---------------------------------------------------------------- full grid
// Tile of the full-grid pass: KF frequencies per thread (1 or 2) and at most
// wpb_cap walkers per workgroup.  Walker rows are sized so that the grid
// keeps >= ~8 workgroups per CU in total and runs as many short rounds of
// resident workgroups (a long-running last round leaves most of the chip
// idle); the per-(chunk, walker) partials, and so the results, do not depend
// on the number of walkers per workgroup, only on KF (the chunking).  The
// default (1, 32) measured fastest for the (2,2) mode on the 1-yr grid.
struct FullShape {
  int kf = 1, wpb_cap = 32;
};

static FullShape full_shape_of(const mbh_ctx *ctx, bool hm) {
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->full_shape.find(hm ? 1 : 0);
  FullShape f;
  if (it != ctx->full_shape.end()) {
    f.kf = it->second.first;
    f.wpb_cap = it->second.second;
  }
  return f;
}

static bool valid_full_shape(int kf, int wpb_cap) {
  return (kf == 1 || kf == 2) && (wpb_cap == 8 || wpb_cap == 16 || wpb_cap == 32 || wpb_cap == 64 || wpb_cap == 128);
}

// Partial sums of one pass are NV x W x n_chunks doubles; walkers are taken
// in groups whose partials fit kFullPartBytes, so that scratch stays bounded
// for any W (each walker's result is independent of the grouping).
constexpr size_t kFullPartBytes = (size_t)1 << 30;

template <int KF, bool DH, bool HM>
static mbh_status full_impl(mbh_ctx *ctx, const mbh_data *d, uint32_t modes, const WalkerC *wc, int64_t W,
                            int wpb_cap, double *lnL, double *dhhh, hipStream_t st, Scratch &sc) {
  const int64_t fpb = (int64_t)kBlock * KF;
  const int64_t n_fc = (d->n_f + fpb - 1) / fpb;
  if (n_fc > 65535 * 64) return mbh_fail(MBH_EINVAL, "grid too large");
  const int nv = DH ? 3 : 1;
  const int64_t group = std::max<int64_t>(1, std::min<int64_t>(W, (int64_t)(kFullPartBytes / ((size_t)nv * n_fc *
                                                                                                sizeof(double)))));
  double *part = nullptr;
  MBH_TRY(sc.get(&part, (size_t)nv * n_fc * group));
  const int64_t target = (int64_t)ctx->n_cu * 8;
  for (int64_t w0 = 0; w0 < W; w0 += group) {
    const int64_t Wg = std::min<int64_t>(group, W - w0);
    int64_t n_wc = std::max<int64_t>(1, std::min<int64_t>(Wg, target / std::max<int64_t>(1, n_fc)));
    int64_t wpb = std::min<int64_t>((Wg + n_wc - 1) / n_wc, wpb_cap);
    wpb = std::max<int64_t>(wpb, (Wg + 65534) / 65535);  // grid y at most 65535
    n_wc = (Wg + wpb - 1) / wpb;
    hipLaunchKernelGGL((k_full<KF, DH, HM>), dim3((unsigned)n_fc, (unsigned)n_wc), dim3(kBlock), 0, st, d->dw64,
                       d->sw64, d->n_chan, d->n_f, d->f0, d->df, d->t_obs, modes, wc + w0, Wg, (int)wpb, part);
    hipLaunchKernelGGL((k_full_reduce<DH ? 3 : 1>), dim3((unsigned)Wg), dim3(kBlock), 0, st, part, (int)n_fc, Wg,
                       d->dd_dev, wc + w0, lnL + w0, dhhh ? dhhh + 2 * w0 : nullptr);
  }
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

template <bool DH, bool HM>
static mbh_status full_kf(mbh_ctx *ctx, const mbh_data *d, uint32_t modes, const WalkerC *wc, int64_t W,
                          FullShape f, double *lnL, double *dhhh, hipStream_t st, Scratch &sc) {
  if (f.kf == 1) return full_impl<1, DH, HM>(ctx, d, modes, wc, W, f.wpb_cap, lnL, dhhh, st, sc);
  return full_impl<2, DH, HM>(ctx, d, modes, wc, W, f.wpb_cap, lnL, dhhh, st, sc);
}

static mbh_status full_run(mbh_ctx *ctx, const mbh_data *d, int model, uint32_t modes, const double *theta_dev,
                           int64_t W, const FullShape &f, double *lnL_dev, double *dh_hh_dev, hipStream_t st,
                           Scratch &sc) {
  WalkerC *wc = nullptr;
  MBH_TRY(sc.get(&wc, (size_t)W));
  const uint32_t m = model == MBH_MODEL_IMR ? modes : 0u;
  hipLaunchKernelGGL(k_walker_setup, dim3((unsigned)((W + 63) / 64)), dim3(128), 0, st, theta_dev, W, model, m, wc);
  if (modes_hm(model, m))
    return dh_hh_dev ? full_kf<true, true>(ctx, d, m, wc, W, f, lnL_dev, dh_hh_dev, st, sc)
                     : full_kf<false, true>(ctx, d, m, wc, W, f, lnL_dev, nullptr, st, sc);
  return dh_hh_dev ? full_kf<true, false>(ctx, d, m, wc, W, f, lnL_dev, dh_hh_dev, st, sc)
                   : full_kf<false, false>(ctx, d, m, wc, W, f, lnL_dev, nullptr, st, sc);
}

extern "C" mbh_status mbh_loglike_full(mbh_ctx *ctx, const mbh_data *data, int model, uint32_t modes,
                                       const double *theta_dev, int64_t W, mbh_precision prec, double *lnL_dev,
                                       double *dh_hh_dev, hipStream_t st) {
  if (!ctx || !data || (W > 0 && (!theta_dev || !lnL_dev))) return mbh_fail(MBH_EINVAL, "null argument");
  if (W < 0 || W > (int64_t)1 << 24) return mbh_fail(MBH_EINVAL, "W = %lld out of range", (long long)W);
  if (prec != MBH_FP64 && prec != MBH_MIXED) return mbh_fail(MBH_EINVAL, "bad precision");
  MBH_TRY(check_model(data, model, modes));
  if (W == 0) return MBH_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  Scratch sc(ctx, st);
  const uint32_t m = model == MBH_MODEL_IMR ? modes : 0u;
  return full_run(ctx, data, model, modes, theta_dev, W, full_shape_of(ctx, modes_hm(model, m)), lnL_dev, dh_hh_dev,
                  st, sc);
}

extern "C" mbh_status mbh_set_full_shape(mbh_ctx *ctx, int higher_modes, int kf, int wpb_cap) {
  if (!ctx) return mbh_fail(MBH_EINVAL, "null argument");
  if (!valid_full_shape(kf, wpb_cap))
    return mbh_fail(MBH_EINVAL, "tile (%d frequencies per thread, %d walkers) not supported", kf, wpb_cap);
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->full_shape[higher_modes ? 1 : 0] = std::make_pair(kf, wpb_cap);
  return MBH_OK;
}

extern "C" mbh_status mbh_full_shape(const mbh_ctx *ctx, int higher_modes, int *kf_out, int *wpb_cap_out) {
  if (!ctx) return mbh_fail(MBH_EINVAL, "null argument");
  const FullShape f = full_shape_of(ctx, higher_modes != 0);
  if (kf_out) *kf_out = f.kf;
  if (wpb_cap_out) *wpb_cap_out = f.wpb_cap;
  return MBH_OK;
}

extern "C" mbh_status mbh_autotune_full(mbh_ctx *ctx, const mbh_data *data, int model, uint32_t modes,
                                        const double *theta_dev, int64_t W, int *kf_out, int *wpb_cap_out) {
  if (!ctx || !data || !theta_dev || W < 1) return mbh_fail(MBH_EINVAL, "bad argument");
  if (W > (int64_t)1 << 24) return mbh_fail(MBH_EINVAL, "W = %lld out of range", (long long)W);
  MBH_TRY(check_model(data, model, modes));
  HIP_TRY(hipSetDevice(ctx->device));
  const uint32_t m = model == MBH_MODEL_IMR ? modes : 0u;
  const bool hm = modes_hm(model, m);
  hipStream_t st;
  HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  mbh_status rc = MBH_OK;
  std::vector<std::pair<float, std::pair<int, int>>> res;
  {
    Scratch sc(ctx, st);
    double *lnL = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((rc = sc.get(&lnL, (size_t)W)) == MBH_OK && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
      for (int kf : {1, 2})
        for (int cap : {8, 16, 32, 64, 128}) {
          FullShape f;
          f.kf = kf;
          f.wpb_cap = cap;
          // one untimed call, then the median of three
          std::vector<float> t;
          for (int r = 0; r < 4 && rc == MBH_OK; ++r) {
            (void)hipEventRecord(e0, st);
            Scratch s2(ctx, st);
            rc = full_run(ctx, data, model, modes, theta_dev, W, f, lnL, nullptr, st, s2);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t.push_back(ms);
          }
          if (rc != MBH_OK) break;
          std::sort(t.begin(), t.end());
          res.emplace_back(t[1], std::make_pair(kf, cap));
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == MBH_OK && (hipGetLastError() != hipSuccess || res.empty()))
      rc = mbh_fail(MBH_EDEVICE, "autotune launches failed");
  }
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (rc != MBH_OK) return rc;
  std::sort(res.begin(), res.end());
  const auto best = res.front().second;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->full_shape[hm ? 1 : 0] = best;
  }
  if (kf_out) *kf_out = best.first;
  if (wpb_cap_out) *wpb_cap_out = best.second;
  return MBH_OK;
}

// ---------------------------------------------------------------- autotuner
// 0 (flattened mapping) or a power of two in [1, 64] (lanes per walker)
static bool valid_lanes(int g) { return g == 0 || g == 1 || g == 2 || g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

extern "C" mbh_status mbh_lanes_for(const mbh_ctx *ctx, int n_bins, int n_modes, mbh_precision prec,
                                    int *lanes_out) {
  if (!ctx || !lanes_out) return mbh_fail(MBH_EINVAL, "null argument");
  *lanes_out = lanes_lookup(ctx, n_bins, n_modes, prec);
  return MBH_OK;
}

extern "C" mbh_status mbh_set_mixed_tolerance(mbh_ctx *ctx, double tol) {
  if (!ctx || !(tol >= 0.0)) return mbh_fail(MBH_EINVAL, "tolerance must be >= 0 (inf allowed)");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->mixed_tol = tol;
  return MBH_OK;
}

extern "C" mbh_status mbh_get_mixed_tolerance(const mbh_ctx *ctx, double *tol_out) {
  if (!ctx || !tol_out) return mbh_fail(MBH_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  *tol_out = ctx->mixed_tol;
  return MBH_OK;
}

extern "C" mbh_status mbh_set_lanes(mbh_ctx *ctx, int n_bins, int n_modes, mbh_precision prec, int lanes) {
  if (!ctx || !valid_lanes(lanes)) return mbh_fail(MBH_EINVAL, "lanes must be 0 or a power of two in [1, 64]");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->lanes[std::make_tuple(n_bins, n_modes, (int)prec)] = lanes;
  return MBH_OK;
}

// Times each mapping of the main heterodyned pass (flattened, and lane groups
// of 16, 32 and 64 lanes per walker) on the reference's shape with W walkers, the
// caller's (theta_dev) or, if null, copies of a fixed valid parameter point
// with small offsets; keeps the fastest.
extern "C" mbh_status mbh_autotune_heterodyned(mbh_ctx *ctx, const mbh_ref *ref, const double *theta_dev,
                                               int64_t W, mbh_precision prec, int *lanes_out) {
  if (!ctx || !ref || W < 1) return mbh_fail(MBH_EINVAL, "bad argument");
  if (prec != MBH_FP64 && prec != MBH_MIXED) return mbh_fail(MBH_EINVAL, "bad precision");
  if (ref->pm) return mbh_fail(MBH_EINVAL, "per-mode references use the flattened mapping only");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st;
  HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  mbh_status rc = MBH_OK;
  {
    Scratch sc(ctx, st);
    WorkItem it = make_item(ctx, ref, 0);
    double *th = nullptr, *lnL = nullptr;
    it.W = W;
    if ((rc = sc.get(&th, (size_t)W * 11)) != MBH_OK || (rc = sc.get(&lnL, (size_t)W)) != MBH_OK ||
        (rc = sc.get(&it.wc, (size_t)W)) != MBH_OK || (rc = sc.get(&it.part, (size_t)W * it.K * 4)) != MBH_OK) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
      return rc;
    }
    it.theta = theta_dev ? theta_dev : th;
    it.lnL = lnL;
    // default walkers: a valid parameter vector of the reference's model
    std::vector<double> h((size_t)W * 11);
    for (int64_t w = 0; w < W; ++w) {
      double *t = &h[(size_t)w * 11];
      const double base[11] = {2e6, 0.5, 0.3, -0.2, 50.0, 1.0, 1.1, 2.0, 0.3, 0.7, ref->t_obs * 0.5};
      for (int i = 0; i < 11; ++i) t[i] = base[i];
      if (ref->model == MBH_MODEL_TF2) {
        t[0] = 3e5;
        t[1] = 1e-21;
        t[2] = 1e4;
        t[3] = 0.5;
      }
      t[0] *= 1.0 + 1e-6 * (double)(w % 7);
    }
    std::vector<std::pair<float, int>> res;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    if (hipMemcpyAsync(th, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess) {
      hipLaunchKernelGGL(k_setup_one, dim3((unsigned)((W + 63) / 64)), dim3(128), 0, st, it);
      for (int G : {0, 16, 32, 64}) {
        it.G = G;
        launch_main(prec, false, it, st);  // warm-up
        (void)hipEventRecord(e0, st);
        const int reps = 20;
        for (int r = 0; r < reps; ++r) launch_main(prec, false, it, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        res.emplace_back(ms / reps, G);
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipGetLastError() != hipSuccess || res.empty()) rc = mbh_fail(MBH_EDEVICE, "autotune launches failed");
    if (rc == MBH_OK) {
      std::sort(res.begin(), res.end());
      int best = res.front().second;
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->lanes[std::make_tuple(ref->n_bins, popcount_modes(ref->modes ? ref->modes : 1u), (int)prec)] = best;
      if (lanes_out) *lanes_out = best;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  return rc;
}

// cache file: one line per entry, "arch n_bins n_modes prec lanes" for the
// heterodyned mapping and "arch full higher_modes kf wpb_cap" for the
// full-grid tile
extern "C" mbh_status mbh_autotune_save(const mbh_ctx *ctx, const char *path) {
  if (!ctx || !path) return mbh_fail(MBH_EINVAL, "null argument");
  FILE *f = fopen(path, "w");
  if (!f) return mbh_fail(MBH_EINVAL, "cannot write %s", path);
  std::lock_guard<std::mutex> g(ctx->mu);
  for (auto &kv : ctx->lanes)
    fprintf(f, "%s %d %d %d %d\n", ctx->arch.c_str(), std::get<0>(kv.first), std::get<1>(kv.first),
            std::get<2>(kv.first), kv.second);
  for (auto &kv : ctx->full_shape)
    fprintf(f, "%s full %d %d %d\n", ctx->arch.c_str(), kv.first, kv.second.first, kv.second.second);
  fclose(f);
  return MBH_OK;
}

extern "C" mbh_status mbh_autotune_load(mbh_ctx *ctx, const char *path) {
  if (!ctx || !path) return mbh_fail(MBH_EINVAL, "null argument");
  FILE *f = fopen(path, "r");
  if (!f) return mbh_fail(MBH_EINVAL, "cannot read %s", path);
  char line[256], arch[128];
  int a, b, c, d;
  std::lock_guard<std::mutex> lk(ctx->mu);
  while (fgets(line, sizeof line, f)) {
    bool full = false;
    if (sscanf(line, "%127s full %d %d %d", arch, &a, &b, &c) == 4)
      full = true;
    else if (sscanf(line, "%127s %d %d %d %d", arch, &a, &b, &c, &d) != 5)
      continue;
    // entries measured on another architecture are ignored
    if (!(ctx->arch.rfind(arch, 0) == 0 || std::string(arch).rfind(ctx->arch, 0) == 0)) continue;
    if (full) {
      if ((a == 0 || a == 1) && valid_full_shape(b, c)) ctx->full_shape[a] = std::make_pair(b, c);
    } else if (valid_lanes(d)) {
      ctx->lanes[std::make_tuple(a, b, c)] = d;
    }
  }
  fclose(f);
  return MBH_OK;
}
