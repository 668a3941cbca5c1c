// mbh_ingest.hip -- data ingest (Sec. 2.1): TDI X, Y, Z time series to the
// A, E, T frequency series the likelihoods work on.
//
// Three steps on the caller's stream: the A, E, T combination of each sample
// with the optional Tukey taper (one kernel, one pass over the samples), the
// real-to-complex transform of the three series (hipFFT, batched), and the
// band extraction with the dt scaling and the start-time phase (one kernel).
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>

#include "mbh.h"
#include "mbh_internal.hpp"

using namespace mbh;

namespace {

// A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3 of sample
// n, times the Tukey window: 0.5 (1 - cos(pi m / e)) at distance m < e from
// either end (e = alpha (N - 1) / 2; e <= 0: no taper).  xyz [3][N], aet [3][N].
__global__ __launch_bounds__(kBlock) void k_tdi_combine(const double *__restrict__ xyz, int64_t N, double e,
                                                        double *__restrict__ aet) {
  for (int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x; n < N; n += (int64_t)gridDim.x * kBlock) {
    const double x = xyz[n], y = xyz[N + n], z = xyz[2 * N + n];
    double w = 1.0;
    const double m = (double)min(n, N - 1 - n);
    if (m < e) {
      double s, c;
      sincos_red<double>(kPi * m / e, s, c);
      w = 0.5 * (1.0 - c);
    }
    aet[n] = w * ((z - x) / kSqrt2);
    aet[N + n] = w * ((x - 2.0 * y + z) / kSqrt6);
    aet[2 * N + n] = w * ((x + y + z) / kSqrt3);
  }
}

// out[c][j] = dt spec[c][k] e^{-2 pi i f_k t0}, k = k_first + j, f_k = k / (N dt);
// the phase in cycles k t0 / (N dt) is reduced to (-1/2, 1/2] before the angle
// is formed.  spec [3][N/2 + 1], out [3][n_freq][2].
__global__ __launch_bounds__(kBlock) void k_band(const double2 *__restrict__ spec, int64_t n_half, int64_t N,
                                                 double dt, double t0, int64_t k_first, int64_t n_freq,
                                                 double *__restrict__ out) {
  const int64_t total = 3 * n_freq;
  const double cyc_per_k = t0 / ((double)N * dt);
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t c = i / n_freq, j = i - c * n_freq, k = k_first + j;
    const double2 v = spec[c * n_half + k];
    double cyc = (double)k * cyc_per_k;
    cyc -= rint(cyc);
    double s, co;
    sincos_red<double>(-kTwoPi * cyc, s, co);
    out[2 * i] = dt * (v.x * co - v.y * s);
    out[2 * i + 1] = dt * (v.x * s + v.y * co);
  }
}

// one element per thread up to 2^28 elements (a partial second pass of a
// capped grid left a third of the combine kernel's threads idle)
int blocks_for(int64_t n) { return (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1 << 20); }

void destroy_plan(void *p) { (void)hipfftDestroy((hipfftHandle)p); }

// The context's plan of three batched D2Z transforms of length N (made on
// first use, without a work area of its own) and the work-area size it needs.
// Caller holds ctx->mu.
hipfftResult plan_for(mbh_ctx *ctx, int64_t N, hipfftHandle *plan, size_t *work) {
  auto it = ctx->fft_plans.find(N);
  if (it != ctx->fft_plans.end()) {
    *plan = (hipfftHandle)it->second;
    return hipfftGetSize(*plan, work);
  }
  hipfftHandle p = nullptr;
  hipfftResult r = hipfftCreate(&p);
  if (r != HIPFFT_SUCCESS) return r;
  int n = (int)N;
  r = hipfftSetAutoAllocation(p, 0);
  if (r == HIPFFT_SUCCESS) r = hipfftMakePlanMany(p, 1, &n, nullptr, 1, n, nullptr, 1, n / 2 + 1, HIPFFT_D2Z, 3, work);
  if (r != HIPFFT_SUCCESS) {
    (void)hipfftDestroy(p);
    return r;
  }
  ctx->fft_plans[N] = (void *)p;
  ctx->fft_plan_destroy = destroy_plan;
  *plan = p;
  return HIPFFT_SUCCESS;
}

}  // namespace

static mbh_status check_ingest(int64_t N, double dt, double t0, double alpha, int64_t k_first, int64_t n_freq) {
  if (N < 4 || N > (int64_t)INT32_MAX) return mbh_fail(MBH_EINVAL, "n_samples = %lld out of range", (long long)N);
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0)) return mbh_fail(MBH_EINVAL, "need dt > 0 and finite t0");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return mbh_fail(MBH_EINVAL, "Tukey alpha must lie in [0, 1]");
  if (k_first < 1 || n_freq < 2 || k_first + n_freq - 1 > N / 2)
    return mbh_fail(MBH_EINVAL, "band k = %lld .. %lld outside 1 .. N/2 = %lld (at least 2 bins)",
                    (long long)k_first, (long long)(k_first + n_freq - 1), (long long)(N / 2));
  return MBH_OK;
}

extern "C" mbh_status mbh_tdi_to_aet_fd(mbh_ctx *ctx, int64_t n_samples, double dt, double t0, const double *xyz_dev,
                                        double tukey_alpha, int64_t k_first, int64_t n_freq, double *aet_dev,
                                        hipStream_t st) {
  if (!ctx || !xyz_dev || !aet_dev) return mbh_fail(MBH_EINVAL, "null argument");
  const int64_t N = n_samples;
  mbh_status s = check_ingest(N, dt, t0, tukey_alpha, k_first, n_freq);
  if (s != MBH_OK) return s;
  if (hipSetDevice(ctx->device) != hipSuccess) return mbh_fail(MBH_EDEVICE, "hipSetDevice");
  const int64_t n_half = N / 2 + 1;
  hipfftHandle plan = nullptr;
  size_t work_bytes = 0;
  hipfftResult fr;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    fr = plan_for(ctx, N, &plan, &work_bytes);
  }
  if (fr != HIPFFT_SUCCESS) return mbh_fail(MBH_EDEVICE, "hipFFT plan error %d", (int)fr);
  double *aet = nullptr;
  double2 *spec = nullptr;
  void *work = nullptr;
  if ((s = ctx_alloc_async(ctx, (void **)&aet, (size_t)3 * N * sizeof(double), st)) != MBH_OK) return s;
  if ((s = ctx_alloc_async(ctx, (void **)&spec, (size_t)3 * n_half * sizeof(double2), st)) != MBH_OK ||
      (s = ctx_alloc_async(ctx, &work, work_bytes, st)) != MBH_OK) {
    ctx_free_async(ctx, spec, (size_t)3 * n_half * sizeof(double2), st);
    ctx_free_async(ctx, aet, (size_t)3 * N * sizeof(double), st);
    return s;
  }
  hipLaunchKernelGGL(k_tdi_combine, dim3(blocks_for(N)), dim3(kBlock), 0, st, xyz_dev, N,
                     tukey_alpha * (double)(N - 1) / 2.0, aet);
  {
    // the plan is shared by the context's calls: stream and work area are set
    // and the transform enqueued under the lock (the launch takes both along)
    std::lock_guard<std::mutex> g(ctx->mu);
    fr = hipfftSetStream(plan, st);
    if (fr == HIPFFT_SUCCESS && work) fr = hipfftSetWorkArea(plan, work);
    if (fr == HIPFFT_SUCCESS) fr = hipfftExecD2Z(plan, aet, (hipfftDoubleComplex *)spec);
  }
  if (fr == HIPFFT_SUCCESS)
    hipLaunchKernelGGL(k_band, dim3(blocks_for(3 * n_freq)), dim3(kBlock), 0, st, spec, n_half, N, dt, t0, k_first,
                       n_freq, aet_dev);
  // stream-ordered frees: the buffers are released after the kernels have run
  ctx_free_async(ctx, work, work_bytes, st);
  ctx_free_async(ctx, spec, (size_t)3 * n_half * sizeof(double2), st);
  ctx_free_async(ctx, aet, (size_t)3 * N * sizeof(double), st);
  if (fr != HIPFFT_SUCCESS) return mbh_fail(MBH_EDEVICE, "hipFFT error %d", (int)fr);
  if (hipGetLastError() != hipSuccess) return mbh_fail(MBH_EDEVICE, "ingest kernels failed to launch");
  return MBH_OK;
}

extern "C" mbh_status mbh_data_create_tdi(mbh_ctx *ctx, int64_t n_samples, double dt, double t0,
                                          const double *xyz_dev, double tukey_alpha, int64_t k_first,
                                          int64_t n_freq, const double *psd_dev, double t_obs, hipStream_t st,
                                          mbh_data **out) {
  if (!ctx || !xyz_dev || !psd_dev || !out) return mbh_fail(MBH_EINVAL, "null argument");
  *out = nullptr;
  mbh_status s = check_ingest(n_samples, dt, t0, tukey_alpha, k_first, n_freq);
  if (s != MBH_OK) return s;
  if (hipSetDevice(ctx->device) != hipSuccess) return mbh_fail(MBH_EDEVICE, "hipSetDevice");
  double *d = nullptr;
  const size_t bytes = (size_t)3 * n_freq * 2 * sizeof(double);
  if ((s = ctx_alloc(ctx, (void **)&d, bytes)) != MBH_OK) return s;
  s = mbh_tdi_to_aet_fd(ctx, n_samples, dt, t0, xyz_dev, tukey_alpha, k_first, n_freq, d, st);
  const double T = (double)n_samples * dt;
  if (s == MBH_OK) s = mbh_data_create(ctx, 3, n_freq, (double)k_first / T, 1.0 / T, t_obs, d, psd_dev, st, out);
  // the whitening has read d once the stream is through
  if (hipStreamSynchronize(st) != hipSuccess && s == MBH_OK) s = mbh_fail(MBH_EDEVICE, "ingest stream");
  ctx_free(ctx, d, bytes);
  if (s != MBH_OK && *out) {
    (void)mbh_data_release(*out);
    *out = nullptr;
  }
  return s;
}
