// mbh_kernels.hpp -- HIP kernels of libmbh (gfx950).
#pragma once

#include "mbh.h"
#include "mbh_device.hpp"

namespace mbh {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- reference
// Everything the heterodyned kernel needs about one reference, as device
// pointers.  coef is [C][Nb][6] FP64: Re/Im (A0-B0), Re/Im (A1-B1)/dF_b, B0,
// B1/dF_b, where dF_b = F_{b+1} - F_b.
// per-edge frequency constants: FreqC's a, Cp, Cm, then FreqPow
constexpr int kFq = 7;

// Scalars of a reference that a refresh on the device may change, kept in
// device memory next to its arrays.
struct RefMeta {
  double lnL0, dh0, hh0;  // lnL(h0), <d|h0>, <h0|h0>
  int32_t ns64, ns32;     // sinc terms over the edges for FP64 / FP32
  int64_t k_lo, k_hi;     // band in grid indices
  // outcome of the last refresh: walker chosen (-1: none), mbh_status,
  // refreshes committed so far
  int64_t pick;
  int32_t status, generation;
};

struct HetRef {
  const double *F;      // [E] bin edges
  const double *fq;     // [E][kFq] response factors a, Cp, Cm and FreqPow of each edge
  const double *psi0;   // [E] carrier phase of h0
  const double *is064;  // [C][E][2] 1/s0
  const double *coef;   // [C][Nb][6]
  const RefMeta *meta;
  double t_obs;
  int32_t n_bins, n_chan;
  uint32_t modes;
  int32_t ns64, ns32;   // meta's sinc term counts, loaded once per workgroup (with_meta)
};

// A reference view whose by-value copies of the scalars that a refresh may
// change are read from its device block: done once at kernel entry, so that
// the per-edge code reads them from registers.
__device__ __forceinline__ HetRef with_meta(HetRef r) {
  // read through the constant address space: the block does not change
  // while a likelihood kernel runs, so the load is a scalar one and the term
  // counts stay in scalar registers
  typedef const RefMeta __attribute__((address_space(4))) ConstMeta;
  ConstMeta *m = (ConstMeta *)(uintptr_t)r.meta;
  r.ns64 = m->ns64;
  r.ns32 = m->ns32;
  return r;
}

// ---------------------------------------------------------------- utilities
// value of lane perm(i) within lane i's row of 16 (DPP control CTRL), for
// both halves of a double
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double x, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                          __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Sum over the 64 lanes of a wavefront, returned (uniform) in every lane, in
// a fixed order: within each row of 16 lanes by data-parallel-primitive
// moves (lane xor 1, xor 2, the mirrored half row, the mirrored row), then
// the four row sums as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// fixed-order block sum of up to 3 values; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double *sh /* [NV][kBlock/64] */) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i * (kBlock / 64) + wv] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int k = 0; k < kBlock / 64; ++k) s += sh[i * (kBlock / 64) + k];
      v[i] = s;
    }
  }
}

// ---------------------------------------------------------------- a1: ingest
// two threads per walker (intrinsic and extrinsic parts), 64 walkers per
// workgroup of 128 threads
static __global__ __launch_bounds__(128) void k_walker_setup(const double *__restrict__ theta, int64_t W, int model,
                                                             uint32_t modes, WalkerC *__restrict__ out) {
  const int64_t w = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (w >= W) return;
  walker_setup(theta + w * 11, model, modes, out[w], threadIdx.x < 64 ? 1 : 2);
}

// ---------------------------------------------------------------- data
// whitening: w = 4 df / S; dw = d sqrt(w); sw = sqrt(w) / kAmpScale.
// Per-block partial of <d|d> = sum |dw|^2.
static __global__ __launch_bounds__(kBlock) void k_whiten(const double *__restrict__ d, const double *__restrict__ psd,
                                                   int64_t n_total, double df, double2 *__restrict__ dw64,
                                                   double *__restrict__ sw64, double *__restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * kBlock) {
    double w = 4.0 * df / psd[i];
    double s = sqrt(w);
    double re = d[2 * i] * s, im = d[2 * i + 1] * s;
    dw64[i] = make_double2(re, im);
    sw64[i] = s / kAmpScale;
    acc += re * re + im * im;
  }
  double v[1] = {acc};
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// out[i] = sum_b part[b * stride + i] for i < n_out: one wavefront per
// output, lanes stride over the partials, fixed butterfly (grid n_out x 64)
static __global__ __launch_bounds__(64) void k_sum_partials(const double *__restrict__ part, int n_part, int stride,
                                                            int n_out, double *__restrict__ out) {
  const int i = blockIdx.x;
  if (i >= n_out) return;
  double s = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < n_part; b += 64) s += part[(int64_t)b * stride + i];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[i] = s;
}

static __global__ void k_init_band(unsigned long long *band) {
  band[0] = ~0ull;
  band[1] = 0ull;
}

// ---------------------------------------------------------------- template on the grid
// h [C][N][2] (unscaled FP64), for signal injection
static __global__ __launch_bounds__(kBlock) void k_template_grid(const WalkerC *__restrict__ wc, uint32_t modes,
                                                          int n_chan, int64_t n_f, double f0, double df,
                                                          double t_obs, double2 *__restrict__ h) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n_f) return;
  const WalkerC &w = wc[0];
  double f = grid_freq(f0, df, k);
  cx<double> s[3];
  double psi;
  const int ns = sinc_terms_for<double>(grid_freq(f0, df, n_f - 1));
  bool any = template_point<double>(w, modes, f, freq_pows(f), freq_consts<double>(f, ns), t_obs, s, psi);
  double sp = 0.0, cp = 1.0;
  if (any) sincos_red<double>(reduce_2pi(psi), sp, cp);
  for (int c = 0; c < n_chan; ++c) {
    cx<double> v = any ? s[c] * mk<double>(cp, -sp) : mk<double>(0.0, 0.0);
    h[c * n_f + k] = make_double2(v.re / kAmpScale, v.im / kAmpScale);
  }
}

// ---------------------------------------------------------------- a9: reference build
// pass 1: whitened h0 on the grid, band ends, and block partials of
// -2 lnL(h0) = sum |dw - h0w|^2, <d|h0>, <h0|h0>
template <bool HM>
__global__ __launch_bounds__(kBlock) void k_ref_grid(const WalkerC *__restrict__ wc, uint32_t modes, int n_chan,
                                                     int64_t n_f, double f0, double df, double t_obs,
                                                     const double2 *__restrict__ dw, const double *__restrict__ sw,
                                                     double2 *__restrict__ h0w, unsigned long long *band,
                                                     double *__restrict__ part, const RefMeta *gate) {
  if (gate && gate->status != 0) return;
  __shared__ double sh[3 * (kBlock / 64)];
  const WalkerC &w = wc[0];
  double a_res = 0.0, a_dh = 0.0, a_hh = 0.0;
  unsigned long long lo = ~0ull, hi = 0ull;
  bool seen = false;
  const int ns = sinc_terms_for<double>(grid_freq(f0, df, n_f - 1));
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_f; k += (int64_t)gridDim.x * kBlock) {
    double f = grid_freq(f0, df, k);
    cx<double> s[3];
    double psi;
    bool any = template_point<double, HM>(w, modes, f, freq_pows(f), freq_consts<double>(f, ns), t_obs, s, psi);
    double sp = 0.0, cp = 1.0;
    if (any) sincos_red<double>(reduce_2pi(psi), sp, cp);
    bool nz = false;
    for (int c = 0; c < n_chan; ++c) {
      int64_t i = c * n_f + k;
      cx<double> h = any ? s[c] * mk<double>(cp, -sp) : mk<double>(0.0, 0.0);
      h = sw[i] * h;
      if (h.re != 0.0 || h.im != 0.0) nz = true;
      h0w[i] = make_double2(h.re, h.im);
      double2 d = dw[i];
      double rr = d.x - h.re, ri = d.y - h.im;
      a_res += rr * rr + ri * ri;
      a_dh += d.x * h.re + d.y * h.im;
      a_hh += h.re * h.re + h.im * h.im;
    }
    if (nz) {
      if (!seen) lo = (unsigned long long)k;
      seen = true;
      hi = (unsigned long long)k;
    }
  }
  if (seen) {
    atomicMin(&band[0], lo);
    atomicMax(&band[1], hi);
  }
  double v[3] = {a_res, a_dh, a_hh};
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = v[0];
    part[blockIdx.x * 3 + 1] = v[1];
    part[blockIdx.x * 3 + 2] = v[2];
  }
}

// pass 2: per (bin, chunk) sums over the bin's grid points of
// (dw - h0w) conj(h0w) {1, (f - f_b)} and |h0w|^2 {1, (f - f_b)} per channel.
// part layout [Nb][n_sub][C][6].
constexpr int kRefChunk = 4096;
static __global__ __launch_bounds__(kBlock) void k_ref_bins(const int64_t *__restrict__ kb, const double *__restrict__ F,
                                                     int n_bins, int n_sub, int n_chan, int64_t n_f, double f0,
                                                     double df, const double2 *__restrict__ dw,
                                                     const double2 *__restrict__ h0w, double *__restrict__ part,
                                                     const RefMeta *gate) {
  if (gate && gate->status != 0) return;
  __shared__ double sh[18 * (kBlock / 64)];
  const int b = blockIdx.x, sub = blockIdx.y;
  const int64_t k_begin = kb[b] + (int64_t)sub * kRefChunk;
  const int64_t k_end = min(kb[b + 1], k_begin + kRefChunk);
  double acc[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) acc[i] = 0.0;
  if (k_begin < k_end) {
    const double fb = 0.5 * (F[b] + F[b + 1]);
    for (int64_t k = k_begin + threadIdx.x; k < k_end; k += kBlock) {
      double x = grid_freq(f0, df, k) - fb;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c >= n_chan) break;
        int64_t i = c * n_f + k;
        double2 d = dw[i], h = h0w[i];
        double rr = d.x - h.x, ri = d.y - h.y;
        // (d - h0) conj(h0)
        double tr = rr * h.x + ri * h.y, ti = ri * h.x - rr * h.y;
        double h2 = h.x * h.x + h.y * h.y;
        acc[c * 6 + 0] += tr;
        acc[c * 6 + 1] += ti;
        acc[c * 6 + 2] += tr * x;
        acc[c * 6 + 3] += ti * x;
        acc[c * 6 + 4] += h2;
        acc[c * 6 + 5] += h2 * x;
      }
    }
  }
  block_sum<18>(acc, sh);
  if (threadIdx.x == 0) {
    double *o = part + ((int64_t)b * n_sub + sub) * 18;
    for (int i = 0; i < 18; ++i) o[i] = acc[i];
  }
}

// sum the chunks of each bin in a fixed order: part [Nb][n_sub][18] -> out
// [Nb][18], one thread per (bin, value); the loads run ahead of the adds
static __global__ __launch_bounds__(256) void k_sum_bins(const double *__restrict__ part, int n_bins, int n_sub,
                                                         double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_bins * 18) return;
  const int b = t / 18, i = t - b * 18;
  const double *p = part + (int64_t)b * n_sub * 18 + i;
  double s = 0.0;
#pragma unroll 8
  for (int sub = 0; sub < n_sub; ++sub) s += p[(int64_t)sub * 18];
  out[t] = s;
}

// pass 3: response factors of the edges, carrier phase and small factors of
// h0 at the edges
static __global__ __launch_bounds__(64) void k_ref_edges(const WalkerC *__restrict__ wc, uint32_t modes, int n_chan,
                                                         int E, const double *__restrict__ F, double t_obs,
                                                         double *__restrict__ fq, double *__restrict__ psi0,
                                                         double2 *__restrict__ s0, const RefMeta *gate) {
  if (gate && gate->status != 0) return;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= E) return;
  FreqC fc;
  freq_consts64(F[j], fc.a, fc.Cp, fc.Cm);
  fc.ns = sinc_terms_for<double>(F[E - 1]);
  const FreqPow pw = freq_pows(F[j]);
  double *q = fq + (int64_t)kFq * j;
  q[0] = fc.a;
  q[1] = fc.Cp;
  q[2] = fc.Cm;
  q[3] = pw.f13;
  q[4] = pw.fm13;
  q[5] = pw.fi;
  q[6] = pw.fm76;
  cx<double> s[3];
  double psi;
  bool any = template_point<double>(wc[0], modes, F[j], pw, fc, t_obs, s, psi);
  psi0[j] = psi;
  for (int c = 0; c < n_chan; ++c) s0[c * E + j] = any ? make_double2(s[c].re, s[c].im) : make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------- reference refresh
// Sec. 3.2 replaces the reference by the highest-likelihood point of the
// population every few thousand sampler iterations.  On the device this is
// the reference build above with its host steps moved into kernels: pick the
// walker, then band, edges and bin assignment, then the coefficients, all
// written to a staging copy that replaces the live reference only if every
// step succeeded.  A failed step sets the staging status and the later
// kernels return at once.

// Best walker (largest finite lnL; the lowest index among equals), its
// walker constants, and the band's initial value.  One block of 256.
static __global__ __launch_bounds__(256) void k_refresh_pick(const double *__restrict__ theta,
                                                             const double *__restrict__ lnL, int64_t W, int model,
                                                             uint32_t modes, WalkerC *__restrict__ wc,
                                                             unsigned long long *band, RefMeta *stg) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  __shared__ double th[11];
  const int t = threadIdx.x;
  double bv = 0.0;
  int64_t bi = -1;
  for (int64_t i = t; i < W; i += 256) {
    const double v = lnL[i];
    if (isfinite(v) && (bi < 0 || v > bv)) {
      bv = v;
      bi = i;
    }
  }
  sv[t] = bv;
  si[t] = bi;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      const double v = sv[t + h];
      const int64_t i = si[t + h];
      if (i >= 0 && (si[t] < 0 || v > sv[t] || (v == sv[t] && i < si[t]))) {
        sv[t] = v;
        si[t] = i;
      }
    }
    __syncthreads();
  }
  const int64_t pick = si[0];
  if (pick >= 0 && t < 11) th[t] = theta[pick * 11 + t];
  __syncthreads();
  if (pick >= 0 && (t == 0 || t == 64)) walker_setup(th, model, modes, wc[0], t == 0 ? 1 : 2);
  __syncthreads();
  if (t == 0) {
    stg->pick = pick;
    stg->status = pick < 0 ? MBH_EINVAL : (wc[0].valid ? MBH_OK : MBH_EINVAL);
    band[0] = ~0ull;
    band[1] = 0ull;
  }
}

// Band, log-spaced edges and the first grid index of each bin, with the same
// roundings as the host build (the interior edges go through the device's
// exp and log).  Fails if the band is empty or a bin holds more than
// max_len grid points (the bound the bin-sum launch was sized for).  One
// block of 256.
#pragma clang fp contract(off)
static __global__ __launch_bounds__(256) void k_refresh_edges(const unsigned long long *band, double f0, double df,
                                                              int n_bins, int64_t max_len, double *__restrict__ F,
                                                              int64_t *__restrict__ kb, RefMeta *stg) {
  if (stg->status != 0) return;
  __shared__ unsigned long long worst;
  const unsigned long long lo = band[0], hi = band[1];
  if (lo == ~0ull || hi <= lo) {
    if (threadIdx.x == 0) stg->status = MBH_EBAND;
    return;
  }
  if (threadIdx.x == 0) worst = 0ull;
  const int64_t k_lo = (int64_t)lo, k_hi = (int64_t)hi;
  const double F0 = grid_freq(f0, df, k_lo), FN = grid_freq(f0, df, k_hi);
  const double l0 = log(F0), span = log(FN) - l0;
  for (int j = threadIdx.x; j <= n_bins; j += blockDim.x) {
    double e;
    int64_t k;
    if (j == 0) {
      e = F0;
      k = k_lo;
    } else if (j == n_bins) {
      e = FN;
      k = k_hi + 1;
    } else {
      e = exp(l0 + (double)j * span / (double)n_bins);
      int64_t a = k_lo, b = k_hi;  // smallest k with f_k >= e
      while (a < b) {
        const int64_t mid = a + (b - a) / 2;
        if (grid_freq(f0, df, mid) >= e) b = mid;
        else a = mid + 1;
      }
      k = a;
    }
    F[j] = e;
    kb[j] = k;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < n_bins; b += blockDim.x) {
    const int64_t len = kb[b + 1] - kb[b];
    if (len > max_len || len < 0) atomicMax(&worst, 1ull);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (worst) stg->status = MBH_EINVAL;
    stg->k_lo = k_lo;
    stg->k_hi = k_hi;
  }
}

// Coefficients from the bin sums (as in the host build), 1/s0, h0 at the
// edges in the paper's units and the reference scalars.  Fails if h0 is zero
// or not finite at an edge.  One block of 256.
static __global__ __launch_bounds__(256) void k_refresh_finish(const double *__restrict__ sums1,
                                                               const double *__restrict__ sums2,
                                                               const double2 *__restrict__ s0,
                                                               const double *__restrict__ F,
                                                               const double *__restrict__ psi0, int n_chan, int n_bins,
                                                               double *__restrict__ coef, double *__restrict__ is064,
                                                               double *__restrict__ paper, double *__restrict__ h0e,
                                                               RefMeta *stg) {
  if (stg->status != 0) return;
  __shared__ int bad;
  const int E = n_bins + 1, t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int i = t; i < n_chan * E; i += blockDim.x) {
    const double2 v = s0[i];
    if (!(v.x != 0.0 || v.y != 0.0) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(&bad, 1);
  }
  __syncthreads();
  if (bad) {
    if (t == 0) stg->status = MBH_EBAND;
    return;
  }
  for (int o = t; o < n_chan * n_bins; o += blockDim.x) {
    const int c = o / n_bins, b = o - c * n_bins;
    const double *q = sums2 + (int64_t)b * 18 + c * 6;
    // the grid sums carry w = 4 df / S; the coefficients carry df / S
    const double amb0r = 0.25 * q[0], amb0i = 0.25 * q[1], amb1r = 0.25 * q[2], amb1i = 0.25 * q[3];
    const double b0 = 0.25 * q[4], b1 = 0.25 * q[5];
    const double idf = 1.0 / (F[b + 1] - F[b]);
    double *k = coef + 6 * (int64_t)o;
    k[0] = amb0r;
    k[1] = amb0i;
    k[2] = amb1r * idf;
    k[3] = amb1i * idf;
    k[4] = b0;
    k[5] = b1 * idf;
    double *p = paper + 6 * (int64_t)o;
    p[0] = amb0r + b0;
    p[1] = amb0i;
    p[2] = amb1r + b1;
    p[3] = amb1i;
    p[4] = b0;
    p[5] = b1;
  }
  for (int i = t; i < n_chan * E; i += blockDim.x) {
    const double re = s0[i].x, im = s0[i].y;
    const double den = re * re + im * im;
    is064[2 * i] = re / den;
    is064[2 * i + 1] = -im / den;
    const int j = i % E;
    const double ph = remainder(psi0[j], 2.0 * kPi);
    const double cp = cos(ph), sp = sin(ph);
    h0e[2 * i] = (re * cp + im * sp) / kAmpScale;
    h0e[2 * i + 1] = (im * cp - re * sp) / kAmpScale;
  }
  if (t == 0) {
    stg->lnL0 = -0.5 * sums1[0];
    stg->dh0 = sums1[1];
    stg->hh0 = sums1[2];
    stg->ns64 = sinc_terms_for<double>(F[E - 1]);
    stg->ns32 = sinc_terms_for<float>(F[E - 1]);
  }
}
#pragma clang fp contract(on)

// Arrays a refresh replaces, staging -> live, in one launch, copied as
// 8-byte words (the doubles bit for bit, and the int64 bin indices).
struct RefreshCopy {
  static constexpr int kMax = 8;
  const uint64_t *src[kMax];
  uint64_t *dst[kMax];
  int64_t n[kMax];
  int count;
};

// Copy staging to live if the refresh succeeded; record its outcome in the
// live scalars either way.
static __global__ __launch_bounds__(256) void k_refresh_commit(RefreshCopy cp, const RefMeta *stg, RefMeta *live) {
  const bool ok = stg->status == 0;
  if (ok) {
    for (int a = 0; a < cp.count; ++a)
      for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cp.n[a];
           i += (int64_t)gridDim.x * blockDim.x)
        cp.dst[a][i] = cp.src[a][i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (ok) {
      live->lnL0 = stg->lnL0;
      live->dh0 = stg->dh0;
      live->hh0 = stg->hh0;
      live->ns64 = stg->ns64;
      live->ns32 = stg->ns32;
      live->k_lo = stg->k_lo;
      live->k_hi = stg->k_hi;
      live->generation += 1;
    }
    live->pick = stg->pick;
    live->status = stg->status;
  }
}

// ---------------------------------------------------------------- a2-a7: heterodyned
// Residual form of the heterodyned likelihood (Sec. 2.2): with delta = r - 1
// at the bin edges, delta_0 its value at the bin centre and delta_1 its slope,
//   lnL = lnL(h0) + sum_b,c { 4 Re[(A0 - B0) delta_0* + (A1 - B1) delta_1*]
//                             - 2 [B0 |delta_0|^2 + 2 B1 Re(delta_0 delta_1*)] },
// which equals -(1/2)(<d|d> + Z[h,h] - 2 Z[d,h]) up to the second-order
// B2 term that the piecewise-linear ratio drops.
//
// Mixed precision: the FP32 parts of the response (sinc series, link phase
// factors) leave a per-edge relative error of ~1e-7 on r - 1, random from
// edge to edge; its effect on lnL is estimated as kMixedErrScale sqrt(S / 2),
// S = sum over bins and channels of |dT/d delta_0|^2 + 4 |dT/d delta_1|^2
// (the gradient of the bin term T with respect to the edge values).
// kMixedErrScale bounds the measured ratio |lnL_mixed - lnL_fp64| / sqrt(S / 2)
// over tempered walker clouds at SNR 100-1000.  The estimate is formed per
// segment (a walker's bins within one wavefront's chunk, or the whole walker
// in a lane-group mapping) and a segment whose share could push the walker's
// estimate above the tolerance tol (default kMixedRouteTol) is recomputed in
// FP64 by the same wavefront right away: a segment of n of the N_b bins is
// kept in FP32 only if kMixedErrScale^2 8 s < tol^2 n / N_b (s the segment's
// sum S / 16), so the kept segments of a walker add up to at most tol.
constexpr double kMixedErrScale = 2.5e-7;
constexpr double kMixedRouteTol = 9e-4;

// Flattened mapping: task t = w E + j is (walker w, edge j).  A wavefront
// takes the 64 tasks 63 c .. 63 c + 63 of chunk c: every lane evaluates its
// edge, and lanes 0..62 close the bin that starts at their edge with the
// value of lane + 1, so each bin is formed exactly once and no lane idles.
constexpr int kChunk = 63;
constexpr int kWaves = kBlock / 64;

// A pointer read from a work item is generic, so loads through it are flat
// loads, which wait on the LDS counter as well; this view of it in the
// global address space (where the work list's arrays live) gives global loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *as_global(const T *p) {
  return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}
// two doubles as a native vector: loads, stores and copies of it work in
// every address space (unlike those of the double2 class)
typedef double dvec2 __attribute__((ext_vector_type(2)));

// Per-mode relative binning (higher modes, each mode with its own bins and
// ratio r_L = h_L / h0_L; Sec. 2.2 applied per mode).  The reference's edge
// arrays (F, fq, psi0, is064) hold the edges of all its modes one mode after
// the other (T1 of them), its coefficient array the bins likewise (NB).
// Cross terms between two modes run over their merged edge grids (T2 merged
// bins in all): merged bin m lies in bin ea of one mode and eb of the other
// (given as the bins' left edges in the edge arrays), at offsets xa, xb from
// the two bins' centres; ia, ib are the reciprocal bin widths.
struct PmCross {
  int32_t ea, eb;
  double xa, xb, ia, ib;
};
struct PmView {
  const int32_t *mode_of;  // [T1] mode index of each edge
  const int32_t *bin_of;   // [T1] bin starting at the edge (-1 at a mode's last edge)
  const PmCross *cross;    // [T2]
  const double *ccoef;     // [C][T2][4]: Re/Im C0, Re/Im C1 of the merged bins
  double2 *dsc;            // [W][T1][C] delta = r - 1 at every edge (per-call scratch)
  int32_t T1, T2;
  int32_t cross_wg;        // > 0: the cross pass runs one workgroup per cross_wg walkers (1 or 2), deltas in LDS
  int32_t pad;
};

// One heterodyned work item: a reference, a walker batch, its outputs and
// per-walker scratch.  G is the number of lanes per walker of the lane-group
// mapping, or 0 for the flattened mapping.
struct WorkItem {
  HetRef ref;
  const double *theta;   // [W][11]
  WalkerC *wc;           // [W] walker constants
  double *lnL;           // [W]
  double *dhhh;          // [W][2] or null
  double *part;          // [W][K][4] per-walker partial sums of the main pass
  unsigned long long *redo;  // running count of segments recomputed in FP64, or null
  // mixed path: a segment of n bins is recomputed in FP64 unless its error
  // sum s[3] is below est_lim n / N_b
  double est_lim;
  int64_t W;
  int64_t offset;        // first walker of this item in its batch
  int32_t E, K, G, model;
  int32_t hm, prec;      // hm: the reference has modes beyond (2,2) (kernels compiled with HM);
                         // prec: MBH_FP64 or MBH_MIXED (batches group their tiles by it)
  // per-mode references (pm.T1 > 0): E = T1 tasks per walker in the edge pass
  // (slots 0..), E2 = T2 + 1 in the cross pass (slots K1..); E2 = 0 otherwise
  PmView pm;
  int32_t E2, K1;
};

// chunks of the flattened main pass (the last bin sits at task W E - 2)
__host__ __device__ inline int64_t flat_chunks(int64_t W, int E) { return (W * E - 2) / kChunk + 1; }
// partial slots per walker: chunks that one walker's bins can touch
__host__ __device__ inline int flat_slots(int E) { return (E - 2) / kChunk + 2; }

// delta = r - 1 at edge j of walker c
template <typename R, bool HM>
__device__ __forceinline__ void het_edge(const HetRef &ref, const WalkerC &c, int j, cx<double> dl[3]) {
  cx<double> s[3];
  double psi;
  const auto *q = as_global(ref.fq + (int64_t)kFq * j);
  const FreqC fc{q[0], q[1], q[2], sizeof(R) == 8 ? ref.ns64 : ref.ns32};
  const FreqPow pw{q[3], q[4], q[5], q[6]};
  template_point<R, HM>(c, ref.modes, *as_global(ref.F + j), pw, fc, ref.t_obs, s, psi);
  // the carrier difference enters every channel of the edge at once: formed
  // and reduced to [-pi, pi] in FP64 in both paths; its sine and cosine in
  // the template precision (in FP32 they add an edge-to-edge random error of
  // the same size as the response's, which the error estimate's calibration
  // covers)
  const double dpsi = reduce_2pi(psi - *as_global(ref.psi0 + j));
  double hs, hc;
  if constexpr (sizeof(R) == 4) {
    float hs32, hc32;
    sincos_red<float>((float)(0.5 * dpsi), hs32, hc32);
    hs = hs32;
    hc = hc32;
  } else {
    sincos_red<double>(0.5 * dpsi, hs, hc);
  }
  // e^{-i dpsi} - 1 = -2 sin^2(dpsi/2) - i sin(dpsi)
  const cx<double> em1 = mk<double>(-2.0 * hs * hs, -2.0 * hs * hc);
  const cx<double> e = mk<double>(1.0 + em1.re, em1.im);
  const int E = ref.n_bins + 1;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if (ch >= ref.n_chan) break;
    const auto *p = as_global(ref.is064 + 2 * (ch * E + j));
    cx<double> is0 = mk<double>(p[0], p[1]);
    cx<double> q = s[ch] * is0;
    q.re -= 1.0;
    dl[ch] = q * e + em1;  // r - 1 without cancellation
  }
}

// bin term of bin b from delta at its left (L) and right (Rt) edges:
// v[0] += lnL - lnL(h0), v[1] += Z[d,h] - <d|h0>, v[2] += Z[h,h] - <h0|h0>,
// v[3] += squared gradient (without its factor 4) for the FP32 error estimate
template <bool EST, bool DH>
__device__ __forceinline__ void bin_terms(const HetRef &ref, int b, const cx<double> L[3], const cx<double> Rt[3],
                                          double v[4]) {
  const int Nb = ref.n_bins;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if (ch >= ref.n_chan) break;
    const auto *k = as_global(ref.coef + ((int64_t)ch * Nb + b) * 6);
    // delta_0 at the bin centre and the edge difference delta_1 dF_b
    const double d0r = 0.5 * (L[ch].re + Rt[ch].re), d0i = 0.5 * (L[ch].im + Rt[ch].im);
    const double d1r = Rt[ch].re - L[ch].re, d1i = Rt[ch].im - L[ch].im;
    const double re_a = k[0] * d0r + k[1] * d0i + k[2] * d1r + k[3] * d1i;
    const double m0 = d0r * d0r + d0i * d0i;
    const double x01 = d0r * d1r + d0i * d1i;
    v[0] += 4.0 * re_a - 2.0 * (k[4] * m0 + 2.0 * k[5] * x01);
    if constexpr (DH) {
      // Z[d,h] - <d|h0> = 4 Re[A0 conj(d0) + A1 conj(d1)], A = (A - B) + B
      v[1] += 4.0 * (re_a + k[4] * d0r + k[5] * d1r);
      // Z[h,h] - <h0|h0> = 4 {B0 (2 Re d0 + |d0|^2) + 2 B1 (Re d1 + Re d0 conj d1)}
      v[2] += 4.0 * (k[4] * (2.0 * d0r + m0) + 2.0 * k[5] * (d1r + x01));
    }
    if constexpr (EST) {
      const double g0r = k[0] - k[4] * d0r - k[5] * d1r, g0i = k[1] - k[4] * d0i - k[5] * d1i;
      const double g1r = k[2] - k[5] * d0r, g1i = k[3] - k[5] * d0i;
      v[3] += g0r * g0r + g0i * g0i + 4.0 * (g1r * g1r + g1i * g1i);
    }
  }
}

// Lane-group mapping: G lanes per walker, lane gl takes edges gl, gl + G, ...
// The right edge of each bin comes from lane gl + 1 (rotation within the
// group); the last lane's bin closes one iteration later with lane 0's next
// edge.  Every lane of the wavefront runs the loop (the rotations read other
// lanes); lanes whose `on` is false evaluate nothing and sum zeros.  Returns
// the group's sums in every lane of the group.
template <typename R, int G, bool EST, bool DH, bool HM>
__device__ __forceinline__ void group_sums(const WorkItem &it, const WalkerC &c, bool on, double v[4]) {
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int Nb = it.ref.n_bins, E = Nb + 1;
  const int n_iter = (E + G - 1) / G;
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = 0.0;
  cx<double> dprev[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) dprev[ch] = mk<double>(0.0, 0.0);
  const int src = (lane & ~(G - 1)) | ((gl + 1) & (G - 1));
  for (int itr = 0; itr < n_iter; ++itr) {
    const int j = itr * G + gl;
    cx<double> dl[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) dl[ch] = mk<double>(0.0, 0.0);
    if (on && j < E) het_edge<R, HM>(it.ref, c, j, dl);
    cx<double> nb[3], lft[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      nb[ch].re = __shfl(dl[ch].re, src, 64);
      nb[ch].im = __shfl(dl[ch].im, src, 64);
      lft[ch] = gl < G - 1 ? dl[ch] : dprev[ch];
    }
    const int b = gl < G - 1 ? j : itr * G - 1;
    if (on && b >= 0 && b < Nb) bin_terms<EST, DH>(it.ref, b, lft, nb, v);
    if (gl == G - 1) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) dprev[ch] = dl[ch];
    }
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], off, 64);
}

// Main pass of walker w in the lane-group mapping: its single slot.  On the
// mixed path a walker whose error sum reaches est_lim is recomputed in FP64
// by its group (the other groups of the wavefront take part in the rotations
// only).
template <typename R, int G, bool DH, bool HM>
__device__ __forceinline__ void het_walker(const WorkItem &it, int64_t w) {
  constexpr bool EST = sizeof(R) == 4;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  // with one walker per wavefront its constants are wave-uniform
  if constexpr (G == 64) w = (int64_t)__builtin_amdgcn_readfirstlane((int)w);
  const bool active = w < it.W;
  const WalkerC &c = it.wc[active ? w : 0];
  const bool valid = active && c.valid;
  double v[4];
  group_sums<R, G, EST, DH, HM>(it, c, valid, v);
  if constexpr (EST) {
    const bool redo = valid && !(v[3] < it.est_lim);
    const uint64_t m = __ballot(redo && gl == 0);
    if (m) {
      double u[4];
      group_sums<double, G, false, DH, HM>(it, c, redo, u);
      if (redo) {
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = u[q];
        v[3] = 0.0;
      }
      if (lane == 0 && it.redo) atomicAdd(it.redo, (unsigned long long)__popcll(m));
    }
  }
  if (active && gl == 0) {
    double *o = it.part + w * it.K * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = v[q];
  }
}

// Bin terms of one lane of a flattened chunk: the lane's edge value, the
// right neighbour's from lane + 1, and the terms of the bin starting at the
// lane's edge (zero where `bin` is false).  Run by every lane of the wavefront.
template <typename R, bool EST, bool DH, bool HM>
__device__ __forceinline__ void chunk_terms(const WorkItem &it, const WalkerC &c, int j, bool edge, bool bin,
                                            double val[4]) {
  cx<double> dl[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) dl[ch] = mk<double>(0.0, 0.0);
  if (edge) het_edge<R, HM>(it.ref, c, j, dl);
  cx<double> nb[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    nb[ch].re = __shfl_down(dl[ch].re, 1, 64);
    nb[ch].im = __shfl_down(dl[ch].im, 1, 64);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) val[q] = 0.0;
  if (bin) bin_terms<EST, DH>(it.ref, j, dl, nb, val);
}

// chunk sums of walker vs (wave-uniform) over the lanes whose walker is vs,
// fixed butterfly order
template <bool EST, bool DH>
__device__ __forceinline__ void segment_sums(const double val[4], bool mine, double s[4]) {
  s[0] = wave_sum(mine ? val[0] : 0.0);
  s[1] = DH ? wave_sum(mine ? val[1] : 0.0) : 0.0;
  s[2] = DH ? wave_sum(mine ? val[2] : 0.0) : 0.0;
  s[3] = EST ? wave_sum(mine ? val[3] : 0.0) : 0.0;
}

// Flattened mapping, one chunk per wavefront: the tasks of the item's W
// walkers, E per walker.  For every walker with bins in the chunk, the
// chunk's sums go to the walker's slot (chunk - first chunk of the walker).
// On the mixed path, the segments whose error sum reaches their share of
// est_lim are recomputed in FP64 by the same wavefront before their slots are
// written.
template <typename R, bool DH, bool HM>
__device__ __forceinline__ void het_chunk(const WorkItem &it, int64_t chunk) {
  constexpr bool EST = sizeof(R) == 4;
  const int lane = threadIdx.x & 63;
  const int E = it.E;
  // chunk is wave-uniform: the first task's walker and edge are scalars, the
  // lanes' offsets from them need only a 32-bit division
  const int64_t t0 = chunk * kChunk;
  const int64_t v0 = t0 / E;
  const int j0 = (int)(t0 - v0 * E);
  const unsigned jl = (unsigned)(j0 + lane);
  const unsigned qv = jl / (unsigned)E;  // v - v0, below 64
  const int64_t v = v0 + qv;
  const int j = (int)(jl - qv * (unsigned)E);
  const bool act = v < it.W;
  const WalkerC &c = it.wc[act ? v : 0];
  const bool valid = act && c.valid;
  const bool is_bin = valid && lane < kChunk && j < E - 1;
  double val[4];
  chunk_terms<R, EST, DH, HM>(it, c, j, valid, is_bin, val);
  // walkers with a bin in the chunk: v0 unless the chunk starts at its last
  // edge, up to the walker of lane kChunk - 1
  const int64_t v_lo = v0 + (j0 == E - 1 ? 1 : 0);
  const int64_t v_hi = min(v0 + (j0 + kChunk - 1) / E, it.W - 1);
  uint64_t redo = 0;  // bit vs - v0: walker vs's segment goes to FP64
  for (int64_t vs = v_lo; vs <= v_hi; ++vs) {
    double s[4];
    segment_sums<EST, DH>(val, is_bin && v == vs, s);
    if constexpr (EST) {
      // n bins of walker vs here (none for an invalid walker: nothing to redo)
      const int n = __popcll(__ballot(is_bin && v == vs));
      if (n > 0 && __builtin_amdgcn_readfirstlane(s[3] * it.ref.n_bins < it.est_lim * n ? 0 : 1)) {
        redo |= 1ull << (vs - v0);
        continue;
      }
    }
    if (lane == 0) {
      double *o = it.part + (vs * it.K + (chunk - (vs * E) / kChunk)) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = s[q];
    }
  }
  if constexpr (EST) {
    if (redo) {
      const bool mine = (redo >> qv) & 1ull;
      chunk_terms<double, false, DH, HM>(it, c, j, valid && mine, is_bin && mine, val);
      for (int64_t vs = v_lo; vs <= v_hi; ++vs) {
        if (!((redo >> (vs - v0)) & 1ull)) continue;
        double s[4];
        segment_sums<false, DH>(val, is_bin && v == vs, s);
        if (lane == 0) {
          double *o = it.part + (vs * it.K + (chunk - (vs * E) / kChunk)) * 4;
#pragma unroll
          for (int q = 0; q < 4; ++q) o[q] = s[q];
        }
      }
      if (lane == 0 && it.redo) atomicAdd(it.redo, (unsigned long long)__popcll(redo));
    }
  }
}

// Walkers of one item handled by one workgroup of the setup and totals
// kernels (kWalkerTile walkers from w_begin), so that the item is uniform.
constexpr int kWalkerTile = 64;
struct WalkerTile {
  int32_t item, pad;
  int64_t w_begin;
  // the item's fields by value: a tile's workgroup reads them in the same
  // round of loads as the tile, not in a second one through the item index
  WorkItem it;
};

struct WalkerTotals {
  double lnL, dh, hh;
};

// lnL, <d|h> and <h|h> of walker w of an item: its partial slots added in
// slot order and the reference's h0 terms added; written to the item's
// outputs and returned
__device__ inline WalkerTotals het_walker_totals(const WorkItem &it, int64_t w) {
  double s[3] = {0.0, 0.0, 0.0};
  int n_slot = 1;
  if (it.G == 0) n_slot = (int)((w * it.E + it.E - 2) / kChunk - (w * it.E) / kChunk) + 1;
  const double *p = it.part + w * it.K * 4;
  for (int k = 0; k < n_slot; ++k)
#pragma unroll
    for (int q = 0; q < 3; ++q) s[q] += p[4 * k + q];
  if (it.E2 > 1) {  // the cross pass of a per-mode reference (one slot when a workgroup took the walker)
    const int n2 = it.pm.cross_wg ? 1 : (int)((w * it.E2 + it.E2 - 2) / kChunk - (w * it.E2) / kChunk) + 1;
    for (int k = 0; k < n2; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) s[q] += p[4 * (it.K1 + k) + q];
  }
  const bool valid = it.wc[w].valid;
  const RefMeta &m = *it.ref.meta;
  const WalkerTotals r{valid ? m.lnL0 + s[0] : -INFINITY, valid ? m.dh0 + s[1] : 0.0, valid ? m.hh0 + s[2] : 0.0};
  it.lnL[w] = r.lnL;
  if (it.dhhh) {
    it.dhhh[2 * w] = r.dh;
    it.dhhh[2 * w + 1] = r.hh;
  }
  return r;
}

// Per-walker totals of the main pass.  One workgroup of kWalkerTile threads
// per walker tile (batches: items != nullptr, the item's fields read from the
// tile) or, for a single item passed by value in `one` with items == nullptr,
// per kWalkerTile consecutive walkers.
static __global__ __launch_bounds__(kWalkerTile) void k_het_final(const WorkItem *__restrict__ items, WorkItem one,
                                                                  const WalkerTile *__restrict__ wtiles) {
  const WorkItem &it = items ? wtiles[blockIdx.x].it : one;
  const int64_t w = (items ? wtiles[blockIdx.x].w_begin : (int64_t)blockIdx.x * kWalkerTile) + threadIdx.x;
  if (w < it.W) (void)het_walker_totals(it, w);
}

// single-item path: walker constants, two threads per walker (intrinsic and
// extrinsic parts), 64 walkers per workgroup of 128 threads
static __global__ __launch_bounds__(128) void k_setup_one(WorkItem one) {
  const int64_t w = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (w < one.W) walker_setup(one.theta + w * 11, one.model, one.ref.modes, one.wc[w], threadIdx.x < 64 ? 1 : 2);
}

// single-item launches of the main pass
template <typename R, int G, bool DH, bool HM>
__global__ __launch_bounds__(kBlock, 2) void k_het_lane(WorkItem one) {
  one.ref = with_meta(one.ref);
  het_walker<R, G, DH, HM>(one, (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G);
}

template <typename R, bool DH, bool HM>
__global__ __launch_bounds__(kBlock, 2) void k_het_flat(WorkItem one, int64_t n_chunks) {
  const int64_t c = (int64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  one.ref = with_meta(one.ref);
  if (c < n_chunks) het_chunk<R, DH, HM>(one, c);
}

// ---------------------------------------------------------------- a8: full grid
// lnL = -1/2 <d-h|d-h> = -1/2 (<d|d> + sum (|h|^2 - 2 Re d* h)) over the
// grid and channels: <d|d> is the data's (FP64, computed once), so the
// points outside the template's support add exactly nothing and the data
// enter only through Re d* h.  FP64 throughout.
//
// Block (fc, wc): KF grid frequencies per thread kept in registers, then a
// loop over the block's walkers (wave-uniform constants); per walker and
// block one FP64 partial of sum (|h|^2 - 2 Re d* h) (and <d|h>, <h|h>).
// part layout [NV][W][n_fchunks] (a walker's partials contiguous for the
// totals kernel).
template <int KF, bool DH, bool HM>
__global__ __launch_bounds__(kBlock, 2) void k_full(const double2 *__restrict__ dw, const double *__restrict__ sw,
                                                 int n_chan, int64_t n_f, double f0, double df, double t_obs,
                                                 uint32_t modes, const WalkerC *__restrict__ wc, int64_t W,
                                                 int w_per_block, double *__restrict__ part) {
  constexpr int NV = DH ? 3 : 1;
  __shared__ double sh[NV * (kBlock / 64)];
  const int64_t n_fc = gridDim.x;
  double2 d[KF][3];
  double s_w[KF][3];
  double fq[KF];
  FreqC fcs[KF];
  bool inr[KF];
  // sinc terms for the highest frequency of this workgroup (uniform)
  const int ns = sinc_terms_for<double>(
      grid_freq(f0, df, min(n_f - 1, (int64_t)blockIdx.x * (kBlock * KF) + kBlock * KF - 1)));
#pragma unroll
  for (int i = 0; i < KF; ++i) {
    int64_t k = (int64_t)blockIdx.x * (kBlock * KF) + i * kBlock + threadIdx.x;
    inr[i] = k < n_f;
    fq[i] = grid_freq(f0, df, inr[i] ? k : 0);
    fcs[i] = freq_consts<double>(fq[i], ns);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < n_chan && inr[i]) {
        d[i][c] = dw[c * n_f + k];
        s_w[i][c] = sw[c * n_f + k];
      } else {
        d[i][c].x = d[i][c].y = 0.0;
        s_w[i][c] = 0.0;
      }
    }
  }
  const int64_t w0 = (int64_t)blockIdx.y * w_per_block;
  const int64_t w1 = min(W, w0 + w_per_block);
  for (int64_t w = w0; w < w1; ++w) {
    const int64_t wu = __builtin_amdgcn_readfirstlane((int)w);
    const WalkerC &c = wc[wu];
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = 0.0;
    if (c.valid) {
#pragma unroll
      for (int i = 0; i < KF; ++i) {
        if (!inr[i]) continue;
        cx<double> s[3];
        double psi;
        if (!template_point<double, HM>(c, modes, fq[i], freq_pows(fq[i]), fcs[i], t_obs, s, psi)) continue;
        double sp, cp;
        sincos_red<double>(reduce_2pi(psi), sp, cp);
        const cx<double> e = mk<double>(cp, -sp);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          if (ch >= n_chan) break;
          const cx<double> h = s_w[i][ch] * (s[ch] * e);
          const double hh = h.re * h.re + h.im * h.im;
          const double dh = d[i][ch].x * h.re + d[i][ch].y * h.im;
          v[0] += hh - 2.0 * dh;
          if constexpr (DH) {
            v[1] += dh;
            v[2] += hh;
          }
        }
      }
    }
    block_sum<NV>(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < NV; ++i) part[((int64_t)i * W + w) * n_fc + blockIdx.x] = v[i];
  }
}

// Totals, one workgroup per walker: its threads stride over the walker's
// contiguous chunk partials, then a fixed-order block sum (the result does
// not depend on W or on the launch).
template <int NV>
static __global__ __launch_bounds__(kBlock) void k_full_reduce(const double *__restrict__ part, int n_fc, int64_t W,
                                                               const double *__restrict__ dd,
                                                               const WalkerC *__restrict__ wc,
                                                               double *__restrict__ lnL, double *__restrict__ dhhh) {
  __shared__ double sh[NV * (kBlock / 64)];
  const int64_t w = blockIdx.x;
  double s[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double *p = part + ((int64_t)i * W + w) * n_fc;
    double a = 0.0;
#pragma unroll 8
    for (int fc = threadIdx.x; fc < n_fc; fc += kBlock) a += p[fc];
    s[i] = a;
  }
  block_sum<NV>(s, sh);
  if (threadIdx.x != 0) return;
  const bool ok = wc[w].valid;
  lnL[w] = ok ? -0.5 * (*dd + s[0]) : -INFINITY;
  if constexpr (NV == 3) {
    if (dhhh) {
      dhhh[2 * w] = ok ? s[1] : 0.0;
      dhhh[2 * w + 1] = ok ? s[2] : 0.0;
    }
  }
}

// ---------------------------------------------------------------- per-mode relative binning
// Reference build, grid pass: each mode's whitened h0_L (at rank r of the
// reference's modes: h0w + r C N), their sum htot, each mode's band (first
// and last grid index where h0_L != 0) and the block partials of
// -2 lnL(h0), <d|h0>, <h0|h0>.  IMR model, three channels.
static __global__ __launch_bounds__(kBlock) void k_pm_ref_grid(const WalkerC *__restrict__ wc, uint32_t modes,
                                                              int64_t n_f, double f0, double df, double t_obs,
                                                              const double2 *__restrict__ dw,
                                                              const double *__restrict__ sw, double2 *__restrict__ h0w,
                                                              double2 *__restrict__ htot, unsigned long long *band,
                                                              double *__restrict__ part) {
  __shared__ double sh[3 * (kBlock / 64)];
  const WalkerC &w = wc[0];
  double a_res = 0.0, a_dh = 0.0, a_hh = 0.0;
  unsigned long long lo[kNumModes], hi[kNumModes];
#pragma unroll
  for (int r = 0; r < kNumModes; ++r) {
    lo[r] = ~0ull;
    hi[r] = 0ull;
  }
  const int ns = sinc_terms_for<double>(grid_freq(f0, df, n_f - 1));
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_f; k += (int64_t)gridDim.x * kBlock) {
    const double f = grid_freq(f0, df, k);
    const FreqPow pw = freq_pows(f);
    const FreqC fc = freq_consts<double>(f, ns);
    cx<double> tot[3] = {mk<double>(0.0, 0.0), mk<double>(0.0, 0.0), mk<double>(0.0, 0.0)};
    int rank = 0;
#pragma unroll 1
    for (int mi = 0; mi < kNumModes; ++mi) {
      if (!(modes & (1u << mi))) continue;
      cx<double> s[3];
      double psi;
      const bool any = mode_point<double>(w, mi, f, pw, fc, t_obs, s, psi);
      double sp = 0.0, cp = 1.0;
      if (any) sincos_red<double>(reduce_2pi(psi), sp, cp);
      bool nz = false;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t i = c * n_f + k;
        cx<double> h = any ? s[c] * mk<double>(cp, -sp) : mk<double>(0.0, 0.0);
        h = sw[i] * h;
        if (h.re != 0.0 || h.im != 0.0) nz = true;
        h0w[((int64_t)rank * 3 + c) * n_f + k] = make_double2(h.re, h.im);
        tot[c] = tot[c] + h;
      }
      if (nz) {
        lo[rank] = min(lo[rank], (unsigned long long)k);
        hi[rank] = (unsigned long long)k;
      }
      ++rank;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = c * n_f + k;
      htot[i] = make_double2(tot[c].re, tot[c].im);
      const double2 d = dw[i];
      const double rr = d.x - tot[c].re, ri = d.y - tot[c].im;
      a_res += rr * rr + ri * ri;
      a_dh += d.x * tot[c].re + d.y * tot[c].im;
      a_hh += tot[c].re * tot[c].re + tot[c].im * tot[c].im;
    }
  }
  for (int r = 0; r < kNumModes; ++r) {
    if (lo[r] != ~0ull) {
      atomicMin(&band[2 * r], lo[r]);
      atomicMax(&band[2 * r + 1], hi[r]);
    }
  }
  double v[3] = {a_res, a_dh, a_hh};
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = v[0];
    part[blockIdx.x * 3 + 1] = v[1];
    part[blockIdx.x * 3 + 2] = v[2];
  }
}

// Mode bins: per (bin, chunk) sums over the bin's grid points of
// (dw - htot) conj(h0w_L) {1, (f - f_b)} and |h0w_L|^2 {1, (f - f_b)} per
// channel (the residual-form A - B and B of the mode), part [Nb][n_sub][18].
static __global__ __launch_bounds__(kBlock) void k_pm_mode_bins(const int64_t *__restrict__ kb,
                                                               const double *__restrict__ F, int n_sub, int64_t n_f,
                                                               double f0, double df, const double2 *__restrict__ dw,
                                                               const double2 *__restrict__ htot,
                                                               const double2 *__restrict__ hL,
                                                               double *__restrict__ part) {
  __shared__ double sh[18 * (kBlock / 64)];
  const int b = blockIdx.x, sub = blockIdx.y;
  const int64_t k_begin = kb[b] + (int64_t)sub * kRefChunk;
  const int64_t k_end = min(kb[b + 1], k_begin + kRefChunk);
  double acc[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) acc[i] = 0.0;
  if (k_begin < k_end) {
    const double fb = 0.5 * (F[b] + F[b + 1]);
    for (int64_t k = k_begin + threadIdx.x; k < k_end; k += kBlock) {
      const double x = grid_freq(f0, df, k) - fb;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t i = c * n_f + k;
        const double2 d = dw[i], t = htot[i], h = hL[i];
        const double rr = d.x - t.x, ri = d.y - t.y;
        const double tr = rr * h.x + ri * h.y, ti = ri * h.x - rr * h.y;
        const double h2 = h.x * h.x + h.y * h.y;
        acc[c * 6 + 0] += tr;
        acc[c * 6 + 1] += ti;
        acc[c * 6 + 2] += tr * x;
        acc[c * 6 + 3] += ti * x;
        acc[c * 6 + 4] += h2;
        acc[c * 6 + 5] += h2 * x;
      }
    }
  }
  block_sum<18>(acc, sh);
  if (threadIdx.x == 0) {
    double *o = part + ((int64_t)b * n_sub + sub) * 18;
    for (int i = 0; i < 18; ++i) o[i] = acc[i];
  }
}

// Merged bins of mode pairs: per (merged bin, chunk) sums over grid points
// kbeg[m] .. kend[m] - 1 of hA conj(hB) {1, (f - fm[m])} per channel, with
// hA, hB the whitened h0 of the modes at ranks ra[m], rb[m];
// part [M][n_sub][12].
static __global__ __launch_bounds__(kBlock) void k_pm_pair_bins(const int64_t *__restrict__ kbeg,
                                                               const int64_t *__restrict__ kend,
                                                               const double *__restrict__ fm,
                                                               const int32_t *__restrict__ ra,
                                                               const int32_t *__restrict__ rb, int n_sub, int64_t n_f,
                                                               double f0, double df, const double2 *__restrict__ h0w,
                                                               double *__restrict__ part) {
  __shared__ double sh[12 * (kBlock / 64)];
  const int m = blockIdx.x, sub = blockIdx.y;
  const int64_t k_begin = kbeg[m] + (int64_t)sub * kRefChunk;
  const int64_t k_end = min(kend[m], k_begin + kRefChunk);
  const double2 *hA = h0w + (int64_t)ra[m] * 3 * n_f, *hB = h0w + (int64_t)rb[m] * 3 * n_f;
  double acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = 0.0;
  if (k_begin < k_end) {
    const double fc = fm[m];
    for (int64_t k = k_begin + threadIdx.x; k < k_end; k += kBlock) {
      const double x = grid_freq(f0, df, k) - fc;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t i = c * n_f + k;
        const double2 a = hA[i], b = hB[i];
        const double tr = a.x * b.x + a.y * b.y, ti = a.y * b.x - a.x * b.y;  // a conj(b)
        acc[c * 4 + 0] += tr;
        acc[c * 4 + 1] += ti;
        acc[c * 4 + 2] += tr * x;
        acc[c * 4 + 3] += ti * x;
      }
    }
  }
  block_sum<12>(acc, sh);
  if (threadIdx.x == 0) {
    double *o = part + ((int64_t)m * n_sub + sub) * 12;
    for (int i = 0; i < 12; ++i) o[i] = acc[i];
  }
}

// sum the chunks of each bin in a fixed order: part [n][n_sub][nv] -> out [n][nv]
static __global__ __launch_bounds__(256) void k_pm_sum(const double *__restrict__ part, int n, int n_sub, int nv,
                                                       double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nv) return;
  const int b = t / nv, i = t - b * nv;
  const double *p = part + (int64_t)b * n_sub * nv + i;
  double s = 0.0;
  for (int sub = 0; sub < n_sub; ++sub) s += p[(int64_t)sub * nv];
  out[t] = s;
}

// the edges of every mode: response factors and frequency powers, and h0_L
// at its own edges (carrier psi0 and small factors s0 [C][T1])
static __global__ __launch_bounds__(64) void k_pm_ref_edges(const WalkerC *__restrict__ wc,
                                                           const int32_t *__restrict__ mode_of, int T1,
                                                           const double *__restrict__ F, int ns, double t_obs,
                                                           double *__restrict__ fq, double *__restrict__ psi0,
                                                           double2 *__restrict__ s0) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= T1) return;
  FreqC fc;
  freq_consts64(F[j], fc.a, fc.Cp, fc.Cm);
  fc.ns = ns;
  const FreqPow pw = freq_pows(F[j]);
  double *q = fq + (int64_t)kFq * j;
  q[0] = fc.a;
  q[1] = fc.Cp;
  q[2] = fc.Cm;
  q[3] = pw.f13;
  q[4] = pw.fm13;
  q[5] = pw.fi;
  q[6] = pw.fm76;
  cx<double> s[3];
  double psi;
  const bool any = mode_point<double>(wc[0], mode_of[j], F[j], pw, fc, t_obs, s, psi);
  psi0[j] = psi;
  for (int c = 0; c < 3; ++c) s0[c * T1 + j] = any ? make_double2(s[c].re, s[c].im) : make_double2(0.0, 0.0);
}

// delta_L = h_L / h0_L - 1 at edge tau (of mode mode_of[tau]) of walker c,
// without cancellation, as het_edge (FP64)
__device__ __forceinline__ void pm_edge(const WorkItem &it, const WalkerC &c, int tau, cx<double> dl[3]) {
  const HetRef &ref = it.ref;
  const auto *q = as_global(ref.fq + (int64_t)kFq * tau);
  const FreqC fc{q[0], q[1], q[2], ref.ns64};
  const FreqPow pw{q[3], q[4], q[5], q[6]};
  cx<double> s[3];
  double psi;
  mode_point<double>(c, *as_global(it.pm.mode_of + tau), *as_global(ref.F + tau), pw, fc, ref.t_obs, s, psi);
  const double dpsi = reduce_2pi(psi - *as_global(ref.psi0 + tau));
  double hs, hc;
  sincos_red<double>(0.5 * dpsi, hs, hc);
  const cx<double> em1 = mk<double>(-2.0 * hs * hs, -2.0 * hs * hc);
  const cx<double> e = mk<double>(1.0 + em1.re, em1.im);
  const int T1 = it.pm.T1;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const auto *p = as_global(ref.is064 + 2 * (ch * T1 + tau));
    const cx<double> is0 = mk<double>(p[0], p[1]);
    cx<double> r = s[ch] * is0;
    r.re -= 1.0;
    dl[ch] = r * e + em1;
  }
}

// the chunk's sums of each walker with bins in it go to the walker's slot
// `slot0 + chunk - first chunk of the walker` (as het_chunk, FP64)
template <bool DH>
__device__ __forceinline__ void pm_store_segments(const WorkItem &it, int64_t chunk, int E, int64_t v0, int j0,
                                                  int64_t v, bool is_bin, const double val[4], int slot0) {
  const int lane = threadIdx.x & 63;
  const int64_t v_lo = v0 + (j0 == E - 1 ? 1 : 0);
  const int64_t v_hi = min(v0 + (j0 + kChunk - 1) / E, it.W - 1);
  for (int64_t vs = v_lo; vs <= v_hi; ++vs) {
    double s[4];
    segment_sums<false, DH>(val, is_bin && v == vs, s);
    if (lane == 0) {
      double *o = it.part + (vs * it.K + slot0 + (chunk - (vs * E) / kChunk)) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = s[q];
    }
  }
}

// Edge pass of a per-mode reference, one chunk per wavefront: task
// t = w T1 + tau is (walker w, edge tau); every lane evaluates its mode at
// its edge and stores delta (for the cross pass), and lanes 0..62 close the
// bin that starts at their edge (unless it is the mode's last edge) with
// the value of lane + 1: data term and the mode's own <h|h> term.
template <bool DH>
__device__ __forceinline__ void pm_chunk_edges(const WorkItem &it, int64_t chunk) {
  const int lane = threadIdx.x & 63;
  const int E = it.E;
  const int64_t t0 = chunk * kChunk;
  const int64_t v0 = t0 / E;
  const int j0 = (int)(t0 - v0 * E);
  const unsigned jl = (unsigned)(j0 + lane);
  const unsigned qv = jl / (unsigned)E;
  const int64_t v = v0 + qv;
  const int tau = (int)(jl - qv * (unsigned)E);
  const bool act = v < it.W;
  const WalkerC &c = it.wc[act ? v : 0];
  const bool valid = act && c.valid;
  const int b = *as_global(it.pm.bin_of + tau);
  const bool is_bin = valid && lane < kChunk && b >= 0;
  cx<double> dl[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) dl[ch] = mk<double>(0.0, 0.0);
  if (valid) pm_edge(it, c, tau, dl);
  if (act) {
    auto *o = as_global((dvec2 *)(it.pm.dsc + ((int64_t)v * E + tau) * 3));
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) o[ch] = dvec2{dl[ch].re, dl[ch].im};
  }
  cx<double> nb[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    nb[ch].re = __shfl_down(dl[ch].re, 1, 64);
    nb[ch].im = __shfl_down(dl[ch].im, 1, 64);
  }
  double val[4] = {0.0, 0.0, 0.0, 0.0};
  if (is_bin) bin_terms<false, DH>(it.ref, b, dl, nb, val);
  pm_store_segments<DH>(it, chunk, E, v0, j0, v, is_bin, val, 0);
}

// Cross pass: task t = w (T2 + 1) + mu is (walker w, merged bin mu) (the
// last task of a walker is empty).  Both modes' lines at the merged centre
// from the deltas of their own bins' edges, and the merged bin's terms:
//   lnL:          -4 Re[C0 P0 + C1 P1],
//   Z[d,h]:       +4 Re[C0 dA + C1 dA1] + 4 Re[C0 dB* + C1 dB1*],
//   Z[h,h]:       +8 Re[C0 (P0 + dA + dB*) + C1 (P1 + dA1 + dB1*)],
// with P0 = dA dB*, P1 = dA1 dB* + dA dB1* (dA, dB the lines at the centre,
// dA1, dB1 their slopes): the cross terms of <h|h> linearised about the
// merged centre, and the parts of the data and <h|h> terms that involve the
// other mode's reference.
// Constants of merged bin mu: its edges, offsets and reciprocal widths, and
// per channel C0, C1 (Re, Im)
struct PmBinC {
  PmCross x;
  double k[12];
};
__device__ __forceinline__ PmBinC pm_bin_consts(const WorkItem &it, int mu) {
  PmBinC b;
  const auto *xp = as_global(it.pm.cross + mu);
  b.x = PmCross{xp->ea, xp->eb, xp->xa, xp->xb, xp->ia, xp->ib};
  const int T2 = it.pm.T2;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const auto *k = as_global(it.pm.ccoef + ((int64_t)ch * T2 + mu) * 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) b.k[4 * ch + q] = k[q];
  }
  return b;
}

// Terms of a merged bin (constants b) from the deltas D of one walker (D:
// LDS or global)
template <bool DH, typename DP>
__device__ __forceinline__ void pm_cross_terms(const PmBinC &b, DP D, double val[4]) {
  const PmCross &x = b.x;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const dvec2 a0 = D[x.ea * 3 + ch], a1 = D[(x.ea + 1) * 3 + ch];
    const dvec2 b0 = D[x.eb * 3 + ch], b1 = D[(x.eb + 1) * 3 + ch];
    const cx<double> sA = mk<double>((a1.x - a0.x) * x.ia, (a1.y - a0.y) * x.ia);
    const cx<double> sB = mk<double>((b1.x - b0.x) * x.ib, (b1.y - b0.y) * x.ib);
    const cx<double> dA = mk<double>(0.5 * (a0.x + a1.x) + sA.re * x.xa, 0.5 * (a0.y + a1.y) + sA.im * x.xa);
    const cx<double> dB = mk<double>(0.5 * (b0.x + b1.x) + sB.re * x.xb, 0.5 * (b0.y + b1.y) + sB.im * x.xb);
    const cx<double> cB = mk<double>(dB.re, -dB.im), cSB = mk<double>(sB.re, -sB.im);
    const cx<double> P0 = dA * cB;
    const cx<double> P1 = sA * cB + dA * cSB;
    const cx<double> C0 = mk<double>(b.k[4 * ch], b.k[4 * ch + 1]), C1 = mk<double>(b.k[4 * ch + 2], b.k[4 * ch + 3]);
    const double q = (C0 * P0).re + (C1 * P1).re;
    val[0] -= 4.0 * q;
    if constexpr (DH) {
      val[1] += 4.0 * ((C0 * dA).re + (C1 * sA).re + (C0 * cB).re + (C1 * cSB).re);
      val[2] += 8.0 * (q + (C0 * dA).re + (C0 * cB).re + (C1 * sA).re + (C1 * cSB).re);
    }
  }
}

template <bool DH>
__device__ __forceinline__ void pm_chunk_cross(const WorkItem &it, int64_t chunk) {
  const int lane = threadIdx.x & 63;
  const int E = it.E2;
  const int T1 = it.pm.T1, T2 = it.pm.T2;
  const int64_t t0 = chunk * kChunk;
  const int64_t v0 = t0 / E;
  const int j0 = (int)(t0 - v0 * E);
  const unsigned jl = (unsigned)(j0 + lane);
  const unsigned qv = jl / (unsigned)E;
  const int64_t v = v0 + qv;
  const int mu = (int)(jl - qv * (unsigned)E);
  const bool act = v < it.W;
  const bool valid = act && it.wc[act ? v : 0].valid;
  const bool is_bin = valid && lane < kChunk && mu < T2;
  double val[4] = {0.0, 0.0, 0.0, 0.0};
  if (is_bin) pm_cross_terms<DH>(pm_bin_consts(it, mu), as_global((const dvec2 *)(it.pm.dsc + (int64_t)v * T1 * 3)), val);
  pm_store_segments<DH>(it, chunk, E, v0, j0, v, is_bin, val, it.K1);
}

// Cross pass with one workgroup of kBlock threads per pm.cross_wg walkers
// (1 or 2; 0 selects the chunked pass): each walker's deltas (T1 x C complex
// values, contiguous) are staged in LDS by coalesced loads, and every merged
// bin reads them there instead of through the caches, its constants loaded
// once for the workgroup's walkers; thread i takes merged bins i,
// i + kBlock, ... in turn, and each walker's fixed-order workgroup sum goes
// to its slot K1.  `sd` is the dynamic LDS, cross_wg x T1 x C double2.
template <bool DH>
__device__ __forceinline__ void pm_walker_cross(const WorkItem &it, int64_t w0, double2 *sd) {
  __shared__ double sh[3 * kWaves];
  const int nw = it.pm.cross_wg;
  const int n = it.pm.T1 * 3;
  bool on[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) on[k] = k < nw && w0 + k < it.W && it.wc[w0 + k].valid;  // uniform
  dvec2 *S = (dvec2 *)sd;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (!on[k]) continue;
    const auto *D = as_global((const dvec2 *)(it.pm.dsc + (w0 + k) * n));
    for (int i = threadIdx.x; i < n; i += kBlock) S[k * n + i] = D[i];
  }
  __syncthreads();
  double val[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  if (on[0] || on[1]) {
    const dvec2 *Sc = S;
    for (int mu = threadIdx.x; mu < it.pm.T2; mu += kBlock) {
      const PmBinC b = pm_bin_consts(it, mu);
      if (on[0]) pm_cross_terms<DH>(b, Sc, val[0]);
      if (on[1]) pm_cross_terms<DH>(b, Sc + n, val[1]);
    }
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= nw || w0 + k >= it.W) break;  // uniform
    block_sum<3>(val[k], sh);
    if (threadIdx.x == 0) {
      double *o = it.part + ((w0 + k) * it.K + it.K1) * 4;
      o[0] = val[k][0];
      o[1] = val[k][1];
      o[2] = val[k][2];
      o[3] = 0.0;
    }
  }
}

// single-item launches of the two passes
template <bool DH>
__global__ __launch_bounds__(kBlock, 2) void k_pm_edges(WorkItem one, int64_t n_chunks) {
  const int64_t c = (int64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  one.ref = with_meta(one.ref);
  if (c < n_chunks) pm_chunk_edges<DH>(one, c);
}
template <bool DH>
__global__ __launch_bounds__(kBlock, 2) void k_pm_cross(WorkItem one, int64_t n_chunks) {
  const int64_t c = (int64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (c < n_chunks) pm_chunk_cross<DH>(one, c);
}
// one workgroup per pm.cross_wg walkers (from blockIdx.x cross_wg); dynamic
// LDS of cross_wg x T1 x C double2
template <bool DH>
__global__ __launch_bounds__(kBlock) void k_pm_cross_wg(WorkItem one) {
  extern __shared__ double2 pm_sd[];
  pm_walker_cross<DH>(one, (int64_t)blockIdx.x * one.pm.cross_wg, pm_sd);
}

}  // namespace mbh
