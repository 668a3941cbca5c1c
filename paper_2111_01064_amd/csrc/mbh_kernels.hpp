// mbh_kernels.hpp -- HIP kernels of libmbh (gfx950).
#pragma once

#include "mbh_device.hpp"

namespace mbh {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- reference
// Everything the heterodyned kernel needs about one reference, as device
// pointers.  coef is [C][Nb][6] FP64: Re/Im (A0-B0), Re/Im (A1-B1)/dF_b, B0,
// B1/dF_b, where dF_b = F_{b+1} - F_b.
struct HetRef {
  const double *F;      // [E] bin edges
  const double *psi0;   // [E] carrier phase of h0
  const double *is064;  // [C][E][2] 1/s0
  const double *coef;   // [C][Nb][6]
  double lnL0, dh0, hh0, t_obs;
  int32_t n_bins, n_chan;
  uint32_t modes;
  int32_t pad;
};

// ---------------------------------------------------------------- utilities
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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
static __global__ __launch_bounds__(128) void k_walker_setup(const double *__restrict__ theta, int64_t W, int model,
                                                             uint32_t modes, WalkerC *__restrict__ out) {
  int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  walker_setup(theta + w * 11, model, modes, out[w]);
}

// ---------------------------------------------------------------- data
// whitening: w = 4 df / S; dw = d sqrt(w); sw = sqrt(w) / kAmpScale.
// Per-block partial of <d|d> = sum |dw|^2.
static __global__ __launch_bounds__(kBlock) void k_whiten(const double *__restrict__ d, const double *__restrict__ psd,
                                                   int64_t n_total, double df, double2 *__restrict__ dw64,
                                                   double *__restrict__ sw64, float2 *__restrict__ dw32,
                                                   float *__restrict__ sw32, double *__restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * kBlock) {
    double w = 4.0 * df / psd[i];
    double s = sqrt(w);
    double re = d[2 * i] * s, im = d[2 * i + 1] * s;
    dw64[i] = make_double2(re, im);
    sw64[i] = s / kAmpScale;
    dw32[i] = make_float2((float)re, (float)im);
    sw32[i] = (float)(s / kAmpScale);
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
  bool any = template_point<double>(w, modes, f, t_obs, s, psi);
  double sp = 0.0, cp = 1.0;
  if (any) sincos(reduce_2pi(psi), &sp, &cp);
  for (int c = 0; c < n_chan; ++c) {
    cx<double> v = any ? s[c] * mk<double>(cp, -sp) : mk<double>(0.0, 0.0);
    h[c * n_f + k] = make_double2(v.re / kAmpScale, v.im / kAmpScale);
  }
}

// ---------------------------------------------------------------- a9: reference build
// pass 1: whitened h0 on the grid, band ends, and block partials of
// -2 lnL(h0) = sum |dw - h0w|^2, <d|h0>, <h0|h0>
static __global__ __launch_bounds__(kBlock) void k_ref_grid(const WalkerC *__restrict__ wc, uint32_t modes, int n_chan,
                                                     int64_t n_f, double f0, double df, double t_obs,
                                                     const double2 *__restrict__ dw, const double *__restrict__ sw,
                                                     double2 *__restrict__ h0w, unsigned long long *band,
                                                     double *__restrict__ part) {
  __shared__ double sh[3 * (kBlock / 64)];
  const WalkerC &w = wc[0];
  double a_res = 0.0, a_dh = 0.0, a_hh = 0.0;
  unsigned long long lo = ~0ull, hi = 0ull;
  bool seen = false;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_f; k += (int64_t)gridDim.x * kBlock) {
    double f = grid_freq(f0, df, k);
    cx<double> s[3];
    double psi;
    bool any = template_point<double>(w, modes, f, t_obs, s, psi);
    double sp = 0.0, cp = 1.0;
    if (any) sincos(reduce_2pi(psi), &sp, &cp);
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
                                                     const double2 *__restrict__ h0w, double *__restrict__ part) {
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

// sum the chunks of each bin in a fixed order: part [Nb][n_sub][18] -> out [Nb][18]
static __global__ void k_sum_bins(const double *__restrict__ part, int n_sub, double *__restrict__ out) {
  const int b = blockIdx.x;
  for (int i = threadIdx.x; i < 18; i += blockDim.x) {
    double s = 0.0;
    for (int sub = 0; sub < n_sub; ++sub) s += part[((int64_t)b * n_sub + sub) * 18 + i];
    out[(int64_t)b * 18 + i] = s;
  }
}

// pass 3: carrier phase and small factors of h0 at the edges
static __global__ __launch_bounds__(64) void k_ref_edges(const WalkerC *__restrict__ wc, uint32_t modes, int n_chan, int E,
                            const double *__restrict__ F, double t_obs, double *__restrict__ psi0,
                            double2 *__restrict__ s0) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= E) return;
  cx<double> s[3];
  double psi;
  bool any = template_point<double>(wc[0], modes, F[j], t_obs, s, psi);
  psi0[j] = psi;
  for (int c = 0; c < n_chan; ++c) s0[c * E + j] = any ? make_double2(s[c].re, s[c].im) : make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------- a2-a7: heterodyned
// FP64 recomputation queue of the mixed path.  The FP32 response leaves a
// per-edge relative error of ~1e-7 on r - 1; its effect on lnL is estimated
// per walker as kMixedErrScale * sqrt(S / 2), S = sum over bins and channels
// of |dT/d delta_0|^2 + 4 |dT/d delta_1|^2 (the gradient of the bin term
// with respect to the edge values).  kMixedErrScale bounds the measured ratio
// |lnL_mixed - lnL_fp64| / sqrt(S / 2) over tempered walker clouds at SNR
// 100-1000; walkers whose estimate exceeds kMixedRouteTol are queued and
// recomputed in FP64, so the mixed result stays within 1e-3 of FP64.
constexpr double kMixedErrScale = 6e-7;
constexpr double kMixedRouteTol = 5e-4;

struct RouteQ {
  unsigned int *count;  // entries queued by the mixed pass (null: no routing)
  int2 *list;           // (item, walker)
  int item;
};

// One lane group of G lanes per walker; lane gl evaluates edges gl, gl+G, ...
// The right neighbour edge of each bin comes from lane gl+1 (rotate within
// the group); the last lane's bin closes one iteration later with lane 0's
// next edge.  Bin terms accumulate in FP64 and are summed over the group with
// a fixed butterfly, so a walker's result depends only on its inputs and G.
template <typename R, int G, bool DH>
__device__ __forceinline__ void het_walker(const HetRef &ref, const WalkerC *__restrict__ wc, int64_t w,
                                           int64_t W, double *__restrict__ lnL, double *__restrict__ dhhh,
                                           RouteQ rq) {
  constexpr bool EST = sizeof(R) == 4;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  // with one walker per wavefront the walker index is wave-uniform: say so,
  // so that the walker constants live in scalar registers
  if constexpr (G == 64) w = (int64_t)__builtin_amdgcn_readfirstlane((int)w);
  const bool active = w < W;
  const WalkerC &c = wc[active ? w : 0];
  const bool valid = active && c.valid;
  const int Nb = ref.n_bins, E = Nb + 1, C = ref.n_chan;
  const int n_iter = (E + G - 1) / G;
  double acc = 0.0, a_dh = 0.0, a_hh = 0.0, a_s = 0.0;
  cx<double> dprev[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) dprev[ch] = mk<double>(0.0, 0.0);
  const int src = (lane & ~(G - 1)) | ((gl + 1) & (G - 1));

  for (int it = 0; it < n_iter; ++it) {
    const int j = it * G + gl;
    cx<double> dl[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) dl[ch] = mk<double>(0.0, 0.0);
    if (valid && j < E) {
      cx<double> s[3];
      double psi;
      template_point<R>(c, ref.modes, ref.F[j], ref.t_obs, s, psi);
      double dpsi = reduce_2pi(psi - ref.psi0[j]);
      R hs_r, hc_r;
      Prec<R>::sincos_r((R)(0.5 * dpsi), hs_r, hc_r);
      const double hs = hs_r, hc = hc_r;
      // e^{-i dpsi} - 1 = -2 sin^2(dpsi/2) - i sin(dpsi)
      cx<double> em1 = mk<double>(-2.0 * hs * hs, -2.0 * hs * hc);
      cx<double> e = mk<double>(1.0 + em1.re, em1.im);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        if (ch >= C) break;
        cx<double> is0 = mk<double>(ref.is064[2 * (ch * E + j)], ref.is064[2 * (ch * E + j) + 1]);
        cx<double> q = s[ch] * is0;
        q.re -= 1.0;
        dl[ch] = q * e + em1;  // r - 1 without cancellation
      }
    }
    cx<double> nb[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      nb[ch].re = __shfl(dl[ch].re, src, 64);
      nb[ch].im = __shfl(dl[ch].im, src, 64);
    }
    int b;
    cx<double> Lft[3];
    if (gl < G - 1) {
      b = j;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) Lft[ch] = dl[ch];
    } else {
      b = it * G - 1;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) Lft[ch] = dprev[ch];
    }
    if (valid && b >= 0 && b < Nb) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        if (ch >= C) break;
        const double *k = ref.coef + ((int64_t)ch * Nb + b) * 6;
        // delta_0 at the bin centre and the edge difference delta_1 dF_b, in FP64
        double d0r = 0.5 * (Lft[ch].re + nb[ch].re);
        double d0i = 0.5 * (Lft[ch].im + nb[ch].im);
        double d1r = nb[ch].re - Lft[ch].re;
        double d1i = nb[ch].im - Lft[ch].im;
        double re_a = k[0] * d0r + k[1] * d0i + k[2] * d1r + k[3] * d1i;
        double m0 = d0r * d0r + d0i * d0i;
        double x01 = d0r * d1r + d0i * d1i;
        acc += 4.0 * re_a - 2.0 * (k[4] * m0 + 2.0 * k[5] * x01);
        if constexpr (EST) {
          // gradient of the bin term (without its factor 4)
          double g0r = k[0] - k[4] * d0r - k[5] * d1r, g0i = k[1] - k[4] * d0i - k[5] * d1i;
          double g1r = k[2] - k[5] * d0r, g1i = k[3] - k[5] * d0i;
          a_s += g0r * g0r + g0i * g0i + 4.0 * (g1r * g1r + g1i * g1i);
        }
        if constexpr (DH) {
          // Z[d,h] - <d|h0> = 4 Re[A0 conj(d0) + A1 conj(d1)], A = (A - B) + B
          a_dh += 4.0 * (re_a + k[4] * d0r + k[5] * d1r);
          // Z[h,h] - <h0|h0> = 4 {B0 (2 Re d0 + |d0|^2) + 2 B1 (Re d1 + Re d0 conj d1)}
          a_hh += 4.0 * (k[4] * (2.0 * d0r + m0) + 2.0 * k[5] * (d1r + x01));
        }
      }
    }
    if (gl == G - 1) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) dprev[ch] = dl[ch];
    }
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    acc += __shfl_xor(acc, off, 64);
    if constexpr (EST) a_s += __shfl_xor(a_s, off, 64);
    if constexpr (DH) {
      a_dh += __shfl_xor(a_dh, off, 64);
      a_hh += __shfl_xor(a_hh, off, 64);
    }
  }
  if constexpr (EST) {
    // S carries the bin-term gradient without its factor 4: sqrt(S_true / 2) = sqrt(8 S)
    if (valid && rq.count && kMixedErrScale * sqrt(8.0 * a_s) > kMixedRouteTol) {
      if (gl == 0) {
        unsigned int slot = atomicAdd(rq.count, 1u);
        rq.list[slot] = make_int2(rq.item, (int)w);
      }
      return;  // the FP64 recomputation writes this walker's outputs
    }
  }
  if (active && gl == 0) {
    lnL[w] = valid ? ref.lnL0 + acc : -INFINITY;
    if constexpr (DH) {
      if (dhhh) {
        dhhh[2 * w] = valid ? ref.dh0 + a_dh : 0.0;
        dhhh[2 * w + 1] = valid ? ref.hh0 + a_hh : 0.0;
      }
    }
  }
}

template <typename R, int G, bool DH>
__global__ __launch_bounds__(kBlock) void k_het(HetRef ref, const WalkerC *__restrict__ wc, int64_t W,
                                                double *__restrict__ lnL, double *__restrict__ dhhh, RouteQ rq) {
  const int64_t w = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G;
  het_walker<R, G, DH>(ref, wc, w, W, lnL, dhhh, rq);
}

static __global__ void k_zero_u32(unsigned int *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- a8: full grid
// Block (fc, wc): KF grid frequencies per thread kept in registers, then a
// loop over the block's walkers (wave-uniform constants); per walker and
// block one FP64 partial of sum |dw - hw|^2 (and <d|h>, <h|h>).
// part layout [NV][n_fchunks][W].
template <typename R>
struct DataPtrs;
template <>
struct DataPtrs<double> {
  using R2 = double2;
};
template <>
struct DataPtrs<float> {
  using R2 = float2;
};

template <typename R, int KF, bool DH>
__global__ __launch_bounds__(kBlock) void k_full(const typename DataPtrs<R>::R2 *__restrict__ dw,
                                                 const R *__restrict__ sw, int n_chan, int64_t n_f, double f0,
                                                 double df, double t_obs, uint32_t modes,
                                                 const WalkerC *__restrict__ wc, int64_t W, int w_per_block,
                                                 double *__restrict__ part) {
  using R2 = typename DataPtrs<R>::R2;
  constexpr int NV = DH ? 3 : 1;
  __shared__ double sh[NV * (kBlock / 64)];
  const int64_t n_fc = gridDim.x;
  R2 d[KF][3];
  R s_w[KF][3];
  double fq[KF];
  bool inr[KF];
#pragma unroll
  for (int i = 0; i < KF; ++i) {
    int64_t k = (int64_t)blockIdx.x * (kBlock * KF) + i * kBlock + threadIdx.x;
    inr[i] = k < n_f;
    fq[i] = grid_freq(f0, df, inr[i] ? k : 0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < n_chan && inr[i]) {
        d[i][c] = dw[c * n_f + k];
        s_w[i][c] = sw[c * n_f + k];
      } else {
        d[i][c].x = d[i][c].y = (R)0;
        s_w[i][c] = (R)0;
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
        bool any = template_point<R>(c, modes, fq[i], t_obs, s, psi);
        R sp = (R)0, cp = (R)1;
        if (any) Prec<R>::sincos_r((R)reduce_2pi(psi), sp, cp);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          if (ch >= n_chan) break;
          cx<R> sr = mk<R>((R)s[ch].re, (R)s[ch].im);
          cx<R> h = any ? sr * mk<R>(cp, -sp) : mk<R>((R)0, (R)0);
          h = s_w[i][ch] * h;
          R rr = d[i][ch].x - h.re, ri = d[i][ch].y - h.im;
          v[0] += (double)(rr * rr + ri * ri);
          if constexpr (DH) {
            v[1] += (double)(d[i][ch].x * h.re + d[i][ch].y * h.im);
            v[2] += (double)(h.re * h.re + h.im * h.im);
          }
        }
      }
    }
    block_sum<NV>(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < NV; ++i) part[((int64_t)i * n_fc + blockIdx.x) * W + w] = v[i];
  }
}

// one wavefront per walker: lanes stride over the frequency chunks, fixed butterfly
static __global__ __launch_bounds__(kBlock) void k_full_reduce(const double *__restrict__ part, int n_fc, int64_t W,
                                                               int nv, const WalkerC *__restrict__ wc,
                                                               double *__restrict__ lnL, double *__restrict__ dhhh) {
  const int64_t w = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  if (w >= W) return;
  const int lane = threadIdx.x & 63;
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < nv; ++i) {
    for (int fc = lane; fc < n_fc; fc += 64) s[i] += part[((int64_t)i * n_fc + fc) * W + w];
    s[i] = wave_sum(s[i]);
  }
  if (lane != 0) return;
  bool ok = wc[w].valid;
  lnL[w] = ok ? -0.5 * s[0] : -INFINITY;
  if (dhhh) {
    dhhh[2 * w] = ok ? s[1] : 0.0;
    dhhh[2 * w + 1] = ok ? s[2] : 0.0;
  }
}

}  // namespace mbh
