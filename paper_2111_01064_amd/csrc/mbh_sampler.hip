// mbh_sampler.hip -- tempered ensemble sampler on the device (Sec. 3 of the
// paper: an affine-invariant ensemble with parallel tempering, ~85 % stretch
// proposals and three kinds of sky-mode hops; the extracted-SNR stopping rule
// of the first search and the maximum-likelihood convergence rule of the
// heterodyned search; the reference moved to the best walker every few
// thousand iterations).  Walkers, proposals and decisions stay in HBM.  With
// the heterodyned likelihood a half step is the sampler's batch's main pass
// between two kernels of the sampler's own (proposals fused with the batch's
// walker setup, the batch's totals fused with the decisions); with the full
// grid it is a full-grid call; a sampler can also send its proposals to a
// request server as one of its clients.  The exchanges between rungs are one
// kernel over all walkers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "mbh.h"
#include "mbh_internal.hpp"

using namespace mbh;

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return mbh_fail(MBH_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)
#define MBH_TRY(x)               \
  do {                           \
    mbh_status s_ = (x);         \
    if (s_ != MBH_OK) return s_; \
  } while (0)

namespace {

constexpr int kDim = 11;
// streams of the random counter's third word
constexpr uint32_t kStreamMove = 1, kStreamSwap = 2;
enum { kStretch = 0, kSkyAll = 1, kSkyLon = 2, kSkyLat = 3 };

// Philox4x32 with ten rounds (Salmon, Moraes, Dror & Shaw, SC 2011): each
// round takes the 32x32 -> 64-bit products of words 0 and 2 with the round
// multipliers, and the new words are (hi1 ^ w1 ^ k0, lo1, hi0 ^ w3 ^ k1, lo0);
// the key advances by the Weyl increments between rounds.
struct U4 {
  double u[4];
};
__device__ __forceinline__ U4 philox_uniforms(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t w0 = c0, w1 = c1, w2 = c2, w3 = c3;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * w0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * w2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ w1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ w3 ^ k1;
    w1 = (uint32_t)p1;
    w3 = (uint32_t)p0;
    w0 = n0;
    w2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  // (w + 1/2) / 2^32: exact in FP64, strictly inside (0, 1)
  U4 o;
  o.u[0] = ((double)w0 + 0.5) * 2.3283064365386962890625e-10;
  o.u[1] = ((double)w1 + 0.5) * 2.3283064365386962890625e-10;
  o.u[2] = ((double)w2 + 0.5) * 2.3283064365386962890625e-10;
  o.u[3] = ((double)w3 + 0.5) * 2.3283064365386962890625e-10;
  return o;
}

// sampling coordinates x = (ln M_T, q, a1, a2, D_L, phi_ref, cos iota,
// lambda, sin beta, psi, t_ref) -> the likelihood's theta
__device__ __forceinline__ void x_to_theta(const double *x, double *th) {
  for (int i = 0; i < kDim; ++i) th[i] = x[i];
  th[0] = exp(x[0]);
  th[6] = acos(fmin(fmax(x[6], -1.0), 1.0));
  th[8] = asin(fmin(fmax(x[8], -1.0), 1.0));
}

struct SmpParams {
  int32_t K, W;
  double a, p_all, p_lon, p_lat;
  uint64_t seed;
  const double *lo, *hi, *betas;
};

// Proposal t of one half (walker half * W/2 + t mod W/2 of rung t div W/2):
// the move kind, then a stretch from a partner of the other half or a
// sky-mode hop.  Roundings as written (no contraction), so that the proposals
// follow the operations of their definition exactly.  The proposal's theta
// also goes to th_out when it is given.
__device__ __forceinline__ void smp_propose_one(const SmpParams &p, int half, uint32_t it, int t,
                                                const double *__restrict__ x, double *__restrict__ y,
                                                double *__restrict__ thy, int32_t *__restrict__ kind,
                                                double *__restrict__ lz, double *th_out) {
  const int H = p.W / 2;
  const int k = t / H, i = t - k * H, w = half * H + i;
  const U4 u = philox_uniforms(p.seed, it, (uint32_t)(k * p.W + w), kStreamMove, (uint32_t)half);
  int kd = kStretch;
  if (u.u[0] < p.p_all) kd = kSkyAll;
  else if (u.u[0] < __dadd_rn(p.p_all, p.p_lon)) kd = kSkyLon;
  else if (u.u[0] < __dadd_rn(__dadd_rn(p.p_all, p.p_lon), p.p_lat)) kd = kSkyLat;
  const double *xi = x + ((int64_t)k * p.W + w) * kDim;
  double yv[kDim];
  double l = 0.0;
  if (kd == kStretch) {
    const int j = (1 - half) * H + min((int)floor(__dmul_rn(u.u[1], (double)H)), H - 1);
    const double *xj = x + ((int64_t)k * p.W + j) * kDim;
    const double s = __dadd_rn(__dmul_rn(__dadd_rn(p.a, -1.0), u.u[2]), 1.0);
    const double z = __ddiv_rn(__dmul_rn(s, s), p.a);
    for (int d = 0; d < kDim; ++d) yv[d] = __dadd_rn(xj[d], __dmul_rn(z, __dadd_rn(xi[d], -xj[d])));
    l = (kDim - 1) * log(z);
  } else {
    for (int d = 0; d < kDim; ++d) yv[d] = xi[d];
    constexpr double kPiD = 3.1415926535897931159979634685441852;     // nearest double to pi
    if (kd == kSkyAll || kd == kSkyLon) {
      const double q = fmin(floor(__dmul_rn(4.0, u.u[1])), 3.0);
      const double turn = __dmul_rn(__dmul_rn(q, 0.5), kPiD);
      yv[7] = fmod(__dadd_rn(yv[7], turn), __dmul_rn(2.0, kPiD));
      yv[9] = fmod(__dadd_rn(yv[9], turn), kPiD);
    }
    if (kd == kSkyLat || (kd == kSkyAll && u.u[2] < 0.5)) {
      yv[8] = -yv[8];
      yv[6] = -yv[6];
      yv[9] = __dadd_rn(kPiD, -yv[9]);
    }
  }
  bool in = true;
  for (int d = 0; d < kDim; ++d) in = in && yv[d] >= p.lo[d] && yv[d] <= p.hi[d];
  double *yo = y + (int64_t)t * kDim;
  double *to = thy + (int64_t)t * kDim;
  for (int d = 0; d < kDim; ++d) yo[d] = yv[d];
  double th[kDim];
  x_to_theta(yv, th);
  if (!in) th[0] = NAN;  // outside the prior: the likelihood returns -inf, the walker stays
  for (int d = 0; d < kDim; ++d) to[d] = th[d];
  if (th_out)
    for (int d = 0; d < kDim; ++d) th_out[d] = th[d];
  kind[t] = kd;
  lz[t] = l;
}

// the proposals of one half, one thread per (rung, walker)
__global__ __launch_bounds__(256) void k_smp_propose(SmpParams p, int half, uint32_t it, const double *__restrict__ x,
                                                     double *__restrict__ y, double *__restrict__ thy,
                                                     int32_t *__restrict__ kind, double *__restrict__ lz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < p.K * (p.W / 2)) smp_propose_one(p, half, it, t, x, y, thy, kind, lz, nullptr);
}

// Metropolis decision of proposal t of one half: accept when
// ln v < ln z^(d-1) + beta (lnL_y - lnL) inside the prior with a finite lnL_y
// (a walker whose lnL is not finite takes any such proposal); an accepted
// proposal replaces the walker, its lnL and overlaps.  The decision's inputs
// other than lnL_y are read first (smp_accept_in), so that a caller can have
// them in flight while it forms lnL_y.
struct AcceptIn {
  double yv[kDim];
  double cur, lzt, logu;
  int64_t o;
  int k, kd;
  bool in;
};
__device__ __forceinline__ AcceptIn smp_accept_in(const SmpParams &p, int half, uint32_t it, int t,
                                                  const double *__restrict__ y, const int32_t *__restrict__ kind,
                                                  const double *__restrict__ lz, const double *__restrict__ lnL) {
  AcceptIn a;
  const int H = p.W / 2;
  a.k = t / H;
  const int i = t - a.k * H, w = half * H + i;
  const U4 v = philox_uniforms(p.seed, it, (uint32_t)(a.k * p.W + w), kStreamMove, (uint32_t)(half + 2));
  const double *yv = y + (int64_t)t * kDim;
  a.in = true;
  for (int d = 0; d < kDim; ++d) {
    a.yv[d] = yv[d];
    a.in = a.in && yv[d] >= p.lo[d] && yv[d] <= p.hi[d];
  }
  a.o = (int64_t)a.k * p.W + w;
  a.cur = lnL[a.o];
  a.lzt = lz[t];
  a.kd = kind[t];
  a.logu = log(v.u[0]);
  return a;
}
// Returns 2 (4 k + kind) + 1 when the proposal was accepted, 2 (4 k + kind)
// if not.
__device__ __forceinline__ int smp_accept_apply(const SmpParams &p, const AcceptIn &a, double ly, double dh,
                                                double hh, bool has_dh, double *__restrict__ x,
                                                double *__restrict__ lnL, double *__restrict__ dhhh) {
  bool acc = false;
  if (a.in && isfinite(ly)) {
    const double la = isfinite(a.cur) ? __dadd_rn(a.lzt, __dmul_rn(p.betas[a.k], __dadd_rn(ly, -a.cur))) : INFINITY;
    acc = a.logu < la;
  }
  const int c = 2 * (a.k * 4 + a.kd);
  if (!acc) return c;
  for (int d = 0; d < kDim; ++d) x[a.o * kDim + d] = a.yv[d];
  lnL[a.o] = ly;
  if (has_dh) {
    dhhh[2 * a.o] = dh;
    dhhh[2 * a.o + 1] = hh;
  }
  return c + 1;
}

// The acceptance counters (accepted, proposed) per rung and move kind, K x 4
// pairs: each workgroup counts in LDS, then adds its nonzero counts.
constexpr int kMaxCounters = 64 * 4;
__device__ __forceinline__ void smp_count(unsigned *cnt, int code) {
  // proposed in the high half, accepted in the low half: one LDS atomic
  if (code >= 0) atomicAdd(&cnt[code >> 1], (1u << 16) + (unsigned)(code & 1));
}
__device__ __forceinline__ void smp_count_flush(const unsigned *cnt, int n_cnt, unsigned long long *counts) {
  for (int c = threadIdx.x; c < n_cnt; c += blockDim.x) {
    const unsigned v = cnt[c];
    if (v & 0xFFFFu) atomicAdd(&counts[2 * c], (unsigned long long)(v & 0xFFFFu));
    if (v >> 16) atomicAdd(&counts[2 * c + 1], (unsigned long long)(v >> 16));
  }
}

// the decisions of one half from the proposals' lnL (and overlaps) in lny, dhy
__global__ __launch_bounds__(256) void k_smp_accept(SmpParams p, int half, uint32_t it, const double *__restrict__ y,
                                                    const int32_t *__restrict__ kind, const double *__restrict__ lz,
                                                    const double *__restrict__ lny, const double *__restrict__ dhy,
                                                    double *__restrict__ x, double *__restrict__ lnL,
                                                    double *__restrict__ dhhh, unsigned long long *__restrict__ counts) {
  __shared__ unsigned cnt[kMaxCounters];
  const int n_cnt = p.K * 4;
  for (int c = threadIdx.x; c < n_cnt; c += blockDim.x) cnt[c] = 0u;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < p.K * (p.W / 2)) {
    const AcceptIn a = smp_accept_in(p, half, it, t, y, kind, lz, lnL);
    smp_count(cnt, smp_accept_apply(p, a, lny[t], dhy ? dhy[2 * t] : 0.0, dhy ? dhy[2 * t + 1] : 0.0,
                                    dhy != nullptr, x, lnL, dhhh));
  }
  __syncthreads();
  smp_count_flush(cnt, n_cnt, counts);
}

// A sampler step with the heterodyned likelihood runs the half batch's main
// pass between two kernels of its own, each fused with the batch stage next
// to it (so a half step is three launches, not five):
//  * proposals and the batch's walker constants: 64 proposals per workgroup
//    of 128 threads; the first 64 threads propose (their theta kept in LDS),
//    then the two threads of each proposal set its intrinsic and extrinsic
//    constants in the batch item that holds it.
//  * totals and decisions: one thread per proposal reads the decision's
//    inputs, adds its partial sums (as the batch's totals stage, writing the
//    item's outputs) and takes the Metropolis decision.
// items[0] holds proposals 0 .. n0-1, items[1] the rest; the first nb0
// workgroups take items[0]'s proposals, the others items[1]'s, so that a
// workgroup's item is uniform.  Proposals, constants, totals and decisions
// are those of the separate kernels bit for bit.
__global__ __launch_bounds__(128) void k_smp_propose_setup(SmpParams p, int half, uint32_t it,
                                                           const double *__restrict__ x, double *__restrict__ y,
                                                           double *__restrict__ thy, int32_t *__restrict__ kind,
                                                           double *__restrict__ lz, const WorkItem *__restrict__ items,
                                                           int n0, int nb0) {
  __shared__ double th_s[64][kDim];
  const int nh = p.K * (p.W / 2);
  const int j = threadIdx.x & 63;
  const bool second = (int)blockIdx.x >= nb0;
  const int t0 = second ? n0 + ((int)blockIdx.x - nb0) * 64 : (int)blockIdx.x * 64;
  const int t = t0 + j, t_end = second ? nh : n0;
  const WorkItem &itm = items[second ? 1 : 0];
  const int model = itm.model;
  const uint32_t modes = itm.ref.modes;
  WalkerC *wc = itm.wc;
  if (threadIdx.x < 64 && t < t_end) smp_propose_one(p, half, it, t, x, y, thy, kind, lz, th_s[j]);
  __syncthreads();
  if (t < t_end) walker_setup(th_s[j], model, modes, wc[second ? t - n0 : t], threadIdx.x < 64 ? 1 : 2);
}

__global__ __launch_bounds__(256) void k_smp_final_accept(SmpParams p, int half, uint32_t it,
                                                          const WorkItem *__restrict__ items, int n0, int nb0,
                                                          const double *__restrict__ y,
                                                          const int32_t *__restrict__ kind,
                                                          const double *__restrict__ lz, double *__restrict__ x,
                                                          double *__restrict__ lnL, double *__restrict__ dhhh,
                                                          unsigned long long *__restrict__ counts) {
  __shared__ unsigned cnt[kMaxCounters];
  const int n_cnt = p.K * 4;
  for (int c = threadIdx.x; c < n_cnt; c += blockDim.x) cnt[c] = 0u;
  __syncthreads();
  const bool second = (int)blockIdx.x >= nb0;
  const int t = (second ? n0 + ((int)blockIdx.x - nb0) * 256 : (int)blockIdx.x * 256) + (int)threadIdx.x;
  if (t < (second ? p.K * (p.W / 2) : n0)) {
    const AcceptIn a = smp_accept_in(p, half, it, t, y, kind, lz, lnL);
    const WorkItem &itm = items[second ? 1 : 0];
    const WalkerTotals r = het_walker_totals(itm, second ? t - n0 : t);
    smp_count(cnt, smp_accept_apply(p, a, r.lnL, r.dh, r.hh, itm.dhhh != nullptr, x, lnL, dhhh));
  }
  __syncthreads();
  smp_count_flush(cnt, n_cnt, counts);
}

// Exchanges between adjacent rungs: pairs k = 0, 1, ... in turn, walker i of
// rung k with walker (i + s_k) mod W of rung k + 1 (s_k uniform per pair),
// accepted when ln v < (beta_k - beta_k+1)(lnL_k+1 - lnL_k) with v uniform
// per (pair, walker i).  The slots p_0 = c, p_k+1 = (p_k + s_k) mod W of
// rungs 0 .. K-1 form chain c, and every pair of an iteration joins two slots
// of one chain: the W chains are independent, so each is one thread's loop
// over the pairs, with the walker that moves up the chain carried along (the
// decisions and their order are those of the pairs taken in turn over all
// walkers).  A workgroup of kExchThreads threads takes T chains (T <= 64, so
// that the deciding threads are one wavefront): the shifts are drawn, the
// chains' slots found, then all threads load the chains' lnL, <d|h>, <h|h>
// and x into LDS (one round of memory reads) and draw their ln v; the T
// deciding threads take the decisions (counted per pair by a ballot); then all
// threads write every slot of the chains from LDS: lnL and the overlaps in
// place, x into x_out.  Dynamic LDS: K (two doubles and an int) + K T (15
// doubles, an int and a byte).
constexpr int kExchThreads = 1024;
__global__ __launch_bounds__(kExchThreads) void k_smp_exchange(SmpParams p, uint32_t it, int T,
                                                               const double *__restrict__ x_in,
                                                               double *__restrict__ x_out, double *__restrict__ lnL,
                                                               double *__restrict__ dhhh,
                                                               unsigned long long *__restrict__ swaps) {
  extern __shared__ double smem[];
  const int K = p.K, W = p.W, tid = threadIdx.x, nt = blockDim.x;
  const int c0 = blockIdx.x * T;            // first chain of the workgroup
  const int Tc = min(T, W - c0);            // chains it holds
  const int KT = K * T;
  double *DB = smem;                        // [K] beta_k - beta_k+1
  double *L = DB + K, *Dh = L + KT, *Hh = Dh + KT, *V = Hh + KT;  // [K][T]
  double *X = V + KT;                       // [K][T][11]
  int32_t *P = (int32_t *)(X + KT * kDim);  // [K][T] the chain's slot in rung k
  int32_t *SH = P + KT;                     // [K] shifts
  uint8_t *S = (uint8_t *)(SH + K);         // [K][T] rung whose walker ends in rung k
  for (int k = tid; k + 1 < K; k += nt) {
    const U4 us = philox_uniforms(p.seed, it, (uint32_t)k, kStreamSwap, 0u);
    SH[k] = min((int)floor(__dmul_rn(us.u[0], (double)W)), W - 1);
  }
  __syncthreads();
  if (tid < Tc) {
    int pk = c0 + tid;
    for (int k = 0; k < K; ++k) {
      P[k * T + tid] = pk;
      if (k + 1 < K) {
        pk += SH[k];
        if (pk >= W) pk -= W;
      }
    }
  }
  __syncthreads();
  for (int k = tid; k + 1 < K; k += nt) DB[k] = __dadd_rn(p.betas[k], -p.betas[k + 1]);
  for (int e = tid; e < KT; e += nt) {
    const int k = e / T, j = e - k * T;
    if (j >= Tc) continue;
    const int64_t slot = (int64_t)k * W + P[e];
    L[e] = lnL[slot];
    Dh[e] = dhhh[2 * slot];
    Hh[e] = dhhh[2 * slot + 1];
    double lv = 0.0;
    if (k + 1 < K) {
      const U4 v = philox_uniforms(p.seed, it, (uint32_t)(k * W + P[e]), kStreamSwap, 1u);
      lv = log(v.u[0]);
    }
    V[e] = lv;
  }
  for (int e = tid; e < KT * kDim; e += nt) {
    const int q = e / kDim, d = e - q * kDim, k = q / T, j = q - k * T;
    if (j >= Tc) continue;
    X[e] = x_in[((int64_t)k * W + P[q]) * kDim + d];
  }
  __syncthreads();
  if (tid < 64) {  // the deciding wavefront
    const bool active = tid < Tc;
    int carry = 0;  // the rung whose walker sits in rung k of the chain before pair k
    for (int k = 0; k + 1 < K; ++k) {
      bool sw = false;
      if (active) {
        const double a = L[carry * T + tid], b = L[(k + 1) * T + tid];
        const double la = __dmul_rn(DB[k], __dadd_rn(b, -a));
        sw = V[k * T + tid] < (isnan(la) ? -INFINITY : la);
        S[k * T + tid] = (uint8_t)(sw ? k + 1 : carry);
        if (!sw) carry = k + 1;
      }
      const unsigned long long m = __ballot(sw);
      if (tid == 0 && m) atomicAdd(&swaps[k], (unsigned long long)__popcll(m));
    }
    if (active) S[(K - 1) * T + tid] = (uint8_t)carry;
  }
  __syncthreads();
  for (int e = tid; e < KT; e += nt) {
    const int k = e / T, j = e - k * T;
    if (j >= Tc) continue;
    const int r = S[e];
    const int64_t slot = (int64_t)k * W + P[e];
    lnL[slot] = L[r * T + j];
    dhhh[2 * slot] = Dh[r * T + j];
    dhhh[2 * slot + 1] = Hh[r * T + j];
  }
  for (int e = tid; e < KT * kDim; e += nt) {
    const int q = e / kDim, d = e - q * kDim, k = q / T, j = q - k * T;
    if (j >= Tc) continue;
    x_out[((int64_t)k * W + P[q]) * kDim + d] = X[((int)S[q] * T + j) * kDim + d];
  }
}

// chains per workgroup of the exchange kernel: 64, or fewer so that its LDS
// stays within 64 KB (K <= 64 rungs)
size_t exchange_lds(int K, int T) {
  return (size_t)K * (sizeof(double) + sizeof(int32_t)) +
         (size_t)K * T * ((4 + kDim) * sizeof(double) + sizeof(int32_t) + 1);
}
int exchange_chains(int K) {
  int T = 64;
  while (T > 1 && exchange_lds(K, T) > 65536) T /= 2;
  return T;
}

// theta of every walker, and whether its x lies in the prior box
__global__ __launch_bounds__(256) void k_smp_theta(int n, const double *__restrict__ x, const double *__restrict__ lo,
                                                   const double *__restrict__ hi, double *__restrict__ th) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double tv[kDim];
  x_to_theta(x + (int64_t)t * kDim, tv);
  bool in = true;
  for (int d = 0; d < kDim; ++d) in = in && x[(int64_t)t * kDim + d] >= lo[d] && x[(int64_t)t * kDim + d] <= hi[d];
  if (!in) tv[0] = NAN;
  for (int d = 0; d < kDim; ++d) th[(int64_t)t * kDim + d] = tv[d];
}

}  // namespace

struct mbh_sampler {
  mbh_ctx *ctx = nullptr;
  CtxHold hold;
  mbh_sampler_config cfg{};
  int K = 0, W = 0, H = 0;
  SmpParams p{};
  double *lo = nullptr, *hi = nullptr, *betas = nullptr;
  double *x_alt = nullptr;        // [K W][11] the other buffer of the walkers (swapped with x)
  double *x = nullptr, *lnL = nullptr, *dhhh = nullptr, *th = nullptr;
  double *y = nullptr, *thy = nullptr, *lny = nullptr, *dhy = nullptr, *lz = nullptr;
  int32_t *kind = nullptr;
  unsigned long long *counts = nullptr, *swaps = nullptr;
  int64_t it = 0;
  std::vector<std::pair<void *, size_t>> allocs;
  // heterodyned likelihood: batches over a half ensemble's proposals and
  // over the whole population, for the reference they were made for
  const mbh_ref *bref = nullptr;
  mbh_batch *half_batch = nullptr, *all_batch = nullptr;
  int half_n0 = 0;  // proposals in the half batch's first item
  // pinned host staging of one half step's proposals and results for a
  // request server (allocated on first use): theta [K W/2][11], lnL, <d|h> <h|h>
  double *h_theta = nullptr, *h_lnl = nullptr, *h_dh = nullptr;
  // their device addresses (coherent pinned memory): the proposal kernel
  // writes theta there and the decision kernel reads lnL and the overlaps
  // there, so a served half step makes no runtime copies
  double *h_theta_d = nullptr, *h_lnl_d = nullptr, *h_dh_d = nullptr;
};

static void sampler_free(mbh_sampler *s) {
  for (double *h : {s->h_theta, s->h_lnl, s->h_dh})
    if (h) (void)hipHostFree(h);
  if (s->half_batch) mbh_batch_release(s->half_batch);
  if (s->all_batch) mbh_batch_release(s->all_batch);
  for (auto &a : s->allocs) ctx_free(s->ctx, a.first, a.second);
  delete s;
}

template <typename T>
static mbh_status smp_alloc(mbh_sampler *s, T **p, size_t n) {
  mbh_status e = ctx_alloc(s->ctx, (void **)p, std::max<size_t>(1, n) * sizeof(T));
  if (e == MBH_OK) s->allocs.emplace_back((void *)*p, std::max<size_t>(1, n) * sizeof(T));
  return e;
}

extern "C" mbh_status mbh_sampler_create(mbh_ctx *ctx, const mbh_sampler_config *cfg, const double *betas_host,
                                         const double *prior_lo_host, const double *prior_hi_host,
                                         mbh_sampler **out) {
  if (!ctx || !cfg || !betas_host || !prior_lo_host || !prior_hi_host || !out) return mbh_fail(MBH_EINVAL, "null argument");
  *out = nullptr;
  const int K = cfg->n_temps, W = cfg->walkers_per_temp;
  if (K < 1 || K > 64 || W < 4 || W % 2 || W > 65536) return mbh_fail(MBH_EINVAL, "n_temps in [1, 64], walkers even in [4, 65536]");
  if (cfg->mixed_rungs < 0) return mbh_fail(MBH_EINVAL, "mixed_rungs must be >= 0");
  if (!(cfg->stretch_a > 1.0) || cfg->p_sky_all < 0 || cfg->p_sky_lon < 0 || cfg->p_sky_lat < 0 ||
      cfg->p_sky_all + cfg->p_sky_lon + cfg->p_sky_lat > 1.0)
    return mbh_fail(MBH_EINVAL, "stretch a > 1 and sky-hop shares in [0, 1] summing to at most 1");
  if (cfg->prec != MBH_FP64 && cfg->prec != MBH_MIXED) return mbh_fail(MBH_EINVAL, "bad precision");
  if (betas_host[0] != 1.0) return mbh_fail(MBH_EINVAL, "betas[0] must be 1");
  for (int k = 1; k < K; ++k)
    if (!(betas_host[k] >= 0.0 && betas_host[k] < betas_host[k - 1]))
      return mbh_fail(MBH_EINVAL, "betas must decrease from 1 and stay >= 0");
  for (int d = 0; d < kDim; ++d)
    if (!(prior_lo_host[d] < prior_hi_host[d])) return mbh_fail(MBH_EINVAL, "prior box: lo < hi in every coordinate");
  HIP_TRY(hipSetDevice(ctx->device));
  mbh_sampler *s = new mbh_sampler();
  s->ctx = ctx;
  s->hold.set(ctx);
  s->cfg = *cfg;
  s->K = K;
  s->W = W;
  s->H = W / 2;
  const size_t n = (size_t)K * W, nh = (size_t)K * (W / 2);
  mbh_status e;
  if ((e = smp_alloc(s, &s->lo, kDim)) || (e = smp_alloc(s, &s->hi, kDim)) || (e = smp_alloc(s, &s->betas, K)) ||
      (e = smp_alloc(s, &s->x, n * kDim)) || (e = smp_alloc(s, &s->lnL, n)) || (e = smp_alloc(s, &s->dhhh, 2 * n)) ||
      (e = smp_alloc(s, &s->th, n * kDim)) || (e = smp_alloc(s, &s->y, nh * kDim)) ||
      (e = smp_alloc(s, &s->thy, nh * kDim)) || (e = smp_alloc(s, &s->lny, nh)) || (e = smp_alloc(s, &s->dhy, 2 * nh)) ||
      (e = smp_alloc(s, &s->lz, nh)) || (e = smp_alloc(s, &s->kind, nh)) || (e = smp_alloc(s, &s->counts, K * 8)) ||
      (e = smp_alloc(s, &s->swaps, K)) ||
      (e = smp_alloc(s, &s->x_alt, n * kDim))) {
    sampler_free(s);
    return e;
  }
  if (hipMemcpy(s->lo, prior_lo_host, kDim * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->hi, prior_hi_host, kDim * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->betas, betas_host, K * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(s->counts, 0, K * 8 * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(s->swaps, 0, K * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(s->dhhh, 0, 2 * n * sizeof(double)) != hipSuccess) {
    sampler_free(s);
    return mbh_fail(MBH_EDEVICE, "sampler upload");
  }
  s->p = SmpParams{K, W, cfg->stretch_a, cfg->p_sky_all, cfg->p_sky_lon, cfg->p_sky_lat, cfg->seed, s->lo, s->hi, s->betas};
  *out = s;
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_destroy(mbh_sampler *s) {
  if (!s) return MBH_OK;
  (void)hipSetDevice(s->ctx->device);
  (void)hipDeviceSynchronize();
  sampler_free(s);
  (void)hipGetLastError();
  return MBH_OK;
}

// batches over the half-ensemble proposals and over the population for the
// heterodyned likelihood of `ref` (made once per reference)
static mbh_status smp_batches(mbh_sampler *s, const mbh_ref *ref) {
  if (s->bref == ref && s->half_batch) return MBH_OK;
  if (s->half_batch) mbh_batch_release(s->half_batch);
  if (s->all_batch) mbh_batch_release(s->all_batch);
  s->half_batch = s->all_batch = nullptr;
  const mbh_precision prec = ref->pm ? MBH_FP64 : s->cfg.prec;
  // rungs [0, m) in prec and [m, K) in FP64: two items over the rung-major arrays
  const int m = (prec == MBH_MIXED && s->cfg.mixed_rungs > 0 && s->cfg.mixed_rungs < s->K) ? s->cfg.mixed_rungs
                                                                                          : s->K;
  const int n_items = m < s->K ? 2 : 1;
  const mbh_ref *r2[2] = {ref, ref};
  const mbh_precision p2[2] = {prec, MBH_FP64};
  for (int b = 0; b < 2; ++b) {
    const int64_t per = b == 0 ? s->H : s->W;  // walkers per rung in the half / whole batch
    double *thb = b == 0 ? s->thy : s->th, *lb = b == 0 ? s->lny : s->lnL, *db = b == 0 ? s->dhy : s->dhhh;
    const double *th[2] = {thb, thb + (int64_t)m * per * kDim};
    double *l[2] = {lb, lb + (int64_t)m * per};
    double *d[2] = {db, db + 2 * (int64_t)m * per};
    const int64_t W2[2] = {(int64_t)m * per, (int64_t)(s->K - m) * per};
    MBH_TRY(mbh_batch_create_prec(s->ctx, n_items, r2, th, W2, l, d, p2, b == 0 ? &s->half_batch : &s->all_batch));
  }
  s->half_n0 = m * s->H;
  s->bref = ref;
  return MBH_OK;
}

static mbh_status check_like(const mbh_sampler *s, const mbh_likelihood *like) {
  if (!like || (!like->ref && !like->data)) return mbh_fail(MBH_EINVAL, "likelihood: a reference or data");
  if (like->ref && (like->ref->ctx != s->ctx || like->ref->model != MBH_MODEL_IMR))
    return mbh_fail(MBH_EINVAL, "likelihood: an IMR reference of the sampler's context");
  if (!like->ref && like->data->n_chan != 3) return mbh_fail(MBH_EINVAL, "likelihood: three-channel data");
  return MBH_OK;
}

// lnL (and <d|h>, <h|h>) of n walkers th [n][11] into lnl, dh
static mbh_status smp_like(mbh_sampler *s, const mbh_likelihood *like, bool half, hipStream_t st) {
  if (like->ref) {
    MBH_TRY(smp_batches(s, like->ref));
    return mbh_batch_launch_direct(half ? s->half_batch : s->all_batch, st);
  }
  const int64_t n = half ? (int64_t)s->K * s->H : (int64_t)s->K * s->W;
  return mbh_loglike_full(s->ctx, like->data, MBH_MODEL_IMR, like->modes, half ? s->thy : s->th, n, s->cfg.prec,
                          half ? s->lny : s->lnL, half ? s->dhy : s->dhhh, st);
}

static mbh_status smp_eval_all(mbh_sampler *s, const mbh_likelihood *like, hipStream_t st) {
  const int n = s->K * s->W;
  hipLaunchKernelGGL(k_smp_theta, dim3((n + 255) / 256), dim3(256), 0, st, n, s->x, s->lo, s->hi, s->th);
  HIP_TRY(hipGetLastError());
  return smp_like(s, like, false, st);
}

extern "C" mbh_status mbh_sampler_set_walkers(mbh_sampler *s, const double *x_host, const double *lnL_host,
                                              const mbh_likelihood *like, hipStream_t st) {
  if (!s || !x_host) return mbh_fail(MBH_EINVAL, "null argument");
  if (!lnL_host) MBH_TRY(check_like(s, like));
  HIP_TRY(hipSetDevice(s->ctx->device));
  const size_t n = (size_t)s->K * s->W;
  HIP_TRY(hipMemcpyAsync(s->x, x_host, n * kDim * sizeof(double), hipMemcpyHostToDevice, st));
  if (!lnL_host) return smp_eval_all(s, like, st);
  HIP_TRY(hipMemcpyAsync(s->lnL, lnL_host, n * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(s->dhhh, 0, 2 * n * sizeof(double), st));
  HIP_TRY(hipStreamSynchronize(st));  // the host buffers may go once this returns
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_propose(mbh_sampler *s, int half, hipStream_t st) {
  if (!s || (half != 0 && half != 1)) return mbh_fail(MBH_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const int nh = s->K * s->H;
  hipLaunchKernelGGL(k_smp_propose, dim3((nh + 255) / 256), dim3(256), 0, st, s->p, half, (uint32_t)s->it, s->x, s->y,
                     s->thy, s->kind, s->lz);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_proposals(mbh_sampler *s, double *x_host, double *theta_host, int32_t *kind_host) {
  if (!s) return mbh_fail(MBH_EINVAL, "null sampler");
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  const size_t nh = (size_t)s->K * s->H;
  if (x_host) HIP_TRY(hipMemcpy(x_host, s->y, nh * kDim * sizeof(double), hipMemcpyDeviceToHost));
  if (theta_host) HIP_TRY(hipMemcpy(theta_host, s->thy, nh * kDim * sizeof(double), hipMemcpyDeviceToHost));
  if (kind_host) HIP_TRY(hipMemcpy(kind_host, s->kind, nh * sizeof(int32_t), hipMemcpyDeviceToHost));
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_accept(mbh_sampler *s, int half, const double *lnL_prop_dev,
                                         const double *dh_hh_prop_dev, hipStream_t st) {
  if (!s || (half != 0 && half != 1) || !lnL_prop_dev) return mbh_fail(MBH_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const int nh = s->K * s->H;
  hipLaunchKernelGGL(k_smp_accept, dim3((nh + 255) / 256), dim3(256), 0, st, s->p, half, (uint32_t)s->it, s->y,
                     s->kind, s->lz, lnL_prop_dev, dh_hh_prop_dev, s->x, s->lnL, s->dhhh, s->counts);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

// the exchanges of the iteration
static mbh_status smp_swap(mbh_sampler *s, hipStream_t st) {
  if (s->K > 1) {
    const int T = exchange_chains(s->K);
    hipLaunchKernelGGL(k_smp_exchange, dim3((s->W + T - 1) / T), dim3(kExchThreads), exchange_lds(s->K, T), st,
                       s->p, (uint32_t)s->it, T, s->x, s->x_alt, s->lnL, s->dhhh, s->swaps);
    std::swap(s->x, s->x_alt);
  }
  HIP_TRY(hipGetLastError());
  s->it += 1;
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_swap(mbh_sampler *s, hipStream_t st) {
  if (!s) return mbh_fail(MBH_EINVAL, "null sampler");
  HIP_TRY(hipSetDevice(s->ctx->device));
  return smp_swap(s, st);
}

// one half step with the heterodyned likelihood: proposals fused with the
// half batch's setup, its main pass, totals fused with the decisions
static mbh_status smp_half_het(mbh_sampler *s, const mbh_ref *ref, int half, hipStream_t st) {
  MBH_TRY(smp_batches(s, ref));
  const int nh = s->K * s->H;
  const WorkItem *items = batch_device_items(s->half_batch);
  const int n0 = s->half_n0, nb0 = (n0 + 63) / 64, nb1 = (nh - n0 + 63) / 64;
  hipLaunchKernelGGL(k_smp_propose_setup, dim3(nb0 + nb1), dim3(128), 0, st, s->p, half, (uint32_t)s->it, s->x, s->y,
                     s->thy, s->kind, s->lz, items, n0, nb0);
  MBH_TRY(mbh_batch_launch_stage(s->half_batch, MBH_STAGE_MAIN, st));
  const int fb0 = (n0 + 255) / 256, fb1 = (nh - n0 + 255) / 256;
  hipLaunchKernelGGL(k_smp_final_accept, dim3(fb0 + fb1), dim3(256), 0, st, s->p, half, (uint32_t)s->it, items, n0,
                     fb0, s->y, s->kind, s->lz, s->x, s->lnL, s->dhhh, s->counts);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_step(mbh_sampler *s, const mbh_likelihood *like, int64_t n_iter, hipStream_t st) {
  if (!s || n_iter < 0) return mbh_fail(MBH_EINVAL, "bad argument");
  MBH_TRY(check_like(s, like));
  HIP_TRY(hipSetDevice(s->ctx->device));
  for (int64_t i = 0; i < n_iter; ++i) {
    if (like->ref) {
      for (int half = 0; half < 2; ++half) MBH_TRY(smp_half_het(s, like->ref, half, st));
      MBH_TRY(smp_swap(s, st));
      continue;
    }
    for (int half = 0; half < 2; ++half) {
      MBH_TRY(mbh_sampler_propose(s, half, st));
      MBH_TRY(smp_like(s, like, true, st));
      MBH_TRY(mbh_sampler_accept(s, half, s->lny, s->dhy, st));
    }
    MBH_TRY(smp_swap(s, st));
  }
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_step_served(mbh_sampler *s, mbh_server *srv, int ref_index, int64_t n_iter,
                                              hipStream_t st, double *latency_s) {
  if (!s || !srv || n_iter < 0) return mbh_fail(MBH_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const int64_t nh = (int64_t)s->K * s->H;
  // staging allocated on first use (each buffer on its own, so a call after a
  // failed allocation tries again)
  if (!s->h_theta) HIP_TRY(hipHostMalloc((void **)&s->h_theta, nh * kDim * sizeof(double), hipHostMallocCoherent));
  if (!s->h_lnl) HIP_TRY(hipHostMalloc((void **)&s->h_lnl, nh * sizeof(double), hipHostMallocCoherent));
  if (!s->h_dh) HIP_TRY(hipHostMalloc((void **)&s->h_dh, 2 * nh * sizeof(double), hipHostMallocCoherent));
  HIP_TRY(hipHostGetDevicePointer((void **)&s->h_theta_d, s->h_theta, 0));
  HIP_TRY(hipHostGetDevicePointer((void **)&s->h_lnl_d, s->h_lnl, 0));
  HIP_TRY(hipHostGetDevicePointer((void **)&s->h_dh_d, s->h_dh, 0));
  const int blocks = (int)((nh + 255) / 256);
  for (int64_t i = 0; i < n_iter; ++i) {
    for (int half = 0; half < 2; ++half) {
      hipLaunchKernelGGL(k_smp_propose, dim3(blocks), dim3(256), 0, st, s->p, half, (uint32_t)s->it, s->x, s->y,
                         s->h_theta_d, s->kind, s->lz);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipStreamSynchronize(st));
      uint64_t id = 0;
      MBH_TRY(mbh_server_submit(srv, ref_index, s->h_theta, nh, &id));
      double lat = 0.0;
      MBH_TRY(mbh_server_wait(srv, id, -1, s->h_lnl, s->h_dh, nh, &lat));
      if (latency_s) latency_s[2 * i + half] = lat;
      MBH_TRY(mbh_sampler_accept(s, half, s->h_lnl_d, s->h_dh_d, st));
    }
    MBH_TRY(smp_swap(s, st));
  }
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_get(mbh_sampler *s, double *x_host, double *lnL_host, double *dh_hh_host,
                                      int64_t *iteration) {
  if (!s) return mbh_fail(MBH_EINVAL, "null sampler");
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  const size_t n = (size_t)s->K * s->W;
  if (x_host) HIP_TRY(hipMemcpy(x_host, s->x, n * kDim * sizeof(double), hipMemcpyDeviceToHost));
  if (lnL_host) HIP_TRY(hipMemcpy(lnL_host, s->lnL, n * sizeof(double), hipMemcpyDeviceToHost));
  if (dh_hh_host) HIP_TRY(hipMemcpy(dh_hh_host, s->dhhh, 2 * n * sizeof(double), hipMemcpyDeviceToHost));
  if (iteration) *iteration = s->it;
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_stats(mbh_sampler *s, uint64_t *accepted, uint64_t *proposed, uint64_t *swaps) {
  if (!s) return mbh_fail(MBH_EINVAL, "null sampler");
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  std::vector<unsigned long long> c((size_t)s->K * 8), sw((size_t)s->K);
  HIP_TRY(hipMemcpy(c.data(), s->counts, c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sw.data(), s->swaps, sw.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  for (int k = 0; k < s->K; ++k)
    for (int kd = 0; kd < 4; ++kd) {
      if (accepted) accepted[k * 4 + kd] = c[(k * 4 + kd) * 2];
      if (proposed) proposed[k * 4 + kd] = c[(k * 4 + kd) * 2 + 1];
    }
  if (swaps)
    for (int k = 0; k + 1 < s->K; ++k) swaps[k] = sw[k];
  return MBH_OK;
}

extern "C" mbh_status mbh_sampler_run(mbh_sampler *s, const mbh_likelihood *like, const mbh_sampler_stop *stop,
                                      hipStream_t st, mbh_sampler_report *rep) {
  if (!s || !stop || !rep) return mbh_fail(MBH_EINVAL, "null argument");
  MBH_TRY(check_like(s, like));
  if (stop->check_every < 1 || stop->max_iter < 0 || stop->lnl_checks < 0)
    return mbh_fail(MBH_EINVAL, "check_every >= 1, max_iter >= 0, lnl_checks >= 0");
  if (stop->refresh_every > 0 && (!like->ref || !stop->refresh_data))
    return mbh_fail(MBH_EINVAL, "reference updates need the heterodyned likelihood and its data");
  HIP_TRY(hipSetDevice(s->ctx->device));
  std::memset(rep, 0, sizeof(*rep));
  const auto t0 = std::chrono::steady_clock::now();
  const size_t n = (size_t)s->K * s->W;
  std::vector<double> lnl(n), dh(2 * n);
  double last_max = -INFINITY;
  int same = 0;
  int64_t done = 0;
  rep->reason = MBH_STOP_MAX_ITER;
  while (done < stop->max_iter) {
    const int64_t chunk = std::min<int64_t>(stop->check_every, stop->max_iter - done);
    for (int64_t i = 0; i < chunk; ++i) {
      MBH_TRY(mbh_sampler_step(s, like, 1, st));
      ++done;
      if (stop->refresh_every > 0 && s->it % stop->refresh_every == 0) {
        // Sec. 3.2: the best walker becomes the reference; every walker's lnL
        // is then re-evaluated against the new reference
        mbh_ref *r = const_cast<mbh_ref *>(like->ref);
        const int nn = (int)n;
        hipLaunchKernelGGL(k_smp_theta, dim3((nn + 255) / 256), dim3(256), 0, st, nn, s->x, s->lo, s->hi, s->th);
        MBH_TRY(mbh_ref_refresh(s->ctx, stop->refresh_data, r, s->th, s->lnL, (int64_t)n, st));
        MBH_TRY(smp_like(s, like, false, st));
        rep->refreshes += 1;
      }
    }
    // stopping checks on the cold rung's best walker (host copies of lnL and overlaps)
    HIP_TRY(hipMemcpyAsync(lnl.data(), s->lnL, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(dh.data(), s->dhhh, 2 * n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double mx = -INFINITY, snr = 0.0;
    for (int w = 0; w < s->W; ++w) {
      if (!(lnl[w] > mx)) continue;
      mx = lnl[w];
      snr = dh[2 * w + 1] > 0.0 ? dh[2 * w] / std::sqrt(dh[2 * w + 1]) : 0.0;
    }
    rep->max_lnL = mx;
    rep->best_snr = snr;
    rep->checks += 1;
    if (stop->snr_stop > 0.0 && snr >= stop->snr_stop) {
      rep->reason = MBH_STOP_SNR;
      break;
    }
    if (stop->lnl_checks > 0) {
      same = (std::isfinite(mx) && std::fabs(mx - last_max) < stop->lnl_tol) ? same + 1 : 0;
      last_max = mx;
      if (same >= stop->lnl_checks) {
        rep->reason = MBH_STOP_CONVERGED;
        break;
      }
    }
  }
  rep->iterations = done;
  rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return MBH_OK;
}
