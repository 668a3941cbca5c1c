// mbh_device.hpp -- device-side physics of libmbh (gfx950).
//
// Template of one walker at one frequency, split into a big FP64 "carrier"
// phase Psi and small per-channel complex factors s^c, so that
//     h^c(f) = s^c(f) * exp(-i Psi(f)).
// The carrier holds every phase that can exceed a few radians: the (2,2)
// phase phi_22(f) (Sec. 2.1 eq. amp_and_phase), the time shift 2 pi f t_ref,
// the guiding-centre Doppler 2 pi f k.p0(t_22(f)) and the common TDI arm
// phase 4 pi f L.  Everything in s^c is bounded by a few radians and is
// evaluated in the template precision R (double for the plain path, float for
// the mixed path).
//
// Waveform: "IMR-lite" (2,2) with 1PN + 1.5PN spin-orbit inspiral phase, a
// C1 arctan merger-ringdown continuation and f^(-7/6) x Lorentzian amplitude;
// reference frequency f_max = argmax f^2 A_22 (Sec. 2.1); higher modes
// phi_lm(f) = (m/2) phi_22(2f/m), t_lm(f) = t_22(2f/m) (eq. tf).
// Response: first-order cartwheel orbit, single-link Doppler transfer,
// first-generation TDI, A/E/T (Sec. 2.1).  The A/E/T combinations are written
// directly in terms of the symmetric (sigma) and antisymmetric (Delta) parts of
// the two directions of each arm; Delta is evaluated from a divided difference
// of the sinc series so that T (which vanishes to leading order at low
// frequency) keeps full relative precision in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbh {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kTwoPi = 6.283185307179586476925286766559005768;
constexpr double kInvTwoPi = 0.159154943091895335768883763372514362;
constexpr double kTwoPiHi = 6.283185307179586231995926937088;   // nearest double to 2 pi
constexpr double kTwoPiLo = 2.4492935982947063544521318e-16;     // 2 pi - kTwoPiHi
constexpr double kSqrt2 = 1.41421356237309504880168872420969808;
constexpr double kSqrt3 = 1.73205080756887729352744634150587237;
constexpr double kSqrt6 = 2.44948974278317809819728407470589139;
constexpr double kMsunS = 4.925490947641267e-6;
constexpr double kClight = 299792458.0;
constexpr double kGpcM = 3.0856775814913673e25;
constexpr double kAuM = 1.495978707e11;
constexpr double kYearS = 31557600.0;
constexpr double kArmS = 2.5e9 / kClight;          // L [s]
constexpr double kOrbR = kAuM / kClight;           // R [s]
constexpr double kEccR = kArmS / (2.0 * kSqrt3);   // e R [s]
constexpr double kKappa = -1.0;                    // merger-ringdown phase weight
// Templates carry a fixed power-of-two scale so that FP32 small factors and
// their reciprocals stay far from the FP32 range limits; the whitening
// weights are stored divided by the same scale.
constexpr double kAmpScale = 18446744073709551616.0;  // 2^64
constexpr double kMaxFreq = 0.1;                      // sinc series domain [Hz]

constexpr int kNumModes = 6;
// mode order (2,2) (3,3) (4,4) (2,1) (3,2) (4,3)
__device__ __constant__ const int kModeM[6] = {2, 3, 4, 1, 2, 3};
__device__ __constant__ const int kModeVPow[6] = {0, 1, 2, 1, 2, 3};

template <typename R>
struct cx {
  R re, im;
};
template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// multiply by -i
template <typename R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }

// x - 2 pi rint(x / 2 pi) with a two-constant split of 2 pi (Cody & Waite)
__device__ __forceinline__ double reduce_2pi(double x) {
  double k = rint(x * kInvTwoPi);
  return fma(-k, kTwoPiLo, fma(-k, kTwoPiHi, x));
}

// Per-walker constants, evaluated once in FP64 from theta.
struct WalkerC {
  int32_t valid, model, pad0, pad1;
  // IMR-lite (2,2)
  double piM;                 // pi M
  double c5, c3, c2;          // phi_raw = c5 v^-5 + c3 v^-3 + c2 v^-2
  double d5, d3, d2;          // f * dphi_raw/df = d5 v^-5 + d3 v^-3 + d2 v^-2
  double f1, fRD, fD, fcut, fmax;
  double P1, dP1, L1, at1;    // inspiral phase, slope at f1; Lorentzian, arctan at f1
  double ph_max, dph_max;     // raw phase and slope at f_max
  double AN;                  // amplitude prefactor (times kAmpScale)
  double lam_num;             // (f1 - fRD)^2 + fD^2
  double inv_fD;              // 1 / fD
  double tref;
  double rel[6];              // relative amplitude coefficient of each mode
  // sky: propagation direction and polarisation basis
  double kx, ky, kz, px, py, pz, qx, qy, qz;
  // polarisation content of each mode: K+ = e^{i m phi} kp, Kx = i e^{i m phi} kc
  double kp[6], kc[6], eph[6][2];
  // chirp model
  double piMc, amp, tc, phic;
};

__device__ __forceinline__ double sq(double x) { return x * x; }

// closed-form spin-weight -2 harmonics (real part at phi = 0) for the
// (l, +-m) pairs of the six modes, in terms of c = cos(iota), s = sin(iota)
// and ch, sh = cos, sin(iota/2)
__device__ inline void ylm_pair(int mi, double c, double s, double ch, double sh, double &yp, double &ym,
                                int &lsign) {
  const double r5_64pi = 0.15769578262626002;  // sqrt(5 / (64 pi))
  const double r5_16pi = 0.31539156525252005;  // sqrt(5 / (16 pi))
  const double r21_2pi = 1.8281831978578629;   // sqrt(21 / (2 pi))
  const double r7_pi = 1.4927053303604616;     // sqrt(7 / pi)
  const double r7_4pi = 0.7463526651802308;    // sqrt(7 / (4 pi))
  const double r7_2pi = 1.0555020614058327;    // sqrt(7 / (2 pi))
  double ch2 = ch * ch, sh2 = sh * sh;
  switch (mi) {
    case 0:  // (2, +-2)
      yp = r5_64pi * (1 + c) * (1 + c);
      ym = r5_64pi * (1 - c) * (1 - c);
      lsign = 1;
      break;
    case 1:  // (3, +-3)
      yp = -r21_2pi * ch2 * ch2 * ch * sh;
      ym = r21_2pi * ch * sh2 * sh2 * sh;
      lsign = -1;
      break;
    case 2:  // (4, +-4)
      yp = 3.0 * r7_pi * ch2 * ch2 * ch2 * sh2;
      ym = 3.0 * r7_pi * ch2 * sh2 * sh2 * sh2;
      lsign = 1;
      break;
    case 3:  // (2, +-1)
      yp = r5_16pi * s * (1 + c);
      ym = r5_16pi * s * (1 - c);
      lsign = 1;
      break;
    case 4:  // (3, +-2)
      yp = 0.5 * r7_pi * ch2 * ch2 * (3 * c - 2);
      ym = r7_4pi * (2 + 3 * c) * sh2 * sh2;
      lsign = -1;
      break;
    default:  // (4, +-3)
      yp = -3.0 * r7_2pi * ch2 * ch2 * ch * (2 * c - 1) * sh;
      ym = 3.0 * r7_2pi * ch * (1 + 2 * c) * sh2 * sh2 * sh;
      lsign = 1;
      break;
  }
}

__device__ inline bool imr_domain_ok(const double *th) {
  for (int i = 0; i < 11; ++i)
    if (!isfinite(th[i])) return false;
  return th[0] > 0.0 && th[1] >= 0.05 && th[1] <= 1.0 && fabs(th[2]) <= 0.99 &&
         fabs(th[3]) <= 0.99 && th[4] > 0.0;
}

// raw (unaligned) (2,2) phase and its slope at frequency f
__device__ inline void raw_phase64(const WalkerC &w, double f, double &ph, double &dph) {
  if (f <= w.f1) {
    double v = cbrt(w.piM * f);
    double iv = 1.0 / v, iv2 = iv * iv, iv3 = iv2 * iv, iv5 = iv3 * iv2;
    ph = w.c5 * iv5 + w.c3 * iv3 + w.c2 * iv2;
    dph = (w.d5 * iv5 + w.d3 * iv3 + w.d2 * iv2) / f;
  } else {
    double x = f - w.f1, y = f - w.fRD;
    double L = w.fD / (y * y + w.fD * w.fD);
    ph = w.P1 + w.dP1 * x + kKappa * (atan(y / w.fD) - w.at1 - w.L1 * x);
    dph = w.dP1 + kKappa * (L - w.L1);
  }
}

__device__ inline void walker_setup(const double *__restrict__ th, int model, uint32_t modes, WalkerC &w) {
  w.model = model;
  w.pad0 = w.pad1 = 0;
  if (model == 1) {  // chirp
    bool ok = isfinite(th[0]) && isfinite(th[1]) && isfinite(th[2]) && isfinite(th[3]) && th[0] > 0.0;
    w.valid = ok ? 1 : 0;
    w.piMc = kPi * th[0] * kMsunS;
    w.amp = th[1] * kAmpScale;
    w.tc = th[2];
    w.phic = th[3];
    return;
  }
  w.valid = imr_domain_ok(th) ? 1 : 0;
  if (!w.valid) return;
  double M = th[0] * kMsunS, q = th[1];
  double m1 = 1.0 / (1.0 + q), m2 = q * m1;
  double eta = m1 * m2, delta = m1 - m2;
  double DL = th[4] * (kGpcM / kClight);
  double psi2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  double beta_so = ((113.0 * m1 * m1 + 75.0 * eta) * th[2] + (113.0 * m2 * m2 + 75.0 * eta) * th[3]) / 12.0;
  double psi3 = -16.0 * kPi + 4.0 * beta_so;
  double i128 = 1.0 / (128.0 * eta);
  w.piM = kPi * M;
  w.c5 = -3.0 * i128;
  w.c3 = w.c5 * psi2;
  w.c2 = w.c5 * psi3;
  w.d5 = 5.0 * i128;
  w.d3 = 3.0 * psi2 * i128;
  w.d2 = 2.0 * psi3 * i128;
  w.f1 = 0.018 / M;
  double Mf = M * (1.0 - 0.19 * eta);
  w.fRD = 0.0595 / Mf;
  w.fD = 0.0142 / Mf;
  w.fcut = 0.2 / M;
  w.fmax = -2.0 * w.fRD + sqrt(9.0 * w.fRD * w.fRD + 5.0 * w.fD * w.fD);
  {
    double v = cbrt(w.piM * w.f1);
    double iv = 1.0 / v, iv2 = iv * iv, iv3 = iv2 * iv, iv5 = iv3 * iv2;
    w.P1 = w.c5 * iv5 + w.c3 * iv3 + w.c2 * iv2;
    w.dP1 = (w.d5 * iv5 + w.d3 * iv3 + w.d2 * iv2) / w.f1;
  }
  w.lam_num = sq(w.f1 - w.fRD) + w.fD * w.fD;
  w.inv_fD = 1.0 / w.fD;
  w.L1 = w.fD / w.lam_num;
  w.at1 = atan((w.f1 - w.fRD) / w.fD);
  raw_phase64(w, w.fmax, w.ph_max, w.dph_max);
  w.AN = kPi * sqrt(2.0 * eta / 3.0) * M * M / DL * kAmpScale;
  w.tref = th[10];
  double a = 1.0 - 3.0 * eta;
  w.rel[0] = 1.0;
  w.rel[1] = 0.75 * sqrt(15.0 / 14.0) * delta;
  w.rel[2] = (4.0 / 9.0) * sqrt(10.0 / 7.0) * a;
  w.rel[3] = delta / 3.0;
  w.rel[4] = sqrt(5.0 / 7.0) / 3.0 * a;
  w.rel[5] = 9.0 / (4.0 * sqrt(70.0)) * delta * (1.0 - 2.0 * eta);
  double lam = th[7], bet = th[8], psi = th[9];
  double cl = cos(lam), sl = sin(lam), cb = cos(bet), sb = sin(bet), cp = cos(psi), sp = sin(psi);
  w.kx = -cb * cl;
  w.ky = -cb * sl;
  w.kz = -sb;
  // u = (sin l, -cos l, 0), v = (-sin b cos l, -sin b sin l, cos b)
  w.px = cp * sl - sp * sb * cl;
  w.py = -cp * cl - sp * sb * sl;
  w.pz = sp * cb;
  w.qx = -sp * sl - cp * sb * cl;
  w.qy = sp * cl - cp * sb * sl;
  w.qz = cp * cb;
  // polarisation weights of the active modes only; e^{i m phi_ref} as powers of e^{i phi_ref}
  double ci, si, chi, shi, s1, c1;
  sincos(th[6], &si, &ci);
  sincos(0.5 * th[6], &shi, &chi);
  sincos(th[5], &s1, &c1);
  for (int mi = 0; mi < kNumModes; ++mi) {
    if (!(modes & (1u << mi))) continue;
    double yp, ym;
    int ls;
    ylm_pair(mi, ci, si, chi, shi, yp, ym, ls);
    double cm = c1, sm = s1;
    for (int k = 1; k < kModeM[mi]; ++k) {
      double t = cm * c1 - sm * s1;
      sm = sm * c1 + cm * s1;
      cm = t;
    }
    w.kp[mi] = 0.5 * (yp + ls * ym);
    w.kc[mi] = 0.5 * (yp - ls * ym);
    w.eph[mi][0] = cm;
    w.eph[mi][1] = sm;
  }
}

// ---- precision-specific primitives ---------------------------------------
// FP64 reciprocal and cube root from hardware FP32 estimates refined by two
// Newton steps in FP64 (quadratic convergence from ~1e-7 to below the FP64
// rounding level); used by both paths in place of IEEE division sequences.
__device__ __forceinline__ double rcp64_nr(double x) {
  double y = (double)__builtin_amdgcn_rcpf((float)x);
  y = y * fma(-x, y, 2.0);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ double cbrt64_nr(double x) {
  double v = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)x) * (1.0f / 3.0f));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double v2 = v * v;
    v = v - fma(v2, v, -x) * (double)__builtin_amdgcn_rcpf((float)(3.0 * v2));
  }
  return v;
}

template <typename R>
struct Prec;

template <>
struct Prec<double> {
  static __device__ __forceinline__ void sincos_r(double x, double &s, double &c) { sincos(x, &s, &c); }
  static __device__ __forceinline__ void sincos_alpha(double a, double &s, double &c) { sincos(a, &s, &c); }
  static __device__ __forceinline__ double atan_small(double x) { return atan(x); }
  static __device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
  static __device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
  static constexpr int kSincTerms = 20;
};

template <>
struct Prec<float> {
  static __device__ __forceinline__ void sincos_r(float x, float &s, float &c) { sincosf(x, &s, &c); }
  static __device__ __forceinline__ void sincos_alpha(double a, double &s, double &c) { sincos(a, &s, &c); }
  static __device__ __forceinline__ float atan_small(float x) { return atanf(x); }
  static __device__ __forceinline__ float rsqrt_r(float x) { return rsqrtf(x); }
  static __device__ __forceinline__ float sqrt_r(float x) { return sqrtf(x); }
  static constexpr int kSincTerms = 14;
};

// (2,2) phase aligned at f_max, its slope, and the amplitude at (2,2)
// frequency fp; amplitude scaled by v^vpow (v = (pi M fp)^(1/3)).  Phase and
// slope are FP64; the frequency-dependent amplitude factor (v^-7/2 times the
// ringdown Lorentzian) is formed in R and multiplied by the per-walker FP64
// prefactor, so its rounding varies from edge to edge and never acts as a
// coherent shift of D_L.
template <typename R>
__device__ __forceinline__ void wf22(const WalkerC &w, double fp, int vpow, double &ph, double &dph,
                                     double &amp) {
  double v = cbrt64_nr(w.piM * fp);
  double iv = rcp64_nr(v);
  R lam2 = (R)1;
  if (fp <= w.f1) {
    double iv2 = iv * iv, iv3 = iv2 * iv, iv5 = iv3 * iv2;
    ph = w.c5 * iv5 + w.c3 * iv3 + w.c2 * iv2;
    dph = (w.d5 * iv5 + w.d3 * iv3 + w.d2 * iv2) * rcp64_nr(fp);
  } else {
    double x = fp - w.f1, y = fp - w.fRD;
    double rden = rcp64_nr(y * y + w.fD * w.fD);
    R Lr = (R)(w.fD * rden);
    R at = Prec<R>::atan_small((R)(y * w.inv_fD));
    // the arctan difference and the slope correction are bounded by a few rad
    ph = w.P1 + w.dP1 * x + kKappa * ((double)(at - (R)w.at1) - w.L1 * x);
    dph = w.dP1 + kKappa * ((double)Lr - w.L1);
    lam2 = (R)(w.lam_num * rden);
  }
  ph = ph - w.ph_max - w.dph_max * (fp - w.fmax);
  dph = dph - w.dph_max;
  R ivr = (R)iv;
  R af = ivr * ivr * ivr * Prec<R>::sqrt_r(ivr * lam2);
  double a = w.AN * (double)af;
  for (int k = 0; k < vpow; ++k) a *= v;
  amp = a;
}

// Taylor coefficients of sinc in y = x^2: c_n = (-1)^n / (2n+1)!
struct SincCoef {
  double c[24];
  constexpr SincCoef() : c() {
    double cn = 1.0;
    c[0] = 1.0;
    for (int n = 1; n < 24; ++n) {
      cn = -cn / ((2.0 * n) * (2.0 * n + 1.0));
      c[n] = cn;
    }
  }
};
constexpr SincCoef kSinc{};

// sinc series S(y) = sum c_n y^n and its divided difference
// S[y1, y2] = (S(y1) - S(y2)) / (y1 - y2), in one downward Horner pass:
// with P_n(y) = sum_{k>=n} c_k y^(k-n), P_n = c_n + y P_{n+1} and
// P_n[y1, y2] = P_{n+1}(y1) + y2 P_{n+1}[y1, y2].
template <typename R>
__device__ __forceinline__ void sinc_pair(R y1, R y2, R &s1, R &dd) {
  constexpr int N = Prec<R>::kSincTerms;
  R p = (R)kSinc.c[N];
  R d = (R)0;
#pragma unroll
  for (int n = N - 1; n >= 0; --n) {
    d = p + y2 * d;
    p = (R)kSinc.c[n] + y1 * p;
  }
  s1 = p;
  dd = d;
}

// A, E, T transfer of a plus-only (Tp) and a cross-only (Tc) wave, without
// the guiding-centre Doppler and the common e^{4 i pi f L}, for spacecraft
// offsets at orbital phase (ca, sa).  Only geometry enters here; the mode's
// polarisation weights are applied by the caller in FP64.
template <typename R>
__device__ __forceinline__ void response_pol(const WalkerC &w, R f, R a, R Cp, R Cm, R ca, R sa, cx<R> Tp[3],
                                             cx<R> Tc[3]) {
  const R eR = (R)kEccR;
  R c2a = ca * ca - sa * sa, s2a = (R)2 * sa * ca;
  // beta_k = 0, 2pi/3, 4pi/3
  const R cbk[3] = {(R)1, (R)-0.5, (R)-0.5};
  const R sbk[3] = {(R)0, (R)(0.5 * kSqrt3), (R)(-0.5 * kSqrt3)};
  R dp[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dp[k][0] = eR * ((R)0.5 * (c2a * cbk[k] + s2a * sbk[k]) - (R)1.5 * cbk[k]);
    dp[k][1] = eR * ((R)0.5 * (s2a * cbk[k] - c2a * sbk[k]) - (R)1.5 * sbk[k]);
    dp[k][2] = -(R)kSqrt3 * eR * (ca * cbk[k] + sa * sbk[k]);
  }
  // projections on the source frame use the FP64 sky vectors: rounding p, q
  // or k to FP32 would change |p|^2 - |q|^2 and act as a coherent amplitude
  // error at every frequency of the walker
  double kdp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    kdp[k] = w.kx * (double)dp[k][0] + w.ky * (double)dp[k][1] + w.kz * (double)dp[k][2];
  const double pif = kPi * (double)f;
  cx<R> Up[3], Vp[3], Uc[3], Vc[3];
  const int li[3] = {0, 1, 2}, lj[3] = {1, 2, 0};
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    int i = li[l], j = lj[l];
    R nx = dp[j][0] - dp[i][0], ny = dp[j][1] - dp[i][1], nz = dp[j][2] - dp[i][2];
    R inv = Prec<R>::rsqrt_r(nx * nx + ny * ny + nz * nz);
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const double ndx = nx, ndy = ny, ndz = nz;
    R kn = (R)(w.kx * ndx + w.ky * ndy + w.kz * ndz);
    double np = w.px * ndx + w.py * ndy + w.pz * ndz;
    double nq = w.qx * ndx + w.qy * ndy + w.qz * ndz;
    R Fp = (R)((np - nq) * (np + nq)), Fc = (R)(2.0 * np * nq);  // n e+ n, n ex n
    R sph, cph;
    Prec<R>::sincos_r((R)(pif * (kdp[i] + kdp[j])), sph, cph);
    R am = a * ((R)1 - kn), ap = a * ((R)1 + kn);
    R s1, dd;
    sinc_pair<R>(am * am, ap * ap, s1, dd);
    R delta = (R)-4 * a * a * kn * dd;  // sinc(x_ij) - sinc(x_ji)
    R sigma = s1 - (R)0.5 * delta;      // (sinc(x_ij) + sinc(x_ji)) / 2
    R us = sigma * Fp, vs = delta * Fp, uc = sigma * Fc, vc = delta * Fc;
    Up[l] = mk<R>(us * cph, us * sph);
    Vp[l] = mk<R>(vs * cph, vs * sph);
    Uc[l] = mk<R>(uc * cph, uc * sph);
    Vc[l] = mk<R>(vc * cph, vc * sph);
  }
  // sqrt2 A = Cp (U1 + U2 - 2 U3) - i Cm (V2 - V1)
  // sqrt6 E = 3 Cp (U2 - U1) - i Cm (2 V3 - V1 - V2)
  // sqrt3 T = -2 i Cm (V1 + V2 + V3)
  // (the 1/sqrt2, 1/sqrt6, 1/sqrt3 normalisations are applied by the caller in FP64)
  Tp[0] = Cp * (Up[0] + Up[1] - (R)2 * Up[2]) + Cm * mul_mi(Vp[1] - Vp[0]);
  Tp[1] = ((R)3 * Cp) * (Up[1] - Up[0]) + Cm * mul_mi((R)2 * Vp[2] - Vp[0] - Vp[1]);
  Tp[2] = ((R)2 * Cm) * mul_mi(Vp[0] + Vp[1] + Vp[2]);
  Tc[0] = Cp * (Uc[0] + Uc[1] - (R)2 * Uc[2]) + Cm * mul_mi(Vc[1] - Vc[0]);
  Tc[1] = ((R)3 * Cp) * (Uc[1] - Uc[0]) + Cm * mul_mi((R)2 * Vc[2] - Vc[0] - Vc[1]);
  Tc[2] = ((R)2 * Cm) * mul_mi(Vc[0] + Vc[1] + Vc[2]);
}

// Frequency-only response factors for a = pi f L:
// Cp = 4 a sin(2a) cos(a), Cm = 2 a sin(2a) sin(a)
template <typename R>
struct FreqC {
  R f, a, Cp, Cm;
};
template <typename R>
__device__ __forceinline__ FreqC<R> freq_consts(double f) {
  FreqC<R> fc;
  double a64 = kPi * f * kArmS;
  fc.f = (R)f;
  fc.a = (R)a64;
  R s, c;
  Prec<R>::sincos_r((R)a64, s, c);
  R s2 = (R)2 * s * c;
  fc.Cp = (R)4 * fc.a * s2 * c;
  fc.Cm = (R)2 * fc.a * s2 * s;
  return fc;
}

// Template of one walker at frequency f: small factors s[c] (FP64) and the
// carrier psi.  Only the response geometry runs in precision R; every
// per-walker constant factor (amplitude, polarisation weights, e^{i m phi_ref},
// mode phase) is applied in FP64, so FP32 rounding cannot act as a coherent
// shift of D_L or phi_ref.  Returns true if any mode is inside its support.
template <typename R>
__device__ __forceinline__ bool template_point(const WalkerC &w, uint32_t modes, double f, double t_obs,
                                               cx<double> s[3], double &psi) {
  if (w.model == 1) {  // 0PN chirp, one channel
    double x = w.piMc * f;
    double cx1 = cbrt64_nr(x);
    double x53 = x * cx1 * cx1;
    psi = w.phic - (3.0 / 128.0) * rcp64_nr(x53) - kTwoPi * f * w.tc;
    R fr = (R)f;
    double a = w.amp * (double)((R)1 / (fr * Prec<R>::sqrt_r(cbrt(fr))));
    s[0] = mk<double>(a, 0.0);
    s[1] = s[2] = mk<double>(0.0, 0.0);
    return true;
  }
  // carrier: (2,2) phase, t_ref shift, guiding-centre Doppler at t_22, arm phase
  double ph22, dph22, amp22;
  wf22<R>(w, f, 0, ph22, dph22, amp22);
  double t22 = w.tref - dph22 * kInvTwoPi;
  double al22 = reduce_2pi(t22 * (kTwoPi / kYearS));
  double sa22, ca22;
  Prec<R>::sincos_alpha(al22, sa22, ca22);
  double dop22 = kTwoPi * f * kOrbR * (w.kx * ca22 + w.ky * sa22);
  psi = ph22 - kTwoPi * f * w.tref - dop22 - 4.0 * kPi * f * kArmS;

  FreqC<R> fc = freq_consts<R>(f);
  s[0] = s[1] = s[2] = mk<double>(0.0, 0.0);
  bool any = false;
#pragma unroll 1
  for (int mi = 0; mi < kNumModes; ++mi) {
    if (!(modes & (1u << mi))) continue;
    int m = kModeM[mi];
    double fp = 2.0 * f / m;
    double tlm, amp, ca, sa;
    cx<double> fm;  // A_lm e^{i m phi_ref} e^{-i (Psi_lm - Psi)}
    if (mi == 0) {
      tlm = t22;
      amp = amp22;
      ca = ca22;
      sa = sa22;
      fm = mk<double>(amp * w.eph[0][0], amp * w.eph[0][1]);
    } else {
      double ph, dph;
      wf22<R>(w, fp, kModeVPow[mi], ph, dph, amp);
      amp *= w.rel[mi];
      tlm = w.tref - dph * kInvTwoPi;
      double al = reduce_2pi(tlm * (kTwoPi / kYearS));
      Prec<R>::sincos_alpha(al, sa, ca);
      double dop = kTwoPi * f * kOrbR * (w.kx * ca + w.ky * sa);
      // Psi_lm - Psi = (m/2 phi_22(2f/m) - phi_22(f)) - (Doppler_lm - Doppler_22)
      double dlt = reduce_2pi((0.5 * m * ph - ph22) - (dop - dop22));
      R sd, cd;
      Prec<R>::sincos_r((R)dlt, sd, cd);
      cx<double> e = mk<double>((double)cd, -(double)sd);
      fm = e * mk<double>(amp * w.eph[mi][0], amp * w.eph[mi][1]);
    }
    if (!(fp <= w.fcut && tlm >= 0.0 && tlm <= t_obs)) continue;
    any = true;
    cx<R> Tp[3], Tc[3];
    response_pol<R>(w, fc.f, fc.a, fc.Cp, fc.Cm, (R)ca, (R)sa, Tp, Tc);
    const double kp = w.kp[mi], kc = w.kc[mi];
    const double nrm[3] = {1.0 / kSqrt2, 1.0 / kSqrt6, 1.0 / kSqrt3};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // K+ T+ + Kx Tx = e^{i m phi} (kp T+ + i kc Tx)
      cx<double> t = mk<double>(nrm[c] * (kp * (double)Tp[c].re - kc * (double)Tc[c].im),
                                nrm[c] * (kp * (double)Tp[c].im + kc * (double)Tc[c].re));
      s[c] = s[c] + fm * t;
    }
  }
  return any;
}

// grid frequency with the two roundings of f0 + k df (no FMA contraction)
__device__ __forceinline__ double grid_freq(double f0, double df, int64_t k) {
  return __dadd_rn(f0, __dmul_rn((double)k, df));
}

}  // namespace mbh
