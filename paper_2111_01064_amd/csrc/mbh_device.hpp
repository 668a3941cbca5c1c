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
// powers of the ratio m / 2 between a mode's frequency argument 2 f / m and
// f: (2/m)^(1/3), (m/2)^(1/3), m/2, (m/2)^(7/6) (decimal expansions rounded)
__device__ __constant__ const double kModeP13[6] = {1.0, 0.87358046473629886905, 0.79370052598409973738,
                                                    1.25992104989487316477, 1.0, 0.87358046473629886905};
__device__ __constant__ const double kModeM13[6] = {1.0, 1.14471424255333186781, 1.25992104989487316477,
                                                    0.79370052598409973738, 1.0, 1.14471424255333186781};
__device__ __constant__ const double kModeHalf[6] = {1.0, 1.5, 2.0, 0.5, 1.0, 1.5};
__device__ __constant__ const double kModeM76[6] = {1.0, 1.60486979090049442633, 2.24492409661874596287,
                                                    0.44544935907016965237, 1.0, 1.60486979090049442633};

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
  // (pi M)^(1/3), (pi M)^(-1/3), AN (pi M)^(-7/6) and sqrt(lam_num): with the
  // frequency powers of FreqPow they give v, 1/v and the amplitude without a
  // root or a division per frequency
  double cpiM, icpiM, AN76, slam;
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

__device__ __forceinline__ bool imr_domain_ok(const double *th) {
  for (int i = 0; i < 11; ++i)
    if (!isfinite(th[i])) return false;
  return th[0] > 0.0 && th[1] >= 0.05 && th[1] <= 1.0 && fabs(th[2]) <= 0.99 &&
         fabs(th[3]) <= 0.99 && th[4] > 0.0;
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
// FP64 reciprocal square root: FP32 estimate and two Newton steps
// t <- t (1 + (1 - x t^2) / 2)
__device__ __forceinline__ double rsq64_nr(double x) {
  double t = (double)__builtin_amdgcn_rsqf((float)x);
#pragma unroll
  for (int k = 0; k < 2; ++k) t = fma(0.5 * t, fma(-x * t, t, 1.0), t);
  return t;
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

// Taylor coefficients of sin(x)/x and cos(x) in y = x^2:
// s_n = (-1)^n / (2n+1)!, c_n = (-1)^n / (2n)!
struct TrigCoef {
  double s[24], c[24];
  constexpr TrigCoef() : s(), c() {
    double sn = 1.0, cn = 1.0;
    s[0] = 1.0;
    c[0] = 1.0;
    for (int n = 1; n < 24; ++n) {
      cn = -cn / ((2.0 * n - 1.0) * (2.0 * n));
      sn = -sn / ((2.0 * n) * (2.0 * n + 1.0));
      s[n] = sn;
      c[n] = cn;
    }
  }
};
constexpr TrigCoef kTrig{};

// sin and cos for the bounded arguments of this library (|x| <= ~1e4): one
// Cody-Waite reduction by pi/2 (two-constant split, exact FMA products), then
// Taylor polynomials on [-pi/4, pi/4] truncated where the next term is below
// the format's rounding (x^17 / x^16 for FP64, x^11 / x^10 for FP32).
template <typename R>
struct TrigConst;
template <>
struct TrigConst<double> {
  static constexpr double kTwoOverPi = 0.636619772367581343075535053490057448;
  static constexpr double kPio2Hi = 1.5707963267948965579989817342720925807952880859375;  // nearest double
  static constexpr double kPio2Lo = 6.123233995736766035868820147291818e-17;            // pi/2 - hi
  static constexpr int kSin = 9, kCos = 9;
};
template <>
struct TrigConst<float> {
  static constexpr float kTwoOverPi = 0.636619772367581343f;
  static constexpr float kPio2Hi = 1.57079637050628662109375f;   // nearest float
  static constexpr float kPio2Lo = -4.37113900018624283e-8f;     // pi/2 - hi
  static constexpr int kSin = 6, kCos = 6;
};

template <typename R>
__device__ __forceinline__ void sincos_red(R x, R &s, R &c) {
  using T = TrigConst<R>;
  const R kq = rint(x * T::kTwoOverPi);
  R r = fma(-kq, T::kPio2Hi, x);
  r = fma(-kq, T::kPio2Lo, r);
  const int q = (int)kq;
  const R r2 = r * r;
  R ps = (R)kTrig.s[T::kSin - 1], pc = (R)kTrig.c[T::kCos - 1];
#pragma unroll
  for (int n = T::kSin - 2; n >= 0; --n) ps = fma(ps, r2, (R)kTrig.s[n]);
#pragma unroll
  for (int n = T::kCos - 2; n >= 0; --n) pc = fma(pc, r2, (R)kTrig.c[n]);
  const R sr = r * ps;
  // x = q pi/2 + r
  R so = (q & 1) ? pc : sr;
  R co = (q & 1) ? -sr : pc;
  if (q & 2) {
    so = -so;
    co = -co;
  }
  s = so;
  c = co;
}

template <typename R>
struct Prec;

template <>
struct Prec<double> {
  static __device__ __forceinline__ void sincos_r(double x, double &s, double &c) { sincos_red<double>(x, s, c); }
  static __device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
};

template <>
struct Prec<float> {
  static __device__ __forceinline__ void sincos_r(float x, float &s, float &c) { sincos_red<float>(x, s, c); }
  static __device__ __forceinline__ float sqrt_r(float x) { return sqrtf(x); }
};

// FP64 arctangent: the FP32 value refined by one Newton step in FP64 on
// g(a) = sin a - z cos a, whose second derivative vanishes at the root
// a = atan z, so the step converges cubically (relative error ~1e-7 -> below
// the FP64 rounding level).  Shorter and far lighter on registers than a
// full FP64 polynomial, and the same in both precision paths.
__device__ __forceinline__ double atan64_nr(double z) {
  const double a = (double)atanf((float)z);
  double s, c;
  sincos_red<double>(a, s, c);
  return a - (s - z * c) * rcp64_nr(fma(z, s, c));
}

// FP64 quotient x / y through the refined reciprocal (within 1 ulp; the
// per-walker constants below need no correctly rounded division)
__device__ __forceinline__ double div64(double x, double y) { return x * rcp64_nr(y); }

// sin and cos of an unbounded parameter angle: reduced to [-pi, pi] first
__device__ __forceinline__ void sincos_param(double x, double &s, double &c) {
  sincos_red<double>(reduce_2pi(x), s, c);
}

// raw (unaligned) (2,2) phase and its slope at frequency f > f1 (merger-
// ringdown continuation; the setup evaluates it at f_max)
__device__ __forceinline__ void raw_phase_mr(const WalkerC &w, double f, double &ph, double &dph) {
  const double x = f - w.f1, y = f - w.fRD;
  const double L = div64(w.fD, y * y + w.fD * w.fD);
  ph = w.P1 + w.dP1 * x + kKappa * (atan64_nr(y * w.inv_fD) - w.at1 - w.L1 * x);
  dph = w.dP1 + kKappa * (L - w.L1);
}

// (pi M f1)^(1/3) with f1 = 0.018 / M: a constant of the model
constexpr double kV1 = 0.38383165853550260132496406524933909994849537353683;

// extrinsic part of walker_setup: sky and polarisation vectors and the mode
// polarisation weights
__device__ __forceinline__ void walker_setup_sky(const double *__restrict__ th, uint32_t modes, WalkerC &w) {
  double t[11];
#pragma unroll
  for (int i = 5; i < 10; ++i) t[i] = th[i];
  double cl, sl, cb, sb, cp, sp;
  sincos_param(t[7], sl, cl);
  sincos_param(t[8], sb, cb);
  sincos_param(t[9], sp, cp);
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
  sincos_param(t[6], si, ci);
  sincos_param(0.5 * t[6], shi, chi);
  sincos_param(t[5], s1, c1);
  for (int mi = 0; mi < kNumModes; ++mi) {
    if (!(modes & (1u << mi))) continue;
    double yp, ym;
    int ls;
    ylm_pair(mi, ci, si, chi, shi, yp, ym, ls);
    double cm = c1, sm = s1;
    for (int k = 1; k < kModeM[mi]; ++k) {
      double tt = cm * c1 - sm * s1;
      sm = sm * c1 + cm * s1;
      cm = tt;
    }
    w.kp[mi] = 0.5 * (yp + ls * ym);
    w.kc[mi] = 0.5 * (yp - ls * ym);
    w.eph[mi][0] = cm;
    w.eph[mi][1] = sm;
  }
}

// Per-walker constants from theta.  part 1 sets the validity and the
// intrinsic constants (masses, spins, distance, t_ref: phase, amplitude and
// frequencies), part 2 the extrinsic ones (sky and polarisation vectors,
// mode polarisation weights); the two write disjoint fields, so two threads
// may build one walker together (part 0 does both).
__device__ __forceinline__ void walker_setup(const double *__restrict__ th, int model, uint32_t modes, WalkerC &w,
                                             int part = 0) {
  if (part == 2) {
    if (model != 1) walker_setup_sky(th, modes, w);
    return;
  }
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
  double t[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) t[i] = th[i];
  w.valid = imr_domain_ok(t) ? 1 : 0;
  if (!w.valid) return;
  const double M = t[0] * kMsunS, q = t[1];
  const double m1 = rcp64_nr(1.0 + q), m2 = q * m1;
  const double eta = m1 * m2, delta = m1 - m2;
  const double DL = t[4] * (kGpcM / kClight);
  const double psi2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  const double beta_so = ((113.0 * m1 * m1 + 75.0 * eta) * t[2] + (113.0 * m2 * m2 + 75.0 * eta) * t[3]) * (1.0 / 12.0);
  const double psi3 = -16.0 * kPi + 4.0 * beta_so;
  const double i128 = rcp64_nr(128.0 * eta);
  const double iM = 1.0 / M;  // IEEE division: M may lie far outside the FP32 range
  w.piM = kPi * M;
  w.c5 = -3.0 * i128;
  w.c3 = w.c5 * psi2;
  w.c2 = w.c5 * psi3;
  w.d5 = 5.0 * i128;
  w.d3 = 3.0 * psi2 * i128;
  w.d2 = 2.0 * psi3 * i128;
  w.f1 = 0.018 * iM;
  const double iMf = iM * rcp64_nr(1.0 - 0.19 * eta);
  w.fRD = 0.0595 * iMf;
  w.fD = 0.0142 * iMf;
  w.fcut = 0.2 * iM;
  w.fmax = -2.0 * w.fRD + sqrt(9.0 * w.fRD * w.fRD + 5.0 * w.fD * w.fD);
  {
    const double iv = 1.0 / kV1, iv2 = iv * iv, iv3 = iv2 * iv, iv5 = iv3 * iv2;
    w.P1 = w.c5 * iv5 + w.c3 * iv3 + w.c2 * iv2;
    w.dP1 = (w.d5 * iv5 + w.d3 * iv3 + w.d2 * iv2) * rcp64_nr(w.f1);
  }
  w.lam_num = sq(w.f1 - w.fRD) + w.fD * w.fD;
  w.inv_fD = rcp64_nr(w.fD);
  w.L1 = div64(w.fD, w.lam_num);
  w.at1 = atan64_nr((w.f1 - w.fRD) * w.inv_fD);
  // f_max lies past f1 (the (2,2) amplitude peaks in the merger-ringdown part)
  raw_phase_mr(w, w.fmax, w.ph_max, w.dph_max);
  w.AN = kPi * sqrt(2.0 * eta / 3.0) * M * M / DL * kAmpScale;
  w.cpiM = cbrt(w.piM);
  w.icpiM = 1.0 / w.cpiM;
  w.AN76 = w.AN * (w.icpiM * w.icpiM * w.icpiM) * sqrt(w.icpiM);
  w.slam = sqrt(w.lam_num);
  w.tref = t[10];
  // mode amplitude relative to (2,2) at the same orbital frequency, without
  // its power of v: leading-order PN mode magnitude |H_lm| times the
  // stationary-phase ratio sqrt(2/m), folded into one constant per mode
  // ((3,3): (3/4) sqrt(15/14) sqrt(2/3) = (3/4) sqrt(5/7); (4,4): (8/9)
  // sqrt(5/7) sqrt(1/2) = (4/9) sqrt(10/7); (2,1): sqrt2 / 3; (3,2): m = 2;
  // (4,3): 9 / (4 sqrt70) sqrt(2/3) = (3/4) sqrt(3/35))
  const double a = 1.0 - 3.0 * eta;
  w.rel[0] = 1.0;
  w.rel[1] = 0.75 * sqrt(5.0 / 7.0) * delta;
  w.rel[2] = (4.0 / 9.0) * sqrt(10.0 / 7.0) * a;
  w.rel[3] = (kSqrt2 / 3.0) * delta;
  w.rel[4] = sqrt(5.0 / 7.0) / 3.0 * a;
  w.rel[5] = 0.75 * sqrt(3.0 / 35.0) * delta * (1.0 - 2.0 * eta);
  if (part == 0) walker_setup_sky(th, modes, w);
}

// Powers of a frequency f used by the waveform: f^(1/3), f^(-1/3), 1/f and
// f^(-7/6), all FP64 (NR-refined estimates, within a few ulp).  The
// heterodyned pass reads them per bin edge from the reference; the grid
// kernels evaluate them per frequency.
struct FreqPow {
  double f13, fm13, fi, fm76;
};
__device__ __forceinline__ FreqPow freq_pows(double f) {
  FreqPow p;
  p.f13 = cbrt64_nr(f);
  p.fm13 = rcp64_nr(p.f13);
  p.fi = rcp64_nr(f);
  p.fm76 = p.fi * sqrt(p.fm13);
  return p;
}
// the powers at the frequency argument 2 f / m of mode mi
__device__ __forceinline__ FreqPow mode_pows(const FreqPow &p, int mi) {
  return FreqPow{p.f13 * kModeP13[mi], p.fm13 * kModeM13[mi], p.fi * kModeHalf[mi], p.fm76 * kModeM76[mi]};
}

// (2,2) phase aligned at f_max, its slope, and the amplitude at (2,2)
// frequency fp with powers pw; amplitude scaled by v^vpow (v = (pi M fp)^(1/3)).
// All FP64: the arctan of the merger-ringdown continuation and the amplitude
// factor would otherwise carry FP32 roundings of per-walker constants
// (arctan at f1) into every edge alike, i.e. coherent phase and amplitude
// shifts.  The inspiral and merger-ringdown forms are both evaluated and
// selected per lane: a wavefront's lanes straddle f1 often, and the
// straight-line code schedules better than the two branches.
__device__ __forceinline__ void wf22(const WalkerC &w, double fp, const FreqPow &pw, int vpow, double &ph,
                                     double &dph, double &amp) {
  const double v = w.cpiM * pw.f13;
  const double iv = w.icpiM * pw.fm13;
  // both branches, selected per lane (no divergent control flow)
  const double iv2 = iv * iv, iv3 = iv2 * iv, iv5 = iv3 * iv2;
  const double ph_i = w.c5 * iv5 + w.c3 * iv3 + w.c2 * iv2;
  const double dph_i = (w.d5 * iv5 + w.d3 * iv3 + w.d2 * iv2) * pw.fi;
  const double x = fp - w.f1, y = fp - w.fRD;
  const double t = rsq64_nr(y * y + w.fD * w.fD);
  const double ph_m = w.P1 + w.dP1 * x + kKappa * ((atan64_nr(y * w.inv_fD) - w.at1) - w.L1 * x);
  const double dph_m = w.dP1 + kKappa * (w.fD * (t * t) - w.L1);
  const bool insp = fp <= w.f1;
  ph = insp ? ph_i : ph_m;
  dph = insp ? dph_i : dph_m;
  const double lam = insp ? 1.0 : w.slam * t;
  ph = ph - w.ph_max - w.dph_max * (fp - w.fmax);
  dph = dph - w.dph_max;
  double a = w.AN76 * pw.fm76 * lam;
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

// Number N of sinc coefficients beyond c_0 that reach the format's rounding
// level for y <= y_max: the truncated terms are below 2^-53 (FP64) or 2^-24
// (FP32) relative to the divided difference (whose leading coefficient is
// -1/6).  ylim[N] is the largest y for which N suffices.
__host__ __device__ inline int sinc_terms(double y_max, bool fp64) {
  constexpr double ylim64[21] = {0, 0, 0, 1.1e-3, 1.08e-2, 5.17e-2, 0.166, 0.412, 0.857, 1.58, 2.64,
                                 4.12, 6.08, 8.58, 11.7, 15.4, 19.8, 25.0, 30.9, 37.5, 45.0};
  constexpr double ylim32[21] = {0, 0, 0, 0.173, 0.602, 1.48, 2.93, 5.08, 8.0, 11.8, 16.4,
                                 22.0, 28.5, 36.1, 44.6, 54.1, 64.7, 76.3, 88.9, 103.0, 117.0};
  const double *lim = fp64 ? ylim64 : ylim32;
  for (int n = 3; n < 20; ++n)
    if (y_max <= lim[n]) return n;
  return 20;
}

// the sinc coefficients in each format, in constant memory (read with
// scalar loads, the loop index being uniform)
struct SincCoef32 {
  float c[24];
  constexpr SincCoef32() : c() {
    for (int n = 0; n < 24; ++n) c[n] = (float)kSinc.c[n];
  }
};
__device__ __constant__ const SincCoef kSincDev64 = SincCoef{};
__device__ __constant__ const SincCoef32 kSincDev32 = SincCoef32{};

// sinc series S(y) = sum_{n<=N} c_n y^n and its divided difference
// S[y1, y2] = (S(y1) - S(y2)) / (y1 - y2) in one downward Horner pass:
// with P_n(y) = sum_{k>=n} c_k y^(k-n), P_n = c_n + y P_{n+1} and
// P_n[y1, y2] = P_{n+1}(y1) + y2 P_{n+1}[y1, y2].  The three links run in
// the same pass (one coefficient load feeds six independent chains).  N
// (<= 20) is uniform across the wavefront, so the loop is scalar-controlled.
template <typename R>
__device__ __forceinline__ void sinc_pairs3(const R y1[3], const R y2[3], int N, R s1[3], R dd[3]) {
  const R *c;
  if constexpr (sizeof(R) == 8) c = (const R *)kSincDev64.c;
  else c = (const R *)kSincDev32.c;
  R p[3] = {(R)0, (R)0, (R)0}, d[3] = {(R)0, (R)0, (R)0};
  for (int n = N; n >= 0; --n) {
    const R cn = c[n];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      d[l] = p[l] + y2[l] * d[l];
      p[l] = cn + y1[l] * p[l];
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    s1[l] = p[l];
    dd[l] = d[l];
  }
}

// Frequency-only response factors for a = pi f L:
// Cp = 4 a sin(2a) cos(a), Cm = 2 a sin(2a) sin(a); ns = sinc terms for the
// precision in use over the frequencies that share this value (uniform)
struct FreqC {
  double a, Cp, Cm;
  int ns;
};
__device__ __forceinline__ void freq_consts64(double f, double &a, double &Cp, double &Cm) {
  a = kPi * f * kArmS;
  double s, c;
  sincos_red<double>(a, s, c);
  const double s2 = 2.0 * s * c;
  Cp = 4.0 * a * s2 * c;
  Cm = 2.0 * a * s2 * s;
}
// sinc terms for frequencies up to f_max (the sinc arguments are a (1 +- k.n) <= 2a)
template <typename R>
__host__ __device__ inline int sinc_terms_for(double f_max) {
  const double x = 2.0 * kPi * f_max * kArmS;
  return sinc_terms(x * x, sizeof(R) == 8);
}
template <typename R>
__device__ __forceinline__ FreqC freq_consts(double f, int ns) {
  FreqC fc;
  freq_consts64(f, fc.a, fc.Cp, fc.Cm);
  fc.ns = ns;
  return fc;
}

// A, E, T transfer of one mode (unnormalised: sqrt2 A, sqrt6 E, sqrt3 T),
// without the guiding-centre Doppler and the common e^{4 i pi f L}, for
// spacecraft offsets at orbital phase (ca, sa).  The geometry (offsets,
// link vectors, projections, polarisation weights w_l = kp F+_l + i kc Fx_l)
// is FP64 in both paths: on this hardware an FP32 operation issues at the
// FP64 rate, so FP32 is used only where it shortens the work (the sinc
// series and the link phase sine/cosine, precision R), and constant-like
// FP32 roundings that would act coherently on every edge never arise.
// In this orbit model every arm has length L exactly, so the link unit
// vectors are offset differences in units of L, and the three offsets sum to
// zero, so the third link phase factor is the conjugate product of the other
// two.
// spacecraft offset k (beta_k = 2 pi k / 3) from the guiding centre in
// units of L at orbital phase a: (cos a, sin a) = (ca, sa),
// (cos 2a, sin 2a) = (c2a, s2a); e R / L = 1 / (2 sqrt3)
__device__ __forceinline__ void sc_offset(int k, double ca, double sa, double c2a, double s2a, double o[3]) {
  constexpr double e = 0.5 / kSqrt3;
  const double cb = k == 0 ? 1.0 : -0.5;
  const double sb = k == 0 ? 0.0 : (k == 1 ? 0.5 * kSqrt3 : -0.5 * kSqrt3);
  o[0] = e * (0.5 * (c2a * cb + s2a * sb) - 1.5 * cb);
  o[1] = e * (0.5 * (s2a * cb - c2a * sb) - 1.5 * sb);
  o[2] = -kSqrt3 * e * (ca * cb + sa * sb);
}

template <typename R>
__device__ __forceinline__ void response_mode(const WalkerC &w, double kp, double kc, const FreqC &fc, double ca,
                                              double sa, cx<double> T[3]) {
  const double c2a = ca * ca - sa * sa, s2a = 2.0 * sa * ca;
  // projections of the offsets on k, p and q: spacecraft 0 and 2 directly,
  // spacecraft 1 from the zero sum; link l runs from l to (l + 1) mod 3, so
  // its unit vector's projection is a difference of two of them
  double kd[3], pd[3], qd[3];
  {
    double o[3];
    sc_offset(0, ca, sa, c2a, s2a, o);
    kd[0] = w.kx * o[0] + w.ky * o[1] + w.kz * o[2];
    pd[0] = w.px * o[0] + w.py * o[1] + w.pz * o[2];
    qd[0] = w.qx * o[0] + w.qy * o[1] + w.qz * o[2];
    sc_offset(2, ca, sa, c2a, s2a, o);
    kd[2] = w.kx * o[0] + w.ky * o[1] + w.kz * o[2];
    pd[2] = w.px * o[0] + w.py * o[1] + w.pz * o[2];
    qd[2] = w.qx * o[0] + w.qy * o[1] + w.qz * o[2];
    kd[1] = -(kd[0] + kd[2]);
    pd[1] = -(pd[0] + pd[2]);
    qd[1] = -(qd[0] + qd[2]);
  }
  // link phase factors z_l = e^{i a k.(p_i + p_j)}: link (0,1) has phase
  // -a k.p_2, link (1,2) -a k.p_0, and z_2 closes
  cx<double> z[3];
  {
    R s0, c0, s1, c1;
    Prec<R>::sincos_r((R)(-fc.a * kd[2]), s0, c0);
    Prec<R>::sincos_r((R)(-fc.a * kd[0]), s1, c1);
    z[0] = mk<double>((double)c0, (double)s0);
    z[1] = mk<double>((double)c1, (double)s1);
    z[2] = z[0] * z[1];
    z[2].im = -z[2].im;
  }
  double kn[3];
  R y1[3], y2[3], s1r[3], ddr[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int m = l == 2 ? 0 : l + 1;
    kn[l] = kd[m] - kd[l];
    const double am = fc.a * (1.0 - kn[l]), ap = fc.a * (1.0 + kn[l]);
    y1[l] = (R)(am * am);
    y2[l] = (R)(ap * ap);
  }
  sinc_pairs3<R>(y1, y2, fc.ns, s1r, ddr);
  // sqrt2 A = Cp SAU - i Cm SAV, sqrt6 E = 3 Cp SEU - i Cm SEV, sqrt3 T = -2 i Cm STV
  cx<double> SAU = mk<double>(0, 0), SEU = mk<double>(0, 0), SAV = mk<double>(0, 0), SEV = mk<double>(0, 0),
             STV = mk<double>(0, 0);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int m = l == 2 ? 0 : l + 1;
    const double np = pd[m] - pd[l], nq = qd[m] - qd[l];
    // n e+ n = np^2 - nq^2, n ex n = 2 np nq
    const cx<double> wl = mk<double>(kp * ((np - nq) * (np + nq)), kc * (2.0 * np * nq));
    const double delta = -4.0 * fc.a * fc.a * kn[l] * (double)ddr[l];  // sinc(x_ij) - sinc(x_ji)
    const double sigma = (double)s1r[l] - 0.5 * delta;                 // (sinc(x_ij) + sinc(x_ji)) / 2
    const cx<double> wz = wl * z[l];
    const cx<double> U = sigma * wz, V = delta * wz;
    if (l == 0) {
      SAU = SAU + U;
      SEU = SEU - U;
      SAV = SAV - V;
      SEV = SEV - V;
    } else if (l == 1) {
      SAU = SAU + U;
      SEU = SEU + U;
      SAV = SAV + V;
      SEV = SEV - V;
    } else {
      SAU = SAU - 2.0 * U;
      SEV = SEV + 2.0 * V;
    }
    STV = STV + V;
  }
  T[0] = fc.Cp * SAU + fc.Cm * mul_mi(SAV);
  T[1] = (3.0 * fc.Cp) * SEU + fc.Cm * mul_mi(SEV);
  T[2] = (2.0 * fc.Cm) * mul_mi(STV);
}

// Template of one walker at frequency f: small factors s[c] (FP64) and the
// carrier psi.  Only the response geometry runs in precision R; every
// per-walker constant factor (amplitude, polarisation weights, e^{i m phi_ref},
// mode phase) is applied in FP64, so FP32 rounding cannot act as a coherent
// shift of D_L or phi_ref.  Returns true if any mode is inside its support.
// HM = false compiles the (2,2) mode alone (callers pass it only for mode
// mask (2,2) or the chirp model): without the higher-mode loop the kernels
// need under half the registers and run at several times the occupancy.
template <typename R, bool HM = true>
__device__ __forceinline__ bool template_point(const WalkerC &w, uint32_t modes, double f, const FreqPow &pw,
                                               const FreqC &fc, double t_obs, cx<double> s[3], double &psi) {
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
  wf22(w, f, pw, 0, ph22, dph22, amp22);
  double t22 = w.tref - dph22 * kInvTwoPi;
  double al22 = reduce_2pi(t22 * (kTwoPi / kYearS));
  double sa22, ca22;
  sincos_red<double>(al22, sa22, ca22);
  double dop22 = kTwoPi * f * kOrbR * (w.kx * ca22 + w.ky * sa22);
  psi = ph22 - kTwoPi * f * w.tref - dop22 - 4.0 * kPi * f * kArmS;

  s[0] = s[1] = s[2] = mk<double>(0.0, 0.0);
  bool any = false;
#pragma unroll 1
  for (int mi = 0; mi < (HM ? kNumModes : 1); ++mi) {
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
      wf22(w, fp, mode_pows(pw, mi), kModeVPow[mi], ph, dph, amp);
      amp *= w.rel[mi];
      tlm = w.tref - dph * kInvTwoPi;
      double al = reduce_2pi(tlm * (kTwoPi / kYearS));
      sincos_red<double>(al, sa, ca);
      double dop = kTwoPi * f * kOrbR * (w.kx * ca + w.ky * sa);
      // Psi_lm - Psi = (m/2 phi_22(2f/m) - phi_22(f)) - (Doppler_lm - Doppler_22)
      double dlt = reduce_2pi((0.5 * m * ph - ph22) - (dop - dop22));
      double sd, cd;
      sincos_red<double>(dlt, sd, cd);
      cx<double> e = mk<double>(cd, -sd);
      fm = e * mk<double>(amp * w.eph[mi][0], amp * w.eph[mi][1]);
    }
    if (!(fp <= w.fcut && tlm >= 0.0 && tlm <= t_obs)) continue;
    any = true;
    cx<double> T[3];
    response_mode<R>(w, w.kp[mi], w.kc[mi], fc, ca, sa, T);
    const double nrm[3] = {1.0 / kSqrt2, 1.0 / kSqrt6, 1.0 / kSqrt3};
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = s[c] + fm * (nrm[c] * T[c]);
  }
  return any;
}

// One mode (index mi) alone at frequency f, for per-mode relative binning:
// the small factors s[c] and the mode's own carrier psi = its phase
// (m/2) phi_22(2f/m), the t_ref shift, the guiding-centre Doppler at
// t_lm(f) and the arm phase.  Returns false (s = 0) outside the mode's
// support.  The same arithmetic as the mode's term in template_point, with
// the mode's phase kept in the carrier instead of relative to (2,2).
template <typename R>
__device__ __forceinline__ bool mode_point(const WalkerC &w, int mi, double f, const FreqPow &pw, const FreqC &fc,
                                           double t_obs, cx<double> s[3], double &psi) {
  const int m = kModeM[mi];
  const double fp = 2.0 * f / m;
  double ph, dph, amp;
  wf22(w, fp, mode_pows(pw, mi), kModeVPow[mi], ph, dph, amp);
  amp *= w.rel[mi];
  const double tlm = w.tref - dph * kInvTwoPi;
  const double al = reduce_2pi(tlm * (kTwoPi / kYearS));
  double sa, ca;
  sincos_red<double>(al, sa, ca);
  const double dop = kTwoPi * f * kOrbR * (w.kx * ca + w.ky * sa);
  psi = 0.5 * m * ph - kTwoPi * f * w.tref - dop - 4.0 * kPi * f * kArmS;
  s[0] = s[1] = s[2] = mk<double>(0.0, 0.0);
  if (!(fp <= w.fcut && tlm >= 0.0 && tlm <= t_obs)) return false;
  cx<double> T[3];
  response_mode<R>(w, w.kp[mi], w.kc[mi], fc, ca, sa, T);
  const cx<double> fm = mk<double>(amp * w.eph[mi][0], amp * w.eph[mi][1]);
  const double nrm[3] = {1.0 / kSqrt2, 1.0 / kSqrt6, 1.0 / kSqrt3};
#pragma unroll
  for (int c = 0; c < 3; ++c) s[c] = fm * (nrm[c] * T[c]);
  return true;
}

// grid frequency with the two roundings of f0 + k df (no FMA contraction)
__device__ __forceinline__ double grid_freq(double f0, double df, int64_t k) {
  return __dadd_rn(f0, __dmul_rn((double)k, df));
}

}  // namespace mbh
