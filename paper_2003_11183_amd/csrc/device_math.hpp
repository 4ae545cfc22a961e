// Device univariate functions of the SOV recursion (FP64).
//
// Phi and log Phi come from erfcx(z) = exp(z^2) erfc(z) (polynomial in
// t = (z - K)/(z + K) up to z = 12, the asymptotic series above), so the
// lower tail is formed as erfcx(|x|/sqrt2) exp(-x^2/2) / 2 with x^2 split
// exactly by an fma; log Phi needs no exp.  Phi^-1(u) = sqrt2 x p(w) with
// x = 2u - 1, w = -log(4 u (1 - u)) and p a polynomial in w or sqrt(w) on
// five intervals (Giles' form of erfinv).  Coefficients: special_tables.hpp,
// written by gen_special.py.  These keep the sweep kernel's register
// footprint small enough for several waves per SIMD.
//
// The chi quantile of the Student-t radius is chi_nu^-1(u) = sqrt(2
// P^-1(nu/2, u)) with P the regularized lower incomplete gamma function,
// solved by Halley's method; P and Q = 1 - P come from the power series
// (x < a + 1) and Legendre's continued fraction evaluated by the modified
// Lentz algorithm otherwise.
#pragma once

#include <hip/hip_runtime.h>

#define TLRQMC_SPECIAL_TABLE static __constant__
#include "special_tables.hpp"

namespace tlrqmc {
namespace dev {

// Read-only global data seen through the constant address space: uniform
// loads from it become scalar loads (one per wave, into SGPRs).
#define TLRQMC_CONST __attribute__((address_space(4)))
typedef const TLRQMC_CONST double *ctab_t;

template <class T>
__device__ __forceinline__ const TLRQMC_CONST T *as_const(const T *p) {
  return (const TLRQMC_CONST T *)p;
}

// A pointer into global memory, marked so: loads through it are global
// loads (counted on the vector memory counter only) rather than flat ones.
#define TLRQMC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const TLRQMC_GLOBAL T *as_global(const T *p) {
  return (const TLRQMC_GLOBAL T *)p;
}

// Word 3 of a raw buffer resource (data format 32, every other field zero);
// loads through it take byte offsets, and an offset past the resource's
// byte count reads zero.
constexpr int kRawBufferWord3 = 0x00020000;

// Copy of a wave-uniform descriptor in device memory, read with scalar
// loads (T is a plain struct of 8-byte multiples).
template <class T>
__device__ __forceinline__ T load_uniform(const T *p) {
  static_assert(sizeof(T) % 8 == 0, "descriptor size");
  T out;
  const auto src = as_const(reinterpret_cast<const uint64_t *>(p));
  uint64_t *dst = reinterpret_cast<uint64_t *>(&out);
#pragma unroll
  for (int i = 0; i < static_cast<int>(sizeof(T) / 8); ++i) dst[i] = src[i];
  return out;
}

// The coefficient table through a pointer the optimizer cannot see through:
// the loads stay inside the loop that calls the function (one scalar load
// per few coefficients) instead of being hoisted, which would pin all 134
// coefficients in registers for the whole kernel.
__device__ __forceinline__ ctab_t special_table() {
  ctab_t p = (ctab_t)kSpecialTable;
  asm volatile("" : "+s"(p));
  return p;
}

// Interval probabilities at or below this value are handled in log space.
constexpr double kTiny = 1e-300;
constexpr double kLogSqrt2Pi = 0.91893853320467274178;
constexpr double kInvSqrtPi = 0.56418958354775628695;
constexpr double kLog4 = 1.38629436111989061883;

// a * b + c with the wave-uniform c read straight from its scalar registers
// (v_fma_f64 takes one scalar operand).  Left to itself the compiler ties
// the accumulator to c and copies c into vector registers first, tripling
// the instruction count of every polynomial step.
__device__ __forceinline__ double fma_s(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

template <int OFF, int N>
__device__ __forceinline__ double horner(ctab_t T, double s) {
  double acc = fma_s(T[OFF + N - 1], s, T[OFF + N - 2]);
#pragma unroll
  for (int i = N - 3; i >= 0; --i) acc = fma_s(acc, s, T[OFF + i]);
  return acc;
}

// a / d for d in a range far from overflow and underflow: hardware
// reciprocal, two Newton steps and one residual correction.
__device__ __forceinline__ double div_safe(double a, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-d, q, a), r, q);
}

constexpr double kLn2Hi = 6.93147180559945286227e-01;
constexpr double kLn2Lo = 2.31904681384629955842e-17;

// exp(x) for x <= 0: x = k ln2 + r with |r| <= ln2/2 (Cody-Waite split of
// ln2), a polynomial for exp(r), then the exponent by ldexp.
__device__ __forceinline__ double exp_nonpos(ctab_t T, double x) {
  if (!(x > -745.2)) return x != x ? x : 0.0;
  const double k = rint(x * M_LOG2E);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
  return ldexp(horner<kOffExp, kNExp>(T, r * kExpH), static_cast<int>(k));
}

// log(x) for x > 0: x = m 2^e with m in [sqrt(1/2), sqrt 2), f = m - 1
// (exact), s = f / (2 + f), log m = 2s + s^3 Q(s^2).
__device__ __forceinline__ double log_pos(ctab_t T, double x) {
  if (!(x > 0.0) || isinf(x)) return x == 0.0 ? -INFINITY : (x > 0.0 ? x : NAN);
  int e = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);
  if (m < M_SQRT1_2) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;
  const double s = div_safe(f, 2.0 + f);
  const double v = s * s;
  const double lm = fma(s * v, horner<kOffLog, kNLog>(T, (v - kLogC) * kLogH), 2.0 * s);
  const double de = static_cast<double>(e);
  return fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
}

// log(1 + x) for x > -1: log of the rounded sum, corrected by its error.
__device__ __forceinline__ double log1p_t(ctab_t T, double x) {
  const double u = 1.0 + x;
  return log_pos(T, u) + (x - (u - 1.0)) / u;
}

// erfcx(z) for z > 12 (z = +inf gives 0): the asymptotic series
// sum_k (-1)^k (2k-1)!! / (2 z^2)^k divided by z sqrt(pi).  Out of line: it
// is reached only below Phi(-17).
__device__ __forceinline__ double erfcx_large(double z) {
  const double v = 0.5 / (z * z);
  double acc = 0.0, coef = 1.0;
  double pw = 1.0;
#pragma unroll
  for (int k = 0; k < kErfcxAsymTerms; ++k) {
    acc = fma(coef, pw, acc);
    pw *= v;
    coef *= -(2.0 * k + 1.0);
  }
  return acc * kInvSqrtPi / z;
}

// erfcx(z) for z >= 0.
__device__ __forceinline__ double erfcx_pos(ctab_t T, double z) {
  if (z <= kErfcxZmax) {
    const double t = div_safe(z - kErfcxK, z + kErfcxK);
    const double g = horner<kOffErfcx, kNErfcx>(T, (t - kErfcxC) * kErfcxH);
    return g * (1.0 - t) * 0.5;
  }
  return erfcx_large(z);
}

// q = Phi(-|x|) and lq = log q, for finite x.
__device__ __forceinline__ void phi_lower(ctab_t T, double x, double &q, double &lq, double &ex) {
  const double z = fabs(x) * M_SQRT1_2;
  ex = 0.5 * erfcx_pos(T, z);
  const double p = x * x;
  const double a = 0.5 * p;
  const double al = 0.5 * fma(x, x, -p);  // x^2 / 2 = a + al exactly
  q = ex * exp_nonpos(T, -a) * (1.0 - al);
  lq = log_pos(T, ex) - a - al;
}

__device__ inline double Phi(ctab_t T, double x) {
  if (isinf(x)) return x > 0 ? 1.0 : 0.0;
  double q, lq, ex;
  phi_lower(T, x, q, lq, ex);
  return x < 0.0 ? q : 1.0 - q;
}

__device__ inline double log_Phi(ctab_t T, double x) {
  if (isinf(x)) return x > 0 ? 0.0 : -INFINITY;
  double q, lq, ex;
  phi_lower(T, x, q, lq, ex);
  return x < 0.0 ? lq : log1p_t(T, -q);
}

// p(w) of Phi^-1 for w >= 6.25 (u outside [5e-4, 1 - 5e-4]), in sqrt(w)
// on four intervals.  Out of line: rare, and it would otherwise add its
// registers to the main path.
__device__ __forceinline__ double inv_poly_tail(ctab_t T, double wv) {
  const double s = sqrt(wv);
  if (s < 4.0) return horner<kOffInv2, kNInv2>(T, (s - kInvC2) * kInvH2);
  if (s < 8.0) return horner<kOffInv3, kNInv3>(T, (s - kInvC3) * kInvH3);
  if (s < 14.0) return horner<kOffInv4, kNInv4>(T, (s - kInvC4) * kInvH4);
  return horner<kOffInv5, kNInv5>(T, (s - kInvC5) * kInvH5);
}

// p(w) of Phi^-1: a polynomial in w on [0, 6.25], the tail beyond.
__device__ __forceinline__ double inv_poly(ctab_t T, double wv) {
  if (wv < 6.25) return horner<kOffInv1, kNInv1>(T, (wv - kInvC1) * kInvH1);
  return inv_poly_tail(T, wv);
}

__device__ inline double Phi_inv(ctab_t T, double u) {
  const double wv = -log_pos(T, 4.0 * u * (1.0 - u));
  const double x = 2.0 * u - 1.0;
  if (!(wv <= 756.25)) return u < 0.5 ? -INFINITY : INFINITY;  // u = 0 or 1
  return M_SQRT2 * x * inv_poly(T, wv);
}

// Phi^-1(exp(lu)) for lu possibly far below the double range.  Above
// lu = -690 this is Phi_inv(exp(lu)).  Below, 1 - u = 1 to double
// precision, so w = -log(4 u (1 - u)) = -log 4 - lu and the tail polynomial
// applies up to w = 756 (lu = -757); further out, Newton steps on log Phi
// from the asymptotic start, with log Phi(y) = log(erfcx(-y/sqrt2)/2) -
// y^2/2 and erfcx from its asymptotic series (-y/sqrt2 > 12 there).
__device__ inline double Phi_inv_log(ctab_t T, double lu) {
  if (lu > -690.0) return Phi_inv(T, exp_nonpos(T, lu));
  const double wv = -kLog4 - lu;
  if (wv <= 756.25) return -M_SQRT2 * inv_poly(T, wv);
  double y = -sqrt(-2.0 * lu - log_pos(T, -4.0 * M_PI * lu));
  for (int it = 0; it < 12; ++it) {
    const double z = -y * M_SQRT1_2;
    const double lp = log_pos(T, 0.5 * erfcx_large(z)) - z * z;
    const double dy = (lp - lu) / exp_nonpos(T, -z * z - kLogSqrt2Pi - lp);
    y -= dy;
    if (fabs(dy) <= 1e-16 * fabs(y)) break;
  }
  return y;
}

__device__ __forceinline__ double log_add_exp(double x, double y) {
  const double mx = fmax(x, y);
  if (mx == -INFINITY) return -INFINITY;
  return mx + log1p(exp(fmin(x, y) - mx));
}

// log(exp(x) - exp(y)) for x >= y.
__device__ __forceinline__ double log_diff_exp(double x, double y) {
  if (y == -INFINITY) return x;
  return x + log1p(-exp(y - x));
}

// One variable of the recursion with conditional limits (ah, bh) and point
// w: returns log(Phi(bh) - Phi(ah)) and sets y to the conditional quantile
// Phi^-1(Phi(ah) + w (Phi(bh) - Phi(ah))).  Where ah > 0 the complement
// CDFs are used; tiny intervals go through log Phi; an empty interval
// gives -inf and y = 0.
__device__ inline double sov_step(double ah, double bh, double w, double &y) {
  ctab_t T = special_table();
  const bool lower = ah <= 0.0;
  const double lo = lower ? ah : -bh;
  const double hi = lower ? bh : -ah;
  const double d = Phi(T, lo);
  const double e = Phi(T, hi);
  const double delta = e - d;
  double ld, yy;
  if (delta > kTiny) {
    const double u = lower ? fma(w, delta, d) : fma(-w, delta, e);
    yy = Phi_inv(T, u);
    ld = log_pos(T, delta);
  } else {
    const double l_lo = log_Phi(T, lo);
    const double l_hi = log_Phi(T, hi);
    ld = (l_hi > l_lo) ? log_diff_exp(l_hi, l_lo) : -INFINITY;
    if (!(ld > -INFINITY)) {
      y = 0.0;
      return -INFINITY;
    }
    const double lw = log_pos(T, w);
    const double lu = lower ? log_add_exp(l_lo, lw + ld) : log_diff_exp(l_hi, lw + ld);
    yy = Phi_inv_log(T, lu);
  }
  if (!(ld > -INFINITY)) {
    y = 0.0;
    return -INFINITY;
  }
  y = lower ? yy : -yy;
  return ld;
}

// One-sided form (a = -inf): returns log Phi(bh), sets y = Phi^-1(w Phi(bh)).
// One log serves both signs of bh: log(ex) - x^2/2 below zero, and
// log(1 - q) corrected to log1p(-q) above.
__device__ inline double sov_step_upper(double bh, double w, double &y) {
  ctab_t T = special_table();
  if (isinf(bh)) {
    if (bh < 0) {
      y = 0.0;
      return -INFINITY;
    }
    y = Phi_inv(T, w);
    return 0.0;
  }
  const double z = fabs(bh) * M_SQRT1_2;
  const double ex = 0.5 * erfcx_pos(T, z);
  const double p = bh * bh;
  const double a = 0.5 * p;
  const double al = 0.5 * fma(bh, bh, -p);
  const double q = ex * exp_nonpos(T, -a) * (1.0 - al);
  const bool neg = bh < 0.0;
  const double e = neg ? q : 1.0 - q;
  const double arg = neg ? ex : e;
  const double L = log_pos(T, arg);
  // e >= 1/2 above zero, so (2 - e) stands in for 1/e in the correction,
  // which is itself below one ulp of 1.
  const double le = neg ? L - a - al : fma((-q) - (e - 1.0), 2.0 - e, L);
  if (e > kTiny) {
    y = Phi_inv(T, w * e);
  } else {
    y = Phi_inv_log(T, log_pos(T, w) + le);
  }
  return le;
}

template <int N>
__device__ __forceinline__ float horner32(const float (&c)[N], float s) {
  float acc = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) acc = fmaf(acc, s, c[i]);
  return acc;
}

// erfcx(z) / 2 in FP32 for 0 <= z <= 8: the rational-map polynomial.
__device__ __forceinline__ float half_erfcx32_poly(float z) {
  const float t = (z - kErfcx32K) * __builtin_amdgcn_rcpf(z + kErfcx32K);
  const float g = horner32(kErfcx32, (t - kErfcx32C) * kErfcx32H);
  return g * (1.0f - t) * 0.25f;
}

// erfcx(z) / 2 in FP32 for z > 8: the asymptotic series 1/(z sqrt(pi)) (1 -
// v + 3v^2 - 15v^3 + 105v^4 - 945v^5), v = 1/(2z^2) (error below 3e-9).
__device__ __forceinline__ float half_erfcx32_asym(float z) {
  const float r = __builtin_amdgcn_rcpf(z);
  const float v = 0.5f * r * r;
  const float sr = fmaf(fmaf(fmaf(fmaf(fmaf(-945.0f, v, 105.0f), v, -15.0f), v, 3.0f), v, -1.0f), v, 1.0f);
  return (0.5f * 0.56418958354775628f) * r * sr;
}

// Phi^-1(exp(lu)) deep in the lower tail (exp(lu) < 1e-36), in FP64 with
// few live values: there 1 - u = 1 to double precision, w' = -log 4 - lu
// >= 81, and Phi^-1 = -sqrt2 p(w') with p in sqrt(w') (the last two tail
// intervals of the FP64 table) up to w' = 756.25; further out, Newton steps
// on log Phi from the asymptotic start.
__device__ __noinline__ double Phi_inv_log_deep(double lu) {
  ctab_t T = special_table();
  const double wv = -kLog4 - lu;
  if (wv <= 756.25) {
    const double s = sqrt(wv);
    const double pw = s < 14.0 ? horner<kOffInv4, kNInv4>(T, (s - kInvC4) * kInvH4)
                               : horner<kOffInv5, kNInv5>(T, (s - kInvC5) * kInvH5);
    return -M_SQRT2 * pw;
  }
  double y = -sqrt(-2.0 * lu - log_pos(T, -4.0 * M_PI * lu));
  for (int it = 0; it < 12; ++it) {
    const double z = -y * M_SQRT1_2;
    const double lp = log_pos(T, 0.5 * erfcx_large(z)) - z * z;
    const double dy = (lp - lu) / exp_nonpos(T, -z * z - kLogSqrt2Pi - lp);
    y -= dy;
    if (fabs(dy) <= 1e-16 * fabs(y)) break;
  }
  return y;
}

// Precision form of the one-sided step: Phi(bh), log Phi(bh) and the
// quantile with FP32 special functions, FP64 where precision is made.
//   q = Phi(-|bh|) = erfcx(|bh|/sqrt2) exp(-bh^2/2) / 2: erfcx in FP32, the
//     exponent bh^2/2 split exactly in FP64 and reduced to 2^-(k + f) there.
//   log Phi(bh) = log(erfcx/2) - bh^2/2 below zero (FP32 log, FP64 sum: valid
//     however far out), and log1p(-q) = -2 atanh(q / (2 - q)) above (FP32
//     series).
//   u = w Phi(bh) and its complement c = 1 - u are formed in FP64 without
//     cancellation (c = (1 - w) + w q above zero), and
//     Phi^-1(u) = sqrt2 (u - c) p(w'), w' = -log(4 p (1 - p)), p = min(u, c),
//     with p(w') in FP32 out to w' = 90 (p down to 1e-36).
//   Below p = 1e-36 (only where bh < 0) the quantile is taken in FP64 from
//     log u = log w + log Phi(bh) (Phi_inv_log_deep).
// The FP32 parts carry about 2e-7 relative error; the running sum of log P
// stays FP64.
__device__ inline double sov_step_upper_fp32(double bh, double w, double &y) {
  constexpr float kLn2f = 0.69314718055994531f;
  if (bh == -INFINITY) {  // an empty interval: a dead sample
    y = 0.0;
    return -INFINITY;
  }
  const double ab = fabs(bh);
  // erfcx(|bh|/sqrt2)/2.  Above zero and beyond z = 8 (bh > 11.3) the
  // complement q is below 1e-29 and leaves e = 1 - q, u, c and log e
  // unchanged in FP64, so any value of the right size will do there: the
  // polynomial at z = 8.  Only the lower tail (bh < -11.3, where q itself is
  // the probability) takes the asymptotic series, in a branch that is
  // skipped unless a lane of the wave needs it.
  const float zf = static_cast<float>(ab * M_SQRT1_2);
  float ex = half_erfcx32_poly(fminf(zf, kErfcx32Zmax));
  if (zf > kErfcx32Zmax && bh < 0.0) ex = half_erfcx32_asym(zf);
  // q = Phi(-|bh|) = ex 2^-(tt) with tt = bh^2 log2(e) / 2 (its FP64 rounding
  // moves q by about 1e-14 relative), split into integer and fraction
  const double tt = fmin(bh * bh * (0.5 * M_LOG2E), 200.0);
  const double kf = floor(tt);
  const float q = __builtin_amdgcn_ldexpf(ex * __builtin_amdgcn_exp2f(-static_cast<float>(tt - kf)),
                                           -static_cast<int>(kf));
  const double qd = static_cast<double>(q);
  double le, u, c;
  if (bh >= 0.0) {
    // log1p(-q) = -2 atanh(q / (2 - q)), u = w (1 - q), c = (1 - w) + w q
    const float v = q * __builtin_amdgcn_rcpf(2.0f - q);
    const float v2 = v * v;
    const float at = fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(1.0f / 15.0f, v2, 1.0f / 13.0f), v2, 1.0f / 11.0f), v2,
                                              1.0f / 9.0f), v2, 1.0f / 7.0f), v2, 0.2f), v2, 1.0f / 3.0f), v2, 1.0f);
    le = static_cast<double>(-2.0f * v * at);
    u = fma(-w, qd, w);
    c = fma(w, qd, 1.0 - w);
  } else {
    // log q = log(erfcx/2) - bh^2/2 with bh^2/2 = a + al split exactly
    const double p2 = bh * bh;
    const double a = 0.5 * p2;
    const double al = 0.5 * fma(bh, bh, -p2);
    le = static_cast<double>(__builtin_amdgcn_logf(ex) * kLn2f) - a - al;
    u = w * qd;
    c = 1.0 - u;
  }
  const double pm = fmin(u, c);
  if (pm >= 1e-36) {
    const float pf = static_cast<float>(pm);
    const float wv = -__builtin_amdgcn_logf(4.0f * pf * (1.0f - pf)) * kLn2f;
    float pw;
    if (wv < 6.25f) {
      pw = horner32(kInv32, (wv - kInv32C) * kInv32H);
    } else {
      const float sq = __builtin_amdgcn_sqrtf(wv);
      pw = sq < kInv32Split ? horner32(kInv32T0, (sq - kInv32T0C) * kInv32T0H)
                            : horner32(kInv32T1, (sq - kInv32T1C) * kInv32T1H);
    }
    y = M_SQRT2 * (u - c) * static_cast<double>(pw);
  } else {
    y = Phi_inv_log_deep(log_pos(special_table(), w) + le);
  }
  return le;
}

// Regularized incomplete gamma: returns P(a, x) and sets q = Q(a, x).
__device__ inline double gamma_pq(double a, double x, double lgam, double &q) {
  if (x <= 0.0) {
    q = 1.0;
    return 0.0;
  }
  const double lpre = a * log(x) - x - lgam;
  if (x < a + 1.0) {
    double ap = a, term = 1.0 / a, sum = term;
    for (int i = 0; i < 600; ++i) {
      ap += 1.0;
      term *= x / ap;
      sum += term;
      if (fabs(term) < fabs(sum) * 1e-17) break;
    }
    const double p = sum * exp(lpre);
    q = 1.0 - p;
    return p;
  }
  // Legendre continued fraction for Q by the modified Lentz algorithm.
  const double tiny = 1e-300;
  double bb = x + 1.0 - a, c = 1.0 / tiny, dd = 1.0 / bb, h = dd;
  for (int i = 1; i < 600; ++i) {
    const double an = -i * (i - a);
    bb += 2.0;
    dd = an * dd + bb;
    if (fabs(dd) < tiny) dd = tiny;
    c = bb + an / c;
    if (fabs(c) < tiny) c = tiny;
    dd = 1.0 / dd;
    const double del = dd * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  q = exp(lpre) * h;
  return 1.0 - q;
}

// Quantile of the chi distribution with nu degrees of freedom.
__device__ inline double chi_inv(double nu, double u) {
  const double a = 0.5 * nu;
  const double lgam = lgamma(a);
  // Wilson-Hilferty start, or the small-x power law when that is not positive.
  const double z = Phi_inv(special_table(), u);
  const double t = 1.0 / (9.0 * a);
  double x = 1.0 - t + z * sqrt(t);
  x = a * x * x * x;
  const double xs = exp((log(u) + lgamma(a + 1.0)) / a);
  if (!(x > 0.0) || xs < x * 0.5) x = fmax(xs, 1e-300);
  const bool upper = u > 0.5;
  const double target = upper ? 1.0 - u : u;
  for (int it = 0; it < 100; ++it) {
    double q;
    const double p = gamma_pq(a, x, lgam, q);
    const double f = upper ? target - q : p - target;  // P(x) - u either way
    const double dens = exp((a - 1.0) * log(x) - x - lgam);
    if (!(dens > 0.0)) break;
    const double tn = f / dens;
    const double dx = tn / (1.0 - 0.5 * tn * ((a - 1.0) / x - 1.0));
    double xn = x - dx;
    if (xn <= 0.0) xn = 0.5 * x;
    if (fabs(xn - x) <= 1e-15 * x) {
      x = xn;
      break;
    }
    x = xn;
  }
  return sqrt(2.0 * x);
}

}  // namespace dev
}  // namespace tlrqmc
