// fastmath.hpp -- lean FP64 elementary functions for the per-bin sweep.
//
// On gfx950 FP64 FMA issues at the full (non-packed) vector rate, so the cost
// of a bin is its VALU instruction count.  The library versions of exp, log
// and division carry range/special-case handling that the objective never
// needs (its arguments are finite and, where it matters, positive normal), so
// these replacements drop it:
//   exp_fast   Cody-Waite reduction by ln 2 and a degree-13 Taylor polynomial
//              on |r| <= ln2/2 (truncation < 1e-17); inputs below -746 give 0.
//   rcp_fast   v_rcp_f64 seed (measured on gfx950: <= 4.7e-8 relative) and
//              one Newton step (<= 2.3e-15); div_fast adds one residual
//              correction, which brings the quotient to about 1 ulp (the
//              refinement the compiler's IEEE division uses, without its
//              scaling for extreme exponents).
//   exp_hw32   the FP32 hardware exp2, for the FP32-per-bin variant: results
//              below about e^-87 are 0 and above e^88 infinite.
//   log_lut    x = 2^e m, m in [1,2); a 1024-entry LDS table of 1/c_j and
//              ln c_j at the midpoints c_j of the top 10 mantissa bits gives
//              f = m/c_j - 1 with |f| < 2^-11, and ln(1+f) is a degree-4
//              polynomial (|f|^5/5 < 1e-17).  Table entries with c_j >= 1.5
//              store ln(c_j/2) and bump e, so arguments just below 1 do not
//              cancel against ln 2.  log_lut(0) is finite (about -709): an
//              empty bin's n ln(n/mu) term is 0 * finite = 0.
// Inputs must be finite; div_fast needs a positive normal divisor.
#pragma once

#include <hip/hip_runtime.h>

namespace hf {

constexpr double kLog2e = 1.4426950408889634074;
// ln 2 split so that k * kLn2Hi is exact for |k| < 2^11 (trailing zero bits).
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;
constexpr double kLn2 = 6.93147180559945309417e-01;

constexpr int kLogLutBits = 10;
constexpr int kLogLut = 1 << kLogLutBits;

__device__ __forceinline__ double exp_fast(double x) {
  x = fmax(x, -746.0);
  const double k = __builtin_rint(x * kLog2e);
  double r = fma(-k, kLn2Hi, x);
  r = fma(-k, kLn2Lo, r);
  double p = 1.0 / 6227020800.0;     // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);  // 1/12!
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, static_cast<int>(k));
}

// e^x through the FP32 hardware exp2 (about 1e-7 relative for |x| < 8).
__device__ __forceinline__ double exp_hw32(double x) {
  return static_cast<double>(__builtin_amdgcn_exp2f(static_cast<float>(x * kLog2e)));
}

__device__ __forceinline__ double rcp_fast(double d) {
  const double y = __builtin_amdgcn_rcp(d);
  return fma(y, fma(-d, y, 1.0), y);
}

// a / d for a positive normal d.  The FP32-per-bin variant keeps the FP64
// seed (an FP32 seed would overflow or vanish for divisors outside FP32's
// range) and drops the residual correction (2.3e-15 relative is ample there).
template <bool F32BIN>
__device__ __forceinline__ double div_fast(double a, double d) {
  const double y = rcp_fast(d);
  const double q = a * y;
  return F32BIN ? q : fma(fma(-d, q, a), y, q);
}

// Clamp of a recurrence ratio's exponent: 0 * exp(a) must stay 0, so exp(a)
// must stay finite in the precision it is taken in (e^88.7 overflows FP32).
template <bool F32BIN>
__device__ __forceinline__ double clamp_ratio_exponent(double a) {
  constexpr double lim = F32BIN ? 80.0 : 700.0;
  return fmin(fmax(a, -lim), lim);
}

// Log table entry j: 1/c_j and ln of c_j (of c_j/2 from 1.5 up), with
// c_j = 1 + (j + 1/2)/kLogLut.  Computed once per context on the host
// (log_lut_host) and copied into each block's LDS by log_lut_load; the block
// must synchronise before the first log_lut call.
__host__ __device__ inline void log_lut_entry(int j, double* ic, double* lnc) {
  const double c = 1.0 + (j + 0.5) / kLogLut;
  *ic = 1.0 / c;
  *lnc = (j >= kLogLut / 2) ? -log(2.0 * *ic) : -log(*ic);
}

__device__ __forceinline__ void log_lut_load(double2* lut, const double2* __restrict__ src) {
  for (int j = threadIdx.x; j < kLogLut; j += blockDim.x) lut[j] = src[j];
}

// Degree of the ln(1+f) polynomial: 4 terms for FP64 accuracy, 3 for the
// FP32-per-bin variant (|f|^4/4 < 1e-14).
template <bool F32BIN>
__device__ __forceinline__ double log_lut(double x, const double2* __restrict__ lut) {
  const int hi = __double2hiint(x);
  const int lo = __double2loint(x);
  const int j = (hi >> (20 - kLogLutBits)) & (kLogLut - 1);
  const int e = ((hi >> 20) - 1023) + (j >> (kLogLutBits - 1));
  const double m = __hiloint2double((hi & 0x000fffff) | 0x3ff00000, lo);
  const double2 t = lut[j];
  const double f = fma(m, t.x, -1.0);
  double p;
  if (F32BIN) {
    p = 1.0 / 3.0;
    p = fma(p, f, -0.5);
    p = fma(p, f, 1.0);
  } else {
    p = -0.25;
    p = fma(p, f, 1.0 / 3.0);
    p = fma(p, f, -0.5);
    p = fma(p, f, 1.0);
  }
  // e ln 2 in one rounding: e = 0 for arguments in [0.75, 1.5), where the
  // objective cancels and needs the log to the last bit; elsewhere |ln x| >
  // 0.28 and the term it enters is large, so ~1e-16 relative is ample.
  const double ed = static_cast<double>(e);
  return fma(p, f, fma(ed, kLn2, t.y));
}

// S(u) = sinh(u)/u and S'(u) = (cosh u - S(u))/u: the average of
// exp(b0 + b1 t) over [t_c - d, t_c + d] is exp(b0 + b1 t_c) S(b1 d).  Taylor
// series to u^10 for |u| < 1/2 (truncation below 4e-14 relative), the
// closed forms beyond, where cosh u - S(u) no longer cancels badly.
__device__ __forceinline__ void sinhc(double u, double& S, double& dS) {
  if (fabs(u) < 0.5) {
    const double u2 = u * u;
    S = 1.0 + u2 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0 * (1.0 + u2 / 72.0 * (1.0 + u2 / 110.0))));
    dS = u / 3.0 * (1.0 + u2 / 10.0 * (1.0 + u2 / 28.0 * (1.0 + u2 / 54.0 * (1.0 + u2 / 88.0))));
  } else {
    S = sinh(u) / u;
    dS = (cosh(u) - S) / u;
  }
}

}  // namespace hf
