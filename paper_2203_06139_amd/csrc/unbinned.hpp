// unbinned.hpp -- extended unbinned NLL and its reverse-mode gradient:
// the binned objective's per-bin code applied to single events at arbitrary
// positions (the per-event batch evaluation of RooFit-style likelihoods).
//
// For events x_e with weights w_e (default 1) and the 1D Gauss + polynomial
// or exponential model read as an intensity lambda(x; theta):
//   L(theta) = Lambda(theta) - sum_e w_e ln lambda(x_e),
//   Lambda   = integral of lambda over [lo, hi]   (the expected count),
// the extended likelihood of a Poisson process (the binned Poisson objective
// as the bins shrink to single events).  Per event the forward sweep
// evaluates lambda, the reverse sweep with adjoint -w/lambda accumulates
// dlambda/dtheta (without the 1/s of the Gaussian mean and width columns,
// applied to the totals); one exp per Gaussian, the table log and a Newton
// reciprocal per event.  Lambda and its gradient are closed forms (per
// Gaussian with z_b = (b - m)/s, e_b = exp(-z_b^2/2)):
//   Lambda_g = A s sqrt(pi/2) [erf(z_hi/sqrt 2) - erf(z_lo/sqrt 2)],
//   d/dA = Lambda_g/A,  d/dm = A (e_lo - e_hi),
//   d/ds = Lambda_g/s + A (z_lo e_lo - z_hi e_hi);
//   polynomial: d/dc_j = t_scale (t_hi^(j+1) - t_lo^(j+1))/(j+1);
//   exponential: (hi - lo) E_c S(b1 d), E_c = exp(b0 + b1 t_c), S = sinh(u)/u;
// thread 0 of block 0 computes them into LDS during the prologue and adds
// them to the partials it publishes.  Events outside
// [lo, hi] are skipped; lambda <= 0 at an event inside is a domain error.
#pragma once

#include "device.hpp"

namespace hf {

struct UnbinnedArgs {
  const double* x;   // [n] event positions
  const float* w;    // [n] or null
  int64_t n;
  double lo, hi;
  const double* theta;
  double* nll_out;
  double* grad_out;  // [P] or null (value only)
  int32_t* status_out;
  int32_t P;
  double t_shift, t_scale;
  double* part;
  int32_t* part_flags;
  const double2* log_lut;
};

// Launches the main kernel and returns the grid it used through *grid_used
// (the caller then launches the finishing kernel over that many partials).
using UnbinnedFn = hipError_t (*)(const UnbinnedArgs&, bool vec, int num_cu, int max_grid,
                                  hipStream_t, int* grid_used);

// Event pairs per thread per step (16-byte loads of two positions); the next
// step's positions are requested while the current step is computed.
// Measured on 1e7 events (two Gaussians + cubic): 4 pairs with the prefetch
// 65.6 us; without it 80.5 us (8 pairs 68.6 us, 2 pairs 86.4 us); 2 pairs
// with it 77.3 us.
constexpr int kUbPairs = 4;

template <int U>
__device__ __forceinline__ void load_pairs(const UnbinnedArgs& a, int64_t q0, int64_t stride,
                                           int64_t npair, double2 (&xv)[U], float2 (&wv)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t q = q0 + u * stride;
    xv[u] = make_double2(__builtin_nan(""), __builtin_nan(""));  // skipped
    wv[u] = make_float2(0.0f, 0.0f);
    if (q < npair) {
      xv[u] = reinterpret_cast<const double2*>(a.x)[q];
      wv[u] = a.w ? reinterpret_cast<const float2*>(a.w)[q] : make_float2(1.0f, 1.0f);
    }
  }
}

template <int NG, int BKG, bool GRAD, int NV>
__device__ __forceinline__ void event_term(const UnbinnedArgs& a, const Model1D<NG, BKG>& M,
                                           const double2* __restrict__ lut, double x, double w,
                                           double (&acc)[NV], int& flags) {
  using S = Shape1D<NG, BKG>;
  const bool in = x >= a.lo && x <= a.hi;
  // a skipped event (outside the range, or NaN) is evaluated at the range's
  // midpoint with weight 0, where every partial is finite: at its own x a
  // polynomial power could overflow and 0 * inf would reach the sums
  x = in ? x : 0.5 * (a.lo + a.hi);
  double lam = 0.0;
  double J[S::P];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const double z = (x - M.m[g]) * M.is[g];
    const double e = exp_fast(-0.5 * z * z);
    const double G = M.A[g] * e;
    lam += G;
    if constexpr (GRAD) {
      const double Gz = G * z;
      J[3 * g] = e;
      J[3 * g + 1] = Gz;
      J[3 * g + 2] = Gz * z;
    }
  }
  if constexpr (BKG == BKG_EXP) {
    const double t = (x - M.tshift) * M.ta;
    const double Eb = exp_fast(fma(M.c[1], t, M.c[0]));
    lam += Eb;
    if constexpr (GRAD) {
      J[3 * NG] = Eb;
      J[3 * NG + 1] = t * Eb;
    }
  } else if constexpr (S::NB > 0) {
    const double t = (x - M.tshift) * M.ta;
    double b = M.c[S::NB - 1];
#pragma unroll
    for (int j = S::NB - 2; j >= 0; --j) b = fma(b, t, M.c[j]);
    lam += b;
    if constexpr (GRAD) {
      double tj = 1.0;
#pragma unroll
      for (int j = 0; j < S::NB; ++j) {
        J[3 * NG + j] = tj;
        tj *= t;
      }
    }
  }
  const bool ok = lam > 0.0;
  flags |= (in && !ok) ? ST_DOMAIN : 0;
  const double we = (in && ok) ? w : 0.0;
  const double lg = log_lut<false>(ok ? lam : 1.0, lut);
  acc[0] = fma(we, lg, acc[0]);
  if constexpr (GRAD) {
    const double r = we * rcp_fast(ok ? lam : 1.0);
#pragma unroll
    for (int k = 0; k < S::P; ++k) acc[1 + k] = fma(r, J[k], acc[1 + k]);
  }
}

// Lambda (out[0]) and dLambda/dtheta_k (out[1 + k], final values).
template <int NG, int BKG>
__device__ void lambda_terms(const UnbinnedArgs& a, const Model1D<NG, BKG>& M, double* out) {
  using S = Shape1D<NG, BKG>;
  constexpr double kRt = 1.2533141373155002512;  // sqrt(pi/2)
  constexpr double kIr2 = 0.70710678118654752440;
  double lam = 0.0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const double s = 1.0 / M.is[g];
    const double zl = (a.lo - M.m[g]) * M.is[g], zh = (a.hi - M.m[g]) * M.is[g];
    const double el = exp(-0.5 * zl * zl), eh = exp(-0.5 * zh * zh);
    const double ia = s * kRt * (erf(zh * kIr2) - erf(zl * kIr2));
    const double lg = M.A[g] * ia;
    lam += lg;
    out[1 + 3 * g] = ia;
    out[2 + 3 * g] = M.A[g] * (el - eh);
    out[3 + 3 * g] = lg * M.is[g] + M.A[g] * (zl * el - zh * eh);
  }
  if constexpr (BKG == BKG_EXP) {
    // (hi - lo) E_c S(b1 d) over the range, E_c at its midpoint t_c, d its
    // half-width in t (S = sinh(u)/u, see sinhc)
    const double tl = (a.lo - M.tshift) * M.ta, th = (a.hi - M.tshift) * M.ta;
    const double tc = 0.5 * (tl + th), d = 0.5 * (th - tl), w = a.hi - a.lo;
    const double Ec = exp(fma(M.c[1], tc, M.c[0]));
    double Sh, dSh;
    sinhc(M.c[1] * d, Sh, dSh);
    lam = fma(w * Ec, Sh, lam);
    out[1 + 3 * NG] = w * Ec * Sh;
    out[2 + 3 * NG] = w * Ec * fma(tc, Sh, d * dSh);
  } else if constexpr (S::NB > 0) {
    const double tl = (a.lo - M.tshift) * M.ta, th = (a.hi - M.tshift) * M.ta;
    double pl = tl, ph = th;
#pragma unroll
    for (int j = 0; j < S::NB; ++j) {
      const double ij = a.t_scale * (ph - pl) / static_cast<double>(j + 1);
      lam = fma(M.c[j], ij, lam);
      out[1 + 3 * NG + j] = ij;
      pl *= tl;
      ph *= th;
    }
  }
  out[0] = lam;
}

template <int NG, int BKG, bool GRAD, bool VEC>
__global__ __launch_bounds__(kBlock) void k_nll_unbinned(UnbinnedArgs a) {
  using S = Shape1D<NG, BKG>;
  constexpr int NV = GRAD ? S::P + 1 : 1;
  __shared__ double2 lut[kLogLut];
  __shared__ double lamd[S::P + 1];
  __shared__ double ff[S::P + 1];
  log_lut_load(lut, a.log_lut);
  Model1D<NG, BKG> M;
  M.init(a.theta, a.t_shift, a.t_scale);
  const bool finite = all_finite(a.theta, S::P);
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0) lambda_terms<NG, BKG>(a, M, lamd);
#pragma unroll
    for (int k = 0; k <= S::P; ++k) ff[k] = M.final_factor(k);
  }
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  if constexpr (VEC) {
    const int64_t npair = a.n / 2;
    const int64_t step = kUbPairs * stride;
    double2 xn[kUbPairs];
    float2 wn[kUbPairs];
    load_pairs(a, tid, stride, npair, xn, wn);
    for (int64_t q0 = tid; q0 < npair; q0 += step) {
      double2 xv[kUbPairs];
      float2 wv[kUbPairs];
#pragma unroll
      for (int u = 0; u < kUbPairs; ++u) {
        xv[u] = xn[u];
        wv[u] = wn[u];
      }
      if (q0 + step < npair) load_pairs(a, q0 + step, stride, npair, xn, wn);
#pragma unroll
      for (int u = 0; u < kUbPairs; ++u) {
        event_term<NG, BKG, GRAD>(a, M, lut, xv[u].x, wv[u].x, acc, flags);
        event_term<NG, BKG, GRAD>(a, M, lut, xv[u].y, wv[u].y, acc, flags);
      }
    }
    if ((a.n & 1) && tid == 0)
      event_term<NG, BKG, GRAD>(a, M, lut, a.x[a.n - 1], a.w ? a.w[a.n - 1] : 1.0f, acc, flags);
  } else {
    for (int64_t e = tid; e < a.n; e += stride)
      event_term<NG, BKG, GRAD>(a, M, lut, a.x[e], a.w ? a.w[e] : 1.0f, acc, flags);
  }
  // L = Lambda - sum w ln lambda: every block publishes -(its sums) times
  // the final factors, and block 0 adds Lambda and its derivatives
  __shared__ double fac[NV];
  if (threadIdx.x < NV) fac[threadIdx.x] = -ff[threadIdx.x];
  grid_publish<NV>(acc, flags | (finite ? 0 : ST_NONFINITE), fac, lamd, a.part, a.part_flags);
}

// Blocks per CU that fit (queried once per variant) bound a single round.
template <int NG, int BKG, bool GRAD, bool VEC>
hipError_t launch_unbinned_v(const UnbinnedArgs& a, int num_cu, int max_grid, hipStream_t s,
                             int* grid_used) {
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_nll_unbinned<NG, BKG, GRAD, VEC>, kBlock,
                                                     0) != hipSuccess || o < 1)
      o = 1;
    return o;
  }();
  const int64_t per = VEC ? 2 * kUbPairs : 1;
  const int64_t need = (a.n + per * kBlock - 1) / (per * kBlock);
  int64_t grid = static_cast<int64_t>(num_cu) * occ;
  if (grid > need) grid = need;
  if (grid > max_grid) grid = max_grid;
  if (grid < 1) grid = 1;
  *grid_used = static_cast<int>(grid);
  hipLaunchKernelGGL((k_nll_unbinned<NG, BKG, GRAD, VEC>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int NG, int BKG>
hipError_t launch_unbinned(const UnbinnedArgs& a, bool vec, int num_cu, int max_grid,
                           hipStream_t s, int* grid_used) {
  if (a.grad_out)
    return vec ? launch_unbinned_v<NG, BKG, true, true>(a, num_cu, max_grid, s, grid_used)
               : launch_unbinned_v<NG, BKG, true, false>(a, num_cu, max_grid, s, grid_used);
  return vec ? launch_unbinned_v<NG, BKG, false, true>(a, num_cu, max_grid, s, grid_used)
             : launch_unbinned_v<NG, BKG, false, false>(a, num_cu, max_grid, s, grid_used);
}

// bkg: the background code (polynomial degree -1..3, or BKG_EXP).
template <int NG>
UnbinnedFn pick_unbinned_ng(int bkg) {
  switch (bkg) {
    case -1:
      if constexpr (NG == 0) return nullptr;
      else return &launch_unbinned<NG, BKG_NONE>;
    case 0:
      return &launch_unbinned<NG, 0>;
    case 1:
      return &launch_unbinned<NG, 1>;
    case 2:
      return &launch_unbinned<NG, 2>;
    case 3:
      return &launch_unbinned<NG, 3>;
    case BKG_EXP:
      return &launch_unbinned<NG, BKG_EXP>;
    default:
      return nullptr;
  }
}

// Defined in unbinned_ng{0..4}.hip.
UnbinnedFn pick_unbinned_ng0(int bkg);
UnbinnedFn pick_unbinned_ng1(int bkg);
UnbinnedFn pick_unbinned_ng2(int bkg);
UnbinnedFn pick_unbinned_ng3(int bkg);
UnbinnedFn pick_unbinned_ng4(int bkg);

}  // namespace hf
