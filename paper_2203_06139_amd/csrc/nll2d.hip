// nll2d.hip -- objective (+ gradient) kernel of the correlated 2D Gaussian
// plus constant over a row-major (x fastest) 2D histogram, with optional
// per-bin weights and the per-bin weight adjoint seed * l_i (the backward of
// a differentiable objective in both theta and w).
//
// Along a row y is fixed and Q = (u^2 - 2 rho u v + v^2)/(1 - rho^2) =
// w^2 + v^2 with w = (u - rho v)/sqrt(1 - rho^2), so exp(-Q/2) is a 1D
// Gaussian in x: a chunk of 16 bins of one row uses the same two-multiply
// recurrence as the 1D kernel (two exps per chunk, valid while
// 16 |dw| <= 1 with dw = hx / (sx sqrt(1 - rho^2)); otherwise per-bin exps).
#include "nll_kernels.hpp"

namespace hf {

// One chunk of len consecutive bins of one row.  RECUR needs len == K.
template <int OBJ, bool GRAD, bool F32BIN, bool RECUR, int K, int NV>
__device__ __forceinline__ void chunk_2d(const Model2D& M, const double2* __restrict__ lut, double u0,
                                         double du, double v, const double (&n)[K],
                                         const double (&w)[K], int len, double (&acc)[NV],
                                         int& flags, double (&lk)[K]) {
  const double sqD = sqrt(M.invD);
  const double dw = du * sqD;
  const double w0 = (u0 - M.rho * v) * sqD;
  double e = 0.0, r = 0.0, Dw = 0.0;
  if constexpr (RECUR) {
    const double q0 = -0.5 * fma(w0, w0, v * v);
    const double a0 = clamp_ratio_exponent<F32BIN>(fma(-dw, w0, -0.5 * dw * dw));
    e = F32BIN ? exp_hw32(q0) : exp_fast(q0);
    r = F32BIN ? exp_hw32(a0) : exp_fast(a0);
    Dw = M.Dw;
  }
  // Reverse sweep of a recurrence piece by moments: only u varies along the
  // row (u_k = u0 + k du), and every adjoint term is mb e times a polynomial
  // of degree <= 2 in u, so E_l = sum_k mb_k e_k k^l (l = 0..2) and
  // sum_k mb_k suffice; they are expanded after the loop.
  constexpr bool MOM = RECUR && GRAD;
  double E0 = 0.0, E1 = 0.0, E2 = 0.0, Mb = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // bins past len (short row tail, !RECUR only) are computed and masked
    const bool in = RECUR || k < len;
    // ---- forward sweep ----
    double ek, u = 0.0, uv = 0.0, Q = 0.0;
    if constexpr (RECUR) {
      ek = e;
    } else {
      u = fma(static_cast<double>(k), du, u0);
      uv = u * v;
      Q = (fma(u, u, v * v) - 2.0 * M.rho * uv) * M.invD;
      ek = F32BIN ? exp_hw32(-0.5 * Q) : exp_fast(-0.5 * Q);
    }
    const double G = M.A * ek;
    const double mu = G + M.c;
    double l, ub;
    const bool dom = objective_t<OBJ, F32BIN>(n[k], mu, lut, l, ub);
    flags |= (dom && in) ? ST_DOMAIN : 0;
    l = in ? l : 0.0;
    lk[k] = l;
    acc[0] = fma(w[k], l, acc[0]);
    if constexpr (MOM) {
      const double mb = w[k] * ub;
      const double kd = static_cast<double>(k);
      const double t = mb * ek;
      E0 += t;
      E1 = fma(t, kd, E1);
      E2 = fma(t, kd * kd, E2);
      Mb += mb;
    } else if constexpr (GRAD) {
      // ---- reverse sweep: mu_bar = w ubar ----
      const double mb = in ? w[k] * ub : 0.0;
      acc[1] = fma(mb, ek, acc[1]);  // A
      // Q_bar = -mu_bar G / 2;  dQ/du = 2(u - rho v)/D, dQ/dv = 2(v - rho u)/D,
      // dQ/drho = 2(rho Q - u v)/D; u = (x-mx)/sx, v = (y-my)/sy.  The common
      // factors (1/D, 1/sx, 1/sy) are applied once to the totals.
      const double gb = mb * G;  // = -2 Q_bar
      const double au = gb * fma(-M.rho, v, u);
      const double av = gb * fma(-M.rho, u, v);
      acc[2] += au;                                  // mx  (x invD/sx)
      acc[3] += av;                                  // my  (x invD/sy)
      acc[4] = fma(au, u, acc[4]);                   // sx  (x invD/sx)
      acc[5] = fma(av, v, acc[5]);                   // sy  (x invD/sy)
      acc[6] = fma(gb, fma(-M.rho, Q, uv), acc[6]);  // rho (x invD)
      acc[7] += mb;                                  // c
    }
    if constexpr (RECUR) {
      e *= r;
      r *= Dw;
    }
  }
  if constexpr (MOM) {
    // with g = mb G = A mb e: S0 = sum g, Su = sum g u, Su2 = sum g u^2
    const double su = fma(du, E1, u0 * E0);
    const double su2 = fma(u0, fma(2.0 * du, E1, u0 * E0), du * du * E2);
    const double S0 = M.A * E0, Su = M.A * su, Su2 = M.A * su2;
    const double rho = M.rho;
    acc[1] += E0;                                              // A
    acc[2] += fma(-rho * v, S0, Su);                           // sum g (u - rho v)
    acc[3] += fma(v, S0, -rho * Su);                           // sum g (v - rho u)
    acc[4] += fma(-rho * v, Su, Su2);                          // sum g (u - rho v) u
    acc[5] += v * fma(v, S0, -rho * Su);                       // sum g (v - rho u) v
    const double sq = fma(v * v, S0, fma(-2.0 * rho * v, Su, Su2));  // sum g (u^2 - 2 rho u v + v^2)
    acc[6] += fma(v, Su, -rho * M.invD * sq);                  // sum g (u v - rho Q)
    acc[7] += Mb;                                              // c
  }
}

template <int OBJ, bool GRAD, bool F32BIN>
__global__ __launch_bounds__(kBlock, kMinWaves) void k_nll_2d(NllArgs a) {
  constexpr int NV = GRAD ? 8 : 1;
  constexpr int K = kChunk2D;
  __shared__ double2 lut[OBJ == OBJ_POISSON ? kLogLut : 1];
  if constexpr (OBJ == OBJ_POISSON) log_lut_load(lut, a.log_lut);
  Model2D M;
  M.init(a.theta);
  const double du = a.hx * M.isx;
  const double dwv = du * sqrt(M.invD);
  M.Dw = exp(-dwv * dwv);
  const bool recur = K * fabs(dwv) <= 1.0;
  if constexpr (OBJ == OBJ_POISSON) __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  // the upstream adjoint scales grad_w here; the finishing kernel applies it
  // to the parameter gradient
  const double seed = (a.grad_w_out && a.seed) ? a.seed[0] : 1.0;
  const bool finite = all_finite(a.theta, a.P);
  const int64_t nx = a.nx;
  const int64_t cpr = (nx + K - 1) / K;  // chunks per row
  const int64_t nitems = cpr * a.ny;
  const double inv_cpr = 1.0 / static_cast<double>(cpr);
  const bool vec = (nx % 4) == 0;  // every row starts 16-byte aligned
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;

  for (int64_t c = tid; c < nitems; c += stride) {
    int64_t iy = static_cast<int64_t>(static_cast<double>(c) * inv_cpr);
    int64_t cx = c - iy * cpr;
    if (cx < 0) {
      --iy;
      cx += cpr;
    } else if (cx >= cpr) {
      ++iy;
      cx -= cpr;
    }
    const int64_t ix0 = cx * K;
    const int len = static_cast<int>(nx - ix0 < K ? nx - ix0 : K);
    const int64_t i0 = iy * nx + ix0;
    double n[K], w[K];
    if (vec && len == K) {
#pragma unroll
      for (int q = 0; q < K / 4; ++q) {
        double t4[4];
        load_counts4(a, i0 + 4 * q, t4);
#pragma unroll
        for (int k = 0; k < 4; ++k) n[4 * q + k] = t4[k];
        if (a.weights) {
          const float4 wv = *reinterpret_cast<const float4*>(a.weights + i0 + 4 * q);
          w[4 * q] = wv.x;
          w[4 * q + 1] = wv.y;
          w[4 * q + 2] = wv.z;
          w[4 * q + 3] = wv.w;
        } else {
          w[4 * q] = w[4 * q + 1] = w[4 * q + 2] = w[4 * q + 3] = 1.0;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool in = k < len;
        n[k] = in ? load_count1(a, i0 + k) : 0.0;
        w[k] = (in && a.weights) ? static_cast<double>(a.weights[i0 + k]) : 1.0;
      }
    }
    const double v = (fma(static_cast<double>(iy), a.hy, a.y0) - M.my) * M.isy;
    const double u0 = (fma(static_cast<double>(ix0), a.hx, a.x0) - M.mx) * M.isx;
    double l[K];
    if (recur && len == K)
      chunk_2d<OBJ, GRAD, F32BIN, true, K>(M, lut, u0, du, v, n, w, K, acc, flags, l);
    else
      chunk_2d<OBJ, GRAD, F32BIN, false, K>(M, lut, u0, du, v, n, w, len, acc, flags, l);
    if (a.grad_w_out) {
      if (vec && len == K) {
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
          float4 o;
          o.x = static_cast<float>(seed * l[4 * q]);
          o.y = static_cast<float>(seed * l[4 * q + 1]);
          o.z = static_cast<float>(seed * l[4 * q + 2]);
          o.w = static_cast<float>(seed * l[4 * q + 3]);
          *reinterpret_cast<float4*>(a.grad_w_out + i0 + 4 * q) = o;
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (k < len) a.grad_w_out[i0 + k] = static_cast<float>(seed * l[k]);
      }
    }
  }

  __shared__ double fac[NV];
  if (threadIdx.x < NV) fac[threadIdx.x] = M.final_factor(threadIdx.x);
  grid_publish<NV>(acc, flags | (finite ? 0 : ST_NONFINITE), fac, nullptr, a.part,
                   a.part_flags);
}

template <int OBJ, bool GRAD, bool F32BIN>
hipError_t launch_2d(const NllArgs& a, int grid, hipStream_t s, int* occ, int* block) {
  return launch_or_occupancy<kBlock>(k_nll_2d<OBJ, GRAD, F32BIN>, a, grid, s, occ, block);
}

template <int OBJ>
LaunchFn pick_2d_obj(bool grad, bool f32) {
  if (grad) return f32 ? &launch_2d<OBJ, true, true> : &launch_2d<OBJ, true, false>;
  return f32 ? &launch_2d<OBJ, false, true> : &launch_2d<OBJ, false, false>;
}

LaunchFn pick_2d(int obj, bool grad, bool f32) {
  switch (obj) {
    case OBJ_NEYMAN:
      return pick_2d_obj<OBJ_NEYMAN>(grad, f32);
    case OBJ_PEARSON:
      return pick_2d_obj<OBJ_PEARSON>(grad, f32);
    case OBJ_POISSON:
      return pick_2d_obj<OBJ_POISSON>(grad, f32);
    default:
      return nullptr;
  }
}

}  // namespace hf
