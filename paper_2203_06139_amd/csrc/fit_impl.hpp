// fit_impl.hpp -- persistent batched BFGS fitter (templates).
//
// Algorithm per histogram (the optimiser step of a gradient-based fit, paper
// sec. 4; BFGS and the first-step scaling follow Nocedal & Wright,
// "Numerical Optimization", ch. 6 and eq. 6.20):
//   scaled coordinates u_k = (theta_k - theta0_k)/sigma_k for the free
//   parameters, sigma by parameter kind (amplitude max(|A0|,1), mean
//   range/100, width |s0|, background max(|c0|,1));  H = I, or with the
//   Fisher start H = inverse expected Hessian at theta0 (Gauss-Newton /
//   Fisher scoring first step; identity if it is not safely positive
//   definite);
//   repeat: p = -H g;  EDM = g^T H g / 2;  stop when EDM < max(edm_tol,
//   4 eps |f|);  if g^T p >= 0 restart from H = I;  backtracking Armijo
//   (c1 = 1e-4, alpha halved up to ls_max times; non-finite f rejected);
//   s = alpha p, y = g_new - g;  if s^T y > 1e-12 |s||y| the BFGS inverse
//   update (scaled by s^T y / y^T y before the first one after an identity
//   start).
// Finally |s| for every width, Gaussians ordered by mean, and the NLL
// re-evaluated with FP64 bins.
//
// Work split: the whole workgroup (or, for small histograms, one wave)
// evaluates the objective and gradient over the histogram's bins (chunk_1d
// in 4- or 8-bin chunks, then a fixed-order group sum); the O(P^2) BFGS
// algebra is spread over the first P or P^2 threads; scalar decisions are
// computed redundantly by every thread from the same LDS values, so control
// flow stays uniform without extra barriers.
#pragma once

#include <float.h>
#include <stdlib.h>

#include "chunk.hpp"
#include "device.hpp"
#include "fit_kernels.hpp"

namespace hf {

enum : int { FIT_CONVERGED = 0, FIT_MAXITER = 1, FIT_LSFAIL = 2, FIT_NONFINITE = 3,
             FIT_DOMAIN = 4, FIT_BADHIST = 5 };

__device__ __forceinline__ double count_at(const void* base, int dtype, int64_t i) {
  if (dtype == DT_U32) return static_cast<const uint32_t*>(base)[i];
  if (dtype == DT_F32) return static_cast<const float*>(base)[i];
  return static_cast<const double*>(base)[i];
}

// Entries of the expected Hessian accumulated per pass over the bins.
constexpr int kFisherPass = 32;

template <int NG, int BKG, int BLK>
struct FitShared {
  static constexpr int P = Shape1D<NG, BKG>::P;
  static constexpr int NV = P + 1;
  double th[P], th0[P], sig[P];
  double u[P], g[P], un[P], gn[P], pv[P], tmp[P], sv[P], yv[P], Hy[P], up[P];
  double H[P * P];   // row stride P; the leading nf x nf block is used
  double Lc[P * P];  // Fisher start: scaled F, its Cholesky factor, the inverse
  double tot[NV];
  double red[BLK / 64][NV];
  double fred[(BLK / 64) * kFisherPass];
  double ftot[kFisherPass];
  double dmax;
  int redf[BLK / 64];
  int fredf[BLK / 64];
  int totf, ftotf;
  int chol_ok;
  int fidx[P];
  int nf;
  int h;
};

// Bins per thread per step of the fit's objective sweep: 8 once every
// thread of a workgroup has a chunk of 8, else 4.  Measured on the
// 4096-histogram Gauss + exponential batch (512-thread workgroups, counts
// in LDS): one evaluation of its longest fit (22,086 bins) 15.2 us with
// 4-bin chunks, 13.5 with 8 and 15.5 with 16; reading the cached counts as
// 16-byte vectors instead of one by one, 12.1 us with 8.
constexpr int kFitChunkSmall = 4;
constexpr int kFitChunkLarge = 8;
// The 8-bin sweep is built where it fits the register budget: 512-thread
// workgroups (two waves per SIMD by construction) of one Gaussian with no,
// a constant or an exponential background, which stay below 256 VGPRs
// without spilling.  With a sloped polynomial background the 8-bin sweep
// spilled at 512 threads (32-144 bytes per lane), and at 256 threads it
// took several models to one wave per SIMD (256 VGPRs plus AGPRs), e.g.
// Gauss + line, Poisson: 0.35 -> 0.46 ms for 512 histograms of 10,000 bins.
template <int NG, int BKG, int BLK>
constexpr bool fit_chunk_large() {
  return BLK == 512 && NG == 1 && (BKG == BKG_NONE || BKG == 0 || BKG == BKG_EXP);
}

// Where a histogram's counts are read from: the workgroup's LDS cache (u32)
// or global memory (any dtype).
struct CountsSrc {
  const uint32_t* lds;  // non-null when cached (16-byte aligned)
  const void* glb;
  int dtype;
  int64_t off;
  __device__ __forceinline__ double at(int64_t i) const {
    return lds ? static_cast<double>(lds[i]) : count_at(glb, dtype, off + i);
  }
  // K consecutive counts from bin i0 (K and i0 multiples of 4)
  template <int K>
  __device__ __forceinline__ void chunk(int64_t i0, double (&n)[K]) const {
    if (lds) {
#pragma unroll
      for (int q = 0; q < K / 4; ++q) {
        const uint4 v = reinterpret_cast<const uint4*>(lds + i0)[q];
        n[4 * q] = v.x;
        n[4 * q + 1] = v.y;
        n[4 * q + 2] = v.z;
        n[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) n[k] = count_at(glb, dtype, off + i0 + k);
    }
  }
};

// The threads that run one fit: the workgroup (BLK = 256 or 512), or one
// wave (BLK = 64) for the small histograms at the end of the longest-first
// queue.  gtid is the thread's index in its group, gsync the group's
// barrier (for a wave: LDS operations stay in program order, so a fence and
// a code-motion barrier are enough), group_sum the group's fixed-order sum.
template <int BLK>
__device__ __forceinline__ int gtid() {
  return BLK == 64 ? static_cast<int>(threadIdx.x & 63u) : static_cast<int>(threadIdx.x);
}

template <int BLK>
__device__ __forceinline__ void gsync() {
  if constexpr (BLK == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int NV, int BLK>
__device__ __forceinline__ void group_sum(double (&v)[NV], int flags, double* tot, int* totf,
                                          double (*red)[NV], int* redf) {
  if constexpr (BLK == 64) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    const int f = (__ballot(flags & ST_DOMAIN) ? ST_DOMAIN : 0) |
                  (__ballot(flags & ST_NONFINITE) ? ST_NONFINITE : 0);
    if ((threadIdx.x & 63u) == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) tot[k] = v[k];
      *totf = f;
    }
    gsync<64>();
  } else {
    block_sum<NV, BLK / 64>(v, flags, tot, totf, red, redf);
  }
}

// Objective (and with GRAD its gradient) of one histogram at sm.th,
// evaluated by the whole group with the chunked sweep (chunk_1d) in K-bin
// chunks.  Leaves f in sm.tot[0] (+inf on a domain error) and dL/dtheta_k
// in sm.tot[1 + k].
template <int NG, int BKG, int OBJ, bool F32BIN, bool GRAD, int BLK, int K>
__device__ __forceinline__ void wg_eval_k(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const double2* lut, const CountsSrc& src, int64_t nb, double x0, double hx) {
  constexpr int NV = GRAD ? FitShared<NG, BKG, BLK>::NV : 1;
  Model1D<NG, BKG> M;
  M.init(sm.th, a.t_shift, a.t_scale);
  M.init_grid(hx, K);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  const int64_t nch = nb / K;
  double w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = 1.0;
  for (int64_t c = gtid<BLK>(); c < nch; c += BLK) {
    const int64_t i0 = c * K;
    double n[K];
    src.chunk<K>(i0, n);
    double l[K];
    const double xs = fma(static_cast<double>(i0), hx, x0);
    if (M.recur)
      chunk_1d<NG, BKG, OBJ, GRAD, F32BIN, true>(M, lut, xs, n, w, acc, flags, l);
    else
      chunk_1d<NG, BKG, OBJ, GRAD, F32BIN, false>(M, lut, xs, n, w, acc, flags, l);
  }
  for (int64_t i = nch * K + gtid<BLK>(); i < nb; i += BLK) {
    const double n1[1] = {src.at(i)};
    const double w1[1] = {1.0};
    double l1[1];
    chunk_1d<NG, BKG, OBJ, GRAD, F32BIN, false>(M, lut, fma(static_cast<double>(i), hx, x0), n1, w1,
                                                acc, flags, l1);
  }
  group_sum<NV, BLK>(acc, flags, sm.tot, &sm.totf, reinterpret_cast<double(*)[NV]>(sm.red),
                          sm.redf);
  if (gtid<BLK>() >= 1 && gtid<BLK>() < NV) sm.tot[gtid<BLK>()] *= M.final_factor(gtid<BLK>());
  if (gtid<BLK>() == 0 && (sm.totf & ST_DOMAIN)) sm.tot[0] = __builtin_inf();
  gsync<BLK>();
}

template <int NG, int BKG, int OBJ, bool F32BIN, bool GRAD, int BLK>
__device__ __forceinline__ void wg_eval(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const double2* lut, const CountsSrc& src, int64_t nb, double x0, double hx) {
  if constexpr (fit_chunk_large<NG, BKG, BLK>()) {
    if (nb >= static_cast<int64_t>(kFitChunkLarge) * BLK) {
      wg_eval_k<NG, BKG, OBJ, F32BIN, GRAD, BLK, kFitChunkLarge>(a, sm, lut, src, nb, x0, hx);
      return;
    }
  }
  wg_eval_k<NG, BKG, OBJ, F32BIN, GRAD, BLK, kFitChunkSmall>(a, sm, lut, src, nb, x0, hx);
}

// mu(x) and dmu/dtheta by their closed forms, one exp per Gaussian (the
// Fisher pass runs once per fit, so it does without the recurrence):
//   dG/dA = e, dG/dm = G z / s, dG/ds = G z^2 / s with z = (x - m)/s;
//   polynomial t^j; exponential E and t E.
template <int NG, int BKG>
__device__ __forceinline__ double mu_partials(const Model1D<NG, BKG>& M, double x,
                                              double (&v)[Shape1D<NG, BKG>::P]) {
  using S = Shape1D<NG, BKG>;
  double mu = 0.0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const double z = (x - M.m[g]) * M.is[g];
    const double e = exp(-0.5 * z * z);
    const double G = M.A[g] * e;
    mu += G;
    v[3 * g] = e;
    v[3 * g + 1] = G * z * M.is[g];
    v[3 * g + 2] = G * z * z * M.is[g];
  }
  const double t = (x - M.tshift) * M.ta;
  if constexpr (BKG == BKG_EXP) {
    const double E = exp(fma(M.c[1], t, M.c[0]));
    mu += E;
    v[3 * NG] = E;
    v[3 * NG + 1] = t * E;
  } else if constexpr (S::NB > 0) {
    double tj = 1.0;
#pragma unroll
    for (int j = 0; j < S::NB; ++j) {
      mu = fma(M.c[j], tj, mu);
      v[3 * NG + j] = tj;
      tj *= t;
    }
  }
  return mu;
}

// Expected Hessian at theta0, F = sum_i c_i (dmu_i/dtheta)(dmu_i/dtheta)^T
// with c_i = d^2 l/d mu^2 at n_i = mu_i (1/mu Poisson, 2/mu Pearson, 2/n for
// n > 0 Neyman); bins whose c_i is not finite and positive are skipped.  The
// upper triangle is accumulated kFisherPass entries per pass over the bins
// and written symmetrically into sm.H.
template <int NG, int BKG, int OBJ, int PASS, int BLK>
__device__ __forceinline__ void fisher_pass(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const CountsSrc& src, int64_t nb, double x0, double hx) {
  constexpr int P = FitShared<NG, BKG, BLK>::P;
  constexpr TriIndex<P> tri{};
  constexpr int E0 = PASS * kFisherPass;
  if constexpr (E0 < TriIndex<P>::N) {
    constexpr int NQ = (TriIndex<P>::N - E0 < kFisherPass) ? TriIndex<P>::N - E0 : kFisherPass;
    Model1D<NG, BKG> M;
    M.init(sm.th0, a.t_shift, a.t_scale);
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int64_t i = gtid<BLK>(); i < nb; i += BLK) {
      double v[P];
      const double mu = mu_partials(M, fma(static_cast<double>(i), hx, x0), v);
      double c;
      if constexpr (OBJ == OBJ_POISSON) c = 1.0 / mu;
      else if constexpr (OBJ == OBJ_PEARSON) c = 2.0 / mu;
      else {
        const double n = src.at(i);
        c = n > 0.0 ? 2.0 / n : 0.0;
      }
      if (c > 0.0 && __builtin_isfinite(c)) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = fma(c * v[tri.a[E0 + q]], v[tri.b[E0 + q]], acc[q]);
      }
    }
    group_sum<NQ, BLK>(acc, 0, sm.ftot, &sm.ftotf, reinterpret_cast<double(*)[NQ]>(sm.fred), sm.fredf);
    if (gtid<BLK>() < NQ) {
      const int r = tri.a[E0 + gtid<BLK>()], c = tri.b[E0 + gtid<BLK>()];
      sm.H[r * P + c] = sm.ftot[gtid<BLK>()];
      sm.H[c * P + r] = sm.ftot[gtid<BLK>()];
    }
    fisher_pass<NG, BKG, OBJ, PASS + 1, BLK>(a, sm, src, nb, x0, hx);
  }
}

// Replaces the identity in sm.H by the inverse of F_u = diag(sigma) F
// diag(sigma) over the free parameters, F already in sm.H: Cholesky
// F_u = L L^T (a pivot must exceed 1e-12 times the largest diagonal entry),
// inv(L) by forward substitution, H = inv(L)^T inv(L).  Falls back to the
// identity when F_u is not safely positive definite or anything is not
// finite.  Returns whether the inverse was taken.
template <int NG, int BKG, int BLK>
__device__ __forceinline__ bool fisher_start(FitShared<NG, BKG, BLK>& sm, int nf) {
  constexpr int P = FitShared<NG, BKG, BLK>::P;
  const int tid = gtid<BLK>();
  gsync<BLK>();
  for (int t = tid; t < nf * nf; t += BLK) {
    const int r = t / nf, c = t % nf;
    sm.Lc[r * P + c] = sm.sig[sm.fidx[r]] * sm.sig[sm.fidx[c]] * sm.H[sm.fidx[r] * P + sm.fidx[c]];
  }
  gsync<BLK>();
  if (tid == 0) {
    double dmax = 0.0;
    for (int r = 0; r < nf; ++r) dmax = fmax(dmax, sm.Lc[r * P + r]);
    sm.dmax = dmax;
    sm.chol_ok = (dmax > 0.0 && __builtin_isfinite(dmax)) ? 1 : 0;
  }
  gsync<BLK>();
  const double dmax = sm.dmax;
  for (int j = 0; j < nf && sm.chol_ok; ++j) {
    if (tid == 0) {
      double d = sm.Lc[j * P + j];
      for (int k = 0; k < j; ++k) d -= sm.Lc[j * P + k] * sm.Lc[j * P + k];
      if (!(d > 1e-12 * dmax) || !__builtin_isfinite(d)) sm.chol_ok = 0;
      else sm.Lc[j * P + j] = sqrt(d);
    }
    gsync<BLK>();
    if (sm.chol_ok && tid > j && tid < nf) {
      double v = sm.Lc[tid * P + j];
      for (int k = 0; k < j; ++k) v -= sm.Lc[tid * P + k] * sm.Lc[j * P + k];
      sm.Lc[tid * P + j] = v / sm.Lc[j * P + j];
    }
    gsync<BLK>();
  }
  if (sm.chol_ok) {
    if (tid < nf) {  // column tid of inv(L), into the lower triangle of H
      const int c = tid;
      for (int i = c; i < nf; ++i) {
        double v = (i == c) ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) v -= sm.Lc[i * P + k] * sm.H[k * P + c];
        sm.H[i * P + c] = v / sm.Lc[i * P + i];
      }
    }
    gsync<BLK>();
    for (int t = tid; t < nf * nf; t += BLK) {
      const int r = t / nf, c = t % nf;
      double v = 0.0;
      for (int k = (r > c ? r : c); k < nf; ++k) v += sm.H[k * P + r] * sm.H[k * P + c];
      sm.Lc[r * P + c] = v;
      if (!__builtin_isfinite(v)) sm.chol_ok = 0;
    }
    gsync<BLK>();
  }
  const bool ok = sm.chol_ok != 0;
  for (int t = tid; t < P * P; t += BLK) {
    const int r = t / P, c = t % P;
    sm.H[t] = (ok && r < nf && c < nf) ? sm.Lc[r * P + c] : (r == c ? 1.0 : 0.0);
  }
  gsync<BLK>();
  return ok;
}

// Sum over q < n of x[q] y[q] (or of x[q] when y is null), in order of q.
// The first P entries are loaded up front, so the LDS reads overlap instead
// of making one round trip per term.
template <int P>
__device__ __forceinline__ double dot_lds(const double* x, const double* y, int n) {
  double v[P], w[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    v[q] = x[q];
    w[q] = y ? y[q] : 1.0;
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < P; ++q)
    if (q < n) s = fma(v[q], w[q], s);
  return s;
}

// f(u) and g_u = sigma * dL/dtheta at theta = theta0 + sigma * u.
template <int NG, int BKG, int OBJ, int BLK>
__device__ __forceinline__ double wg_objective(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const double2* lut, const CountsSrc& src, const double* uu, double* gout, bool f32, int64_t nb,
    double x0, double hx) {
  constexpr int P = FitShared<NG, BKG, BLK>::P;
  const int tid = gtid<BLK>();
  if (tid < P) sm.th[tid] = sm.th0[tid];
  gsync<BLK>();
  if (tid < sm.nf) {
    const int k = sm.fidx[tid];
    sm.th[k] = fma(sm.sig[k], uu[tid], sm.th0[k]);
  }
  gsync<BLK>();
  if (f32)
    wg_eval<NG, BKG, OBJ, true, true, BLK>(a, sm, lut, src, nb, x0, hx);
  else
    wg_eval<NG, BKG, OBJ, false, true, BLK>(a, sm, lut, src, nb, x0, hx);
  if (tid < sm.nf) {
    const int k = sm.fidx[tid];
    gout[tid] = sm.sig[k] * sm.tot[1 + k];
  }
  const double f = sm.tot[0];
  gsync<BLK>();
  return f;
}

// f(u) alone (FP64 bins): the value the finite-difference gradient and its
// line search need.
template <int NG, int BKG, int OBJ, int BLK>
__device__ __forceinline__ double wg_value(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const double2* lut, const CountsSrc& src, const double* uu, int64_t nb, double x0, double hx) {
  constexpr int P = FitShared<NG, BKG, BLK>::P;
  const int tid = gtid<BLK>();
  if (tid < P) sm.th[tid] = sm.th0[tid];
  gsync<BLK>();
  if (tid < sm.nf) {
    const int k = sm.fidx[tid];
    sm.th[k] = fma(sm.sig[k], uu[tid], sm.th0[k]);
  }
  gsync<BLK>();
  wg_eval<NG, BKG, OBJ, false, false, BLK>(a, sm, lut, src, nb, x0, hx);
  const double f = sm.tot[0];
  gsync<BLK>();
  return f;
}

// Central differences in the scaled coordinates, the gradient a fitter
// without derivatives of the model uses: g_q = (f(u + h e_q) - f(u - h e_q))
// / (2h) with h = kFdStep max(1, |u_q|), 2 nf objective sweeps.
constexpr double kFdStep = 1e-4;

template <int NG, int BKG, int OBJ, int BLK>
__device__ __forceinline__ void wg_fd_grad(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const double2* lut, const CountsSrc& src, const double* uu, double* gout, int64_t nb, double x0,
    double hx) {
  const int tid = gtid<BLK>();
  const int nf = sm.nf;
  for (int q = 0; q < nf; ++q) {
    const double h = kFdStep * fmax(1.0, fabs(uu[q]));
    const double up = uu[q] + h, um = uu[q] - h;
    if (tid < nf) sm.up[tid] = (tid == q) ? up : uu[tid];
    const double fp = wg_value<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.up, nb, x0, hx);
    if (tid < nf) sm.up[tid] = (tid == q) ? um : uu[tid];
    const double fm = wg_value<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.up, nb, x0, hx);
    if (tid == 0) gout[q] = (fp - fm) / (up - um);
  }
  gsync<BLK>();
}

template <int NG, int BKG, int OBJ, int BLK>
__device__ __forceinline__ void fit_one(const FitArgs& a, FitShared<NG, BKG, BLK>& sm,
    const double2* lut, uint32_t* cache, int cache_cap, int b) {
  constexpr int P = FitShared<NG, BKG, BLK>::P;
  constexpr int NB = Shape1D<NG, BKG>::NB;
  const int tid = gtid<BLK>();
  const int64_t off = a.offsets[b];
  const int64_t nb = a.offsets[b + 1] - off;
  const double lo = a.ranges[2 * b], hi = a.ranges[2 * b + 1];
  if (!(nb >= 1) || !(hi > lo) || !__builtin_isfinite(lo) || !__builtin_isfinite(hi)) {
    if (tid < P) a.theta_out[static_cast<int64_t>(b) * P + tid] = a.theta0[static_cast<int64_t>(b) * P + tid];
    if (tid == 0) {
      a.nll_out[b] = __builtin_nan("");
      a.status[b] = FIT_BADHIST;
      a.iters[b] = 0;
      a.nevals[b] = 0;
    }
    gsync<BLK>();
    return;
  }
  const double hx = (hi - lo) / static_cast<double>(nb);
  const double x0 = lo + 0.5 * hx;
  CountsSrc src{nullptr, a.counts, a.dtype, off};
  if (a.dtype == DT_U32 && nb <= cache_cap) {  // keep the counts in LDS for all evaluations
    const uint32_t* g = static_cast<const uint32_t*>(a.counts) + off;
    for (int64_t i = tid; i < nb; i += BLK) cache[i] = g[i];
    src.lds = cache;
  }

  if (tid < P) sm.th0[tid] = a.theta0[static_cast<int64_t>(b) * P + tid];
  gsync<BLK>();
  if (tid == 0) {
    const double rx = hi - lo;
    int k = 0;
    for (int g = 0; g < NG; ++g, k += 3) {
      sm.sig[k] = fmax(fabs(sm.th0[k]), 1.0);
      sm.sig[k + 1] = rx / 100.0;
      sm.sig[k + 2] = fabs(sm.th0[k + 2]) > 0.0 ? fabs(sm.th0[k + 2]) : rx / 100.0;
    }
    for (int j = 0; j < NB; ++j) sm.sig[k + j] = fmax(fabs(sm.th0[k + j]), 1.0);
    int nf = 0;
    for (int q = 0; q < P; ++q)
      if (a.free_mask == 0u || ((a.free_mask >> q) & 1u)) sm.fidx[nf++] = q;
    sm.nf = nf;
  }
  if (tid < P) sm.u[tid] = 0.0;
  for (int t = tid; t < P * P; t += BLK) sm.H[t] = (t / P == t % P) ? 1.0 : 0.0;
  gsync<BLK>();
  const int nf = sm.nf;
  bool first = true;
  if (a.hessian_init == 1 && nf > 0) {
    fisher_pass<NG, BKG, OBJ, 0, BLK>(a, sm, src, nb, x0, hx);
    first = !fisher_start(sm, nf);  // no first-update scaling after a Fisher start
  }

  bool f32 = a.f32 != 0;
  const bool fd = a.fd_grad != 0;  // central differences (FP64 bins only)
  double f;
  int nev = 1, it = 0, status = FIT_MAXITER;
  if (fd) {
    f = wg_value<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.u, nb, x0, hx);
    if (__builtin_isfinite(f)) {
      wg_fd_grad<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.u, sm.g, nb, x0, hx);
      nev += 2 * nf;
    }
  } else {
    f = wg_objective<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.u, sm.g, f32, nb, x0, hx);
  }
  if (!__builtin_isfinite(f)) {
    status = (f == __builtin_inf()) ? FIT_DOMAIN : FIT_NONFINITE;
  } else {
    while (it < a.max_iter) {
      if (tid < nf) {
        double hg = 0.0;
        hg = dot_lds<P>(&sm.H[tid * P], sm.g, nf);
        sm.pv[tid] = -hg;
        sm.tmp[tid] = sm.g[tid] * hg;
      }
      gsync<BLK>();
      double edm = 0.0;
      edm = dot_lds<P>(sm.tmp, nullptr, nf);
      edm *= 0.5;
      const double goal = fmax(a.edm_tol, 4.0 * DBL_EPSILON * fabs(f));
      if (f32 && a.polish_edm > 0.0 && edm < a.polish_edm) {
        // switch to FP64 bins for the rest of the fit
        f32 = false;
        f = wg_objective<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.u, sm.g, false, nb, x0, hx);
        ++nev;
        if (!__builtin_isfinite(f)) {
          status = (f == __builtin_inf()) ? FIT_DOMAIN : FIT_NONFINITE;
          break;
        }
        continue;
      }
      if (!a.fixed_iters && edm < goal) {
        status = FIT_CONVERGED;
        break;
      }
      double slope = 0.0;
      slope = dot_lds<P>(sm.g, sm.pv, nf);
      if (!(slope < 0.0)) {  // H lost positive definiteness: restart from I
        gsync<BLK>();
        for (int t = tid; t < P * P; t += BLK) sm.H[t] = (t / P == t % P) ? 1.0 : 0.0;
        if (tid < nf) sm.pv[tid] = -sm.g[tid];
        first = true;
        gsync<BLK>();
        slope = 0.0;
        slope = -dot_lds<P>(sm.g, sm.g, nf);
      }
      double alpha = 1.0, fn = 0.0;
      bool accepted = false;
      for (int ls = 0; ls < a.ls_max; ++ls) {
        if (tid < nf) sm.un[tid] = sm.u[tid] + alpha * sm.pv[tid];
        gsync<BLK>();
        fn = fd ? wg_value<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.un, nb, x0, hx)
                : wg_objective<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.un, sm.gn, f32, nb, x0, hx);
        ++nev;
        if (__builtin_isfinite(fn) && fn <= f + 1e-4 * alpha * slope) {
          accepted = true;
          break;
        }
        alpha *= 0.5;
      }
      if (!accepted) {
        status = (edm < goal) ? FIT_CONVERGED : FIT_LSFAIL;
        break;
      }
      ++it;
      if (fd) {  // the gradient only at the accepted point
        wg_fd_grad<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.un, sm.gn, nb, x0, hx);
        nev += 2 * nf;
      }
      if (tid < nf) {
        sm.sv[tid] = sm.un[tid] - sm.u[tid];
        sm.yv[tid] = sm.gn[tid] - sm.g[tid];
      }
      gsync<BLK>();
      const double sy = dot_lds<P>(sm.sv, sm.yv, nf);
      const double yy = dot_lds<P>(sm.yv, sm.yv, nf);
      const double ss = dot_lds<P>(sm.sv, sm.sv, nf);
      if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
        if (first) {
          const double gam = sy / yy;
          for (int t = tid; t < nf * nf; t += BLK) sm.H[(t / nf) * P + t % nf] *= gam;
          first = false;
          gsync<BLK>();
        }
        if (tid < nf) {
          double hy = 0.0;
          hy = dot_lds<P>(&sm.H[tid * P], sm.yv, nf);
          sm.Hy[tid] = hy;
        }
        gsync<BLK>();
        double yHy = 0.0;
        yHy = dot_lds<P>(sm.yv, sm.Hy, nf);
        const double rho = 1.0 / sy;
        const double cc = rho * rho * yHy + rho;
        for (int t = tid; t < nf * nf; t += BLK) {
          const int r = t / nf, c = t % nf;
          sm.H[r * P + c] += -rho * (sm.Hy[r] * sm.sv[c] + sm.sv[r] * sm.Hy[c]) + cc * sm.sv[r] * sm.sv[c];
        }
      }
      if (tid < nf) {
        sm.u[tid] = sm.un[tid];
        sm.g[tid] = sm.gn[tid];
      }
      gsync<BLK>();
      f = fn;
    }
  }
  double nll = f;
  if (f32 && __builtin_isfinite(f)) nll = wg_objective<NG, BKG, OBJ, BLK>(a, sm, lut, src, sm.u, sm.gn, false, nb, x0, hx);
  // final parameters, canonicalised
  if (tid < P) sm.th[tid] = sm.th0[tid];
  gsync<BLK>();
  if (tid < nf) {
    const int k = sm.fidx[tid];
    sm.th[k] = fma(sm.sig[k], sm.u[tid], sm.th0[k]);
  }
  gsync<BLK>();
  if (tid == 0) {
    for (int g = 0; g < NG; ++g) sm.th[3 * g + 2] = fabs(sm.th[3 * g + 2]);
    for (int p = 1; p < NG; ++p)
      for (int q = p; q > 0 && sm.th[3 * q + 1] < sm.th[3 * (q - 1) + 1]; --q)
        for (int r = 0; r < 3; ++r) {
          const double t = sm.th[3 * q + r];
          sm.th[3 * q + r] = sm.th[3 * (q - 1) + r];
          sm.th[3 * (q - 1) + r] = t;
        }
    a.nll_out[b] = nll;
    a.status[b] = status;
    a.iters[b] = it;
    a.nevals[b] = nev;
  }
  gsync<BLK>();
  if (tid < P) a.theta_out[static_cast<int64_t>(b) * P + tid] = sm.th[tid];
  gsync<BLK>();
}

// Bytes of dynamic LDS one wave takes in wave mode: its fit state, then an
// LDS copy of up to wave_bins u32 counts, each rounded up to 16 bytes so
// that every slot's counts start 16-byte aligned.
template <int NG, int BKG>
constexpr size_t wave_slot_bytes(int wave_bins) {
  return ((sizeof(FitShared<NG, BKG, 64>) + 15) / 16) * 16 +
         ((4 * static_cast<size_t>(wave_bins) + 15) / 16) * 16;
}

template <int NG, int BKG, int OBJ, int BLK>
__global__ __launch_bounds__(BLK) void k_fit(FitArgs a) {
  __shared__ FitShared<NG, BKG, BLK> sm;
  __shared__ double2 lut[OBJ == OBJ_POISSON ? kLogLut : 1];
  // the workgroup's count cache, or the waves' slots
  extern __shared__ __attribute__((aligned(16))) uint32_t cache[];
  const int tid = threadIdx.x;
  if constexpr (OBJ == OBJ_POISSON) log_lut_load(lut, a.log_lut);
  // wave mode needs the longest-first order: the first histogram of at most
  // wave_bins bins is followed by smaller ones only
  const bool waves = a.wave_bins > 0 && a.sorted;
  int h;
  for (;;) {
    if (tid == 0) sm.h = static_cast<int>(atomicAdd(&a.counters[0], 1u));
    __syncthreads();
    h = sm.h;
    __syncthreads();
    if (h >= a.B) break;
    const int b = a.sorted ? a.order[h] : h;
    if (waves && a.offsets[b + 1] - a.offsets[b] <= a.wave_bins) break;
    fit_one<NG, BKG, OBJ, BLK>(a, sm, lut, cache, a.cache_bins, b);
  }
  if (waves && h < a.B) {
    // from here on every wave fits its own histograms: wave 0 the one just
    // taken, the others and every later one from the queue
    const int w = tid >> 6;
    char* slot = reinterpret_cast<char*>(cache) + w * wave_slot_bytes<NG, BKG>(a.wave_bins);
    auto& sw = *reinterpret_cast<FitShared<NG, BKG, 64>*>(slot);
    uint32_t* wc = reinterpret_cast<uint32_t*>(slot + wave_slot_bytes<NG, BKG>(0));
    int hw = h;
    if (w != 0) {
      int t = 0;
      if ((tid & 63) == 0) t = static_cast<int>(atomicAdd(&a.counters[0], 1u));
      hw = __shfl(t, 0);
    }
    while (hw < a.B) {
      fit_one<NG, BKG, OBJ, 64>(a, sw, lut, wc, a.wave_bins, a.order[hw]);
      int t = 0;
      if ((tid & 63) == 0) t = static_cast<int>(atomicAdd(&a.counters[0], 1u));
      hw = __shfl(t, 0);
    }
  }
  __syncthreads();  // every wave is past the queue before the workgroup leaves
  // the last workgroup to leave re-arms the queue for the next launch
  if (tid == 0) {
    __threadfence();
    const unsigned d = atomicAdd(&a.counters[1], 1u);
    if (d == gridDim.x - 1) {
      atomicExch(&a.counters[0], 0u);
      atomicExch(&a.counters[1], 0u);
    }
  }
}

template <int NG, int BKG, int OBJ, int BLK>
hipError_t launch_fit_kernel(const FitArgs& a, int grid, hipStream_t s, int* max_cache) {
  if (grid <= 0) {
    // grid 0: the largest dynamic LDS cache (u32 bins) that still fits;
    // grid -1: the largest wave_bins whose per-wave slots fit
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(k_fit<NG, BKG, OBJ, BLK>));
    if (e != hipSuccess) return e;
    int dev = 0, lds = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    const long free_bytes = static_cast<long>(lds) - static_cast<long>(attr.sharedSizeBytes);
    if (grid == 0) {
      *max_cache = static_cast<int>(free_bytes / 4);
    } else {
      const long per_wave = free_bytes / (BLK / 64) - static_cast<long>(wave_slot_bytes<NG, BKG>(0));
      *max_cache = per_wave > 0 ? static_cast<int>(per_wave / 16) * 4 : 0;
    }
    return hipSuccess;
  }
  size_t dyn = sizeof(uint32_t) * static_cast<size_t>(a.cache_bins);
  if (a.wave_bins > 0) {
    const size_t w = (BLK / 64) * wave_slot_bytes<NG, BKG>(a.wave_bins);
    dyn = w > dyn ? w : dyn;
  }
  hipLaunchKernelGGL((k_fit<NG, BKG, OBJ, BLK>), dim3(grid), dim3(BLK), dyn, s, a);
  return hipGetLastError();
}

using FitLaunchFn = hipError_t (*)(const FitArgs&, int, hipStream_t, int*);

// Workgroup sizes the fitter is built for: 256 threads (one wave per SIMD)
// or 512 (two), the second for batches whose longest fits set the time.
template <int NG, int BKG, int OBJ>
FitLaunchFn pick_fit_blk(int blk) {
  if (blk == 256) return &launch_fit_kernel<NG, BKG, OBJ, 256>;
  if (blk == 512) return &launch_fit_kernel<NG, BKG, OBJ, 512>;
  return nullptr;
}

template <int NG, int BKG>
FitLaunchFn pick_fit_obj(int obj, int blk) {
  switch (obj) {
    case OBJ_NEYMAN:
      return pick_fit_blk<NG, BKG, OBJ_NEYMAN>(blk);
    case OBJ_PEARSON:
      return pick_fit_blk<NG, BKG, OBJ_PEARSON>(blk);
    case OBJ_POISSON:
      return pick_fit_blk<NG, BKG, OBJ_POISSON>(blk);
    default:
      return nullptr;
  }
}

template <int NG>
FitLaunchFn pick_fit_ng(int bkg, int obj, int blk) {
  switch (bkg) {
    case BKG_NONE:
      if constexpr (NG == 0) return nullptr;
      else return pick_fit_obj<NG, BKG_NONE>(obj, blk);
    case 0:
      return pick_fit_obj<NG, 0>(obj, blk);
    case 1:
      return pick_fit_obj<NG, 1>(obj, blk);
    case 2:
      return pick_fit_obj<NG, 2>(obj, blk);
    case 3:
      return pick_fit_obj<NG, 3>(obj, blk);
    case BKG_EXP:
      return pick_fit_obj<NG, BKG_EXP>(obj, blk);
    default:
      return nullptr;
  }
}

FitLaunchFn pick_fit_ng0(int bkg, int obj, int blk);
FitLaunchFn pick_fit_ng1(int bkg, int obj, int blk);
FitLaunchFn pick_fit_ng2(int bkg, int obj, int blk);
FitLaunchFn pick_fit_ng3(int bkg, int obj, int blk);
FitLaunchFn pick_fit_ng4(int bkg, int obj, int blk);

}  // namespace hf
