// device.hpp -- per-bin model, objective and adjoint code for gfx950, plus the
// deterministic FP64 block reduction shared by the objective and fit kernels.
//
// The per-bin code is written the way a source-transformation AD tool emits a
// reverse-mode gradient (paper sec. 3, Listing 1 and the text after it: the
// generated gradient of a device function is called from a kernel that
// supplies the parallel schedule): a forward sweep of elementary statements
// whose intermediates stay in registers, then a reverse sweep that propagates
// the adjoint of the objective term back to the parameters.  The adjoints of
// parameters shared by all bins are written by every bin -- the "parallel
// reads become parallel writes" hazard the paper names in sec. 3 -- so each
// thread accumulates them privately and the block/grid reduction below sums
// them in a fixed order (no floating-point atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

enum : int { OBJ_NEYMAN = 0, OBJ_PEARSON = 1, OBJ_POISSON = 2 };
enum : int { ST_DOMAIN = 1, ST_NONFINITE = 2 };
enum : int { DT_U32 = 0, DT_F32 = 1, DT_F64 = 2 };

// Background selector of the 1D models: -1 none, 0..3 polynomial degree,
// BKG_EXP the exponential exp(b0 + b1 t).
constexpr int BKG_NONE = -1;
constexpr int BKG_EXP = 4;

template <int NG, int BKG>
struct Shape1D {
  static constexpr int NB = (BKG == BKG_EXP) ? 2 : BKG + 1;
  static constexpr int P = 3 * NG + NB;
};

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// --------------------------------------------------------------------------
// FP32 hardware transcendentals used by the FP32-per-bin variant.  On gfx950
// FP64 FMA issues at the same rate as non-packed FP32, so that variant keeps
// ordinary arithmetic in FP64 and narrows only the steps that have cheap
// FP32 instructions: exp2, log2 and the reciprocal.
// --------------------------------------------------------------------------
__device__ __forceinline__ double exp_f32hw(double q) {
  // e^q = 2^(q log2 e); the exponent is rounded to FP32 once.
  const float y = static_cast<float>(q * 1.4426950408889634);
  return static_cast<double>(__builtin_amdgcn_exp2f(y));
}

__device__ __forceinline__ double rcp_f32hw(double d) {
  // FP32 reciprocal seed refined by one FP64 Newton step (~1e-14 relative).
  const double r0 = static_cast<double>(__builtin_amdgcn_rcpf(static_cast<float>(d)));
  return r0 * fma(-d, r0, 2.0);
}

__device__ __forceinline__ double log_f32hw(double x) {
  return 0.6931471805599453 * static_cast<double>(__builtin_amdgcn_logf(static_cast<float>(x)));
}

// r - log(1 + r) for r > -1 without cancellation: with u = r/(2+r),
// log(1+r) = 2 atanh(u) = 2(u + u^3/3 + u^5/5 + ...) and r - 2u = r u, so
// r - log1p(r) = r u - 2 u^3 (1/3 + u^2/5 + u^4/7 + ...).  The series is
// used for |u| < 1/3 (-0.5 < r < 1), the direct form elsewhere.
__device__ __forceinline__ double rmlog1p_f32hw(double r) {
  const double u = r * rcp_f32hw(2.0 + r);
  if (fabs(u) < (1.0 / 3.0)) {
    const double v = u * u;
    double p = 1.0 / 15.0;
    p = fma(p, v, 1.0 / 13.0);
    p = fma(p, v, 1.0 / 11.0);
    p = fma(p, v, 1.0 / 9.0);
    p = fma(p, v, 1.0 / 7.0);
    p = fma(p, v, 1.0 / 5.0);
    p = fma(p, v, 1.0 / 3.0);
    return fma(r, u, -2.0 * u * v * p);
  }
  return r - log_f32hw(1.0 + r);
}

// --------------------------------------------------------------------------
// Objective term l(n, mu) and its adjoint seed ubar = dl/dmu.
// Returns 0 for a regular term, 1 for a domain error (l = +inf, ubar = 0),
// 2 for a skipped bin (l = 0, ubar = 0).
// --------------------------------------------------------------------------
template <bool F32BIN>
__device__ __forceinline__ int objective(int obj, double n, double mu, double& l, double& ub) {
  if (obj == OBJ_NEYMAN) {
    if (!(n > 0.0)) {
      l = 0.0;
      ub = 0.0;
      return 2;
    }
    const double inv = F32BIN ? rcp_f32hw(n) : 1.0 / n;
    const double d = mu - n;
    l = d * d * inv;
    ub = 2.0 * d * inv;
    return 0;
  }
  if (obj == OBJ_PEARSON) {
    if (!(mu > 0.0)) {
      l = __builtin_inf();
      ub = 0.0;
      return 1;
    }
    const double inv = F32BIN ? rcp_f32hw(mu) : 1.0 / mu;
    const double d = n - mu;
    const double r = n * inv;
    l = d * d * inv;
    ub = fma(-r, r, 1.0);
    return 0;
  }
  // Poisson, saturated form
  if (n > 0.0) {
    if (!(mu > 0.0)) {
      l = __builtin_inf();
      ub = 0.0;
      return 1;
    }
    if (F32BIN) {
      // l = n (r - log1p r) with r = (mu - n)/n; ubar = (mu - n)/mu
      const double d = mu - n;
      l = n * rmlog1p_f32hw(d * rcp_f32hw(n));
      ub = d * rcp_f32hw(mu);
    } else {
      const double inv = 1.0 / mu;
      const double r = n * inv;
      l = mu - n + n * log(r);
      ub = 1.0 - r;
    }
    return 0;
  }
  if (mu < 0.0) {
    l = __builtin_inf();
    ub = 0.0;
    return 1;
  }
  l = mu;
  ub = 1.0;
  return 0;
}

// --------------------------------------------------------------------------
// 1D models.  Uniform constants derived once per thread from theta.
// --------------------------------------------------------------------------
template <int NG, int BKG>
struct Model1D {
  using S = Shape1D<NG, BKG>;
  double A[NG > 0 ? NG : 1], m[NG > 0 ? NG : 1], is[NG > 0 ? NG : 1];
  double c[S::NB > 0 ? S::NB : 1];
  double tshift, ta;  // t = (x - tshift) * ta; the subtraction first keeps t exact near 0
  // Uniform-grid constants for a chunk of consecutive bins of width h:
  // dz = h/s per Gaussian, D = exp(-dz^2), dt = h/t_scale; `recur` is set
  // when every Gaussian satisfies K |dz| <= 1 (see chunk_1d).
  double dz[NG > 0 ? NG : 1], D[NG > 0 ? NG : 1];
  double dt;
  bool recur;

  __device__ __forceinline__ void init(const double* __restrict__ th, double t_shift,
                                       double t_scale) {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      A[g] = th[3 * g];
      m[g] = th[3 * g + 1];
      is[g] = 1.0 / th[3 * g + 2];
    }
#pragma unroll
    for (int j = 0; j < S::NB; ++j) c[j] = th[3 * NG + j];
    tshift = t_shift;
    ta = 1.0 / t_scale;
  }

  __device__ __forceinline__ void init_grid(double h, int K) {
    recur = true;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      dz[g] = h * is[g];
      D[g] = exp(-dz[g] * dz[g]);
      recur = recur && (K * fabs(dz[g]) <= 1.0);
    }
    dt = h * ta;
  }

  // Factor applied to accumulated adjoint component k (0 = NLL) at the end:
  // the per-bin sweep leaves out the 1/s of dmu/dm and dmu/ds.
  __device__ __forceinline__ double final_factor(int k) const {
    if (k >= 1 && k <= 3 * NG) {
      const int p = k - 1;
      const int g = p / 3;
      if (p % 3 != 0) {
#pragma unroll
        for (int q = 0; q < NG; ++q)
          if (q == g) return is[q];
      }
    }
    return 1.0;
  }
};

// One bin of a 1D model: forward sweep, objective, reverse sweep.
// acc[0] accumulates w l; acc[1..P] the parameter adjoints (see final_factor).
template <int NG, int BKG, bool GRAD, bool F32BIN, int NV>
__device__ __forceinline__ double bin_1d(const Model1D<NG, BKG>& M, int obj, double x, double n,
                                         double w, double (&acc)[NV], int& flags) {
  using S = Shape1D<NG, BKG>;
  // ---- forward sweep ----
  double z[NG > 0 ? NG : 1], e[NG > 0 ? NG : 1], G[NG > 0 ? NG : 1];
  double mu = 0.0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    z[g] = (x - M.m[g]) * M.is[g];
    const double q = -0.5 * z[g] * z[g];
    e[g] = F32BIN ? exp_f32hw(q) : exp(q);
    G[g] = M.A[g] * e[g];
    mu += G[g];
  }
  const double t = (x - M.tshift) * M.ta;
  double E = 0.0;
  if constexpr (BKG == BKG_EXP) {
    const double a = fma(M.c[1], t, M.c[0]);
    E = F32BIN ? exp_f32hw(a) : exp(a);
    mu += E;
  } else if constexpr (S::NB > 0) {
    double b = M.c[S::NB - 1];
#pragma unroll
    for (int j = S::NB - 2; j >= 0; --j) b = fma(b, t, M.c[j]);
    mu += b;
  }
  double l, ub;
  const int rc = objective<F32BIN>(obj, n, mu, l, ub);
  flags |= (rc == 1) ? ST_DOMAIN : 0;
  acc[0] = fma(w, l, acc[0]);
  if constexpr (GRAD) {
    // ---- reverse sweep: mu_bar = w * ubar ----
    const double mb = w * ub;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      // G = A e:  A_bar += mb e ;  e_bar = mb A
      // e = exp(q): q_bar = e_bar e = mb G ; q = -z^2/2: z_bar = -q_bar z
      // z = (x - m)/s: m_bar = -z_bar/s ; s_bar = -z_bar z / s  (1/s deferred)
      acc[1 + 3 * g] = fma(mb, e[g], acc[1 + 3 * g]);
      const double zb = mb * G[g] * z[g];  // = -z_bar
      acc[2 + 3 * g] += zb;
      acc[3 + 3 * g] = fma(zb, z[g], acc[3 + 3 * g]);
    }
    constexpr int k0 = 1 + 3 * NG;
    if constexpr (BKG == BKG_EXP) {
      // E = exp(b0 + b1 t): b0_bar += mb E ; b1_bar += mb E t
      const double eb = mb * E;
      acc[k0] += eb;
      acc[k0 + 1] = fma(eb, t, acc[k0 + 1]);
    } else if constexpr (S::NB > 0) {
      double tj = mb;
#pragma unroll
      for (int j = 0; j < S::NB; ++j) {
        acc[k0 + j] += tj;
        tj *= t;
      }
    }
  }
  return l;
}

// --------------------------------------------------------------------------
// 2D correlated Gaussian + constant.
// --------------------------------------------------------------------------
struct Model2D {
  double A, mx, my, isx, isy, rho, c, invD;
  __device__ __forceinline__ void init(const double* __restrict__ th) {
    A = th[0];
    mx = th[1];
    my = th[2];
    isx = 1.0 / th[3];
    isy = 1.0 / th[4];
    rho = th[5];
    c = th[6];
    invD = 1.0 / (1.0 - rho * rho);
  }
  // order: A, mx, my, sx, sy, rho, c
  __device__ __forceinline__ double final_factor(int k) const {
    switch (k) {
      case 2:
      case 4:
        return invD * isx;
      case 3:
      case 5:
        return invD * isy;
      case 6:
        return invD;
      default:
        return 1.0;
    }
  }
};

template <bool GRAD, bool F32BIN, int NV>
__device__ __forceinline__ double bin_2d(const Model2D& M, int obj, double u, double v, double n,
                                         double w, double (&acc)[NV], int& flags) {
  // ---- forward sweep ----
  const double uv = u * v;
  const double Q = (fma(u, u, v * v) - 2.0 * M.rho * uv) * M.invD;
  const double e = F32BIN ? exp_f32hw(-0.5 * Q) : exp(-0.5 * Q);
  const double G = M.A * e;
  const double mu = G + M.c;
  double l, ub;
  const int rc = objective<F32BIN>(obj, n, mu, l, ub);
  flags |= (rc == 1) ? ST_DOMAIN : 0;
  acc[0] = fma(w, l, acc[0]);
  if constexpr (GRAD) {
    // ---- reverse sweep: mu_bar = w ubar ----
    const double mb = w * ub;
    acc[1] = fma(mb, e, acc[1]);  // A
    // Q_bar = -mu_bar G / 2;  dQ/du = 2(u - rho v)/D, dQ/dv = 2(v - rho u)/D,
    // dQ/drho = 2(rho Q - u v)/D; u = (x-mx)/sx, v = (y-my)/sy.
    const double gb = mb * G;  // = -2 Q_bar
    const double au = gb * fma(-M.rho, v, u);
    const double av = gb * fma(-M.rho, u, v);
    acc[2] += au;                               // mx  (x invD/sx)
    acc[3] += av;                               // my  (x invD/sy)
    acc[4] = fma(au, u, acc[4]);                // sx  (x invD/sx)
    acc[5] = fma(av, v, acc[5]);                // sy  (x invD/sy)
    acc[6] = fma(gb, fma(-M.rho, Q, uv), acc[6]);  // rho (x invD)
    acc[7] += mb;                               // c
  }
  return l;
}

// --------------------------------------------------------------------------
// Deterministic reductions.
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums v[0..NV) over the block; on return tot[k] holds the block total of
// component k and *totf the OR of flags.  Ends with a barrier.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], int flags, double* tot, int* totf,
                                          double (*red)[NV], int* redf) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  const int f = (__ballot(flags & ST_DOMAIN) ? ST_DOMAIN : 0) |
                (__ballot(flags & ST_NONFINITE) ? ST_NONFINITE : 0);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wid][k] = v[k];
    redf[wid] = f;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = red[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += red[w][threadIdx.x];
    tot[threadIdx.x] = s;
  }
  if (threadIdx.x == 0) {
    int o = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) o |= redf[w];
    *totf = o;
  }
  __syncthreads();
}

__device__ __forceinline__ double load_relaxed(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide deterministic completion of a multi-value sum.  Every block
// publishes its block totals to part[k * G + block]; the block that takes the
// last ticket sums the G partials of each component in block order (strided
// over its threads, then the fixed block_sum tree) and returns true with the
// grand totals in tot/totf.  That block also re-arms the ticket to 0, so the
// counter needs clearing only once, when it is allocated.
//
// Ordering: the partials are written by lanes of wave 0 only (NV <= 64), and
// the same wave issues an agent-scope release fence before lane 0 takes the
// ticket, so one L2 write-back per block publishes them; only the last block
// pays the acquire (L2 invalidate) before reading them.  A seq_cst fence in
// every wave of every block costs an order of magnitude more on gfx950.
template <int NV>
__device__ __forceinline__ bool grid_sum(double (&v)[NV], int flags, double* __restrict__ part,
                                         int* __restrict__ part_flags, unsigned* ticket,
                                         double* tot, int* totf) {
  static_assert(NV <= 64, "partials must be published by one wave");
  __shared__ double red[kWaves][NV];
  __shared__ int redf[kWaves];
  __shared__ int is_last;
  const int G = gridDim.x;
  block_sum<NV>(v, flags, tot, totf, red, redf);
  if (threadIdx.x < 64) {
    if (threadIdx.x < NV) store_relaxed(&part[threadIdx.x * G + blockIdx.x], tot[threadIdx.x]);
    if (threadIdx.x == 0) store_relaxed(&part_flags[blockIdx.x], *totf);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) {
      const unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      is_last = (t == static_cast<unsigned>(G - 1));
    }
  }
  __syncthreads();
  if (!is_last) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double a[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) a[k] = 0.0;
  int f = 0;
  for (int b = threadIdx.x; b < G; b += kBlock) {
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] += load_relaxed(&part[k * G + b]);
    f |= load_relaxed(&part_flags[b]);
  }
  block_sum<NV>(a, f, tot, totf, red, redf);
  if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

__device__ __forceinline__ bool all_finite(const double* __restrict__ th, int P) {
  bool ok = true;
  for (int k = 0; k < P; ++k) ok = ok && (__builtin_isfinite(th[k]) != 0);
  return ok;
}

}  // namespace hf
