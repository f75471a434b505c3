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

#include "fastmath.hpp"

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
// 1D models.  Uniform constants derived once per thread from theta.
// --------------------------------------------------------------------------
template <int NG, int BKG>
struct Model1D {
  using S = Shape1D<NG, BKG>;
  double A[NG > 0 ? NG : 1], m[NG > 0 ? NG : 1], is[NG > 0 ? NG : 1];
  double c[S::NB > 0 ? S::NB : 1];
  double tshift, ta;  // t = (x - tshift) * ta; the subtraction first keeps t exact near 0
  // Uniform-grid constants for a chunk of consecutive bins of width h:
  // dz = h/s per Gaussian, D = exp(-dz^2), dt = h/t_scale, qE = exp(b1 dt);
  // `recur` is set when every Gaussian satisfies K |dz| <= 1 and the
  // exponential background K |b1 dt| <= 1 (see chunk_1d).
  double dz[NG > 0 ? NG : 1], D[NG > 0 ? NG : 1];
  double dt;
  double qE;  // exponential background: ratio exp(b1 dt) of neighbouring bins
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
      D[g] = exp_fast(-dz[g] * dz[g]);
      recur = recur && (K * fabs(dz[g]) <= 1.0);
    }
    dt = h * ta;
    qE = 1.0;
    if constexpr (BKG == BKG_EXP) {
      // E_{k+1} = E_k exp(b1 dt): exact ratio on the grid; K |b1 dt| <= 1
      // keeps q^K within [1/e, e], so the product loses no range
      qE = exp_fast(c[1] * dt);
      recur = recur && (K * fabs(c[1] * dt) <= 1.0);
    }
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

// --------------------------------------------------------------------------
// 2D correlated Gaussian + constant.
// --------------------------------------------------------------------------
struct Model2D {
  double A, mx, my, isx, isy, rho, c, invD;
  double Dw = 0.0;  // exp(-dw^2) of the row recurrence, set by the kernel
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

// Row and column of entry e of the upper triangle of a P x P matrix,
// row-major (a <= b).
template <int P>
struct TriIndex {
  static constexpr int N = P * (P + 1) / 2;
  int a[N], b[N];
  constexpr TriIndex() : a(), b() {
    int e = 0;
    for (int r = 0; r < P; ++r)
      for (int c = r; c < P; ++c, ++e) {
        a[e] = r;
        b[e] = c;
      }
  }
};

// --------------------------------------------------------------------------
// Deterministic reductions.
// --------------------------------------------------------------------------
// One DPP move of a double (both 32-bit halves) within each row of 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes of a full wave in a fixed order; the result is
// wave-uniform.  Within each row of 16 lanes: neighbours (quad_perm
// [1,0,3,2]), pairs (quad_perm [2,3,0,1]), then rotations by 4 and 8 lanes,
// after which lane 16 r holds its row's sum; the rows combine as
// (r0 + r1) + (r2 + r3).  DPP moves and readlanes stay in the VALU, where
// the LDS round trips of lane shuffles would serialise the wave.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_row<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_row<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_row<0x124>(v);  // row_ror:4
  v += dpp_row<0x128>(v);  // row_ror:8
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sums v[0..NV) over the block; on return tot[k] holds the block total of
// component k and *totf the OR of flags.  Ends with a barrier.
template <int NV, int WAVES = kWaves>
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
    for (int w = 1; w < WAVES; ++w) s += red[w][threadIdx.x];
    tot[threadIdx.x] = s;
  }
  if (threadIdx.x == 0) {
    int o = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) o |= redf[w];
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

// Grid-wide deterministic completion of a multi-value sum in one kernel
// (used for the gradient map's shared sums, which its own kernel writes).  Every block publishes its block totals
// to part[k * G + block]; the block that takes the last ticket sums the G
// partials of each component in block order (strided over its threads, then
// the fixed block_sum tree) and returns true with the grand totals in
// tot/totf.  That block also re-arms the ticket to 0, so the counter needs
// clearing only once, when it is allocated.
//
// Ordering: the partials are written by lanes of wave 0 only (NV <= 64), and
// the same wave issues an agent-scope release fence before lane 0 takes the
// ticket; only the last block pays the acquire before reading them, and it
// requests every partial it sums before the first one is used (one memory
// round trip: a loaded value that is then added before the next load is
// requested would make one round trip per block stride).
template <int NV, int BLOCK = kBlock>
__device__ __forceinline__ bool grid_sum(double (&v)[NV], int flags, double* __restrict__ part,
                                         int* __restrict__ part_flags, unsigned* ticket,
                                         double* tot, int* totf) {
  static_assert(NV <= 64, "partials must be published by one wave");
  constexpr int WAVES = BLOCK / 64;
  __shared__ double red[WAVES][NV];
  __shared__ int redf[WAVES];
  __shared__ int is_last;
  const int G = gridDim.x;
  block_sum<NV, WAVES>(v, flags, tot, totf, red, redf);
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
  // U strides' partials are requested together (fewer for wide NV, whose
  // values already fill many registers); indices past G are clamped into
  // range and their values dropped
  constexpr int U = NV <= 17 ? 4 : 1;
  for (int b0 = 0; b0 < G; b0 += U * BLOCK) {
    double x[U][NV];
    int fl[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int b = min(b0 + q * BLOCK + static_cast<int>(threadIdx.x), G - 1);
#pragma unroll
      for (int k = 0; k < NV; ++k) x[q][k] = load_relaxed(&part[k * G + b]);
      fl[q] = load_relaxed(&part_flags[b]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const bool in = b0 + q * BLOCK + static_cast<int>(threadIdx.x) < G;
#pragma unroll
      for (int k = 0; k < NV; ++k) a[k] += in ? x[q][k] : 0.0;
      f |= in ? fl[q] : 0;
    }
  }
  block_sum<NV, WAVES>(a, f, tot, totf, red, redf);
  if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// First half of the two-kernel completion of the objective calls and the
// expected Hessian: every block sums v over its threads (fixed tree) and
// publishes
//   part[k * G + block] = total_k * fac[k] + (block 0 ? add[k] : 0)
// and its status flags; fac and add are block-shared arrays of NV values or
// null (1 and 0).  A finishing kernel (finish.hip) then sums the G partials
// of each value in block order.  Completion of the kernel makes the partials
// visible to the next one on the stream, so no fence, ticket or atomic is
// needed, and every partial is overwritten by every call.
template <int NV, int BLOCK = kBlock>
__device__ __forceinline__ void grid_publish(double (&v)[NV], int flags, const double* fac,
                                             const double* add, double* __restrict__ part,
                                             int* __restrict__ part_flags) {
  static_assert(NV <= BLOCK, "one thread per published value");
  constexpr int WAVES = BLOCK / 64;
  __shared__ double red[WAVES][NV];
  __shared__ int redf[WAVES];
  __shared__ double tot[NV];
  __shared__ int totf;
  const int G = gridDim.x;
  block_sum<NV, WAVES>(v, flags, tot, &totf, red, redf);
  const int k = threadIdx.x;
  if (k < NV) {
    double x = fac ? tot[k] * fac[k] : tot[k];
    if (add && blockIdx.x == 0) x += add[k];
    part[k * G + blockIdx.x] = x;
  }
  if (k == 0) part_flags[blockIdx.x] = totf;
}

__device__ __forceinline__ bool all_finite(const double* __restrict__ th, int P) {
  bool ok = true;
  for (int k = 0; k < P; ++k) ok = ok && (__builtin_isfinite(th[k]) != 0);
  return ok;
}

}  // namespace hf
