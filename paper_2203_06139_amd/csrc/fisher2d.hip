// fisher2d.hip -- Fisher information of the correlated 2D Gaussian plus
// constant over a row-major (x fastest) histogram, in 16-bin pieces of one
// row like the objective kernel.
//
// dmu/dtheta with u = (x - mx)/sx, v = (y - my)/sy, D = 1 - rho^2,
// Q = (u^2 - 2 rho u v + v^2)/D, G = A exp(-Q/2):
//   A: exp(-Q/2);  mx: G (u - rho v)/(D sx);  my: G (v - rho u)/(D sy);
//   sx: G u (u - rho v)/(D sx);  sy: G v (v - rho u)/(D sy);
//   rho: G (u v - rho Q)/D;  c: 1.
// The 1/(D sx), 1/(D sy) and 1/D factors are applied to the totals
// (Model2D::final_factor).  Along a row Q = w^2 + v^2 with
// w = (u - rho v)/sqrt(D), so exp(-Q/2) follows the same two-multiply
// recurrence as the objective kernel (two exps per piece while
// 16 |dw| <= 1, dw = hx/(sx sqrt(D)); otherwise one exp per bin): a
// per-bin exp is a long chain of dependent FP64 operations, the recurrence
// one multiply per bin.
#include "fisher_kernels.hpp"

namespace hf {

// Where a 16-bin work item (piece of one row) lies.
struct Piece2D {
  int64_t i0;  // flat index of its first bin
  int64_t ix0, iy;
  int len;     // bins in the piece (the last piece of a row may be short)
  bool full;   // len == K and rows 16-byte aligned: 16-byte loads
};

template <int K>
__device__ __forceinline__ Piece2D piece_of(int64_t c, int64_t nx, int64_t cpr, double inv_cpr,
                                            bool vec) {
  Piece2D p;
  int64_t iy = static_cast<int64_t>(static_cast<double>(c) * inv_cpr);
  int64_t cx = c - iy * cpr;
  if (cx < 0) {
    --iy;
    cx += cpr;
  } else if (cx >= cpr) {
    ++iy;
    cx -= cpr;
  }
  p.iy = iy;
  p.ix0 = cx * K;
  p.len = static_cast<int>(nx - p.ix0 < K ? nx - p.ix0 : K);
  p.i0 = iy * nx + p.ix0;
  p.full = vec && p.len == K;
  return p;
}

// Counts (Neyman, 4-byte dtypes) and weights of a whole piece.
template <bool NEY, int K>
__device__ __forceinline__ void load_piece(const FisherArgs& a, const Piece2D& p,
                                           FisherRaw4 (&raw)[K / 4]) {
  if (p.full) {
#pragma unroll
    for (int j = 0; j < K / 4; ++j) raw[j] = fisher_load4<NEY>(a, p.i0 + 4 * j);
    return;
  }
  const bool cnt = NEY && a.dtype != DT_F64;
#pragma unroll
  for (int j = 0; j < K / 4; ++j) {
    raw[j] = FisherRaw4{};
    const int rem = p.len - 4 * j;
    if (cnt) {
      const uint32_t* cp = static_cast<const uint32_t*>(a.counts) + p.i0 + 4 * j;
      raw[j].n.x = rem > 0 ? cp[0] : 0u;
      raw[j].n.y = rem > 1 ? cp[1] : 0u;
      raw[j].n.z = rem > 2 ? cp[2] : 0u;
      raw[j].n.w = rem > 3 ? cp[3] : 0u;
    }
    if (a.weights) {
      const float* wp = a.weights + p.i0 + 4 * j;
      raw[j].w.x = rem > 0 ? wp[0] : 0.0f;
      raw[j].w.y = rem > 1 ? wp[1] : 0.0f;
      raw[j].w.z = rem > 2 ? wp[2] : 0.0f;
      raw[j].w.w = rem > 3 ? wp[3] : 0.0f;
    }
  }
}

// One piece of len (<= K) bins of one row starting at bin i0, with
// u0, v the standardised coordinates of its first bin.  RECUR needs
// len == K.
template <bool NEY, bool RECUR, int K, int NQ>
__device__ __forceinline__ void fisher_piece_2d(const FisherArgs& a, const Model2D& M,
                                                const Piece2D& p, const FisherRaw4 (&raw)[K / 4],
                                                double u0, double v, double du, double sqD,
                                                double (&acc)[NQ]) {
  constexpr int P = 7;
  double e = 0.0, r = 0.0;
  if constexpr (RECUR) {
    const double dw = du * sqD;
    const double w0 = (u0 - M.rho * v) * sqD;
    const double a0 = fmin(fmax(fma(-dw, w0, -0.5 * dw * dw), -700.0), 700.0);
    e = exp_fast(-0.5 * fma(w0, w0, v * v));
    r = exp_fast(a0);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool in = k < p.len;
    double n = 0.0, w = 0.0;
    if (in) fisher_nw4<NEY>(a, raw[k / 4], k % 4, p.i0 + k, n, w);
    const double u = fma(static_cast<double>(k), du, u0);
    const double uv = u * v;
    const double Q = (fma(u, u, v * v) - 2.0 * M.rho * uv) * M.invD;
    double ek;
    if constexpr (RECUR) {
      ek = e;
      e *= r;
      r *= M.Dw;
    } else {
      ek = exp_fast(-0.5 * Q);
    }
    const double G = M.A * ek;
    const double mu = G + M.c;
    double J[P];
    J[0] = ek;
    J[1] = G * fma(-M.rho, v, u);
    J[2] = G * fma(-M.rho, u, v);
    J[3] = J[1] * u;
    J[4] = J[2] * v;
    J[5] = G * fma(-M.rho, Q, uv);
    J[6] = 1.0;
    bool ok;
    const double cw = fisher_weight<NEY>(n, mu, w, ok);
    fisher_rank1<P, 0, NQ>(J, cw, acc);
  }
}

// Grid-stride loop over the pieces, the next piece's counts and weights
// requested while the current one is computed; the first piece's before the
// model set-up, so the two latencies overlap.
template <bool NEY>
__global__ __launch_bounds__(kBlock, 1) void k_fisher_2d(FisherArgs a) {
  constexpr int P = 7;
  constexpr int NQ = TriIndex<P>::N;
  constexpr int K = kFisherChunk;
  const int64_t nx = a.nx;
  const int64_t cpr = (nx + K - 1) / K;  // pieces per row
  const int64_t nitems = cpr * a.ny;
  const double inv_cpr = 1.0 / static_cast<double>(cpr);
  const bool vec = (nx % 4) == 0;  // every row starts 16-byte aligned
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  Piece2D nxp{};
  FisherRaw4 nxt[K / 4];
  if (tid < nitems) {
    nxp = piece_of<K>(tid, nx, cpr, inv_cpr, vec);
    load_piece<NEY, K>(a, nxp, nxt);
  }
  Model2D M;
  M.init(a.theta);
  const bool finite = all_finite(a.theta, P);
  const double du = a.hx * M.isx;
  const double sqD = sqrt(M.invD);
  const double dw = du * sqD;
  M.Dw = exp_fast(-dw * dw);
  const bool recur = K * fabs(dw) <= 1.0;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t c = tid; c < nitems; c += stride) {
    const Piece2D cp = nxp;
    FisherRaw4 cur[K / 4];
#pragma unroll
    for (int j = 0; j < K / 4; ++j) cur[j] = nxt[j];
    if (c + stride < nitems) {
      nxp = piece_of<K>(c + stride, nx, cpr, inv_cpr, vec);
      load_piece<NEY, K>(a, nxp, nxt);
    }
    const double v = (fma(static_cast<double>(cp.iy), a.hy, a.y0) - M.my) * M.isy;
    const double u0 = (fma(static_cast<double>(cp.ix0), a.hx, a.x0) - M.mx) * M.isx;
    if (recur && cp.len == K)
      fisher_piece_2d<NEY, true, K>(a, M, cp, cur, u0, v, du, sqD, acc);
    else
      fisher_piece_2d<NEY, false, K>(a, M, cp, cur, u0, v, du, sqD, acc);
  }
  fisher_publish<P, 0, NQ>(a, M, acc, finite);
}

template <bool NEY>
hipError_t launch_fisher_2d(const FisherArgs& a, int pass, int grid, hipStream_t s, int* occ) {
  if (pass != 0) return hipErrorInvalidValue;
  if (grid <= 0) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_fisher_2d<NEY>, kBlock, 0);
  hipLaunchKernelGGL(k_fisher_2d<NEY>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

FisherFn pick_fisher_2d(bool ney) { return ney ? &launch_fisher_2d<true> : &launch_fisher_2d<false>; }

}  // namespace hf
