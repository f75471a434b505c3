// fisher_kernels.hpp -- expected Hessian (Fisher information) of the binned
// objective over one histogram, and the batched inverse that turns it into
// the parameters' covariance.
//
// The paper's fit computes the gradient by reverse-mode AD and leaves the
// Hessian to numerical differentiation; moving the second derivatives to the
// GPU is the step it names next (sec. 4, the HessianPar discussion).  Near
// the minimum the second-order term of the Hessian is weighted by the
// residuals, so the Gauss-Newton / Fisher form
//   F_jk = sum_i w_i c_i (dmu_i/dtheta_j)(dmu_i/dtheta_k),
//   c_i = d^2 l/d mu^2 at n_i = mu_i: 1/mu (Poisson), 2/mu (Pearson),
//         2/n for n > 0 (Neyman),
// is the matrix a fit's parameter errors come from (bins whose c_i is not
// finite and positive are skipped).  It is a contraction over the bins of
// the per-bin Jacobian J_i = dmu_i/dtheta, J^T diag(w c) J: P(P+1)/2 FMAs
// per bin on top of the model.
//
// Schedule: the same grid-stride chunks as the objective kernel (16
// consecutive bins per thread, with the Gaussian and exponential recurrences
// when they are valid), each thread keeping up to kFisherQ entries of the
// upper triangle in registers; more entries (P > 10) take further passes
// (launches), each over all bins.  Every block publishes its totals
// (grid_publish) and a finishing kernel adds them in block order.
// On gfx950 the FP64 matrix cores have the same peak as the FP64 vector
// FMAs, and a 16x16 tile would spend 256 products per bin on the
// P(P+1)/2 = 55 (P = 10) that are needed, so the contraction stays on the
// vector units.
#pragma once

#include "device.hpp"

namespace hf {

struct FisherArgs {
  const void* counts;
  const float* weights;
  int64_t nx, ny;
  int32_t dtype;
  int32_t P;
  double x0, hx;  // centre of bin 0 and bin width along x
  double y0, hy;  // same along y (2D)
  double cfac;    // 1 (Poisson) or 2 (Pearson, Neyman): c_i = cfac / mu or cfac / n
  const double* theta;
  double* fisher_out;  // P x P, row-major
  int32_t* status_out;
  double t_shift, t_scale;
  double* part;
  int32_t* part_flags;
};

// Upper-triangle entries per pass (one block publishes at most 64).
#ifndef HF_FISHER_Q
#define HF_FISHER_Q 64
#endif
constexpr int kFisherQ = HF_FISHER_Q;
constexpr int kFisherChunk = 16;
// 4-bin groups of a 1D chunk unrolled together.  Measured on the 1e7-bin
// two-Gaussian + cubic workload: all four 64.2 us, one at a time 68.1 us.
#ifndef HF_FISHER_UNROLL
#define HF_FISHER_UNROLL 4
#endif

constexpr int fisher_passes(int P) { return (P * (P + 1) / 2 + kFisherQ - 1) / kFisherQ; }

// Launches pass `pass` with `grid` blocks; grid <= 0 instead returns through
// *occ how many blocks fit on one CU.
using FisherFn = hipError_t (*)(const FisherArgs&, int pass, int grid, hipStream_t, int* occ);

// Counts (read by the Neyman weight c = 2/n only) and weights of one chunk,
// requested together before the chunk is computed so that one memory
// latency covers all K bins.  4-byte counts travel as raw bits; FP64 counts
// are read per bin.  VEC: 16-byte loads (i0 a multiple of 4, rows 16-byte
// aligned, all K bins inside); otherwise one load per bin below len.
template <int K>
struct FisherRaw {
  uint32_t n[K];
  float w[K];
};

template <int K, bool NEY>
__device__ __forceinline__ void fisher_load(const FisherArgs& a, int64_t i0, bool vec, int len,
                                            FisherRaw<K>& r) {
  const bool cnt = NEY && a.dtype != DT_F64;
  if (vec) {
#pragma unroll
    for (int q = 0; q < K / 4; ++q) {
      if (cnt) {
        const uint4 c = reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.counts) + i0)[q];
        r.n[4 * q] = c.x;
        r.n[4 * q + 1] = c.y;
        r.n[4 * q + 2] = c.z;
        r.n[4 * q + 3] = c.w;
      }
      if (a.weights) {
        const float4 v = reinterpret_cast<const float4*>(a.weights + i0)[q];
        r.w[4 * q] = v.x;
        r.w[4 * q + 1] = v.y;
        r.w[4 * q + 2] = v.z;
        r.w[4 * q + 3] = v.w;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool in = k < len;
      if (cnt) r.n[k] = in ? static_cast<const uint32_t*>(a.counts)[i0 + k] : 0u;
      if (a.weights) r.w[k] = in ? a.weights[i0 + k] : 0.0f;
    }
  }
}

// Count and weight of bin k of a loaded chunk (`in`: k is inside the chunk;
// FP64 counts are read here, only for bins inside).
template <int K, bool NEY>
__device__ __forceinline__ void fisher_unpack(const FisherArgs& a, const FisherRaw<K>& r,
                                              int64_t i0, int k, bool in, double& n, double& w) {
  n = 0.0;
  if constexpr (NEY) {
    if (a.dtype == DT_U32) n = r.n[k];
    else if (a.dtype == DT_F32) n = __uint_as_float(r.n[k]);
    else n = in ? static_cast<const double*>(a.counts)[i0 + k] : 0.0;
  }
  w = a.weights ? static_cast<double>(r.w[k]) : 1.0;
}

__device__ __forceinline__ double fisher_count1(const FisherArgs& a, int64_t i) {
  if (a.dtype == DT_U32) return static_cast<const uint32_t*>(a.counts)[i];
  if (a.dtype == DT_F32) return static_cast<const float*>(a.counts)[i];
  return static_cast<const double*>(a.counts)[i];
}

// w c of one bin, 0 when c is not finite and positive (the bin is skipped).
template <bool NEY>
__device__ __forceinline__ double fisher_weight(double n, double mu, double w, bool& ok) {
  const double c = rcp_fast(NEY ? n : mu);
  ok = c > 0.0 && c < __builtin_inf();
  return ok ? w * c : 0.0;
}

// acc[q] += (cw J_a) J_b over the pass's entries q = E0 .. E0 + NQ - 1.
template <int P, int E0, int NQ>
__device__ __forceinline__ void fisher_rank1(const double (&J)[P], double cw, double (&acc)[NQ]) {
  constexpr TriIndex<P> tri{};
  double cJ[P];
#pragma unroll
  for (int j = 0; j < P; ++j) cJ[j] = cw * J[j];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = fma(cJ[tri.a[E0 + q]], J[tri.b[E0 + q]], acc[q]);
}

// Counts and weights of 4 consecutive bins (16-byte loads; i0 a multiple of
// 4).  FP64 counts are read per bin by fisher_nw4.
struct FisherRaw4 {
  uint4 n;
  float4 w;
};

template <bool NEY>
__device__ __forceinline__ FisherRaw4 fisher_load4(const FisherArgs& a, int64_t i0) {
  FisherRaw4 r{};
  if (NEY && a.dtype != DT_F64)
    r.n = *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.counts) + i0);
  if (a.weights) r.w = *reinterpret_cast<const float4*>(a.weights + i0);
  return r;
}

template <bool NEY>
__device__ __forceinline__ void fisher_nw4(const FisherArgs& a, const FisherRaw4& r, int kk,
                                           int64_t i, double& n, double& w) {
  const uint32_t nb = kk == 0 ? r.n.x : kk == 1 ? r.n.y : kk == 2 ? r.n.z : r.n.w;
  const float wb = kk == 0 ? r.w.x : kk == 1 ? r.w.y : kk == 2 ? r.w.z : r.w.w;
  n = 0.0;
  if constexpr (NEY) {
    if (a.dtype == DT_U32) n = nb;
    else if (a.dtype == DT_F32) n = __uint_as_float(nb);
    else n = static_cast<const double*>(a.counts)[i];
  }
  w = a.weights ? static_cast<double>(wb) : 1.0;
}

// Per-thread state of a chunk of consecutive bins of a 1D model: the
// Gaussian factors e_k = exp(-z_k^2/2) and their ratios r_k (recurrence
// e_{k+1} = e_k r_k, r_{k+1} = r_k D) and the exponential background E_k.
template <int NG, int BKG, bool RECUR>
struct FisherChunk1D {
  static constexpr int G1 = NG > 0 ? NG : 1;
  double z0[G1], e[G1], r[G1];
  double t0, Eb;
  __device__ __forceinline__ FisherChunk1D(const Model1D<NG, BKG>& M, double xs) {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      z0[g] = (xs - M.m[g]) * M.is[g];
      if constexpr (RECUR) {
        const double a0 = fmin(fmax(fma(-M.dz[g], z0[g], -0.5 * M.dz[g] * M.dz[g]), -700.0), 700.0);
        e[g] = exp_fast(-0.5 * z0[g] * z0[g]);
        r[g] = exp_fast(a0);
      }
    }
    t0 = (xs - M.tshift) * M.ta;
    Eb = 0.0;
    if constexpr (RECUR && BKG == BKG_EXP) Eb = exp_fast(fma(M.c[1], t0, M.c[0]));
  }

  // Bin k of the chunk (k counts from the chunk's first bin; bins are taken
  // in order when RECUR).  J holds dmu/dtheta without the 1/s of the
  // Gaussian mean and width columns (Model1D::final_factor, applied to the
  // totals):  A: e;  m: G z;  s: G z^2;  polynomial: t^j;  exponential:
  // E, t E.
  template <bool NEY, int E0, int NQ>
  __device__ __forceinline__ void bin(const Model1D<NG, BKG>& M, double kd, double nk, double wk,
                                      double (&acc)[NQ]) {
    using S = Shape1D<NG, BKG>;
    constexpr int P = S::P;
    double J[P];
    double mu = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const double z = fma(kd, M.dz[g], z0[g]);
      const double ek = RECUR ? e[g] : exp_fast(-0.5 * z * z);
      const double G = M.A[g] * ek;
      const double Gz = G * z;
      mu += G;
      J[3 * g] = ek;
      J[3 * g + 1] = Gz;
      J[3 * g + 2] = Gz * z;
    }
    const double t = fma(kd, M.dt, t0);
    double E = 0.0;
    if constexpr (BKG == BKG_EXP) {
      if constexpr (RECUR) {
        E = Eb;
        Eb *= M.qE;
      } else {
        E = exp_fast(fma(M.c[1], t, M.c[0]));
      }
      mu += E;
    } else if constexpr (S::NB > 0) {
      double b = M.c[S::NB - 1];
#pragma unroll
      for (int j = S::NB - 2; j >= 0; --j) b = fma(b, t, M.c[j]);
      mu += b;
      double tj = 1.0;
#pragma unroll
      for (int j = 0; j < S::NB; ++j) {
        J[3 * NG + j] = tj;
        tj *= t;
      }
    }
    bool ok;
    const double cw = fisher_weight<NEY>(nk, mu, wk, ok);
    if constexpr (BKG == BKG_EXP) {
      // an overflowing background makes mu infinite and the bin skipped;
      // its columns are zeroed so that 0 * inf does not reach the sums
      J[3 * NG] = ok ? E : 0.0;
      J[3 * NG + 1] = ok ? t * E : 0.0;
    }
    fisher_rank1<P, E0, NQ>(J, cw, acc);
    if constexpr (RECUR) {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        e[g] *= r[g];
        r[g] *= M.D[g];
      }
    }
  }
};

// One chunk of K consecutive bins (K a multiple of 4) starting at bin i0:
// groups of 4 bins, the next group's counts and weights requested while the
// current group is computed.
template <int NG, int BKG, bool NEY, bool RECUR, int K, int E0, int NQ>
__device__ __forceinline__ void fisher_chunk_1d(const FisherArgs& a, const Model1D<NG, BKG>& M,
                                                int64_t i0, double (&acc)[NQ]) {
  static_assert(K % 4 == 0, "chunk of whole 4-bin groups");
  FisherChunk1D<NG, BKG, RECUR> st(M, fma(static_cast<double>(i0), a.hx, a.x0));
  FisherRaw4 nxt = fisher_load4<NEY>(a, i0);
  // chunks without the recurrences (narrow Gaussians) go one group at a
  // time, so that their per-bin exps do not set the kernel's register count
  constexpr int U = RECUR ? HF_FISHER_UNROLL : 1;
#pragma unroll U
  for (int j = 0; j < K / 4; ++j) {
    const FisherRaw4 cur = nxt;
    if (j + 1 < K / 4) nxt = fisher_load4<NEY>(a, i0 + 4 * (j + 1));
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      double nk, wk;
      fisher_nw4<NEY>(a, cur, kk, i0 + 4 * j + kk, nk, wk);
      st.template bin<NEY, E0, NQ>(M, static_cast<double>(4 * j + kk), nk, wk, acc);
    }
  }
}

// ---------------------------------------------------------------------------
// Moment form of a recurrence chunk (every entry of F in one pass).
//
// Where the recurrences hold, every column of J is a group factor times a
// polynomial in the bin's offset k within the chunk (z = z0 + k dz,
// t = t0 + k dt):
//   Gaussian g, factor e_g:  A: 1;  m: A z;  s: A z^2
//   polynomial, factor 1:    t^j
//   exponential, factor E:   E: 1;  t E: t
// so the chunk's share of F_ab is a combination of the moments
//   M_XY,m = sum_k c_k w_k f_X,k f_Y,k u^m,   m <= deg X + deg Y,
// of the pair of groups (X, Y) the two columns belong to, in the distance
// u = K-1-k from the chunk's last bin (z = z_e - u dz, t = t_e - u dt).
// Per bin, the moments are kept in the binomial basis C(u, l) by nested
// running sums (R_l += R_{l-1} from the top, then R_0 += weight: only adds,
// no per-bin constants); once per chunk they are turned into powers of u,
// u^m = sum_l l! S(m, l) C(u, l) with S the Stirling numbers of the second
// kind, and expanded into the entries, column polynomial by column
// polynomial.  34 running sums for two Gaussians and a cubic, against 55
// entries per bin.
// ---------------------------------------------------------------------------
template <int NG, int BKG>
struct FisherMoments {
  using S = Shape1D<NG, BKG>;
  static constexpr int P = S::P;
  static constexpr bool EXPB = BKG == BKG_EXP;
  static constexpr int NGRP = NG + (S::NB > 0 ? 1 : 0);
  static constexpr int NPAIR = NGRP * (NGRP + 1) / 2;
  static constexpr int deg(int X) { return X < NG ? 2 : (S::NB > 0 ? S::NB - 1 : 0); }
  static constexpr int group(int j) { return j < 3 * NG ? j / 3 : NG; }
  static constexpr int cdeg(int j) { return j < 3 * NG ? j % 3 : j - 3 * NG; }
  static constexpr int first(int X) { return 3 * X; }  // first column of group X
  static constexpr int pair(int X, int Y) { return X * NGRP - X * (X - 1) / 2 + (Y - X); }
  static constexpr int entry(int a, int b) { return a * P - a * (a - 1) / 2 + (b - a); }
  int off[NPAIR + 1];  // first moment of each pair
  int px[NPAIR], py[NPAIR];
  constexpr FisherMoments() : off(), px(), py() {
    int p = 0, o = 0;
    for (int X = 0; X < NGRP; ++X)
      for (int Y = X; Y < NGRP; ++Y, ++p) {
        px[p] = X;
        py[p] = Y;
        off[p] = o;
        o += deg(X) + deg(Y) + 1;
      }
    off[NPAIR] = o;
  }
  static constexpr int count() {
    int o = 0;
    for (int X = 0; X < NGRP; ++X)
      for (int Y = X; Y < NGRP; ++Y) o += deg(X) + deg(Y) + 1;
    return o;
  }
  static constexpr int NMOM = count();
};

// A chunk of K consecutive bins starting at bin i0, by moments; every entry
// of F (NQ = P(P+1)/2) is accumulated into acc.
template <int NG, int BKG, bool NEY, int K, int NQ>
__device__ __forceinline__ void fisher_chunk_moments(const FisherArgs& a, const Model1D<NG, BKG>& M,
                                                     int64_t i0, double (&acc)[NQ]) {
  using FM = FisherMoments<NG, BKG>;
  using S = Shape1D<NG, BKG>;
  constexpr int P = S::P;
  constexpr int NGRP = FM::NGRP;
  constexpr int NMOM = FM::NMOM;
  constexpr FM fm{};
  static_assert(NQ == P * (P + 1) / 2, "moment form takes every entry in one pass");
  static_assert(K % 4 == 0 && K <= 16, "chunk of whole 4-bin groups");
  FisherChunk1D<NG, BKG, true> st(M, fma(static_cast<double>(i0), a.hx, a.x0));
  double mom[NMOM];
#pragma unroll
  for (int q = 0; q < NMOM; ++q) mom[q] = 0.0;
  FisherRaw4 nxt = fisher_load4<NEY>(a, i0);
#pragma unroll
  for (int j = 0; j < K / 4; ++j) {
    const FisherRaw4 cur = nxt;
    if (j + 1 < K / 4) nxt = fisher_load4<NEY>(a, i0 + 4 * (j + 1));
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * j + kk;
      double nk, wk;
      fisher_nw4<NEY>(a, cur, kk, i0 + k, nk, wk);
      double f[NGRP > 0 ? NGRP : 1];
      double mu = 0.0;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        f[g] = st.e[g];
        mu = fma(M.A[g], st.e[g], mu);
      }
      double E = 0.0;
      if constexpr (FM::EXPB) {
        E = st.Eb;
        st.Eb *= M.qE;
        mu += E;
      } else if constexpr (S::NB > 0) {
        const double t = fma(static_cast<double>(k), M.dt, st.t0);
        double b = M.c[S::NB - 1];
#pragma unroll
        for (int q = S::NB - 2; q >= 0; --q) b = fma(b, t, M.c[q]);
        mu += b;
      }
      bool ok;
      const double cw = fisher_weight<NEY>(nk, mu, wk, ok);
      if constexpr (S::NB > 0) f[NG] = FM::EXPB ? (ok ? E : 0.0) : 1.0;
      double cf[NGRP > 0 ? NGRP : 1];
#pragma unroll
      for (int X = 0; X < NGRP; ++X) cf[X] = cw * f[X];
#pragma unroll
      for (int p = 0; p < FM::NPAIR; ++p) {
        const double w = (fm.py[p] == NG && !FM::EXPB) ? cf[fm.px[p]] : cf[fm.px[p]] * f[fm.py[p]];
#pragma unroll
        for (int l = fm.off[p + 1] - fm.off[p] - 1; l >= 1; --l)
          mom[fm.off[p] + l] += mom[fm.off[p] + l - 1];
        mom[fm.off[p]] += w;
      }
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        st.e[g] *= st.r[g];
        st.r[g] *= M.D[g];
      }
    }
  }
  // binomial basis -> powers of u (m! S(m, l), m <= 6)
  constexpr double kStir[7][7] = {{1, 0, 0, 0, 0, 0, 0},        {0, 1, 0, 0, 0, 0, 0},
                                  {0, 1, 2, 0, 0, 0, 0},        {0, 1, 6, 6, 0, 0, 0},
                                  {0, 1, 14, 36, 24, 0, 0},     {0, 1, 30, 150, 240, 120, 0},
                                  {0, 1, 62, 540, 1560, 1800, 720}};
#pragma unroll
  for (int p = 0; p < FM::NPAIR; ++p) {
#pragma unroll
    for (int m = fm.off[p + 1] - fm.off[p] - 1; m >= 2; --m) {
      double v = mom[fm.off[p] + 1];
#pragma unroll
      for (int l = 2; l <= m; ++l) v = fma(kStir[m][l], mom[fm.off[p] + l], v);
      mom[fm.off[p] + m] = v;
    }
  }
  // column polynomials in u (about the chunk's last bin) and their scales
  double cc[P][4];
  double sc[P];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const double dz = -M.dz[g];
    const double z0 = fma(static_cast<double>(K - 1), M.dz[g], st.z0[g]);
    cc[3 * g][0] = 1.0;
    sc[3 * g] = 1.0;
    cc[3 * g + 1][0] = z0;
    cc[3 * g + 1][1] = dz;
    sc[3 * g + 1] = M.A[g];
    cc[3 * g + 2][0] = z0 * z0;
    cc[3 * g + 2][1] = 2.0 * z0 * dz;
    cc[3 * g + 2][2] = dz * dz;
    sc[3 * g + 2] = M.A[g];
  }
  if constexpr (S::NB > 0) {
    // (t_e - u dt)^j by the binomial theorem
    const double t0 = fma(static_cast<double>(K - 1), M.dt, st.t0), dt = -M.dt;
    double tp[S::NB], dp[S::NB];
    tp[0] = 1.0;
    dp[0] = 1.0;
#pragma unroll
    for (int j = 1; j < S::NB; ++j) {
      tp[j] = tp[j - 1] * t0;
      dp[j] = dp[j - 1] * dt;
    }
#pragma unroll
    for (int j = 0; j < S::NB; ++j) {
      double binom = 1.0;
#pragma unroll
      for (int l = 0; l <= j; ++l) {
        cc[3 * NG + j][l] = binom * tp[j - l] * dp[l];
        binom = binom * static_cast<double>(j - l) / static_cast<double>(l + 1);
      }
      sc[3 * NG + j] = 1.0;
    }
  }
  // F_ab += sc_a sc_b sum_i cc_a,i W_b,i with W_b,i = sum_j cc_b,j M_XY,i+j
#pragma unroll
  for (int b = 0; b < P; ++b) {
    const int Y = FM::group(b);
    const int db = FM::cdeg(b);
#pragma unroll
    for (int X = 0; X < NGRP; ++X) {
      if (X > Y) continue;
      const int p = FM::pair(X, Y);
      const int dX = FM::deg(X);
      double W[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i > dX) continue;
        double w = 0.0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (jj <= db) w = fma(cc[b][jj], mom[fm.off[p] + i + jj], w);
        W[i] = w;
      }
      const int a0 = FM::first(X);
      const int a1 = X < NG ? a0 + 3 : P;
#pragma unroll
      for (int aa = 0; aa < P; ++aa) {
        if (aa < a0 || aa >= a1 || aa > b) continue;
        double sv = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i <= FM::cdeg(aa)) sv = fma(cc[aa][i], W[i], sv);
        const int q = FM::entry(aa, b);
        acc[q] = fma(sc[aa] * sc[b], sv, acc[q]);
      }
    }
  }
}

// A single bin i (the ragged tail), with its own exps.
template <int NG, int BKG, bool NEY, int E0, int NQ>
__device__ __forceinline__ void fisher_bin_1d(const FisherArgs& a, const Model1D<NG, BKG>& M,
                                              int64_t i, double (&acc)[NQ]) {
  FisherChunk1D<NG, BKG, false> st(M, fma(static_cast<double>(i), a.hx, a.x0));
  const double nk = NEY ? fisher_count1(a, i) : 0.0;
  const double wk = a.weights ? static_cast<double>(a.weights[i]) : 1.0;
  st.template bin<NEY, E0, NQ>(M, 0.0, nk, wk, acc);
}

// Publishes the block's totals of the pass's entries, each already times the
// columns' final factors and cfac (grid_publish); the finishing kernel
// (launch_finish_sym) adds them in block order and writes both triangles.
// A theta that is not finite is passed on as ST_NONFINITE (NaN entries).
template <int P, int E0, int NQ, class M>
__device__ __forceinline__ void fisher_publish(const FisherArgs& a, const M& model,
                                               double (&acc)[NQ], bool finite) {
  // the columns' factors go through LDS: indexing the model's arrays with a
  // thread-dependent column would place them in scratch memory
  __shared__ double ff[P];
  __shared__ double fac[NQ];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < P; ++j) ff[j] = model.final_factor(1 + j);
  }
  __syncthreads();
  const int q = threadIdx.x;
  if (q < NQ) {
    // row r and column c of upper-triangle entry E0 + q (rows of P - r entries)
    int r = 0, e = E0 + q;
    while (e >= P - r) {
      e -= P - r;
      ++r;
    }
    fac[q] = ff[r] * ff[r + e] * a.cfac;
  }
  // (block_sum's barriers inside grid_publish order these writes before use)
  grid_publish<NQ>(acc, finite ? 0 : ST_NONFINITE, fac, nullptr, a.part, a.part_flags);
}

template <int NG, int BKG, bool NEY, int PASS>
__global__ __launch_bounds__(kBlock, 1) void k_fisher_1d(FisherArgs a) {
  constexpr int P = Shape1D<NG, BKG>::P;
  constexpr int E0 = PASS * kFisherQ;
  constexpr int NQ = (TriIndex<P>::N - E0 < kFisherQ) ? TriIndex<P>::N - E0 : kFisherQ;
  constexpr int K = kFisherChunk;
  Model1D<NG, BKG> M;
  M.init(a.theta, a.t_shift, a.t_scale);
  M.init_grid(a.hx, K);
  const bool finite = all_finite(a.theta, P);
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  const int64_t nb = a.nx;
  const int64_t nfull = nb / K;
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t c = tid; c < nfull; c += stride) {
    if (M.recur) {
      if constexpr (NQ == TriIndex<P>::N)
        fisher_chunk_moments<NG, BKG, NEY, K, NQ>(a, M, c * K, acc);
      else
        fisher_chunk_1d<NG, BKG, NEY, true, K, E0, NQ>(a, M, c * K, acc);
    } else {
      fisher_chunk_1d<NG, BKG, NEY, false, K, E0, NQ>(a, M, c * K, acc);
    }
  }
  const int64_t tail = nb - nfull * K;
  if (tid < tail) fisher_bin_1d<NG, BKG, NEY, E0, NQ>(a, M, nfull * K + tid, acc);
  fisher_publish<P, E0, NQ>(a, M, acc, finite);
}

template <int NG, int BKG, bool NEY, int PASS>
hipError_t launch_fisher_pass_1d(const FisherArgs& a, int grid, hipStream_t s, int* occ) {
  auto kern = k_fisher_1d<NG, BKG, NEY, PASS>;
  if (grid <= 0) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, kBlock, 0);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int NG, int BKG, bool NEY>
hipError_t launch_fisher_1d(const FisherArgs& a, int pass, int grid, hipStream_t s, int* occ) {
  constexpr int NP = fisher_passes(Shape1D<NG, BKG>::P);
  static_assert(NP <= 3, "P <= 16");
  switch (pass) {
    case 0:
      return launch_fisher_pass_1d<NG, BKG, NEY, 0>(a, grid, s, occ);
    case 1:
      if constexpr (NP > 1) return launch_fisher_pass_1d<NG, BKG, NEY, 1>(a, grid, s, occ);
      break;
    case 2:
      if constexpr (NP > 2) return launch_fisher_pass_1d<NG, BKG, NEY, 2>(a, grid, s, occ);
      break;
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <int NG, int BKG>
FisherFn pick_fisher_bkg(bool ney) {
  return ney ? &launch_fisher_1d<NG, BKG, true> : &launch_fisher_1d<NG, BKG, false>;
}

template <int NG>
FisherFn pick_fisher_ng(int bkg, bool ney) {
  switch (bkg) {
    case BKG_NONE:
      if constexpr (NG == 0) return nullptr;
      else return pick_fisher_bkg<NG, BKG_NONE>(ney);
    case 0:
      return pick_fisher_bkg<NG, 0>(ney);
    case 1:
      return pick_fisher_bkg<NG, 1>(ney);
    case 2:
      return pick_fisher_bkg<NG, 2>(ney);
    case 3:
      return pick_fisher_bkg<NG, 3>(ney);
    case BKG_EXP:
      return pick_fisher_bkg<NG, BKG_EXP>(ney);
    default:
      return nullptr;
  }
}

// Defined in fisher_ng{0..4}.hip and fisher2d.hip.
FisherFn pick_fisher_ng0(int bkg, bool ney);
FisherFn pick_fisher_ng1(int bkg, bool ney);
FisherFn pick_fisher_ng2(int bkg, bool ney);
FisherFn pick_fisher_ng3(int bkg, bool ney);
FisherFn pick_fisher_ng4(int bkg, bool ney);
FisherFn pick_fisher_2d(bool ney);

// Batched covariance from Fisher matrices (fisher_cov.hip): for each of B
// row-major P x P matrices, cov = scale * inverse of the free block, zero in
// the rows and columns of fixed parameters; status 1 (and NaN) when the free
// block is not safely positive definite.
hipError_t fisher_covariance(int B, int P, const double* F, uint32_t free_mask, double scale,
                             double* cov, int32_t* status, hipStream_t s);

}  // namespace hf
