// nll_avg.hpp -- objective (+ gradient) kernels of the bin-average 1D model
// and of histograms with bins of any widths.
//
// Bin average: mu_i is the Gauss + polynomial model's integral over bin i
// divided by the bin width, instead of its value at the bin centre (the
// "integral of the function in the bin" form of a binned fit).  Bins of any
// widths (a.x_edges: nx + 1 ascending edges): the bin-average kernel takes
// its edges from the array, and k_nll_1d_edges evaluates the centre model
// at each bin's midpoint (one exp per Gaussian and bin: the uniform grid's
// recurrences do not apply).
//
// Per Gaussian, with edges a < b of the bin, z_x = (x - m)/s and
// e_x = exp(-z_x^2/2):
//   mu_g   = A s sqrt(pi/2) [erf(z_b/sqrt 2) - erf(z_a/sqrt 2)] / h
//   dmu/dA = s sqrt(pi/2) [erf difference] / h
//   dmu/dm = A (e_a - e_b) / h
//   dmu/ds = mu_g / s + A (z_a e_a - z_b e_b) / h
// and for the polynomial in t the exact bin averages of t^j
//   1, t_c, t_c^2 + d^2/3, t_c^3 + t_c d^2   (d = h / (2 t_scale)),
// for the exponential exp(b0 + b1 t) its exact average E_c S(b1 d) with
// E_c = exp(b0 + b1 t_c) and S(u) = sinh(u)/u (d/db1 = E_c (t_c S + d S')).
// A thread walks a chunk of consecutive bins edge to edge: each bin
// evaluates erf and exp at its right edge and hands them to the next bin, so
// a bin costs one erf and one exp per Gaussian.  On uniform bins narrower
// than a sixteenth of every width, the Gaussians' averages and partials come
// instead from a Hermite series about the bin centre, with exp at the
// centres by the two-multiply recurrence (no erf; see k_nll_1d_avg).  The objective terms, the
// reverse sweep (w ubar times the partials above) and the reduction are the
// centre model's.  FP64 only.
#pragma once

#include "chunk.hpp"
#include "nll_kernels.hpp"

namespace hf {

// Bins per thread per step of the bin-average kernel.
constexpr int kAvgChunk = 8;

// Terms of the bin-average Hermite series (see k_nll_1d_avg): at most 7.
constexpr int kHermMax = 6;

// sum_{k<=NH} He_2k(z) c_k, sum He_2k+1(z) c_k and sum_{k<=NH} He_2k+2(z) c_k
// (He by He_{n+1} = z He_n - n He_{n-1}).
template <int NH>
__device__ __forceinline__ void herm_series(double z, const double (&c)[kHermMax + 1], double& sv,
                                            double& tv, double& ux) {
  double hm = 1.0, hc = z;
  sv = c[0];
  tv = c[0] * z;
  ux = 0.0;
#pragma unroll
  for (int n = 1; n <= 2 * NH + 1; ++n) {
    const double hn = fma(z, hc, -static_cast<double>(n) * hm);  // He_{n+1}
    hm = hc;
    hc = hn;
    const int m = n + 1;
    if (m % 2 == 0) {
      if (m / 2 <= NH) sv = fma(c[m / 2], hn, sv);
      ux = fma(c[m / 2 - 1], hn, ux);
    } else if ((m - 1) / 2 <= NH) {
      tv = fma(c[(m - 1) / 2], hn, tv);
    }
  }
}

// a.x0 holds the left edge of bin 0 (not its centre) for these kernels.
// EDGES: the bins' edges come from a.x_edges (any widths), else from the
// uniform grid.
template <int NG, int BKG, int OBJ, bool GRAD, bool EDGES>
__global__ __launch_bounds__(kBlock) void k_nll_1d_avg(NllArgs a) {
  using S = Shape1D<NG, BKG>;
  constexpr int P = S::P;
  constexpr int NV = GRAD ? P + 1 : 1;
  constexpr int G1 = NG > 0 ? NG : 1;
  constexpr double kRt = 1.2533141373155002512;   // sqrt(pi/2)
  constexpr double kIr2 = 0.70710678118654752440;  // 1/sqrt(2)
  __shared__ double2 lut[OBJ == OBJ_POISSON ? kLogLut : 1];
  if constexpr (OBJ == OBJ_POISSON) log_lut_load(lut, a.log_lut);
  Model1D<NG, BKG> M;
  M.init(a.theta, a.t_shift, a.t_scale);
  double sg[G1];
#pragma unroll
  for (int g = 0; g < NG; ++g) sg[g] = a.theta[3 * g + 2];
  const double invh = 1.0 / a.hx;
  const double d = 0.5 * a.hx * M.ta;
  // Uniform bins narrow against every width (16 |dz| <= 1, dz = h/s): the
  // Gaussians' bin averages by the Hermite series about the bin centres,
  // with exp at the centres by the two-multiply recurrence, instead of erf at
  // the edges.  With phi(z) = exp(-z^2/2), phi^(n) = (-1)^n He_n phi, so over
  // a bin [z_c - delta, z_c + delta] (delta = dz/2)
  //   avg phi     = phi(z_c) sum_k He_2k(z_c)   c_k,
  //   avg z phi   = phi(z_c) sum_k He_2k+1(z_c) c_k,
  //   avg z^2 phi = phi(z_c) sum_k (He_2k+2 + He_2k)(z_c) c_k,
  // c_k = delta^2k / (2k+1)!, and mu_g = A avg phi, dmu/dm = (A/s) avg z phi,
  // dmu/ds = (A/s) avg z^2 phi.  The first omitted term is at most about
  // (13 delta)^(2N+2)/(2N+3)! relative for |z_c| <= 9 (He_n(z) <= (|z| +
  // sqrt n)^n) and phi < 3e-18 beyond; N = 1, 3 or 6 terms after the first
  // keep it below 1e-19, 1e-19 and 3e-18 for delta up to 4.5e-6, 1.6e-3 and
  // 1/32.
  bool series = !EDGES && NG > 0;
  double dmax = 0.0;
  double dzs[G1], Dz[G1], cs[G1][kHermMax + 1];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    dzs[g] = a.hx * M.is[g];
    series = series && 16.0 * fabs(dzs[g]) <= 1.0;
    dmax = fmax(dmax, 0.5 * fabs(dzs[g]));
    Dz[g] = exp_fast(-dzs[g] * dzs[g]);
    const double d2 = 0.25 * dzs[g] * dzs[g];
    cs[g][0] = 1.0;
#pragma unroll
    for (int k = 1; k <= kHermMax; ++k)
      cs[g][k] = cs[g][k - 1] * d2 / static_cast<double>((2 * k) * (2 * k + 1));
  }
  const int nh = dmax <= 4.5e-6 ? 1 : (dmax <= 1.6e-3 ? 3 : kHermMax);
  if constexpr (OBJ == OBJ_POISSON) __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  const double seed = (a.grad_w_out && a.seed) ? a.seed[0] : 1.0;  // for grad_w
  const bool finite = all_finite(a.theta, a.P);
  const int64_t nb = a.nx;
  const int64_t nch = (nb + kAvgChunk - 1) / kAvgChunk;
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t c = tid; c < nch; c += stride) {
    const int64_t i0 = c * kAvgChunk;
    const int len = static_cast<int>(nb - i0 < kAvgChunk ? nb - i0 : kAvgChunk);
    const double* __restrict__ E = EDGES ? a.x_edges : nullptr;
    // erf path: z, erf and phi at the left edge of the current bin; series
    // path: za = z at the chunk's first centre, ea = phi at the current
    // centre and Ea its ratio to the next one
    double za[G1], Ea[G1], ea[G1];
    double xa = EDGES ? E[i0] : fma(static_cast<double>(i0), a.hx, a.x0);
    if (series) {
      const double xc = fma(static_cast<double>(i0) + 0.5, a.hx, a.x0);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        za[g] = (xc - M.m[g]) * M.is[g];  // z at the first centre
        ea[g] = exp_fast(-0.5 * za[g] * za[g]);
        Ea[g] = exp_fast(fmin(fmax(fma(-dzs[g], za[g], -0.5 * dzs[g] * dzs[g]), -700.0), 700.0));
      }
    } else {
      const double x = xa;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        za[g] = (x - M.m[g]) * M.is[g];
        Ea[g] = erf(za[g] * kIr2);
        ea[g] = exp_fast(-0.5 * za[g] * za[g]);
      }
    }
    // the next bin's count, weight and right edge are requested while the
    // current bin is computed (one bin's latency hidden behind its erfs)
    double n_nx = load_count1(a, i0);
    double w_nx = a.weights ? static_cast<double>(a.weights[i0]) : 1.0;
    double xb_nx = EDGES ? E[i0 + 1] : 0.0;
    for (int k = 0; k < len; ++k) {
      const int64_t i = i0 + k;
      const double n = n_nx, w = w_nx;
      const double xb = EDGES ? xb_nx : fma(static_cast<double>(i + 1), a.hx, a.x0);
      if (k + 1 < len) {
        n_nx = load_count1(a, i + 1);
        w_nx = a.weights ? static_cast<double>(a.weights[i + 1]) : 1.0;
        if (EDGES) xb_nx = E[i + 2];
      }
      const double ih = EDGES ? 1.0 / (xb - xa) : invh;
      double mu = 0.0;
      double J[P];
      if (series) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const double z = fma(static_cast<double>(k), dzs[g], za[g]);  // centre
          double sv, tv, ux;
          if (nh == 1)
            herm_series<1>(z, cs[g], sv, tv, ux);
          else if (nh == 3)
            herm_series<3>(z, cs[g], sv, tv, ux);
          else
            herm_series<kHermMax>(z, cs[g], sv, tv, ux);
          const double es = ea[g] * sv;
          const double mg = M.A[g] * es;
          mu += mg;
          if constexpr (GRAD) {
            const double ae = M.A[g] * M.is[g] * ea[g];
            J[3 * g] = es;
            J[3 * g + 1] = ae * tv;
            J[3 * g + 2] = ae * (sv + ux);
          }
          ea[g] *= Ea[g];  // phi at the next centre
          Ea[g] *= Dz[g];
        }
      } else {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const double zb = (xb - M.m[g]) * M.is[g];
          const double Eb = erf(zb * kIr2);
          const double eb = exp_fast(-0.5 * zb * zb);
          const double ia = sg[g] * kRt * (Eb - Ea[g]) * ih;
          const double mg = M.A[g] * ia;
          mu += mg;
          if constexpr (GRAD) {
            J[3 * g] = ia;
            J[3 * g + 1] = M.A[g] * (ea[g] - eb) * ih;
            J[3 * g + 2] = fma(mg, M.is[g], M.A[g] * fma(za[g], ea[g], -zb * eb) * ih);
          }
          za[g] = zb;
          Ea[g] = Eb;
          ea[g] = eb;
        }
      }
      if constexpr (BKG == BKG_EXP) {
        const double xc = EDGES ? 0.5 * (xa + xb) : fma(static_cast<double>(i) + 0.5, a.hx, a.x0);
        const double tc = (xc - M.tshift) * M.ta;
        const double dh = EDGES ? 0.5 * (xb - xa) * M.ta : d;
        const double Ec = exp_fast(fma(M.c[1], tc, M.c[0]));
        double Sh, dSh;
        sinhc(M.c[1] * dh, Sh, dSh);
        const double eb = Ec * Sh;
        mu += eb;
        if constexpr (GRAD) {
          J[3 * NG] = eb;
          J[3 * NG + 1] = Ec * fma(tc, Sh, dh * dSh);
        }
      } else if constexpr (S::NB > 0) {
        const double xc = EDGES ? 0.5 * (xa + xb) : fma(static_cast<double>(i) + 0.5, a.hx, a.x0);
        const double tc = (xc - M.tshift) * M.ta;
        const double dh = EDGES ? 0.5 * (xb - xa) * M.ta : d;
        const double d2 = dh * dh;
        double avg[4];
        avg[0] = 1.0;
        avg[1] = tc;
        avg[2] = fma(tc, tc, d2 * (1.0 / 3.0));
        avg[3] = tc * fma(tc, tc, d2);
#pragma unroll
        for (int j = 0; j < S::NB; ++j) {
          mu = fma(M.c[j], avg[j], mu);
          if constexpr (GRAD) J[3 * NG + j] = avg[j];
        }
      }
      double l, ub;
      flags |= objective_t<OBJ, false>(n, mu, lut, l, ub) ? ST_DOMAIN : 0;
      acc[0] = fma(w, l, acc[0]);
      if constexpr (GRAD) {
        const double mb = w * ub;
#pragma unroll
        for (int p = 0; p < P; ++p) acc[1 + p] = fma(mb, J[p], acc[1 + p]);
      }
      if (a.grad_w_out) a.grad_w_out[i] = static_cast<float>(seed * l);
      xa = xb;
    }
  }
  // exact partials: no final factors
  grid_publish<NV>(acc, flags | (finite ? 0 : ST_NONFINITE), nullptr, nullptr, a.part,
                   a.part_flags);
}

// Centre model on bins of any widths: mu at each bin's midpoint, with the
// closed-form partials (A: e; m: G z; s: G z^2, the 1/s applied to the
// totals; polynomial t^j; exponential E and t E), one exp per Gaussian.
// A thread takes kEdgeChunk consecutive bins per step (their kEdgeChunk + 1
// edges are shared between neighbours), computed together so that their
// exp chains interleave, and requests the next step's edges, counts and
// weights while the current step is computed.
constexpr int kEdgeChunk = 4;

struct EdgeChunk {
  double e[kEdgeChunk + 1], n[kEdgeChunk], w[kEdgeChunk];
};

__device__ __forceinline__ void load_edge_chunk(const NllArgs& a, int64_t i0, int len,
                                                EdgeChunk& c) {
#pragma unroll
  for (int k = 0; k <= kEdgeChunk; ++k) c.e[k] = k <= len ? a.x_edges[i0 + k] : 0.0;
#pragma unroll
  for (int k = 0; k < kEdgeChunk; ++k) {
    c.n[k] = k < len ? load_count1(a, i0 + k) : 0.0;
    c.w[k] = (k < len && a.weights) ? static_cast<double>(a.weights[i0 + k]) : (k < len ? 1.0 : 0.0);
  }
}

template <int NG, int BKG, int OBJ, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_nll_1d_edges(NllArgs a) {
  using S = Shape1D<NG, BKG>;
  constexpr int P = S::P;
  constexpr int NV = GRAD ? P + 1 : 1;
  constexpr int K = kEdgeChunk;
  __shared__ double2 lut[OBJ == OBJ_POISSON ? kLogLut : 1];
  if constexpr (OBJ == OBJ_POISSON) log_lut_load(lut, a.log_lut);
  Model1D<NG, BKG> M;
  M.init(a.theta, a.t_shift, a.t_scale);
  if constexpr (OBJ == OBJ_POISSON) __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  const double seed = (a.grad_w_out && a.seed) ? a.seed[0] : 1.0;  // for grad_w
  const bool finite = all_finite(a.theta, a.P);
  const int64_t nb = a.nx;
  const int64_t nch = (nb + K - 1) / K;
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  EdgeChunk nxt;
  if (tid < nch) {
    const int64_t i0 = tid * K;
    load_edge_chunk(a, i0, static_cast<int>(nb - i0 < K ? nb - i0 : K), nxt);
  }
  for (int64_t c = tid; c < nch; c += stride) {
    const EdgeChunk cur = nxt;
    const int64_t i0 = c * K;
    const int len = static_cast<int>(nb - i0 < K ? nb - i0 : K);
    if (c + stride < nch) {
      const int64_t j0 = (c + stride) * K;
      load_edge_chunk(a, j0, static_cast<int>(nb - j0 < K ? nb - j0 : K), nxt);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool in = k < len;
      // bins past len (the last chunk) are computed at a valid point and
      // masked: their weight is 0 and their terms are dropped
      const double x = in ? 0.5 * (cur.e[k] + cur.e[k + 1]) : cur.e[0];
      double mu = 0.0;
      double J[P];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const double z = (x - M.m[g]) * M.is[g];
        const double e = exp_fast(-0.5 * z * z);
        const double G = M.A[g] * e;
        mu += G;
        if constexpr (GRAD) {
          const double Gz = G * z;
          J[3 * g] = e;
          J[3 * g + 1] = Gz;
          J[3 * g + 2] = Gz * z;
        }
      }
      const double t = (x - M.tshift) * M.ta;
      if constexpr (BKG == BKG_EXP) {
        const double Eb = exp_fast(fma(M.c[1], t, M.c[0]));
        mu += Eb;
        if constexpr (GRAD) {
          J[3 * NG] = Eb;
          J[3 * NG + 1] = t * Eb;
        }
      } else if constexpr (S::NB > 0) {
        double b = M.c[S::NB - 1];
#pragma unroll
        for (int j = S::NB - 2; j >= 0; --j) b = fma(b, t, M.c[j]);
        mu += b;
        if constexpr (GRAD) {
          double tj = 1.0;
#pragma unroll
          for (int j = 0; j < S::NB; ++j) {
            J[3 * NG + j] = tj;
            tj *= t;
          }
        }
      }
      double l, ub;
      const bool dom = objective_t<OBJ, false>(cur.n[k], mu, lut, l, ub);
      flags |= (dom && in) ? ST_DOMAIN : 0;
      l = in ? l : 0.0;
      acc[0] = fma(cur.w[k], l, acc[0]);
      if constexpr (GRAD) {
        const double mb = in ? cur.w[k] * ub : 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) acc[1 + p] = fma(mb, J[p], acc[1 + p]);
      }
      if (in && a.grad_w_out) a.grad_w_out[i0 + k] = static_cast<float>(seed * l);
    }
  }
  __shared__ double fac[NV];
  if (threadIdx.x < NV) fac[threadIdx.x] = M.final_factor(threadIdx.x);
  grid_publish<NV>(acc, flags | (finite ? 0 : ST_NONFINITE), fac, nullptr, a.part,
                   a.part_flags);
}

template <int NG, int BKG, int OBJ, bool GRAD>
hipError_t launch_1d_edges(const NllArgs& a, int grid, hipStream_t s, int* occ, int* block) {
  return launch_or_occupancy<kBlock>(k_nll_1d_edges<NG, BKG, OBJ, GRAD>, a, grid, s, occ, block);
}

template <int NG, int BKG>
LaunchFn pick_edges_obj(int obj, bool grad) {
  switch (obj) {
    case OBJ_NEYMAN:
      return grad ? &launch_1d_edges<NG, BKG, OBJ_NEYMAN, true>
                  : &launch_1d_edges<NG, BKG, OBJ_NEYMAN, false>;
    case OBJ_PEARSON:
      return grad ? &launch_1d_edges<NG, BKG, OBJ_PEARSON, true>
                  : &launch_1d_edges<NG, BKG, OBJ_PEARSON, false>;
    case OBJ_POISSON:
      return grad ? &launch_1d_edges<NG, BKG, OBJ_POISSON, true>
                  : &launch_1d_edges<NG, BKG, OBJ_POISSON, false>;
    default:
      return nullptr;
  }
}

template <int NG>
LaunchFn pick_edges_ng(int bkg, int obj, bool grad) {
  switch (bkg) {
    case BKG_NONE:
      if constexpr (NG == 0) return nullptr;
      else return pick_edges_obj<NG, BKG_NONE>(obj, grad);
    case 0:
      return pick_edges_obj<NG, 0>(obj, grad);
    case 1:
      return pick_edges_obj<NG, 1>(obj, grad);
    case 2:
      return pick_edges_obj<NG, 2>(obj, grad);
    case 3:
      return pick_edges_obj<NG, 3>(obj, grad);
    case BKG_EXP:
      return pick_edges_obj<NG, BKG_EXP>(obj, grad);
    default:
      return nullptr;
  }
}

template <int NG, int BKG, int OBJ, bool GRAD, bool EDGES>
hipError_t launch_1d_avg(const NllArgs& a, int grid, hipStream_t s, int* occ, int* block) {
  return launch_or_occupancy<kBlock>(k_nll_1d_avg<NG, BKG, OBJ, GRAD, EDGES>, a, grid, s, occ,
                                     block);
}

template <int NG, int BKG, bool EDGES>
LaunchFn pick_avg_obj_e(int obj, bool grad) {
  switch (obj) {
    case OBJ_NEYMAN:
      return grad ? &launch_1d_avg<NG, BKG, OBJ_NEYMAN, true, EDGES>
                  : &launch_1d_avg<NG, BKG, OBJ_NEYMAN, false, EDGES>;
    case OBJ_PEARSON:
      return grad ? &launch_1d_avg<NG, BKG, OBJ_PEARSON, true, EDGES>
                  : &launch_1d_avg<NG, BKG, OBJ_PEARSON, false, EDGES>;
    case OBJ_POISSON:
      return grad ? &launch_1d_avg<NG, BKG, OBJ_POISSON, true, EDGES>
                  : &launch_1d_avg<NG, BKG, OBJ_POISSON, false, EDGES>;
    default:
      return nullptr;
  }
}

template <int NG, int BKG>
LaunchFn pick_avg_obj(int obj, bool grad, bool edges) {
  return edges ? pick_avg_obj_e<NG, BKG, true>(obj, grad) : pick_avg_obj_e<NG, BKG, false>(obj, grad);
}

// bkg: the background code (polynomial degree -1..3, or BKG_EXP).
template <int NG>
LaunchFn pick_avg_ng(int bkg, int obj, bool grad, bool edges) {
  switch (bkg) {
    case -1:
      if constexpr (NG == 0) return nullptr;
      else return pick_avg_obj<NG, BKG_NONE>(obj, grad, edges);
    case 0:
      return pick_avg_obj<NG, 0>(obj, grad, edges);
    case 1:
      return pick_avg_obj<NG, 1>(obj, grad, edges);
    case 2:
      return pick_avg_obj<NG, 2>(obj, grad, edges);
    case 3:
      return pick_avg_obj<NG, 3>(obj, grad, edges);
    case BKG_EXP:
      return pick_avg_obj<NG, BKG_EXP>(obj, grad, edges);
    default:
      return nullptr;
  }
}

// Defined in nll1d_avg_ng{0..4}.hip.
LaunchFn pick_edges_ng0(int bkg, int obj, bool grad);
LaunchFn pick_edges_ng1(int bkg, int obj, bool grad);
LaunchFn pick_edges_ng2(int bkg, int obj, bool grad);
LaunchFn pick_edges_ng3(int bkg, int obj, bool grad);
LaunchFn pick_edges_ng4(int bkg, int obj, bool grad);
LaunchFn pick_avg_ng0(int bkg, int obj, bool grad, bool edges);
LaunchFn pick_avg_ng1(int bkg, int obj, bool grad, bool edges);
LaunchFn pick_avg_ng2(int bkg, int obj, bool grad, bool edges);
LaunchFn pick_avg_ng3(int bkg, int obj, bool grad, bool edges);
LaunchFn pick_avg_ng4(int bkg, int obj, bool grad, bool edges);

}  // namespace hf
