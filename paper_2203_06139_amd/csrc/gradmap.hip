// gradmap.hip -- elementwise Gaussian and its reverse-mode gradient over N
// independent parameter sets (the device-function example of paper sec. 3,
// Listing 1, generalised).
//
// Per element i, with d = x_i - p_i and s = sigma_i:
//   g_i = (2 pi)^(-1/2) s^(-a) exp(t),  t = -d^2 / (2 s^2),
//   a = 1/2 (the normalisation as the listing prints it) or 1 (the normal pdf);
//   reverse sweep with upstream adjoint w_i (seed_i, or 1):
//     x_bar = w g (-d / s^2),  p_bar = -x_bar,
//     s_bar = w g (d^2 / s^3 - a / s).
// Per-element inputs give per-element adjoints: no two elements write the
// same output, so the map is a pure stream (8 bytes per input and output per
// element), bound by HBM.  When p or sigma is one value shared by every
// element, the listing's parallel reads of it become parallel writes of its
// adjoint (the hazard the paper names in sec. 3): that adjoint is then a sum
// over the elements, taken with the fixed-order grid reduction instead of
// atomics.
#include "device.hpp"
#include "gradmap.hpp"

namespace hf {

__device__ __forceinline__ void gradmap_point(const GradMapArgs& a, double x, double p, double s,
                                              double w, double& g, double& gx, double& gs) {
  const double d = x - p;
  const double is = 1.0 / s;
  const double is2 = is * is;
  const double t = -0.5 * d * d * is2;
  constexpr double kInvSqrt2Pi = 0.39894228040143267794;
  const bool pdf = a.norm == GRADMAP_NORM_PDF;
  const double cn = pdf ? kInvSqrt2Pi * is : kInvSqrt2Pi / sqrt(s);
  g = cn * exp_fast(t);
  const double wg = w * g;
  gx = -wg * d * is2;
  gs = wg * is * fma(d * d, is2, pdf ? -1.0 : -0.5);
}

// One element: loads, evaluation, stores; shared-input adjoints go to acc.
template <bool PSH, bool SSH>
__device__ __forceinline__ void gradmap_one(const GradMapArgs& a, int64_t i, double p0, double s0,
                                            double (&acc)[2]) {
  const double x = a.x[i];
  const double p = PSH ? p0 : a.p[i];
  const double s = SSH ? s0 : a.sigma[i];
  const double w = a.seed ? a.seed[i] : 1.0;
  double g, gx, gs;
  gradmap_point(a, x, p, s, w, g, gx, gs);
  if (a.g) a.g[i] = g;
  if (a.dx) a.dx[i] = gx;
  if (PSH) acc[0] -= gx;
  else if (a.dp) a.dp[i] = -gx;
  if (SSH) acc[1] += gs;
  else if (a.ds) a.ds[i] = gs;
}

// Pairs of consecutive elements with 16-byte loads and stores (every array
// 16-byte aligned).  A thread takes kPairs pairs per step, pair u of step c
// being c * kPairs * stride + u * stride + tid: each load instruction of a
// wave reads 1 KiB contiguous, and all of a step's loads are in flight before
// its first element is computed (a thread streams 16-32 bytes per element
// for about 40 FP64 operations, so the loads' latency, not the arithmetic,
// sets the pace).
// Measured on 2^27 elements (listing configuration / every input and output
// per element): 8 pairs 837 / 1579 us, 4 pairs 950 / 1654 us, 2 pairs
// 820 / 1673 us.
#ifndef HF_GM_PAIRS
#define HF_GM_PAIRS 8
#endif
constexpr int kPairs = HF_GM_PAIRS;

// Non-temporal loads and stores (each element is touched once): measured on
// 2^27 elements, 937 vs 997 us for the listing's configuration, 1653 vs 1682
// us with every input and output per element.
#ifndef HF_GRADMAP_NT
#define HF_GRADMAP_NT 1
#endif
typedef double gm_d2 __attribute__((ext_vector_type(2)));

// 16-byte store of (u, v) at p and 16-byte load, non-temporal with
// HF_GRADMAP_NT.
__device__ __forceinline__ void store2(double* p, double u, double v) {
  gm_d2 t;
  t.x = u;
  t.y = v;
  if (HF_GRADMAP_NT)
    __builtin_nontemporal_store(t, reinterpret_cast<gm_d2*>(p));
  else
    *reinterpret_cast<gm_d2*>(p) = t;
}

__device__ __forceinline__ double2 load2(const double* p) {
  if (HF_GRADMAP_NT) {
    const gm_d2 t = __builtin_nontemporal_load(reinterpret_cast<const gm_d2*>(p));
    return make_double2(t.x, t.y);
  }
  return *reinterpret_cast<const double2*>(p);
}

template <bool PSH, bool SSH>
__device__ __forceinline__ void gradmap_pairs(const GradMapArgs& a, int64_t q0, int64_t stride,
                                              int64_t npair, double p0, double s0, bool redp,
                                              bool reds, double (&acc)[2]) {
  const double* __restrict__ xa = a.x;
  const double* __restrict__ pa = a.p;
  const double* __restrict__ sa = a.sigma;
  const double* __restrict__ wa = a.seed;
  double2 x[kPairs], p[kPairs], s[kPairs], w[kPairs];
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int64_t q = q0 + u * stride;
    if (q < npair) {
      x[u] = load2(xa + 2 * q);
      p[u] = PSH ? make_double2(p0, p0) : load2(pa + 2 * q);
      s[u] = SSH ? make_double2(s0, s0) : load2(sa + 2 * q);
      w[u] = wa ? load2(wa + 2 * q) : make_double2(1.0, 1.0);
    }
  }
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int64_t q = q0 + u * stride;
    if (q >= npair) continue;
    const int64_t i = 2 * q;
    double2 g, gx, gs;
    gradmap_point(a, x[u].x, p[u].x, s[u].x, w[u].x, g.x, gx.x, gs.x);
    gradmap_point(a, x[u].y, p[u].y, s[u].y, w[u].y, g.y, gx.y, gs.y);
    if (a.g) store2(a.g + i, g.x, g.y);
    if (a.dx) store2(a.dx + i, gx.x, gx.y);
    if (PSH) {
      if (redp) acc[0] -= gx.x + gx.y;
    } else if (a.dp) {
      store2(a.dp + i, -gx.x, -gx.y);
    }
    if (SSH) {
      if (reds) acc[1] += gs.x + gs.y;
    } else if (a.ds) {
      store2(a.ds + i, gs.x, gs.y);
    }
  }
}

template <bool PSH, bool SSH, bool VEC>
__global__ __launch_bounds__(kBlock) void k_gauss_grad_map(GradMapArgs a) {
  // a shared input's adjoint is reduced only when it is asked for
  const bool redp = PSH && a.dp, reds = SSH && a.ds;
  const double p0 = PSH ? a.p[0] : 0.0;
  const double s0 = SSH ? a.sigma[0] : 0.0;
  double acc[2] = {0.0, 0.0};
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  if constexpr (VEC) {
    const int64_t npair = a.n / 2;
    for (int64_t q0 = tid; q0 < npair; q0 += kPairs * stride)
      gradmap_pairs<PSH, SSH>(a, q0, stride, npair, p0, s0, redp, reds, acc);
    if ((a.n & 1) && tid == 0) gradmap_one<PSH, SSH>(a, a.n - 1, p0, s0, acc);
  } else {
    for (int64_t i = tid; i < a.n; i += stride) gradmap_one<PSH, SSH>(a, i, p0, s0, acc);
  }
  if (redp || reds) {
    __shared__ double tot[2];
    __shared__ int totf;
    if (grid_sum<2>(acc, 0, a.part, a.part_flags, a.ticket, tot, &totf) && threadIdx.x == 0) {
      if (redp) a.dp[0] = tot[0];
      if (reds) a.ds[0] = tot[1];
    }
  }
}

// Blocks of one variant that fit on a CU at once (queried once per variant).
template <bool PSH, bool SSH, bool VEC>
int gradmap_occupancy() {
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_gauss_grad_map<PSH, SSH, VEC>, kBlock,
                                                     0) != hipSuccess || o < 1)
      o = 1;
    return o;
  }();
  return occ;
}

// One round of resident blocks (no more than the work needs), each thread
// streaming kPairs pairs per step.
template <bool PSH, bool SSH, bool VEC>
hipError_t launch_gradmap(const GradMapArgs& a, int num_cu, int max_grid, hipStream_t s) {
  const int64_t per_thread_step = VEC ? 2 * kPairs : 1;
  const int64_t need = (a.n + per_thread_step * kBlock - 1) / (per_thread_step * kBlock);
  int64_t grid = static_cast<int64_t>(num_cu) * gradmap_occupancy<PSH, SSH, VEC>();
  if (grid > need) grid = need;
  if (grid > max_grid) grid = max_grid;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_gauss_grad_map<PSH, SSH, VEC>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <bool PSH, bool SSH>
hipError_t launch_gradmap_v(const GradMapArgs& a, bool vec, int num_cu, int max_grid,
                            hipStream_t s) {
  return vec ? launch_gradmap<PSH, SSH, true>(a, num_cu, max_grid, s)
             : launch_gradmap<PSH, SSH, false>(a, num_cu, max_grid, s);
}

hipError_t gauss_grad_map(const GradMapArgs& a, bool vec, int num_cu, int max_grid, hipStream_t s) {
  if (a.p_shared) {
    return a.sigma_shared ? launch_gradmap_v<true, true>(a, vec, num_cu, max_grid, s)
                          : launch_gradmap_v<true, false>(a, vec, num_cu, max_grid, s);
  }
  return a.sigma_shared ? launch_gradmap_v<false, true>(a, vec, num_cu, max_grid, s)
                        : launch_gradmap_v<false, false>(a, vec, num_cu, max_grid, s);
}

}  // namespace hf
