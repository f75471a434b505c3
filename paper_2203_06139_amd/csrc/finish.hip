// finish.hip -- the finishing kernels of the objective calls and of the
// expected Hessian.
//
// The main kernel's blocks each publish their totals of the objective and
// its gradient components (grid_publish); this one-block kernel sums them in
// block order and writes the outputs.  The kernel boundary orders the two:
// the partials written by the main kernel are visible here without fences,
// tickets or atomics.  Every partial of a component is requested before the
// first one is added, so the sum costs one memory round trip.
//
// Outputs (as nll_eval / nll_grad document them): a status bit ST_NONFINITE
// (theta not finite) makes every output NaN; ST_DOMAIN (a bin outside the
// objective's domain) makes L = +inf and the gradient NaN, since L has no
// gradient there; otherwise L = sum, dL/dtheta_k = seed * sum_k, and 0 for
// parameters whose free_mask bit is clear.
#include "device.hpp"
#include "finish.hpp"

namespace hf {

namespace {

// 256 threads: with 1024 the finishing kernel took 1.8 us longer per call on
// the 1e7-bin workload (245 partials), the block reduction over 16 waves
// outweighing the shorter load loop.
constexpr int kFinishBlock = 256;

// Adds this thread's partials of blocks b0 + threadIdx.x + q kFinishBlock,
// q < Q, all requested before the first is added.
template <int NV, int Q>
__device__ __forceinline__ void load_partials(const FinishArgs& a, int b0, double (&v)[NV],
                                              int& f) {
  const int G = a.G;
  double x[Q][NV];
  int fl[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    // clamped into range; the select below drops what lies past G
    const int b = min(b0 + static_cast<int>(threadIdx.x) + q * kFinishBlock, G - 1);
#pragma unroll
    for (int k = 0; k < NV; ++k) x[q][k] = a.part[k * G + b];
    fl[q] = a.part_flags[b];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const bool in = b0 + static_cast<int>(threadIdx.x) + q * kFinishBlock < G;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += in ? x[q][k] : 0.0;
    f |= in ? fl[q] : 0;
  }
}

template <int NV>
__global__ __launch_bounds__(kFinishBlock) void k_finish_objective(FinishArgs a) {
  constexpr int WAVES = kFinishBlock / 64;
  __shared__ double red[WAVES][NV];
  __shared__ int redf[WAVES];
  __shared__ double tot[NV];
  __shared__ int totf;
  const double seed = a.seed ? a.seed[0] : 1.0;  // requested with the partials
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  int f = 0;
  const int nq = (a.G + kFinishBlock - 1) / kFinishBlock;
  if (nq <= 1) {
    load_partials<NV, 1>(a, 0, v, f);
  } else if (nq <= 2) {
    load_partials<NV, 2>(a, 0, v, f);
  } else if (nq <= 4) {
    load_partials<NV, 4>(a, 0, v, f);
  } else {
    for (int b0 = 0; b0 < a.G; b0 += 8 * kFinishBlock) load_partials<NV, 8>(a, b0, v, f);
  }
  block_sum<NV, WAVES>(v, f, tot, &totf, red, redf);
  const int k = threadIdx.x;
  const double nan = __builtin_nan("");
  const bool finite = (totf & ST_NONFINITE) == 0;
  const bool domain = (totf & ST_DOMAIN) != 0;
  if (k == 0) {
    a.nll_out[0] = !finite ? nan : (domain ? __builtin_inf() : tot[0]);
    if (a.status_out) a.status_out[0] = totf;
  }
  if (NV > 1 && k >= 1 && k < NV) {
    const bool free = (a.free_mask == 0u) || ((a.free_mask >> (k - 1)) & 1u);
    a.grad_out[k - 1] = (!finite || domain) ? nan : (free ? tot[k] * seed : 0.0);
  }
}

template <int NV>
hipError_t launch_nv(const FinishArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_objective<NV>, dim3(1), dim3(kFinishBlock), 0, s, a);
  return hipGetLastError();
}

using FinishFn = hipError_t (*)(const FinishArgs&, hipStream_t);

constexpr FinishFn kFinish[18] = {
    nullptr,        &launch_nv<1>,  &launch_nv<2>,  &launch_nv<3>,  &launch_nv<4>,
    &launch_nv<5>,  &launch_nv<6>,  &launch_nv<7>,  &launch_nv<8>,  &launch_nv<9>,
    &launch_nv<10>, &launch_nv<11>, &launch_nv<12>, &launch_nv<13>, &launch_nv<14>,
    &launch_nv<15>, &launch_nv<16>, &launch_nv<17>};

// One block per entry: the block's threads take the G partials in a fixed
// assignment (thread t: blocks t, t + 256, ...), all requested before the
// first add, and block_sum adds them up.
__global__ __launch_bounds__(kFinishBlock) void k_finish_sym(FinishSymArgs a) {
  constexpr int WAVES = kFinishBlock / 64;
  constexpr int U = 8;
  __shared__ double red[WAVES][1];
  __shared__ int redf[WAVES];
  __shared__ double tot[1];
  __shared__ int totf;
  const int q = blockIdx.x;
  const int G = a.G;
  const double* col = a.part + static_cast<int64_t>(q) * G;
  double v[1] = {0.0};
  int f = 0;
  for (int b0 = 0; b0 < G; b0 += U * kFinishBlock) {
    double x[U];
    int fl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = min(b0 + static_cast<int>(threadIdx.x) + u * kFinishBlock, G - 1);
      x[u] = col[b];
      fl[u] = a.part_flags[b];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = b0 + static_cast<int>(threadIdx.x) + u * kFinishBlock < G;
      v[0] += in ? x[u] : 0.0;
      f |= in ? fl[u] : 0;
    }
  }
  block_sum<1, WAVES>(v, f, tot, &totf, red, redf);
  if (threadIdx.x == 0) {
    int r = 0, e = a.E0 + q;
    while (e >= a.P - r) {
      e -= a.P - r;
      ++r;
    }
    const int c = r + e;
    const bool finite = (totf & ST_NONFINITE) == 0;
    const double val = finite ? tot[0] : __builtin_nan("");
    a.out[r * a.P + c] = val;
    a.out[c * a.P + r] = val;
    if (q == 0 && a.E0 == 0 && a.status_out) a.status_out[0] = finite ? 0 : ST_NONFINITE;
  }
}

}  // namespace

hipError_t launch_finish_sym(const FinishSymArgs& a, hipStream_t s) {
  if (a.G < 1 || a.NQ < 1 || a.P < 1 || a.E0 < 0 || a.E0 + a.NQ > a.P * (a.P + 1) / 2 || !a.out)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finish_sym, dim3(a.NQ), dim3(kFinishBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs& a, hipStream_t s) {
  if (a.NV < 1 || a.NV > 17 || a.G < 1) return hipErrorInvalidValue;
  if (a.NV > 1 && !a.grad_out) return hipErrorInvalidValue;
  return kFinish[a.NV](a, s);
}

}  // namespace hf
