// finish.hip -- the finishing kernels of the objective calls and of the
// expected Hessian.
//
// The main kernel's blocks each publish their totals of the objective and
// its gradient components (grid_publish); these kernels sum them in block
// order, one block per output value, and write the outputs.  The kernel boundary orders the two:
// the partials written by the main kernel are visible here without fences,
// tickets or atomics.  Every partial of a value is requested before the
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

// One 256-thread block per output value.  Measured on the 1e7-bin workload
// (245 partials of 11 values): one 1024-thread block for all values took
// 35.7 us per call, one 256-thread block 33.5 us, a block per value 32.5 us.
constexpr int kFinishBlock = 256;

// One block per output value: block k sums the G partials of value k (thread
// t takes blocks t, t + 256, ..., all requested before the first add) and
// every block ORs all the status flags, so the NV sums run side by side.
__global__ __launch_bounds__(kFinishBlock) void k_finish_split(FinishArgs a) {
  constexpr int WAVES = kFinishBlock / 64;
  constexpr int U = 8;
  __shared__ double red[WAVES][1];
  __shared__ int redf[WAVES];
  __shared__ double tot[1];
  __shared__ int totf;
  const int k = blockIdx.x;
  const int G = a.G;
  const double seed = (k > 0 && a.seed) ? a.seed[0] : 1.0;  // requested with the partials
  const double* col = a.part + static_cast<int64_t>(k) * G;
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
    const double nan = __builtin_nan("");
    const bool finite = (totf & ST_NONFINITE) == 0;
    const bool domain = (totf & ST_DOMAIN) != 0;
    if (k == 0) {
      a.nll_out[0] = !finite ? nan : (domain ? __builtin_inf() : tot[0]);
      if (a.status_out) a.status_out[0] = totf;
    } else {
      const bool free = (a.free_mask == 0u) || ((a.free_mask >> (k - 1)) & 1u);
      a.grad_out[k - 1] = (!finite || domain) ? nan : (free ? tot[0] * seed : 0.0);
    }
  }
}

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
  hipLaunchKernelGGL(k_finish_split, dim3(a.NV), dim3(kFinishBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace hf
