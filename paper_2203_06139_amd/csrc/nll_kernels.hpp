// nll_kernels.hpp -- objective (+ gradient) kernels over one histogram.
//
// One launch evaluates L(theta) = sum_i w_i l(n_i, mu_i(theta)) and, when GRAD,
// its reverse-mode gradient, over every bin of a 1D or 2D histogram
// (paper sec. 4, Fig. 2a: the fit objective whose parameter gradient Clad
// generates; sec. 2: reverse accumulation for a scalar function of many
// parameters).  Schedule: a grid-stride loop over 4-bin chunks (one 16-byte
// load of u32 counts per lane, so a wave reads 1 KiB contiguous), each thread
// keeping P+1 FP64 accumulators in registers, then grid_sum() for the fixed
// order reduction.  Bin centres are computed, never stored.
#pragma once

#include "device.hpp"

namespace hf {

struct NllArgs {
  const void* counts;
  const float* weights;
  int64_t nx, ny;
  int32_t dtype;
  int32_t obj;
  double x0, hx;  // centre of bin 0 and bin width along x
  double y0, hy;  // same along y (2D)
  const double* theta;
  const double* seed;
  double* nll_out;
  double* grad_out;
  float* grad_w_out;
  int32_t* status_out;
  uint32_t free_mask;
  int32_t P;
  double t_shift, t_scale;
  double* part;
  int32_t* part_flags;
  unsigned* ticket;
};

using LaunchFn = hipError_t (*)(const NllArgs&, int grid, hipStream_t);

__device__ __forceinline__ void load_counts4(const NllArgs& a, int64_t i0, double (&n)[4]) {
  if (a.dtype == DT_U32) {
    const uint4 c = *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.counts) + i0);
    n[0] = c.x;
    n[1] = c.y;
    n[2] = c.z;
    n[3] = c.w;
  } else if (a.dtype == DT_F32) {
    const float* p = static_cast<const float*>(a.counts) + i0;
#pragma unroll
    for (int k = 0; k < 4; ++k) n[k] = p[k];
  } else {
    const double* p = static_cast<const double*>(a.counts) + i0;
#pragma unroll
    for (int k = 0; k < 4; ++k) n[k] = p[k];
  }
}

__device__ __forceinline__ double load_count1(const NllArgs& a, int64_t i) {
  if (a.dtype == DT_U32) return static_cast<const uint32_t*>(a.counts)[i];
  if (a.dtype == DT_F32) return static_cast<const float*>(a.counts)[i];
  return static_cast<const double*>(a.counts)[i];
}

// Final stage shared by both kernels: the last block writes the outputs.
template <int NV, class M>
__device__ __forceinline__ void write_outputs(const NllArgs& a, const M& model, const double* tot,
                                              int totf) {
  const int k = threadIdx.x;
  if (k == 0) {
    a.nll_out[0] = tot[0];
    if (a.status_out) {
      const int nf = all_finite(a.theta, a.P) ? 0 : ST_NONFINITE;
      a.status_out[0] = totf | nf;
    }
  }
  if (NV > 1 && k >= 1 && k < NV) {
    const double seed = a.seed ? a.seed[0] : 1.0;
    const bool free = (a.free_mask == 0u) || ((a.free_mask >> (k - 1)) & 1u);
    a.grad_out[k - 1] = free ? tot[k] * model.final_factor(k) * seed : 0.0;
  }
}

template <int NG, int BKG, bool GRAD, bool F32BIN>
__global__ __launch_bounds__(kBlock) void k_nll_1d(NllArgs a) {
  using S = Shape1D<NG, BKG>;
  constexpr int NV = GRAD ? S::P + 1 : 1;
  Model1D<NG, BKG> M;
  M.init(a.theta, a.t_shift, a.t_scale);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  const int obj = a.obj;
  const double seed = (a.grad_w_out && a.seed) ? a.seed[0] : 1.0;
  const int64_t nb = a.nx;
  const int64_t nfull = nb >> 2;
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;

  for (int64_t c = tid; c < nfull; c += stride) {
    const int64_t i0 = c << 2;
    double n[4];
    load_counts4(a, i0, n);
    double w[4] = {1.0, 1.0, 1.0, 1.0};
    if (a.weights) {
      const float4 wv = *reinterpret_cast<const float4*>(a.weights + i0);
      w[0] = wv.x;
      w[1] = wv.y;
      w[2] = wv.z;
      w[3] = wv.w;
    }
    const double xb = fma(static_cast<double>(i0), a.hx, a.x0);
    double l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double x = fma(static_cast<double>(k), a.hx, xb);
      l[k] = bin_1d<NG, BKG, GRAD, F32BIN>(M, obj, x, n[k], w[k], acc, flags);
    }
    if (a.grad_w_out) {
      float4 o;
      o.x = static_cast<float>(seed * l[0]);
      o.y = static_cast<float>(seed * l[1]);
      o.z = static_cast<float>(seed * l[2]);
      o.w = static_cast<float>(seed * l[3]);
      *reinterpret_cast<float4*>(a.grad_w_out + i0) = o;
    }
  }
  // ragged tail: at most 3 bins, one per thread of the first threads
  const int64_t tail = nb - (nfull << 2);
  if (tid < tail) {
    const int64_t i = (nfull << 2) + tid;
    const double n = load_count1(a, i);
    const double w = a.weights ? static_cast<double>(a.weights[i]) : 1.0;
    const double x = fma(static_cast<double>(i), a.hx, a.x0);
    const double l = bin_1d<NG, BKG, GRAD, F32BIN>(M, obj, x, n, w, acc, flags);
    if (a.grad_w_out) a.grad_w_out[i] = static_cast<float>(seed * l);
  }

  __shared__ double tot[NV];
  __shared__ int totf;
  if (grid_sum<NV>(acc, flags, a.part, a.part_flags, a.ticket, tot, &totf))
    write_outputs<NV>(a, M, tot, totf);
}

template <int NG, int BKG, bool GRAD, bool F32BIN>
hipError_t launch_1d(const NllArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_nll_1d<NG, BKG, GRAD, F32BIN>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int NG, int BKG>
LaunchFn pick_grad_prec(bool grad, bool f32) {
  if (grad) return f32 ? &launch_1d<NG, BKG, true, true> : &launch_1d<NG, BKG, true, false>;
  return f32 ? &launch_1d<NG, BKG, false, true> : &launch_1d<NG, BKG, false, false>;
}

template <int NG>
LaunchFn pick_1d_ng(int bkg, bool grad, bool f32) {
  switch (bkg) {
    case BKG_NONE:
      if constexpr (NG == 0) return nullptr;
      else return pick_grad_prec<NG, BKG_NONE>(grad, f32);
    case 0:
      return pick_grad_prec<NG, 0>(grad, f32);
    case 1:
      return pick_grad_prec<NG, 1>(grad, f32);
    case 2:
      return pick_grad_prec<NG, 2>(grad, f32);
    case 3:
      return pick_grad_prec<NG, 3>(grad, f32);
    case BKG_EXP:
      return pick_grad_prec<NG, BKG_EXP>(grad, f32);
    default:
      return nullptr;
  }
}

// Defined in nll1d_ng{0..4}.hip and nll2d.hip.
LaunchFn pick_1d_ng0(int bkg, bool grad, bool f32);
LaunchFn pick_1d_ng1(int bkg, bool grad, bool f32);
LaunchFn pick_1d_ng2(int bkg, bool grad, bool f32);
LaunchFn pick_1d_ng3(int bkg, bool grad, bool f32);
LaunchFn pick_1d_ng4(int bkg, bool grad, bool f32);
LaunchFn pick_2d(bool grad, bool f32);

}  // namespace hf
