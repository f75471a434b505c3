// nll2d.hip -- objective (+ gradient) kernel of the correlated 2D Gaussian
// plus constant over a row-major (x fastest) 2D histogram, with optional
// per-bin weights and the per-bin weight adjoint seed * l_i (the backward of
// a differentiable objective in both theta and w).
#include "nll_kernels.hpp"

namespace hf {

// (iy, ix) of flat bin i; i < 2^53, so the FP64 quotient is off by at most
// one and the remainder test fixes it.
__device__ __forceinline__ void split_index(int64_t i, int64_t nx, double inv_nx, int64_t& iy,
                                            int64_t& ix) {
  iy = static_cast<int64_t>(static_cast<double>(i) * inv_nx);
  ix = i - iy * nx;
  if (ix < 0) {
    --iy;
    ix += nx;
  } else if (ix >= nx) {
    ++iy;
    ix -= nx;
  }
}

template <bool GRAD, bool F32BIN>
__global__ __launch_bounds__(kBlock) void k_nll_2d(NllArgs a) {
  constexpr int NV = GRAD ? 8 : 1;
  Model2D M;
  M.init(a.theta);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  const int obj = a.obj;
  const double seed = (a.grad_w_out && a.seed) ? a.seed[0] : 1.0;
  const int64_t nx = a.nx;
  const int64_t nb = a.nx * a.ny;
  const double inv_nx = 1.0 / static_cast<double>(nx);
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
    int64_t iy, ix;
    split_index(i0, nx, inv_nx, iy, ix);
    double v = (fma(static_cast<double>(iy), a.hy, a.y0) - M.my) * M.isy;
    double l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (ix == nx) {  // the chunk crosses into the next row
        ix = 0;
        ++iy;
        v = (fma(static_cast<double>(iy), a.hy, a.y0) - M.my) * M.isy;
      }
      const double u = (fma(static_cast<double>(ix), a.hx, a.x0) - M.mx) * M.isx;
      l[k] = bin_2d<GRAD, F32BIN>(M, obj, u, v, n[k], w[k], acc, flags);
      ++ix;
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
  const int64_t tail = nb - (nfull << 2);
  if (tid < tail) {
    const int64_t i = (nfull << 2) + tid;
    int64_t iy, ix;
    split_index(i, nx, inv_nx, iy, ix);
    const double n = load_count1(a, i);
    const double w = a.weights ? static_cast<double>(a.weights[i]) : 1.0;
    const double u = (fma(static_cast<double>(ix), a.hx, a.x0) - M.mx) * M.isx;
    const double v = (fma(static_cast<double>(iy), a.hy, a.y0) - M.my) * M.isy;
    const double l = bin_2d<GRAD, F32BIN>(M, obj, u, v, n, w, acc, flags);
    if (a.grad_w_out) a.grad_w_out[i] = static_cast<float>(seed * l);
  }

  __shared__ double tot[NV];
  __shared__ int totf;
  if (grid_sum<NV>(acc, flags, a.part, a.part_flags, a.ticket, tot, &totf))
    write_outputs<NV>(a, M, tot, totf);
}

template <bool GRAD, bool F32BIN>
hipError_t launch_2d(const NllArgs& a, int grid, hipStream_t s, int* occ) {
  return launch_or_occupancy(k_nll_2d<GRAD, F32BIN>, a, grid, s, occ);
}

LaunchFn pick_2d(bool grad, bool f32) {
  if (grad) return f32 ? &launch_2d<true, true> : &launch_2d<true, false>;
  return f32 ? &launch_2d<false, true> : &launch_2d<false, false>;
}

}  // namespace hf
