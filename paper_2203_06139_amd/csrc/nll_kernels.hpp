// nll_kernels.hpp -- objective (+ gradient) kernels over one histogram.
//
// One launch evaluates L(theta) = sum_i w_i l(n_i, mu_i(theta)) and, when GRAD,
// its reverse-mode gradient, over every bin of a 1D or 2D histogram
// (paper sec. 4, Fig. 2a: the fit objective whose parameter gradient Clad
// generates; sec. 2: reverse accumulation for a scalar function of many
// parameters).  Schedule: a grid-stride loop over 16-bin chunks (16-byte
// loads of u32 counts), each thread keeping P+1 FP64 accumulators in
// registers; every block publishes its totals (grid_publish) and the
// finishing kernel (finish.hip) adds them in block order.  Bin centres are
// computed, never stored.
#pragma once

#include "chunk.hpp"
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
  const double2* log_lut;  // kLogLut entries, see log_lut_entry
  const double* x_edges;   // 1D bins of any widths: nx + 1 ascending edges, or null
};

// Launches a kernel variant with `grid` blocks; grid <= 0 instead returns,
// through *occ, how many blocks of that kernel fit on one CU at once, and
// through *block its threads per block.  The main kernel only publishes
// per-block partials (grid_publish); the caller launches the finishing
// kernel (launch_finish) after it.
using LaunchFn = hipError_t (*)(const NllArgs&, int grid, hipStream_t, int* occ, int* block);

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

// Bins per thread per step (K) and waves per SIMD (W) the 1D kernel is built
// for.  Every bin of a chunk is interleaved with the others, so registers
// grow with K.  Measured with every call reading its 1e7 bins from HBM:
//   two Gaussians + cubic, Poisson: 16 bins at two waves per SIMD (256
//     VGPRs, a few spilled outside the chunk loop) 44.0 us, at one wave
//     47.3 us; 12 bins at two waves 59.7 us (12-bin chunks win only while
//     the histogram stays in the last-level cache);
//   other Poisson models with up to two Gaussians: two waves 1-3% faster;
//   two Gaussians + line, Neyman (no log, about half the work per bin):
//     two waves 41.8 us, one wave 27.0 us.
// So two waves for the Poisson objective with up to two Gaussians, one wave
// otherwise (three or more Gaussians need well over 256 VGPRs at 16 bins).
// K is a multiple of 4 (16-byte loads).
// Threads per block (BLOCK): 64 x 4 SIMDs x W, so one block fills a CU at
// the kernel's occupancy and the grid has one block per CU (half as many
// partials to publish and sum as two 256-thread blocks).
template <int NG, int OBJ>
struct Chunking {
  static constexpr int K = 16;
  static constexpr int W = (NG <= 2 && OBJ == OBJ_POISSON) ? 2 : 1;
  static constexpr int BLOCK = 256 * W;
  static_assert(K % 4 == 0, "chunk must be a multiple of 4 bins");
};
constexpr int chunk_bins(int) { return 16; }
constexpr int kMinWaves = 1;  // the 2D kernel: one wave per SIMD

// Counts of one chunk as loaded: 4-byte dtypes travel as raw 16-byte vectors
// so the next chunk can be fetched while the current one is computed.
template <int K>
struct ChunkRaw {
  uint4 c[K / 4];
  float4 w[K / 4];
};

template <bool SPEC, int K>
__device__ __forceinline__ void load_raw(const NllArgs& a, int64_t i0, ChunkRaw<K>& r) {
  const uint4* cp = reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.counts) + i0);
#pragma unroll
  for (int q = 0; q < K / 4; ++q) r.c[q] = cp[q];
  if (!SPEC && a.weights) {
    const float4* wp = reinterpret_cast<const float4*>(a.weights + i0);
#pragma unroll
    for (int q = 0; q < K / 4; ++q) r.w[q] = wp[q];
  }
}

// SPEC: the counts are u32 and there are no weights (the common case, with
// the conversions and weight products folded away); otherwise the dtype and
// the weights are checked at run time.
template <bool SPEC, int K>
__device__ __forceinline__ void unpack_raw(const NllArgs& a, const ChunkRaw<K>& r, double (&n)[K],
                                           double (&w)[K]) {
#pragma unroll
  for (int q = 0; q < K / 4; ++q) {
    if (SPEC || a.dtype == DT_U32) {
      n[4 * q] = r.c[q].x;
      n[4 * q + 1] = r.c[q].y;
      n[4 * q + 2] = r.c[q].z;
      n[4 * q + 3] = r.c[q].w;
    } else {
      n[4 * q] = __uint_as_float(r.c[q].x);
      n[4 * q + 1] = __uint_as_float(r.c[q].y);
      n[4 * q + 2] = __uint_as_float(r.c[q].z);
      n[4 * q + 3] = __uint_as_float(r.c[q].w);
    }
    if (!SPEC && a.weights) {
      w[4 * q] = r.w[q].x;
      w[4 * q + 1] = r.w[q].y;
      w[4 * q + 2] = r.w[q].z;
      w[4 * q + 3] = r.w[q].w;
    } else {
      w[4 * q] = w[4 * q + 1] = w[4 * q + 2] = w[4 * q + 3] = 1.0;
    }
  }
}

template <int NG, int BKG, int OBJ, bool GRAD, bool F32BIN, int K, int NV>
__device__ __forceinline__ void chunk_step(const NllArgs& a, const Model1D<NG, BKG>& M,
                                           const double2* lut, int64_t i0, const double (&n)[K],
                                           const double (&w)[K], double seed,
                                           double (&acc)[NV], int& flags) {
  const double xs = fma(static_cast<double>(i0), a.hx, a.x0);
  double l[K];
  if (M.recur)
    chunk_1d<NG, BKG, OBJ, GRAD, F32BIN, true>(M, lut, xs, n, w, acc, flags, l);
  else
    chunk_1d<NG, BKG, OBJ, GRAD, F32BIN, false>(M, lut, xs, n, w, acc, flags, l);
  if (a.grad_w_out) {
#pragma unroll
    for (int q = 0; q < K / 4; ++q) {
      float4 o;
      o.x = static_cast<float>(seed * l[4 * q]);
      o.y = static_cast<float>(seed * l[4 * q + 1]);
      o.z = static_cast<float>(seed * l[4 * q + 2]);
      o.w = static_cast<float>(seed * l[4 * q + 3]);
      reinterpret_cast<float4*>(a.grad_w_out + i0)[q] = o;
    }
  }
}

// Grid-stride loop over the full chunks of 4-byte counts, with the next chunk
// loaded while the current one is computed.  `nxt` holds the thread's first
// chunk (chunk tid), loaded by the caller when tid < nfull.
template <int NG, int BKG, int OBJ, bool GRAD, bool F32BIN, bool SPEC, int K, int NV>
__device__ __forceinline__ void stream_chunks(const NllArgs& a, const Model1D<NG, BKG>& M,
                                              const double2* lut, int64_t nfull, int64_t tid,
                                              int64_t stride, double seed, ChunkRaw<K> nxt,
                                              double (&acc)[NV], int& flags) {
  for (int64_t c = tid; c < nfull; c += stride) {
    const ChunkRaw<K> cur = nxt;
    if (c + stride < nfull) load_raw<SPEC>(a, (c + stride) * K, nxt);
    double n[K], w[K];
    unpack_raw<SPEC>(a, cur, n, w);
    chunk_step<NG, BKG, OBJ, GRAD, F32BIN>(a, M, lut, c * K, n, w, seed, acc, flags);
  }
}

template <int NG, int BKG, int OBJ, bool GRAD, bool F32BIN>
__global__ __launch_bounds__((Chunking<NG, OBJ>::BLOCK), (Chunking<NG, OBJ>::W)) void k_nll_1d(
    NllArgs a) {
  constexpr int K = Chunking<NG, OBJ>::K;
  constexpr int BLOCK = Chunking<NG, OBJ>::BLOCK;
  using S = Shape1D<NG, BKG>;
  constexpr int NV = GRAD ? S::P + 1 : 1;
  const int64_t nb = a.nx;
  const int64_t nfull = nb / K;
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * BLOCK;
  const bool spec = a.dtype == DT_U32 && !a.weights;
  // the first chunk's counts are requested before the log table, so the two
  // memory latencies overlap instead of adding up
  ChunkRaw<K> first;
  if (a.dtype != DT_F64 && tid < nfull) {
    if (spec)
      load_raw<true>(a, tid * K, first);
    else
      load_raw<false>(a, tid * K, first);
  }
  __shared__ double2 lut[kLogLut];
  if constexpr (OBJ == OBJ_POISSON) log_lut_load(lut, a.log_lut);
  Model1D<NG, BKG> M;
  M.init(a.theta, a.t_shift, a.t_scale);
  M.init_grid(a.hx, K);
  if constexpr (OBJ == OBJ_POISSON) __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  int flags = 0;
  // the upstream adjoint scales grad_w here; the finishing kernel applies it
  // to the parameter gradient
  const double seed = (a.grad_w_out && a.seed) ? a.seed[0] : 1.0;
  const bool finite = all_finite(a.theta, a.P);

  if (spec) {
    stream_chunks<NG, BKG, OBJ, GRAD, F32BIN, true>(a, M, lut, nfull, tid, stride, seed, first, acc,
                                                    flags);
  } else if (a.dtype != DT_F64) {
    stream_chunks<NG, BKG, OBJ, GRAD, F32BIN, false>(a, M, lut, nfull, tid, stride, seed, first, acc,
                                                     flags);
  } else {
    for (int64_t c = tid; c < nfull; c += stride) {
      const int64_t i0 = c * K;
      double n[K], w[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        n[k] = static_cast<const double*>(a.counts)[i0 + k];
        w[k] = a.weights ? static_cast<double>(a.weights[i0 + k]) : 1.0;
      }
      chunk_step<NG, BKG, OBJ, GRAD, F32BIN>(a, M, lut, i0, n, w, seed, acc, flags);
    }
  }
  // ragged tail: fewer than K bins, one per thread of the first threads
  const int64_t tail = nb - nfull * K;
  if (tid < tail) {
    const int64_t i = nfull * K + tid;
    const double n[1] = {load_count1(a, i)};
    const double w[1] = {a.weights ? static_cast<double>(a.weights[i]) : 1.0};
    double l[1];
    chunk_1d<NG, BKG, OBJ, GRAD, F32BIN, false>(M, lut, fma(static_cast<double>(i), a.hx, a.x0),
                                                  n, w, acc, flags, l);
    if (a.grad_w_out) a.grad_w_out[i] = static_cast<float>(seed * l[0]);
  }

  __shared__ double fac[NV];
  if (threadIdx.x < NV) fac[threadIdx.x] = M.final_factor(threadIdx.x);
  grid_publish<NV, BLOCK>(acc, flags | (finite ? 0 : ST_NONFINITE), fac, nullptr, a.part,
                          a.part_flags);
}

template <int BLOCK, class K>
hipError_t launch_or_occupancy(K kernel, const NllArgs& a, int grid, hipStream_t s, int* occ,
                               int* block) {
  if (grid <= 0) {
    *block = BLOCK;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kernel, BLOCK, 0);
  }
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLOCK), 0, s, a);
  return hipGetLastError();
}

template <int NG, int BKG, int OBJ, bool GRAD, bool F32BIN>
hipError_t launch_1d(const NllArgs& a, int grid, hipStream_t s, int* occ, int* block) {
  return launch_or_occupancy<Chunking<NG, OBJ>::BLOCK>(k_nll_1d<NG, BKG, OBJ, GRAD, F32BIN>, a,
                                                       grid, s, occ, block);
}

template <int NG, int BKG, int OBJ>
LaunchFn pick_grad_prec(bool grad, bool f32) {
  if (grad) return f32 ? &launch_1d<NG, BKG, OBJ, true, true> : &launch_1d<NG, BKG, OBJ, true, false>;
  return f32 ? &launch_1d<NG, BKG, OBJ, false, true> : &launch_1d<NG, BKG, OBJ, false, false>;
}

template <int NG, int BKG>
LaunchFn pick_obj(int obj, bool grad, bool f32) {
  switch (obj) {
    case OBJ_NEYMAN:
      return pick_grad_prec<NG, BKG, OBJ_NEYMAN>(grad, f32);
    case OBJ_PEARSON:
      return pick_grad_prec<NG, BKG, OBJ_PEARSON>(grad, f32);
    case OBJ_POISSON:
      return pick_grad_prec<NG, BKG, OBJ_POISSON>(grad, f32);
    default:
      return nullptr;
  }
}

template <int NG>
LaunchFn pick_1d_ng(int bkg, int obj, bool grad, bool f32) {
  switch (bkg) {
    case BKG_NONE:
      if constexpr (NG == 0) return nullptr;
      else return pick_obj<NG, BKG_NONE>(obj, grad, f32);
    case 0:
      return pick_obj<NG, 0>(obj, grad, f32);
    case 1:
      return pick_obj<NG, 1>(obj, grad, f32);
    case 2:
      return pick_obj<NG, 2>(obj, grad, f32);
    case 3:
      return pick_obj<NG, 3>(obj, grad, f32);
    case BKG_EXP:
      return pick_obj<NG, BKG_EXP>(obj, grad, f32);
    default:
      return nullptr;
  }
}

// Defined in nll1d_ng{0..4}.hip and nll2d.hip.
LaunchFn pick_1d_ng0(int bkg, int obj, bool grad, bool f32);
LaunchFn pick_1d_ng1(int bkg, int obj, bool grad, bool f32);
LaunchFn pick_1d_ng2(int bkg, int obj, bool grad, bool f32);
LaunchFn pick_1d_ng3(int bkg, int obj, bool grad, bool f32);
LaunchFn pick_1d_ng4(int bkg, int obj, bool grad, bool f32);
LaunchFn pick_2d(int obj, bool grad, bool f32);
constexpr int kChunk2D = 16;  // bins of one row per 2D work item

}  // namespace hf
