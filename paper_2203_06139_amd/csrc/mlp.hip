// mlp.hip -- learned initialiser: rebinning, default starts, and the BF16
// MFMA training / inference kernels of the 256-512-512-512-5 GELU network.
//
// Dense layers use v_mfma_f32_16x16x32_bf16 (gfx950): one wave computes a
// 32x32 output tile as 2x2 MFMA tiles, each lane feeding 8 consecutive K
// values of one A row and one B row per instruction, loaded as 16 bytes
// straight from L2 (the operands of this network are at most a few MB).
// Every GEMM is "NT": C[m][n] = sum_k A[m][k] B[n][k] with K contiguous in
// both operands, so the layers also keep transposed copies of activations,
// adjoints and weights; epilogues fuse bias, GELU, GELU' and BF16 rounding.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "mlp.hpp"

namespace hf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  if (m0 >= g.M || n0 >= g.N) return;  // whole wave; the kernel has no barriers
  const int r = lane & 15, kq = (lane >> 4) * 8;
  const uint16_t* a0p = g.A + static_cast<int64_t>(m0 + r) * g.lda + kq;
  const uint16_t* a1p = a0p + 16 * g.lda;
  const uint16_t* b0p = g.B + static_cast<int64_t>(n0 + r) * g.ldb + kq;
  const uint16_t* b1p = b0p + 16 * g.ldb;
  f32x4 c00 = {0.f, 0.f, 0.f, 0.f}, c01 = c00, c10 = c00, c11 = c00;
  // kStages K-steps of operands in flight: each step's loads are issued
  // kStages steps before its MFMAs, so L2 latency overlaps the matrix work
  // (a plain loop waits for every step's loads in turn).
  constexpr int kStages = 4;
  bf16x8 ra0[kStages], ra1[kStages], rb0[kStages], rb1[kStages];
#pragma unroll
  for (int s = 0; s < kStages; ++s) {
    if (s * 32 < g.K) {
      ra0[s] = *reinterpret_cast<const bf16x8*>(a0p + s * 32);
      ra1[s] = *reinterpret_cast<const bf16x8*>(a1p + s * 32);
      rb0[s] = *reinterpret_cast<const bf16x8*>(b0p + s * 32);
      rb1[s] = *reinterpret_cast<const bf16x8*>(b1p + s * 32);
    }
  }
  for (int k0 = 0; k0 < g.K; k0 += kStages * 32) {
#pragma unroll
    for (int s = 0; s < kStages; ++s) {
      const int k = k0 + s * 32;
      if (k < g.K) {
        c00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra0[s], rb0[s], c00, 0, 0, 0);
        c01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra0[s], rb1[s], c01, 0, 0, 0);
        c10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra1[s], rb0[s], c10, 0, 0, 0);
        c11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra1[s], rb1[s], c11, 0, 0, 0);
        const int kn = k + kStages * 32;
        if (kn < g.K) {
          ra0[s] = *reinterpret_cast<const bf16x8*>(a0p + kn);
          ra1[s] = *reinterpret_cast<const bf16x8*>(a1p + kn);
          rb0[s] = *reinterpret_cast<const bf16x8*>(b0p + kn);
          rb1[s] = *reinterpret_cast<const bf16x8*>(b1p + kn);
        }
      }
    }
  }
  // lane holds D[4 (lane/16) + q][lane % 16] of each 16x16 tile
  const f32x4 acc[2][2] = {{c00, c01}, {c10, c11}};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 16 * i + 4 * (lane >> 4) + q;
        const int n = n0 + 16 * j + r;
        float v = acc[i][j][q];
        if (g.epi == EPI_BIAS_GELU || g.epi == EPI_BIAS) v += g.bias[n];
        if (g.epi == EPI_BIAS_GELU) {
          if (g.cf) g.cf[static_cast<int64_t>(m) * g.ldcf + n] = v;  // pre-activation, for GELU'
          v = gelu(v);
        } else if (g.epi == EPI_GELU_PRIME) {
          v *= gelu_prime(g.zin[static_cast<int64_t>(m) * g.ldz + n]);
        } else {
          g.cf[static_cast<int64_t>(m) * g.ldcf + n] = v;
        }
        if (g.cb) {
          const uint16_t b = f2bf(v);
          g.cb[static_cast<int64_t>(m) * g.ldcb + n] = b;
          if (g.cbt) g.cbt[static_cast<int64_t>(n) * g.ldcbt + m] = b;
        }
      }
}

// Rejects what the kernel cannot index safely: shapes off the 32 grid, row
// strides that break the 16-byte operand loads, and a missing output or
// epilogue operand.
hipError_t gemm_nt(const GemmArgs& g, hipStream_t s) {
  if (g.M < 32 || g.N < 32 || g.K < 32 || g.M % 32 || g.N % 32 || g.K % 32) return hipErrorInvalidValue;
  if (!g.A || !g.B || g.lda < g.K || g.ldb < g.K || g.lda % 8 || g.ldb % 8) return hipErrorInvalidValue;
  const bool bias = g.epi == EPI_BIAS || g.epi == EPI_BIAS_GELU;
  if (bias && !g.bias) return hipErrorInvalidValue;
  if ((g.epi == EPI_PLAIN || g.epi == EPI_BIAS) && (!g.cf || g.ldcf < g.N)) return hipErrorInvalidValue;
  if (g.epi == EPI_BIAS_GELU && g.cf && g.ldcf < g.N) return hipErrorInvalidValue;
  if (g.epi == EPI_GELU_PRIME && (!g.zin || g.ldz < g.N || !g.cb)) return hipErrorInvalidValue;
  if (g.epi == EPI_BIAS_GELU && !g.cb) return hipErrorInvalidValue;
  if ((g.cb && g.ldcb < g.N) || (g.cbt && g.ldcbt < g.M)) return hipErrorInvalidValue;
  if (g.epi < EPI_PLAIN || g.epi > EPI_GELU_PRIME) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm_nt, dim3((g.N + 63) / 64, (g.M + 63) / 64), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Elementwise helpers of the training step
// ---------------------------------------------------------------------------
// W fp32 [N][K] -> W bf16 [N][K] and its transpose [K][N].
__global__ void k_cast_nt(const float* __restrict__ w, int N, int K, uint16_t* __restrict__ wb,
                          uint16_t* __restrict__ wt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(N) * K) return;
  const int n = static_cast<int>(i / K), k = static_cast<int>(i % K);
  const uint16_t b = f2bf(w[i]);
  wb[i] = b;
  if (wt) wt[static_cast<int64_t>(k) * N + n] = b;
}

hipError_t cast_nt(const float* w, int N, int K, uint16_t* wb, uint16_t* wt, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(N) * K;
  hipLaunchKernelGGL(k_cast_nt, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, w, N,
                     K, wb, wt);
  return hipGetLastError();
}

// loss = sum_{m, n<5} (y - t)^2 / (5B); dZ = bf16(2 (y - t) / (5B)), zero for
// the padding columns; written [B][32] and transposed [32][B].  Each block
// of 256 threads takes 8 rows and writes its FP64 partial sum of squares to
// part[block]; k_mse_loss then sums the partials in block order.
__global__ __launch_bounds__(256) void k_mse_grad(const float* __restrict__ y,
                                                  const float* __restrict__ t, int B,
                                                  uint16_t* dz, uint16_t* dzt,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const int i = blockIdx.x * 256 + threadIdx.x;  // B * 32 is a multiple of 256
  const int m = i / kMlpOutPad, n = i % kMlpOutPad;
  const float scale = 2.0f / (5.0f * static_cast<float>(B));
  float d = 0.0f;
  double acc = 0.0;
  if (n < kMlpOut) {
    d = y[i] - t[m * kMlpOut + n];
    acc = static_cast<double>(d) * d;
  }
  const uint16_t bv = f2bf(scale * d);
  dz[i] = bv;
  dzt[static_cast<int64_t>(n) * B + m] = bv;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_mse_loss(const double* __restrict__ part, int nparts, int B,
                                                  float* loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int q = threadIdx.x; q < nparts; q += 256) acc += part[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = static_cast<float>(red[0] / (5.0 * B));
}

hipError_t mse(const float* y, const float* t, int B, float* loss, uint16_t* dz, uint16_t* dzt,
               double* part, hipStream_t s) {
  const int nblk = B * kMlpOutPad / 256;
  hipLaunchKernelGGL(k_mse_grad, dim3(nblk), dim3(256), 0, s, y, t, B, dz, dzt, part);
  hipLaunchKernelGGL(k_mse_loss, dim3(1), dim3(256), 0, s, part, nblk, B, loss);
  return hipGetLastError();
}

// db[n] = sum_m dZ[m][n] (BF16 adjoints, FP32 sums).  A block of 1024
// threads takes 64 columns: 16 row groups each sum rows g, g+16, ... of one
// column (coalesced across the 64 lanes), then the 16 group sums are added
// in group order.
__global__ __launch_bounds__(1024) void k_bias_grad(const uint16_t* __restrict__ dz, int B, int N,
                                                    float* __restrict__ db) {
  __shared__ float red[16][64];
  const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float acc = 0.0f;
  if (n < N)
    for (int m = grp; m < B; m += 16) acc += bf2f(dz[static_cast<int64_t>(m) * N + n]);
  red[grp][c] = acc;
  __syncthreads();
  if (grp == 0 && n < N) {
    float v = red[0][c];
#pragma unroll
    for (int q = 1; q < 16; ++q) v += red[q][c];
    db[n] = v;
  }
}

hipError_t bias_grad(const uint16_t* dz, int B, int N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_bias_grad, dim3((N + 63) / 64), dim3(1024), 0, s, dz, B, N, db);
  return hipGetLastError();
}

// AdamW with decoupled weight decay (Loshchilov & Hutter), FP32 state.
__global__ void k_adamw(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                        const float* __restrict__ g, int64_t n, float lr, float wd, float bc1,
                        float bc2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  p[i] -= lr * (mh / (sqrtf(vh) + 1e-8f) + wd * p[i]);
}

hipError_t adamw(float* p, float* m, float* v, const float* g, int64_t n, float lr, float wd,
                 int step, hipStream_t s) {
  const float bc1 = 1.0f - powf(0.9f, static_cast<float>(step));
  const float bc2 = 1.0f - powf(0.999f, static_cast<float>(step));
  hipLaunchKernelGGL(k_adamw, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, m,
                     v, g, n, lr, wd, bc1, bc2);
  return hipGetLastError();
}

// x fp32 [B][256] -> bf16 [B][256] and transposed [256][B].
__global__ void k_cast_input(const float* __restrict__ x, int B, uint16_t* a, uint16_t* at) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kMlpIn) return;
  const int m = i / kMlpIn, k = i % kMlpIn;
  const uint16_t b = f2bf(x[i]);
  a[i] = b;
  if (at) at[static_cast<int64_t>(k) * B + m] = b;
}

hipError_t cast_input(const float* x, int B, uint16_t* a, uint16_t* at, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_input, dim3((B * kMlpIn + 255) / 256), dim3(256), 0, s, x, B, a, at);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Histogram -> network input, default starts, target maps, column statistics
// ---------------------------------------------------------------------------
__device__ __forceinline__ double count_any(const void* base, int dtype, int64_t i) {
  if (dtype == DT_U32) return static_cast<const uint32_t*>(base)[i];
  if (dtype == DT_F32) return static_cast<const float*>(base)[i];
  return static_cast<const double*>(base)[i];
}

// One block per histogram; coarse sums accumulate as exact FP64 sums of
// integer-valued (or given) counts in a fixed order per coarse bin.
__global__ __launch_bounds__(256) void k_rebin_lognorm(const void* counts, int dtype,
                                                       const int64_t* __restrict__ offsets,
                                                       float in_mean, float in_std,
                                                       float* __restrict__ out) {
  const int b = blockIdx.x;
  const int64_t off = offsets[b];
  const int64_t nb = offsets[b + 1] - off;
  const int j = threadIdx.x;  // coarse bin
  // fine bin i goes to coarse bin floor((2i+1) 256 / (2 nb)); the fine bins
  // of coarse bin j are i in [lo(j), lo(j+1)) with lo(j) the count of i whose
  // (2i+1) 256 < 2 j nb, i.e. lo(j) = ceil((2 j nb - 256) / 512) clamped.
  auto lo_of = [nb](int jj) -> int64_t {
    const int64_t num = 2 * static_cast<int64_t>(jj) * nb - kMlpIn;
    if (num <= 0) return 0;
    const int64_t q = (num + 2 * kMlpIn - 1) / (2 * kMlpIn);
    return q < nb ? q : nb;
  };
  const int64_t i0 = lo_of(j), i1 = (j + 1 == kMlpIn) ? nb : lo_of(j + 1);
  double c = 0.0;
  for (int64_t i = i0; i < i1; ++i) c += count_any(counts, dtype, off + i);
  const double k = static_cast<double>(i1 - i0);
  const double v = k > 0.0 ? log1p(c / k) : 0.0;
  out[static_cast<int64_t>(b) * kMlpIn + j] = static_cast<float>((v - in_mean) / in_std);
}

hipError_t rebin_lognorm(int B, const void* counts, int dtype, const int64_t* offsets, float mean,
                         float std, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rebin_lognorm, dim3(B), dim3(kMlpIn), 0, s, counts, dtype, offsets, mean, std,
                     out);
  return hipGetLastError();
}

// Default starting point for Gauss + exp(b0 + b1 t); one block per histogram.
//   background: mean counts of the first and last ne = max(nb/25, 1) bins
//     (at least 1), an exponential through the two edge-block centres (the
//     model's own background form; a straight line would leave a false
//     excess at the steep edge of a falling or rising background);
//   peak: the window position i in [W, nb - W), W = max(nb/256, 1), with the
//     largest integer excess e(i) = rint(S(i) - (2W+1) bg(i)), S(i) the sum
//     of counts over [i - W, i + W] (first such i on ties);
//   width: walking out from the peak while 2 e >= e_max, the half-maximum
//     bounds give the FWHM.
// The window positions are split among the block's four waves in
// contiguous ranges; a wave walks its range 64 positions per step, lane l
// at position s + l, with coalesced loads: the window sum at position i is
// the sum at the range's first position plus the lane prefix sum of the
// differences c[i + W] - c[i - W - 1] (S(i) - S(i - 1)).  Sums of
// integer-valued counts are exact in FP64 in any order, so every window sum
// and decision matches a direct evaluation; the excess is evaluated without
// FMA contraction (separate products and sums).  The walk for the width
// becomes a search for the nearest positions left and right of the peak
// with 2 e < e_max.
struct Excess {
  double lb0, dlb, c0, cden, wlen;
  __device__ __forceinline__ int64_t operator()(double S, int64_t i) const {
#pragma clang fp contract(off)
    const double bg = exp(lb0 + dlb * ((static_cast<double>(i) + 0.5 - c0) / cden));
    return static_cast<int64_t>(__builtin_rint(S - wlen * bg));
  }
};

// Calls fn(S, i) for every window position i of [q0, q1) (one wave, lane l
// taking positions q0 + l, q0 + 64 + l, ...), S the window sum over
// [i - W, i + W].
template <class Fn>
__device__ __forceinline__ void window_walk(const void* counts, int dtype, int64_t off, int64_t q0,
                                            int64_t q1, int64_t W, Fn fn) {
  if (q0 >= q1) return;
  const int lane = static_cast<int>(threadIdx.x & 63u);
  double s0 = 0.0;
  for (int64_t q = q0 - W + lane; q <= q0 + W; q += 64) s0 += count_any(counts, dtype, off + q);
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) s0 += __shfl_xor(s0, k);
  double carry = s0;  // S(q0), then S of the previous step's last position
  for (int64_t base = q0; base < q1; base += 64) {
    const int64_t i = base + lane;
    double d = 0.0;
    if (i > q0 && i < q1)
      d = count_any(counts, dtype, off + i + W) - count_any(counts, dtype, off + i - W - 1);
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
      const double u = __shfl_up(d, k);
      if (lane >= k) d += u;
    }
    const double S = carry + d;
    if (i < q1) fn(S, i);
    carry = __shfl(S, 63);
  }
}

// Threads per histogram: 16 waves (a histogram of 65,536 bins walks 64
// steps of 64 positions per wave and pass).  Measured on the 4096-histogram
// Gauss + exponential batch: 0.89 ms with 16 waves, 0.91 ms with four, and
// 2.86 ms when each thread walked its own segment of positions with
// scattered loads.  Per position the background's exp and the division
// before it now dominate; both stay, since the excess must round as the
// direct evaluation does.
constexpr int kDsThreads = 1024;
constexpr int kDsWaves = kDsThreads / 64;

__global__ __launch_bounds__(kDsThreads) void k_default_starts(const void* counts, int dtype,
                                                               const int64_t* __restrict__ offsets,
                                                               const double* __restrict__ ranges,
                                                               double t_shift, double t_scale,
                                                               double* __restrict__ theta0) {
  __shared__ double red_d[2][kDsWaves];
  __shared__ int64_t red_e[kDsWaves];
  __shared__ int64_t red_i[kDsWaves];
  __shared__ int64_t red_j[kDsWaves];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int64_t off = offsets[b];
  const int64_t nb = offsets[b + 1] - off;
  if (nb < 1) {  // empty histogram: no start (uniform over the block)
    if (t < 5) theta0[static_cast<int64_t>(b) * 5 + t] = __builtin_nan("");
    return;
  }
  const double lo = ranges[2 * b], hi = ranges[2 * b + 1];
  const double h = (hi - lo) / static_cast<double>(nb);
  const int64_t ne = nb / 25 > 0 ? nb / 25 : 1;  // 4% of the bins at each edge
  // edge sums (integer-valued: exact in any order)
  double sl = 0.0, sr = 0.0;
  for (int64_t i = t; i < ne; i += kDsThreads) {
    sl += count_any(counts, dtype, off + i);
    sr += count_any(counts, dtype, off + nb - ne + i);
  }
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) {
    sl += __shfl_xor(sl, k);
    sr += __shfl_xor(sr, k);
  }
  if (lane == 0) {
    red_d[0][wv] = sl;
    red_d[1][wv] = sr;
  }
  __syncthreads();
  double esl = 0.0, esr = 0.0;
#pragma unroll
  for (int w = 0; w < kDsWaves; ++w) {
    esl += red_d[0][w];
    esr += red_d[1][w];
  }
  const double bk0 = fmax(esl / static_cast<double>(ne), 1.0);
  const double bk1 = fmax(esr / static_cast<double>(ne), 1.0);
  const double c0 = 0.5 * static_cast<double>(ne);
  const double c1 = static_cast<double>(nb) - 0.5 * static_cast<double>(ne);
  const int64_t W = nb / 256 > 1 ? nb / 256 : 1;
  const double lb0 = log(bk0);
  const Excess ex{lb0, log(bk1) - lb0, c0, c1 - c0, static_cast<double>(2 * W + 1)};
  // this wave's range [q0, q1) of the window positions [W, nb - W)
  const int64_t nv = nb - 2 * W > 0 ? nb - 2 * W : 0;
  const int64_t Lw = (nv + kDsWaves - 1) / kDsWaves;
  const int64_t q0 = W + wv * Lw;
  const int64_t q1 = (W + (wv + 1) * Lw < nb - W) ? W + (wv + 1) * Lw : nb - W;
  // pass 1: largest excess, first position (per lane, positions increase)
  int64_t be = INT64_MIN, bi = 0;
  window_walk(counts, dtype, off, q0, q1, W, [&](double S, int64_t i) {
    const int64_t e = ex(S, i);
    if (e > be) {
      be = e;
      bi = i;
    }
  });
  // the largest excess, the first position among equals: over the lanes,
  // then over the waves
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) {
    const int64_t oe = __shfl_xor(be, k), oi = __shfl_xor(bi, k);
    if (oe > be || (oe == be && oi < bi)) {
      be = oe;
      bi = oi;
    }
  }
  if (lane == 0) {
    red_e[wv] = be;
    red_i[wv] = bi;
  }
  __syncthreads();
  int64_t emax = INT64_MIN, imax = nb / 2;
#pragma unroll
  for (int w = 0; w < kDsWaves; ++w)
    if (red_e[w] > emax || (red_e[w] == emax && red_i[w] < imax)) {
      emax = red_e[w];
      imax = red_i[w];
    }
  if (emax == INT64_MIN) {  // histogram shorter than one window
    emax = 0;
    imax = nb / 2;
  }
  __syncthreads();
  // pass 2: nearest positions left / right of the peak with 2 e < emax
  int64_t pl = INT64_MIN, pr = INT64_MAX;
  window_walk(counts, dtype, off, q0, q1, W, [&](double S, int64_t i) {
    if (i != imax && 2 * ex(S, i) < emax) {
      if (i < imax) pl = i > pl ? i : pl;  // the largest below the peak
      else pr = i < pr ? i : pr;           // the smallest above it
    }
  });
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) {
    const int64_t ol = __shfl_xor(pl, k), orr = __shfl_xor(pr, k);
    pl = ol > pl ? ol : pl;
    pr = orr < pr ? orr : pr;
  }
  if (lane == 0) {
    red_e[wv] = pl;
    red_j[wv] = pr;
  }
  __syncthreads();
  if (t == 0) {
    int64_t l = INT64_MIN, r = INT64_MAX;
    for (int q = 0; q < kDsWaves; ++q) {
      l = red_e[q] > l ? red_e[q] : l;
      r = red_j[q] < r ? red_j[q] : r;
    }
    // the walk stops just inside the first failing position, or at the edge
    // of the window range; it never moves when that range is empty
    const int64_t left = l == INT64_MIN ? W : (l + 1 > W ? l + 1 : W);
    const int64_t right = r == INT64_MAX ? nb - W - 1 : (r - 1 < nb - W - 1 ? r - 1 : nb - W - 1);
    const int64_t b0i = left < imax ? left : imax;
    const int64_t b1i = right > imax ? right : imax;
    const double range = hi - lo;
    const double fwhm = static_cast<double>(b1i - b0i + 1) * h;
    const double s = fmin(fmax(fwhm / 2.3548200450309493, 0.005 * range), 0.1 * range);
    const double A = fmax(static_cast<double>(emax) / ex.wlen, 1.0);
    const double m = lo + (static_cast<double>(imax) + 0.5) * h;
    const double t0 = (lo + c0 * h - t_shift) / t_scale;
    const double t1 = (lo + c1 * h - t_shift) / t_scale;
    const double b1 = log(bk1 / bk0) / (t1 - t0);
    const double b0v = log(bk0) - b1 * t0;
    double* th = theta0 + static_cast<int64_t>(b) * 5;
    th[0] = A;
    th[1] = m;
    th[2] = s;
    th[3] = b0v;
    th[4] = b1;
  }
}

hipError_t default_starts(int B, const void* counts, int dtype, const int64_t* offsets,
                          const double* ranges, double t_shift, double t_scale, double* theta0,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_default_starts, dim3(B), dim3(kDsThreads), 0, s, counts, dtype, offsets, ranges,
                     t_shift, t_scale, theta0);
  return hipGetLastError();
}

__global__ void k_theta_to_target(int B, const double* __restrict__ th, const float* mean,
                                  const float* std, float* __restrict__ t) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double* p = th + static_cast<int64_t>(b) * 5;
  const double raw[5] = {p[1], log(fabs(p[2])), log(fabs(p[0])), p[3], p[4]};
  for (int k = 0; k < 5; ++k)
    t[static_cast<int64_t>(b) * 5 + k] = static_cast<float>((raw[k] - mean[k]) / std[k]);
}

__global__ void k_target_to_theta(int B, const float* __restrict__ y, const float* mean,
                                  const float* std, double* __restrict__ th) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double v[5];
  for (int k = 0; k < 5; ++k)
    v[k] = static_cast<double>(y[static_cast<int64_t>(b) * kMlpOutPad + k]) * std[k] + mean[k];
  double* p = th + static_cast<int64_t>(b) * 5;
  p[0] = exp(v[2]);
  p[1] = v[0];
  p[2] = exp(v[1]);
  p[3] = v[3];
  p[4] = v[4];
}

hipError_t theta_to_target(int B, const double* th, const float* mean, const float* std, float* t,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_theta_to_target, dim3((B + 255) / 256), dim3(256), 0, s, B, th, mean, std, t);
  return hipGetLastError();
}

hipError_t target_to_theta(int B, const float* y, const float* mean, const float* std, double* th,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_target_to_theta, dim3((B + 255) / 256), dim3(256), 0, s, B, y, mean, std, th);
  return hipGetLastError();
}

// One block per column: FP64 sum and sum of squares over rows in a fixed
// (strided, then tree) order.
__global__ __launch_bounds__(256) void k_column_stats(int64_t n, int cols, const float* __restrict__ x,
                                                      float* mean, float* stdv) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0.0, q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = x[i * cols + c];
    a += v;
    q += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / static_cast<double>(n);
    const double var = fmax(s2[0] / static_cast<double>(n) - mu * mu, 0.0);
    mean[c] = static_cast<float>(mu);
    stdv[c] = static_cast<float>(var > 0.0 ? sqrt(var) : 1.0);
  }
}

hipError_t column_stats(int64_t n, int cols, const float* x, float* mean, float* stdv,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_column_stats, dim3(cols), dim3(256), 0, s, n, cols, x, mean, stdv);
  return hipGetLastError();
}

}  // namespace hf
