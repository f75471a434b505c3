// fisher_cov.hip -- parameter covariance from Fisher matrices, one wave per
// matrix.
//
// For the free parameters (free_mask bit set, or all when the mask is 0):
//   S = diag(F)^(-1/2),  R = S F S (unit diagonal),
//   R = L L^T (Cholesky; every pivot must exceed 1e-12 and be finite),
//   cov = scale * S inv(L)^T inv(L) S.
// Scaling to unit diagonal first makes the pivot test independent of the
// parameters' units (an amplitude of 1e4 counts next to a width of 0.01).
// The rows and columns of fixed parameters are 0.  A free block that is not
// safely positive definite (or a non-positive diagonal entry) gives NaN in
// the free entries and status 1.
#include "fisher_kernels.hpp"

namespace hf {

constexpr int kCovMaxP = 16;

__global__ __launch_bounds__(64) void k_fisher_cov(const double* __restrict__ F, int P,
                                                   uint32_t free_mask, double scale,
                                                   double* __restrict__ cov,
                                                   int32_t* __restrict__ status) {
  constexpr int S = kCovMaxP;
  __shared__ double L[S * S], Li[S * S], sc[S];
  __shared__ int fidx[S], pos[S];
  __shared__ int nf, ok;
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  const double* Fb = F + b * P * P;
  double* Cb = cov + b * P * P;
  if (tid == 0) {
    int k = 0;
    for (int p = 0; p < P; ++p) {
      const bool fr = free_mask == 0u || ((free_mask >> p) & 1u);
      pos[p] = fr ? k : -1;
      if (fr) fidx[k++] = p;
    }
    nf = k;
    ok = 1;
  }
  __syncthreads();
  if (tid < nf) {
    const double d = Fb[fidx[tid] * P + fidx[tid]];
    if (!(d > 0.0) || !__builtin_isfinite(d)) ok = 0;  // benign race: every writer stores 0
    sc[tid] = 1.0 / sqrt(d);
  }
  __syncthreads();
  for (int t = tid; t < nf * nf; t += 64) {
    const int r = t / nf, c = t % nf;
    L[r * S + c] = ok ? Fb[fidx[r] * P + fidx[c]] * sc[r] * sc[c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nf && ok; ++j) {
    if (tid == 0) {
      double d = L[j * S + j];
      for (int k = 0; k < j; ++k) d -= L[j * S + k] * L[j * S + k];
      if (!(d > 1e-12) || !__builtin_isfinite(d)) ok = 0;
      else L[j * S + j] = sqrt(d);
    }
    __syncthreads();
    if (ok && tid > j && tid < nf) {
      double v = L[tid * S + j];
      for (int k = 0; k < j; ++k) v -= L[tid * S + k] * L[j * S + k];
      L[tid * S + j] = v / L[j * S + j];
    }
    __syncthreads();
  }
  if (ok && tid < nf) {  // column tid of inv(L)
    const int c = tid;
    for (int i = c; i < nf; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= L[i * S + k] * Li[k * S + c];
      Li[i * S + c] = v / L[i * S + i];
    }
  }
  __syncthreads();
  const double nan = __builtin_nan("");
  for (int t = tid; t < P * P; t += 64) {
    const int pr = pos[t / P], pc = pos[t % P];
    double v = 0.0;
    if (pr >= 0 && pc >= 0) {
      if (ok) {
        for (int k = (pr > pc ? pr : pc); k < nf; ++k) v += Li[k * S + pr] * Li[k * S + pc];
        v *= scale * sc[pr] * sc[pc];
      } else {
        v = nan;
      }
    }
    Cb[t] = v;
  }
  if (tid == 0 && status) status[b] = ok ? 0 : 1;
}

hipError_t fisher_covariance(int B, int P, const double* F, uint32_t free_mask, double scale,
                             double* cov, int32_t* status, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (P < 1 || P > kCovMaxP) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fisher_cov, dim3(B), dim3(64), 0, s, F, P, free_mask, scale, cov, status);
  return hipGetLastError();
}

}  // namespace hf
