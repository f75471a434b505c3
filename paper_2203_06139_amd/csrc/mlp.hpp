// mlp.hpp -- kernels of the learned initialiser (see mlp.hip) and the host
// routines that sequence them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

constexpr int kMlpIn = 256;
constexpr int kMlpHidden = 512;
constexpr int kMlpOut = 5;
constexpr int kMlpOutPad = 32;

enum : int { EPI_PLAIN = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_PRIME = 3 };

// C[m][n] = sum_k A[m][k] B[n][k] (BF16 in, FP32 accumulate); M, N, K
// multiples of 32, rows 16-byte aligned.  Epilogue:
//   EPI_PLAIN       cf = C
//   EPI_BIAS        cf = C + bias
//   EPI_BIAS_GELU   cf = z = C + bias (if cf), cb/cbt = bf16(GELU(z))
//   EPI_GELU_PRIME  cb/cbt = bf16(C * GELU'(zin))
struct GemmArgs {
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  int M, N, K;
  int epi;
  const float* bias;
  const float* zin;
  int64_t ldz;
  float* cf;
  int64_t ldcf;
  uint16_t* cb;
  int64_t ldcb;
  uint16_t* cbt;
  int64_t ldcbt;
};

hipError_t gemm_nt(const GemmArgs& g, hipStream_t s);
hipError_t cast_nt(const float* w, int N, int K, uint16_t* wb, uint16_t* wt, hipStream_t s);
hipError_t cast_input(const float* x, int B, uint16_t* a, uint16_t* at, hipStream_t s);
hipError_t mse(const float* y, const float* t, int B, float* loss, uint16_t* dz, uint16_t* dzt,
               double* part, hipStream_t s);
hipError_t bias_grad(const uint16_t* dz, int B, int N, float* db, hipStream_t s);
hipError_t adamw(float* p, float* m, float* v, const float* g, int64_t n, float lr, float wd,
                 int step, hipStream_t s);
hipError_t rebin_lognorm(int B, const void* counts, int dtype, const int64_t* offsets, float mean,
                         float std, float* out, hipStream_t s);
hipError_t default_starts(int B, const void* counts, int dtype, const int64_t* offsets,
                          const double* ranges, double t_shift, double t_scale, double* theta0,
                          hipStream_t s);
hipError_t theta_to_target(int B, const double* th, const float* mean, const float* std, float* t,
                           hipStream_t s);
hipError_t target_to_theta(int B, const float* y, const float* mean, const float* std, double* th,
                           hipStream_t s);
hipError_t column_stats(int64_t n, int cols, const float* x, float* mean, float* stdv,
                        hipStream_t s);

// Parameter layout (offsets in floats) and workspace carving.
struct MlpLayout {
  static constexpr int64_t kW[4] = {0, 131584, 394240, 656896};
  static constexpr int64_t kB[4] = {131072, 393728, 656384, 673280};
  static constexpr int kIn[4] = {kMlpIn, kMlpHidden, kMlpHidden, kMlpHidden};
  static constexpr int kOutDim[4] = {kMlpHidden, kMlpHidden, kMlpHidden, kMlpOutPad};
  static constexpr int64_t kTotal = 673312;
};

struct MlpWorkspace {
  uint16_t* a[4];   // a[0] = x, a[1..3] hidden activations, [B][in]
  uint16_t* at[4];  // transposed [in][B]
  float* z[4];      // z[1..3] hidden pre-activations [B][512]
  float* y;         // [B][32]
  uint16_t* dz[5];  // dz[1..4] layer adjoints [B][out]
  uint16_t* dzt[5]; // transposed
  uint16_t* wb[4];  // layer weights bf16 [out][in]
  uint16_t* wt[4];  // transposed [in][out]
  double* loss_part;  // B*32/256 partial sums of the loss
};

int64_t mlp_workspace_bytes(int B);
MlpWorkspace mlp_carve(void* base, int B);
hipError_t mlp_forward(int B, const float* params, const float* x, float* y, void* ws, hipStream_t s);
hipError_t mlp_train_step(int B, float* params, float* m, float* v, int step, float lr, float wd,
                          const float* x, const float* t, float* grads, float* loss, void* ws,
                          hipStream_t s);

}  // namespace hf
