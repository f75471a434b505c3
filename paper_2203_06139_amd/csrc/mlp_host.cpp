// mlp_host.cpp -- sequencing of the learned initialiser's forward pass and
// training step (kernels in mlp.hip).
#include "mlp.hpp"

namespace hf {

constexpr int64_t MlpLayout::kW[4];
constexpr int64_t MlpLayout::kB[4];
constexpr int MlpLayout::kIn[4];
constexpr int MlpLayout::kOutDim[4];

namespace {

struct Carver {
  char* p;
  int64_t used = 0;
  template <class T>
  T* take(int64_t n) {
    const int64_t bytes = (static_cast<int64_t>(sizeof(T)) * n + 255) & ~int64_t(255);
    T* r = p ? reinterpret_cast<T*>(p + used) : nullptr;
    used += bytes;
    return r;
  }
};

MlpWorkspace carve(Carver& c, int B) {
  MlpWorkspace w{};
  for (int l = 0; l < 4; ++l) {
    const int in = MlpLayout::kIn[l], out = MlpLayout::kOutDim[l];
    w.a[l] = c.take<uint16_t>(static_cast<int64_t>(B) * in);
    w.at[l] = c.take<uint16_t>(static_cast<int64_t>(B) * in);
    w.wb[l] = c.take<uint16_t>(static_cast<int64_t>(in) * out);
    w.wt[l] = c.take<uint16_t>(static_cast<int64_t>(in) * out);
    w.dz[l + 1] = c.take<uint16_t>(static_cast<int64_t>(B) * out);
    w.dzt[l + 1] = c.take<uint16_t>(static_cast<int64_t>(B) * out);
    if (l >= 1) w.z[l] = c.take<float>(static_cast<int64_t>(B) * in);
  }
  w.y = c.take<float>(static_cast<int64_t>(B) * kMlpOutPad);
  w.loss_part = c.take<double>(static_cast<int64_t>(B) * kMlpOutPad / 256);
  return w;
}

#define HF_TRY(x)                      \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

GemmArgs gemm_args(const uint16_t* A, int64_t lda, const uint16_t* Bm, int64_t ldb, int M, int N,
                   int K, int epi) {
  GemmArgs g{};
  g.A = A;
  g.lda = lda;
  g.B = Bm;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.epi = epi;
  return g;
}

// Casts the weights and runs the four layers; `train` keeps transposed
// activations and pre-activations for the backward pass.
hipError_t forward(int B, const float* params, const float* x, const MlpWorkspace& w, bool train,
                   float* y, hipStream_t s) {
  for (int l = 0; l < 4; ++l)
    HF_TRY(cast_nt(params + MlpLayout::kW[l], MlpLayout::kOutDim[l], MlpLayout::kIn[l], w.wb[l],
                   train ? w.wt[l] : nullptr, s));
  HF_TRY(cast_input(x, B, w.a[0], train ? w.at[0] : nullptr, s));
  for (int l = 0; l < 3; ++l) {
    const int in = MlpLayout::kIn[l], out = MlpLayout::kOutDim[l];
    GemmArgs g = gemm_args(w.a[l], in, w.wb[l], in, B, out, in, EPI_BIAS_GELU);
    g.bias = params + MlpLayout::kB[l];
    g.cf = train ? w.z[l + 1] : nullptr;
    g.ldcf = out;
    g.cb = w.a[l + 1];
    g.ldcb = out;
    g.cbt = train ? w.at[l + 1] : nullptr;
    g.ldcbt = B;
    HF_TRY(gemm_nt(g, s));
  }
  GemmArgs g = gemm_args(w.a[3], kMlpHidden, w.wb[3], kMlpHidden, B, kMlpOutPad, kMlpHidden,
                         EPI_BIAS);
  g.bias = params + MlpLayout::kB[3];
  g.cf = y;
  g.ldcf = kMlpOutPad;
  return gemm_nt(g, s);
}

}  // namespace

int64_t mlp_workspace_bytes(int B) {
  Carver c{nullptr};
  carve(c, B);
  return c.used;
}

MlpWorkspace mlp_carve(void* base, int B) {
  Carver c{static_cast<char*>(base)};
  return carve(c, B);
}

hipError_t mlp_forward(int B, const float* params, const float* x, float* y, void* ws,
                       hipStream_t s) {
  const MlpWorkspace w = mlp_carve(ws, B);
  return forward(B, params, x, w, false, y, s);
}

hipError_t mlp_train_step(int B, float* params, float* m, float* v, int step, float lr, float wd,
                          const float* x, const float* t, float* grads, float* loss, void* ws,
                          hipStream_t s) {
  const MlpWorkspace w = mlp_carve(ws, B);
  HF_TRY(forward(B, params, x, w, true, w.y, s));
  HF_TRY(mse(w.y, t, B, loss, w.dz[4], w.dzt[4], w.loss_part, s));
  for (int l = 3; l >= 0; --l) {
    const int in = MlpLayout::kIn[l], out = MlpLayout::kOutDim[l];
    // dW_l[n][k] = sum_b dZ_l[b][n] A_{l-1}[b][k]
    GemmArgs gw = gemm_args(w.dzt[l + 1], B, w.at[l], B, out, in, B, EPI_PLAIN);
    gw.cf = grads + MlpLayout::kW[l];
    gw.ldcf = in;
    HF_TRY(gemm_nt(gw, s));
    HF_TRY(bias_grad(w.dz[l + 1], B, out, grads + MlpLayout::kB[l], s));
    if (l > 0) {
      // dZ_{l-1}[b][k] = bf16( GELU'(z_{l-1}) * sum_n dZ_l[b][n] W_l[n][k] )
      GemmArgs gx = gemm_args(w.dz[l + 1], out, w.wt[l], out, B, in, out, EPI_GELU_PRIME);
      gx.zin = w.z[l];
      gx.ldz = in;
      gx.cb = w.dz[l];
      gx.ldcb = in;
      gx.cbt = w.dzt[l];
      gx.ldcbt = B;
      HF_TRY(gemm_nt(gx, s));
    }
  }
  return adamw(params, m, v, grads, MlpLayout::kTotal, lr, wd, step, s);
}

}  // namespace hf
