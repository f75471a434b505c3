// fp64_issue_probe.hip -- measures the VALU issue rate gfx950 reaches on
// chains of FP64 FMA / mul / add, v_rcp_f64 and FP32<->FP64 conversions, at
// 1..8 independent chains per thread (ILP) and 1..8 resident 256-thread
// blocks per CU (waves per SIMD).  It sets the achievable denominator next to
// the nominal 256 CU x 64 lanes x 2.4 GHz = 3.93e13 lane-instructions/s.
//
// Build and run on the GPU (not part of the library):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o fp64_issue_probe paper_2203_06139_amd/probes/fp64_issue_probe.hip && ./fp64_issue_probe
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)

template <int ILP, int OP>
__global__ __launch_bounds__(256) void k_chain(double* out, int iters, double b, double c) {
  double a[ILP];
#pragma unroll
  for (int i = 0; i < ILP; ++i) a[i] = threadIdx.x * 1e-3 + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < ILP; ++i) {
      if (OP == 0) a[i] = fma(a[i], b, c);
      else if (OP == 1) a[i] = a[i] * b;
      else if (OP == 2) a[i] = a[i] + c;
      else if (OP == 3) a[i] = __builtin_amdgcn_rcp(a[i]);
      else if (OP == 4) a[i] = static_cast<double>(static_cast<float>(a[i]) * 1.0001f);
    }
  }
  double s = 0;
#pragma unroll
  for (int i = 0; i < ILP; ++i) s += a[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int ILP, int OP>
int run(const char* name, double* d, int ncu, int bpc) {
  const int iters = 2048;
  const int grid = ncu * bpc;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0)); CK(hipEventCreate(&e1));
  hipLaunchKernelGGL((k_chain<ILP, OP>), dim3(grid), dim3(256), 0, 0, d, iters, 0.999999, 1e-7);
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int r = 0; r < 5; ++r)
    hipLaunchKernelGGL((k_chain<ILP, OP>), dim3(grid), dim3(256), 0, 0, d, iters, 0.999999, 1e-7);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double inst = 5.0 * grid * 256.0 * iters * ILP;  // lane-instructions
  printf("%-6s ILP=%d blocks/CU=%d: %.3f ms  %.2f T lane-instr/s  (%.1f%% of 3.93e13)\n", name, ILP,
         bpc, ms, inst / (ms * 1e-3) / 1e12, 100.0 * inst / (ms * 1e-3) / 3.93e13);
  return 0;
}

int main() {
  int ncu = 0;
  CK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  printf("device %s, %d CUs, clock %d kHz\n", p.gcnArchName, ncu, p.clockRate);
  double* d;
  CK(hipMalloc(&d, sizeof(double) * 256 * ncu * 16));
  for (int bpc : {1, 2, 4, 8}) {
    run<1, 0>("fma", d, ncu, bpc);
    run<2, 0>("fma", d, ncu, bpc);
    run<4, 0>("fma", d, ncu, bpc);
    run<8, 0>("fma", d, ncu, bpc);
  }
  for (int bpc : {2, 4}) {
    run<4, 1>("mul", d, ncu, bpc);
    run<4, 2>("add", d, ncu, bpc);
    run<4, 3>("rcp", d, ncu, bpc);
    run<4, 4>("cvt32", d, ncu, bpc);
  }
  CK(hipFree(d));
  return 0;
}
