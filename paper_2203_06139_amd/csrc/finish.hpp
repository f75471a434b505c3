// finish.hpp -- second kernel of every objective call (nll_eval, nll_grad,
// nll_unbinned): the fixed-order sum of the per-block partials published by
// grid_publish, and the outputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

struct FinishArgs {
  const double* part;      // [NV][G] block partials (factors already applied)
  const int32_t* part_flags;  // [G] status bits per block
  int32_t G;               // blocks of the main kernel
  int32_t NV;              // 1 (value) or P + 1 (value and gradient)
  const double* seed;      // upstream adjoint of L, or null (1)
  double* nll_out;
  double* grad_out;        // P values, or null when NV == 1
  int32_t* status_out;     // or null
  uint32_t free_mask;
};

// Launches the finishing kernel on `s` after the main kernel; G >= 1,
// 1 <= NV <= 17.
hipError_t launch_finish(const FinishArgs& a, hipStream_t s);

}  // namespace hf
