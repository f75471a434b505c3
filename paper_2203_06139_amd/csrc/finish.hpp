// finish.hpp -- second kernel of every objective call (nll_eval, nll_grad,
// nll_unbinned) and of the expected Hessian: the fixed-order sum of the
// per-block partials published by grid_publish, and the outputs.
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

// Finishing kernel of a symmetric matrix published entry by entry (the
// expected Hessian): NQ upper-triangle entries E0 .. E0+NQ-1 of a P x P
// row-major matrix, each the block-order sum of its G partials, written to
// both triangles of out; NaN where a block flags ST_NONFINITE.  status_out
// (if not null, and E0 == 0) gets 0 or ST_NONFINITE.
struct FinishSymArgs {
  const double* part;         // [NQ][G]
  const int32_t* part_flags;  // [G]
  int32_t G, NQ, E0, P;
  double* out;
  int32_t* status_out;
};

hipError_t launch_finish_sym(const FinishSymArgs& a, hipStream_t s);

}  // namespace hf
