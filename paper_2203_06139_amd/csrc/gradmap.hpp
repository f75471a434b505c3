// gradmap.hpp -- arguments of the elementwise Gaussian gradient map
// (gradmap.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

enum : int { GRADMAP_NORM_LISTING = 0, GRADMAP_NORM_PDF = 1 };

struct GradMapArgs {
  int64_t n;
  const double* x;      // [n]
  const double* p;      // [n], or [1] when p_shared
  const double* sigma;  // [n], or [1] when sigma_shared
  const double* seed;   // [n] upstream adjoints, or null (1)
  int32_t p_shared, sigma_shared;
  int32_t norm;
  double* g;   // [n] or null
  double* dx;  // [n] or null
  double* dp;  // [n], [1] when p_shared, or null
  double* ds;  // [n], [1] when sigma_shared, or null
  double* part;
  int32_t* part_flags;
  unsigned* ticket;
};

// vec: every non-null array is 16-byte aligned (pairs of elements move as
// 16-byte vectors).  The grid is one round of resident blocks on num_cu CUs,
// at most max_grid (the partials scratch's block count).
hipError_t gauss_grad_map(const GradMapArgs& a, bool vec, int num_cu, int max_grid, hipStream_t s);

}  // namespace hf
