// fit_kernels.hpp -- batched histogram fitting on the device.
//
// A gradient-based fit of a parametric function to a histogram (paper sec. 4,
// Fig. 2a, where ROOT's minimiser takes the Clad gradient) repeated over B
// independent histograms in one launch.  Every workgroup is persistent: it
// takes the next histogram from an atomic work queue (longest first), runs
// BFGS on it with the objective and gradient evaluated by the whole
// workgroup, writes the result and takes the next one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

struct FitArgs {
  int32_t B;
  int32_t dtype;
  const void* counts;
  const int64_t* offsets;
  const double* ranges;
  int32_t obj;
  int32_t f32;
  const double* theta0;
  double* theta_out;
  double* nll_out;
  int32_t* status;
  int32_t* iters;
  int32_t* nevals;
  int32_t max_iter;
  int32_t ls_max;
  int32_t fixed_iters;
  uint32_t free_mask;
  double edm_tol;
  double polish_edm;
  double t_shift, t_scale;
  int32_t P;
  int32_t sorted;
  int32_t* order;     // device i32[B]: queue position -> histogram index
  unsigned* counters; // [0] queue head, [1] finished workgroups
  const double2* log_lut;  // kLogLut entries (Poisson)
  int32_t cache_bins;      // LDS cache capacity (u32 counts); 0 = no cache
  int32_t hessian_init;    // 0 identity, 1 inverse expected Hessian at theta0
  int32_t fd_grad;         // 1: central-difference gradient (FP64 bins)
  int32_t wave_bins;       // histograms of at most this many bins are fitted one per wave (0: off)
};

// Device scratch of the fitter, owned by the context.  `order` grows with B;
// the two counters are cleared once at creation and re-armed by the kernel.
struct FitScratch {
  int32_t* order = nullptr;
  int64_t cap = 0;
  unsigned* counters = nullptr;
  int wg_per_cu = 2;   // persistent workgroups per CU
  int cache_bins = 0;  // histograms with at most this many u32 bins live in LDS
  int block = 256;     // threads per workgroup (256 or 512)
  int wave_bins = 0;   // one wave per histogram of at most this many bins (0: off)
};

hipError_t fit_scratch_init(FitScratch* s);
void fit_scratch_free(FitScratch* s);

// Returns hipErrorNotSupported for a model without a fit kernel.
hipError_t launch_fit(int n_gauss, int bkg, FitArgs a, int num_cu, FitScratch* s, hipStream_t st);

// Largest LDS cache (in u32 bins) a fit workgroup of `block` threads can
// hold for this model and objective next to its own state.
int fit_max_cache_bins(int n_gauss, int bkg, int obj, int block);

// Largest wave_bins whose per-wave slots (fit state + counts) fit in the
// LDS a workgroup of `block` threads has next to its own state.
int fit_max_wave_bins(int n_gauss, int bkg, int obj, int block);

}  // namespace hf
