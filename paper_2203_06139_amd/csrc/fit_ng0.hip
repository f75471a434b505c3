// fit_ng0.hip -- batched fitter kernels for models with 0 Gaussian(s).
#include "fit_impl.hpp"

namespace hf {
FitLaunchFn pick_fit_ng0(int bkg, int obj, int blk) { return pick_fit_ng<0>(bkg, obj, blk); }
}  // namespace hf
