// fit_ng3.hip -- batched fitter kernels for models with 3 Gaussian(s).
#include "fit_impl.hpp"

namespace hf {
FitLaunchFn pick_fit_ng3(int bkg, int obj, int blk) { return pick_fit_ng<3>(bkg, obj, blk); }
}  // namespace hf
