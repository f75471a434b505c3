// fit_ng1.hip -- batched fitter kernels for models with 1 Gaussian(s).
#include "fit_impl.hpp"

namespace hf {
FitLaunchFn pick_fit_ng1(int bkg, int obj, int blk) { return pick_fit_ng<1>(bkg, obj, blk); }
}  // namespace hf
