// fit_ng2.hip -- batched fitter kernels for models with 2 Gaussian(s).
#include "fit_impl.hpp"

namespace hf {
FitLaunchFn pick_fit_ng2(int bkg, int obj, int blk) { return pick_fit_ng<2>(bkg, obj, blk); }
}  // namespace hf
