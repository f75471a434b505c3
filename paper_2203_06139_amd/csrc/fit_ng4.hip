// fit_ng4.hip -- batched fitter kernels for models with 4 Gaussian(s).
#include "fit_impl.hpp"

namespace hf {
FitLaunchFn pick_fit_ng4(int bkg, int obj, int blk) { return pick_fit_ng<4>(bkg, obj, blk); }
}  // namespace hf
