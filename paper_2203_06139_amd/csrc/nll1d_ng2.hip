// nll1d_ng2.hip -- 1D objective kernels with 2 Gaussian(s); one translation
// unit per Gaussian count so the instantiations compile in parallel.
#include "nll_kernels.hpp"

namespace hf {
LaunchFn pick_1d_ng2(int bkg, int obj, bool grad, bool f32) {
  return pick_1d_ng<2>(bkg, obj, grad, f32);
}
}  // namespace hf
