// nll1d_avg_ng1.hip -- bin-average and explicit-edge objective kernels with
// 1 Gaussian(s); one translation unit per Gaussian count so the
// instantiations compile in parallel.
#include "nll_avg.hpp"

namespace hf {
LaunchFn pick_avg_ng1(int bkg, int obj, bool grad, bool edges) {
  return pick_avg_ng<1>(bkg, obj, grad, edges);
}
LaunchFn pick_edges_ng1(int bkg, int obj, bool grad) { return pick_edges_ng<1>(bkg, obj, grad); }
}  // namespace hf
