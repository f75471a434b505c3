// nll1d_avg_ng4.hip -- bin-average and explicit-edge objective kernels with
// 4 Gaussian(s); one translation unit per Gaussian count so the
// instantiations compile in parallel.
#include "nll_avg.hpp"

namespace hf {
LaunchFn pick_avg_ng4(int bkg, int obj, bool grad, bool edges) {
  return pick_avg_ng<4>(bkg, obj, grad, edges);
}
LaunchFn pick_edges_ng4(int bkg, int obj, bool grad) { return pick_edges_ng<4>(bkg, obj, grad); }
}  // namespace hf
