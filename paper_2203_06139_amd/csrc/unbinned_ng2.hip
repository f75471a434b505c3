// unbinned_ng2.hip -- unbinned-NLL kernels of the models with 2 Gaussian(s);
// one translation unit per Gaussian count so the instantiations compile in
// parallel.
#include "unbinned.hpp"

namespace hf {
UnbinnedFn pick_unbinned_ng2(int bkg) { return pick_unbinned_ng<2>(bkg); }
}  // namespace hf
