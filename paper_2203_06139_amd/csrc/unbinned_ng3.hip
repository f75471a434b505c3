// unbinned_ng3.hip -- unbinned-NLL kernels of the models with 3 Gaussian(s);
// one translation unit per Gaussian count so the instantiations compile in
// parallel.
#include "unbinned.hpp"

namespace hf {
UnbinnedFn pick_unbinned_ng3(int bkg) { return pick_unbinned_ng<3>(bkg); }
}  // namespace hf
