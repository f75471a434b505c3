// unbinned_ng0.hip -- unbinned-NLL kernels of the models with 0 Gaussian(s);
// one translation unit per Gaussian count so the instantiations compile in
// parallel.
#include "unbinned.hpp"

namespace hf {
UnbinnedFn pick_unbinned_ng0(int bkg) { return pick_unbinned_ng<0>(bkg); }
}  // namespace hf
