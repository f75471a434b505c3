// unbinned_ng1.hip -- unbinned-NLL kernels of the models with 1 Gaussian(s);
// one translation unit per Gaussian count so the instantiations compile in
// parallel.
#include "unbinned.hpp"

namespace hf {
UnbinnedFn pick_unbinned_ng1(int bkg) { return pick_unbinned_ng<1>(bkg); }
}  // namespace hf
