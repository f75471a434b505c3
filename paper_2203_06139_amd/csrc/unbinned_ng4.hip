// unbinned_ng4.hip -- unbinned-NLL kernels of the models with 4 Gaussian(s);
// one translation unit per Gaussian count so the instantiations compile in
// parallel.
#include "unbinned.hpp"

namespace hf {
UnbinnedFn pick_unbinned_ng4(int bkg) { return pick_unbinned_ng<4>(bkg); }
}  // namespace hf
