// fisher_ng0.hip -- Fisher-information kernels of the 1D models with 0
// Gaussian(s); one translation unit per Gaussian count so the instantiations
// compile in parallel.
#include "fisher_kernels.hpp"

namespace hf {
FisherFn pick_fisher_ng0(int bkg, bool ney) { return pick_fisher_ng<0>(bkg, ney); }
}  // namespace hf
