// fisher_ng3.hip -- Fisher-information kernels of the 1D models with 3
// Gaussian(s); one translation unit per Gaussian count so the instantiations
// compile in parallel.
#include "fisher_kernels.hpp"

namespace hf {
FisherFn pick_fisher_ng3(int bkg, bool ney) { return pick_fisher_ng<3>(bkg, ney); }
}  // namespace hf
