// fisher_ng1.hip -- Fisher-information kernels of the 1D models with 1
// Gaussian(s); one translation unit per Gaussian count so the instantiations
// compile in parallel.
#include "fisher_kernels.hpp"

namespace hf {
FisherFn pick_fisher_ng1(int bkg, bool ney) { return pick_fisher_ng<1>(bkg, ney); }
}  // namespace hf
