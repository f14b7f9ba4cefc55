// Kernel instantiations for the MWC32 generator.
#include "rng_kernels.hpp"

namespace rngx {
RNGX_INSTANTIATE(GenMWC32)
RNGX_INSTANTIATE_TREE_HEAD(GenMWC32)
}  // namespace rngx
