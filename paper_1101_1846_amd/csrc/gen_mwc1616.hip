// Kernel instantiations for the MWC1616 generator.
#include "rng_kernels.hpp"

namespace rngx {
RNGX_INSTANTIATE(GenMWC1616)
RNGX_INSTANTIATE_TREE_HEAD(GenMWC1616)
}  // namespace rngx
