// Kernel instantiations for the XS32 generator.
#include "rng_kernels.hpp"

namespace rngx {
RNGX_INSTANTIATE(GenXS32)
RNGX_INSTANTIATE_TREE_HEAD(GenXS32)
}  // namespace rngx
