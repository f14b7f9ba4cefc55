// Kernel instantiations for the XS256 generator.
#include "rng_kernels.hpp"

namespace rngx {
RNGX_INSTANTIATE(GenXS256)
RNGX_INSTANTIATE_TREE_HEAD(GenXS256)
}  // namespace rngx
