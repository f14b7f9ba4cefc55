// Kernel instantiations for the KISS generator.
#include "rng_kernels.hpp"

namespace rngx {
RNGX_INSTANTIATE(GenKISS)
RNGX_INSTANTIATE_TREE_HEAD(GenKISS)
}  // namespace rngx
