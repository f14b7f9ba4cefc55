// batch_gen_64.hip -- the batched path's persistent generation kernel for
// 64-lane workgroups, every unroll (one translation unit per workgroup size).
#include "rng_batch_gen.hpp"

namespace rngx {
RNGX_BATCH_GEN_INSTANTIATE(64)
}  // namespace rngx
