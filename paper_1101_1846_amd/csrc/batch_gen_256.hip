// batch_gen_256.hip -- the batched path's persistent generation kernel for
// 256-lane workgroups, every unroll (one translation unit per workgroup size).
#include "rng_batch_gen.hpp"

namespace rngx {
RNGX_BATCH_GEN_INSTANTIATE(256)
}  // namespace rngx
