// batch_gen_1024.hip -- the batched path's persistent generation kernel for
// 1024-lane workgroups, every unroll (one translation unit per workgroup size).
#include "rng_batch_gen.hpp"

namespace rngx {
RNGX_BATCH_GEN_INSTANTIATE(1024)
}  // namespace rngx
