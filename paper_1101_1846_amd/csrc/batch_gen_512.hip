// batch_gen_512.hip -- the batched path's persistent generation kernel for
// 512-lane workgroups, every unroll (one translation unit per workgroup size).
#include "rng_batch_gen.hpp"

namespace rngx {
RNGX_BATCH_GEN_INSTANTIATE(512)
}  // namespace rngx
