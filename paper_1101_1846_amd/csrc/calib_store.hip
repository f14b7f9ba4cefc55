// calib_store.hip -- the achievable write rate of the bulk store schedule.
// The paper measured its achievable bandwidth beside its kernels (Sec. V);
// a plain fill gives the linear ceiling, but the generators write
// stream-major rows through the LDS transpose.  This runs the generation
// kernel itself (same resident schedule, tiles, pipelined 16-byte stores,
// one-word state read and write-back) with a counter in place of a
// generator, so the only difference from a generator launch is the
// arithmetic per sample.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_abi_internal.hpp"
#include "rng_kernels.hpp"

namespace rngx {

namespace {

// Sample k of a stream whose state word is y is y + k + 1 (mod 2^32), and the
// state advances by the number of samples.  Its id is no generator's, so the
// kernel takes none of the generator-specific paths (the rotated row order).
struct GenCount {
    static constexpr int kId = 0, W = 1, D = 1;
    uint32_t y;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t, uint64_t s, const DevTables &) { y = st[s]; }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t, uint64_t s) const { st[s] = y; }
    __device__ __forceinline__ uint32_t next() { return ++y; }
    __device__ __forceinline__ void jump(uint64_t k, const DevTables &) { y += (uint32_t)k; }
};

}  // namespace

}  // namespace rngx

using namespace rngx;

extern "C" int rng_calibrate_store(uint32_t *d_state, uint64_t n_streams, uint64_t n, void *d_out, uint32_t wg,
                                   uint32_t unroll, void *stream)
{
    if (!valid_shape(wg, unroll)) return fail(RNG_EINVAL, "launch shape wg=%u unroll=%u", wg, unroll);
    if (n_streams == 0 || n == 0) return RNG_OK;
    if (!d_state || !d_out) return fail(RNG_EINVAL, "NULL state or output");
    if (((uintptr_t)d_state & 3) || ((uintptr_t)d_out & 3))
        return fail(RNG_EINVAL, "state and output must be 4-byte aligned");
    if (int rc = check_sizes(n_streams, n, 1)) return rc;
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    GenArgs a{};
    a.state = d_state;
    a.ld = n_streams;
    a.S = n_streams;
    a.N = n;
    a.out = d_out;
    a.C = n;  // one chunk per stream: the bulk schedule
    a.P = 1;
    a.vec4 = (n % 4 == 0) && (((uintptr_t)d_out & 15) == 0);
    a.tab = tab;
    return check_launch(launch_generate_wg<GenCount, RNG_DT_U32>(a, (int)wg, (int)unroll, true, (hipStream_t)stream),
                        "rng_calibrate_store");
}
