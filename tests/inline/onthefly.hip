// A consumer kernel written the way a user of the library would write one: it
// includes only the public headers, loads each stream's state from the
// layout rng_seed wrote, draws n numbers on the fly (no output buffer), and
// stores the state back.  Per stream it reports the XOR of the n outputs and
// how many of their FP32 uniforms fall below one half.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_inline.hpp"

template <class G>
__global__ __launch_bounds__(256) void k_onthefly(uint32_t *state, uint64_t S, uint64_t n, uint32_t *xor_out,
                                                  uint32_t *below_half)
{
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    G g;
    g.load(state, S, s);
    uint32_t x = 0, h = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t u = g.next();
        x ^= u;
        h += rng_inline::to_unit_f32(u) < 0.5f;
    }
    g.store(state, S, s);
    xor_out[s] = x;
    below_half[s] = h;
}

template <class G>
static int launch(uint32_t *state, uint64_t S, uint64_t n, uint32_t *x, uint32_t *h, hipStream_t st)
{
    const uint64_t blocks = (S + 255) / 256;
    if (blocks == 0) return 0;
    hipLaunchKernelGGL(k_onthefly<G>, dim3((unsigned)blocks), dim3(256), 0, st, state, S, n, x, h);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// gen: an rng_gen_t; state: [kWords][S] device words; x, h: [S] device words.
// Returns 0, -1 on a launch error, -2 for an unknown generator.
extern "C" int onthefly_draw(int gen, uint32_t *state, uint64_t S, uint64_t n, uint32_t *x, uint32_t *h,
                             void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (gen) {
    case RNG_MWC32: return launch<rng_inline::MWC32>(state, S, n, x, h, st);
    case RNG_XS256: return launch<rng_inline::XS256>(state, S, n, x, h, st);
    case RNG_XS32: return launch<rng_inline::XS32>(state, S, n, x, h, st);
    case RNG_KISS: return launch<rng_inline::KISS>(state, S, n, x, h, st);
    case RNG_MWC1616: return launch<rng_inline::MWC1616>(state, S, n, x, h, st);
    }
    return -2;
}
