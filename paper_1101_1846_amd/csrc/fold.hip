// fold.hip -- the "without write-back" mode of the paper's tables (Sec.
// III.B, Tables I-III) for every generator: each stream draws n numbers
// (uint32 or their FP32 bit patterns), nothing is stored but the XOR of them
// and the final state.  Every number is computed (the XOR keeps it live and
// checkable), so the rate is the generator's VALU-bound rate.  Few streams
// are cut into chunks whose starts come from jump-ahead (uniform per wave);
// chunk folds combine by atomic XOR, and the states are then advanced by a
// separate skip launch (no chunk may overwrite a start state others read).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_abi_internal.hpp"

namespace rngx {

namespace {

struct FoldArgs {
    uint32_t *state;
    uint64_t ld, S, N;
    uint64_t C;  // chunk length
    uint32_t P;  // chunks per stream
    uint32_t *fold;
    DevTables tab;
};

template <int DT>
__device__ __forceinline__ uint32_t fold_bits(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

template <class G, int DT, int U>
__global__ __launch_bounds__(256) void k_fold(FoldArgs a)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint64_t sb = wave / a.P, j = wave - sb * a.P;
    const uint64_t s0 = sb * 64;
    if (s0 >= a.S) return;
    const uint64_t kb = j * a.C;
    if (kb >= a.N) return;
    const uint64_t ke = min(kb + a.C, a.N);
    const bool valid = s0 + lane < a.S;
    const uint64_t s = valid ? s0 + lane : s0;
    G g;
    g.load(a.state, a.ld, s, a.tab);
    if (j) g.jump(kb, a.tab);
    uint32_t acc = 0;
    uint64_t k = kb;
    for (; k + U <= ke; k += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= fold_bits<DT>(g.next());
    }
    for (; k < ke; ++k) acc ^= fold_bits<DT>(g.next());
    if (!valid) return;
    if (a.P == 1) a.fold[s] ^= acc;
    else atomicXor(&a.fold[s], acc);
    if (a.P == 1) g.store(a.state, a.ld, s);  // P > 1: the host skips the states by N
}

template <class G>
int launch_fold(int dt, const FoldArgs &a, hipStream_t st)
{
    const uint64_t waves = ((a.S + 63) / 64) * a.P;
    const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    if (dt == RNG_F32) hipLaunchKernelGGL((k_fold<G, RNG_DT_F32, 8>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_fold<G, RNG_DT_U32, 8>), grid, block, 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

}  // namespace rngx

using namespace rngx;

extern "C" int rng_generate_fold(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t, uint32_t *d_fold,
                                 void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (n_streams == 0 || n == 0) return RNG_OK;
    if (!d_state || !d_fold) return fail(RNG_EINVAL, "NULL state or fold");
    if (((uintptr_t)d_state & 3) || ((uintptr_t)d_fold & 3)) return fail(RNG_EINVAL, "misaligned pointer");
    if (int rc = check_sizes(n_streams, n, gen_words(g))) return rc;
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    FoldArgs a{};
    a.state = d_state;
    a.ld = n_streams;
    a.S = n_streams;
    a.N = n;
    a.fold = d_fold;
    a.tab = tab;
    choose_chunks(g, n_streams, n, 8, &a.C, &a.P, (uint64_t)1 << 17);
    hipStream_t st = (hipStream_t)stream;
    int rc = -2;
    switch (g) {
    case RNG_MWC32: rc = launch_fold<GenMWC32>(t, a, st); break;
    case RNG_XS256: rc = launch_fold<GenXS256>(t, a, st); break;
    case RNG_XS32: rc = launch_fold<GenXS32>(t, a, st); break;
    case RNG_KISS: rc = launch_fold<GenKISS>(t, a, st); break;
    case RNG_MWC1616: rc = launch_fold<GenMWC1616>(t, a, st); break;
    }
    if (int e = check_launch(rc, "rng_generate_fold")) return e;
    if (a.P == 1) return RNG_OK;
    return check_launch(dispatch_skip(g, d_state, n_streams, n_streams, n, tab, st), "rng_generate_fold: state");
}
