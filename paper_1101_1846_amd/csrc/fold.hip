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
    uint64_t C;      // chunk length
    uint32_t P;      // chunks per stream
    uint32_t lanes;  // fewer streams than lanes: lane v takes chunk v mod P of stream v / P
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
    uint64_t s, kb, ke;
    bool valid;
    if (a.lanes) {
        // one chunk per lane: its own stream, start and (per-lane) jump
        const uint64_t total = a.S * a.P, v = wave * 64 + lane;
        if (wave * 64 >= total) return;  // whole waves
        valid = v < total;
        s = valid ? v / a.P : 0;
        kb = valid ? (v - s * a.P) * a.C : 0;
        ke = valid ? min(kb + a.C, a.N) : 0;
    } else {
        const uint64_t sb = wave / a.P, j = wave - sb * a.P;
        const uint64_t s0 = sb * 64;
        if (s0 >= a.S) return;
        kb = j * a.C;
        if (kb >= a.N) return;
        ke = min(kb + a.C, a.N);
        valid = s0 + lane < a.S;
        s = valid ? s0 + lane : s0;
    }
    G g;
    g.load(a.state, a.ld, s, a.tab);
    if (kb) g.jump(kb, a.tab);
    uint32_t acc = 0;
    uint64_t k = kb;
    for (; k + U <= ke; k += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= fold_bits<DT>(g.next());
    }
    for (; k < ke; ++k) acc ^= fold_bits<DT>(g.next());
    if (a.lanes) {
        // Many lanes hold chunks of one stream: XOR them within the wave first
        // (the streams of the first and the last lane), so that a wave issues
        // at most two atomics there instead of 64 on one word.
        const uint32_t sl = (uint32_t)s;
        const uint32_t s_first = __shfl(sl, 0, 64), s_last = __shfl(sl, 63, 64);
        const bool valid_last = __shfl((int)valid, 63, 64) != 0;
        uint32_t x0 = valid && sl == s_first ? acc : 0u;
        uint32_t x1 = valid && sl == s_last && sl != s_first ? acc : 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            x0 ^= (uint32_t)__shfl_xor((int)x0, off, 64);
            x1 ^= (uint32_t)__shfl_xor((int)x1, off, 64);
        }
        if (lane == 0) atomicXor(&a.fold[s_first], x0);
        if (lane == 63 && valid_last && s_last != s_first) atomicXor(&a.fold[s_last], x1);
        if (valid && sl != s_first && sl != s_last) atomicXor(&a.fold[s], acc);  // streams between them
        return;  // P > 1: the host skips the states by N
    }
    if (!valid) return;
    if (a.P == 1) a.fold[s] ^= acc;
    else atomicXor(&a.fold[s], acc);
    if (a.P == 1) g.store(a.state, a.ld, s);  // P > 1: the host skips the states by N
}

template <class G>
int launch_fold(int dt, const FoldArgs &a, hipStream_t st)
{
    const uint64_t waves = a.lanes ? (a.S * a.P + 63) / 64 : ((a.S + 63) / 64) * a.P;
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
    if (n_streams < 64) {
        lane_chunks(g, n_streams, n, &a.C, &a.P);
        a.lanes = a.P > 1;
        if (a.P == 1) a.C = n;
    } else {
        choose_chunks(g, n_streams, n, 8, &a.C, &a.P, (uint64_t)1 << 17);
    }
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
