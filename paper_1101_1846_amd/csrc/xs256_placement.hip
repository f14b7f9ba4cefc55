// xs256_placement.hip -- the paper's XorShift placement comparison (Sec.
// III.A.2, Table II) on gfx950: the r = 8 XorShift of eq. (5) with its state
//   0  in LDS, addressed through a runtime circular index (the form of the
//      reference C code, one number per call);
//   1  in LDS, with the circular buffer made explicit by an 8-fold unroll
//      (constant offsets, no index arithmetic);
//   2  in VGPRs (the explicit buffer in registers; the library's form).
// Each thread owns one stream.  In LDS its eight words are blockDim-strided
// (word i of thread t at i * 256 + t), the paper's conflict-free layout, and
// every access is volatile so the state really lives there.  All three
// produce the same numbers: one tap function (rng_inline::XS256::step).
//
// Output is either every number, sample-major (number k of stream s at
// out[k * S + s]: one coalesced 256-byte row per wave and number, the same
// store for all three placements), or, with no output, the XOR of each
// stream's numbers (so that the generation is live but nothing is stored).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_abi_internal.hpp"

namespace rngx {

namespace {

template <int DT>
__device__ __forceinline__ uint32_t emit_bits(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

constexpr int kWG = 256;

// LDS words accessed as such: volatile keeps every read and write, and the
// explicit address space keeps them ds_read / ds_write rather than FLAT.
typedef __attribute__((address_space(3))) volatile uint32_t lds_word;

template <int PLACE, int DT, bool FOLD>
__global__ __launch_bounds__(kWG) void k_xs256_placement(uint32_t *__restrict__ st, uint64_t S, uint64_t N,
                                                         uint32_t *__restrict__ out, uint32_t *__restrict__ fold)
{
    __shared__ uint32_t lds[PLACE == 2 ? 1 : 8 * kWG];
    const uint64_t s = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (s >= S) return;  // no barriers below: each thread's LDS words are its own
    uint32_t acc = 0;
    uint32_t *o = FOLD ? nullptr : out + s;
    auto emit = [&](uint64_t k, uint32_t u) {
        const uint32_t b = emit_bits<DT>(u);
        if constexpr (FOLD) acc ^= b;
        else o[k * S] = b;
    };
    using rng_inline::XS256;
    if constexpr (PLACE == 2) {
        GenXS256 g;
        g.load(st, S, s);
        uint64_t k = 0;
        for (; k + 8 <= N; k += 8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) emit(k + j, g.next());
        }
        for (; k < N; ++k) emit(k, g.next());
        g.store(st, S, s);
    } else {
        lds_word *w = (lds_word *)lds + threadIdx.x;  // word i at w[i * kWG]
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i * kWG] = st[i * S + s];
        // c: slot of v_{n-8}; the slot after it holds v_{n-7}, ..., c + 7 holds v_{n-1}
        uint32_t c = 0;
        uint64_t k = 0;
        if constexpr (PLACE == 1) {
            for (; k + 8 <= N; k += 8) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t vn = XS256::step(w[((j + 7) & 7) * kWG], w[((j + 4) & 7) * kWG],
                                                    w[((j + 3) & 7) * kWG], w[((j + 1) & 7) * kWG], w[j * kWG]);
                    w[j * kWG] = vn;
                    emit(k + j, vn);
                }
            }
        }
#pragma unroll 1
        for (; k < N; ++k) {
            const uint32_t vn = XS256::step(w[((c + 7) & 7) * kWG], w[((c + 4) & 7) * kWG], w[((c + 3) & 7) * kWG],
                                            w[((c + 1) & 7) * kWG], w[c * kWG]);
            w[c * kWG] = vn;
            c = (c + 1) & 7;
            emit(k, vn);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) st[i * S + s] = w[((c + i) & 7) * kWG];
    }
    if constexpr (FOLD) fold[s] = acc;
}

template <int PLACE, int DT>
int launch_placement(uint32_t *st, uint64_t S, uint64_t N, uint32_t *out, uint32_t *fold, hipStream_t stream)
{
    const dim3 grid((unsigned)((S + kWG - 1) / kWG)), block(kWG);
    if (fold) hipLaunchKernelGGL((k_xs256_placement<PLACE, DT, true>), grid, block, 0, stream, st, S, N, out, fold);
    else hipLaunchKernelGGL((k_xs256_placement<PLACE, DT, false>), grid, block, 0, stream, st, S, N, out, fold);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int PLACE>
int launch_dt(int dt, uint32_t *st, uint64_t S, uint64_t N, uint32_t *out, uint32_t *fold, hipStream_t stream)
{
    return dt == RNG_F32 ? launch_placement<PLACE, RNG_DT_F32>(st, S, N, out, fold, stream)
                         : launch_placement<PLACE, RNG_DT_U32>(st, S, N, out, fold, stream);
}

}  // namespace

}  // namespace rngx

using namespace rngx;

extern "C" int rng_xs256_placement(int placement, uint32_t *d_state, uint64_t n_streams, uint64_t n, int dtype,
                                   void *d_out, uint32_t *d_fold, void *stream)
{
    if (placement < RNG_XS_LDS_INDEXED || placement > RNG_XS_VGPR)
        return fail(RNG_EINVAL, "unknown state placement %d", placement);
    if (dtype != RNG_U32 && dtype != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", dtype);
    if ((d_out == nullptr) == (d_fold == nullptr))
        return fail(RNG_EINVAL, "exactly one of d_out and d_fold must be given");
    if (n_streams == 0) return RNG_OK;
    if (!d_state || ((uintptr_t)d_state & 3)) return fail(RNG_EINVAL, "d_state is NULL or not 4-byte aligned");
    if (d_out && ((uintptr_t)d_out & 3)) return fail(RNG_EINVAL, "d_out not 4-byte aligned");
    if (d_fold && ((uintptr_t)d_fold & 3)) return fail(RNG_EINVAL, "d_fold not 4-byte aligned");
    if (int rc = check_sizes(n_streams, n, 8)) return rc;
    if (n_streams > ((uint64_t)1 << 31)) return fail(RNG_ERANGE, "n_streams above 2^31");
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;  // also checks for a gfx950 device
    uint32_t *out = (uint32_t *)d_out;
    hipStream_t st = (hipStream_t)stream;
    int rc = -2;
    switch (placement) {
    case RNG_XS_LDS_INDEXED: rc = launch_dt<0>(dtype, d_state, n_streams, n, out, d_fold, st); break;
    case RNG_XS_LDS_UNROLLED: rc = launch_dt<1>(dtype, d_state, n_streams, n, out, d_fold, st); break;
    case RNG_XS_VGPR: rc = launch_dt<2>(dtype, d_state, n_streams, n, out, d_fold, st); break;
    }
    return check_launch(rc, "rng_xs256_placement");
}
