// rng_aux_kernels.hpp -- the kernels around generation: seeding, the
// radix-16 thread-start tree of split and leapfrogged sequences, and a
// state copy, with their launchers (instantiated per generator together with
// the generation kernels of rng_kernels.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng_device.hpp"
#include "rng_internal.hpp"

namespace rngx {

inline unsigned grid_for(uint64_t lanes, int wg) { return (unsigned)((lanes + wg - 1) / wg); }

// ------------------------------------------------------------------ seeding
template <class G>
__global__ __launch_bounds__(256) void k_seed(uint32_t *__restrict__ st, uint64_t S, uint64_t seed,
                                              uint64_t first, DevTables tab)
{
    uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    uint64_t d[4];
#pragma unroll
    for (int j = 0; j < G::D; ++j) d[j] = splitmix64_at(seed, (first + s) * G::D + j);
    G g;
    g.seed(d, tab);
    g.store(st, S, s);
}

// One level of the radix-16 tree that starts the threads of a split
// sequence: thread t in [16^l, min(16^(l+1), T)), t = q 16^l + r with q in
// 1..15, starts where thread r starts, jumped by q 16^l unit samples.  For
// XS256 with a power-of-two unit, each workgroup stages the lookup tables of
// M^(unit 16^l 2^k), k < 4, in LDS (128 KiB: one 1024-lane workgroup per CU,
// 16 waves sharing them) and applies the set bits of q; the grid strides over
// the level.
constexpr int kTreeWG = 1024;

template <class G>
__global__ __launch_bounds__(kTreeWG) void k_tree_level(uint32_t *__restrict__ ws, uint64_t T, uint32_t shift,
                                                        uint64_t unit, DevTables tab)
{
    const uint64_t lo = (uint64_t)1 << shift;
    const uint64_t hi = min(lo << 4, T);
    const uint64_t n = hi - lo;
    const uint64_t first = (uint64_t)blockIdx.x * kTreeWG + threadIdx.x, stride = (uint64_t)gridDim.x * kTreeWG;
    if constexpr (G::kId == G_XS256) {
        __shared__ uint4 s_t4[4][2048];
        const uint32_t b0 = (uint32_t)__builtin_ctzll(unit) + shift;
        const bool staged = (unit & (unit - 1)) == 0 && b0 <= 60;
        if (staged) {
            stage_quads<kTreeWG, 4 * 2048>(&s_t4[0][0], tab.xs256_t4 + (size_t)b0 * 2048);  // tables b0 .. b0+3
            __syncthreads();
        }
        for (uint64_t i = first; i < n; i += stride) {
            const uint64_t t = lo + i, r = t & (lo - 1);
            G g;
            g.load(ws, T, r, tab);
            if (staged) {
                const uint32_t q = (uint32_t)(t >> shift);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if ((q >> k) & 1) g.jump_table(s_t4[k]);
            } else {
                g.jump((t - r) * unit, tab);
            }
            g.store(ws, T, t);
        }
    } else {
        for (uint64_t i = first; i < n; i += stride) {
            const uint64_t t = lo + i, r = t & (lo - 1);
            G g;
            g.load(ws, T, r, tab);
            g.jump((t - r) * unit, tab);
            g.store(ws, T, t);
        }
    }
}

// ------------------------------------------------------------------ helpers
// Copy one stream's state between a [W] contiguous buffer and slot `idx` of
// a [W][T] structure-of-arrays buffer.
template <int W>
__global__ void k_state_copy(const uint32_t *__restrict__ src, uint64_t src_stride, uint64_t src_idx,
                             uint32_t *__restrict__ dst, uint64_t dst_stride, uint64_t dst_idx)
{
    int w = threadIdx.x;
    if (w < W) dst[w * dst_stride + dst_idx] = src[w * src_stride + src_idx];
}

// ------------------------------------------------------------------ launchers

template <class G>
int launch_seed_t(uint64_t seed, uint64_t first, uint64_t S, uint32_t *st, const DevTables &tab,
                  hipStream_t stream)
{
    hipLaunchKernelGGL(k_seed<G>, dim3(grid_for(S, 256)), dim3(256), 0, stream, st, S, seed, first, tab);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class G>
int launch_tree_level_t(uint32_t *ws, uint64_t T, uint32_t shift, uint64_t unit, const DevTables &tab,
                        hipStream_t stream)
{
    // XS256 workgroups each stage 128 KiB of tables: one per CU, striding
    const uint64_t lo = (uint64_t)1 << shift, hi = (lo << 4) < T ? (lo << 4) : T;
    const unsigned cap = G::kId == G_XS256 ? 256 : 2048, blocks = grid_for(hi - lo, kTreeWG);
    hipLaunchKernelGGL(k_tree_level<G>, dim3(blocks < cap ? blocks : cap), dim3(kTreeWG), 0, stream, ws, T, shift,
                       unit, tab);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class G>
int launch_state_copy_t(const uint32_t *src, uint64_t ss, uint64_t si, uint32_t *dst, uint64_t ds,
                        uint64_t di, hipStream_t stream)
{
    hipLaunchKernelGGL(k_state_copy<G::W>, dim3(1), dim3(64), 0, stream, src, ss, si, dst, ds, di);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rngx
