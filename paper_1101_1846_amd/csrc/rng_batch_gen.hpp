// rng_batch_gen.hpp -- the persistent generation kernel of the batched path,
// included by one translation unit per workgroup size (batch_gen_*.hip) so
// that its 25 (workgroup, unroll) shapes compile in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng_batch_internal.hpp"
#include "rng_device.hpp"
#include "rng_internal.hpp"

namespace rngx {

#define RNGX_COMPILER_FENCE() asm volatile("" ::: "memory")
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Pointers read from the request table are generic to the compiler, which
// would address through FLAT instructions; FLAT accesses also count as LDS
// traffic and serialise with the tile's LDS reads.  These buffers are device
// global memory: say so, so that loads and stores are global_*.
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) u32x4 gu32x4;

__device__ __forceinline__ gu32 *global_ptr(uint32_t *p) { return (gu32 *)p; }

// LDS tile depth of the generation kernel: kBatchTile samples per row, or 32
// for 1024-lane workgroups, whose 16 tiles of 64 rows would not fit in the
// 160 KiB of LDS at 64 (chunk lengths are multiples of kBatchTile, so of both).
constexpr int batch_tile_depth(int wg) { return wg >= 1024 ? 32 : kBatchTile; }

template <int DT>
__device__ __forceinline__ uint32_t bits_of(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

// One 64-chunk tile: lane l generates chunk chunk0 + l of the group into its
// LDS row, K samples at a time; rows are then stored with consecutive lanes on
// consecutive words of one chunk's output.
template <class G, int DT, int U, int K>
__device__ void batch_tile(const BatchArgs &a, const BatchGroup &gr, uint32_t tile, uint32_t *lds_tile,
                           uint32_t **row_ptr, uint32_t *row_len)
{
    static_assert(K % U == 0 && K % 4 == 0 && kBatchTile % K == 0, "tile depth");
    constexpr int LD = K + 4;
    const BatchHeader &h = *a.hdr;
    const int lane = threadIdx.x & 63;
    const uint32_t c0 = (tile - gr.tile_begin) * 64;
    const bool active = c0 + lane < gr.nchunks;
    const uint32_t c = active ? c0 + lane : c0;
    // the chunk's request (the root and tree kernels wrote the map)
    const BatchReq q = plan_at<const BatchReq>(a.hdr, h.off_reqs)[a.chunk_req[gr.tile_begin * 64 + c]];
    const uint64_t j = c - q.chunk_base;
    const uint64_t start = j * h.C;
    const uint32_t len = active ? (uint32_t)min<uint64_t>(h.C, q.length - start) : 0;
    uint32_t *dst = q.out + start;

    G g;
    g.load(a.ws + gr.ws_off, gr.nchunks_pad, c, a.tab);

    row_ptr[lane] = dst;
    row_len[lane] = len;
    uint32_t maxlen = len;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlen = max(maxlen, (uint32_t)__shfl_xor((int)maxlen, off, 64));
    const bool aligned = __all(((uintptr_t)dst & 15) == 0);
    uint32_t *row = lds_tile + lane * LD;

    for (uint32_t k0 = 0; k0 < maxlen; k0 += K) {
        // Lanes with a whole block left take the unrolled path together; only
        // the lanes in the final partial block of their chunk (the last chunk
        // of a request) step one sample at a time, so that they stop exactly
        // at the chunk's end.
        if (k0 + K <= len) {
#pragma unroll 1
            for (int k = 0; k < K; k += U) {
                uint32_t v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = bits_of<DT>(g.next());
                if constexpr (U % 4 == 0) {
#pragma unroll
                    for (int u = 0; u < U; u += 4) *(uint4 *)&row[k + u] = make_uint4(v[u], v[u + 1], v[u + 2], v[u + 3]);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) row[k + u] = v[u];
                }
            }
        } else if (k0 < len) {
            for (uint32_t k = 0; k < len - k0; ++k) row[k] = bits_of<DT>(g.next());
        }
        RNGX_COMPILER_FENCE();
        if (aligned) {
            constexpr int QPR = K / 4, RPI = 64 / QPR;
            const int rr = lane / QPR, qq = lane % QPR;
#pragma unroll 4
            for (int i = 0; i < QPR; ++i) {
                const int r = i * RPI + rr;
                const uint32_t col = k0 + 4 * qq, n = row_len[r];
                gu32 *p = global_ptr(row_ptr[r]) + col;
                const uint32_t *s = lds_tile + r * LD + 4 * qq;
                if (col + 4 <= n) {
                    *(gu32x4 *)p = *(const u32x4 *)s;
                } else if (col < n) {
                    for (uint32_t e = 0; e < n - col; ++e) p[e] = s[e];
                }
            }
        } else {
            constexpr int RPI = 64 / K;
            const int rr = lane / K, cc = lane % K;
#pragma unroll 4
            for (int i = 0; i < K; ++i) {
                const int r = i * RPI + rr;
                const uint32_t col = k0 + cc;
                if (col < row_len[r]) global_ptr(row_ptr[r])[col] = lds_tile[r * LD + cc];
            }
        }
        RNGX_COMPILER_FENCE();
    }
    if (active && j + 1 == q.nchunks) g.store(q.state, q.stride, 0);
}

// Persistent generation.  Wave w of the grid's W waves takes tile w first;
// the tiles from W on are pulled from an atomic counter (reset by the root
// kernel), so a batch with fewer tiles than waves issues no atomics and the
// waves without a tile leave at once.
template <int WG, int U>
__global__ __launch_bounds__(WG) void k_batch_gen(BatchArgs a)
{
    constexpr int K = batch_tile_depth(WG), NW = WG / 64, LD = K + 4;
    __shared__ __attribute__((aligned(16))) uint32_t lds[NW * 64 * LD];
    __shared__ uint32_t *rptr[NW * 64];
    __shared__ uint32_t rlen[NW * 64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const BatchHeader &h = *a.hdr;
    const uint32_t nwaves = gridDim.x * NW;
    uint32_t t = blockIdx.x * NW + wv;
    for (;; ) {
        if (t >= h.n_tiles) break;
        uint32_t gi = 0;
        while (gi + 1 < h.ngroups && t >= h.groups[gi].tile_end) ++gi;
        const BatchGroup &gr = h.groups[gi];
        const uint32_t key = gr.gen * 2 + gr.dtype;
        uint32_t *tile = &lds[wv * 64 * LD];
        switch (key) {
#define RNGX_BATCH_CASE(GEN, ID)                                                                   \
    case ID * 2 + RNG_DT_U32: batch_tile<GEN, RNG_DT_U32, U, K>(a, gr, t, tile, &rptr[wv * 64], &rlen[wv * 64]); break; \
    case ID * 2 + RNG_DT_F32: batch_tile<GEN, RNG_DT_F32, U, K>(a, gr, t, tile, &rptr[wv * 64], &rlen[wv * 64]); break;
            RNGX_BATCH_CASE(GenMWC32, G_MWC32)
            RNGX_BATCH_CASE(GenXS256, G_XS256)
            RNGX_BATCH_CASE(GenXS32, G_XS32)
            RNGX_BATCH_CASE(GenKISS, G_KISS)
            RNGX_BATCH_CASE(GenMWC1616, G_MWC1616)
#undef RNGX_BATCH_CASE
        }
        if (nwaves >= h.n_tiles) break;  // every tile was handed out statically
        uint32_t next = 0;
        if (lane == 0) next = atomicAdd(a.counter, 1u);
        t = nwaves + __builtin_amdgcn_readfirstlane(__shfl(next, 0, 64));
    }
}


template <int WG, int U>
static int gen_t(const BatchArgs &a, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch_gen<WG, U>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int WG, int U>
static int occ_t(int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_gen<WG, U>, WG, 0) == hipSuccess ? 0 : -1;
}

// Launch (occupancy query with grid == 0 and blocks != nullptr) for one
// workgroup size and any unroll in {1, 2, 4, 8, 16}; -2 for other unrolls.
template <int WG>
int batch_gen_wg(const BatchArgs &a, int unroll, unsigned grid, hipStream_t s, int *blocks)
{
    switch (unroll) {
#define RNGX_U(U) case U: return blocks ? occ_t<WG, U>(blocks) : gen_t<WG, U>(a, grid, s);
    RNGX_U(1) RNGX_U(2) RNGX_U(4) RNGX_U(8) RNGX_U(16)
#undef RNGX_U
    }
    return -2;
}

#define RNGX_BATCH_GEN_INSTANTIATE(WG) \
    template int batch_gen_wg<WG>(const BatchArgs &, int, unsigned, hipStream_t, int *);

}  // namespace rngx
