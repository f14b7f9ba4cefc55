// rng_batch_kernels.hip -- kernels of the batched path: chunk start states by
// jump-ahead (a root jump per request, then a radix-16 tree), and one
// persistent generation kernel whose wavefronts pull 64-chunk tiles from an
// atomic counter until the batch is done.
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

// Calls F.template operator()<Generator>() for the generator id g.
template <class F>
__device__ __forceinline__ void with_gen(uint32_t g, F &&f)
{
    switch (g) {
    case G_MWC32: f.template operator()<GenMWC32>(); break;
    case G_XS256: f.template operator()<GenXS256>(); break;
    case G_XS32: f.template operator()<GenXS32>(); break;
    case G_KISS: f.template operator()<GenKISS>(); break;
    case G_MWC1616: f.template operator()<GenMWC1616>(); break;
    }
}

// Root of each request's tree and its first level, 16 lanes per request:
// the leading lane jumps the request's state by `offset` (the start of chunk
// 0, or, for an empty request, the state written straight back) and passes it
// through LDS to the other 15, and lane j < nchunks starts chunk j from it,
// jumped by j C (level 0 of the radix-16 tree).  Also clears the generation
// kernel's tile counter.
constexpr int kRootWG = 256;

__global__ __launch_bounds__(kRootWG) void k_batch_root(BatchArgs a)
{
    __shared__ uint32_t s_st[8 * kRootWG];  // leader states, [word][lane]
    const BatchHeader &h = *a.hdr;
    const BatchReq *reqs = plan_at<const BatchReq>(a.hdr, h.off_reqs);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counter[0] = 0;  // tile counter of the generation kernel
    const uint32_t j = threadIdx.x & 15, lead = threadIdx.x & ~15u;
    // uniform over the workgroup: every lane takes part in each barrier
    for (uint32_t base = blockIdx.x * kRootWG; base < h.n * 16; base += gridDim.x * kRootWG) {
        const uint32_t r = (base + threadIdx.x) >> 4;
        const bool live = r < h.n;
        const BatchReq q = reqs[live ? r : 0];
        const BatchGroup &gr = h.groups[q.group];
        if (live && j == 0) {
            if (q.nchunks) a.chunk_req[gr.tile_begin * 64 + q.chunk_base] = r;
            with_gen(gr.gen, [&]<class G>() {
                G g;
                g.load(q.state, q.stride, 0, a.tab);
                if (q.offset) g.jump(q.offset, a.tab);
                if (q.nchunks == 0) g.store(q.state, q.stride, 0);
                else g.store(a.ws + gr.ws_off, gr.nchunks_pad, q.chunk_base);
                g.store(s_st, kRootWG, threadIdx.x);
            });
        }
        __syncthreads();
        if (live && j > 0 && j < q.nchunks) {
            const uint32_t c = q.chunk_base + j;
            a.chunk_req[gr.tile_begin * 64 + c] = r;
            with_gen(gr.gen, [&]<class G>() {
                G g;
                g.load(s_st, kRootWG, lead, a.tab);
                g.jump((uint64_t)j * h.C, a.tab);
                g.store(a.ws + gr.ws_off, gr.nchunks_pad, c);
            });
        }
        __syncthreads();  // the leaders' LDS slots are read before the next round writes them
    }
}

// Level l >= 1 of the radix-16 tree: chunk j in [16^l, min(16^(l+1), nchunks)) of
// every request, j = q 16^l + r, starts where chunk r starts, jumped by
// q 16^l C.  A block takes kLevelWG consecutive work items: it loads the
// kLevelWG segments from its first item's segment on (a block spans at most
// that many) into LDS, and every thread finds its request there.  XS256
// applies the set bits of q with the lookup tables of M^(C 16^l 2^k), k < 4,
// staged in LDS once per block (128 KiB: one 1024-lane block per CU).
__global__ __launch_bounds__(kLevelWG) void k_batch_level(BatchArgs a, uint32_t level)
{
    __shared__ uint4 s_t4[kRadixBits][2048];
    __shared__ uint32_t s_pre[kLevelWG], s_req[kLevelWG];
    const BatchHeader &h = *a.hdr;
    if (level >= h.levels) return;
    const BatchReq *reqs = plan_at<const BatchReq>(a.hdr, h.off_reqs);
    const uint2 *seg = plan_at<const uint2>(a.hdr, h.off_seg);
    const uint32_t *blk_first = plan_at<const uint32_t>(a.hdr, h.off_blk);
    const LevelInfo L = h.lvl[level];
    const uint32_t total = h.level_total[level];
    const uint32_t nblk = (total + kLevelWG - 1) / kLevelWG;
    if (blockIdx.x >= nblk) return;
    // pow is 0xFFFFFFFF when C is no power of two: compare without adding to it
    const bool staged = h.has_xs256 && L.pow <= 64 - kRadixBits;
    if (staged) {
#pragma unroll
        for (int k = 0; k < kRadixBits; ++k) stage_t4(s_t4[k], a.tab.xs256_t4 + (size_t)(L.pow + k) * 2048);
    }
    const uint32_t lo = 1u << L.shift;
    for (uint32_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const uint32_t k = blk_first[L.blk_off + blk] + threadIdx.x;
        __syncthreads();  // the previous block's segments are consumed (and the tables are staged)
        if (k < L.seg_n) {
            const uint2 sg = seg[L.seg_off + k];
            s_req[threadIdx.x] = sg.x;
            s_pre[threadIdx.x] = sg.y;
        } else {
            s_req[threadIdx.x] = 0;
            s_pre[threadIdx.x] = 0xFFFFFFFFu;
        }
        __syncthreads();
        const uint32_t t = blk * kLevelWG + threadIdx.x;
        if (t >= total) continue;
        uint32_t i = 0;  // largest i with s_pre[i] <= t (s_pre[0] <= t by construction)
#pragma unroll
        for (uint32_t step = kLevelWG / 2; step; step >>= 1)
            if (s_pre[i + step] <= t) i += step;
        const uint32_t r = s_req[i];
        const BatchReq q = reqs[r];
        const BatchGroup &gr = h.groups[q.group];
        const uint32_t j = lo + (t - s_pre[i]);  // chunk within the request
        const uint32_t rem = j & (lo - 1);       // the chunk it starts from
        const uint32_t qd = j >> L.shift;        // in 1 .. 15
        const uint32_t c = q.chunk_base + j;
        a.chunk_req[gr.tile_begin * 64 + c] = r;
        uint32_t *ws = a.ws + gr.ws_off;
        with_gen(gr.gen, [&]<class G>() {
            G g;
            g.load(ws, gr.nchunks_pad, q.chunk_base + rem, a.tab);
            if constexpr (G::kId == G_XS256) {
                if (staged) {
#pragma unroll
                    for (int b = 0; b < kRadixBits; ++b)
                        if ((qd >> b) & 1) g.jump_table(s_t4[b]);
                } else {
                    g.jump((uint64_t)(j - rem) * h.C, a.tab);
                }
            } else {
                g.jump((uint64_t)(j - rem) * h.C, a.tab);
            }
            g.store(ws, gr.nchunks_pad, c);
        });
    }
}

template <int DT>
__device__ __forceinline__ uint32_t bits_of(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

// One 64-chunk tile: lane l generates chunk chunk0 + l of the group into its
// LDS row; rows are then stored with consecutive lanes on consecutive words of
// one chunk's output.
template <class G, int DT, int U>
__device__ void batch_tile(const BatchArgs &a, const BatchGroup &gr, uint32_t tile, uint32_t *lds_tile,
                           uint32_t **row_ptr, uint32_t *row_len)
{
    constexpr int K = kBatchTile, LD = K + 4;
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
    constexpr int NW = WG / 64, LD = kBatchTile + 4;
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
    case ID * 2 + RNG_DT_U32: batch_tile<GEN, RNG_DT_U32, U>(a, gr, t, tile, &rptr[wv * 64], &rlen[wv * 64]); break; \
    case ID * 2 + RNG_DT_F32: batch_tile<GEN, RNG_DT_F32, U>(a, gr, t, tile, &rptr[wv * 64], &rlen[wv * 64]); break;
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

// ------------------------------------------------------------------ launchers
int launch_batch_root(const BatchArgs &a, uint32_t max_requests, hipStream_t s)
{
    const uint64_t lanes = (uint64_t)max_requests * 16, blocks = (lanes + kRootWG - 1) / kRootWG;
    const unsigned grid = (unsigned)(blocks < 1024 ? blocks : 1024);
    hipLaunchKernelGGL(k_batch_root, dim3(grid ? grid : 1), dim3(kRootWG), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_level(const BatchArgs &a, uint32_t level, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_level, dim3(grid), dim3(kLevelWG), 0, s, a, level);
    return hipGetLastError() == hipSuccess ? 0 : -1;
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

#define RNGX_BATCH_SHAPES(X) \
    X(64, 8) X(128, 8) X(256, 8) X(512, 8) X(256, 1) X(256, 2) X(256, 4) X(256, 16)

int launch_batch_gen(const BatchArgs &a, int wg, int unroll, unsigned grid, hipStream_t s)
{
#define X(W, U) if (wg == W && unroll == U) return gen_t<W, U>(a, grid, s);
    RNGX_BATCH_SHAPES(X)
#undef X
    return -2;
}

int batch_gen_occupancy(int wg, int unroll, int *blocks_per_cu)
{
#define X(W, U) if (wg == W && unroll == U) return occ_t<W, U>(blocks_per_cu);
    RNGX_BATCH_SHAPES(X)
#undef X
    return -2;
}

}  // namespace rngx
