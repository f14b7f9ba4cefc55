// rng_batch_kernels.hip -- kernels of the batched path: chunk start states by
// jump-ahead (a root jump per request, then a radix-16 tree), and the
// dispatch to the persistent generation kernel (rng_batch_gen.hpp, built per
// workgroup size in batch_gen_*.hip), whose wavefronts pull 64-chunk tiles
// from an atomic counter until the batch is done.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng_batch_internal.hpp"
#include "rng_device.hpp"
#include "rng_internal.hpp"

namespace rngx {

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

__global__ __launch_bounds__(kRootWG) void k_batch_root(BatchArgs a, PlanInline pin)
{
    __shared__ uint32_t s_st[8 * kRootWG];  // leader states, [word][lane]
    const BatchHeader *hp = pin.bytes ? (const BatchHeader *)pin.q : a.hdr;
    if (pin.bytes && blockIdx.x == 0)  // the plan for the kernels after this one
        for (uint32_t i = threadIdx.x; i * 16 < pin.bytes; i += kRootWG) ((uint4 *)a.hdr)[i] = pin.q[i];
    const BatchHeader &h = *hp;
    const BatchReq *reqs = plan_at<const BatchReq>(hp, h.off_reqs);
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
        // tables L.pow .. L.pow + kRadixBits - 1, adjacent in memory
        stage_quads<kLevelWG, kRadixBits * 2048>(&s_t4[0][0], a.tab.xs256_t4 + (size_t)L.pow * 2048);
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

// Small batches (the plan in the kernel's arguments, at most 16^3 chunks per
// request): the whole radix-16 tree of each request in one launch, with the
// levels separated by barriers instead of launches.  Each request takes four
// workgroups that need nothing from each other: every one jumps the
// request's state by `offset` (as the root kernel's leader) and builds
// chunks 0 .. 255 (levels 0 and 1: chunk j of level l starts from chunk
// j mod 16^l, jumped by (j - j mod 16^l) C) in its own LDS, workgroup 0
// writes them out, and the four share level 2 (chunks 256 .. 4095), so its
// jumps spread over four CUs.  XS256 stages the tables of M^(C 16^l 2^k),
// k < 4, in LDS when C is a power of two; its level 2 then runs four lanes
// per source chunk: lane k starts chunk r + 256 (k + 1) with the tables of
// the set bits of k + 1, then each chunk 1024 further on with one product by
// M^(1024 C), at most 5 products in a row (the bit tables: up to 4 for each
// of up to 4 chunks per lane, on one CU, before).
constexpr int kTreeSmallWG = 256;
constexpr uint32_t kTreeSmallBlocks = 4;  // workgroups per request

__global__ __launch_bounds__(kTreeSmallWG) void k_batch_tree_small(BatchArgs a, PlanInline pin)
{
    __shared__ uint4 s_t4[kRadixBits * 2048];
    __shared__ uint32_t s_st[8 * 256];  // chunks 0 .. 255, [word][chunk]
    const BatchHeader &h = *(const BatchHeader *)pin.q;
    if (blockIdx.x == 0) {  // the plan for the generation kernel, and its tile counter
        for (uint32_t i = threadIdx.x; i * 16 < pin.bytes; i += kTreeSmallWG) ((uint4 *)a.hdr)[i] = pin.q[i];
        if (threadIdx.x == 0) a.counter[0] = 0;
    }
    const uint32_t r = blockIdx.x / kTreeSmallBlocks, b = blockIdx.x % kTreeSmallBlocks;
    if (r >= h.n) return;  // uniform per workgroup
    const BatchReq q = plan_at<const BatchReq>(&h, h.off_reqs)[r];
    if (b > 0 && q.nchunks <= 256) return;  // no level 2: workgroup 0 does it all
    const BatchGroup &gr = h.groups[q.group];
    uint32_t *ws = a.ws + gr.ws_off;
    uint32_t *map = a.chunk_req + gr.tile_begin * 64 + q.chunk_base;
    const uint32_t ld = gr.nchunks_pad, tid = threadIdx.x;
    if (tid == 0) {
        with_gen(gr.gen, [&]<class G>() {
            G g;
            g.load(q.state, q.stride, 0, a.tab);
            if (q.offset) g.jump(q.offset, a.tab);
            if (b == 0) {
                if (q.nchunks == 0) g.store(q.state, q.stride, 0);
                else g.store(ws, ld, q.chunk_base);
            }
            g.store(s_st, 256, 0);
        });
        if (b == 0 && q.nchunks) map[0] = r;
    }
    const bool xs = gr.gen == (uint32_t)G_XS256;
    const uint32_t pow0 = h.lvl[0].pow;  // log2 C, or 0xFFFFFFFF
    // levels 0 and 1: chunks [1, 16) and [16, 256) into LDS
    for (uint32_t l = 0, lo = 1; l < 2 && lo < q.nchunks; ++l, lo <<= kRadixBits) {
        const uint32_t pw = pow0 == 0xFFFFFFFFu ? 0xFFFFFFFFu : pow0 + kRadixBits * l;
        const bool staged = xs && pw <= 64 - kRadixBits;  // uniform per workgroup
        __syncthreads();  // the previous level's states are in LDS, and its tables read
        if (staged) {
            stage_quads<kTreeSmallWG, kRadixBits * 2048>(s_t4, a.tab.xs256_t4 + (size_t)pw * 2048);
            __syncthreads();
        }
        const uint32_t hi = min(lo << kRadixBits, q.nchunks), j = lo + tid;
        if (j < hi) {
            const uint32_t rem = j & (lo - 1), qd = j >> (kRadixBits * l);  // qd in 1 .. 15
            with_gen(gr.gen, [&]<class G>() {
                G g;
                g.load(s_st, 256, rem, a.tab);
                if constexpr (G::kId == G_XS256) {
                    if (staged) {
#pragma unroll
                        for (int k = 0; k < kRadixBits; ++k)
                            if ((qd >> k) & 1) g.jump_table(s_t4 + k * 2048);
                    } else {
                        g.jump((uint64_t)(j - rem) * h.C, a.tab);
                    }
                } else {
                    g.jump((uint64_t)(j - rem) * h.C, a.tab);
                }
                g.store(s_st, 256, j);
                if (b == 0) g.store(ws, ld, q.chunk_base + j);
            });
            if (b == 0) map[j] = r;
        }
    }
    // level 2: chunks [256, hi) from the 256 in LDS
    if (q.nchunks <= 256) return;  // uniform
    const uint32_t hi = min(256u << kRadixBits, q.nchunks);
    const uint32_t pw = pow0 == 0xFFFFFFFFu ? 0xFFFFFFFFu : pow0 + 2 * kRadixBits;
    __syncthreads();
    if (xs && pw <= 64 - kRadixBits) {
        stage_quads<kTreeSmallWG, 3 * 2048>(s_t4, a.tab.xs256_t4 + (size_t)pw * 2048);  // M^(256 C 2^k), k < 3
        __syncthreads();
        const uint32_t k = tid >> 6, src = b * 64 + (tid & 63);  // four lanes per source chunk
        if (src + 256 >= hi) return;
        const uint32_t room = (hi - 1 - src) >> 8;  // largest qd with src + 256 qd < hi
        GenXS256 g;
        g.load(s_st, 256, src, a.tab);
        for (uint32_t qd = k + 1; qd <= room; qd += 4) {
            if (qd == k + 1) {
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if ((qd >> e) & 1) g.jump_table(s_t4 + e * 2048);
            } else {
                g.jump_table(s_t4 + 2 * 2048);
            }
            const uint32_t j = src + (qd << 8);
            map[j] = r;
            g.store(ws, ld, q.chunk_base + j);
        }
        return;
    }
    for (uint32_t j = 256 + b * kTreeSmallWG + tid; j < hi; j += kTreeSmallBlocks * kTreeSmallWG) {
        const uint32_t rem = j & 255;
        map[j] = r;
        with_gen(gr.gen, [&]<class G>() {
            G g;
            g.load(s_st, 256, rem, a.tab);
            g.jump((uint64_t)(j - rem) * h.C, a.tab);
            g.store(ws, ld, q.chunk_base + j);
        });
    }
}

// ------------------------------------------------------------------ launchers
int launch_batch_root(const BatchArgs &a, const PlanInline &pin, uint32_t max_requests, hipStream_t s)
{
    const uint64_t lanes = (uint64_t)max_requests * 16, blocks = (lanes + kRootWG - 1) / kRootWG;
    const unsigned grid = (unsigned)(blocks < 1024 ? blocks : 1024);
    hipLaunchKernelGGL(k_batch_root, dim3(grid ? grid : 1), dim3(kRootWG), 0, s, a, pin);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_tree_small(const BatchArgs &a, const PlanInline &pin, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_tree_small, dim3(n ? n * kTreeSmallBlocks : 1), dim3(kTreeSmallWG), 0, s, a, pin);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_level(const BatchArgs &a, uint32_t level, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_level, dim3(grid), dim3(kLevelWG), 0, s, a, level);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int WG>
int batch_gen_wg(const BatchArgs &a, int unroll, unsigned grid, hipStream_t s, int *blocks);

static int batch_gen_dispatch(const BatchArgs &a, int wg, int unroll, unsigned grid, hipStream_t s, int *blocks)
{
    switch (wg) {
    case 64: return batch_gen_wg<64>(a, unroll, grid, s, blocks);
    case 128: return batch_gen_wg<128>(a, unroll, grid, s, blocks);
    case 256: return batch_gen_wg<256>(a, unroll, grid, s, blocks);
    case 512: return batch_gen_wg<512>(a, unroll, grid, s, blocks);
    case 1024: return batch_gen_wg<1024>(a, unroll, grid, s, blocks);
    }
    return -2;
}

int launch_batch_gen(const BatchArgs &a, int wg, int unroll, unsigned grid, hipStream_t s)
{
    return batch_gen_dispatch(a, wg, unroll, grid, s, nullptr);
}

int batch_gen_occupancy(int wg, int unroll, int *blocks_per_cu)
{
    if (!blocks_per_cu) return -1;
    return batch_gen_dispatch(BatchArgs{}, wg, unroll, 0, nullptr, blocks_per_cu);
}

}  // namespace rngx
