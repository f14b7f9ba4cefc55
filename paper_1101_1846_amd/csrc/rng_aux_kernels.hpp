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
// 1..15, starts where thread r starts, jumped by q 16^l unit samples; the
// grid strides over the level.  (XS256 takes k_tree_stride below.)
constexpr int kTreeWG = 1024;

template <class G>
__global__ __launch_bounds__(kTreeWG) void k_tree_level(uint32_t *__restrict__ ws, uint64_t T, uint32_t shift,
                                                        uint64_t unit, DevTables tab)
{
    const uint64_t lo = (uint64_t)1 << shift;
    const uint64_t hi = min(lo << 4, T);
    const uint64_t n = hi - lo;
    const uint64_t first = (uint64_t)blockIdx.x * kTreeWG + threadIdx.x, stride = (uint64_t)gridDim.x * kTreeWG;
    for (uint64_t i = first; i < n; i += stride) {
        const uint64_t t = lo + i, r = t & (lo - 1);
        G g;
        g.load(ws, T, r, tab);
        g.jump((t - r) * unit, tab);
        g.store(ws, T, t);
    }
}

// XS256 tree levels with a power-of-two unit u: the 15 threads r + q lo
// (lo = 2^shift, q = 1 .. 15) that start from thread r are split over four
// lanes by q mod 4.  Lane k starts thread r + (k + 1) lo with the products
// of M^(lo u 2^i) for the set bits i of k + 1, then each further thread,
// 4 lo on, with one product by M^(4 lo u): 16 products per r, at most 5 in a
// row.  (The bit tables alone take 32 products per r; one chain per r takes
// 15, all in a row, and a lone wave pays about 1.8 us for each.)  Tables
// M^(2^(b + i)), i < 3, in LDS (96 KiB); tb points at M^(2^b).
template <class G>
__device__ __forceinline__ void tree_stride4(G &g, uint32_t *__restrict__ ws, uint64_t T, uint64_t r, uint32_t k,
                                             uint32_t shift, uint64_t hi, const uint4 *tb)
{
    const uint64_t room = (hi - 1 - r) >> shift;  // largest q with r + q lo < hi
    uint32_t q = k + 1;
    if (q > room) return;
    if (q & 1) g.jump_table(tb);
    if (q & 2) g.jump_table(tb + 2048);
    if (q & 4) g.jump_table(tb + 4096);
    g.store(ws, T, r + ((uint64_t)q << shift));
    for (q += 4; q <= room; q += 4) {
        g.jump_table(tb + 4096);
        g.store(ws, T, r + ((uint64_t)q << shift));
    }
}

// First of the three tables M^(2^(b + i)) to stage: tables run to 2^63, and a
// table past it is never applied (a thread it would start lies beyond T).
__host__ __device__ constexpr uint32_t stride4_first_table(uint32_t b) { return b < 61 ? b : 61; }

// Tables of M^D, M^(2D), M^(4D) (XS256) for a jump D that is no power of
// two, built by the workgroup in LDS: lanes c < 256 carry column c of the
// identity through the global digit tables of M^(d 16^j) for the nonzero
// hexadecimal digits of D (each staged in t[1] first), which gives the
// columns of M^D; each table is then built from its columns (entry v of
// nibble p: the XOR of columns 4p + k over the set bits k of v), and the
// columns of M^(2D) and M^(4D) are those of the previous power times its own
// table.  t holds three tables of 2048 quads, cols 256 x 8 words.
__device__ __forceinline__ void xs256_cols_to_table(uint4 *t, const uint32_t *cols, uint32_t tid, uint32_t wg)
{
    for (uint32_t q = tid; q < 2048; q += wg) {
        const uint32_t p = q >> 5, h = (q >> 4) & 1, v = q & 15;
        uint32_t r[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if ((v >> k) & 1)
#pragma unroll
                for (int w = 0; w < 4; ++w) r[w] ^= cols[(4 * p + k) * 8 + 4 * h + w];
        t[q] = make_uint4(r[0], r[1], r[2], r[3]);
    }
}

template <int WG>
__device__ void xs256_power_tables(uint64_t D, uint4 *t, uint32_t *cols, const DevTables &tab)
{
    const uint32_t tid = threadIdx.x;
    const bool colt = tid < 256;  // lane c carries column c
    uint32_t col[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) col[i] = (uint32_t)(tid / 32 == (uint32_t)i) << (tid % 32);
    for (int j = 0; j < 16; ++j) {
        const uint32_t d = (uint32_t)(D >> (4 * j)) & 15u;  // uniform
        if (!d) continue;
        __syncthreads();  // the previous digit's table is read
        stage_quads<WG, 2048>(t + 2048, tab.xs256_t4w + ((size_t)j * 15 + (d - 1)) * 2048);
        __syncthreads();
        if (colt) gf2_apply256_t4(t + 2048, col);
    }
    for (int e = 0; e < 3; ++e) {
        if (e) {
            if (colt) gf2_apply256_t4(t + (e - 1) * 2048, col);  // columns of M^(2^e D)
        }
        __syncthreads();  // the digit table, or the previous table's build, is done with
        if (colt)
#pragma unroll
            for (int i = 0; i < 8; ++i) cols[tid * 8 + i] = col[i];
        __syncthreads();
        xs256_cols_to_table(t + e * 2048, cols, tid, WG);
        __syncthreads();
    }
}

// Workgroups of 256 lanes (64 values of r, one wave per k) for small
// levels, spread over many CUs; of 1024 lanes once the level fills every CU
// with them (16 waves sharing the tables and hiding each other's latency).
// b: the tables are M^(2^(b + i)) (a power-of-two unit), or with b = 64 the
// workgroup builds the tables of M^(lo unit 2^i) itself (xs256_power_tables,
// about 20 us, against some 7 global digit-table products for each thread
// of the level without them).
constexpr unsigned kStrideMaxBlocks = 2048;
constexpr uint32_t kStrideBuild = 64;

template <class G, int WG>
__global__ __launch_bounds__(WG) void k_tree_stride(uint32_t *__restrict__ ws, uint64_t T, uint32_t shift,
                                                   uint32_t b, uint64_t unit, DevTables tab)
{
    constexpr int RPB = WG / 4;  // values of r per workgroup
    __shared__ uint4 s_t[3 * 2048];
    __shared__ uint32_t s_col[256 * 8];
    const uint64_t lo = (uint64_t)1 << shift, hi = min(lo << 4, T);
    const uint4 *tb = s_t;
    if (b < kStrideBuild) {  // uniform
        const uint32_t b1 = stride4_first_table(b);
        stage_quads<WG, 3 * 2048>(s_t, tab.xs256_t4 + (size_t)b1 * 2048);
        __syncthreads();
        tb = s_t + (b - b1) * 2048;
    } else {
        xs256_power_tables<WG>(lo * unit, s_t, s_col, tab);
    }
    const uint64_t nr = min(lo, hi - lo);  // threads below lo with a successor
    const uint32_t k = (threadIdx.x >> 6) & 3, off = (threadIdx.x >> 8) * 64 + (threadIdx.x & 63);
    for (uint64_t r = (uint64_t)blockIdx.x * RPB + off; r < nr; r += (uint64_t)gridDim.x * RPB) {
        G g;
        g.load(ws, T, r, tab);
        tree_stride4(g, ws, T, r, k, shift, hi, tb);
    }
}

// The copy of the start state and the first three levels of that tree
// (threads 0 .. min(T, 4096) - 1) in one launch.  Every workgroup rebuilds
// threads 0 .. 255 in LDS (levels 0 and 1: 255 jumps), workgroup 0 also
// writes them out, and the workgroups share level 2, so no workgroup waits
// for another.  XS256 with a power-of-two unit stages the bit tables of
// levels 0 and 1 in LDS and runs level 2 by the four-lane scheme of
// k_tree_stride, 64 values of r per workgroup; other units give every
// level-2 thread a lane of its own.
constexpr uint32_t kTreeHeadThreads = 4096;  // threads the head kernel starts (levels 0 .. 2)
constexpr unsigned kTreeHeadBlocksXs256 = 4;  // workgroups of the four-lane level 2

template <class G>
constexpr int tree_head_wg()
{
    return G::kId == G_XS256 ? 256 : 1024;
}

template <class G>
__device__ __forceinline__ void tree_jump(G &g, uint32_t q, uint64_t k, const uint4 *t4, bool staged,
                                          const DevTables &tab)
{
    if constexpr (G::kId == G_XS256) {
        if (staged) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if ((q >> b) & 1) g.jump_table(t4 + b * 2048);
            return;
        }
    }
    g.jump(k, tab);
}

template <class G>
__global__ __launch_bounds__(tree_head_wg<G>()) void k_tree_head(const uint32_t *__restrict__ st0,
                                                                uint32_t *__restrict__ ws, uint64_t T,
                                                                uint64_t unit, DevTables tab)
{
    constexpr int WG = tree_head_wg<G>();
    __shared__ uint32_t s_st[G::W * 256];  // threads 0 .. 255, [word][thread]
    __shared__ uint4 s_t4[G::kId == G_XS256 ? 4 * 2048 : 1];
    const uint32_t tid = threadIdx.x;
    const uint64_t n = min<uint64_t>(T, kTreeHeadThreads);
    const uint32_t b0 = unit && (unit & (unit - 1)) == 0 ? (uint32_t)__builtin_ctzll(unit) : 64u;
    if (tid == 0) {
        G g;
        g.load(st0, 1, 0, tab);
        g.store(s_st, 256, 0);
        if (blockIdx.x == 0) g.store(ws, T, 0);
    }
    // levels 0 and 1: threads [1, 16) and [16, 256) into LDS
    for (uint32_t l = 0; l < 2; ++l) {
        const uint64_t lo = (uint64_t)1 << (4 * l);
        if (lo >= n) return;  // uniform
        const uint64_t hi = min<uint64_t>(lo << 4, n);
        const bool staged = G::kId == G_XS256 && b0 + 4 * l + 4 <= 64;
        __syncthreads();  // the previous level's states are in LDS, and its tables read
        if constexpr (G::kId == G_XS256) {
            if (staged) {
                stage_quads<WG, 4 * 2048>(s_t4, tab.xs256_t4 + (size_t)(b0 + 4 * l) * 2048);
                __syncthreads();
            }
        }
        const uint64_t t = lo + tid;
        if (t < hi) {
            const uint64_t r = t & (lo - 1);
            G g;
            g.load(s_st, 256, r, tab);
            tree_jump(g, (uint32_t)(t >> (4 * l)), (t - r) * unit, s_t4, staged, tab);
            g.store(s_st, 256, t);
            if (blockIdx.x == 0) g.store(ws, T, t);
        }
    }
    // level 2: threads [256, n) from the 256 in LDS
    if (n <= 256) return;  // uniform
    __syncthreads();
    if constexpr (G::kId == G_XS256) {
        if (b0 + 8 <= 63) {
            const uint32_t b1 = stride4_first_table(b0 + 8);
            stage_quads<WG, 3 * 2048>(s_t4, tab.xs256_t4 + (size_t)b1 * 2048);  // M^(256 u 2^i), i < 3
            __syncthreads();
            for (uint32_t r = blockIdx.x * 64 + (tid & 63); r < 256; r += gridDim.x * 64) {
                G g;
                g.load(s_st, 256, r, tab);
                tree_stride4(g, ws, T, r, tid >> 6, 8, n, s_t4 + (b0 + 8 - b1) * 2048);
            }
            return;
        }
    }
    for (uint64_t t = 256 + (uint64_t)blockIdx.x * WG + tid; t < n; t += (uint64_t)gridDim.x * WG) {
        const uint64_t r = t & 255;
        G g;
        g.load(s_st, 256, r, tab);
        g.jump((t - r) * unit, tab);
        g.store(ws, T, t);
    }
}

template <class G>
int launch_tree_head_t(const uint32_t *st0, uint32_t *ws, uint64_t T, uint64_t unit, const DevTables &tab,
                       hipStream_t stream)
{
    constexpr int WG = tree_head_wg<G>();
    const uint64_t n = T < kTreeHeadThreads ? T : kTreeHeadThreads;
    const bool stride4 = G::kId == G_XS256 && unit && (unit & (unit - 1)) == 0;  // level 2 on four workgroups
    unsigned blocks = 1;
    if (n > 256) blocks = stride4 ? kTreeHeadBlocksXs256 : (unsigned)((n - 256 + WG - 1) / WG);
    hipLaunchKernelGGL(k_tree_head<G>, dim3(blocks), dim3(WG), 0, stream, st0, ws, T, unit, tab);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define RNGX_INSTANTIATE_TREE_HEAD(G)                                                                   \
    template int launch_tree_head_t<G>(const uint32_t *, uint32_t *, uint64_t, uint64_t, const DevTables &, \
                                       hipStream_t);

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
    const uint64_t lo = (uint64_t)1 << shift, hi = (lo << 4) < T ? (lo << 4) : T;
    if constexpr (G::kId == G_XS256) {
        if (unit && hi > lo) {  // (lo * unit < 2^64: the caller checked T * unit)
            const uint64_t nr = hi - lo < lo ? hi - lo : lo;
            const uint32_t b =
                (unit & (unit - 1)) == 0 ? (uint32_t)__builtin_ctzll(unit) + shift : kStrideBuild;
            if (nr >= 256 * 256) {
                const uint64_t want = (nr + 255) / 256;
                const unsigned blocks = want < kStrideMaxBlocks ? (unsigned)want : kStrideMaxBlocks;
                hipLaunchKernelGGL((k_tree_stride<G, 1024>), dim3(blocks), dim3(1024), 0, stream, ws, T, shift, b, unit,
                                   tab);
            } else {
                hipLaunchKernelGGL((k_tree_stride<G, 256>), dim3((unsigned)((nr + 63) / 64)), dim3(256), 0, stream, ws,
                                   T, shift, b, unit, tab);
            }
            return hipGetLastError() == hipSuccess ? 0 : -1;
        }
    }
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
