// rng_kernels.hpp -- kernel templates and their launchers.  Each generator's
// translation unit (gen_*.hip) includes this file and instantiates the
// launchers for its generator only, so the five units compile in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "rng_device.hpp"
#include "rng_internal.hpp"
#include "rng_aux_kernels.hpp"

namespace rngx {

// Compiler-only ordering point between the LDS writes of a tile and the LDS
// reads of the transposed store (and the next tile's writes).  A wavefront's
// LDS instructions execute in issue order, so no hardware wait is needed.
#define RNGX_COMPILER_FENCE() asm volatile("" ::: "memory")

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int DT>
__device__ __forceinline__ uint32_t out_bits(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

// ------------------------------------------------------------------ tile store
// Write a wave's LDS tile [64][K] (row stride K + 4 words) to rows s0.. of the
// stream-major output, columns k0 .. k0 + cnt.  Consecutive lanes take
// consecutive 16-byte quads (vec4) or words of one row, so every store
// instruction covers 64 / (K/4) rows x K words contiguous per row.  Full
// tiles read every LDS quad first and then issue every store, keeping all of
// them in flight; partial tiles take a predicated path.
template <int K>
__device__ __forceinline__ void store_tile(const uint32_t *tile, uint32_t *out, uint64_t s0, uint64_t N,
                                           uint64_t k0, uint32_t rows, uint32_t cnt, int lane, uint32_t vec4,
                                           uint32_t nt)
{
    constexpr int LD = K + 4;
    if (vec4) {
        constexpr int QPR = K / 4;       // quads per row
        constexpr int RPI = 64 / QPR;    // rows per store instruction
        const int r0 = lane / QPR, q = lane % QPR;
        const uint32_t *src = tile + r0 * LD + 4 * q;
        uint32_t *dst = out + (s0 + r0) * N + k0 + 4 * q;
        if (rows == 64 && cnt == K) {
            u32x4 v[QPR];
#pragma unroll
            for (int i = 0; i < QPR; ++i) v[i] = *(const u32x4 *)(src + i * RPI * LD);
#pragma unroll
            for (int i = 0; i < QPR; ++i) {
                u32x4 *d = (u32x4 *)(dst + (uint64_t)(i * RPI) * N);
                if (nt) __builtin_nontemporal_store(v[i], d);
                else *d = v[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < QPR; ++i) {
                if ((uint32_t)(r0 + i * RPI) < rows && (uint32_t)(4 * q) < cnt) {
                    u32x4 val = *(const u32x4 *)(src + i * RPI * LD);
                    *(u32x4 *)(dst + (uint64_t)(i * RPI) * N) = val;
                }
            }
        }
    } else {
        // word stores: each instruction covers RPI rows x W consecutive words
        constexpr int W = K < 64 ? K : 64, RPI = 64 / W, CPR = K / W;
        const int r0 = lane / W, c = lane % W;
        const uint32_t *src = tile + r0 * LD + c;
        uint32_t *dst = out + (s0 + r0) * N + k0 + c;
        const bool full = rows == 64 && cnt == K;
#pragma unroll 4
        for (int i = 0; i < 64 / RPI; ++i) {
#pragma unroll
            for (int j = 0; j < CPR; ++j) {
                const uint32_t r = r0 + i * RPI, col = j * W + c;
                if (full || (r < rows && col < cnt)) {
                    uint32_t *d = dst + (uint64_t)(i * RPI) * N + j * W;
                    const uint32_t v = src[i * RPI * LD + j * W];
                    if (nt) __builtin_nontemporal_store(v, d);
                    else *d = v;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ generate
// Lane mapping: wave w serves streams [64 sb, 64 sb + 64) for chunk j, with
// sb = w / P and j = w % P.  Chunk j covers samples [j C, min((j+1) C, N)) of
// each of its streams and starts from the stream state jumped by j C (the
// jump distance is uniform across the wave).  With one chunk per stream the
// kernel writes the state back.  With several, the last chunk may write it
// only once every chunk has read the start state: when one workgroup holds
// all of a group's chunks a barrier orders that; otherwise nothing does, the
// launcher reports it, and the host advances the states by N in a separate
// launch after this one.
//
// Store paths.  kMode 0: every lane stores its own row straight from
// registers.  kMode 1 and 2 stage through a wave-private LDS tile
// [64][K + 4]: each lane writes K consecutive samples of its own stream, and
// the wave then stores the tile row by row so that consecutive lanes write
// consecutive 16-byte quads of one stream (instead of 64 lanes each touching
// a different row).  kMode 1 issues the whole tile's stores at once after
// generating it; kMode 2 software-pipelines: the transposed quads of tile t
// are held in VGPRs and their stores are spread evenly through the
// generation of tile t + 1, so the write stream leaves the CU at a steady
// rate while the VALU keeps generating.
template <class G, int DT, int U>
__device__ __forceinline__ void gen_to_row(G &g, uint32_t *row, int k)
{
    uint32_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = out_bits<DT>(g.next());
    if constexpr (U % 4 == 0) {
#pragma unroll
        for (int u = 0; u < U; u += 4) *(uint4 *)&row[k + u] = make_uint4(v[u], v[u + 1], v[u + 2], v[u + 3]);
    } else if constexpr (U == 2) {
        *(uint2 *)&row[k] = make_uint2(v[0], v[1]);
    } else {
        row[k] = v[0];
    }
}

// Resident form of the pipelined schedule, for launches with one chunk per
// stream, whole 64-stream groups and N a multiple of K.  The grid holds the
// waves that fit on the device; wave w takes groups w, w + W, w + 2W, ... (at
// most MG).  It loads all their states first and waits for them
// once, before its first store, then only writes: the vector memory counter
// retires loads and stores in issue order, so any later wait for a load
// would also wait for every store still in flight.  The store pipeline runs
// across group boundaries, and the states move down a register queue.
template <class G, int DT, int U, int K, int MG>
__device__ __forceinline__ void gen_resident(const GenArgs &a, uint32_t *tile, int lane, uint64_t wave,
                                             uint64_t nwaves)
{
    constexpr int LD = K + 4, QPR = K / 4, RPI = 64 / QPR;
    const int r0 = lane / QPR, q = lane % QPR;
    const uint32_t *src = tile + r0 * LD + 4 * q;
    uint32_t *row = tile + lane * LD;
    const uint64_t N = a.N, groups = a.S / 64;
    if (wave >= groups) return;
    const uint32_t ng = (uint32_t)((groups - wave + nwaves - 1) / nwaves);
    const uint32_t T = (uint32_t)(N / K);
    uint32_t *out = (uint32_t *)a.out;
    G gs[MG];
#pragma unroll
    for (int i = 0; i < MG; ++i)
        if ((uint32_t)i < ng) gs[i].load(a.state, a.ld, (wave + (uint64_t)i * nwaves) * 64 + lane, a.tab);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every state is in before the first store
    G g = gs[0];
    uint64_t sb = wave;
    u32x4 P[QPR];
#pragma unroll
    for (int k = 0; k < K; k += U) gen_to_row<G, DT, U>(g, row, k);
    RNGX_COMPILER_FENCE();
#pragma unroll
    for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
    RNGX_COMPILER_FENCE();
    uint32_t *pdst = out + (sb * 64 + r0) * N + 4 * q;
    uint32_t t = 1;
    for (uint32_t gi = 0;;) {
        for (; t < T; ++t) {
#pragma unroll
            for (int k = 0; k < K; k += U) {
                gen_to_row<G, DT, U>(g, row, k);
#pragma unroll
                for (int i = k * QPR / K; i < (k + U) * QPR / K; ++i)
                    *(u32x4 *)(pdst + (uint64_t)(i * RPI) * N) = P[i];
                __builtin_amdgcn_sched_barrier(0);
            }
            RNGX_COMPILER_FENCE();
#pragma unroll
            for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
            RNGX_COMPILER_FENCE();
            pdst = out + (sb * 64 + r0) * N + (uint64_t)t * K + 4 * q;
        }
        g.store(a.state, a.ld, sb * 64 + lane);
        if (++gi == ng) break;
        sb += nwaves;
#pragma unroll
        for (int i = 0; i + 1 < MG; ++i) gs[i] = gs[i + 1];
        g = gs[0];
        t = 0;
    }
#pragma unroll
    for (int i = 0; i < QPR; ++i) *(u32x4 *)(pdst + (uint64_t)(i * RPI) * N) = P[i];
}

// Rows that are whole multiples of 4 KiB: with every wave at the same tile
// index, all concurrent writes share address bits 9-11 and the HBM write
// rate drops by a sixth.  Wave w therefore starts each of its rows at tile
// (w mod 4) T / 4: it jumps the state ahead by d N / 4 with d = w mod 4,
// writes to the end of the row, writes the state back, and wraps round to
// write the first tiles from the original state.  The jump is one product
// per word with constants that every stream of the launch shares: a^(d N/4)
// for MWC32, the columns of the xorshift32 M^(d N/4) and the LCG's A, C from
// the host; for the MWC16 words, whose multiplier varies by stream,
// a_i^(d N/4) for all 392 multipliers, built by each workgroup in LDS.
// XS256 (a 256 x 256 product per row) keeps the plain order.
struct RotMwc16 {
    const uint16_t *t392;  // LDS: the ascending multipliers
    const uint32_t *c16;   // LDS: [3][392], a_i^(d N / 4) * 2^48 mod m_i for d = 1..3
};

__device__ __forceinline__ uint32_t rot_xs32(const uint32_t *cols, uint32_t y)
{
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) r ^= cols[j] & (0u - ((y >> j) & 1u));
    return r;
}

template <class G>
__device__ __forceinline__ void rot_jump(G &g, const GenArgs &a, uint32_t d, const RotMwc16 &r)
{
    if constexpr (G::kId == G_MWC32) {
        const uint64_t z = mwc32_mulmod((uint64_t)g.c << 32 | g.x, a.rot_mwc32[d], a.tab.mwc32_a, a.tab.mwc32_m);
        g.x = (uint32_t)z;
        g.c = (uint32_t)(z >> 32);
    } else if constexpr (G::kId == G_XS32) {
        g.y = rot_xs32(a.rot_xs32[d], g.y);
    } else {  // MWC1616, KISS
        const uint32_t *c = r.c16 + (d - 1) * 392;
        g.z = mwc16_mulmod(g.z, c[t392_index(r.t392, g.a1)], g.a1);
        g.w = mwc16_mulmod(g.w, c[t392_index(r.t392, g.a2)], g.a2);
        if constexpr (G::kId == G_KISS) {
            g.jsr = rot_xs32(a.rot_xs32[d], g.jsr);
            g.jcong = a.rot_lcg[d][0] * g.jcong + a.rot_lcg[d][1];
        }
    }
}

template <class G, int DT, int U, int K, int MG>
__device__ __forceinline__ void gen_resident_rot(const GenArgs &a, uint32_t *tile, int lane, uint64_t wave,
                                                 uint64_t nwaves, const RotMwc16 &rt)
{
    constexpr int LD = K + 4, QPR = K / 4, RPI = 64 / QPR;
    const int r0 = lane / QPR, q = lane % QPR;
    const uint32_t *src = tile + r0 * LD + 4 * q;
    uint32_t *row = tile + lane * LD;
    const uint64_t N = a.N, groups = a.S / 64;
    if (wave >= groups) return;
    const uint32_t ng = (uint32_t)((groups - wave + nwaves - 1) / nwaves);
    const uint32_t T = (uint32_t)(N / K);
    const uint32_t d = (uint32_t)(wave & 3), t0 = d * (T / 4);  // first tile of every row of this wave
    uint32_t *out = (uint32_t *)a.out;
    G gs[MG];
#pragma unroll
    for (int i = 0; i < MG; ++i)
        if ((uint32_t)i < ng) gs[i].load(a.state, a.ld, (wave + (uint64_t)i * nwaves) * 64 + lane, a.tab);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every state is in before the first store
    G g0 = gs[0], g = g0;                // g0: the row's start, kept for the wrap
    if (d) rot_jump(g, a, d, rt);
    uint64_t sb = wave;
    u32x4 P[QPR];
#pragma unroll
    for (int k = 0; k < K; k += U) gen_to_row<G, DT, U>(g, row, k);
    RNGX_COMPILER_FENCE();
#pragma unroll
    for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
    RNGX_COMPILER_FENCE();
    uint32_t *pdst = out + (sb * 64 + r0) * N + (uint64_t)t0 * K + 4 * q;
    uint32_t n = 1;  // tiles of the current row done
    for (uint32_t gi = 0;;) {
        for (; n < T; ++n) {
            uint32_t t = t0 + n;
            if (t >= T) t -= T;
            if (t == 0 && n != 0) {  // wrapped: g holds the end-of-row state
                g.store(a.state, a.ld, sb * 64 + lane);
                g = g0;
            }
#pragma unroll
            for (int k = 0; k < K; k += U) {
                gen_to_row<G, DT, U>(g, row, k);
#pragma unroll
                for (int i = k * QPR / K; i < (k + U) * QPR / K; ++i)
                    *(u32x4 *)(pdst + (uint64_t)(i * RPI) * N) = P[i];
                __builtin_amdgcn_sched_barrier(0);
            }
            RNGX_COMPILER_FENCE();
#pragma unroll
            for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
            RNGX_COMPILER_FENCE();
            pdst = out + (sb * 64 + r0) * N + (uint64_t)t * K + 4 * q;
        }
        if (t0 == 0) g.store(a.state, a.ld, sb * 64 + lane);  // no wrap: g is the end-of-row state
        if (++gi == ng) break;
        sb += nwaves;
#pragma unroll
        for (int i = 0; i + 1 < MG; ++i) gs[i] = gs[i + 1];
        g0 = gs[0];
        g = g0;
        if (d) rot_jump(g, a, d, rt);
        n = 0;
    }
#pragma unroll
    for (int i = 0; i < QPR; ++i) *(u32x4 *)(pdst + (uint64_t)(i * RPI) * N) = P[i];
}

template <class G, int DT, int WG, int U>
__global__ __launch_bounds__(WG) void k_generate_rot(GenArgs a)
{
    constexpr int K = 128, LD = K + 4, NW = WG / 64;
    constexpr bool kMwc16 = G::kId == G_MWC1616 || G::kId == G_KISS;
    __shared__ __attribute__((aligned(16))) uint32_t lds[NW * 64 * LD];
    __shared__ uint16_t s_t392[kMwc16 ? 392 : 1];
    __shared__ uint32_t s_c16[kMwc16 ? 3 * 392 : 1];
    if constexpr (kMwc16) {
        // a_i^q, a_i^2q, a_i^3q (q = N / 4) in the fold domain of m_i: the
        // bits of q over the table of a_i^(2^b), then two products
        const uint64_t q = a.N / 4;
        for (uint32_t i = threadIdx.x; i < 392u; i += WG) {
            const uint32_t ai = a.tab.t392[i];
            const uint32_t *p = a.tab.mwc16_pow + (size_t)i * 64;
            uint32_t c = (uint32_t)(((uint64_t)1 << 48) % (ai * 65536u - 1u));  // fold image of 1
            for (int b = 0; b < 64 && (q >> b); ++b)
                if ((q >> b) & 1) c = mwc16_mulmod(c, p[b], ai);
            const uint32_t c2 = mwc16_mulmod(c, c, ai);
            s_t392[i] = (uint16_t)ai;
            s_c16[i] = c;
            s_c16[392 + i] = c2;
            s_c16[784 + i] = mwc16_mulmod(c2, c, ai);
        }
        __syncthreads();  // before any wave returns
    }
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * NW + wv;
    gen_resident_rot<G, DT, U, K, resident_groups(WG, K)>(a, &lds[wv * 64 * LD], lane, wave,
                                                          (uint64_t)gridDim.x * NW, RotMwc16{s_t392, s_c16});
}

// Rows of 4 or 8 KiB as 16 KiB runs.  In [S][N] the rows of consecutive
// streams are adjacent, so lane L of a group takes the seg streams seg L ..
// seg L + seg - 1 one after the other and writes their rows as one run of
// seg N samples: the wave's tiles then step through rows of 16 KiB, which
// write faster than rows of 4 or 8 KiB (measured), with no jump: the lane
// switches to the next stream's state every N / K tiles and writes back the
// one it finished.  The register queue holds the seg states of each of the
// wave's groups (at most MG / seg groups, checked by the launcher).
template <class G, int DT, int U, int K, int MG>
__device__ __forceinline__ void gen_resident_seg(const GenArgs &a, uint32_t *tile, int lane, uint64_t wave,
                                                 uint64_t nwaves)
{
    constexpr int LD = K + 4, QPR = K / 4, RPI = 64 / QPR;
    const int r0 = lane / QPR, q = lane % QPR;
    const uint32_t *src = tile + r0 * LD + 4 * q;
    uint32_t *row = tile + lane * LD;
    const uint32_t seg = a.seg;
    const uint64_t N = a.N, R = N * seg, groups = a.S / (64 * seg);
    if (wave >= groups) return;
    const uint32_t ng = (uint32_t)((groups - wave + nwaves - 1) / nwaves);
    const uint32_t TS = (uint32_t)(N / K), T = TS * seg;
    uint32_t *out = (uint32_t *)a.out;
    G gs[MG];
#pragma unroll
    for (int k = 0; k < MG; ++k) {
        const uint32_t j = (uint32_t)k / seg, i = (uint32_t)k - j * seg;
        if (j < ng) gs[k].load(a.state, a.ld, ((wave + (uint64_t)j * nwaves) * 64 + lane) * seg + i, a.tab);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every state is in before the first store
    G g = gs[0];
    uint64_t sb = wave;
    uint32_t si = 0, tn = TS;  // stream of the run being generated, and the tile that starts the next
    u32x4 P[QPR];
#pragma unroll
    for (int k = 0; k < K; k += U) gen_to_row<G, DT, U>(g, row, k);
    RNGX_COMPILER_FENCE();
#pragma unroll
    for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
    RNGX_COMPILER_FENCE();
    uint32_t *pdst = out + (sb * 64 + r0) * R + 4 * q;
    uint32_t t = 1;
    for (uint32_t gi = 0;;) {
        for (; t < T; ++t) {
            if (t == tn) {  // the next stream of the run
                g.store(a.state, a.ld, (sb * 64 + lane) * seg + si);
                ++si;
                tn += TS;
#pragma unroll
                for (int i = 0; i + 1 < MG; ++i) gs[i] = gs[i + 1];
                g = gs[0];
            }
#pragma unroll
            for (int k = 0; k < K; k += U) {
                gen_to_row<G, DT, U>(g, row, k);
#pragma unroll
                for (int i = k * QPR / K; i < (k + U) * QPR / K; ++i)
                    *(u32x4 *)(pdst + (uint64_t)(i * RPI) * R) = P[i];
                __builtin_amdgcn_sched_barrier(0);
            }
            RNGX_COMPILER_FENCE();
#pragma unroll
            for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
            RNGX_COMPILER_FENCE();
            pdst = out + (sb * 64 + r0) * R + (uint64_t)t * K + 4 * q;
        }
        g.store(a.state, a.ld, (sb * 64 + lane) * seg + si);
        if (++gi == ng) break;
        sb += nwaves;
#pragma unroll
        for (int i = 0; i + 1 < MG; ++i) gs[i] = gs[i + 1];
        g = gs[0];
        si = 0;
        tn = TS;
        t = 0;
    }
#pragma unroll
    for (int i = 0; i < QPR; ++i) *(u32x4 *)(pdst + (uint64_t)(i * RPI) * R) = P[i];
}

template <class G, int DT, int WG, int U>
__global__ __launch_bounds__(WG) void k_generate_seg(GenArgs a)
{
    constexpr int K = 128, LD = K + 4, NW = WG / 64;
    __shared__ __attribute__((aligned(16))) uint32_t lds[NW * 64 * LD];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * NW + wv;
    gen_resident_seg<G, DT, U, K, resident_groups(WG, K)>(a, &lds[wv * 64 * LD], lane, wave,
                                                          (uint64_t)gridDim.x * NW);
}

template <class G, int DT, int WG, int U, int K, int kMode>
__global__ __launch_bounds__(WG) void k_generate(GenArgs a)
{
    static_assert(K % U == 0 && K % 4 == 0, "tile depth");
    constexpr bool kStaged = kMode != 0;
    constexpr int LD = K + 4;
    constexpr int NW = WG / 64;
    __shared__ __attribute__((aligned(16))) uint32_t lds[kStaged ? NW * 64 * LD : 1];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * NW + wv;
    if constexpr (kMode == 2) {
        if (a.resident) {
            gen_resident<G, DT, U, K, resident_groups(WG, K)>(a, &lds[wv * 64 * LD], lane, wave,
                                                              (uint64_t)gridDim.x * NW);
            return;
        }
    }
    const uint64_t sb = wave / a.P, j = wave - sb * a.P;
    const uint64_t s0 = sb * 64;
    const uint64_t kb = j * a.C;
    // When the workgroup holds every chunk of its groups, a barrier after all
    // of them have read their start states lets the last chunk write back.
    const bool sync_wb = chunks_in_workgroup(a.P, NW);
    if (s0 >= a.S || kb >= a.N) {  // uniform per wave
        if (sync_wb) __syncthreads();
        return;
    }
    const uint64_t ke = min(kb + a.C, a.N);
    const uint32_t rows = (uint32_t)min<uint64_t>(64, a.S - s0);
    const bool valid = (uint32_t)lane < rows;
    const uint64_t s = valid ? s0 + lane : s0;

    G g;
    g.load(a.state, a.ld, s, a.tab);
    if (sync_wb) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's start state has arrived
        __syncthreads();
    }
    if (j) g.jump(kb, a.tab);

    uint32_t *tile = kStaged ? &lds[wv * 64 * LD] : nullptr;
    uint32_t *out = (uint32_t *)a.out;
    const uint64_t N = a.N;
    uint64_t k0 = kb;

    if constexpr (kMode == 2) {
        if (a.vec4 && rows == 64 && k0 + K <= ke) {
            constexpr int QPR = K / 4, RPI = 64 / QPR;
            const int r0 = lane / QPR, q = lane % QPR;
            const uint32_t *src = tile + r0 * LD + 4 * q;
            uint32_t *row = tile + lane * LD;
            u32x4 P[QPR];
            // first tile: generate only
#pragma unroll
            for (int k = 0; k < K; k += U) gen_to_row<G, DT, U>(g, row, k);
            RNGX_COMPILER_FENCE();
#pragma unroll
            for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
            RNGX_COMPILER_FENCE();
            uint32_t *pdst = out + (s0 + r0) * N + k0 + 4 * q;
            for (k0 += K; k0 + K <= ke; k0 += K) {
#pragma unroll
                for (int k = 0; k < K; k += U) {
                    gen_to_row<G, DT, U>(g, row, k);
#pragma unroll
                    for (int i = k * QPR / K; i < (k + U) * QPR / K; ++i)
                        *(u32x4 *)(pdst + (uint64_t)(i * RPI) * N) = P[i];
                    // keep each group of stores between its generation chunks
                    __builtin_amdgcn_sched_barrier(0);
                }
                RNGX_COMPILER_FENCE();
#pragma unroll
                for (int i = 0; i < QPR; ++i) P[i] = *(const u32x4 *)(src + i * RPI * LD);
                RNGX_COMPILER_FENCE();
                pdst += K;
            }
#pragma unroll
            for (int i = 0; i < QPR; ++i) *(u32x4 *)(pdst + (uint64_t)(i * RPI) * N) = P[i];
        }
    }

    for (; k0 < ke; k0 += K) {
        const uint32_t cnt = (uint32_t)min<uint64_t>(K, ke - k0);
        if constexpr (kStaged) {
            uint32_t *row = tile + lane * LD;
            if (cnt == K) {
#pragma unroll 1
                for (int k = 0; k < K; k += U) gen_to_row<G, DT, U>(g, row, k);
            } else {
                for (uint32_t k = 0; k < cnt; ++k) row[k] = out_bits<DT>(g.next());
            }
            RNGX_COMPILER_FENCE();
            store_tile<K>(tile, out, s0, N, k0, rows, cnt, lane, a.vec4, a.nt);
            RNGX_COMPILER_FENCE();
        } else {
            uint32_t *dst = out + s * N + k0;
            if (cnt == K) {
#pragma unroll 1
                for (int k = 0; k < K; k += U) {
                    uint32_t v[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) v[u] = out_bits<DT>(g.next());
                    if (valid) {
                        bool done = false;
                        if constexpr (U % 4 == 0) {
                            if (a.vec4) {
#pragma unroll
                                for (int u = 0; u < U; u += 4)
                                    *(uint4 *)&dst[k + u] = make_uint4(v[u], v[u + 1], v[u + 2], v[u + 3]);
                                done = true;
                            }
                        }
                        if (!done) {
#pragma unroll
                            for (int u = 0; u < U; ++u) dst[k + u] = v[u];
                        }
                    }
                }
            } else {
                for (uint32_t k = 0; k < cnt; ++k) {
                    uint32_t v = out_bits<DT>(g.next());
                    if (valid) dst[k] = v;
                }
            }
        }
    }
    if (valid && ke == a.N && (a.P == 1 || sync_wb)) g.store(a.state, a.ld, s);
}

// ------------------------------------------------------------------ fused pi
// 1 when i^2 + j^2 < 2^48 for 24-bit i, j (x^2 + y^2 < 1 for the exact FP32
// uniforms x = i 2^-24, y = j 2^-24): i^2 = hi 2^32 + lo with hi < 2^16, so
// the 48-bit sum is tested on its high word after the carry.
__device__ __forceinline__ uint32_t in_quarter_circle(uint32_t x, uint32_t y)
{
    const uint64_t px = (uint64_t)x * x, py = (uint64_t)y * y;  // 24 x 24 -> 48 bits
    const uint32_t xl = (uint32_t)px, xh = (uint32_t)(px >> 32);
    const uint32_t yl = (uint32_t)py, yh = (uint32_t)(py >> 32);
    const uint32_t lo = xl + yl;
    const uint32_t hi = xh + yh + (lo < xl);
    return hi < 65536u;
}

// Pairs (u_{2k}, u_{2k+1}) -> i = u >> 8, j = u >> 8; count i^2 + j^2 < 2^48
// with 24-bit multiplies: i^2 = hi * 2^32 + lo, hi < 2^16.  Chunk lengths are
// even so that pairs never straddle chunks.
template <class G, int WG, int U>
__global__ __launch_bounds__(WG) void k_fused_pi(FusedArgs a)
{
    static_assert(U % 2 == 0, "pairs");
    constexpr int NW = WG / 64;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * NW + wv;
    uint64_t s, kb, ke;
    bool valid;
    if (a.lanes) {
        // one chunk per lane: its own stream, start and (per-lane) jump
        const uint64_t total_chunks = a.S * a.P, v = wave * 64 + lane;
        if (wave * 64 >= total_chunks) return;  // whole waves
        valid = v < total_chunks;
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
        const uint32_t rows = (uint32_t)min<uint64_t>(64, a.S - s0);
        valid = (uint32_t)lane < rows;
        s = valid ? s0 + lane : s0;
    }

    G g;
    g.load(a.state, a.ld, s, a.tab);
    if (kb) g.jump(kb, a.tab);

    const uint64_t n = ke - kb;
    const uint64_t full = n / U;
    uint64_t total = 0;
    uint32_t cnt = 0;
    for (uint64_t it = 0; it < full; ++it) {
#pragma unroll
        for (int u = 0; u < U; u += 2) {
            const uint32_t x = g.next() >> 8, y = g.next() >> 8;
            cnt += in_quarter_circle(x, y);
        }
        if ((it & 0xFFFF) == 0xFFFF) { total += cnt; cnt = 0; }
    }
    for (uint64_t r = full * U; r + 1 < n; r += 2) {
        uint32_t x = g.next() >> 8, y = g.next() >> 8;
        uint64_t q = (uint64_t)x * x + (uint64_t)y * y;
        cnt += (q >> 48) == 0;
    }
    if (n & 1) g.next();
    total += cnt;
    if (!valid) total = 0;
    // wave reduction, one 64-bit atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
    if (lane == 0 && total) atomicAdd((unsigned long long *)a.count, (unsigned long long)total);
    if (valid && a.P == 1) g.store(a.state, a.ld, s);  // P > 1: the host skips the states by N
}

// ------------------------------------------------------------------ launchers
template <class G, int DT, int WG, int U, int kMode>
int launch_generate_shape(const GenArgs &a, hipStream_t stream)
{
    uint64_t waves = ((a.S + 63) / 64) * a.P;
    uint64_t blocks = (waves + WG / 64 - 1) / (WG / 64);
    // tile depth: kGenTile unless the workgroup's tiles would not fit in the
    // 160 KiB of LDS, then 32 (chunk lengths are multiples of kGenTile, so
    // of both depths)
    constexpr int K = gen_tile_depth(WG);
    GenArgs b = a;
    b.resident = 0;
    if constexpr (kMode == 2) {
        if (a.P == 1 && a.vec4 && a.S % 64 == 0 && a.N % K == 0) {
            // the workgroups resident at once on the current device (queried
            // once per device); each wave then takes at most
            // resident_groups(WG, K) groups
            static std::atomic<uint64_t> cache[kMaxDevices];
            uint64_t resident = 0;
            int dev = 0;
            if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) {
                resident = cache[dev].load(std::memory_order_relaxed);
                int per_cu = 0, cus = 0;
                if (!resident &&
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_generate<G, DT, WG, U, K, kMode>, WG, 0) ==
                        hipSuccess) {
                    resident = (uint64_t)per_cu * (uint64_t)cus;
                    cache[dev].store(resident, std::memory_order_relaxed);
                }
            }
            if (resident && blocks <= resident * resident_groups(WG, K)) {
                b.resident = 1;
                if (blocks > resident) blocks = resident;
            }
        }
    }
    bool launched = false;
    if constexpr (kMode == 2 && K == 128 &&
                  (G::kId == G_MWC32 || G::kId == G_XS32 || G::kId == G_KISS || G::kId == G_MWC1616 ||
                   G::kId == G_XS256)) {
        // runs of seg adjacent rows per lane.  S / 64 groups fit the resident
        // waves' queues (MG states each) exactly when S / (64 seg) runs fit
        // MG / seg per wave, so residency carries over; the grid is at most
        // the resident one, and smaller when the runs need fewer waves.
        if (b.resident && (a.seg == 2 || a.seg == 4) && a.S % (64 * (uint64_t)a.seg) == 0) {
            const uint64_t sw = a.S / (64 * (uint64_t)a.seg), sblocks = (sw + WG / 64 - 1) / (WG / 64);
            hipLaunchKernelGGL((k_generate_seg<G, DT, WG, U>), dim3((unsigned)min(sblocks, blocks)), dim3(WG), 0,
                               stream, b);
            launched = true;
        }
    }
    if constexpr (kMode == 2 && K == 128 &&
                  (G::kId == G_MWC32 || G::kId == G_XS32 || G::kId == G_KISS || G::kId == G_MWC1616)) {
        if (!launched && b.resident && a.rot) {
            hipLaunchKernelGGL((k_generate_rot<G, DT, WG, U>), dim3((unsigned)blocks), dim3(WG), 0, stream, b);
            launched = true;
        }
    }
    if (!launched)
        hipLaunchKernelGGL((k_generate<G, DT, WG, U, K, kMode>), dim3((unsigned)blocks), dim3(WG), 0, stream, b);
    if (hipGetLastError() != hipSuccess) return -1;
    return a.P > 1 && !chunks_in_workgroup(a.P, WG / 64) ? kStatesNotWritten : 0;
}

template <class G, int DT, int WG>
int launch_generate_u(const GenArgs &a, int unroll, bool staged, hipStream_t stream)
{
    if (!staged) return launch_generate_shape<G, DT, WG, 8, 0>(a, stream);
    switch (unroll) {
    case 1: return launch_generate_shape<G, DT, WG, 1, kStoreMode>(a, stream);
    case 2: return launch_generate_shape<G, DT, WG, 2, kStoreMode>(a, stream);
    case 4: return launch_generate_shape<G, DT, WG, 4, kStoreMode>(a, stream);
    case 8: return launch_generate_shape<G, DT, WG, 8, kStoreMode>(a, stream);
    case 16: return launch_generate_shape<G, DT, WG, 16, kStoreMode>(a, stream);
    }
    return -2;
}

template <class G, int DT>
int launch_generate_wg(const GenArgs &a, int wg, int unroll, bool staged, hipStream_t stream)
{
    switch (wg) {
    case 64: return launch_generate_u<G, DT, 64>(a, unroll, staged, stream);
    case 128: return launch_generate_u<G, DT, 128>(a, unroll, staged, stream);
    case 256: return launch_generate_u<G, DT, 256>(a, unroll, staged, stream);
    case 512: return launch_generate_u<G, DT, 512>(a, unroll, staged, stream);
    case 1024: return launch_generate_u<G, DT, 1024>(a, unroll, staged, stream);
    }
    return -2;
}

template <class G>
int launch_generate_t(int dt, const GenArgs &a, int wg, int unroll, bool staged, hipStream_t stream)
{
    return dt == RNG_DT_F32 ? launch_generate_wg<G, RNG_DT_F32>(a, wg, unroll, staged, stream)
                            : launch_generate_wg<G, RNG_DT_U32>(a, wg, unroll, staged, stream);
}

template <class G>
int launch_fused_pi_t(const FusedArgs &a, hipStream_t stream)
{
    constexpr int WG = 256;
    const uint64_t waves = a.lanes ? (a.S * a.P + 63) / 64 : ((a.S + 63) / 64) * a.P;
    const uint64_t blocks = (waves + WG / 64 - 1) / (WG / 64);
    hipLaunchKernelGGL((k_fused_pi<G, WG, 8>), dim3((unsigned)blocks), dim3(WG), 0, stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define RNGX_INSTANTIATE(G)                                                                            \
    template int launch_seed_t<G>(uint64_t, uint64_t, uint64_t, uint32_t *, const DevTables &,        \
                                  hipStream_t);                                                        \
    template int launch_tree_level_t<G>(uint32_t *, uint64_t, uint32_t, uint64_t, const DevTables &,  \
                                        hipStream_t);                                                  \
    template int launch_state_copy_t<G>(const uint32_t *, uint64_t, uint64_t, uint32_t *, uint64_t,  \
                                        uint64_t, hipStream_t);                                        \
    template int launch_generate_t<G>(int, const GenArgs &, int, int, bool, hipStream_t);             \
    template int launch_fused_pi_t<G>(const FusedArgs &, hipStream_t);

}  // namespace rngx
