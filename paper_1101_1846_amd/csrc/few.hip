// few.hip -- bulk generation for fewer streams than a wave has lanes.  One
// wave per (64-stream group, chunk) would leave 64 - S lanes idle; here lane
// v of the grid takes chunk j = v mod P of stream s = v / P instead (chunks of
// C samples, the last one of each stream shorter), starting from the stream's
// state jumped by j C (Sec. II.A.4).  Each lane writes its chunk as one row of
// the wave's LDS tile, and the tile goes out row by row through per-row
// destination pointers, consecutive lanes on consecutive 16-byte quads.  No
// chunk writes the state back (the others read it at unordered times): the
// host advances the states by N with a skip launch afterwards.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_abi_internal.hpp"

namespace rngx {

namespace {

constexpr int kLaneWG = 256;
constexpr int kLaneTile = 64;  // samples per LDS tile row

struct LaneArgs {
    const uint32_t *state;  // [W][ld]
    uint64_t ld, S, N, C;
    uint64_t P;             // chunks per stream
    uint32_t *out;          // [S][N]
    DevTables tab;
};

// Global-memory views of the output (generic pointers would compile to FLAT,
// which also counts against LDS traffic).
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;

template <int DT>
__device__ __forceinline__ uint32_t lane_bits(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

template <class G, int DT, int U>
__global__ __launch_bounds__(kLaneWG) void k_generate_lanes(LaneArgs a)
{
    constexpr int K = kLaneTile, LD = K + 4, NW = kLaneWG / 64;
    __shared__ __attribute__((aligned(16))) uint32_t s_tile[NW * 64 * LD];
    __shared__ uint32_t *s_ptr[NW][64];
    __shared__ uint32_t s_len[NW][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t total = a.S * a.P, v0 = (uint64_t)blockIdx.x * kLaneWG + (uint64_t)wv * 64;
    if (v0 >= total) return;  // whole waves only
    const uint64_t v = v0 + lane;
    const bool active = v < total;
    const uint64_t s = active ? v / a.P : 0, j = active ? v - s * a.P : 0;
    const uint64_t start = j * a.C;
    const uint32_t len = active ? (uint32_t)min<uint64_t>(a.C, a.N - start) : 0;
    uint32_t *dst = a.out + s * a.N + start;

    G g;
    g.load(a.state, a.ld, s, a.tab);
    if (start) g.jump(start, a.tab);  // per-lane distance

    uint32_t **row_ptr = s_ptr[wv];
    uint32_t *row_len = s_len[wv];
    uint32_t *tile = s_tile + wv * 64 * LD;
    row_ptr[lane] = dst;
    row_len[lane] = len;
    uint32_t maxlen = len;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlen = max(maxlen, (uint32_t)__shfl_xor((int)maxlen, off, 64));
    const bool aligned = __all(((uintptr_t)dst & 15) == 0);
    uint32_t *row = tile + lane * LD;

    for (uint32_t k0 = 0; k0 < maxlen; k0 += K) {
        if (k0 + K <= len) {
#pragma unroll 1
            for (int k = 0; k < K; k += U) {
                uint32_t w[U];
#pragma unroll
                for (int u = 0; u < U; ++u) w[u] = lane_bits<DT>(g.next());
                if constexpr (U % 4 == 0) {
#pragma unroll
                    for (int u = 0; u < U; u += 4) *(uint4 *)&row[k + u] = make_uint4(w[u], w[u + 1], w[u + 2], w[u + 3]);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) row[k + u] = w[u];
                }
            }
        } else if (k0 < len) {
            for (uint32_t k = 0; k < len - k0; ++k) row[k] = lane_bits<DT>(g.next());
        }
        asm volatile("" ::: "memory");  // LDS writes before the transposed reads (one wavefront: in order)
        if (aligned) {
            constexpr int QPR = K / 4, RPI = 64 / QPR;
            const int rr = lane / QPR, qq = lane % QPR;
#pragma unroll 4
            for (int i = 0; i < QPR; ++i) {
                const int r = i * RPI + rr;
                const uint32_t col = k0 + 4 * qq, n = row_len[r];
                gu32 *p = (gu32 *)row_ptr[r] + col;
                const uint32_t *src = tile + r * LD + 4 * qq;
                if (col + 4 <= n) {
                    *(gu32x4 *)p = *(const u32x4 *)src;
                } else if (col < n) {
                    for (uint32_t e = 0; e < n - col; ++e) p[e] = src[e];
                }
            }
        } else {
            constexpr int RPI = 64 / K;
            const int rr = lane / K, cc = lane % K;
#pragma unroll 4
            for (int i = 0; i < K; ++i) {
                const int r = i * RPI + rr;
                const uint32_t col = k0 + cc;
                if (col < row_len[r]) ((gu32 *)row_ptr[r])[col] = tile[r * LD + cc];
            }
        }
        asm volatile("" ::: "memory");  // the tile is read before the next block overwrites it
    }
}

template <class G, int DT>
int launch_lanes(const LaneArgs &a, hipStream_t st)
{
    const uint64_t blocks = (a.S * a.P + kLaneWG - 1) / kLaneWG;
    hipLaunchKernelGGL((k_generate_lanes<G, DT, 8>), dim3((unsigned)blocks), dim3(kLaneWG), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class G>
int launch_lanes_t(int dt, const LaneArgs &a, hipStream_t st)
{
    return dt == RNG_DT_F32 ? launch_lanes<G, RNG_DT_F32>(a, st) : launch_lanes<G, RNG_DT_U32>(a, st);
}

}  // namespace

int generate_few(int g, int dt, uint32_t *d_state, uint64_t ld, uint64_t S, uint64_t N, uint64_t C, uint64_t P,
                 void *d_out, const DevTables &tab, hipStream_t st)
{
    LaneArgs a{};
    a.state = d_state;
    a.ld = ld;
    a.S = S;
    a.N = N;
    a.C = C;
    a.P = P;
    a.out = (uint32_t *)d_out;
    a.tab = tab;
    int rc = -2;
    switch (g) {
    case RNG_MWC32: rc = launch_lanes_t<GenMWC32>(dt, a, st); break;
    case RNG_XS256: rc = launch_lanes_t<GenXS256>(dt, a, st); break;
    case RNG_XS32: rc = launch_lanes_t<GenXS32>(dt, a, st); break;
    case RNG_KISS: rc = launch_lanes_t<GenKISS>(dt, a, st); break;
    case RNG_MWC1616: rc = launch_lanes_t<GenMWC1616>(dt, a, st); break;
    }
    if (rc) return rc;
    return dispatch_skip(g, d_state, ld, S, N, tab, st);  // the states advance by N after every chunk read them
}

}  // namespace rngx
