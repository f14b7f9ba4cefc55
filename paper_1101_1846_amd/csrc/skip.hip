// skip.hip -- jump-ahead of many states by one distance k (Sec. II.A.4: the
// MWC congruence z <- a^k z mod m that follows from eqs. (2)-(3), the k-th power of the GF(2)
// step matrix of eqs. (5) and (6), and the affine LCG map).  Every state moves
// by the same k, so the k-step map is built once -- on the host for the
// constants that do not depend on the state, once per workgroup in LDS for
// the rest -- and each state then pays a single application:
//   MWC32    one fold-domain multiply by a^k                (host constant)
//   MWC16    one multiply per word by a_i^k of its multiplier (392 constants, LDS)
//   XS32     M^k y by four byte lookups                     (host columns, LDS tables)
//   XS256    M^k v by 64 nibble lookups                     (LDS table of M^k)
//   LCG      X <- A_k X + C_k                               (host constants)
// The XS256 table is built per workgroup: thread c carries column c of the
// identity through the staged table of M^(d 16^j) for every nonzero
// hexadecimal digit d at position j of k, and the 256 columns then give the
// nibble table of M^k.  That costs a few us per nonzero digit of k whatever
// the number of states, so below kXs256TableMin states every state jumps on
// its own (one product per nonzero digit, from the global tables), which is
// as fast there and has a lower latency floor.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_math.hpp"
#include "rng.h"
#include "rng_abi_internal.hpp"

namespace rngx {

namespace {

constexpr int kSkipWG = 256;
// XS256 workgroups take 1024 lanes: the first 256 carry one column of M^k
// each while the table is built, then all of them apply it (16 waves per CU
// share the LDS reads; with four, each wave's products ran one after the
// other and the launch took 0.10 ms for 2^20 states).  Splitting each
// column's products over the four lanes of a quad (nibbles 4m + s on lane s,
// partial sums combined by DPP) made it slower, 84 against 70 us: the four
// lanes read four table rows at once, whose entries share LDS banks.
constexpr int kSkipXs256WG = 1024;
template <class G>
constexpr int skip_wg()
{
    return G::kId == G_XS256 ? kSkipXs256WG : kSkipWG;
}
constexpr uint64_t kXs256TableMin = (uint64_t)1 << 16;

struct SkipArgs {
    uint32_t *st;           // [W][ld]
    uint64_t ld, S, k;
    uint64_t mwc32_f;       // a^k * 2^64 mod m (fold domain)
    uint32_t lcg_a, lcg_c;  // k steps of the LCG
    uint32_t xs32[32];      // columns of M^k, xorshift32
    DevTables tab;
};

__device__ __forceinline__ uint32_t xs32_by_bytes(const uint32_t *t8, uint32_t y)
{
    return xor3(t8[y & 255], t8[256 + ((y >> 8) & 255)], t8[512 + ((y >> 16) & 255)]) ^ t8[768 + (y >> 24)];
}

__device__ __forceinline__ uint32_t lds_t392_index(const uint16_t *t, uint32_t a)
{
    uint32_t lo = 0, hi = kMwc16Count;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (t[mid] <= a) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <class G>
__global__ __launch_bounds__(skip_wg<G>()) void k_skip_by(SkipArgs a)
{
    constexpr int WG = skip_wg<G>();
    constexpr bool kMwc16 = G::kId == G_MWC1616 || G::kId == G_KISS;
    constexpr bool kXs32 = G::kId == G_XS32 || G::kId == G_KISS;
    constexpr bool kXs256 = G::kId == G_XS256;
    __shared__ uint16_t s_t392[kMwc16 ? kMwc16Count : 1];
    __shared__ uint32_t s_c16[kMwc16 ? kMwc16Count : 1];  // a_i^k * 2^48 mod m_i
    __shared__ uint32_t s_t8[kXs32 ? 1024 : 1];           // byte tables of the xorshift32 M^k
    __shared__ uint4 s_t4[kXs256 ? 2 * 2048 : 1];          // staged M^(2^b) (two buffers), then M^k
    __shared__ uint32_t s_col[kXs256 ? 256 * 8 : 1];       // columns of M^k
    const uint32_t tid = threadIdx.x;
    if constexpr (kMwc16) {
        for (uint32_t i = tid; i < (uint32_t)kMwc16Count; i += WG) {
            const uint32_t ai = a.tab.t392[i];
            const uint32_t *p = a.tab.mwc16_pow + (size_t)i * 64;
            uint32_t c = (uint32_t)(((uint64_t)1 << 48) % (ai * 65536u - 1u));  // fold image of 1
            for (int b = 0; b < 64 && (a.k >> b); ++b)
                if ((a.k >> b) & 1) c = mwc16_mulmod(c, p[b], ai);
            s_t392[i] = (uint16_t)ai;
            s_c16[i] = c;
        }
    }
    if constexpr (kXs32) {
        // entry p * 256 + v: XOR of columns 8p + j over the set bits j of v
        for (uint32_t e = tid; e < 1024; e += WG) {
            const uint32_t p = e >> 8, v = e & 255;
            uint32_t r = 0;
            for (int j = 0; j < 8; ++j)
                if ((v >> j) & 1) r ^= a.xs32[8 * p + j];
            s_t8[e] = r;
        }
    }
    if constexpr (kXs256) {
        const bool colt = tid < 256;  // thread c < 256 carries column c
        uint32_t col[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = (uint32_t)(tid / 32 == (uint32_t)i) << (tid % 32);
        // Nonzero hexadecimal digits of k in increasing position (uniform: k
        // is the same for every thread).  The table of the next one is loaded
        // into registers while the current one is applied; buffer b & 1 is
        // rewritten only after the barrier that follows the previous write,
        // which every thread reaches after applying what that buffer held.
        constexpr int Q = 2048 / WG;
        uint32_t rest = 0;  // non-zero: the host returns before launching for k = 0
        for (int j = 0; j < 16; ++j)
            if ((a.k >> (4 * j)) & 15) rest |= 1u << j;
        auto table = [&](int j) {
            return a.tab.xs256_t4w + ((size_t)j * 15 + (((a.k >> (4 * j)) & 15) - 1)) * 2048;
        };
        uint4 pre[Q];
        const uint4 *src = table(__builtin_ctz(rest));
#pragma unroll
        for (int i = 0; i < Q; ++i) pre[i] = src[tid + i * WG];
        for (uint32_t buf = 0;; buf ^= 1) {
            uint4 *t = s_t4 + buf * 2048;
#pragma unroll
            for (int i = 0; i < Q; ++i) t[tid + i * WG] = pre[i];
            __syncthreads();
            rest &= rest - 1;
            if (rest) {
                src = table(__builtin_ctz(rest));
#pragma unroll
                for (int i = 0; i < Q; ++i) pre[i] = src[tid + i * WG];
            }
            if (colt) gf2_apply256_t4(t, col);
            if (!rest) break;
        }
        if (colt)
#pragma unroll
            for (int i = 0; i < 8; ++i) s_col[tid * 8 + i] = col[i];
        __syncthreads();
        // quad q = (2p + h) * 16 + v: words 4h .. 4h+3 of the XOR of columns 4p + j over the set bits j of v
        for (uint32_t q = tid; q < 2048; q += WG) {
            const uint32_t p = q >> 5, h = (q >> 4) & 1, v = q & 15;
            uint32_t r[4] = {0, 0, 0, 0};
            for (int j = 0; j < 4; ++j)
                if ((v >> j) & 1)
                    for (int w = 0; w < 4; ++w) r[w] ^= s_col[(4 * p + j) * 8 + 4 * h + w];
            s_t4[q] = make_uint4(r[0], r[1], r[2], r[3]);
        }
    }
    if constexpr (kMwc16 || kXs32 || kXs256) __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * WG;
    for (uint64_t s = (uint64_t)blockIdx.x * WG + tid; s < a.S; s += stride) {
        G g;
        g.load(a.st, a.ld, s, a.tab);
        if constexpr (G::kId == G_MWC32) {
            const uint64_t z = mwc32_mulmod((uint64_t)g.c << 32 | g.x, a.mwc32_f, a.tab.mwc32_a, a.tab.mwc32_m);
            g.x = (uint32_t)z;
            g.c = (uint32_t)(z >> 32);
        } else if constexpr (kXs256) {
            gf2_apply256_t4(s_t4, g.v);
        } else if constexpr (G::kId == G_XS32) {
            g.y = xs32_by_bytes(s_t8, g.y);
        } else {  // MWC1616, KISS
            g.z = mwc16_mulmod(g.z, s_c16[lds_t392_index(s_t392, g.a1)], g.a1);
            g.w = mwc16_mulmod(g.w, s_c16[lds_t392_index(s_t392, g.a2)], g.a2);
            if constexpr (G::kId == G_KISS) {
                g.jsr = xs32_by_bytes(s_t8, g.jsr);
                g.jcong = a.lcg_a * g.jcong + a.lcg_c;
            }
        }
        g.store(a.st, a.ld, s);
    }
}

// Each state jumps by k on its own (the generator's own jump).
template <class G>
__global__ __launch_bounds__(kSkipWG) void k_skip_each(SkipArgs a)
{
    const uint64_t s = (uint64_t)blockIdx.x * kSkipWG + threadIdx.x;
    if (s >= a.S) return;
    G g;
    g.load(a.st, a.ld, s, a.tab);
    g.jump(a.k, a.tab);
    g.store(a.st, a.ld, s);
}

template <class G>
int launch_skip_by(const SkipArgs &a, hipStream_t stream)
{
    if (G::kId == G_XS256 && a.S < kXs256TableMin) {  // see the file comment
        hipLaunchKernelGGL(k_skip_each<G>, dim3((unsigned)((a.S + kSkipWG - 1) / kSkipWG)), dim3(kSkipWG), 0, stream,
                           a);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    // workgroups that build LDS tables stride over the states: one per CU
    // for XS256 (one staged table per nonzero hexadecimal digit of k), two
    // for MWC16
    constexpr int WG = skip_wg<G>();
    const uint64_t cap = G::kId == G_XS256 ? 256 : (G::kId == G_MWC1616 || G::kId == G_KISS) ? 512 : 4096;
    const uint64_t need = (a.S + WG - 1) / WG;
    const unsigned blocks = (unsigned)(need < cap ? need : cap);
    hipLaunchKernelGGL(k_skip_by<G>, dim3(blocks), dim3(WG), 0, stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int dispatch_skip(int g, uint32_t *st, uint64_t ld, uint64_t S, uint64_t k, const DevTables &tab, hipStream_t s)
{
    if (S == 0 || k == 0) return 0;
    SkipArgs a{};
    a.st = st;
    a.ld = ld;
    a.S = S;
    a.k = k;
    a.tab = tab;
    if (g == RNG_MWC32) a.mwc32_f = mwc32_fold_const(k);
    if (g == RNG_XS32 || g == RNG_KISS) xs32_lcg_jump(k, a.xs32, &a.lcg_a, &a.lcg_c);
    switch (g) {
    case RNG_MWC32: return launch_skip_by<GenMWC32>(a, s);
    case RNG_XS256: return launch_skip_by<GenXS256>(a, s);
    case RNG_XS32: return launch_skip_by<GenXS32>(a, s);
    case RNG_KISS: return launch_skip_by<GenKISS>(a, s);
    case RNG_MWC1616: return launch_skip_by<GenMWC1616>(a, s);
    }
    return -2;
}

}  // namespace rngx
