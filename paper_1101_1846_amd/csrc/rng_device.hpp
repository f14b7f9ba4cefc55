// rng_device.hpp -- the library's device view of the generators of
// Hissoiny, Despres & Ozell (arXiv:1101.1846).  Each Gen* struct is the
// public step type of include/rng_inline.hpp (state in VGPRs, load/store of
// the structure-of-arrays [W][S] layout, next() = step then emit, eq. (1))
// plus what the library's kernels also need:
//   load(state, S, s, tab)   as load(state, S, s)
//   jump(k, tab)             advance by k steps (device tables below)
//   seed(d, tab)             state from SplitMix64 draws d[]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng_inline.hpp"

namespace rngx {

// Device copies of the host tables (host_math.hpp), one set per device.
struct DevTables {
    const uint16_t *t392;          // [392] base-2^16 multipliers, ascending
    const uint64_t *mwc32_pow;     // [64] a^(2^b) * 2^64 mod m
    const uint32_t *lcg_pow;       // [64][2] (A, C) of 2^b LCG steps
    const uint32_t *xs32_pow;      // [64][32] columns of M^(2^b)
    const uint32_t *mwc16_pow;     // [392][64] a_i^(2^b) * 2^48 mod m_i
    const uint4 *xs256_t4;         // [64][64][2][16] 4-bit lookup tables of M^(2^b)
    const uint4 *xs256_t4w;        // [16][15][64][2][16] 4-bit lookup tables of M^(d 16^j), d = 1..15
    uint32_t mwc32_a;              // 65274
    uint64_t mwc32_m;              // a * 2^32 - 1
};

using rng_inline::detail::xor3;
using rng_inline::detail::mwc16_step;
using rng_inline::to_unit_f32;

// SplitMix64 output number n of a generator started at `seed`
// (Steele, Lea & Flood 2014): mix(seed + (n+1) * gamma).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------- MWC algebra
// For base b = 2^w and m = a*b - 1 we have a*b = 1 (mod m), so for any X,
// fold(X) = (X >> w) + a * (X mod b) is congruent to a*X.  A product z*A is
// reduced with a constant stored pre-multiplied by b^(-f) = a^f (f folds):
// a^f * (z * A * b^f) = z*A (mod m).  The bounds below keep every fold exact.

// m = a*2^32 - 1 < 2^48; z in [1, m-1]; Af = A * 2^64 mod m.  Two folds.
__device__ __forceinline__ uint64_t mwc32_mulmod(uint64_t z, uint64_t Af, uint32_t a, uint64_t m)
{
    uint32_t zl = (uint32_t)z, zh = (uint32_t)(z >> 32);
    uint32_t fl = (uint32_t)Af, fh = (uint32_t)(Af >> 32);
    uint64_t t0 = (uint64_t)zl * fl;
    // P = z*Af < m^2 < 0.993 * 2^96; P_hi = P >> 32 < 0.993 * 2^64
    uint64_t phi = (t0 >> 32) + (uint64_t)zl * fh + (uint64_t)zh * fl + ((uint64_t)(zh * fh) << 32);
    uint64_t y1 = phi + (uint64_t)a * (uint32_t)t0;         // < 2^64
    uint64_t y2 = (y1 >> 32) + (uint64_t)a * (uint32_t)y1;  // < m + 2^32 < 2m
    return y2 >= m ? y2 - m : y2;
}

// m = a*2^16 - 1 < 2^32; z in [1, m-1]; Af = A * 2^48 mod m.  Three folds.
__device__ __forceinline__ uint32_t mwc16_mulmod(uint32_t z, uint32_t Af, uint32_t a)
{
    uint32_t m = a * 65536u - 1u;
    uint64_t p = (uint64_t)z * Af;                               // < 2^64
    uint64_t y1 = (p >> 16) + (uint64_t)a * (uint32_t)(p & 0xFFFFu);   // < 2^48 + 2^32
    uint64_t y2 = (y1 >> 16) + (uint64_t)a * (uint32_t)(y1 & 0xFFFFu); // < 2^32 + 2^16 (a+1)
    uint32_t y3 = (uint32_t)(y2 >> 16) + a * (uint32_t)(y2 & 0xFFFFu);  // < m + 2^16 + 3 < 2m
    return y3 >= m ? y3 - m : y3;
}

// Index of multiplier a in the ascending table (binary search).
__device__ __forceinline__ uint32_t t392_index(const uint16_t *t, uint32_t a)
{
    uint32_t lo = 0, hi = 392;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (t[mid] <= a) lo = mid; else hi = mid;
    }
    return lo;
}

// MWC16 word from 16+16 seed bits with c < a and z outside {0, a*2^16 - 1}.
__device__ __forceinline__ uint32_t mwc16_seed_word(uint32_t h, uint32_t a)
{
    uint32_t z = ((h >> 16) % a) << 16 | (h & 0xFFFFu);
    uint32_t m = a * 65536u - 1u;
    z = z == 0 ? 1u : z;
    return z == m ? m - 1u : z;
}

__device__ __forceinline__ void mwc16_pair(uint64_t d, const uint16_t *t, uint32_t &a1, uint32_t &a2)
{
    uint32_t i = (uint32_t)d % 392u;
    uint32_t j = (i + 1u + (uint32_t)(d >> 32) % 391u) % 392u;
    a1 = t[i];
    a2 = t[j];
}

// ---------------------------------------------------------------- GF(2)
// y <- M y for a 32x32 bit matrix given by its 32 columns.
__device__ __forceinline__ uint32_t gf2_apply32(const uint32_t *__restrict__ col, uint32_t y)
{
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        uint32_t mask = (uint32_t)__builtin_amdgcn_sbfe((int)y, b, 1);
        r ^= col[b] & mask;
    }
    return r;
}

// x <- M x for a 256x256 GF(2) matrix M given by its 4-bit lookup table T
// (2048 quads, 32 KiB): quads (2p + h) * 16 + v hold words 4h .. 4h+3 of the
// XOR of columns 4p + k over the set bits k of v.  The product is the XOR of
// the two quads selected by each of the 64 nibbles of x: 128 independent
// 16-byte lookups instead of 256 masked column XORs.  T may sit in LDS (a
// staged table) or in global memory; inlined, the loads take that space.
__device__ __forceinline__ void gf2_apply256_t4(const uint4 *T, uint32_t (&x)[8])
{
    uint32_t r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < 64; p += 2) {
        const uint32_t n0 = (x[p >> 3] >> (4 * (p & 7))) & 15u;
        const uint32_t n1 = (x[p >> 3] >> (4 * (p & 7) + 4)) & 15u;
        const uint4 a0 = T[(2 * p) * 16 + n0], a1 = T[(2 * p + 1) * 16 + n0];
        const uint4 b0 = T[(2 * p + 2) * 16 + n1], b1 = T[(2 * p + 3) * 16 + n1];
        r[0] = xor3(r[0], a0.x, b0.x);
        r[1] = xor3(r[1], a0.y, b0.y);
        r[2] = xor3(r[2], a0.z, b0.z);
        r[3] = xor3(r[3], a0.w, b0.w);
        r[4] = xor3(r[4], a1.x, b1.x);
        r[5] = xor3(r[5], a1.y, b1.y);
        r[6] = xor3(r[6], a1.z, b1.z);
        r[7] = xor3(r[7], a1.w, b1.w);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = r[i];
}

// Copies NQ consecutive 16-byte quads (whole lookup tables of 2048 quads,
// 32 KiB) into LDS with a workgroup of WG lanes, every global load issued
// before the first LDS write: one memory round trip, where a loop strided by
// the runtime workgroup size waits for each quad in turn.  The caller
// synchronises before use.
template <int WG, int NQ>
__device__ __forceinline__ void stage_quads(uint4 *lds, const uint4 *T)
{
    static_assert(NQ % WG == 0, "whole rows of the workgroup");
    constexpr int PER = NQ / WG;
    uint4 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) v[i] = T[i * WG + threadIdx.x];
#pragma unroll
    for (int i = 0; i < PER; ++i) lds[i * WG + threadIdx.x] = v[i];
}

// ---------------------------------------------------------------- generators
enum { G_MWC32 = 1, G_XS256 = 2, G_XS32 = 3, G_KISS = 4, G_MWC1616 = 5 };

// Eq. (2)-(3), b = 2^32 (rng_inline::MWC32).
struct GenMWC32 : rng_inline::MWC32 {
    static constexpr int kId = G_MWC32, W = 2, D = 1;
    using rng_inline::MWC32::load;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s, const DevTables &)
    {
        load(st, S, s);
    }
    __device__ void jump(uint64_t k, const DevTables &tab)
    {
        uint64_t z = (uint64_t)c << 32 | x;
        for (int b = 0; b < 64 && (k >> b); ++b)
            if ((k >> b) & 1) z = mwc32_mulmod(z, tab.mwc32_pow[b], tab.mwc32_a, tab.mwc32_m);
        x = (uint32_t)z;
        c = (uint32_t)(z >> 32);
    }
    __device__ void seed(const uint64_t *d, const DevTables &tab)
    {
        uint64_t z = (uint64_t)((uint32_t)(d[0] >> 32) % tab.mwc32_a) << 32 | (uint32_t)d[0];
        z = z == 0 ? 1 : z;
        z = z == tab.mwc32_m ? tab.mwc32_m - 1 : z;
        x = (uint32_t)z;
        c = (uint32_t)(z >> 32);
    }
};

// Eq. (5), r = 8 (rng_inline::XS256): window v[0..7] = (v_{n-8} .. v_{n-1}).
// 14 VALU operations per number on gfx950 (7 shifts, 2 two-input and 5
// three-input xors) against the paper's 18 two-input operations.
struct GenXS256 : rng_inline::XS256 {
    static constexpr int kId = G_XS256, W = 8, D = 4;
    using rng_inline::XS256::load;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s, const DevTables &)
    {
        load(st, S, s);
    }
    // M^k v as one product per nonzero hexadecimal digit d_j of k, by the
    // table of M^(d_j 16^j) (the powers commute, so the order is free).
    __device__ void jump(uint64_t k, const DevTables &tab)
    {
        for (int j = 0; j < 16 && (k >> (4 * j)); ++j) {
            const uint32_t d = (uint32_t)(k >> (4 * j)) & 15u;
            if (d) gf2_apply256_t4(tab.xs256_t4w + ((size_t)j * 15 + (d - 1)) * 2048, v);
        }
    }
    // One jump by the power of two whose lookup table T holds (staged in LDS).
    __device__ __forceinline__ void jump_table(const uint4 *T) { gf2_apply256_t4(T, v); }
    __device__ void seed(const uint64_t *d, const DevTables &)
    {
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = (uint32_t)d[i];
            v[2 * i + 1] = (uint32_t)(d[i] >> 32);
            any |= v[2 * i] | v[2 * i + 1];
        }
        if (!any) v[7] = 1;
    }
};

// Eq. (6) (rng_inline::XS32).
struct GenXS32 : rng_inline::XS32 {
    static constexpr int kId = G_XS32, W = 1, D = 1;
    using rng_inline::XS32::load;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s, const DevTables &)
    {
        load(st, S, s);
    }
    __device__ void jump(uint64_t k, const DevTables &tab)
    {
        for (int b = 0; b < 64 && (k >> b); ++b)
            if ((k >> b) & 1) y = gf2_apply32(tab.xs32_pow + b * 32, y);
    }
    __device__ void seed(const uint64_t *d, const DevTables &)
    {
        y = (uint32_t)d[0];
        y = y ? y : 1u;
    }
};


// Sec. III.A.1: two base-2^16 MWC words (rng_inline::MWC1616).
struct GenMWC1616 : rng_inline::MWC1616 {
    static constexpr int kId = G_MWC1616, W = 4, D = 2;
    using rng_inline::MWC1616::load;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s, const DevTables &)
    {
        load(st, S, s);
    }
    __device__ void jump(uint64_t k, const DevTables &tab)
    {
        const uint32_t *p1 = tab.mwc16_pow + t392_index(tab.t392, a1) * 64;
        const uint32_t *p2 = tab.mwc16_pow + t392_index(tab.t392, a2) * 64;
        for (int b = 0; b < 64 && (k >> b); ++b)
            if ((k >> b) & 1) {
                z = mwc16_mulmod(z, p1[b], a1);
                w = mwc16_mulmod(w, p2[b], a2);
            }
    }
    __device__ void seed(const uint64_t *d, const DevTables &tab)
    {
        mwc16_pair(d[0], tab.t392, a1, a2);
        z = mwc16_seed_word((uint32_t)d[1], a1);
        w = mwc16_seed_word((uint32_t)(d[1] >> 32), a2);
    }
};

// Sec. II.A.3 / III.A.3: KISS = (MWC1616 xor LCG) + XS32, LCG of eq. (7).
struct GenKISS : rng_inline::KISS {
    static constexpr int kId = G_KISS, W = 6, D = 3;
    using rng_inline::KISS::load;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s, const DevTables &)
    {
        load(st, S, s);
    }
    __device__ void jump(uint64_t k, const DevTables &tab)
    {
        const uint32_t *p1 = tab.mwc16_pow + t392_index(tab.t392, a1) * 64;
        const uint32_t *p2 = tab.mwc16_pow + t392_index(tab.t392, a2) * 64;
        for (int b = 0; b < 64 && (k >> b); ++b)
            if ((k >> b) & 1) {
                z = mwc16_mulmod(z, p1[b], a1);
                w = mwc16_mulmod(w, p2[b], a2);
                jsr = gf2_apply32(tab.xs32_pow + b * 32, jsr);
                jcong = tab.lcg_pow[2 * b] * jcong + tab.lcg_pow[2 * b + 1];
            }
    }
    __device__ void seed(const uint64_t *d, const DevTables &tab)
    {
        mwc16_pair(d[0], tab.t392, a1, a2);
        z = mwc16_seed_word((uint32_t)d[1], a1);
        w = mwc16_seed_word((uint32_t)(d[1] >> 32), a2);
        jsr = (uint32_t)d[2];
        jsr = jsr ? jsr : 1u;
        jcong = (uint32_t)(d[2] >> 32);
    }
};

}  // namespace rngx
