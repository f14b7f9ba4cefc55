// rng_inline.hpp -- the generators of Hissoiny, Despres & Ozell
// (arXiv:1101.1846) as HIP device code, for drawing numbers inside another
// kernel "on the fly" (the use discussed in Sec. III.A.2 and III.B) instead
// of reading them from a buffer that rng_generate filled.
//
// State layout is the library's (include/rng.h): structure of arrays, word i
// of stream s at state[i * stride + s] with stride >= the number of streams,
// as rng_seed writes it.  A kernel loads one stream's state into registers
// with load(), calls next() as often as it needs, and writes the state back
// with store().  The numbers are exactly those rng_generate would have
// produced for that stream at that point, and a later rng_generate or
// rng_skip call on the same states continues after them.  The library's own
// kernels step the generators with these same functions.
//
//   type     kWords  state words (in order)           definition
//   MWC32    2       x, c                             eq. (2)-(3), b = 2^32, a = 65274
//   XS256    8       v_{n-8} ... v_{n-1}              eq. (5), r = 8
//   XS32     1       y                                eq. (6), shifts 13, 17, 5
//   MWC1616  4       z, w, a1, a2                     Sec. III.A.1: two base-2^16 MWC
//   KISS     6       z, w, jsr, jcong, a1, a2         Sec. III.A.3: (MWC1616 ^ LCG) + XS32, eq. (7)
//
// next() steps the recurrence once and returns the new 32-bit output (the
// step-then-emit convention of eq. (1)); last() returns the output of the
// most recent step again (every output is a function of the state the step
// left).  to_unit_f32(u) maps an output to the exact single-precision
// uniform (u >> 8) * 2^-24 in [0, 1).
//
// Header only, written for gfx950; it allocates nothing, launches nothing and
// holds no global state.  load() and store() must be called with the same
// stride the states were seeded with; two threads must not step the same
// stream concurrently (each would continue from the same point).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rng_inline {

namespace detail {
// a ^ b ^ c in one gfx950 v_bitop3 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One base-2^16 MWC word z = c * 2^16 + x: z <- a * (z & 0xFFFF) + (z >> 16)
// (eq. (2)-(3) with the mask and shift of Sec. II.A.1).  v_mad_u32_u16 reads
// only the low 16 bits of both factors, so the mask costs no instruction: a
// shift and one multiply-add per word (for the same expression in C the
// compiler emits an AND and a 24-bit multiply-add).
__device__ __forceinline__ uint32_t mwc16_step(uint32_t z, uint32_t a)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(z), "v"(z >> 16));
    return r;
}
}  // namespace detail

// The exact FP32 uniform: top 24 bits times 2^-24.
__device__ __forceinline__ float to_unit_f32(uint32_t u)
{
    return (float)(u >> 8) * 0x1p-24f;
}

// Eq. (2)-(3) with b = 2^32: t = a * x + c, x <- t mod 2^32, c <- t div 2^32.
struct MWC32 {
    static constexpr int kWords = 2;
    static constexpr uint32_t kA = 65274u;
    uint32_t x, c;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s)
    {
        x = st[s];
        c = st[S + s];
    }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t S, uint64_t s) const
    {
        st[s] = x;
        st[S + s] = c;
    }
    __device__ __forceinline__ uint32_t next()
    {
        const uint64_t t = (uint64_t)kA * x + c;
        x = (uint32_t)t;
        c = (uint32_t)(t >> 32);
        return x;
    }
    __device__ __forceinline__ uint32_t last() const { return x; }
};

// Eq. (5), r = 8: v_n = (I+L^9)(I+L^13) v_{n-1} + (I+L^7) v_{n-4}
//                     + (I+R^3) v_{n-5} + (I+R^10) v_{n-7} + (I+L^24)(I+R^7) v_{n-8}.
// The eight words are an explicit circular buffer shifted by one per step;
// in an unrolled loop the shifts are register renames.
struct XS256 {
    static constexpr int kWords = 8;
    uint32_t v[8];
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s)
    {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = st[i * S + s];
    }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t S, uint64_t s) const
    {
#pragma unroll
        for (int i = 0; i < 8; ++i) st[i * S + s] = v[i];
    }
    // v_n from the five taps of eq. (5): v_{n-1}, v_{n-4}, v_{n-5}, v_{n-7}, v_{n-8}.
    static __device__ __forceinline__ uint32_t step(uint32_t m1, uint32_t m4, uint32_t m5, uint32_t m7,
                                                    uint32_t m8)
    {
        using detail::xor3;
        const uint32_t u1 = m1 ^ (m1 << 13);             // (I+L^13) v_{n-1}
        const uint32_t u8 = m8 ^ (m8 >> 7);              // (I+R^7) v_{n-8}
        const uint32_t p = xor3(u1, u1 << 9, m4);        // (I+L^9)(.) + v_{n-4}
        const uint32_t q = xor3(m4 << 7, m5, m5 >> 3);   // L^7 v_{n-4} + (I+R^3) v_{n-5}
        const uint32_t r = xor3(m7, m7 >> 10, u8);       // (I+R^10) v_{n-7} + u8
        return xor3(p, q, r) ^ (u8 << 24);               // + L^24 u8
    }
    __device__ __forceinline__ uint32_t next()
    {
        const uint32_t vn = step(v[7], v[4], v[3], v[1], v[0]);
#pragma unroll
        for (int i = 0; i < 7; ++i) v[i] = v[i + 1];
        v[7] = vn;
        return vn;
    }
    __device__ __forceinline__ uint32_t last() const { return v[7]; }
};

// Eq. (6): y ^= y << 13; y ^= y >> 17; y ^= y << 5.
struct XS32 {
    static constexpr int kWords = 1;
    uint32_t y;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t, uint64_t s) { y = st[s]; }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t, uint64_t s) const { st[s] = y; }
    __device__ __forceinline__ uint32_t next()
    {
        y ^= y << 13;
        y ^= y >> 17;
        y ^= y << 5;
        return y;
    }
    __device__ __forceinline__ uint32_t last() const { return y; }
};

// Sec. III.A.1: two base-2^16 MWC words with their own multipliers (carried in
// the state), output (z << 16) + w.
struct MWC1616 {
    static constexpr int kWords = 4;
    uint32_t z, w, a1, a2;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s)
    {
        z = st[s];
        w = st[S + s];
        a1 = st[2 * S + s];
        a2 = st[3 * S + s];
    }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t S, uint64_t s) const
    {
        st[s] = z;
        st[S + s] = w;
        st[2 * S + s] = a1;
        st[3 * S + s] = a2;
    }
    __device__ __forceinline__ uint32_t next()
    {
        z = detail::mwc16_step(z, a1);
        w = detail::mwc16_step(w, a2);
        return (z << 16) + w;
    }
    __device__ __forceinline__ uint32_t last() const { return (z << 16) + w; }
};

// Sec. II.A.3 / III.A.3: KISS = ((MWC1616 output) ^ LCG) + XS32, with the
// LCG of eq. (7), jcong <- 69069 jcong + 1234567 (mod 2^32), and XS32 as eq. (6).
struct KISS {
    static constexpr int kWords = 6;
    uint32_t z, w, jsr, jcong, a1, a2;
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t s)
    {
        z = st[s];
        w = st[S + s];
        jsr = st[2 * S + s];
        jcong = st[3 * S + s];
        a1 = st[4 * S + s];
        a2 = st[5 * S + s];
    }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t S, uint64_t s) const
    {
        st[s] = z;
        st[S + s] = w;
        st[2 * S + s] = jsr;
        st[3 * S + s] = jcong;
        st[4 * S + s] = a1;
        st[5 * S + s] = a2;
    }
    __device__ __forceinline__ uint32_t next()
    {
        z = detail::mwc16_step(z, a1);
        w = detail::mwc16_step(w, a2);
        jcong = 69069u * jcong + 1234567u;
        jsr ^= jsr << 13;
        jsr ^= jsr >> 17;
        jsr ^= jsr << 5;
        return last();
    }
    __device__ __forceinline__ uint32_t last() const { return (((z << 16) + w) ^ jcong) + jsr; }
};

}  // namespace rng_inline
