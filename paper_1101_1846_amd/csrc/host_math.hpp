// host_math.hpp -- host-side number theory and GF(2) algebra that the
// library needs before it can launch anything: the multiplier tables, the
// MWC32 multiplier, and the jump-ahead power tables uploaded to the device.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace rngx {

constexpr int kMwc16Count = 392;  // Sec. III.A.1 counts 392 base-2^16 multipliers
constexpr int kPowBits = 64;      // jump distances are 64-bit

// 64-bit modular arithmetic (exact, via 128-bit products).
uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m);
uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m);
bool is_prime_u64(uint64_t n);  // deterministic Miller-Rabin for all 64-bit n

// Safe-prime multiplier rule of Sec. II.A.1: a*b - 1 and (a*b - 2)/2 prime.
const std::vector<uint16_t> &mwc16_multipliers();  // 392 entries, ascending
uint32_t mwc32_multiplier();                         // largest a < 2^16 for b = 2^32

// A W-word GF(2)-linear state map (W = 1 for xorshift32, 8 for the r = 8
// XorShift of eq. (5)), stored column-major: col(b) is the image of the unit
// state with only bit b set (bit b = bit b%32 of word b/32).
template <int W>
struct Gf2Mat {
    uint32_t c[32 * W][W];
    static Gf2Mat identity();
    void apply(const uint32_t *in, uint32_t *out) const;
    Gf2Mat operator*(const Gf2Mat &rhs) const;  // (this * rhs) x = this(rhs(x))
    bool operator==(const Gf2Mat &o) const;
};

Gf2Mat<8> xs256_step_matrix();  // eq. (5)
Gf2Mat<1> xs32_step_matrix();   // eq. (6)

// Device-side jump tables, written once per device.  All multiplicative
// constants are stored in the "fold" domain used by the device modular
// multiply (see rng_device.hpp): MWC32 constants pre-multiplied by 2^64 mod m,
// MWC16 constants by 2^48 mod m_i.
struct HostTables {
    uint32_t mwc32_a;
    uint64_t mwc32_m;
    uint16_t t392[kMwc16Count];
    uint64_t mwc32_pow_fold[kPowBits];         // a^(2^b) * 2^64 mod m
    uint32_t lcg_pow[kPowBits][2];             // (A, C) of 2^b LCG steps
    uint32_t xs32_pow[kPowBits][32];           // M^(2^b), 32 columns
    uint32_t mwc16_pow_fold[kMwc16Count][kPowBits];  // a_i^(2^b) * 2^48 mod m_i
    std::vector<uint32_t> xs256_pow;           // [64][256][8]: M^(2^b)
    std::vector<uint32_t> xs256_t4;            // [64][64][2][16][4]: 4-bit lookup tables of M^(2^b)
    std::vector<uint32_t> xs256_t4w;           // [16][15][8192]: 4-bit lookup tables of M^(d 16^j), d = 1..15
};

// 4-bit lookup table of a 256x256 GF(2) matrix given by its 256 columns of 8
// words: entry (p, h, v) holds words 4h .. 4h+3 of the XOR of the columns 4p+k
// over the set bits k of v (p < 64, h < 2, v < 16; 32 KiB).  M x is then the
// XOR over p of entries (p, 0, v_p) and (p, 1, v_p), v_p the p-th nibble of x.
void xs256_nibble_table(const uint32_t *cols, uint32_t *t4);
const HostTables &host_tables();

// Constants of a k-step map, composed from the power tables on the host (for
// the kernels that move many states, or many threads, by one distance).
uint64_t mwc32_fold_const(uint64_t k);
// Columns of M^k for xorshift32 (eq. (6)) and the (A_k, C_k) of k LCG steps.
void xs32_lcg_jump(uint64_t k, uint32_t cols[32], uint32_t *lcg_a, uint32_t *lcg_c);

}  // namespace rngx
