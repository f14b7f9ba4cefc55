// host_math.cpp -- see host_math.hpp.
#include "host_math.hpp"

#include <cstring>
#include <mutex>

namespace rngx {

using u128 = unsigned __int128;

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod64(r, a, m);
        a = mulmod64(a, a, m);
        e >>= 1;
    }
    return r;
}

// Miller-Rabin with the first twelve primes as bases: deterministic for
// every n < 3.3e24, hence for all 64-bit n.
bool is_prime_u64(uint64_t n)
{
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t p : bases)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; ++r; }
    for (uint64_t a : bases) {
        uint64_t x = powmod64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int i = 1; i < r; ++i) {
            x = mulmod64(x, x, n);
            if (x == n - 1) { composite = false; break; }
        }
        if (composite) return false;
    }
    return true;
}

static bool safe_prime_rule(uint64_t a, int log2b)
{
    uint64_t m = (a << log2b) - 1;
    return is_prime_u64(m) && is_prime_u64((m - 1) / 2);
}

const std::vector<uint16_t> &mwc16_multipliers()
{
    static std::vector<uint16_t> t = [] {
        std::vector<uint16_t> v;
        for (uint64_t a = 2; a < 65536; ++a)
            if (safe_prime_rule(a, 16)) v.push_back((uint16_t)a);
        return v;
    }();
    return t;
}

uint32_t mwc32_multiplier()
{
    static uint32_t a = [] {
        for (uint64_t c = 65535; c > 1; --c)
            if (safe_prime_rule(c, 32)) return (uint32_t)c;
        return 0u;
    }();
    return a;
}

// ---------------------------------------------------------------- GF(2)
template <int W>
Gf2Mat<W> Gf2Mat<W>::identity()
{
    Gf2Mat m;
    std::memset(m.c, 0, sizeof(m.c));
    for (int b = 0; b < 32 * W; ++b) m.c[b][b >> 5] = 1u << (b & 31);
    return m;
}

template <int W>
void Gf2Mat<W>::apply(const uint32_t *in, uint32_t *out) const
{
    uint32_t r[W] = {};
    for (int w = 0; w < W; ++w) {
        uint32_t word = in[w];
        while (word) {
            int bit = __builtin_ctz(word);
            word &= word - 1;
            const uint32_t *col = c[32 * w + bit];
            for (int i = 0; i < W; ++i) r[i] ^= col[i];
        }
    }
    std::memcpy(out, r, sizeof(r));
}

template <int W>
Gf2Mat<W> Gf2Mat<W>::operator*(const Gf2Mat &rhs) const
{
    Gf2Mat out;
    for (int b = 0; b < 32 * W; ++b) apply(rhs.c[b], out.c[b]);
    return out;
}

template <int W>
bool Gf2Mat<W>::operator==(const Gf2Mat &o) const
{
    return std::memcmp(c, o.c, sizeof(c)) == 0;
}

template struct Gf2Mat<1>;
template struct Gf2Mat<8>;

// 32x32 building blocks: I, L^k (bit i -> bit i+k), R^k (bit i -> bit i-k),
// as column arrays, composed as matrices.
using M32 = Gf2Mat<1>;

static M32 shift_mat(int k, bool left)
{
    M32 m;
    std::memset(m.c, 0, sizeof(m.c));
    for (int i = 0; i < 32; ++i) {
        int j = left ? i + k : i - k;
        if (j >= 0 && j < 32) m.c[i][0] = 1u << j;
    }
    return m;
}

static M32 add(const M32 &a, const M32 &b)
{
    M32 r;
    for (int i = 0; i < 32; ++i) r.c[i][0] = a.c[i][0] ^ b.c[i][0];
    return r;
}

static M32 I_plus_L(int k) { return add(M32::identity(), shift_mat(k, true)); }
static M32 I_plus_R(int k) { return add(M32::identity(), shift_mat(k, false)); }

// Eq. (5) as a block companion matrix on the window (v_{n-8} .. v_{n-1}):
// the new word is sum_j A_j v_{n-j}, the other words slide down by one.
Gf2Mat<8> xs256_step_matrix()
{
    M32 A[9];
    for (auto &a : A) std::memset(a.c, 0, sizeof(a.c));
    A[1] = I_plus_L(9) * I_plus_L(13);
    A[4] = I_plus_L(7);
    A[5] = I_plus_R(3);
    A[7] = I_plus_R(10);
    A[8] = I_plus_L(24) * I_plus_R(7);
    Gf2Mat<8> M;
    std::memset(M.c, 0, sizeof(M.c));
    for (int w = 0; w < 8; ++w) {       // input word w holds v_{n-8+w}
        int lag = 8 - w;
        for (int bit = 0; bit < 32; ++bit) {
            uint32_t *col = M.c[32 * w + bit];
            if (w >= 1) col[w - 1] = 1u << bit;  // slides to position w-1
            col[7] = A[lag].c[bit][0];           // contribution to v_n
        }
    }
    return M;
}

// Eq. (6), applied as written: first (I+L^13), then (I+R^17), then (I+L^5).
Gf2Mat<1> xs32_step_matrix() { return I_plus_L(5) * I_plus_R(17) * I_plus_L(13); }

// ---------------------------------------------------------------- tables
static HostTables *build_tables()
{
    auto *T = new HostTables();
    T->mwc32_a = mwc32_multiplier();
    T->mwc32_m = ((uint64_t)T->mwc32_a << 32) - 1;
    const auto &t = mwc16_multipliers();
    for (int i = 0; i < kMwc16Count; ++i) T->t392[i] = t[i];

    const uint64_t m = T->mwc32_m;
    const uint64_t two64 = mulmod64(((uint64_t)1 << 32) % m, ((uint64_t)1 << 32) % m, m);
    uint64_t p = T->mwc32_a;  // a^(2^0)
    for (int b = 0; b < kPowBits; ++b) {
        T->mwc32_pow_fold[b] = mulmod64(p, two64, m);
        p = mulmod64(p, p, m);
    }

    uint32_t A = 69069u, C = 1234567u;  // eq. (7)
    for (int b = 0; b < kPowBits; ++b) {
        T->lcg_pow[b][0] = A;
        T->lcg_pow[b][1] = C;
        C = A * C + C;  // (A,C) o (A,C)
        A = A * A;
    }

    M32 x = xs32_step_matrix();
    for (int b = 0; b < kPowBits; ++b) {
        for (int i = 0; i < 32; ++i) T->xs32_pow[b][i] = x.c[i][0];
        x = x * x;
    }

    for (int i = 0; i < kMwc16Count; ++i) {
        uint64_t a = t[i], mi = (a << 16) - 1;
        uint64_t two48 = powmod64(2, 48, mi);
        uint64_t q = a;
        for (int b = 0; b < kPowBits; ++b) {
            T->mwc16_pow_fold[i][b] = (uint32_t)mulmod64(q, two48, mi);
            q = mulmod64(q, q, mi);
        }
    }

    T->xs256_pow.resize((size_t)kPowBits * 256 * 8);
    auto *M = new Gf2Mat<8>(xs256_step_matrix());
    for (int b = 0; b < kPowBits; ++b) {
        std::memcpy(&T->xs256_pow[(size_t)b * 2048], M->c, sizeof(M->c));
        *M = (*M) * (*M);
    }
    delete M;
    T->xs256_t4.resize((size_t)kPowBits * 8192);
    for (int b = 0; b < kPowBits; ++b) xs256_nibble_table(&T->xs256_pow[(size_t)b * 2048], &T->xs256_t4[(size_t)b * 8192]);
    // One table per hexadecimal digit d != 0 at position j: a jump by k then
    // takes one product per nonzero digit of k instead of one per set bit.
    T->xs256_t4w.resize((size_t)16 * 15 * 8192);
    auto *base = new Gf2Mat<8>, *P = new Gf2Mat<8>;
    for (int j = 0; j < 16; ++j) {
        std::memcpy(base->c, &T->xs256_pow[(size_t)(4 * j) * 2048], sizeof(base->c));
        *P = *base;
        for (int d = 1; d <= 15; ++d) {
            if (d > 1) *P = (*P) * (*base);
            xs256_nibble_table(&P->c[0][0], &T->xs256_t4w[((size_t)j * 15 + (d - 1)) * 8192]);
        }
    }
    delete base;
    delete P;
    return T;
}

void xs256_nibble_table(const uint32_t *cols, uint32_t *t4)
{
    for (int p = 0; p < 64; ++p)
        for (int h = 0; h < 2; ++h)
            for (int v = 0; v < 16; ++v)
                for (int w = 0; w < 4; ++w) {
                    uint32_t x = 0;
                    for (int k = 0; k < 4; ++k)
                        if ((v >> k) & 1) x ^= cols[(4 * p + k) * 8 + 4 * h + w];
                    t4[((p * 2 + h) * 16 + v) * 4 + w] = x;
                }
}

const HostTables &host_tables()
{
    static HostTables *T = build_tables();
    return *T;
}

uint64_t mwc32_fold_const(uint64_t k)
{
    const HostTables &T = host_tables();
    const uint64_t m = T.mwc32_m;
    const uint64_t two64 = mulmod64(((uint64_t)1 << 32) % m, ((uint64_t)1 << 32) % m, m);
    return mulmod64(powmod64(T.mwc32_a, k, m), two64, m);
}

void xs32_lcg_jump(uint64_t k, uint32_t cols[32], uint32_t *lcg_a, uint32_t *lcg_c)
{
    const HostTables &T = host_tables();
    uint32_t A = 1, C = 0;  // identity affine map
    for (int i = 0; i < 32; ++i) cols[i] = 1u << i;
    for (int b = 0; b < kPowBits; ++b) {
        if (!((k >> b) & 1)) continue;
        const uint32_t pa = T.lcg_pow[b][0], pc = T.lcg_pow[b][1];
        C = pa * C + pc;  // 2^b more steps after the current map
        A = pa * A;
        // column i <- M^(2^b) column i, branch-free with the columns innermost
        // (data-dependent branches here cost more than the arithmetic)
        uint32_t next[32] = {0};
        for (int j = 0; j < 32; ++j) {
            const uint32_t pj = T.xs32_pow[b][j];
            for (int i = 0; i < 32; ++i) next[i] ^= pj & (0u - ((cols[i] >> j) & 1u));
        }
        for (int i = 0; i < 32; ++i) cols[i] = next[i];
    }
    *lcg_a = A;
    *lcg_c = C;
}

}  // namespace rngx
