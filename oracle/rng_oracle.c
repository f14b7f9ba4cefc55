/*
 * rng_oracle.c -- plain, serial, obviously-correct CPU reference for the
 * generators studied in Hissoiny, Despres & Ozell, "Using graphics processing
 * units to generate random numbers" (arXiv:1101.1846).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * generator with the HIP path: every constant below is re-derived here from
 * the paper's text or from mathematics.
 *
 * Everything is unsigned integer arithmetic; 32-bit words wrap mod 2^32.
 * Convention (Sec. II.A, eq. (1)): the seed is never emitted; sample k is the
 * value produced by the (k+1)-th application of the transition ("step, then
 * emit").
 *
 * State layout shared with the library's C ABI (an interface, not code):
 * structure-of-arrays, word w of stream s at state[w * n_streams + s].
 *   MWC32   : x, c                      (2 words)
 *   XS256   : v0..v7, v0 the oldest     (8 words)
 *   XS32    : y                         (1 word)
 *   KISS    : z, w, jsr, jcong, a1, a2  (6 words)
 *   MWC1616 : z, w, a1, a2              (4 words)
 * Output layout: stream-major, sample k of stream s at out[s * n + k].
 *
 * Pinned by tests/test_oracle_pins.py (multiplier count, periods, the MWC
 * congruence, jump == brute force, SplitMix64 vectors, the FP32 map).  The
 * absolute output values of the generators have no external test vector in
 * the paper: see the "parity unpinned" notes next to the affected readings.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_MWC32 = 1, ORC_XS256 = 2, ORC_XS32 = 3, ORC_KISS = 4, ORC_MWC1616 = 5 };
enum { ORC_U32 = 0, ORC_F32 = 1 };

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Primality by trial division: slow and plainly correct.                    */
/* ------------------------------------------------------------------------ */
static int is_prime_td(uint64_t n)
{
    if (n < 2) return 0;
    if (n % 2 == 0) return n == 2;
    for (uint64_t d = 3; d <= n / d; d += 2)
        if (n % d == 0) return 0;
    return 1;
}

/* Sec. II.A.1 and III.A.1: with base b = 2^16 the multiplier a must be below
 * 2^16 and a*b - 1 must be a safe prime, i.e. a*2^16 - 1 and
 * (a*2^16 - 2)/2 = a*2^15 - 1 both prime.  The paper counts 392 such a.
 * Writes them ascending into out (up to cap) and returns the count. */
int orc_mwc16_table(uint16_t *out, int cap)
{
    int n = 0;
    for (uint64_t a = 1; a < 65536; a++) {
        if (!is_prime_td(a * 32768u - 1)) continue;
        if (!is_prime_td(a * 65536u - 1)) continue;
        if (out && n < cap) out[n] = (uint16_t)a;
        n++;
    }
    return n;
}

/* Base b = 2^32: the paper prints no multiplier, so the multiplier is the
 * largest a < 2^16 with a*2^32 - 1 and (a*2^32 - 2)/2 both prime (the same
 * safe-prime rule of Sec. II.A.1).  Cached after the first call. */
uint32_t orc_mwc32_multiplier(void)
{
    static uint32_t cached = 0;
    if (cached) return cached;
    for (uint64_t a = 65535; a >= 1; a--) {
        uint64_t m = (a << 32) - 1;
        if (!is_prime_td((m - 1) / 2)) continue;
        if (!is_prime_td(m)) continue;
        cached = (uint32_t)a;
        return cached;
    }
    return 0;
}

int orc_is_prime(uint64_t n) { return is_prime_td(n); }

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the seeding generator.     */
/* ------------------------------------------------------------------------ */
#define SM64_GAMMA 0x9E3779B97F4A7C15ull

uint64_t orc_sm64_next(uint64_t *s)
{
    uint64_t z = (*s += SM64_GAMMA);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* The recurrences, one step each, emitting the new value.                   */
/* ------------------------------------------------------------------------ */

/* Eq. (2)-(3) with b = 2^32: t = a*x + c; x' = t mod b; c' = floor(t / b). */
uint32_t orc_step_mwc32(uint32_t a, uint32_t *x, uint32_t *c)
{
    uint64_t t = (uint64_t)a * (*x) + (*c);
    *x = (uint32_t)t;
    *c = (uint32_t)(t >> 32);
    return *x;
}

/* Eq. (2)-(3) with b = 2^16, the carry kept in the upper half of one 32-bit
 * word z = c*2^16 + x (Sec. II.A.1: the mod is a mask, the carry a shift). */
uint32_t orc_step_mwc16(uint32_t a, uint32_t *z)
{
    uint32_t x = *z & 0xFFFFu, c = *z >> 16;
    *z = a * x + c;
    return *z;
}

/* Sec. III.A.1: two base-2^16 MWCs with distinct multipliers, their two
 * 16-bit values joined into one 32-bit number.  Reading: (z << 16) + w on the
 * full new words, the form whose operation count matches the ten operations
 * the paper counts (3 shifts, 2 ands, 2 multiplies, 3 adds).  Parity unpinned
 * against any external implementation. */
uint32_t orc_step_mwc1616(uint32_t a1, uint32_t a2, uint32_t *z, uint32_t *w)
{
    orc_step_mwc16(a1, z);
    orc_step_mwc16(a2, w);
    return (*z << 16) + *w;
}

/* Eq. (6): A_1 = (I + L^13)(I + R^17)(I + L^5), applied in the order written
 * (Marsaglia's row-vector convention): <<13, then >>17, then <<5.  L is C's
 * left shift.  The reverse order is also full period, so parity of the order
 * is unpinned. */
uint32_t orc_step_xs32(uint32_t *y)
{
    uint32_t v = *y;
    v ^= v << 13;
    v ^= v >> 17;
    v ^= v << 5;
    *y = v;
    return v;
}

/* Eq. (7) with a = 69069, c = 1234567, m = 2^32 (Sec. II.A.3). */
uint32_t orc_step_lcg(uint32_t *X)
{
    *X = 69069u * (*X) + 1234567u;
    return *X;
}

/* Eq. (5), Panneton's r = 8, w = 32 generator.  v[0..7] is the window
 * (v_{n-8}, ..., v_{n-1}), oldest first:
 *   v_n = (I+L^9)(I+L^13) v_{n-1} + (I+L^7) v_{n-4} + (I+R^3) v_{n-5}
 *       + (I+R^10) v_{n-7} + (I+L^24)(I+R^7) v_{n-8}      (sums over GF(2)).
 * A product of matrices acts on a column vector right factor first, so
 * (I+L^24)(I+R^7) y applies >>7 first, then <<24 (parity of this order is
 * unpinned; both orders give a full-period generator). */
uint32_t orc_step_xs256(uint32_t v[8])
{
    uint32_t y, t1, t4, t5, t7, t8;
    y = v[7];  y ^= y << 13;  t1 = y ^ (y << 9);     /* v_{n-1} */
    y = v[4];  t4 = y ^ (y << 7);                     /* v_{n-4} */
    y = v[3];  t5 = y ^ (y >> 3);                     /* v_{n-5} */
    y = v[1];  t7 = y ^ (y >> 10);                    /* v_{n-7} */
    y = v[0];  y ^= y >> 7;  t8 = y ^ (y << 24);     /* v_{n-8} */
    uint32_t vn = t1 ^ t4 ^ t5 ^ t7 ^ t8;
    for (int i = 0; i < 7; i++) v[i] = v[i + 1];
    v[7] = vn;
    return vn;
}

/* Sec. II.A.3: KISS = (MWC xor LCG) + XorShift, with the MWC the paper's
 * dual base-2^16 generator (Sec. III.A.3). */
uint32_t orc_step_kiss(uint32_t a1, uint32_t a2, uint32_t *z, uint32_t *w,
                       uint32_t *jsr, uint32_t *jcong)
{
    uint32_t mwc = orc_step_mwc1616(a1, a2, z, w);
    uint32_t lcg = orc_step_lcg(jcong);
    uint32_t xs = orc_step_xs32(jsr);
    return (mwc ^ lcg) + xs;
}

/* The FP32 map: the top 24 bits of u scaled by 2^-24.  (u >> 8) has at most
 * 24 significant bits, so both the conversion and the power-of-two scaling
 * are exact and the result lies in [0, 1 - 2^-24]. */
float orc_to_f32(uint32_t u)
{
    return (float)(u >> 8) * (1.0f / 16777216.0f);
}

/* ------------------------------------------------------------------------ */
/* Seeding: per-stream initial states from SplitMix64(seed).                 */
/* Stream s (global id g = first_stream + s) takes SplitMix64 outputs        */
/* g*D .. g*D + D-1, D = 1 (MWC32, XS32), 2 (MWC1616), 3 (KISS), 4 (XS256).  */
/* ------------------------------------------------------------------------ */
static int draws_per_stream(int gen)
{
    switch (gen) {
    case ORC_MWC32: return 1;
    case ORC_XS32: return 1;
    case ORC_MWC1616: return 2;
    case ORC_KISS: return 3;
    case ORC_XS256: return 4;
    }
    return 0;
}

int orc_state_words(int gen)
{
    switch (gen) {
    case ORC_MWC32: return 2;
    case ORC_XS256: return 8;
    case ORC_XS32: return 1;
    case ORC_KISS: return 6;
    case ORC_MWC1616: return 4;
    }
    return 0;
}

static uint16_t g_t392[392];
static int g_t392_n = 0;

static const uint16_t *t392(void)
{
    if (!g_t392_n) g_t392_n = orc_mwc16_table(g_t392, 392);
    return g_t392;
}

/* MWC state (x, c) with c < a and z = c*b + x outside the two fixed points
 * z = 0 and z = a*b - 1 of the map z -> a*z mod (a*b - 1). */
static uint32_t mwc16_word_from(uint32_t h, uint32_t a)
{
    uint32_t x = h & 0xFFFFu, c = (h >> 16) % a;
    uint32_t z = (c << 16) | x;
    if (z == 0) z = 1;
    if (z == a * 65536u - 1) z = a * 65536u - 2;
    return z;
}

static void mwc_pair_from(uint64_t d, uint32_t *a1, uint32_t *a2)
{
    const uint16_t *T = t392();
    uint32_t i = (uint32_t)d % 392u;
    uint32_t j = (i + 1u + (uint32_t)(d >> 32) % 391u) % 392u;
    *a1 = T[i];
    *a2 = T[j];
}

void orc_seed(int gen, uint64_t seed, uint64_t first_stream, uint64_t n_streams,
              uint32_t *state)
{
    const int D = draws_per_stream(gen);
    const uint64_t S = n_streams;
    uint64_t sm = seed;
    /* advance serially to the first draw of stream first_stream */
    for (uint64_t i = 0; i < first_stream * (uint64_t)D; i++) orc_sm64_next(&sm);
    uint32_t a32 = gen == ORC_MWC32 ? orc_mwc32_multiplier() : 0;
    for (uint64_t s = 0; s < S; s++) {
        uint64_t d[4] = {0, 0, 0, 0};
        for (int j = 0; j < D; j++) d[j] = orc_sm64_next(&sm);
        switch (gen) {
        case ORC_MWC32: {
            uint64_t x = (uint32_t)d[0], c = (uint32_t)(d[0] >> 32) % a32;
            uint64_t m = ((uint64_t)a32 << 32) - 1;
            uint64_t z = (c << 32) | x;
            if (z == 0) z = 1;
            if (z == m) z = m - 1;
            state[0 * S + s] = (uint32_t)z;
            state[1 * S + s] = (uint32_t)(z >> 32);
            break;
        }
        case ORC_XS32: {
            uint32_t y = (uint32_t)d[0];
            state[s] = y ? y : 1u;
            break;
        }
        case ORC_XS256: {
            uint32_t v[8], any = 0;
            for (int i = 0; i < 4; i++) {
                v[2 * i] = (uint32_t)d[i];
                v[2 * i + 1] = (uint32_t)(d[i] >> 32);
            }
            for (int i = 0; i < 8; i++) any |= v[i];
            if (!any) v[7] = 1;
            for (int i = 0; i < 8; i++) state[(uint64_t)i * S + s] = v[i];
            break;
        }
        case ORC_MWC1616:
        case ORC_KISS: {
            uint32_t a1, a2;
            mwc_pair_from(d[0], &a1, &a2);
            uint32_t z = mwc16_word_from((uint32_t)d[1], a1);
            uint32_t w = mwc16_word_from((uint32_t)(d[1] >> 32), a2);
            if (gen == ORC_MWC1616) {
                state[0 * S + s] = z;
                state[1 * S + s] = w;
                state[2 * S + s] = a1;
                state[3 * S + s] = a2;
            } else {
                uint32_t jsr = (uint32_t)d[2];
                state[0 * S + s] = z;
                state[1 * S + s] = w;
                state[2 * S + s] = jsr ? jsr : 1u;
                state[3 * S + s] = (uint32_t)(d[2] >> 32);
                state[4 * S + s] = a1;
                state[5 * S + s] = a2;
            }
            break;
        }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Serial generation of streams [s_begin, s_end) of an S-stream state array. */
/* ------------------------------------------------------------------------ */
static uint32_t step_one(int gen, uint32_t *st, uint32_t a32)
{
    switch (gen) {
    case ORC_MWC32: return orc_step_mwc32(a32, &st[0], &st[1]);
    case ORC_XS256: return orc_step_xs256(st);
    case ORC_XS32: return orc_step_xs32(&st[0]);
    case ORC_KISS: return orc_step_kiss(st[4], st[5], &st[0], &st[1], &st[2], &st[3]);
    case ORC_MWC1616: return orc_step_mwc1616(st[2], st[3], &st[0], &st[1]);
    }
    return 0;
}

static void load_stream(int gen, const uint32_t *state, uint64_t S, uint64_t s, uint32_t *st)
{
    int W = orc_state_words(gen);
    for (int w = 0; w < W; w++) st[w] = state[(uint64_t)w * S + s];
}

static void store_stream(int gen, uint32_t *state, uint64_t S, uint64_t s, const uint32_t *st)
{
    int W = orc_state_words(gen);
    for (int w = 0; w < W; w++) state[(uint64_t)w * S + s] = st[w];
}

void orc_generate_range(int gen, uint32_t *state, uint64_t n_streams, uint64_t s_begin,
                        uint64_t s_end, uint64_t n, int dtype, void *out)
{
    uint32_t a32 = gen == ORC_MWC32 ? orc_mwc32_multiplier() : 0;
    uint32_t st[8];
    for (uint64_t s = s_begin; s < s_end; s++) {
        load_stream(gen, state, n_streams, s, st);
        for (uint64_t k = 0; k < n; k++) {
            uint32_t u = step_one(gen, st, a32);
            if (dtype == ORC_F32) ((float *)out)[s * n + k] = orc_to_f32(u);
            else ((uint32_t *)out)[s * n + k] = u;
        }
        store_stream(gen, state, n_streams, s, st);
    }
}

void orc_generate(int gen, uint32_t *state, uint64_t n_streams, uint64_t n, int dtype, void *out)
{
    orc_generate_range(gen, state, n_streams, 0, n_streams, n, dtype, out);
}

/* One logical stream stepped serially: the reference for sequence splitting
 * (Sec. II.A.4).  Samples at the sorted positions pos[0..npos) are written to
 * out_pos; the first n_head and the last n_tail samples are written to head
 * and tail; st (one stream, words contiguous) ends advanced by total steps. */
void orc_serial_sample(int gen, uint32_t *st, uint64_t total, const uint64_t *pos,
                       uint64_t npos, uint32_t *out_pos, uint64_t n_head, uint32_t *head,
                       uint64_t n_tail, uint32_t *tail)
{
    uint32_t a32 = gen == ORC_MWC32 ? orc_mwc32_multiplier() : 0;
    uint64_t p = 0;
    for (uint64_t k = 0; k < total; k++) {
        uint32_t u = step_one(gen, st, a32);
        if (k < n_head) head[k] = u;
        if (k + n_tail >= total) tail[k - (total - n_tail)] = u;
        while (p < npos && pos[p] == k) out_pos[p++] = u;
    }
}

/* ------------------------------------------------------------------------ */
/* Fused consumer: pairs of uniforms tested against the unit quarter circle. */
/* Sample pair (u_{2k}, u_{2k+1}) of one stream gives i = u_{2k} >> 8 and    */
/* j = u_{2k+1} >> 8; the pair counts when i^2 + j^2 < 2^48, which is the    */
/* real test x^2 + y^2 < 1 for x = i / 2^24, y = j / 2^24 done exactly.  An  */
/* odd trailing sample advances the state but is not counted.                */
/* ------------------------------------------------------------------------ */
uint64_t orc_fused_pi_range(int gen, uint32_t *state, uint64_t n_streams, uint64_t s_begin,
                            uint64_t s_end, uint64_t n)
{
    uint32_t a32 = gen == ORC_MWC32 ? orc_mwc32_multiplier() : 0;
    uint32_t st[8];
    uint64_t count = 0;
    for (uint64_t s = s_begin; s < s_end; s++) {
        load_stream(gen, state, n_streams, s, st);
        for (uint64_t p = 0; p < n / 2; p++) {
            uint64_t i = step_one(gen, st, a32) >> 8;
            uint64_t j = step_one(gen, st, a32) >> 8;
            if (i * i + j * j < (1ull << 48)) count++;
        }
        if (n & 1) step_one(gen, st, a32);
        store_stream(gen, state, n_streams, s, st);
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Jump-ahead.  Sec. II.A.4 needs the i-th number without the intermediate   */
/* ones for sequence splitting and leapfrogging; the paper gives no method.  */
/* The exponent k is a little-endian array of nk 32-bit words so that a jump */
/* by a full period (2^256 - 1 for eq. (5)) can be expressed.                */
/* ------------------------------------------------------------------------ */
static int big_bit(const uint32_t *k, int nk, int i)
{
    return (i / 32 < nk) ? (int)((k[i / 32] >> (i % 32)) & 1u) : 0;
}

/* MWC: write z = c*b + x.  By eq. (2)-(3) one step gives c'*b + x' = a*x + c,
 * and a*z = a*b*c + a*x is congruent to c + a*x modulo m = a*b - 1 because
 * a*b = 1 (mod m).  So z' = a*z mod m for z in [1, m-1], and k steps multiply
 * z by a^k mod m. */
static uint64_t mulmod(uint64_t x, uint64_t y, uint64_t m)
{
    return (uint64_t)(((u128)x * y) % m);
}

static uint64_t powmod_big(uint64_t a, const uint32_t *k, int nk, uint64_t m)
{
    uint64_t r = 1 % m, p = a % m;
    for (int i = 0; i < 32 * nk; i++) {
        if (big_bit(k, nk, i)) r = mulmod(r, p, m);
        p = mulmod(p, p, m);
    }
    return r;
}

/* LCG mod 2^32: k steps of X -> A X + C compose to X -> A_k X + C_k.
 * Square-and-combine: (A,C) o (A,C) = (A^2, A C + C). */
static void lcg_pow_big(const uint32_t *k, int nk, uint32_t *Ak, uint32_t *Ck)
{
    uint32_t rA = 1, rC = 0, pA = 69069u, pC = 1234567u;
    for (int i = 0; i < 32 * nk; i++) {
        if (big_bit(k, nk, i)) { rC = pA * rC + pC; rA = pA * rA; }
        pC = pA * pC + pC;
        pA = pA * pA;
    }
    *Ak = rA;
    *Ck = rC;
}

/* GF(2)-linear generators (eq. (4)): the step is a 32W x 32W bit matrix M,
 * stored column by column, column b = the state reached in one step from the
 * unit state e_b.  W = 1 for XS32, 8 for XS256. */
typedef struct { int W; uint32_t *col; } gf2mat;

static gf2mat mat_new(int W)
{
    gf2mat m = {W, (uint32_t *)calloc((size_t)32 * W * W, sizeof(uint32_t))};
    return m;
}

static void mat_free(gf2mat m) { free(m.col); }

static void mat_vec(const gf2mat *M, const uint32_t *v, uint32_t *out)
{
    int W = M->W;
    uint32_t r[8] = {0};
    for (int b = 0; b < 32 * W; b++)
        if ((v[b / 32] >> (b % 32)) & 1u)
            for (int w = 0; w < W; w++) r[w] ^= M->col[(size_t)b * W + w];
    memcpy(out, r, sizeof(uint32_t) * W);
}

static void mat_mul(const gf2mat *A, const gf2mat *B, gf2mat *C)
{
    int W = A->W;
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * 32 * W * W);
    for (int b = 0; b < 32 * W; b++) mat_vec(A, &B->col[(size_t)b * W], &tmp[(size_t)b * W]);
    memcpy(C->col, tmp, sizeof(uint32_t) * 32 * W * W);
    free(tmp);
}

static gf2mat step_matrix(int gen)
{
    int W = gen == ORC_XS256 ? 8 : 1;
    gf2mat M = mat_new(W);
    for (int b = 0; b < 32 * W; b++) {
        uint32_t st[8] = {0};
        st[b / 32] = 1u << (b % 32);
        if (gen == ORC_XS256) orc_step_xs256(st);
        else orc_step_xs32(st);
        memcpy(&M.col[(size_t)b * W], st, sizeof(uint32_t) * W);
    }
    return M;
}

static gf2mat mat_pow_big(int gen, const uint32_t *k, int nk)
{
    gf2mat P = step_matrix(gen);
    int W = P.W;
    gf2mat R = mat_new(W);
    for (int b = 0; b < 32 * W; b++) R.col[(size_t)b * W + b / 32] = 1u << (b % 32);
    int top = 32 * nk - 1;
    while (top >= 0 && !big_bit(k, nk, top)) top--;
    for (int i = 0; i <= top; i++) {
        if (big_bit(k, nk, i)) mat_mul(&P, &R, &R);
        if (i < top) mat_mul(&P, &P, &P);
    }
    mat_free(P);
    return R;
}

/* Advance every stream by k steps. */
void orc_skip_big(int gen, uint32_t *state, uint64_t n_streams, const uint32_t *k, int nk)
{
    const uint64_t S = n_streams;
    uint32_t st[8];
    if (gen == ORC_MWC32) {
        uint64_t a = orc_mwc32_multiplier(), m = (a << 32) - 1;
        uint64_t ak = powmod_big(a, k, nk, m);
        for (uint64_t s = 0; s < S; s++) {
            load_stream(gen, state, S, s, st);
            uint64_t z = ((uint64_t)st[1] << 32) | st[0];
            z = mulmod(ak, z, m);
            st[0] = (uint32_t)z;
            st[1] = (uint32_t)(z >> 32);
            store_stream(gen, state, S, s, st);
        }
        return;
    }
    if (gen == ORC_XS32 || gen == ORC_XS256) {
        gf2mat Mk = mat_pow_big(gen, k, nk);
        for (uint64_t s = 0; s < S; s++) {
            load_stream(gen, state, S, s, st);
            mat_vec(&Mk, st, st);
            store_stream(gen, state, S, s, st);
        }
        mat_free(Mk);
        return;
    }
    /* MWC1616 and KISS: each component jumps on its own. */
    gf2mat Mk = mat_pow_big(ORC_XS32, k, nk);
    uint32_t Ak, Ck;
    lcg_pow_big(k, nk, &Ak, &Ck);
    for (uint64_t s = 0; s < S; s++) {
        load_stream(gen, state, S, s, st);
        int ia = gen == ORC_KISS ? 4 : 2;
        for (int c = 0; c < 2; c++) {
            uint64_t a = st[ia + c], m = a * 65536u - 1;
            st[c] = (uint32_t)mulmod(powmod_big(a, k, nk, m), st[c], m);
        }
        if (gen == ORC_KISS) {
            mat_vec(&Mk, &st[2], &st[2]);
            st[3] = Ak * st[3] + Ck;
        }
        store_stream(gen, state, S, s, st);
    }
    mat_free(Mk);
}

void orc_skip(int gen, uint32_t *state, uint64_t n_streams, uint64_t k)
{
    uint32_t kw[2] = {(uint32_t)k, (uint32_t)(k >> 32)};
    orc_skip_big(gen, state, n_streams, kw, 2);
}

/* ------------------------------------------------------------------------ */
/* Brute-force periods (for the pins): steps until the state first returns. */
/* ------------------------------------------------------------------------ */
uint64_t orc_period_xs32(uint32_t y0)
{
    uint32_t y = y0;
    uint64_t n = 0;
    do { orc_step_xs32(&y); n++; } while (y != y0);
    return n;
}

uint64_t orc_period_lcg(uint32_t x0)
{
    uint32_t x = x0;
    uint64_t n = 0;
    do { orc_step_lcg(&x); n++; } while (x != x0);
    return n;
}

uint64_t orc_period_mwc16(uint32_t a, uint32_t z0)
{
    uint32_t z = z0;
    uint64_t n = 0;
    do { orc_step_mwc16(a, &z); n++; } while (z != z0);
    return n;
}

/* Generic MWC with base 2^bits (bits <= 16) for small-word period checks. */
uint64_t orc_period_mwc_small(uint32_t a, int bits, uint32_t x0, uint32_t c0)
{
    uint32_t mask = (1u << bits) - 1, x = x0, c = c0;
    uint64_t n = 0;
    do {
        uint32_t t = a * x + c;
        x = t & mask;
        c = t >> bits;
        n++;
    } while (x != x0 || c != c0);
    return n;
}
