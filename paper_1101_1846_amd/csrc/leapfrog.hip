// leapfrog.hip -- leapfrog parallelisation of one sequence (Sec. II.A.4):
// thread j of T emits R_j, R_{j+T}, R_{j+2T}, ..., so that number i of the
// sequence lands at out[i] and every wave stores 64 consecutive numbers.
// Each thread starts at state_j (a radix-16 tree of jumps, as for sequence
// splitting), steps once, and then leaps T steps per number with the
// generator's T-step map:
//   MWC32    z <- (a^T mod m) z mod m         one fold-domain multiply (eqs. (2)-(3))
//   MWC1616  z, w <- a_i^T z mod m_i           two; constants from the state's multipliers
//   XS32     y <- M^T y                        32x32 GF(2) product, byte tables in LDS
//   XS256    v <- M^T v                        256x256 GF(2) product, 4-bit table in LDS
//   KISS     MWC1616 and XS32 parts as above, LCG jcong <- A_T jcong + C_T
// The constants that depend only on T come from the host's jump tables; the
// MWC16 ones (per multiplier pair) and the XS256 table are built on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "host_math.hpp"
#include "rng.h"
#include "rng_abi_internal.hpp"

namespace rngx {

namespace {

constexpr uint64_t kConstBytes = 256;                 // MWC16 fold constants
constexpr uint64_t kColBytes = 256 * 8 * 4;           // XS256 columns of M^T
constexpr uint64_t kTableBytes = 2048 * 16;           // XS256 4-bit table of M^T
constexpr uint64_t kByteTableBytes = 4 * 256 * 4;     // xorshift32 byte tables of M^T

uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

struct LeapArgs {
    const uint32_t *ws;      // [W][T] thread start states (state_j)
    const uint32_t *dconst;  // device-built constants: [0], [1] MWC16 fold constants; XS256 table at
                             // +kConstBytes+kColBytes; xorshift32 byte tables at +kConstBytes
    uint64_t T, total;
    uint32_t *out;           // [total]
    uint32_t *final_state;   // [W]
    uint64_t mwc32_af;       // a^T * 2^64 mod m
    uint32_t lcg_a, lcg_c;   // T steps of the LCG
    uint32_t xs32[32];       // columns of M^T (xorshift32)
    DevTables tab;
};

template <int DT>
__device__ __forceinline__ uint32_t bits(uint32_t u)
{
    if constexpr (DT == RNG_DT_F32) return __float_as_uint(to_unit_f32(u));
    else return u;
}

// Fold-domain constants a_i^T * 2^48 mod m_i of a stream's two MWC16 words
// (multipliers at state words wa1, wa2): jump the fold image of 1.
__global__ void k_leap_mwc16(const uint32_t *state_one, uint32_t wa1, uint32_t wa2, uint64_t T, uint32_t *dconst,
                             DevTables tab)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t a[2] = {state_one[wa1], state_one[wa2]};
    for (int i = 0; i < 2; ++i) {
        const uint32_t m = a[i] * 65536u - 1u;
        const uint32_t *p = tab.mwc16_pow + t392_index(tab.t392, a[i]) * 64;
        uint32_t z = (uint32_t)(((uint64_t)1 << 48) % m);
        for (int b = 0; b < 64 && (T >> b); ++b)
            if ((T >> b) & 1) z = mwc16_mulmod(z, p[b], a[i]);
        dconst[i] = z;
    }
}

// Column c of M^T for the r = 8 XorShift: the unit state e_c jumped by T.
__global__ __launch_bounds__(256) void k_leap_xs256_cols(uint64_t T, uint32_t *cols, DevTables tab)
{
    const uint32_t c = threadIdx.x;
    GenXS256 g;
#pragma unroll
    for (int i = 0; i < 8; ++i) g.v[i] = (uint32_t)(c / 32 == (uint32_t)i) << (c % 32);
    g.jump(T, tab);
#pragma unroll
    for (int i = 0; i < 8; ++i) cols[c * 8 + i] = g.v[i];
}

// Quad q = (2p + h) * 16 + v of the 4-bit table: words 4h .. 4h+3 of the XOR
// of columns 4p + k over the set bits k of v.
__global__ __launch_bounds__(256) void k_leap_xs256_table(const uint32_t *cols, uint4 *t4)
{
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    const uint32_t p = q >> 5, h = (q >> 4) & 1, v = q & 15;
    uint32_t r[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
        if ((v >> k) & 1)
            for (int w = 0; w < 4; ++w) r[w] ^= cols[(4 * p + k) * 8 + 4 * h + w];
    t4[q] = make_uint4(r[0], r[1], r[2], r[3]);
}

// Byte tables of the xorshift32 M^T: entry p * 256 + v is the XOR of columns
// 8p + k over the set bits k of v, so M^T y is the XOR of the four entries
// selected by the bytes of y.
__global__ __launch_bounds__(256) void k_leap_xs32_table(LeapArgs a, uint32_t *t8)
{
    const uint32_t e = blockIdx.x * 256 + threadIdx.x;
    const uint32_t p = e >> 8, v = e & 255;
    uint32_t r = 0;
    for (int k = 0; k < 8; ++k)
        if ((v >> k) & 1) r ^= a.xs32[8 * p + k];
    t8[e] = r;
}

__device__ __forceinline__ uint32_t xs32_bytes(const uint32_t *t8, uint32_t y)
{
    return xor3(t8[y & 255], t8[256 + ((y >> 8) & 255)], t8[512 + ((y >> 16) & 255)]) ^ t8[768 + (y >> 24)];
}

template <class G>
__device__ __forceinline__ void leap(G &g, const LeapArgs &a, uint32_t m16a, uint32_t m16b, const uint4 *t4,
                                     const uint32_t *t8)
{
    if constexpr (G::kId == G_MWC32) {
        uint64_t z = (uint64_t)g.c << 32 | g.x;
        z = mwc32_mulmod(z, a.mwc32_af, a.tab.mwc32_a, a.tab.mwc32_m);
        g.x = (uint32_t)z;
        g.c = (uint32_t)(z >> 32);
    } else if constexpr (G::kId == G_XS256) {
        gf2_apply256_t4(t4, g.v);
    } else if constexpr (G::kId == G_XS32) {
        g.y = xs32_bytes(t8, g.y);
    } else if constexpr (G::kId == G_MWC1616) {
        g.z = mwc16_mulmod(g.z, m16a, g.a1);
        g.w = mwc16_mulmod(g.w, m16b, g.a2);
    } else {
        g.z = mwc16_mulmod(g.z, m16a, g.a1);
        g.w = mwc16_mulmod(g.w, m16b, g.a2);
        g.jsr = xs32_bytes(t8, g.jsr);
        g.jcong = a.lcg_a * g.jcong + a.lcg_c;
    }
}

// Thread j: state_j -> one step (R_j) -> leaps of T steps (R_{j+T}, ...).
// The thread that emits R_{total-1} writes the final state.
template <class G, int DT>
__global__ __launch_bounds__(256) void k_leapfrog(LeapArgs a)
{
    constexpr bool kTable = G::kId == G_XS256;
    constexpr bool kBytes = G::kId == G_XS32 || G::kId == G_KISS;
    __shared__ uint4 s_t4[kTable ? 2048 : 1];
    __shared__ uint32_t s_t8[kBytes ? 1024 : 1];
    if constexpr (kTable) {
        stage_quads<256, 2048>(s_t4, (const uint4 *)((const char *)a.dconst + kConstBytes + kColBytes));
        __syncthreads();
    }
    if constexpr (kBytes) {
        const uint32_t *t8 = (const uint32_t *)((const char *)a.dconst + kConstBytes);
        uint32_t v[4];  // every load in flight before the LDS writes
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = t8[i * 256 + threadIdx.x];
#pragma unroll
        for (int i = 0; i < 4; ++i) s_t8[i * 256 + threadIdx.x] = v[i];
        __syncthreads();
    }
    const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.T) return;
    uint32_t m16a = 0, m16b = 0;
    if constexpr (G::kId == G_MWC1616 || G::kId == G_KISS) {
        m16a = a.dconst[0];
        m16b = a.dconst[1];
    }
    G g;
    g.load(a.ws, a.T, j);
    uint32_t u = g.next();
    for (uint64_t pos = j;;) {
        a.out[pos] = bits<DT>(u);
        if (pos == a.total - 1) g.store(a.final_state, 1, 0);
        pos += a.T;
        if (pos >= a.total) break;
        leap(g, a, m16a, m16b, s_t4, s_t8);
        u = g.last();
    }
}

template <class G>
int launch_leapfrog(int dt, const LeapArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.T + 255) / 256)), block(256);
    if (dt == RNG_F32) hipLaunchKernelGGL((k_leapfrog<G, RNG_DT_F32>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_leapfrog<G, RNG_DT_U32>), grid, block, 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Host-side T-step constants from the power tables.
void host_leap_constants(uint64_t T, LeapArgs &a)
{
    a.mwc32_af = mwc32_fold_const(T);
    xs32_lcg_jump(T, a.xs32, &a.lcg_a, &a.lcg_c);
}

}  // namespace

}  // namespace rngx

using namespace rngx;

extern "C" {

int rng_leapfrog_workspace_bytes(int g, uint64_t n_threads, uint64_t *bytes)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (!bytes) return fail(RNG_EINVAL, "bytes is NULL");
    if (n_threads > ((uint64_t)1 << 36)) return fail(RNG_ERANGE, "n_threads above 2^36");
    const bool bytes_t = g == RNG_XS32 || g == RNG_KISS;
    *bytes = align256(n_threads * gen_words(g) * 4) + kConstBytes + (g == RNG_XS256 ? kColBytes + kTableBytes : 0) +
             (bytes_t ? kByteTableBytes : 0);
    return RNG_OK;
}

int rng_generate_leapfrog(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads, int t,
                          void *d_out, uint32_t *d_final_state, void *d_workspace, uint64_t workspace_bytes,
                          void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!d_state_one || !d_final_state) return fail(RNG_EINVAL, "NULL state");
    hipStream_t st = (hipStream_t)stream;
    if (total == 0) {
        if (d_final_state == d_state_one) return RNG_OK;
        hipError_t e = hipMemcpyAsync(d_final_state, d_state_one, gen_words(g) * 4, hipMemcpyDeviceToDevice, st);
        return e == hipSuccess ? RNG_OK : hip_fail(e, "hipMemcpyAsync");
    }
    if (!d_out || !d_workspace) return fail(RNG_EINVAL, "NULL output or workspace");
    if (n_threads == 0) return fail(RNG_EINVAL, "n_threads is 0");
    if (((uintptr_t)d_out & 3) || ((uintptr_t)d_workspace & 255) || ((uintptr_t)d_state_one & 3) ||
        ((uintptr_t)d_final_state & 3))
        return fail(RNG_EINVAL, "misaligned pointer");
    if (int rc = check_sizes(1, total, 1)) return rc;
    const uint64_t T = n_threads < total ? n_threads : total;
    uint64_t need = 0;
    if (int rc = rng_leapfrog_workspace_bytes(g, T, &need)) return rc;
    if (workspace_bytes < need)
        return fail(RNG_ENOMEM, "workspace %llu bytes < %llu", (unsigned long long)workspace_bytes,
                    (unsigned long long)need);
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    uint32_t *ws = (uint32_t *)d_workspace;
    uint32_t *dconst = (uint32_t *)((char *)d_workspace + align256(T * gen_words(g) * 4));
    // thread j starts at state_j: a radix-16 tree, its first three levels (with
    // the copy of state_0) in one launch
    int rc = check_launch(dispatch_tree_head(g, d_state_one, ws, T, 1, tab, st), "leapfrog: tree head");
    for (uint32_t shift = kTreeHeadShift; !rc && ((uint64_t)1 << shift) < T; shift += 4)
        rc = check_launch(dispatch_tree_level(g, ws, T, shift, 1, tab, st), "leapfrog: tree level");
    if (rc) return rc;
    if (g == RNG_MWC1616 || g == RNG_KISS) {
        const uint32_t wa1 = g == RNG_MWC1616 ? 2 : 4;
        hipLaunchKernelGGL(k_leap_mwc16, dim3(1), dim3(64), 0, st, d_state_one, wa1, wa1 + 1, T, dconst, tab);
        if (hipGetLastError() != hipSuccess) return fail(RNG_EHIP, "leapfrog: MWC16 constants");
    }
    if (g == RNG_XS256) {
        uint32_t *cols = (uint32_t *)((char *)dconst + kConstBytes);
        uint4 *t4 = (uint4 *)((char *)cols + kColBytes);
        hipLaunchKernelGGL(k_leap_xs256_cols, dim3(1), dim3(256), 0, st, T, cols, tab);
        hipLaunchKernelGGL(k_leap_xs256_table, dim3(8), dim3(256), 0, st, (const uint32_t *)cols, t4);
        if (hipGetLastError() != hipSuccess) return fail(RNG_EHIP, "leapfrog: XS256 table");
    }
    LeapArgs a{};
    a.ws = ws;
    a.dconst = dconst;
    a.T = T;
    a.total = total;
    a.out = (uint32_t *)d_out;
    a.final_state = d_final_state;
    a.tab = tab;
    host_leap_constants(T, a);
    if (g == RNG_XS32 || g == RNG_KISS) {
        hipLaunchKernelGGL(k_leap_xs32_table, dim3(4), dim3(256), 0, st, a, (uint32_t *)((char *)dconst + kConstBytes));
        if (hipGetLastError() != hipSuccess) return fail(RNG_EHIP, "leapfrog: xorshift32 tables");
    }
    switch (g) {
    case RNG_MWC32: rc = launch_leapfrog<GenMWC32>(t, a, st); break;
    case RNG_XS256: rc = launch_leapfrog<GenXS256>(t, a, st); break;
    case RNG_XS32: rc = launch_leapfrog<GenXS32>(t, a, st); break;
    case RNG_KISS: rc = launch_leapfrog<GenKISS>(t, a, st); break;
    case RNG_MWC1616: rc = launch_leapfrog<GenMWC1616>(t, a, st); break;
    }
    return check_launch(rc, "rng_generate_leapfrog");
}

}  // extern "C"
