// rng_abi.cpp -- the C ABI declared in include/rng.h: argument checks,
// per-device tables, launch-shape selection, and the call sequences of the
// multi-kernel operations (sequence splitting).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "host_math.hpp"
#include "rng.h"
#include "rng_abi_internal.hpp"
#include "rng_internal.hpp"

namespace rngx {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(RNG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- tables
namespace {
struct DevEntry {
    bool ready = false;
    void *blob = nullptr;
    DevTables tab{};
};
std::mutex g_mu;
DevEntry g_dev[kMaxDevices];
}  // namespace

int device_tables(DevTables *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RNG_ENODEV, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    DevEntry &d = g_dev[dev];
    if (!d.ready) {
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(RNG_ENODEV, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
        const HostTables &H = host_tables();
        const size_t o_t392 = 0, n_t392 = sizeof(H.t392);
        const size_t o_m32 = 1024, n_m32 = sizeof(H.mwc32_pow_fold);
        const size_t o_lcg = o_m32 + 1024, n_lcg = sizeof(H.lcg_pow);
        const size_t o_x32 = o_lcg + 1024, n_x32 = sizeof(H.xs32_pow);
        const size_t o_m16 = o_x32 + n_x32, n_m16 = sizeof(H.mwc16_pow_fold);
        const size_t o_x256 = (o_m16 + n_m16 + 255) & ~(size_t)255;
        const size_t n_x256 = H.xs256_t4.size() * sizeof(uint32_t);
        const size_t o_x256w = o_x256 + n_x256, n_x256w = H.xs256_t4w.size() * sizeof(uint32_t);
        const size_t total = o_x256w + n_x256w;
        std::string host(total, '\0');
        std::memcpy(&host[o_t392], H.t392, n_t392);
        std::memcpy(&host[o_m32], H.mwc32_pow_fold, n_m32);
        std::memcpy(&host[o_lcg], H.lcg_pow, n_lcg);
        std::memcpy(&host[o_x32], H.xs32_pow, n_x32);
        std::memcpy(&host[o_m16], H.mwc16_pow_fold, n_m16);
        std::memcpy(&host[o_x256], H.xs256_t4.data(), n_x256);
        std::memcpy(&host[o_x256w], H.xs256_t4w.data(), n_x256w);
        void *blob = nullptr;
        if ((e = hipMalloc(&blob, total)) != hipSuccess) return hip_fail(e, "hipMalloc(tables)");
        if ((e = hipMemcpy(blob, host.data(), total, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(blob);
            return hip_fail(e, "hipMemcpy(tables)");
        }
        char *b = (char *)blob;
        d.tab.t392 = (const uint16_t *)(b + o_t392);
        d.tab.mwc32_pow = (const uint64_t *)(b + o_m32);
        d.tab.lcg_pow = (const uint32_t *)(b + o_lcg);
        d.tab.xs32_pow = (const uint32_t *)(b + o_x32);
        d.tab.mwc16_pow = (const uint32_t *)(b + o_m16);
        d.tab.xs256_t4 = (const uint4 *)(b + o_x256);
        d.tab.xs256_t4w = (const uint4 *)(b + o_x256w);
        d.tab.mwc32_a = H.mwc32_a;
        d.tab.mwc32_m = H.mwc32_m;
        d.blob = blob;
        d.ready = true;
    }
    *out = d.tab;
    return RNG_OK;
}

int device_tables_if_ready(DevTables *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RNG_ENODEV, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev[dev].ready) return fail(RNG_EINVAL, "device %d has no tables yet: call rng_init() on it first", dev);
    *out = g_dev[dev].tab;
    return RNG_OK;
}

int shutdown_tables()
{
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int i = 0; i < kMaxDevices; ++i) {
        if (!g_dev[i].ready) continue;
        (void)hipSetDevice(i);
        (void)hipFree(g_dev[i].blob);
        g_dev[i] = DevEntry();
    }
    (void)hipSetDevice(cur);
    return RNG_OK;
}

// ---------------------------------------------------------------- shapes
int gen_words(int g)
{
    switch (g) {
    case RNG_MWC32: return 2;
    case RNG_XS256: return 8;
    case RNG_XS32: return 1;
    case RNG_KISS: return 6;
    case RNG_MWC1616: return 4;
    }
    return 0;
}

static std::mutex g_shape_mu;
static Shape g_shape[2][6][2] = {};  // [rows written as runs][generator][dtype]

// Rows of 4 or 8 KiB (n = 1024, 2048) over whole groups of 64 runs are
// written as 16 KiB runs of 4 or 2 adjacent rows per lane (on workgroups of
// up to 256 lanes, when the launch is resident): streams per run, else 0.
uint32_t run_rows(uint64_t S, uint64_t N)
{
    if (N != 1024 && N != 2048) return 0;
    const uint32_t seg = (uint32_t)(4096 / N);
    return S && S % (64 * (uint64_t)seg) == 0 ? seg : 0;
}

// Untuned defaults: 256 lanes, unroll 8 (measured on 1 KiB rows), and for
// runs 64 lanes, unroll 16 (within about 1 % of the fastest shape for every
// generator at 2^20 x 1024; 256 x 8 ran 15 % slower for XS256 and KISS).
Shape tuned_shape(int g, int dt, bool runs)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    Shape s = g_shape[runs][g][dt];
    if (!s.wg) s = runs ? Shape{64, 16} : Shape{256, 8};
    return s;
}

// XS256 rows of an odd number of 4 KiB (N = 1024 (2i + 1)) run as four
// jumped chunks on 512- and 1024-lane workgroups: chunk c starts c N bytes
// into its row, so the four chunks of a row cover four column slots of 1 KiB.
// For an even number the chunk starts share at most two slots (N = 2048) or
// one (N = 4096 m), and the plain order is faster.
bool xs256_chunked_rows(uint64_t N) { return N % 1024 == 0 && (N / 1024) % 2 == 1; }

// The shape rng_generate uses for S streams of n samples: the one tuned for
// runs when the rows are written as runs, else the other one, except that
// XS256 rows taking the four-chunk path get 512-lane workgroups (the tuned
// shape is measured on other row lengths).
Shape row_shape(int g, int dt, uint64_t S, uint64_t n)
{
    if (run_rows(S, n)) return tuned_shape(g, dt, true);
    Shape s = tuned_shape(g, dt, false);
    if (g == RNG_XS256 && xs256_chunked_rows(n) && s.wg < 512) s.wg = 512;
    return s;
}

void set_tuned_shape(int g, int dt, bool runs, Shape s)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shape[runs][g][dt] = s;
}

bool valid_shape(uint32_t wg, uint32_t unroll)
{
    return (wg == 64 || wg == 128 || wg == 256 || wg == 512 || wg == 1024) &&
           (unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8 || unroll == 16);
}

// Smallest chunk worth a jump: the jump costs a few modular multiplies for
// MWC/LCG words and 32x32 mat-vecs for xorshift32, but 256x256 mat-vecs for
// the r = 8 XorShift.
static uint64_t min_chunk(int g)
{
    switch (g) {
    case RNG_MWC32: return 64;
    case RNG_XS32: return 128;
    case RNG_MWC1616: return 128;
    case RNG_KISS: return 256;
    case RNG_XS256: return 4096;
    }
    return 1u << 30;
}

// Split each stream into P chunks when there are too few streams to fill the
// chip (256 CUs x 4 SIMDs; aim for >= 2 waves per SIMD).
// Fewer streams than a wave has lanes: one lane per chunk, about 2^17 lanes,
// chunks a multiple of 64 samples and at least the generator's minimum.
void lane_chunks(int g, uint64_t S, uint64_t N, uint64_t *C, uint32_t *P)
{
    const uint64_t p = ((uint64_t)1 << 17) / S;
    uint64_t c = std::max<uint64_t>(min_chunk(g), (N + p - 1) / p);
    c = (c + 63) / 64 * 64;
    *C = c;
    *P = (uint32_t)((N + c - 1) / c);
}

// Lanes that chunked bulk generation aims for: the waves the device holds at
// once with 128-deep LDS tiles (4 per CU, 256 CUs) times 64.  Measured
// against 2^17 and 2^15 over 64..65536 streams: 2^16 is 15-40 % faster than
// 2^17 for MWC32 and KISS and equal for XS256; 2^15 slows XS256 and KISS.
constexpr uint64_t kGenLanes = (uint64_t)1 << 16;

void choose_chunks(int g, uint64_t S, uint64_t N, uint64_t align, uint64_t *C, uint32_t *P, uint64_t target_lanes)
{
    uint64_t p = 1;
    while (S * p * 2 <= target_lanes && N / (p * 2) >= min_chunk(g)) p *= 2;
    if (p == 1) {
        *C = N;
        *P = 1;
        return;
    }
    uint64_t c = (N + p - 1) / p;
    c = (c + align - 1) / align * align;
    *C = c;
    *P = (uint32_t)((N + c - 1) / c);
}

int dispatch_generate(int g, int dt, const GenArgs &a, int wg, int unroll, bool staged, hipStream_t st)
{
    switch (g) {
    case RNG_MWC32: return launch_generate_t<GenMWC32>(dt, a, wg, unroll, staged, st);
    case RNG_XS256: return launch_generate_t<GenXS256>(dt, a, wg, unroll, staged, st);
    case RNG_XS32: return launch_generate_t<GenXS32>(dt, a, wg, unroll, staged, st);
    case RNG_KISS: return launch_generate_t<GenKISS>(dt, a, wg, unroll, staged, st);
    case RNG_MWC1616: return launch_generate_t<GenMWC1616>(dt, a, wg, unroll, staged, st);
    }
    return -2;
}

#define RNGX_GEN_SWITCH(g, call)                                        \
    switch (g) {                                                        \
    case RNG_MWC32: { using G = GenMWC32; return call; }                \
    case RNG_XS256: { using G = GenXS256; return call; }                \
    case RNG_XS32: { using G = GenXS32; return call; }                  \
    case RNG_KISS: { using G = GenKISS; return call; }                  \
    case RNG_MWC1616: { using G = GenMWC1616; return call; }            \
    }                                                                   \
    return -2;

int dispatch_seed(int g, uint64_t seed, uint64_t first, uint64_t S, uint32_t *st, const DevTables &tab,
                  hipStream_t s)
{
    RNGX_GEN_SWITCH(g, launch_seed_t<G>(seed, first, S, st, tab, s))
}

int dispatch_tree_head(int g, const uint32_t *st0, uint32_t *ws, uint64_t T, uint64_t unit, const DevTables &tab,
                       hipStream_t s)
{
    RNGX_GEN_SWITCH(g, launch_tree_head_t<G>(st0, ws, T, unit, tab, s))
}

int dispatch_tree_level(int g, uint32_t *ws, uint64_t T, uint32_t shift, uint64_t unit, const DevTables &tab,
                        hipStream_t s)
{
    RNGX_GEN_SWITCH(g, launch_tree_level_t<G>(ws, T, shift, unit, tab, s))
}

int dispatch_state_copy(int g, const uint32_t *src, uint64_t ss, uint64_t si, uint32_t *dst, uint64_t ds,
                        uint64_t di, hipStream_t s)
{
    RNGX_GEN_SWITCH(g, launch_state_copy_t<G>(src, ss, si, dst, ds, di, s))
}

int dispatch_fused(int g, const FusedArgs &a, hipStream_t s)
{
    RNGX_GEN_SWITCH(g, launch_fused_pi_t<G>(a, s))
}

int check_launch(int rc, const char *what)
{
    if (rc == 0) return RNG_OK;
    if (rc == -2) return fail(RNG_EINVAL, "%s: unsupported launch shape", what);
    hipError_t e = hipGetLastError();
    return fail(RNG_EHIP, "%s: launch failed: %s", what, hipGetErrorString(e));
}

static bool mul_overflows(uint64_t a, uint64_t b, uint64_t *r)
{
    return __builtin_mul_overflow(a, b, r);
}

// Jump constants of the rotated tile order (d N / 4 samples, d = 0..3).  The
// xorshift32 columns cost about 12 us of host time per distance, so the last
// few row lengths are cached.  MWC1616 needs none from the host: the MWC16
// words' constants depend on the stream's multiplier and are built in LDS.
static void rot_constants(int g, uint64_t N, GenArgs &a)
{
    if (g == RNG_MWC32) {
        for (int d = 0; d < 4; ++d) a.rot_mwc32[d] = mwc32_fold_const((uint64_t)d * (N / 4));
        return;
    }
    if (g == RNG_MWC1616) return;
    struct Entry {
        uint64_t N = 0;
        uint32_t cols[4][32];
        uint32_t lcg[4][2];
    };
    static std::mutex mu;
    static Entry cache[8];
    static unsigned next = 0;
    std::lock_guard<std::mutex> lk(mu);
    const Entry *hit = nullptr;
    for (const Entry &e : cache)
        if (e.N == N) hit = &e;
    if (!hit) {
        Entry &e = cache[next++ % 8];
        for (int d = 0; d < 4; ++d) xs32_lcg_jump((uint64_t)d * (N / 4), e.cols[d], &e.lcg[d][0], &e.lcg[d][1]);
        e.N = N;
        hit = &e;
    }
    std::memcpy(a.rot_xs32, hit->cols, sizeof(hit->cols));
    std::memcpy(a.rot_lcg, hit->lcg, sizeof(hit->lcg));
}

// Shared by rng_generate and the split path: one generate launch over
// S streams whose states live at stride ld.
int generate_impl(int g, int dt, uint32_t *d_state, uint64_t ld, uint64_t S, uint64_t N, void *d_out,
                  Shape shape, bool staged, hipStream_t st)
{
    if (S == 0 || N == 0) return RNG_OK;
    DevTables tab;
    int rc = device_tables(&tab);
    if (rc) return rc;
    GenArgs a{};
    a.state = d_state;
    a.ld = ld;
    a.S = S;
    a.N = N;
    a.out = d_out;
    a.vec4 = (N % 4 == 0) && (((uintptr_t)d_out & 15) == 0);
    a.nt = 0;  // plain stores: the streaming hint measured slower for these writes
    a.tab = tab;
    if (staged && S < 64) {
        uint64_t c;
        uint32_t P;
        lane_chunks(g, S, N, &c, &P);
        if (P > 1) return check_launch(generate_few(g, dt, d_state, ld, S, N, c, P, d_out, tab, st), "rng_generate");
    }
    choose_chunks(g, S, N, kGenTile, &a.C, &a.P, kGenLanes);
    // XS256 rows of an odd number of 4 KiB (no rotated order: a row would need
    // a 256 x 256 jump inside the write stream): four chunks per stream, each
    // jumped once at its start, before any store (one table product per
    // nonzero hexadecimal digit of j N / 4: one for N = 1024), so that the
    // waves of a group write four different column slots at once.  Only with
    // workgroups of 8+ waves: they hold all four chunks of their groups and
    // write the states back themselves, and their 32-sample tiles measured
    // faster here than 4-wave workgroups with 128-sample tiles (XS256 2^20 x
    // 1024: 832-867 us at 512 lanes against 1090-1127 at 256 and 883-949 for
    // the plain order).
    // rows of 4 or 8 KiB on workgroups of up to 256 lanes: runs of 4 or 2
    // adjacent rows per lane, 16 KiB each (when the launch is resident; else
    // the orders below)
    if (staged && a.P == 1 && a.vec4 && shape.wg <= 256) a.seg = run_rows(S, N);
    if (g == RNG_XS256 && staged && a.P == 1 && a.vec4 && S % 64 == 0 && xs256_chunked_rows(N) && shape.wg >= 512) {
        a.C = N / kXs256RowChunks;
        a.P = kXs256RowChunks;
    }
    // rows of whole 4 KiB multiples on the resident schedule: rotated tile order
    if (g != RNG_XS256 && staged && a.P == 1 && a.vec4 && S % 64 == 0 && N % 1024 == 0) {
        a.rot = 1;
        rot_constants(g, N, a);
    }
    rc = dispatch_generate(g, dt, a, (int)shape.wg, (int)shape.unroll, staged, st);
    if (rc != kStatesNotWritten) return check_launch(rc, "rng_generate");
    // chunks of one stream in several workgroups: the states advance after
    // every chunk has read them
    return check_launch(dispatch_skip(g, d_state, ld, S, N, tab, st), "rng_generate: state");
}

int check_gen(int g) { return gen_words(g) ? RNG_OK : fail(RNG_EINVAL, "unknown generator %d", g); }

int check_sizes(uint64_t S, uint64_t N, uint64_t words)
{
    uint64_t t;
    if (mul_overflows(S, N, &t) || mul_overflows(t, 4, &t))
        return fail(RNG_ERANGE, "n_streams * n * 4 overflows 64 bits");
    if (mul_overflows(S, words, &t) || mul_overflows(t, 4, &t))
        return fail(RNG_ERANGE, "state size overflows 64 bits");
    // keeps every grid below 2^31 workgroups (64-lane groups, <= 2^30 waves)
    if (S > ((uint64_t)1 << 36)) return fail(RNG_ERANGE, "n_streams above 2^36");
    return RNG_OK;
}

// Sequence splitting after the argument checks of the entry points: thread
// states in ws ([W][T] words, ws_bytes available), a radix-16 tree of jumps,
// then the generation launch(es) and the final state.  Launches only.
int split_args_check(uint64_t total, uint64_t n_threads, const void *d_out, const uint32_t *d_state_one,
                     const uint32_t *d_final_state)
{
    if (!d_out) return fail(RNG_EINVAL, "NULL output");
    if (n_threads == 0) return fail(RNG_EINVAL, "n_threads is 0");
    if (((uintptr_t)d_out & 3) || ((uintptr_t)d_state_one & 3) || ((uintptr_t)d_final_state & 3))
        return fail(RNG_EINVAL, "misaligned pointer");
    return check_sizes(1, total, 1);
}

int split_run(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads, int t, void *d_out,
              uint32_t *d_final_state, uint32_t *ws, uint64_t ws_bytes, const DevTables &tab, hipStream_t st)
{
    const uint64_t C = (total + n_threads - 1) / n_threads;
    const uint64_t T = (total + C - 1) / C;  // threads with work
    uint64_t need;
    if (int rc = split_scratch_bytes(g, total, n_threads, &need)) return rc;
    if (ws_bytes < need)
        return fail(RNG_ENOMEM, "workspace %llu bytes < %llu", (unsigned long long)ws_bytes, (unsigned long long)need);
    // radix-16 tree: level l starts threads [16^l, 16^(l+1)) from threads below 16^l;
    // the start state's copy and levels 0 .. 2 in one launch
    uint64_t far;
    if (mul_overflows(C, T, &far)) return fail(RNG_ERANGE, "jump distance overflows");
    int rc = check_launch(dispatch_tree_head(g, d_state_one, ws, T, C, tab, st), "split: tree head");
    if (rc) return rc;
    for (uint32_t shift = kTreeHeadShift; ((uint64_t)1 << shift) < T; shift += 4) {
        rc = check_launch(dispatch_tree_level(g, ws, T, shift, C, tab, st), "split: tree level");
        if (rc) return rc;
    }
    const uint64_t rem = total - (T - 1) * C;  // samples of the last thread
    const uint64_t full = rem == C ? T : T - 1;
    Shape shape = row_shape(g, t, full / 64 * 64, C);
    // whole 64-thread groups in one launch (the resident schedule needs them),
    // the rest of the full threads in a second
    const uint64_t full64 = full / 64 * 64;
    if (full64) {
        rc = generate_impl(g, t, ws, T, full64, C, d_out, shape, true, st);
        if (rc) return rc;
    }
    if (full > full64) {
        rc = generate_impl(g, t, ws + full64, T, full - full64, C, (uint32_t *)d_out + full64 * C, shape, true, st);
        if (rc) return rc;
    }
    if (full < T) {
        rc = generate_impl(g, t, ws + (T - 1), T, 1, rem, (uint32_t *)d_out + (T - 1) * C, shape, true, st);
        if (rc) return rc;
    }
    return check_launch(dispatch_state_copy(g, ws, T, T - 1, d_final_state, 1, 0, st), "split: final");
}

// Workspace bytes a split of `total` samples over n_threads threads uses:
// one state per thread with work.
int split_scratch_bytes(int g, uint64_t total, uint64_t n_threads, uint64_t *bytes)
{
    if (n_threads == 0) return fail(RNG_EINVAL, "n_threads is 0");
    const uint64_t C = (total + n_threads - 1) / n_threads;
    const uint64_t T = C ? (total + C - 1) / C : 0;
    if (mul_overflows(T, (uint64_t)gen_words(g) * 4, bytes)) return fail(RNG_ERANGE, "n_threads too large");
    return RNG_OK;
}

}  // namespace rngx

using namespace rngx;

// ====================================================================== ABI
extern "C" {

const char *rng_strerror(int code)
{
    switch (code) {
    case RNG_OK: return "success";
    case RNG_EINVAL: return "invalid argument";
    case RNG_ERANGE: return "size out of range";
    case RNG_ENOMEM: return "insufficient memory or workspace";
    case RNG_EHIP: return "HIP runtime error";
    case RNG_ENODEV: return "no usable gfx950 device";
    case RNG_EAGAIN: return "not ready";
    }
    return "unknown error";
}

const char *rng_last_error(void) { return g_last_error.c_str(); }

int rng_init(void)
{
    DevTables t;
    if (int rc = device_tables(&t)) return rc;
    return scratch_init_current_device();
}

int rng_shutdown(void) { return shutdown_tables(); }

int rng_state_words(int g, uint32_t *words)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (!words) return fail(RNG_EINVAL, "words is NULL");
    *words = (uint32_t)gen_words(g);
    return RNG_OK;
}

int rng_mwc32_multiplier(uint32_t *a)
{
    if (!a) return fail(RNG_EINVAL, "a is NULL");
    *a = mwc32_multiplier();
    return RNG_OK;
}

int rng_mwc16_multipliers(uint16_t *h_out, uint32_t cap, uint32_t *count)
{
    if (!count) return fail(RNG_EINVAL, "count is NULL");
    const auto &t = mwc16_multipliers();
    *count = (uint32_t)t.size();
    if (h_out) {
        if (cap < t.size()) return fail(RNG_ERANGE, "cap %u < %zu", cap, t.size());
        std::memcpy(h_out, t.data(), t.size() * sizeof(uint16_t));
    }
    return RNG_OK;
}

int rng_seed(int g, uint64_t seed, uint64_t first_stream, uint64_t n_streams, uint32_t *d_state,
             void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (n_streams == 0) return RNG_OK;
    if (!d_state) return fail(RNG_EINVAL, "d_state is NULL");
    if ((uintptr_t)d_state & 3) return fail(RNG_EINVAL, "d_state not 4-byte aligned");
    if (int rc = check_sizes(n_streams, 1, gen_words(g))) return rc;
    uint64_t end;
    if (__builtin_add_overflow(first_stream, n_streams, &end) ||
        mul_overflows(end, 4, &end))
        return fail(RNG_ERANGE, "first_stream + n_streams too large");
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    return check_launch(dispatch_seed(g, seed, first_stream, n_streams, d_state, tab, (hipStream_t)stream),
                        "rng_seed");
}

int rng_generate_ex(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t, void *d_out,
                    uint32_t wg, uint32_t unroll, void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!valid_shape(wg, unroll)) return fail(RNG_EINVAL, "launch shape wg=%u unroll=%u", wg, unroll);
    if (n_streams == 0 || n == 0) return RNG_OK;
    if (!d_state || !d_out) return fail(RNG_EINVAL, "NULL state or output");
    if (((uintptr_t)d_state & 3) || ((uintptr_t)d_out & 3))
        return fail(RNG_EINVAL, "state and output must be 4-byte aligned");
    if (int rc = check_sizes(n_streams, n, gen_words(g))) return rc;
    return generate_impl(g, t, d_state, n_streams, n_streams, n, d_out, Shape{wg, unroll}, true,
                         (hipStream_t)stream);
}

int rng_generate(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t, void *d_out, void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    Shape s = row_shape(g, t, n_streams, n);
    return rng_generate_ex(g, d_state, n_streams, n, t, d_out, s.wg, s.unroll, stream);
}

int rng_skip(int g, uint32_t *d_state, uint64_t n_streams, uint64_t k, void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (n_streams == 0 || k == 0) return RNG_OK;
    if (!d_state) return fail(RNG_EINVAL, "d_state is NULL");
    if ((uintptr_t)d_state & 3) return fail(RNG_EINVAL, "d_state not 4-byte aligned");
    if (int rc = check_sizes(n_streams, 1, gen_words(g))) return rc;
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    return check_launch(dispatch_skip(g, d_state, n_streams, n_streams, k, tab, (hipStream_t)stream), "rng_skip");
}

int rng_split_workspace_bytes(int g, uint64_t n_threads, uint64_t *bytes)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (!bytes) return fail(RNG_EINVAL, "bytes is NULL");
    uint64_t b;
    if (mul_overflows(n_threads, (uint64_t)gen_words(g) * 4, &b)) return fail(RNG_ERANGE, "n_threads too large");
    *bytes = b;
    return RNG_OK;
}

int rng_generate_split(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads, int t,
                       void *d_out, uint32_t *d_final_state, void *d_workspace, uint64_t workspace_bytes,
                       void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!d_state_one || !d_final_state) return fail(RNG_EINVAL, "NULL state");
    if (total == 0) {
        // nothing generated: the final state is the initial one
        if (d_final_state == d_state_one) return RNG_OK;
        hipError_t e = hipMemcpyAsync(d_final_state, d_state_one, gen_words(g) * 4, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream);
        return e == hipSuccess ? RNG_OK : hip_fail(e, "hipMemcpyAsync");
    }
    if (int rc = split_args_check(total, n_threads, d_out, d_state_one, d_final_state)) return rc;
    if (!d_workspace) return fail(RNG_EINVAL, "NULL workspace");
    if ((uintptr_t)d_workspace & 255) return fail(RNG_EINVAL, "misaligned pointer");
    uint64_t need;
    if (int rc = split_scratch_bytes(g, total, n_threads, &need)) return rc;
    if (workspace_bytes < need)
        return fail(RNG_ENOMEM, "workspace %llu bytes < %llu", (unsigned long long)workspace_bytes,
                    (unsigned long long)need);
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    return split_run(g, d_state_one, total, n_threads, t, d_out, d_final_state, (uint32_t *)d_workspace,
                     workspace_bytes, tab, (hipStream_t)stream);
}

int rng_fused_pi(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, uint64_t *d_count, void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (n_streams == 0 || n == 0) return RNG_OK;
    if (!d_state || !d_count) return fail(RNG_EINVAL, "NULL state or count");
    if (((uintptr_t)d_state & 3) || ((uintptr_t)d_count & 7)) return fail(RNG_EINVAL, "misaligned pointer");
    if (int rc = check_sizes(n_streams, n, gen_words(g))) return rc;
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    FusedArgs a{};
    a.state = d_state;
    a.ld = n_streams;
    a.S = n_streams;
    a.N = n;
    a.count = d_count;
    a.tab = tab;
    if (n_streams < 64) {
        lane_chunks(g, n_streams, n, &a.C, &a.P);
        a.lanes = a.P > 1;
    } else {
        choose_chunks(g, n_streams, n, 8, &a.C, &a.P, (uint64_t)1 << 17);
    }
    if (a.P == 1) a.C = n;
    if (int rc = check_launch(dispatch_fused(g, a, (hipStream_t)stream), "rng_fused_pi")) return rc;
    if (a.P == 1) return RNG_OK;
    return check_launch(dispatch_skip(g, d_state, n_streams, n_streams, n, tab, (hipStream_t)stream),
                        "rng_fused_pi: state");
}

}  // extern "C"
