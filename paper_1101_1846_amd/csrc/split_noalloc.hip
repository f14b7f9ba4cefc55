// split_noalloc.hip -- sequence splitting (Sec. II.A.4) for callers that cannot
// allocate: the per-thread start states live in a file-scope device array
// instead of a caller workspace, so the entry point makes no hipMalloc,
// hipFree or other allocating call.  Each device that loads the library holds
// its own copy of the array until the process ends; its address on a device
// is looked up once, by rng_init() with that device current.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rng.h"
#include "rng_abi_internal.hpp"

namespace rngx {

namespace {

constexpr uint64_t kScratchBytes = RNG_SPLIT_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// Thread start states of rng_generate_split_noalloc ([W][T] words).  In host
// code this name is a stand-in, not a device address: kernels get the
// address from hipGetSymbolAddress (g_scratch below).
static __device__ __align__(256) uint32_t scratch[kScratchBytes / 4];

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // the array's address on each device, once looked up

}  // namespace

int scratch_init_current_device()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RNG_ENODEV, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev]) return RNG_OK;
    void *p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
        return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255)) return fail(RNG_EHIP, "scratch array address %p not 256-byte aligned", p);
    g_scratch[dev] = p;
    return RNG_OK;
}

}  // namespace rngx

using namespace rngx;

extern "C" int rng_generate_split_noalloc(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads,
                                          int t, void *d_out, uint32_t *d_final_state, void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!d_state_one || !d_final_state) return fail(RNG_EINVAL, "NULL state");
    if (total == 0) {
        // nothing generated: the final state is the initial one (an asynchronous
        // device copy, no allocation)
        if (d_final_state == d_state_one) return RNG_OK;
        hipError_t e = hipMemcpyAsync(d_final_state, d_state_one, gen_words(g) * 4, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream);
        return e == hipSuccess ? RNG_OK : hip_fail(e, "hipMemcpyAsync");
    }
    if (int rc = split_args_check(total, n_threads, d_out, d_state_one, d_final_state)) return rc;
    uint64_t need;
    if (int rc = split_scratch_bytes(g, total, n_threads, &need)) return rc;
    if (need > kScratchBytes)
        return fail(RNG_ERANGE, "split needs %llu bytes of thread states; the allocation-free form holds %llu",
                    (unsigned long long)need, (unsigned long long)kScratchBytes);
    DevTables tab;
    if (int rc = device_tables_if_ready(&tab)) return rc;  // never builds (allocates) tables here
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ws = g_scratch[dev];
    }
    if (!ws) return fail(RNG_EINVAL, "device %d: call rng_init() on it first", dev);
    return split_run(g, d_state_one, total, n_threads, t, d_out, d_final_state, (uint32_t *)ws, kScratchBytes, tab,
                     (hipStream_t)stream);
}
