// rng_calib.hip -- device calibration of the integer VALU rate.  The paper
// derived its integer-operation peak from the FP rate (one third of the
// FLOP figure, Sec. V) and measured only its memory bandwidth; here the
// integer rate is measured: independent accumulator chains per lane keep
// every SIMD busy with one opcode class.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_abi_internal.hpp"
#include "rng_kernels.hpp"

namespace rngx {

// OP 0: v_add_u32 + v_xor_b32 (2 ops per chain step); 1: v_mad_u32_u24; 2: v_mul_lo_u32.
template <int OP>
__global__ __launch_bounds__(256) void k_valu(uint32_t *out, uint32_t iters, uint32_t b, uint32_t c)
{
    uint32_t a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 8 + i + blockIdx.x;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if constexpr (OP == 0) a[i] = (a[i] + b) ^ c;
            else if constexpr (OP == 1) a[i] = __umul24(a[i], b) + c;
            else a[i] = a[i] * b;
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r ^= a[i];
    if (r == 0x9E3779B9u) out[blockIdx.x * 256 + threadIdx.x] = r;  // keeps the chains alive
}

// OP 3: the fused consumer's own loop body (a KISS number pair and the exact
// quarter-circle test, eight numbers per stream and iteration, as
// k_fused_pi runs it) on NS independent streams per lane, interleaved, so
// that an instruction need not wait for the previous one's result: the rate
// the VALU sustains for that instruction mix.  In lane-samples per second,
// the fastest of NS = 1, 2, 4, 8.
template <int NS>
__global__ __launch_bounds__(256) void k_valu_fused(uint32_t *out, uint32_t iters, uint32_t seed)
{
    rng_inline::KISS g[NS];
    const uint32_t id = blockIdx.x * 256 + threadIdx.x;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        g[s].z = seed ^ (id * 2654435761u + s) | 1u;
        g[s].w = (id + 77u * s) | 1u;
        g[s].jsr = id * 40503u + s + 1u;
        g[s].jcong = id + s;
        g[s].a1 = 18000u + 2u * s;  // any 16-bit multipliers: only the instruction mix matters
        g[s].a2 = 30903u + 2u * s;
    }
    uint32_t cnt = 0;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint32_t x = g[s].next() >> 8, y = g[s].next() >> 8;
                cnt += in_quarter_circle(x, y);
            }
        }
    }
    if (cnt == 0x9E3779B9u) out[id] = cnt;  // keeps the chains alive
}


}  // namespace rngx

using namespace rngx;

// One timed measurement: 1 warm-up and 3 timed launches; ns = independent
// streams per lane of the fused-mix loop (op 3).
static int calib_once(int op, int ns, double *lane_ops_per_s, void *stream)
{
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    const unsigned blocks = (unsigned)cus * 16;  // 16 workgroups of 256 lanes per CU (several rounds of 8 waves per SIMD)
    const uint32_t iters = 4096;
    hipStream_t st = (hipStream_t)stream;
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipMalloc((void **)&out, (size_t)blocks * 256 * 4)) != hipSuccess) return hip_fail(e, "hipMalloc");
    int rc = RNG_OK;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) rc = hip_fail(e, "event");
    auto launch = [&]() {
        if (op == 0) hipLaunchKernelGGL(k_valu<0>, dim3(blocks), dim3(256), 0, st, out, iters, 0x9E3779B9u, 0x7F4A7C15u);
        else if (op == 1) hipLaunchKernelGGL(k_valu<1>, dim3(blocks), dim3(256), 0, st, out, iters, 69069u, 1234567u);
        else if (op == 2) hipLaunchKernelGGL(k_valu<2>, dim3(blocks), dim3(256), 0, st, out, iters, 69069u, 0u);
        else if (ns == 1) hipLaunchKernelGGL(k_valu_fused<1>, dim3(blocks), dim3(256), 0, st, out, iters / 64, 0x2545F491u);
        else if (ns == 2) hipLaunchKernelGGL(k_valu_fused<2>, dim3(blocks), dim3(256), 0, st, out, iters / 64, 0x2545F491u);
        else if (ns == 4) hipLaunchKernelGGL(k_valu_fused<4>, dim3(blocks), dim3(256), 0, st, out, iters / 64, 0x2545F491u);
        else hipLaunchKernelGGL(k_valu_fused<8>, dim3(blocks), dim3(256), 0, st, out, iters / 64, 0x2545F491u);
        return hipGetLastError();
    };
    if (!rc && (e = launch()) != hipSuccess) rc = hip_fail(e, "launch");
    if (!rc) {
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 3 && !rc; ++r)
            if ((e = launch()) != hipSuccess) rc = hip_fail(e, "launch");
        (void)hipEventRecord(e1, st);
    }
    float ms = 0;
    if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
    if (!rc) (void)hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc) return rc;
    if (op == 3) {  // lane-samples: 8 numbers per stream and iteration
        *lane_ops_per_s = (double)blocks * 256 * (iters / 64) * 8 * ns * 3 / (ms * 1e-3);
        return RNG_OK;
    }
    const double ops_per_step = op == 0 ? 2.0 : 1.0;
    *lane_ops_per_s = (double)blocks * 256 * iters * 8 * ops_per_step * 3 / (ms * 1e-3);
    return RNG_OK;
}

extern "C" int rng_calibrate_valu(int op, double *lane_ops_per_s, void *stream)
{
    if (!lane_ops_per_s || op < 0 || op > 3) return fail(RNG_EINVAL, "bad argument");
    if (op < 3) return calib_once(op, 0, lane_ops_per_s, stream);
    // the fused mix: the fastest of 1, 2, 4 and 8 independent streams per lane
    double best = 0;
    for (int ns : {1, 2, 4, 8}) {
        double r = 0;
        if (int rc = calib_once(3, ns, &r, stream)) return rc;
        best = r > best ? r : best;
    }
    *lane_ops_per_s = best;
    return RNG_OK;
}
