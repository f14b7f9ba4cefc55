// rng_tune.cpp -- launch-shape autotuner for the store-mode generator.
// The paper picked block sizes with an occupancy calculator and unrolled its
// main loop with a pragma (Sec. III.A, III.B); here every (workgroup size,
// unroll) pair is timed on the device and the fastest is kept per
// (generator, dtype) and row class: rows written as 16 KiB runs (4 or 8 KiB
// rows) or any other rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "rng.h"
#include "rng_abi_internal.hpp"

using namespace rngx;

extern "C" {

int rng_set_shape(int g, int t, uint32_t wg, uint32_t unroll)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!valid_shape(wg, unroll)) return fail(RNG_EINVAL, "launch shape wg=%u unroll=%u", wg, unroll);
    set_tuned_shape(g, t, false, Shape{wg, unroll});
    return RNG_OK;
}

int rng_get_shape(int g, int t, uint32_t *wg, uint32_t *unroll)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!wg || !unroll) return fail(RNG_EINVAL, "NULL output");
    Shape s = tuned_shape(g, t, false);
    *wg = s.wg;
    *unroll = s.unroll;
    return RNG_OK;
}

int rng_set_row_shape(int g, int t, uint64_t n_streams, uint64_t n, uint32_t wg, uint32_t unroll)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!valid_shape(wg, unroll)) return fail(RNG_EINVAL, "launch shape wg=%u unroll=%u", wg, unroll);
    set_tuned_shape(g, t, run_rows(n_streams, n) != 0, Shape{wg, unroll});
    return RNG_OK;
}

int rng_row_shape(int g, int t, uint64_t n_streams, uint64_t n, uint32_t *wg, uint32_t *unroll)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!wg || !unroll) return fail(RNG_EINVAL, "NULL output");
    Shape s = row_shape(g, t, n_streams, n);
    *wg = s.wg;
    *unroll = s.unroll;
    return RNG_OK;
}

int rng_autotune(int g, int t, uint64_t n_streams, uint64_t n, uint32_t *d_state_scratch,
                 void *d_out_scratch, uint32_t reps, uint32_t *best_wg, uint32_t *best_unroll,
                 float *best_us, void *stream)
{
    if (check_gen(g)) return RNG_EINVAL;
    if (t != RNG_U32 && t != RNG_F32) return fail(RNG_EINVAL, "unknown dtype %d", t);
    if (!d_state_scratch || !d_out_scratch || !best_wg || !best_unroll)
        return fail(RNG_EINVAL, "NULL argument");
    if (n_streams == 0 || n == 0 || reps == 0) return fail(RNG_EINVAL, "empty tuning problem");
    if (int rc = check_sizes(n_streams, n, gen_words(g))) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    static const uint32_t wgs[] = {64, 128, 256, 512, 1024};
    static const uint32_t uns[] = {1, 2, 4, 8, 16};
    float best = 1e30f;
    Shape bs{256, 8};
    int rc = RNG_OK;
    for (uint32_t wg : wgs) {
        for (uint32_t un : uns) {
            // one warm-up launch, then reps timed launches
            rc = generate_impl(g, t, d_state_scratch, n_streams, n_streams, n, d_out_scratch, Shape{wg, un},
                               true, st);
            if (rc) break;
            (void)hipEventRecord(e0, st);
            for (uint32_t r = 0; r < reps && !rc; ++r)
                rc = generate_impl(g, t, d_state_scratch, n_streams, n_streams, n, d_out_scratch,
                                   Shape{wg, un}, true, st);
            (void)hipEventRecord(e1, st);
            if (rc) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                rc = hip_fail(e, "hipEventSynchronize");
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            float us = ms * 1000.0f / reps;
            if (us < best) {
                best = us;
                bs = Shape{wg, un};
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    set_tuned_shape(g, t, run_rows(n_streams, n) != 0, bs);
    *best_wg = bs.wg;
    *best_unroll = bs.unroll;
    if (best_us) *best_us = best;
    return RNG_OK;
}

}  // extern "C"
