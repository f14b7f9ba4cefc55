// rng_abi_internal.hpp -- helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"
#include "rng_internal.hpp"

namespace rngx {

struct Shape {
    uint32_t wg, unroll;
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int check_launch(int rc, const char *what);
int check_gen(int g);
int check_sizes(uint64_t S, uint64_t N, uint64_t words);
int device_tables(DevTables *out);
int gen_words(int g);
bool valid_shape(uint32_t wg, uint32_t unroll);
uint32_t run_rows(uint64_t S, uint64_t N);
Shape tuned_shape(int g, int dt, bool runs);
Shape row_shape(int g, int dt, uint64_t S, uint64_t n);
void set_tuned_shape(int g, int dt, bool runs, Shape s);
// Chunks per stream: the largest power of two p with S p <= target_lanes and
// chunks of at least the generator's minimum length.
void choose_chunks(int g, uint64_t S, uint64_t N, uint64_t align, uint64_t *C, uint32_t *P, uint64_t target_lanes);
// Chunks for one lane per chunk (fewer streams than a wave has lanes).
void lane_chunks(int g, uint64_t S, uint64_t N, uint64_t *C, uint32_t *P);
int generate_impl(int g, int dt, uint32_t *d_state, uint64_t ld, uint64_t S, uint64_t N, void *d_out,
                  Shape shape, bool staged, hipStream_t st);
int dispatch_generate(int g, int dt, const GenArgs &a, int wg, int unroll, bool staged, hipStream_t st);
int dispatch_skip(int g, uint32_t *st, uint64_t ld, uint64_t S, uint64_t k, const DevTables &tab, hipStream_t s);
// One radix-16 level of a thread-start tree: threads [2^shift, min(2^(shift+4), T))
// of ws ([W][T]) from the threads below 2^shift, unit samples per thread index.
int dispatch_tree_level(int g, uint32_t *ws, uint64_t T, uint32_t shift, uint64_t unit, const DevTables &tab,
                        hipStream_t s);
// Thread starts 0 .. min(T, 4096) - 1 of a split or leapfrogged sequence
// from one state (k_tree_head); the further tree levels start at shift 12.
template <class G>
int launch_tree_head_t(const uint32_t *st0, uint32_t *ws, uint64_t T, uint64_t unit, const DevTables &tab,
                       hipStream_t stream);
int dispatch_tree_head(int g, const uint32_t *st0, uint32_t *ws, uint64_t T, uint64_t unit, const DevTables &tab,
                       hipStream_t s);
constexpr uint32_t kTreeHeadShift = 12;
int dispatch_state_copy(int g, const uint32_t *src, uint64_t ss, uint64_t si, uint32_t *dst, uint64_t ds,
                        uint64_t di, hipStream_t s);

// Fewer streams than a wave has lanes: lane v takes chunk v mod P of stream
// v / P (chunks of C samples), then the states advance by N (few.hip).
int generate_few(int g, int dt, uint32_t *d_state, uint64_t ld, uint64_t S, uint64_t N, uint64_t C, uint64_t P,
                 void *d_out, const DevTables &tab, hipStream_t st);

// Tables of the current device only if they exist already (never allocates).
int device_tables_if_ready(DevTables *out);
// Looks up, once per device, the address of the allocation-free entry
// point's scratch array on the current device (called by rng_init).
int scratch_init_current_device();
// Sequence splitting: argument checks, the workspace a split needs, and the
// launches themselves (thread states in ws, [W][T] words).
int split_args_check(uint64_t total, uint64_t n_threads, const void *d_out, const uint32_t *d_state_one,
                     const uint32_t *d_final_state);
int split_scratch_bytes(int g, uint64_t total, uint64_t n_threads, uint64_t *bytes);
int split_run(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads, int t, void *d_out,
              uint32_t *d_final_state, uint32_t *ws, uint64_t ws_bytes, const DevTables &tab, hipStream_t st);

// rng_batch_set without the check that no two requests share a state (for
// callers that keep one request per state).
int batch_set_distinct(rng_batch_t *h, const rng_request_t *reqs, uint32_t n);
}  // namespace rngx
