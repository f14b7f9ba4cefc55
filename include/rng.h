/*
 * rng.h -- C ABI of the MI355X bulk pseudo-random stream library.
 *
 * The library generates many independent 32-bit streams of the recurrences
 * studied in Hissoiny, Despres & Ozell, "Using graphics processing units to
 * generate random numbers" (arXiv:1101.1846):
 *   RNG_MWC32   multiply-with-carry, eq. (2)-(3), base b = 2^32, multiplier
 *               a = 65274 (the largest a < 2^16 with a*b - 1 a safe prime,
 *               the rule of Sec. II.A.1; the paper prints no value);
 *   RNG_MWC1616 the paper's MWC of Sec. III.A.1: two base-2^16 MWCs with
 *               distinct multipliers from the 392-entry safe-prime table,
 *               output (z << 16) + w;
 *   RNG_XS256   Panneton's r = 8, w = 32 XorShift, eq. (5), period 2^256 - 1;
 *   RNG_XS32    Marsaglia's xorshift32, eq. (6): y ^= y<<13; y ^= y>>17;
 *               y ^= y<<5;
 *   RNG_KISS    Sec. II.A.3: (MWC1616 xor LCG) + XS32, with the LCG of eq. (7)
 *               X <- 69069 X + 1234567 mod 2^32.
 * Every output is the value after a step ("step, then emit", eq. (1)); the
 * seed itself is never emitted.
 *
 * Conventions common to all calls
 *  - Pointers named d_* are device (HBM) pointers on the current HIP device;
 *    h_* are host pointers.  The caller allocates and frees every state and
 *    output buffer; the library never frees memory it did not allocate.
 *  - State layout (the paper keeps per-thread seeds and multipliers in global
 *    memory, fetched coalesced, Sec. III.A.1): structure of arrays, word w of
 *    stream s at d_state[w * n_streams + s].  Words per stream:
 *      MWC32 2 (x, c)   MWC1616 4 (z, w, a1, a2)   XS256 8 (v0..v7, v0 oldest)
 *      XS32 1 (y)       KISS 6 (z, w, jsr, jcong, a1, a2)
 *    State arrays are in/out: every generating call writes the advanced state
 *    back (the paper includes this write-back in its timing, Sec. III.B).
 *  - Output layout: stream-major, sample k of stream s at d_out[s * n + k]
 *    (the paper's output pool, Sec. III.B, whose layout it leaves open).
 *    RNG_U32 writes uint32 values; RNG_F32 writes float (u >> 8) * 2^-24,
 *    exact, in [0, 1 - 2^-24] (the [0,1) uniforms of Sec. III.B with the
 *    scaling fixed to the top 24 bits so that the map is exact).
 *  - Asynchrony: work is queued on the HIP stream passed as void*
 *    (hipStream_t, NULL = the null stream) and the call returns without
 *    waiting; argument checks happen before anything is queued.
 *  - Errors: 0 on success, a negative RNG_E* code otherwise; no exception
 *    crosses the ABI.  rng_strerror() describes a code, rng_last_error()
 *    gives the message of the calling thread's last failure.
 *  - Device tables (multiplier table, jump-ahead power tables) are built on
 *    the host and uploaded once per device, lazily on first use or by
 *    rng_init(); they are owned by the library until rng_shutdown().
 *  - rng_seed, rng_generate(_ex), rng_skip, rng_generate_split and
 *    rng_fused_pi only launch kernels on the given stream once the device
 *    tables exist, so they may be captured into a HIP graph after rng_init()
 *    (call each shape once outside the capture first).
 */
#ifndef RNG_MI355X_H
#define RNG_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { RNG_MWC32 = 1, RNG_XS256 = 2, RNG_XS32 = 3, RNG_KISS = 4, RNG_MWC1616 = 5 } rng_gen_t;
typedef enum { RNG_U32 = 0, RNG_F32 = 1 } rng_dtype_t;

#define RNG_OK 0
#define RNG_EINVAL (-1)  /* bad generator, dtype, null pointer or misaligned pointer */
#define RNG_ERANGE (-2)  /* a size or a size product overflows, or exceeds a limit */
#define RNG_ENOMEM (-3)  /* admission or workspace too small / allocation failed */
#define RNG_EHIP (-4)    /* a HIP runtime call failed; see rng_last_error() */
#define RNG_ENODEV (-5)  /* no usable gfx950 device */
#define RNG_EAGAIN (-6)  /* not ready yet (server polling) */

const char *rng_strerror(int code);
const char *rng_last_error(void);

/* Build and upload the device tables for the current device (idempotent). */
int rng_init(void);
/* Free the device tables of every device the library touched. */
int rng_shutdown(void);

/* Number of 32-bit state words per stream for generator g. */
int rng_state_words(int g, uint32_t *words);

/* The MWC32 multiplier (65274) and the 392 base-2^16 multipliers, ascending
 * (Sec. III.A.1).  h_out must hold cap entries; *count receives 392. */
int rng_mwc32_multiplier(uint32_t *a);
int rng_mwc16_multipliers(uint16_t *h_out, uint32_t cap, uint32_t *count);

/* Seed n_streams states from SplitMix64(seed) (Steele, Lea & Flood 2014).
 * Stream s uses the SplitMix64 outputs D*(first_stream+s) ... +D-1 with
 * D = 1 (MWC32, XS32), 2 (MWC1616), 3 (KISS), 4 (XS256); each stream gets its
 * own seeds and, for MWC1616/KISS, its own multiplier pair: the paper's
 * parametrisation plus independent seeds (Sec. II.A.4, III.A.1, III.A.3).
 * Fixed points are avoided: MWC c < a and z = c*b + x not in {0, a*b - 1};
 * XorShift states non-zero.  d_state: [words][n_streams] uint32, written. */
int rng_seed(int g, uint64_t seed, uint64_t first_stream, uint64_t n_streams,
             uint32_t *d_state, void *stream);

/* Bulk generation, Sec. III.A / III.B: n_streams streams, n samples each.
 * d_state [words][n_streams] in/out; d_out [n_streams][n] of dtype t, 4-byte
 * aligned (16-byte alignment with n % 4 == 0 takes 128-bit stores).
 * n = 0 or n_streams = 0 is a no-op.  When n_streams is small the library
 * splits each stream into chunks that start from jumped-ahead states, so the
 * output is still the serial sequence of every stream.  The states are then
 * written back only after every chunk has read them: inside the kernel when
 * one workgroup holds all chunks of its streams, else by a second launch on
 * the same stream that advances them by n. */
int rng_generate(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t,
                 void *d_out, void *stream);

/* Same, with an explicit launch shape: wg in {64,128,256,512,1024} lanes per
 * workgroup and unroll in {1,2,4,8,16} samples per generation-loop step.
 * rng_generate uses the autotuned shape when one is loaded, else a default;
 * rows of 4 or 8 KiB over whole groups of runs have a shape of their own
 * (below), and for other XS256 rows of an odd number of 4 KiB
 * (n = 1024 (2i + 1)) it takes at least 512 lanes, which generate each row
 * as four jumped chunks so that concurrent writes spread over four column
 * slots (for an even number the chunk starts would share one or two slots,
 * so those rows keep the plain order at every shape). */
int rng_generate_ex(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t,
                    void *d_out, uint32_t wg, uint32_t unroll, void *stream);

/* Launch shape used by rng_generate for (g, t): set, read, or pick by timing
 * every (wg, unroll) pair on the given problem (d_state_scratch and
 * d_out_scratch are overwritten; reps timed launches per shape).  The paper
 * chose block sizes with an occupancy calculator and unrolled its main loop
 * (Sec. III.A.1, III.B); the choice here is measured.
 *
 * Shapes are kept per row class.  Rows of 4 or 8 KiB (n = 1024 or 2048)
 * over a stream count that is a multiple of 256 or 128 are written as 16 KiB
 * runs of 4 or 2 adjacent rows per lane (on workgroups of up to 256 lanes),
 * and have a shape of their own (default 64 lanes, unroll 16); every other
 * problem uses the shape that rng_set_shape / rng_get_shape address (default
 * 256 lanes, unroll 8).  rng_autotune keeps its pick for the class of the
 * problem it timed; rng_set_row_shape sets, and rng_row_shape reads, the
 * shape rng_generate will use for n_streams x n (for XS256 rows of an odd
 * number of 4 KiB outside the run class, at least 512 lanes). */
int rng_set_shape(int g, int t, uint32_t wg, uint32_t unroll);
int rng_get_shape(int g, int t, uint32_t *wg, uint32_t *unroll);
int rng_set_row_shape(int g, int t, uint64_t n_streams, uint64_t n, uint32_t wg, uint32_t unroll);
int rng_row_shape(int g, int t, uint64_t n_streams, uint64_t n, uint32_t *wg, uint32_t *unroll);
int rng_autotune(int g, int t, uint64_t n_streams, uint64_t n, uint32_t *d_state_scratch,
                 void *d_out_scratch, uint32_t reps, uint32_t *best_wg, uint32_t *best_unroll,
                 float *best_us, void *stream);

/* Measured 32-bit integer VALU rate of the current device in lane-operations
 * per second, for op 0 (add + xor), 1 (24-bit multiply-add), 2 (32-bit
 * multiply low): eight independent chains per lane on every SIMD.  op 3
 * returns lane-samples per second of the fused consumer's own loop body
 * (rng_fused_pi's KISS pairs and exact quarter-circle test), the fastest of
 * 1, 2, 4 and 8 independent streams per lane interleaved: the ceiling of
 * that instruction mix.  The paper derived its integer peak
 * as a third of the FP rate (Sec. V) and measured only bandwidth; this
 * measures the integer rate.  Synchronous. */
int rng_calibrate_valu(int op, double *lane_ops_per_s, void *stream);

/* Achievable write rate of the bulk store schedule (Sec. V measured its
 * achievable bandwidth beside its kernels the same way): the generation
 * kernel with its resident schedule, LDS transpose and pipelined 16-byte
 * stores, run with a counter in place of a generator.  Sample k of stream s is
 * d_state[s] + k + 1 (mod 2^32), written to d_out[s][k], and d_state[s]
 * advances by n; every stream is one chunk.  d_state holds n_streams words,
 * d_out n_streams x n words, both 4-byte aligned and owned by the caller (a
 * 16-byte aligned d_out with n a multiple of 4 takes the 128-bit stores); wg
 * and unroll as for rng_generate_ex.  Asynchronous on stream.  RNG_EINVAL for
 * a bad shape, NULL or misaligned pointers, RNG_ERANGE for sizes the ABI's
 * size checks reject (as rng_generate). */
int rng_calibrate_store(uint32_t *d_state, uint64_t n_streams, uint64_t n, void *d_out, uint32_t wg,
                        uint32_t unroll, void *stream);

/* Advance every stream by k steps without producing output: sequence
 * splitting needs the i-th number without the intermediate ones (Sec.
 * II.A.4).  MWC: z <- a^k z mod (a*b - 1) with z = c*b + x; XorShift: the
 * k-th power of the GF(2) step matrix; LCG: the k-fold affine map. */
int rng_skip(int g, uint32_t *d_state, uint64_t n_streams, uint64_t k, void *stream);

/* Sequence splitting (Sec. II.A.4): one logical stream, d_state_one
 * ([words] uint32, device, read only), produces `total` samples divided
 * across n_threads GPU threads, thread t writing samples
 * [t*C, min((t+1)*C, total)) with C = ceil(total / n_threads), each thread
 * starting from the jumped-ahead state, so that d_out[0 .. total) equals the
 * serial sequence.  The advanced state is written to d_final_state ([words],
 * device; may alias d_state_one).  d_workspace of at least
 * rng_split_workspace_bytes(g, n_threads) bytes, 256-byte aligned, caller
 * owned, holds the per-thread states. */
int rng_split_workspace_bytes(int g, uint64_t n_threads, uint64_t *bytes);
int rng_generate_split(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads,
                       int t, void *d_out, uint32_t *d_final_state, void *d_workspace,
                       uint64_t workspace_bytes, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): rng_generate_split without a
 * workspace argument.  The thread states live in a device array of
 * RNG_SPLIT_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends; the call itself makes no hipMalloc, hipFree
 * or other allocating call.  rng_init() must have run on the current device
 * (it builds the tables and looks up the array's address), else RNG_EINVAL.
 * A split needs 4 * W * T bytes (W state words, T = ceil(total / C) threads
 * with work, C = ceil(total / n_threads)); larger splits return RNG_ERANGE
 * (32 MiB holds 2^20 threads of every generator).  Every call on one device
 * shares the array and leaves it holding its thread states, so calls that
 * overlap on one device (other streams, other host threads) race: serialise
 * them.  Arguments, output and errors otherwise as rng_generate_split. */
#define RNG_SPLIT_NOALLOC_SCRATCH_BYTES (32u << 20)
int rng_generate_split_noalloc(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads,
                               int t, void *d_out, uint32_t *d_final_state, void *stream);

/* Leapfrogging (Sec. II.A.4): the same sequence and output as
 * rng_generate_split, computed the other way round.  With T = min(n_threads,
 * total) threads, thread j emits numbers j, j + T, j + 2T, ... of the serial
 * sequence, so d_out[i] is number i and every wave stores 64 consecutive
 * numbers.  Thread j starts at the state after j steps (a radix-16 tree of
 * jumps), steps once, and then advances T steps per number with the
 * generator's T-step map: one modular multiply per MWC word, a 32x32 GF(2)
 * product for xorshift32, a 256x256 one for XS256 (through a 4-bit table of
 * M^T in LDS), an affine map for the LCG.  d_out[0 .. total) equals the
 * serial sequence; the advanced state goes to d_final_state ([words], device;
 * may alias d_state_one).  d_workspace of at least
 * rng_leapfrog_workspace_bytes(g, T) bytes, 256-byte aligned, caller owned,
 * holds the thread states and the T-step constants.  Errors as
 * rng_generate_split. */
int rng_leapfrog_workspace_bytes(int g, uint64_t n_threads, uint64_t *bytes);
int rng_generate_leapfrog(int g, const uint32_t *d_state_one, uint64_t total, uint64_t n_threads,
                          int t, void *d_out, uint32_t *d_final_state, void *d_workspace,
                          uint64_t workspace_bytes, void *stream);

/* Fused consumer (the paper's "without write-back" mode, Sec. III.B, made to
 * consume every sample): each stream draws n samples; consecutive pairs
 * (u_{2k}, u_{2k+1}) give i = u_{2k} >> 8, j = u_{2k+1} >> 8 and count when
 * i^2 + j^2 < 2^48, i.e. x^2 + y^2 < 1 exactly for the FP32 uniforms
 * x = i 2^-24, y = j 2^-24.  The count of all streams is ADDED to *d_count
 * (device uint64; clear it first).  No sample is stored; states are written
 * back.  An odd trailing sample is drawn but not counted. */
int rng_fused_pi(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n,
                 uint64_t *d_count, void *stream);

/* The "without write-back" mode of the paper's Tables I-III (Sec. III.B),
 * for every generator: each stream draws n numbers (uint32, or their FP32
 * bit patterns for t = RNG_F32) and d_fold[s] ([n_streams] uint32, device)
 * is XORed with the XOR of stream s's n outputs; nothing else is stored and
 * the states are written back.  Every number is computed, so the rate is the
 * generator's arithmetic-bound one.  Clear d_fold first for the plain XOR.
 * Few streams are cut into jumped chunks whose folds combine by atomic XOR;
 * their states are then advanced by a second launch. */
int rng_generate_fold(int g, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t,
                      uint32_t *d_fold, void *stream);

/* The paper's XorShift placement comparison (Sec. III.A.2, Table II): the
 * r = 8 XorShift (eq. (5)) with each thread's eight state words
 *   RNG_XS_LDS_INDEXED   in LDS, read and written through a runtime
 *                        circular index (the reference C code's form);
 *   RNG_XS_LDS_UNROLLED  in LDS, circular buffer made explicit by an 8-fold
 *                        unroll (constant offsets);
 *   RNG_XS_VGPR          in registers (the library's own form).
 * The state words sit blockDim-strided in LDS (word i of thread t at
 * i * 256 + t), the paper's bank-conflict-free layout, and every LDS access is
 * a real load or store.  All three give the same numbers as rng_generate.
 * One thread per stream, 256-thread workgroups; d_state is [8][n_streams]
 * (as rng_seed writes it) and is advanced by n.
 *   d_out  : with write-back, [n][n_streams] sample-major (number k of stream
 *            s at d_out[k * n_streams + s]), uint32 or FP32 per t;
 *   d_fold : without write-back, [n_streams] XOR of each stream's n outputs
 *            (FP32 bit patterns when t = RNG_F32); nothing else is stored.
 * Exactly one of d_out and d_fold is non-NULL (else RNG_EINVAL); n_streams
 * at most 2^31.  Meant for measuring what the placement costs, not as a
 * faster path. */
typedef enum { RNG_XS_LDS_INDEXED = 0, RNG_XS_LDS_UNROLLED = 1, RNG_XS_VGPR = 2 } rng_xs_placement_t;
int rng_xs256_placement(int placement, uint32_t *d_state, uint64_t n_streams, uint64_t n, int t,
                        void *d_out, uint32_t *d_fold, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched generation: thousands of independent requests of uneven length  */
/* in one persistent generation launch (after the root and tree launches,   */
/* issued directly or replayed as a captured HIP graph).  Each request is a */
/* slice [offset, offset + length) of one stream's serial sequence; the     */
/* stream's state is advanced by offset + length.  Requests are cut into    */
/* chunks of C samples whose start states come from jump-ahead: one jump    */
/* per request, then a radix-16 tree (level l starts chunk q 16^l + r from  */
/* chunk r, q < 16: at most four jumps by powers of two per chunk; level 0  */
/* in the root's launch, one launch per further level); a persistent kernel */
/* pulls 64-chunk tiles from an atomic counter.                             */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t gen;            /* rng_gen_t */
    int32_t dtype;          /* rng_dtype_t */
    uint32_t *d_state;      /* word 0 of the stream's state (device), in/out */
    uint64_t state_stride;  /* word stride of that state: 1 for a contiguous
                               [words] state, n_streams for stream s of a
                               [words][n_streams] pool (d_state = pool + s) */
    uint64_t offset;        /* samples skipped before the first output */
    uint64_t length;        /* samples produced (0: only the skip) */
    void *d_out;            /* [length] outputs of dtype, 4-byte aligned; a
                               128-byte aligned d_out keeps every chunk's
                               stores on whole cache lines (the fast path:
                               misaligned rows write partial lines and run
                               up to 2x slower) */
} rng_request_t;

typedef struct rng_batch rng_batch_t;

/* A batch handle for up to max_requests requests of at most max_samples
 * samples in total; it owns its device workspace (chunk states, plan) and
 * pinned staging buffers, and its graphs.  Created on the current device. */
int rng_batch_create(uint32_t max_requests, uint64_t max_samples, rng_batch_t **h);
/* Plan a batch from a host table of n requests (copied; the caller may reuse
 * its table).  No two requests may share a stream state (the same d_state
 * twice is RNG_EINVAL; overlapping strided states are not detected).  Blocks
 * until the previous launch's plan upload has left the staging buffers. */
int rng_batch_set(rng_batch_t *h, const rng_request_t *h_reqs, uint32_t n);
/* Queue the planned batch on stream: one plan upload, then the root jumps
 * (with tree level 0), the further tree levels and the persistent
 * generation kernel. */
int rng_batch_launch(rng_batch_t *h, void *stream);
/* use_graph = 1: rng_batch_launch replays a HIP graph of those kernels,
 * captured once per (tree depth, shape) on the handle's own stream;
 * 0 (the default): it launches them directly.  Both give the same results.
 * On MI355X with ROCm 7 a graph replay of 2-6 kernels costs about 21 us of
 * host time against 2.6 us per direct launch, so the direct launches give
 * the lower latency. */
int rng_batch_set_graph(rng_batch_t *h, int use_graph);
/* Persistent-kernel shape: wg lanes per workgroup in {64, 128, 256, 512,
 * 1024} and unroll (samples per generation step) in {1, 2, 4, 8, 16}, every
 * pair built (others RNG_EINVAL; 1024-lane workgroups stage 32-sample LDS
 * tiles, the others 64); and chunk length C (a multiple of 64).  0 keeps the current value.  chunk = RNG_BATCH_CHUNK_AUTO lets every plan
 * choose C: the power of two in [64, 4096] that cuts the batch into about
 * 2^17 chunks (as many 64-chunk tiles as the device holds waves), so that
 * small batches still spread over the device; the workspace is sized for
 * 256-sample chunks (more for handles of more than 2^36 samples), and a plan
 * goes below that only while its chunks fit.  A changed C applies to the
 * last planned table at once (it is planned again). */
#define RNG_BATCH_CHUNK_AUTO 0xFFFFFFFFu
int rng_batch_set_shape(rng_batch_t *h, uint32_t wg, uint32_t unroll, uint32_t chunk);
/* The current shape; chunk reads RNG_BATCH_CHUNK_AUTO in automatic mode. */
int rng_batch_get_shape(rng_batch_t *h, uint32_t *wg, uint32_t *unroll, uint32_t *chunk);
/* Time the planned batch under every persistent-kernel shape (the 25 pairs
 * wg x unroll) and chunk length in {512, 1024, 2048, 4096}, reps launches
 * each after one warm-up launch, and keep the fastest.  Every trial launch runs the batch, so the request states
 * advance and the outputs are overwritten. */
int rng_batch_autotune(rng_batch_t *h, uint32_t reps, uint32_t *best_wg, uint32_t *best_unroll,
                       uint32_t *best_chunk, float *best_us, void *stream);
int rng_batch_destroy(rng_batch_t *h);

/* ---------------------------------------------------------------------- */
/* Serving: a request loop over resident stream states with continuous     */
/* batching.  A worker thread admits queued requests while output memory    */
/* (a device pool) and in-flight slots allow, launches each admitted set as */
/* one batch on one of `inflight` HIP streams (batches overlap on the       */
/* device), and stamps each request's completion.  Requests for the same   */
/* stream are served in arrival order, so request i of a stream returns the */
/* samples [L_0 + ... + L_{i-1}, + L_i) of that stream's serial sequence.   */
/* While batches are in flight the worker polls their events in a loop (it  */
/* keeps one host core busy, for latency); when none are, it keeps polling  */
/* for idle_spin_us after its last activity (so that a new request finds it */
/* awake) and then sleeps until a submission wakes it.  Every batch picks   */
/* its chunk length automatically (RNG_BATCH_CHUNK_AUTO).                   */
/* ---------------------------------------------------------------------- */
typedef struct {
    uint64_t n_streams;            /* resident streams; stream s runs gens[s % n_gens] */
    int32_t gens[5];
    uint32_t n_gens;
    uint64_t seed;                 /* generator kind k is seeded from SplitMix64(seed + k),
                                      stream s being entry s / n_gens of its kind's pool */
    uint64_t pool_bytes;           /* output memory budget used for admission */
    uint32_t max_batch_requests;   /* per launched batch */
    uint64_t max_batch_samples;    /* per launched batch; also the largest request */
    uint32_t inflight;             /* batches in flight, 1..8 */
    uint32_t auto_release;         /* 1: free each output as soon as it completes */
    uint32_t idle_spin_us;         /* idle polling window before the worker sleeps (0: sleep at once) */
} rng_server_config_t;

typedef struct {
    uint64_t submitted, completed, batches, samples, admission_waits;
    double p50_us, p99_us, mean_us, max_us;  /* arrival -> completion latency */
    double wall_s;                           /* first arrival -> last completion */
    double gsamples_per_s;
    double mean_batch_requests;
    /* mean_us in three parts: arrival -> admission into a batch (queue),
     * admission -> its launches enqueued (host: plan and launch calls),
     * enqueued -> completion seen by the worker (device, and the poll) */
    double mean_queue_us, mean_submit_us, mean_device_us;
} rng_server_stats_t;

typedef struct rng_server rng_server_t;

int rng_server_create(const rng_server_config_t *cfg, rng_server_t **h);
/* Queue one request (thread-safe); *ticket identifies it. */
int rng_server_submit(rng_server_t *h, uint64_t stream_id, uint64_t length, int dtype, uint64_t *ticket);
/* RNG_OK with *done = 1 and *d_out = its device output once complete (NULL if
 * released), RNG_EAGAIN with *done = 0 before. */
int rng_server_poll(rng_server_t *h, uint64_t ticket, int *done, void **d_out);
/* Return a completed request's output memory to the pool. */
int rng_server_release(rng_server_t *h, uint64_t ticket);
/* Block until every submitted request has completed.  Admission needs free
 * output memory: with auto_release = 0, requests beyond the pool complete
 * only as the caller releases earlier outputs (from another thread), so a
 * caller that drains without releasing waits for ever once the pool fills. */
int rng_server_drain(rng_server_t *h);
/* Copy one idle stream's resident state to the host ([words] uint32): the
 * resident states are the server's checkpoint.  RNG_EAGAIN while a request
 * for that stream is in flight; a request submitted concurrently may still
 * overtake the copy, so read states with no request pending for them. */
int rng_server_read_state(rng_server_t *h, uint64_t stream_id, uint32_t *h_state);
int rng_server_stats(rng_server_t *h, rng_server_stats_t *st);
int rng_server_reset_stats(rng_server_t *h);
/* Submit n requests at the given arrival times (seconds from the call,
 * ascending) in real time, then drain; tickets (may be NULL) receives their ids. */
int rng_server_replay(rng_server_t *h, const double *t_arrival_s, const uint64_t *stream_ids,
                      const uint64_t *lengths, const int32_t *dtypes, uint64_t n, uint64_t *tickets);
/* Stop the worker and free the server: batches in flight complete, pending
 * requests that can still be admitted run, and those waiting for output
 * memory that is never released are abandoned. */
int rng_server_destroy(rng_server_t *h);

#ifdef __cplusplus
}
#endif

#endif /* RNG_MI355X_H */
