// rng_batch.cpp -- the batched path of the C ABI: plans a batch of
// independent requests (chunking, grouping by generator and dtype, the
// radix-16 tree work lists), ships the plan through pinned host memory, and
// replays one captured HIP graph per batch shape: root jumps (which also
// reset the tile counter), tree levels, persistent generation kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "rng.h"
#include "rng_abi_internal.hpp"
#include "rng_batch_internal.hpp"

namespace rngx {
int launch_batch_root(const BatchArgs &a, const PlanInline &pin, uint32_t max_requests, hipStream_t s);
int launch_batch_level(const BatchArgs &a, uint32_t level, unsigned grid, hipStream_t s);
int launch_batch_tree_small(const BatchArgs &a, const PlanInline &pin, uint32_t n, hipStream_t s);
int launch_batch_gen(const BatchArgs &a, int wg, int unroll, unsigned grid, hipStream_t s);
int batch_gen_occupancy(int wg, int unroll, int *blocks_per_cu);
}  // namespace rngx

using namespace rngx;

struct rng_batch {
    std::mutex mu;
    int device = 0;
    uint32_t max_requests = 0;
    uint64_t max_samples = 0;
    uint64_t C = 1024;
    bool chunk_auto = false;  // C chosen per plan (RNG_BATCH_CHUNK_AUTO)
    uint32_t wg = 256, unroll = 8;
    uint64_t ws_words = 0;
    char *d_plan = nullptr, *h_plan = nullptr;  // packed plan (BatchHeader first), device and pinned staging
    uint64_t plan_cap = 0;                      // bytes of each
    uint32_t *d_ws = nullptr, *d_counter = nullptr, *d_map = nullptr;
    hipEvent_t copied = nullptr;
    hipStream_t capture = nullptr;  // private stream the graphs are recorded on
    bool copy_pending = false;
    bool planned = false;
    struct Graph {
        uint32_t levels, wg, unroll;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    bool use_graph = false;               // replay a captured graph instead of launching directly
    uint32_t occ_wg = 0, occ_unroll = 0;  // shape of the cached occupancy
    unsigned gen_full = 0;                // generation workgroups resident at once for that shape
    int num_cu = 256;
    std::vector<rng_request_t> last;  // last planned table, re-planned on a chunk change
    BatchHeader &hdr() { return *(BatchHeader *)h_plan; }
};

// Automatic chunk length: a power of two in [64, 4096] that cuts the batch
// into about 2^17 chunks (2048 tiles of 64: the waves the device holds at
// once), so that a small batch still spreads over the device.  The workspace
// is sized for chunks of auto_chunk_min (256, more for huge handles); shorter
// chunks are taken only while the plan's chunks fit it.
constexpr uint64_t kAutoChunkMax = 4096;
constexpr uint64_t kAutoChunkFloor = kBatchTile;
constexpr uint64_t kSmallBatch = (uint64_t)1 << 19;  // samples
constexpr uint64_t kAutoChunks = (uint64_t)1 << 17;
static uint64_t auto_chunk_min(uint64_t max_samples)
{
    uint64_t c = 256;  // keeps the chunk capacity below 2^28
    while (c < kAutoChunkMax && max_samples / c > ((uint64_t)1 << 28)) c *= 2;
    return c;
}

static uint64_t chunk_capacity(const rng_batch *h, uint64_t C)
{
    return (h->max_samples + C - 1) / C + h->max_requests + (uint64_t)kBatchMaxGroups * 64;
}

// Segments of all levels: at most one per request and level.
static uint64_t seg_capacity(const rng_batch *h) { return (uint64_t)kBatchMaxLevels * h->max_requests; }

// Block starts of all levels: the levels' work items sum to fewer than the
// chunks, so sum(ceil(items / kLevelWG)) <= chunks / kLevelWG + levels.
static uint64_t blk_capacity(const rng_batch *h, uint64_t C)
{
    return chunk_capacity(h, C) / kLevelWG + kBatchMaxLevels + 1;
}

static uint64_t align16(uint64_t x) { return (x + 15) & ~(uint64_t)15; }

// Packed plan: header, requests, segments, block starts (16-byte aligned each).
static uint64_t plan_capacity(const rng_batch *h, uint64_t C)
{
    return align16(sizeof(BatchHeader)) + align16(sizeof(BatchReq) * (uint64_t)h->max_requests) +
           align16(8 * seg_capacity(h)) + 4 * blk_capacity(h, C);
}

// Sizes the chunk workspace, the chunk-to-request map and the level work
// lists for chunk length C.  Growing any of them drops the captured graphs,
// which hold the old addresses.
static int alloc_ws(rng_batch *h, uint64_t C)
{
    const uint64_t chunks = chunk_capacity(h, C);
    const uint64_t words = chunks * 8;  // widest state: 8 words
    const uint64_t plan_bytes = plan_capacity(h, C);
    if (words <= h->ws_words && plan_bytes <= h->plan_cap) return RNG_OK;
    if (plan_bytes >= ((uint64_t)1 << 32)) return fail(RNG_ENOMEM, "batch plan above 4 GiB");
    if (chunks >= ((uint64_t)1 << 32)) return fail(RNG_ENOMEM, "more than 2^32 chunks of %llu samples",
                                                   (unsigned long long)C);
    for (auto &g : h->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
    (void)hipDeviceSynchronize();  // no launch may still use the old buffers
    if (h->d_ws) (void)hipFree(h->d_ws);
    if (h->d_map) (void)hipFree(h->d_map);
    if (h->d_plan) (void)hipFree(h->d_plan);
    if (h->h_plan) (void)hipHostFree(h->h_plan);
    h->d_ws = h->d_map = nullptr;
    h->d_plan = h->h_plan = nullptr;
    h->ws_words = h->plan_cap = 0;
    h->planned = false;  // the plan lived in the old staging buffer
    hipError_t e;
    if ((e = hipMalloc((void **)&h->d_ws, words * 4)) != hipSuccess) return hip_fail(e, "hipMalloc(batch workspace)");
    if ((e = hipMalloc((void **)&h->d_map, chunks * 4)) != hipSuccess) return hip_fail(e, "hipMalloc(chunk map)");
    if ((e = hipMalloc((void **)&h->d_plan, plan_bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(batch plan)");
    if ((e = hipHostMalloc((void **)&h->h_plan, plan_bytes, hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "hipHostMalloc(batch plan)");
    std::memset(h->h_plan, 0, sizeof(BatchHeader));
    h->ws_words = words;
    h->plan_cap = plan_bytes;
    return RNG_OK;
}

static void free_batch(rng_batch *h)
{
    for (auto &g : h->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    if (h->copied) (void)hipEventDestroy(h->copied);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    if (h->d_plan) (void)hipFree(h->d_plan);
    if (h->d_map) (void)hipFree(h->d_map);
    if (h->d_ws) (void)hipFree(h->d_ws);
    if (h->d_counter) (void)hipFree(h->d_counter);
    if (h->h_plan) (void)hipHostFree(h->h_plan);
    delete h;
}

static bool shape_ok(uint32_t wg, uint32_t unroll)
{
    int b = 0;
    return batch_gen_occupancy((int)wg, (int)unroll, &b) == 0;
}

static BatchArgs make_args(rng_batch *h, const DevTables &tab)
{
    BatchArgs a{};
    a.hdr = (const BatchHeader *)h->d_plan;
    a.chunk_req = h->d_map;
    a.ws = h->d_ws;
    a.counter = h->d_counter;
    a.tab = tab;
    return a;
}

static int plan(rng_batch_t *h, const rng_request_t *reqs, uint32_t n);

extern "C" {

int rng_batch_create(uint32_t max_requests, uint64_t max_samples, rng_batch_t **out)
{
    if (!out) return fail(RNG_EINVAL, "NULL handle pointer");
    if (max_requests == 0) return fail(RNG_EINVAL, "max_requests is 0");
    if (max_samples > ((uint64_t)1 << 40)) return fail(RNG_ERANGE, "max_samples above 2^40");
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    auto *h = new rng_batch();
    h->max_requests = max_requests;
    h->max_samples = max_samples;
    (void)hipGetDevice(&h->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) h->num_cu = prop.multiProcessorCount;
    hipError_t e = hipSuccess;
    int rc = RNG_OK;
    if ((e = hipMalloc((void **)&h->d_counter, 256)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->copied, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking)) != hipSuccess)
        rc = hip_fail(e, "rng_batch_create");
    if (!rc) rc = alloc_ws(h, h->C);
    if (rc) {
        free_batch(h);
        return rc;
    }
    *out = h;
    return RNG_OK;
}

int rng_batch_destroy(rng_batch_t *h)
{
    if (!h) return RNG_OK;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (h->copy_pending) (void)hipEventSynchronize(h->copied);
    }
    free_batch(h);
    return RNG_OK;
}

int rng_batch_set_shape(rng_batch_t *h, uint32_t wg, uint32_t unroll, uint32_t chunk)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    std::lock_guard<std::mutex> lk(h->mu);
    uint32_t w = wg ? wg : h->wg, u = unroll ? unroll : h->unroll;
    if (!shape_ok(w, u)) return fail(RNG_EINVAL, "batch launch shape wg=%u unroll=%u not available", w, u);
    if (chunk) {
        const bool autoc = chunk == RNG_BATCH_CHUNK_AUTO;
        if (!autoc && chunk % kBatchTile)
            return fail(RNG_EINVAL, "chunk %u is not a multiple of %d", chunk, kBatchTile);
        if (h->copy_pending) (void)hipEventSynchronize(h->copied);
        const uint64_t cmin = autoc ? auto_chunk_min(h->max_samples) : chunk;
        if (int rc = alloc_ws(h, cmin)) return rc;
        h->chunk_auto = autoc;
        h->C = autoc ? cmin : chunk;
        h->planned = false;  // the plan depends on the chunk length
        if (!h->last.empty()) {
            std::vector<rng_request_t> t = h->last;
            if (int rc = plan(h, t.data(), (uint32_t)t.size())) return rc;
        }
    }
    h->wg = w;
    h->unroll = u;
    return RNG_OK;
}

int rng_batch_set_graph(rng_batch_t *h, int use_graph)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    if (use_graph != 0 && use_graph != 1) return fail(RNG_EINVAL, "use_graph must be 0 or 1");
    std::lock_guard<std::mutex> lk(h->mu);
    h->use_graph = use_graph == 1;
    return RNG_OK;
}

int rng_batch_get_shape(rng_batch_t *h, uint32_t *wg, uint32_t *unroll, uint32_t *chunk)
{
    if (!h || !wg || !unroll || !chunk) return fail(RNG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(h->mu);
    *wg = h->wg;
    *unroll = h->unroll;
    *chunk = h->chunk_auto ? RNG_BATCH_CHUNK_AUTO : (uint32_t)h->C;
    return RNG_OK;
}

int rng_batch_set(rng_batch_t *h, const rng_request_t *reqs, uint32_t n)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    if (n && !reqs) return fail(RNG_EINVAL, "NULL request table");
    if (n > h->max_requests) return fail(RNG_ENOMEM, "%u requests > capacity %u", n, h->max_requests);
    if (n > 1) {
        // two requests on one state would race on its write-back
        std::vector<uintptr_t> p(n);
        for (uint32_t i = 0; i < n; ++i) p[i] = (uintptr_t)reqs[i].d_state;
        std::sort(p.begin(), p.end());
        if (std::adjacent_find(p.begin(), p.end()) != p.end())
            return fail(RNG_EINVAL, "two requests share one d_state");
    }
    return batch_set_distinct(h, reqs, n);
}

}  // extern "C"

// rng_batch_set for callers that already keep one request per state (the
// server's batches).
int rngx::batch_set_distinct(rng_batch_t *h, const rng_request_t *reqs, uint32_t n)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    if (n && !reqs) return fail(RNG_EINVAL, "NULL request table");
    std::lock_guard<std::mutex> lk(h->mu);
    int rc = plan(h, reqs, n);
    if (rc == RNG_OK) h->last.assign(reqs, reqs + n);
    return rc;
}

extern "C" {

static int plan(rng_batch_t *h, const rng_request_t *reqs, uint32_t n)
{
    if (n > h->max_requests) return fail(RNG_ENOMEM, "%u requests > capacity %u", n, h->max_requests);
    uint64_t total_samples = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const rng_request_t &r = reqs[i];
        if (check_gen(r.gen)) return fail(RNG_EINVAL, "request %u: unknown generator %d", i, r.gen);
        if (r.dtype != RNG_U32 && r.dtype != RNG_F32) return fail(RNG_EINVAL, "request %u: dtype %d", i, r.dtype);
        if (!r.d_state || ((uintptr_t)r.d_state & 3)) return fail(RNG_EINVAL, "request %u: bad state pointer", i);
        if (r.state_stride == 0) return fail(RNG_EINVAL, "request %u: state_stride is 0", i);
        if (r.length && (!r.d_out || ((uintptr_t)r.d_out & 3))) return fail(RNG_EINVAL, "request %u: bad output", i);
        if (__builtin_add_overflow(total_samples, r.length, &total_samples))
            return fail(RNG_ERANGE, "total length overflows");
    }
    if (total_samples > h->max_samples)
        return fail(RNG_ENOMEM, "batch of %llu samples > capacity %llu", (unsigned long long)total_samples,
                    (unsigned long long)h->max_samples);
    if (h->chunk_auto) {
        // The workspace holds max_samples in chunks of auto_chunk_min.  A
        // small batch (its time is the serial work per lane) takes shorter
        // chunks, down to one 64-sample tile, while they fit; larger ones keep
        // the longer minimum, since more chunks mean more tree work.
        const uint64_t cmin = auto_chunk_min(h->max_samples), fit = (h->max_samples + cmin - 1) / cmin;
        uint64_t c = total_samples <= kSmallBatch ? kAutoChunkFloor : cmin;
        while (c < kAutoChunkMax && (total_samples / (2 * c) >= kAutoChunks || (total_samples + c - 1) / c > fit))
            c *= 2;
        h->C = c;
    }
    // The pinned staging buffers are about to be rewritten: wait for the
    // previous launch's copies to leave them.
    if (h->copy_pending) {
        hipError_t e = hipEventSynchronize(h->copied);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        h->copy_pending = false;
    }
    // group requests by (generator, dtype), stable
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    auto key = [&](uint32_t i) { return reqs[i].gen * 2 + reqs[i].dtype; };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return key(x) < key(y); });
    const uint64_t C = h->C;

    h->planned = false;  // until this plan is complete: a failure below leaves nothing to launch
    BatchHeader &H = h->hdr();
    std::memset(&H, 0, sizeof(H));
    H.C = C;
    H.n = n;
    H.off_reqs = (uint32_t)align16(sizeof(BatchHeader));
    BatchReq *Q = plan_at<BatchReq>(&H, H.off_reqs);
    uint64_t ws_off = 0, tiles = 0, max_chunks = 0;
    uint32_t i = 0;
    while (i < n) {
        const int k = key(order[i]);
        BatchGroup &G = H.groups[H.ngroups];
        G.gen = (uint32_t)reqs[order[i]].gen;
        G.dtype = (uint32_t)reqs[order[i]].dtype;
        G.words = (uint32_t)gen_words(reqs[order[i]].gen);
        G.req_begin = i;
        uint64_t chunks = 0;
        for (; i < n && key(order[i]) == k; ++i) {
            const rng_request_t &r = reqs[order[i]];
            BatchReq &q = Q[i];
            q.state = r.d_state;
            q.stride = r.state_stride;
            q.offset = r.offset;
            q.length = r.length;
            q.out = (uint32_t *)r.d_out;
            q.chunk_base = (uint32_t)chunks;
            q.nchunks = (uint32_t)((r.length + C - 1) / C);
            q.group = H.ngroups;
            q.pad = 0;
            chunks += q.nchunks;
            max_chunks = std::max<uint64_t>(max_chunks, q.nchunks);
        }
        G.req_end = i;
        G.nchunks = (uint32_t)chunks;
        G.nchunks_pad = (uint32_t)((chunks + 63) / 64 * 64);
        G.tile_begin = (uint32_t)tiles;
        tiles += G.nchunks_pad / 64;
        G.tile_end = (uint32_t)tiles;
        G.ws_off = ws_off;
        ws_off += (uint64_t)G.words * G.nchunks_pad;
        H.ngroups++;
    }
    if (ws_off > h->ws_words) return fail(RNG_ENOMEM, "batch needs %llu workspace words > %llu",
                                          (unsigned long long)ws_off, (unsigned long long)h->ws_words);
    H.n_tiles = (uint32_t)tiles;
    // radix-16 levels: 16^levels >= the largest request's chunk count
    uint32_t levels = 0;
    while (((uint64_t)1 << (kRadixBits * levels)) < max_chunks) ++levels;
    if (levels > (uint32_t)kBatchMaxLevels) return fail(RNG_ERANGE, "a request needs more than 2^40 chunks");
    H.levels = levels;
    for (uint32_t g = 0; g < H.ngroups; ++g) H.has_xs256 |= H.groups[g].gen == (uint32_t)RNG_XS256;
    H.off_seg = (uint32_t)align16(H.off_reqs + sizeof(BatchReq) * (uint64_t)n);
    uint2 *segs = plan_at<uint2>(&H, H.off_seg);
    const bool pow2 = (C & (C - 1)) == 0;
    const uint32_t lc = (uint32_t)__builtin_ctzll(C);
    uint32_t S = 0, B = 0;
    H.lvl[0] = LevelInfo{};  // level 0 is done by the root kernel: only its table power (small-batch tree)
    H.lvl[0].pow = pow2 && lc + kRadixBits <= 64 ? lc : 0xFFFFFFFFu;
    for (uint32_t l = 1; l < levels; ++l) {
        LevelInfo &L = H.lvl[l];
        L.seg_off = S;
        L.shift = kRadixBits * l;
        L.pow = pow2 && lc + L.shift + kRadixBits <= 64 ? lc + L.shift : 0xFFFFFFFFu;
        L.pad = 0;
        const uint64_t lo = (uint64_t)1 << L.shift, hi = lo << kRadixBits;
        uint64_t acc = 0;
        for (uint32_t r = 0; r < n; ++r) {
            const uint64_t nc = Q[r].nchunks;
            if (nc <= lo) continue;
            segs[S++] = make_uint2(r, (uint32_t)acc);
            acc += std::min(nc, hi) - lo;
        }
        L.seg_n = S - L.seg_off;
        H.level_total[l] = (uint32_t)acc;
    }
    // block starts after all segments: the segment of each level's block's first item
    H.off_blk = (uint32_t)align16(H.off_seg + 8ull * S);
    uint64_t nblk = 0;
    for (uint32_t l = 1; l < levels; ++l) nblk += (H.level_total[l] + kLevelWG - 1) / kLevelWG;
    if (H.off_blk + 4 * nblk > h->plan_cap) return fail(RNG_ENOMEM, "batch plan exceeds its buffer");
    uint32_t *blks = plan_at<uint32_t>(&H, H.off_blk);
    for (uint32_t l = 1; l < levels; ++l) {
        LevelInfo &L = H.lvl[l];
        L.blk_off = B;
        uint32_t k = 0;
        for (uint64_t t0 = 0; t0 < H.level_total[l]; t0 += kLevelWG) {
            while (k + 1 < L.seg_n && segs[L.seg_off + k + 1].y <= t0) ++k;
            blks[B++] = k;
        }
    }
    H.plan_bytes = H.off_blk + 4 * B;
    h->planned = true;
    return RNG_OK;
}

int rng_batch_launch(rng_batch_t *h, void *stream)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    std::lock_guard<std::mutex> lk(h->mu);
    if (!h->planned) return fail(RNG_EINVAL, "rng_batch_set has not been called since the last shape change");
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != h->device) return fail(RNG_EINVAL, "batch created on device %d, current device %d", h->device, dev);
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const BatchHeader &H = h->hdr();
    hipError_t e;
    // a small plan in the root kernel's arguments (direct launches), else the
    // whole plan in one copy
    static thread_local PlanInline pin;
    pin.bytes = 0;
    if (!h->use_graph && H.plan_bytes <= kInlinePlanBytes) {
        pin.bytes = H.plan_bytes;
        std::memcpy(pin.q, h->h_plan, H.plan_bytes);
    } else {
        if ((e = hipMemcpyAsync(h->d_plan, h->h_plan, H.plan_bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(e, "rng_batch_launch: upload");
        if ((e = hipEventRecord(h->copied, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        h->copy_pending = true;
    }

    if (h->occ_wg != h->wg || h->occ_unroll != h->unroll) {
        int per_cu = 0;
        if (batch_gen_occupancy((int)h->wg, (int)h->unroll, &per_cu) || per_cu <= 0) per_cu = 1;
        h->gen_full = (unsigned)(h->num_cu * per_cu);
        h->occ_wg = h->wg;
        h->occ_unroll = h->unroll;
    }
    const unsigned gen_grid = h->gen_full;
    const unsigned level_grid =
        (unsigned)std::min<uint64_t>((chunk_capacity(h, h->C) + kLevelWG - 1) / kLevelWG, 256);
    if (!h->use_graph) {
        // root (and tree level 0), the further tree levels, persistent generation
        const BatchArgs a = make_args(h, tab);
        int rc;
        if (pin.bytes && H.levels <= kSmallTreeLevels && H.n <= kSmallTreeRequests) {
            // the whole tree of each request in one launch instead of 1 + levels - 1
            rc = launch_batch_tree_small(a, pin, H.n, st);
        } else {
            rc = launch_batch_root(a, pin, h->max_requests, st);
            for (uint32_t l = 1; !rc && l < H.levels; ++l) rc = launch_batch_level(a, l, level_grid, st);
        }
        if (!rc) rc = launch_batch_gen(a, (int)h->wg, (int)h->unroll, gen_grid, st);
        return check_launch(rc, "rng_batch_launch");
    }
    rng_batch::Graph *gp = nullptr;
    for (auto &g : h->graphs)
        if (g.levels == H.levels && g.wg == h->wg && g.unroll == h->unroll) gp = &g;
    if (!gp) {
        const BatchArgs a = make_args(h, tab);
        rng_batch::Graph g{H.levels, h->wg, h->unroll, nullptr, nullptr};
        // Recorded on the handle's own stream (the caller's may be the null
        // stream, which cannot capture); nothing runs while recording.
        hipStream_t cs = h->capture;
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        pin.bytes = 0;  // the graph's root kernel reads the uploaded plan
        int rc = launch_batch_root(a, pin, h->max_requests, cs);
        // level 0 (chunks 1..15 of every request) is done by the root kernel
        for (uint32_t l = 1; !rc && l < H.levels; ++l) rc = launch_batch_level(a, l, level_grid, cs);
        if (!rc) rc = launch_batch_gen(a, (int)h->wg, (int)h->unroll, gen_grid, cs);
        e = hipStreamEndCapture(cs, &g.graph);
        if (rc) {
            if (g.graph) (void)hipGraphDestroy(g.graph);
            return check_launch(rc, "rng_batch_launch: capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g.graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        h->graphs.push_back(g);
        gp = &h->graphs.back();
    }
    if ((e = hipGraphLaunch(gp->exec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return RNG_OK;
}

int rng_batch_autotune(rng_batch_t *h, uint32_t reps, uint32_t *best_wg, uint32_t *best_unroll,
                       uint32_t *best_chunk, float *best_us, void *stream)
{
    if (!h || !best_wg || !best_unroll || !best_chunk) return fail(RNG_EINVAL, "NULL argument");
    if (reps == 0) return fail(RNG_EINVAL, "reps is 0");
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (h->last.empty()) return fail(RNG_EINVAL, "no planned batch to tune on");
    }
    // every built shape: workgroups of 64..1024 lanes x unroll 1..16 (the
    // paper chose its block size by occupancy and unrolled its main loop)
    static const uint32_t wgs[] = {64, 128, 256, 512, 1024}, unrolls[] = {1, 2, 4, 8, 16};
    uint32_t shapes[25][2];
    for (int i = 0; i < 25; ++i) {
        shapes[i][0] = wgs[i / 5];
        shapes[i][1] = unrolls[i % 5];
    }
    static const uint32_t chunks[] = {512, 1024, 2048, 4096};
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    float best = 1e30f;
    uint32_t bw = h->wg, bu = h->unroll, bc = (uint32_t)h->C;
    int rc = RNG_OK;
    for (uint32_t c : chunks) {
        for (auto &sh : shapes) {
            if ((rc = rng_batch_set_shape(h, sh[0], sh[1], c))) break;
            if ((rc = rng_batch_launch(h, stream))) break;  // warm-up (and graph capture)
            (void)hipEventRecord(e0, st);
            for (uint32_t r = 0; r < reps && !rc; ++r) rc = rng_batch_launch(h, stream);
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
                bw = sh[0];
                bu = sh[1];
                bc = c;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = rng_batch_set_shape(h, bw, bu, bc))) return rc;
    *best_wg = bw;
    *best_unroll = bu;
    *best_chunk = bc;
    if (best_us) *best_us = best;
    return RNG_OK;
}

}  // extern "C"
