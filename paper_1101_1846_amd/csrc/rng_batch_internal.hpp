// rng_batch_internal.hpp -- device-side layout of a batch of independent
// generation requests (shared by the host planner and the batch kernels).
//
// Every request is cut into chunks of C samples (the last one shorter).
// Requests are grouped by (generator, dtype); inside a group the chunks of
// all its requests are numbered consecutively and padded to whole 64-lane
// tiles.  Chunk states live in a structure-of-arrays workspace per group.
#pragma once
#include <stdint.h>

#include "rng_device.hpp"

namespace rngx {

constexpr int kBatchMaxGroups = 10;   // 5 generators x 2 dtypes
constexpr int kBatchMaxLevels = 10;   // radix-16 tree levels (chunks per request < 2^40)
constexpr int kBatchTile = 64;        // LDS tile depth of the batch kernel

struct BatchReq {
    uint32_t *state;      // word 0 of the stream's state
    uint64_t stride;      // word stride of that state
    uint64_t offset;      // samples skipped before the first output
    uint64_t length;      // samples produced
    uint32_t *out;        // [length]
    uint32_t chunk_base;  // index of the first chunk inside the group
    uint32_t nchunks;     // ceil(length / C)
    uint32_t group;
    uint32_t pad;
};

struct BatchGroup {
    uint32_t gen, dtype, words;
    uint32_t req_begin, req_end;  // requests [req_begin, req_end) of the sorted table
    uint32_t nchunks;             // chunks of the group
    uint32_t nchunks_pad;         // rounded up to whole tiles (SoA stride)
    uint32_t tile_begin, tile_end;
    uint32_t pad;
    uint64_t ws_off;              // word offset of the group's [words][nchunks_pad] states
};

// Work list of one level of the radix-16 tree that gives every chunk its
// start state.  Level l covers the chunks j in [16^l, 16^(l+1)) of every
// request with more than 16^l chunks: with j = q 16^l + r (q in 1..15,
// r < 16^l), chunk j starts where chunk r starts, jumped by q 16^l C samples
// (level 0, chunk j < 16 from chunk 0 by j C, is done by the root kernel and
// has no work list).  Those requests are the level's segments, in table order, each with the exclusive prefix of the
// work items before it.  Items are handled in blocks of kLevelWG; the block
// start table gives the segment holding each block's first item, so that a
// block needs only its kLevelWG following segments.
constexpr int kRadixBits = 4;    // 16-way levels: up to 4 jumps by powers of two per chunk
constexpr int kLevelWG = 1024;   // lanes (and work items) per level workgroup

struct LevelInfo {
    uint32_t seg_off;  // first segment of the level in the segment array
    uint32_t seg_n;    // segments (requests with more than 16^l chunks)
    uint32_t blk_off;  // first entry of the level in the block start array
    uint32_t shift;    // 4 l
    uint32_t pow;      // b with C 16^l = 2^b, or 0xFFFFFFFF when C is no power of two
    uint32_t pad;
};

// Per-batch header, rewritten before every launch (the captured graph only
// holds a pointer to it).  It heads the packed plan that one copy uploads:
// the header, then the request table, the level segments and the block
// starts, each at the byte offset the header gives (16-byte aligned).
struct BatchHeader {
    uint64_t C;           // chunk length
    uint32_t n;           // requests
    uint32_t ngroups;
    uint32_t n_tiles;
    uint32_t levels;      // radix-16 tree levels used
    uint32_t has_xs256;   // some group is XS256 (its level's four tables are staged in LDS)
    uint32_t off_reqs;    // BatchReq [n], sorted by group
    uint32_t off_seg;     // uint2 level segments: (sorted request index, exclusive item prefix)
    uint32_t off_blk;     // uint32 per level and kLevelWG-item block: segment (within the level) of its first item
    uint32_t plan_bytes;  // bytes of the packed plan
    uint32_t pad;
    uint32_t level_total[kBatchMaxLevels];  // work items per level
    LevelInfo lvl[kBatchMaxLevels];
    BatchGroup groups[kBatchMaxGroups];
};

// Plans of at most kInlinePlanBytes travel in the root kernel's arguments
// instead of an upload (direct launches only: a captured graph keeps the
// arguments it was recorded with).  The root kernel reads the plan there, and
// its first workgroup writes it to the device plan buffer for the kernels
// that follow it on the stream.  This saves the copy and the wait for it.
constexpr uint32_t kInlinePlanBytes = 2048;

// Small plans whose requests need at most kSmallTreeLevels radix-16 levels
// (16^3 chunks) and that hold at most kSmallTreeRequests requests build every
// request's tree in one launch, four workgroups per request
// (k_batch_tree_small).
constexpr uint32_t kSmallTreeLevels = 3;
constexpr uint32_t kSmallTreeRequests = 64;

struct PlanInline {
    uint32_t bytes;  // 0: the plan was uploaded to BatchArgs::hdr
    uint32_t pad[3];
    uint4 q[kInlinePlanBytes / 16];
};

struct BatchArgs {
    const BatchHeader *hdr;       // the packed plan
    uint32_t *chunk_req;          // [64 * n_tiles] sorted request index of every chunk (padded group order)
    uint32_t *ws;                 // chunk-state workspace
    uint32_t *counter;            // [0] tile counter of the persistent kernel
    DevTables tab;
};

template <class T>
__host__ __device__ inline T *plan_at(const BatchHeader *p, uint32_t off)
{
    return (T *)((const char *)p + off);
}

}  // namespace rngx
