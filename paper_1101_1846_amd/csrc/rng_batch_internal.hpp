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
constexpr int kBatchMaxLevels = 40;   // doubling-tree levels (chunks per request < 2^40)
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

// Per-batch header, rewritten before every launch (the captured graph only
// holds pointers to it).
struct BatchHeader {
    uint64_t C;           // chunk length
    uint32_t n;           // requests
    uint32_t ngroups;
    uint32_t n_tiles;
    uint32_t levels;      // doubling-tree levels used
    uint32_t level_total[kBatchMaxLevels];  // work items per level
    BatchGroup groups[kBatchMaxGroups];
};

struct BatchArgs {
    const BatchHeader *hdr;
    const BatchReq *reqs;          // [n], sorted by group
    const uint32_t *level_prefix;  // [levels][n + 1] exclusive prefix of per-request work per level
    uint32_t max_requests;         // row stride of level_prefix is max_requests + 1
    uint32_t *ws;                  // chunk-state workspace
    uint32_t *counter;             // [0] tile counter of the persistent kernel
    DevTables tab;
};

}  // namespace rngx
