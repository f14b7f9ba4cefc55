// rng_internal.hpp -- interface between the C ABI layer and the per-generator
// kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng_device.hpp"

namespace rngx {

enum { RNG_DT_U32 = 0, RNG_DT_F32 = 1 };

// Samples each lane produces into its LDS tile between two transposed
// stores (the tile is [64][kGenTile + 4] words per wavefront).
#ifndef RNGX_GEN_TILE
#define RNGX_GEN_TILE 64
#endif
constexpr int kGenTile = RNGX_GEN_TILE;

// Staged store schedule: 1 = whole tile at once, 2 = software-pipelined.
#ifndef RNGX_STORE_MODE
#define RNGX_STORE_MODE 2
#endif
constexpr int kStoreMode = RNGX_STORE_MODE;

// Resident schedule for one-chunk launches of whole stream groups: a wave
// preloads the states of up to kResidentGroups groups before its first store.
#ifndef RNGX_RESIDENT_GROUPS
#define RNGX_RESIDENT_GROUPS 8
#endif
constexpr int kResidentGroups = RNGX_RESIDENT_GROUPS;

struct GenArgs {
    uint32_t *state;  // [W][ld]
    uint64_t ld;      // state word stride (>= S)
    uint64_t S, N;    // streams, samples per stream
    void *out;        // [S][N]
    uint64_t C;       // chunk length (multiple of kGenTile unless P == 1)
    uint32_t P;       // chunks per stream
    uint32_t vec4;    // rows 16-byte aligned: 128-bit stores
    uint32_t nt;      // non-temporal store hint
    uint32_t resident; // waves stride over 64-stream groups with preloaded states (set by the launcher)
    DevTables tab;
};

struct FusedArgs {
    uint32_t *state;
    uint64_t ld;
    uint64_t S, N;
    uint64_t C;  // even chunk length
    uint32_t P;
    uint64_t *count;
    DevTables tab;
};

template <class G>
int launch_seed_t(uint64_t seed, uint64_t first, uint64_t S, uint32_t *st, const DevTables &tab,
                  hipStream_t stream);
template <class G>
int launch_skip_t(uint32_t *st, uint64_t S, uint64_t k, const DevTables &tab, hipStream_t stream);
template <class G>
int launch_tree_level_t(uint32_t *ws, uint64_t T, uint64_t lo, uint64_t dist, const DevTables &tab,
                        hipStream_t stream);
template <class G>
int launch_state_copy_t(const uint32_t *src, uint64_t ss, uint64_t si, uint32_t *dst, uint64_t ds,
                        uint64_t di, hipStream_t stream);
template <class G>
int launch_generate_t(int dt, const GenArgs &a, int wg, int unroll, bool staged, hipStream_t stream);
template <class G>
int launch_fused_pi_t(const FusedArgs &a, hipStream_t stream);

}  // namespace rngx
