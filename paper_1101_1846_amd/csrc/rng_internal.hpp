// rng_internal.hpp -- interface between the C ABI layer and the per-generator
// kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng_device.hpp"

namespace rngx {

enum { RNG_DT_U32 = 0, RNG_DT_F32 = 1 };

// Samples each lane produces into its LDS tile between two transposed
// stores (the tile is [64][depth + 4] words per wavefront).  Workgroups whose
// tiles would not fit in the 160 KiB of LDS take 32.
#ifndef RNGX_GEN_TILE
#define RNGX_GEN_TILE 128
#endif
constexpr int kGenTile = RNGX_GEN_TILE;

constexpr int gen_tile_depth(int wg) { return wg * (kGenTile + 4) * 4 <= 160 * 1024 ? kGenTile : 32; }

// Chunks per row for XS256 rows of whole 4 KiB multiples on 512- and
// 1024-lane workgroups (measured at 2^20 x 1024: 4 chunks 836 us; 8 chunks,
// with jumps by multiples of 128 samples, 1244 us or more).
constexpr uint32_t kXs256RowChunks = 4;

// Staged store schedule: 1 = whole tile at once, 2 = software-pipelined.
#ifndef RNGX_STORE_MODE
#define RNGX_STORE_MODE 2
#endif
constexpr int kStoreMode = RNGX_STORE_MODE;

// Chunked launches (P > 1 chunks per stream) whose workgroups each hold every
// chunk of their 64-stream groups: the kernel orders the start-state reads
// before the write-back with a barrier.
__host__ __device__ constexpr bool chunks_in_workgroup(uint32_t P, int nw) { return P > 1 && nw % P == 0; }

// Launcher result: launched, but the states were not written back (the
// caller advances them by N with a skip launch).
constexpr int kStatesNotWritten = 1;

// Devices whose launch facts (occupancy) are cached per process.
constexpr int kMaxDevices = 64;

// Resident schedule for one-chunk launches of whole stream groups: a wave
// preloads the states of all its groups before its first store.  The register
// queue holds up to this many groups: enough for 2^20 streams on the waves the
// device holds at once with each shape (4 per CU with 128-deep tiles, 16 with
// 32-deep ones), within the registers each shape leaves.
constexpr int resident_groups(int wg, int depth) { return depth >= 128 ? 16 : (wg >= 1024 ? 4 : 8); }

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
    uint32_t rot;      // rows of whole 4 KiB multiples (all but XS256): rotated tile order (constants below)
    uint32_t seg;      // > 1: rows of 4 or 8 KiB written as runs of seg adjacent rows per lane (if resident)
    DevTables tab;
    uint64_t rot_mwc32[4];     // a^(d N / 4) * 2^64 mod m, d = 0..3
    uint32_t rot_xs32[4][32];  // columns of the xorshift32 M^(d N / 4) (XS32, KISS)
    uint32_t rot_lcg[4][2];    // A, C of d N / 4 LCG steps (KISS); the MWC16 words' constants are built in LDS
};

struct FusedArgs {
    uint32_t *state;
    uint64_t ld;
    uint64_t S, N;
    uint64_t C;  // even chunk length
    uint32_t P;
    uint32_t lanes;  // fewer streams than lanes: lane v takes chunk v mod P of stream v / P
    uint64_t *count;
    DevTables tab;
};

template <class G>
int launch_seed_t(uint64_t seed, uint64_t first, uint64_t S, uint32_t *st, const DevTables &tab,
                  hipStream_t stream);
template <class G>
int launch_tree_level_t(uint32_t *ws, uint64_t T, uint32_t shift, uint64_t unit, const DevTables &tab,
                        hipStream_t stream);
template <class G>
int launch_state_copy_t(const uint32_t *src, uint64_t ss, uint64_t si, uint32_t *dst, uint64_t ds,
                        uint64_t di, hipStream_t stream);
template <class G>
int launch_generate_t(int dt, const GenArgs &a, int wg, int unroll, bool staged, hipStream_t stream);
template <class G>
int launch_fused_pi_t(const FusedArgs &a, hipStream_t stream);

}  // namespace rngx
