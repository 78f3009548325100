// Host-side view of the gfx950 KmerCo kernels: launch constants, the
// per-handle workspace and the launchers used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc_device.hpp"
#include "kc_profile.hpp"

namespace kc {

constexpr int kTile = 1024;    // positions (or keys) per workgroup
constexpr int kWG = 256;       // threads per workgroup (4 wavefronts of 64)
constexpr int kScanWG = 1024;  // threads of the single-workgroup scan
constexpr uint32_t kStatusRange = 1u;  // sticky device status: an output overflowed

// Largest chunk of positions resolved at once: occurrence indices t = p - c0
// must stay below kIdle.  A multiple of kTile.
constexpr uint64_t kChunk = 1ull << 31;

// Per-call workspace (device memory owned by the handle).
struct Workspace {
    uint32_t *codes = nullptr;    // code_words(cap) 2-bit packed bases
    uint32_t *inv = nullptr;      // mask_words(cap) invalid-base bits
    uint32_t *rs = nullptr;       // mask_words(cap) read-start bits
    uint64_t *flags = nullptr;    // flag_words(cap) distinct / trustworthy bits
    uint32_t *tile_a = nullptr;   // tiles(cap) per-tile counts
    uint32_t *tile_b = nullptr;   // tiles(cap) per-tile counts
    uint64_t *tile_off = nullptr; // tiles(cap) scanned offsets
    uint64_t *totals = nullptr;   // 2 scan totals
    uint64_t cap = 0;             // positions (bases or keys) the buffers hold
};

inline uint64_t tiles(uint64_t n) { return (n + kTile - 1) / kTile; }
inline uint64_t mask_words(uint64_t n) { return tiles(n) * (kTile / 32) + 2; }
inline uint64_t code_words(uint64_t n) { return tiles(n) * (kTile / 16) + 4; }
inline uint64_t flag_words(uint64_t n) { return tiles(n) * (kTile / 64); }

hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);

// Phase ids for the profiler (same values as kc_phase in kmerco.h).
enum Phase {
    kPhIngest = 0, kPhClaim, kPhIncrement, kPhClaimIncrement, kPhResolve, kPhScan, kPhScatter,
    kPhClassifyMark, kPhClassifyScatter, kPhQuery, kPhReset, kPhCount
};

hipError_t launch_ingest(const uint8_t *reads, uint64_t n_bases, const uint64_t *offsets,
                         uint64_t n_reads, const Workspace &W, hipStream_t s, Profiler *P);
hipError_t launch_insert_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                               bool zero_filter, const Workspace &W, hipStream_t s, Profiler *P);
hipError_t launch_distinct(const ReadsArgs &R, const Workspace &W, uint64_t *distinct,
                           uint64_t cap, uint64_t *n_distinct, uint64_t *n_windows,
                           uint32_t *status, hipStream_t s, Profiler *P);
hipError_t launch_classify(const FilterArgs &F, const uint64_t *keys, const uint64_t *n_keys,
                           uint64_t cap, uint32_t tau, uint64_t *trust, uint64_t *n_trust,
                           uint64_t *err, uint64_t *n_err, const Workspace &W, hipStream_t s,
                           Profiler *P);
hipError_t launch_query(const FilterArgs &F, const uint64_t *keys, uint64_t n, uint32_t *freq,
                        hipStream_t s, Profiler *P);

}  // namespace kc
