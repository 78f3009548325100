// Host-side view of the gfx950 KmerCo kernels: launch constants, the
// per-handle workspace and the launchers used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc_device.hpp"
#include "kc_profile.hpp"

namespace kc {

constexpr int kTile = 1024;    // positions (or keys) per workgroup of the tile kernels
constexpr int kWG = 256;       // threads per workgroup of the tile kernels
constexpr uint32_t kStatusRange = 1u;  // sticky device status: an output overflowed

// Direct path: positions resolved per first-seen chunk (t = p - c0 < 2^32).
constexpr uint64_t kChunk = 1ull << 31;

// Binned path
constexpr int kBinWG = 512;                  // threads per bin workgroup
constexpr uint64_t kBinTileMin = 65536;      // positions per bin workgroup (at least)
constexpr uint64_t kBinTileFloor = 4096;     // ... for chunks of fewer than kBinSpread tiles
constexpr uint64_t kBinSpread = 2048;        // bin workgroups a small chunk is spread over
constexpr int kRegionWG = 1024;              // threads per region workgroup
constexpr int kRegionCounters = 16384;       // counters per region: hits + first = 128 KiB LDS
constexpr int kSmallRegionCounters = 8192;   // the smaller region choice: 64 KiB
constexpr uint32_t kMaxRegions = 16384;      // LDS histogram of the bin kernels: 64 KiB
constexpr uint64_t kMaxMatrix = 1ull << 25;  // (region, bin workgroup) counts per chunk
constexpr uint64_t kBinChunk = 1ull << 28;   // positions per binned chunk (entries < 2^31)
constexpr uint32_t kMaxBuckets = 64;         // level-1 buckets (groups of regions)
constexpr uint32_t kMaxRegionsPerBucket = kMaxRegions / kMaxBuckets;
constexpr int kStage = 4096;                 // entries staged per batch in LDS: 32 KiB
constexpr uint32_t kStageLog = 12;           // kStage == 1 << kStageLog
constexpr uint32_t kSlice = 32;              // bin workgroups per level-2 workgroup
constexpr int kTileGrid = 2048;              // workgroups of the persistent tile kernels
// Partitioned binned path, for countBFs of more than kMaxRegions regions:
// partition p holds regions [p * kMaxRegions, (p + 1) * kMaxRegions)
constexpr uint32_t kPartLog = 14;            // kMaxRegions == 1 << kPartLog
constexpr uint32_t kMaxParts = 256;          // partitions (4M regions: 64 GB at alpha = 8)
// positions per partitioned chunk: entry offsets and chunk-relative positions
// are 32-bit (chunk * k_h < 2^32, t < 2^32 - 1, the idle first-seen value),
// and a multiple of the largest bin tile; the countBF is read and written
// once per chunk, so an 8 Gbase insert takes two passes over it
constexpr uint64_t kPartChunk = (1ull << 32) - (1ull << 16);
constexpr uint32_t kListWGs = 4096;          // list workgroups over all partitions, about
constexpr uint32_t kMaxListG = 512;          // list workgroups per partition (at most)
constexpr uint64_t kMaxCoarse = 1ull << 19;  // (partition bucket, list workgroup) counts
constexpr int kSuper = 4;                    // tiles per iteration of the tile kernels
constexpr uint32_t kWinCursors = 256 + 256 * 32;  // winner passes: level-A and block cursors

struct BinPlan {
    uint32_t region_shift;  // log2(cells per region)
    uint32_t n_regions;
    uint32_t bucket_shift;  // log2(regions per bucket)
    uint32_t n_buckets;
    uint32_t G;             // bin workgroups of the chunk
    uint32_t slice;         // bin workgroups per level-2 workgroup
    uint32_t n_slices;
    uint64_t tile;          // positions per bin workgroup (multiple of kBinWG)
    uint64_t entries_cap;   // capacity of each entry list
    uint32_t n_parts;       // partitioned path: partitions (0: regions binned directly)
    uint32_t part_log;      // partitioned path: log2(regions per partition) <= kPartLog
    uint32_t region0;       // global index of region 0 of the launch (0 but in tests)
    uint32_t list_g;        // partitioned path: list workgroups per partition
    uint32_t region_counters;  // counters per region (kRegionCounters or kSmallRegionCounters)
};

// Per-handle workspace (device memory owned by the handle).
struct Workspace {
    // per-position buffers of an insert call (cap positions)
    uint32_t *codes = nullptr;    // code_words(cap) 2-bit packed bases
    uint32_t *inv = nullptr;      // mask_words(cap) invalid-base bits
    uint32_t *rs = nullptr;       // mask_words(cap) read-start bits
    uint32_t *valid = nullptr;    // mask_words(cap) valid-window bits (binned paths)
    uint8_t *flags8 = nullptr;    // tiles(cap)*kTile flag bytes
    uint64_t cap = 0;
    // per-tile buffers (tile_cap tiles of positions or keys)
    uint32_t *tile_a = nullptr, *tile_b = nullptr, *tile_c = nullptr;
    uint64_t *off_a = nullptr, *off_b = nullptr, *off_c = nullptr;
    uint64_t *tmask = nullptr;    // tile_cap * kTile / 64 classification bits
    uint64_t *partial64 = nullptr;
    uint64_t tile_cap = 0;
    // binned path (per chunk)
    uint32_t *matrix = nullptr;   // matrix_cap region counts, scanned in place to offsets
    uint32_t *matrix_t = nullptr; // matrix_cap counts as the bin workgroups write them
                                  // (workgroup-major), transposed into matrix
    uint32_t *coarse = nullptr;   // coarse_cap bucket counts, scanned in place to offsets
    uint32_t *partial32 = nullptr;
    uint64_t matrix_cap = 0, coarse_cap = 0;
    uint32_t *slots = nullptr;    // slots_cap slot ids (position-major per hash function)
    uint64_t slots_cap = 0;
    uint64_t *bucketed = nullptr; // entries_cap entries grouped by bucket
    uint64_t *entries = nullptr;  // entries_cap entries grouped by region
    uint64_t entries_cap = 0;
    // partitioned binned path (per chunk): slot ids and partition bytes in
    // `bucketed`, the partition lists in `entries` (see launch_parts_chunk)
    uint32_t *pmat = nullptr;     // pmat_cap (partition, bin workgroup) counts -> offsets
    uint64_t pmat_cap = 0;
    uint32_t *pbounds = nullptr;  // kMaxParts + 1 partition starts in plist
    uint64_t *pdesc = nullptr;    // kMaxParts x (list start, entries, list tile)
    // scalars
    uint64_t *totals = nullptr;   // 8 scan totals / saved counters
    uint32_t *n_entries = nullptr;  // 4 entry totals
    uint32_t *win_cursors = nullptr;  // kWinCursors: the winner passes' bucket cursors
    // carried first-seen records (classification by the last chunk's region
    // pass): chunk j < last keeps its records (t, local counter) at
    // [j * carry_cap + region offset) of two arrays, 32-bit t words then
    // 16-bit halves, and each region's offset and record count at
    // [j * carry_regions + region) of carry_off and carry_n
    uint16_t *carry = nullptr;    // 3 * carry_cap halves: the words, then the halves
    uint64_t carry_cap = 0;       // records per carried chunk x carried chunks
    uint32_t *carry_off = nullptr;
    uint32_t *carry_n = nullptr;
    uint64_t carry_idx_cap = 0;   // regions x carried chunks
    // the buffers were carved from caller memory once: they never grow, and a
    // call that needs more than they hold fails instead
    bool fixed = false;
};

inline uint64_t tiles(uint64_t n) { return (n + kTile - 1) / kTile; }

// Exclusive sum over a workgroup of kWG threads; `total` receives the sum.
// Every thread of the workgroup must call it (it synchronises).
__device__ __forceinline__ uint32_t wg_exclusive_u32(uint32_t v, uint32_t *s_wave,
                                                     uint32_t &total) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    uint32_t incl = v;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += o;
    }
    if (lane == 63)
        s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (uint32_t w = 0; w < kWG / 64; w++) {
        const uint32_t t = s_wave[w];
        if (w < wave)
            before += t;
        total += t;
    }
    __syncthreads();
    return before + incl - v;
}
// Exclusive sum over one wavefront (lane = threadIdx.x & 63); `total`
// receives the wavefront's sum on every lane.
__device__ __forceinline__ uint32_t wave_exclusive(uint32_t v, uint32_t lane, uint32_t &total) {
    uint32_t incl = v;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += o;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}

// The flagged positions among a lane's 16 flag bytes x (flags are 0, 1 =
// distinct or 3 = distinct and trustworthy; byte i is tile position
// 16 lane + i), in position order: entry rd, rd + 1, ... of lpos gets the
// tile position and of ltb the trustworthy count before it (from rt) with
// bit 15 set for a trustworthy one.  Bit 0 and bit 1 of the bytes are
// gathered into 16-bit masks four bytes at a time by one multiply (bits 0,
// 8, 16, 24 -> bits 21..24), and only the set bits are visited.
__device__ __forceinline__ void list_flags(const uint32_t (&x)[4], uint32_t lane, uint32_t rd,
                                           uint32_t rt, uint16_t *lpos, uint16_t *ltb) {
    uint32_t m16 = 0, t16 = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        m16 |= (((x[u] & 0x01010101u) * 0x204081u) >> 21 & 0xFu) << (4 * u);
        t16 |= ((((x[u] >> 1) & 0x01010101u) * 0x204081u) >> 21 & 0xFu) << (4 * u);
    }
    while (m16) {
        const uint32_t b = (uint32_t)__builtin_ctz(m16);
        m16 &= m16 - 1u;
        const uint32_t tr = (t16 >> b) & 1u;
        lpos[rd] = (uint16_t)(16u * lane + b);
        ltb[rd] = (uint16_t)(rt | (tr << 15));
        rd++;
        rt += tr;
    }
}

inline uint64_t mask_words(uint64_t n) { return tiles(n) * (kTile / 32) + 2; }
inline uint64_t code_words(uint64_t n) { return tiles(n) * (kTile / 16) + 4; }

// Phase ids for the profiler (same values as kc_phase in kmerco.h).
enum Phase {
    kPhIngest = 0, kPhClaim, kPhIncrement, kPhClaimIncrement, kPhResolve, kPhScan, kPhScatter,
    kPhClassifyMark, kPhClassifyScatter, kPhQuery, kPhReset, kPhBinCount, kPhBinBucket, kPhRegion,
    kPhTileCount, kPhBinRegion, kPhBinPart, kPhPartCount, kPhValid, kPhWinners, kPhCount
};

hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// out[c * rows + r] = in[r * cols + c]: a rows x cols matrix, row-major, to
// its transpose (rows / 64 <= 65535)
hipError_t transpose_u32(const uint32_t *in, uint32_t *out, uint64_t rows, uint64_t cols,
                         hipStream_t s);
// The same for consecutive rows x cols blocks of a rows x total_cols matrix
// stored block by block (block z: columns z*cols .. , the last one cut at
// total_cols); out is the total_cols x rows transpose.
hipError_t transpose_u32_blocks(const uint32_t *in, uint32_t *out, uint64_t rows, uint64_t cols,
                                uint64_t total_cols, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);

uint64_t scan_partials(uint64_t n);
hipError_t scan_u32_u64(const uint32_t *in, uint64_t *out, uint64_t n, const uint64_t *base,
                        uint64_t *total, uint64_t *partial, hipStream_t s);
hipError_t scan_u32_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total,
                        uint32_t *partial, hipStream_t s);

hipError_t launch_ingest(const uint8_t *reads, uint64_t n_bases, const uint64_t *offsets,
                         uint64_t n_reads, const Workspace &W, hipStream_t s, Profiler *P);
// The valid-window bitmap of k-base windows into W.valid (binned paths),
// from the bitmaps launch_ingest wrote.
hipError_t launch_valid_windows(uint64_t n_bases, uint32_t k, const Workspace &W, hipStream_t s,
                                Profiler *P);
hipError_t launch_insert_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                               bool zero_filter, const Workspace &W, hipStream_t s, Profiler *P);
// Binned-path plan for chunks of chunk_positions; false when the countBF
// has too many regions even for the partitioned path.  part_log sets the
// partition size (regions) for countBFs of more than 2^part_log regions.
bool bin_plan(const FilterArgs &F, uint64_t chunk_positions, BinPlan &B,
              uint32_t part_log = kPartLog, uint32_t region_counters = kRegionCounters);
// Carried classification of a multi-chunk insert with one hash function:
// the region passes of the chunks before the last keep their first-seen
// records (Carry::kOut, chunk j of the carry arrays) instead of writing
// flags; the last chunk's region pass (Carry::kIn, chunks 0 .. n_prev - 1)
// marks each carried record trustworthy or not from its counter's final
// value, and the winner passes then write every carried chunk's flags.
struct Carry {
    enum Mode : uint32_t { kNone = 0, kOut = 1, kIn = 2 };
    uint32_t mode = kNone;
    uint32_t chunk = 0;          // kOut: this chunk's index j
    uint32_t n_prev = 0;         // kIn: carried chunks
    uint32_t stride = 0;         // regions per carried chunk in carry_off / carry_n
    uint64_t cap = 0;            // records per carried chunk
    uint32_t *word = nullptr;    // t words of chunk 0 (chunk j at + j * cap)
    uint16_t *half = nullptr;    // local counters, then marks, of chunk 0
    uint32_t *off = nullptr;     // region offsets of chunk 0 (chunk j at + j * stride)
    uint32_t *n = nullptr;       // region record counts of chunk 0
};
// The carry arrays of W viewed for n_chunks chunks of chunk_positions (k_h
// = 1), or a kNone carry when W does not hold them.
Carry carry_of(const Workspace &W, const BinPlan &plan, uint64_t chunk_positions,
               uint64_t n_chunks);
// Whether a plan's regions can take the carried classification: their cells
// fit the region pass's staged-cell array (eta >= 8).
bool carry_fits(const BinPlan &plan);
// plan.n_parts > 0 takes the partitioned path
hipError_t launch_binned_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                               const BinPlan &plan, const Workspace &W, bool classify,
                               uint32_t tau, const Carry &carry, hipStream_t s, Profiler *P);
// The winner passes of carried chunk j (positions [c0, c0 + len)) after the
// last chunk's region pass has marked its records.
hipError_t launch_carried_winners(const BinPlan &plan, const Carry &carry, uint32_t j, uint64_t c0,
                                  uint64_t len, const Workspace &W, hipStream_t s, Profiler *P);
// windows_counted: the insert passes already added this call's valid-window
// count to W.totals[5] (else the tile pass counts them)
hipError_t launch_distinct(const ReadsArgs &R, const Workspace &W, uint64_t *distinct,
                           uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows,
                           uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                           uint64_t cap_te, uint32_t *status, bool windows_counted,
                           hipStream_t s, Profiler *P);
hipError_t launch_classify(const FilterArgs &F, const uint64_t *keys, const uint64_t *n_keys,
                           const uint64_t *key_base, uint64_t grid_cap, uint64_t cap,
                           uint32_t tau, uint64_t *trust, uint64_t *n_trust, uint64_t *err,
                           uint64_t *n_err, uint64_t cap_out, uint32_t *status,
                           const Workspace &W, hipStream_t s, Profiler *P, bool wide = false);
// Marks the distinct flags of positions [0, n_positions) (a multiple of
// kTile, or the call's end) trustworthy where the k-mer's frequency in the
// countBF is above tau (Query-II), so that launch_distinct splits the list.
hipError_t launch_classify_flags(const FilterArgs &F, const ReadsArgs &R, const Workspace &W,
                                 uint64_t n_positions, uint32_t tau, hipStream_t s, Profiler *P);
// wide: keys of 33..64 bases, (low, high) word pairs
hipError_t launch_query(const FilterArgs &F, const uint64_t *keys, uint64_t n, uint32_t *freq,
                        hipStream_t s, Profiler *P, bool wide = false);

}  // namespace kc
