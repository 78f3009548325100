// Batched insertion (many read sets, each with its own countBF) -- host view.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc_device.hpp"
#include "kc_kernels.hpp"

namespace kc {

constexpr uint64_t kSetAlign = (uint64_t)kSuper * kTile;  // set bases: multiples of 4096
constexpr uint32_t kBatchMaxRegions = 2048;                // regions of one set's filter
constexpr uint32_t kNoSet = 0xFFFFFFFFu;                   // tile owned by no set (padding)

// One read set of a batch, as the kernels see it.
struct SetDesc {
    FilterArgs F;             // the set's countBF
    uint64_t base;            // first position (multiple of kSetAlign)
    uint64_t n_bases;
    uint64_t slot_base;       // first slot id of the set (slot ids are per set, per hash fn)
    uint64_t mat_base;        // first count of the set's block (n_regions x G)
    uint32_t k, tau;
    uint32_t region_shift, n_regions;
    uint32_t region_base;     // global index of the set's first region
    uint32_t G;               // work items of the set
    uint32_t item_base;       // global index of the set's first work item
    uint32_t fused;           // the split is taken from the region pass
    uint64_t *distinct;
    uint64_t cap_d;
    uint64_t *n_distinct;
    uint64_t *n_windows;
    uint64_t *trust, *n_trust, *err, *n_err;
    uint64_t cap_te;
    uint32_t *status;         // the filter's sticky status
};

struct BatchPlan {
    uint32_t n_sets;
    uint32_t n_items;
    uint64_t tile;            // positions per work item (multiple of kBinWG)
    uint64_t n_matrix;        // total counts of all sets' blocks
    uint32_t n_regions;       // total regions of all sets
    uint32_t max_G;           // most work items of one set
    uint32_t max_regions;     // most regions of one set
    uint64_t n_tiles;         // 1024-position tiles of the whole buffer
    uint64_t n_slots;
    uint64_t entries_cap;
    uint32_t fast;            // every set has the hashing kernel's fast layout
};

struct BatchBuffers {
    SetDesc *sets = nullptr;          // device copy of the descriptors
    uint32_t *item_set = nullptr;     // set of each work item
    uint32_t *region_set = nullptr;   // set of each region
    uint32_t *tile_set = nullptr;     // set of each tile (kNoSet for padding)
    uint32_t *slots = nullptr;
    uint32_t *matrix = nullptr;       // per set: region-major counts, scanned to offsets
    uint32_t *matrix_t = nullptr;     // per set: the work items' counts, one row per item
    uint32_t *partial32 = nullptr;
    uint32_t *n_entries = nullptr;
    uint64_t *entries = nullptr;
    unsigned long long *valid = nullptr;  // valid windows per set
    uint64_t *saved = nullptr;        // per set: distinct count at the start of the call
    Workspace *W = nullptr;           // per-position and per-tile buffers
};

hipError_t launch_tile_count(const ReadsArgs &R, const Workspace &W, uint64_t n_tiles,
                             hipStream_t s);
hipError_t launch_batch_bins(const BatchPlan &bp, const BatchBuffers &Bf, const ReadsArgs &R,
                             hipStream_t s, Profiler *P);
hipError_t launch_batch(const BatchPlan &bp, const BatchBuffers &Bf, const ReadsArgs &R,
                        bool reset, hipStream_t s, Profiler *P);
hipError_t launch_save_bases(const BatchBuffers &Bf, uint32_t n_sets, hipStream_t s);

}  // namespace kc
