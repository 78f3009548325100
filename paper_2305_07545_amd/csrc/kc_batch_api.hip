// C ABI of the batched form (declared in include/kmerco.h): many read sets,
// each with its own countBF, inserted (and classified) by one launch per
// phase; optional HIP-graph capture and replay; work-item size autotuning.
//
// Sets the fused phase kernels cannot take (a countBF of more than
// kBatchMaxRegions regions, more than kBinChunk bases, or k > 32) run the
// single-set pipeline over their range of the batch's ingested buffer, on up
// to kSideLanes side streams forked from the call's stream after the ingest
// and joined before the call ends, each lane with a workspace of its own, so
// that they overlap each other and the fused phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "kc_batched.hpp"
#include "kc_bin_hash.hpp"
#include "kc_handle.hpp"
#include "kc_kernels.hpp"
#include "kmerco.h"

using namespace kcapi;

constexpr int kSideLanes = 3;

struct kc_batch {
    int device = 0;
    kc::Workspace W;
    // side lanes for the sets of the single-set pipeline
    hipStream_t side[kSideLanes] = {};
    hipEvent_t forked = nullptr, joined[kSideLanes] = {};
    kc::Workspace side_ws[kSideLanes];
    uint8_t *stage = nullptr;        // pinned staging of the plan's tables
    uint64_t stage_cap = 0;
    hipEvent_t staged = nullptr;     // the last upload from it
    std::vector<uint32_t> big;       // the call's sets of the single-set pipeline
    std::vector<int> big_lane;       // their lanes
    uint32_t lanes_used = 0;
    kc::BatchBuffers B;
    uint64_t cap_sets = 0, cap_items = 0, cap_regions = 0, cap_tiles = 0, cap_slots = 0,
             cap_matrix = 0, cap_entries = 0;
    std::vector<kc::SetDesc> h_sets;
    std::vector<uint32_t> h_items, h_regions, h_tiles;
    uint64_t tile = 65536;           // positions per work item (autotuned)
    hipStream_t last = nullptr;
    // graph of the last KC_BATCH_GRAPH call and the arguments it was built for
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint8_t> graph_key;
    kc::Profiler prof;
};

namespace {

constexpr uint64_t kTileCandidates[] = {16384, 32768, 65536, 131072, 262144};

// Whether the fused phase kernels take a set (else the single-set pipeline).
bool fused_form(const kc_set &q) {
    kc::BinPlan bp{};
    return q.k <= 32 && q.n_bases <= kc::kBinChunk && kc::bin_plan(q.filter->F, q.n_bases, bp) &&
           bp.n_regions <= kc::kBatchMaxRegions;
}


void free_batch_buffers(kc_batch *b) {
    kc::BatchBuffers &B = b->B;
    dev_free(B.sets);
    dev_free(B.item_set);
    dev_free(B.region_set);
    dev_free(B.tile_set);
    dev_free(B.slots);
    dev_free(B.matrix);
    dev_free(B.matrix_t);
    dev_free(B.partial32);
    dev_free(B.n_entries);
    dev_free(B.entries);
    dev_free(B.valid);
    dev_free(B.saved);
    b->cap_sets = b->cap_items = b->cap_regions = b->cap_tiles = b->cap_slots = b->cap_matrix =
        b->cap_entries = 0;
}

void drop_graph(kc_batch *b) {
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
}

template <typename T>
kc_status grow(T **p, uint64_t &cap, uint64_t need) {
    if (*p && need <= cap)
        return KC_OK;
    dev_free(*p);
    cap = 0;
    uint64_t n = need + need / 8 + 16;
    if (!dev_alloc(p, n))
        return KC_ENOMEM;
    cap = n;
    return KC_OK;
}

// Plan of a batch for work-item size `tile`: descriptors, work items, regions,
// tile owners, sizes.
kc::BatchPlan make_plan(kc_batch *b, const kc_set *sets, uint32_t n_sets, uint64_t n_bases,
                        uint64_t tile) {
    kc::BatchPlan P{};
    P.tile = tile;
    P.n_tiles = kc::tiles(n_bases);
    P.fast = 1;
    b->h_sets.clear();
    b->h_items.clear();
    b->h_regions.clear();
    b->h_tiles.assign(P.n_tiles + kc::kSuper, kc::kNoSet);
    uint64_t mat = 0, slot = 0;
    uint32_t reg = 0, item = 0;
    for (uint32_t i = 0; i < n_sets; i++) {
        const kc_set &q = sets[i];
        if (q.n_bases == 0 || !fused_form(q))
            continue;
        kc_filter *f = q.filter;
        kc::BinPlan bp{};
        (void)kc::bin_plan(f->F, q.n_bases, bp);  // validated by the caller
        kc::SetDesc d{};
        d.F = f->F;
        if (!kc::fast_layout(f->F))
            P.fast = 0;
        d.base = q.first_base;
        d.n_bases = q.n_bases;
        d.slot_base = slot;
        d.mat_base = mat;
        d.k = q.k;
        d.tau = q.tau;
        d.region_shift = bp.region_shift;
        d.n_regions = bp.n_regions;
        d.region_base = reg;
        d.G = (uint32_t)((q.n_bases + tile - 1) / tile);
        d.item_base = item;
        d.fused = (q.trust_dev && f->F.k_h == 1) ? 1u : 0u;
        d.distinct = q.distinct_dev;
        d.cap_d = q.distinct_cap;
        d.n_distinct = q.n_distinct_dev;
        d.n_windows = q.n_windows_dev;
        d.trust = q.trust_dev;
        d.n_trust = q.n_trust_dev;
        d.err = q.err_dev;
        d.n_err = q.n_err_dev;
        d.cap_te = q.class_cap;
        d.status = f->status;
        const uint32_t s = (uint32_t)b->h_sets.size();
        b->h_sets.push_back(d);
        for (uint32_t j = 0; j < d.G; j++)
            b->h_items.push_back(s);
        for (uint32_t r = 0; r < d.n_regions; r++)
            b->h_regions.push_back(s);
        const uint64_t t0 = q.first_base / kc::kTile;
        const uint64_t t1 = kc::tiles(q.first_base + q.n_bases);
        for (uint64_t t = t0; t < t1; t++)
            b->h_tiles[t] = s;
        item += d.G;
        reg += d.n_regions;
        P.max_G = d.G > P.max_G ? d.G : P.max_G;
        P.max_regions = d.n_regions > P.max_regions ? d.n_regions : P.max_regions;
        mat += (uint64_t)d.n_regions * d.G;
        slot += (q.n_bases * f->F.k_h + 3u) & ~3ull;  // slot bases stay 16-byte aligned
    }
    P.n_sets = (uint32_t)b->h_sets.size();
    P.n_items = item;
    P.n_regions = reg;
    P.n_matrix = mat;
    P.n_slots = slot;
    P.entries_cap = slot;
    return P;
}

kc_status ensure_batch(kc_batch *b, const kc::BatchPlan &P, hipStream_t s) {
    kc::BatchBuffers &B = b->B;
    if (B.sets && P.n_sets <= b->cap_sets && P.n_items <= b->cap_items &&
        P.n_regions <= b->cap_regions && b->h_tiles.size() <= b->cap_tiles &&
        P.n_slots <= b->cap_slots && P.n_matrix <= b->cap_matrix && P.entries_cap <= b->cap_entries)
        return KC_OK;
    (void)hipStreamSynchronize(s);
    drop_graph(b);
    kc_status st = KC_OK;
    uint64_t c_sets = b->cap_sets, c_tmp;
    if ((st = grow(&B.sets, c_sets, P.n_sets)) != KC_OK)
        return st;
    c_tmp = c_sets;
    dev_free(B.valid);
    dev_free(B.saved);
    if (!dev_alloc(&B.valid, c_tmp) || !dev_alloc(&B.saved, c_tmp))
        return KC_ENOMEM;
    b->cap_sets = c_sets;
    if ((st = grow(&B.item_set, b->cap_items, P.n_items)) != KC_OK ||
        (st = grow(&B.region_set, b->cap_regions, P.n_regions)) != KC_OK ||
        (st = grow(&B.tile_set, b->cap_tiles, b->h_tiles.size())) != KC_OK ||
        (st = grow(&B.slots, b->cap_slots, P.n_slots)) != KC_OK ||
        (st = grow(&B.entries, b->cap_entries, P.entries_cap)) != KC_OK)
        return st;
    if (!B.matrix || P.n_matrix > b->cap_matrix) {
        dev_free(B.matrix);
        dev_free(B.matrix_t);
        dev_free(B.partial32);
        b->cap_matrix = 0;
        uint64_t n = P.n_matrix + P.n_matrix / 8 + 16;
        if (!dev_alloc(&B.matrix, n) || !dev_alloc(&B.matrix_t, n) ||
            !dev_alloc(&B.partial32, kc::scan_partials(n)))
            return KC_ENOMEM;
        b->cap_matrix = n;
    }
    if (!B.n_entries && !dev_alloc(&B.n_entries, 2))
        return KC_ENOMEM;
    return KC_OK;
}

// The plan's tables to the device through pinned staging: the copies are
// asynchronous, and only a later upload waits for them (before it rewrites
// the staging), so that the host never waits for the stream here.
kc_status upload(kc_batch *b, const kc::BatchPlan &P, hipStream_t s) {
    kc::BatchBuffers &B = b->B;
    const uint64_t b_sets = P.n_sets * sizeof(kc::SetDesc);
    const uint64_t b_items = P.n_items * sizeof(uint32_t);
    const uint64_t b_regions = P.n_regions * sizeof(uint32_t);
    const uint64_t b_tiles = b->h_tiles.size() * sizeof(uint32_t);
    const uint64_t need = b_sets + b_items + b_regions + b_tiles;
    if (b->staged && hipEventSynchronize(b->staged) != hipSuccess)
        return KC_EDEVICE;
    if (need > b->stage_cap) {
        if (b->stage)
            (void)hipHostFree(b->stage);
        b->stage = nullptr;
        b->stage_cap = 0;
        const uint64_t cap = need + need / 4 + 4096;
        if (hipHostMalloc((void **)&b->stage, cap, hipHostMallocDefault) != hipSuccess)
            return KC_ENOMEM;
        b->stage_cap = cap;
    }
    if (!b->staged && hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess)
        return KC_EDEVICE;
    uint8_t *h = b->stage;
    std::memcpy(h, b->h_sets.data(), b_sets);
    std::memcpy(h + b_sets, b->h_items.data(), b_items);
    std::memcpy(h + b_sets + b_items, b->h_regions.data(), b_regions);
    std::memcpy(h + b_sets + b_items + b_regions, b->h_tiles.data(), b_tiles);
    hipError_t e = hipMemcpyAsync(B.sets, h, b_sets, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && P.n_items)
        e = hipMemcpyAsync(B.item_set, h + b_sets, b_items, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && P.n_regions)
        e = hipMemcpyAsync(B.region_set, h + b_sets + b_items, b_regions, hipMemcpyHostToDevice,
                           s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.tile_set, h + b_sets + b_items + b_regions, b_tiles,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipEventRecord(b->staged, s);
    return e == hipSuccess ? KC_OK : KC_EDEVICE;
}

// The call's sets of the single-set pipeline (and its empty sets, which only
// reset and zero their outputs), largest first, each on the least loaded
// side lane; their lanes' workspaces are sized for them (this may allocate,
// and waits for a lane's earlier work before its workspace moves).
kc_status plan_side(kc_batch *b, const kc_set *sets, uint32_t n_sets) {
    b->big.clear();
    b->big_lane.clear();
    b->lanes_used = 0;
    for (uint32_t i = 0; i < n_sets; i++)
        if (sets[i].n_bases == 0 || !fused_form(sets[i]))
            b->big.push_back(i);
    if (b->big.empty())
        return KC_OK;
    std::stable_sort(b->big.begin(), b->big.end(), [&](uint32_t x, uint32_t y) {
        return sets[x].n_bases > sets[y].n_bases;
    });
    uint64_t load[kSideLanes] = {};
    for (uint32_t i : b->big) {
        int l = 0;
        for (int j = 1; j < kSideLanes; j++)
            if (load[j] < load[l])
                l = j;
        load[l] += sets[i].n_bases + 1;
        b->big_lane.push_back(l);
        if ((uint32_t)l + 1 > b->lanes_used)
            b->lanes_used = (uint32_t)l + 1;
    }
    if (!b->forked && hipEventCreateWithFlags(&b->forked, hipEventDisableTiming) != hipSuccess)
        return KC_EDEVICE;
    for (uint32_t l = 0; l < b->lanes_used; l++) {
        // default priority (the streams of one process share the hardware
        // queues fairly)
        if (!b->side[l] && hipStreamCreateWithFlags(&b->side[l], hipStreamNonBlocking) != hipSuccess)
            return KC_EDEVICE;
        if (!b->joined[l] &&
            hipEventCreateWithFlags(&b->joined[l], hipEventDisableTiming) != hipSuccess)
            return KC_EDEVICE;
    }
    for (size_t j = 0; j < b->big.size(); j++) {
        kc_filter *f = sets[b->big[j]].filter;
        const int l = b->big_lane[j];
        kc::Workspace *own = f->W;
        f->W = &b->side_ws[l];
        f->last = b->side[l];
        const kc_status st = prepare_range(f, sets[b->big[j]].n_bases);
        f->W = own;
        if (st != KC_OK)
            return st;
    }
    return KC_OK;
}

// Launch sequence of one call: the ingest of the whole buffer; the side
// lanes' sets forked after it; the fused phases and the per-set split of the
// sets the region pass cannot classify; the join.
kc_status launch_all(kc_batch *b, const kc::BatchPlan &P, const kc_set *sets, uint32_t n_sets,
                     const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads,
                     uint64_t n_bases, bool reset, bool replayed, hipStream_t s,
                     kc::Profiler *prof) {
    hipError_t e = kc::launch_ingest(reads, n_bases, offsets, n_reads, b->W, s, prof);
    if (e != hipSuccess)
        return KC_EDEVICE;
    kc_status st = KC_OK;
    const bool side = !b->big.empty();
    if (side) {
        if (hipEventRecord(b->forked, s) != hipSuccess)
            return KC_EDEVICE;
        for (uint32_t l = 0; l < b->lanes_used; l++)
            if (hipStreamWaitEvent(b->side[l], b->forked, 0) != hipSuccess)
                return KC_EDEVICE;
        for (size_t j = 0; j < b->big.size() && st == KC_OK; j++) {
            const kc_set &q = sets[b->big[j]];
            const int l = b->big_lane[j];
            kc_filter *f = q.filter;
            kc::Workspace *own = f->W;
            f->W = &b->side_ws[l];
            st = insert_range(f, b->W, q.first_base, q.n_bases, q.k, reset, replayed,
                              q.distinct_dev, q.distinct_cap, q.n_distinct_dev, q.n_windows_dev,
                              q.tau, q.trust_dev, q.n_trust_dev, q.err_dev, q.n_err_dev,
                              q.class_cap, b->side[l], prof);
            f->W = own;
        }
        for (uint32_t l = 0; l < b->lanes_used; l++)
            if (hipEventRecord(b->joined[l], b->side[l]) != hipSuccess)
                st = KC_EDEVICE;
    }
    kc::ReadsArgs R{b->W.codes, b->W.inv, b->W.rs, n_bases, 0, b->W.valid};
    if (st == KC_OK && P.n_sets && kc::launch_batch(P, b->B, R, reset, s, prof) != hipSuccess)
        st = KC_EDEVICE;
    uint32_t di = 0;
    for (uint32_t i = 0; i < n_sets && st == KC_OK; i++) {
        const kc_set &q = sets[i];
        if (q.n_bases == 0 || !fused_form(q))
            continue;
        const kc::SetDesc &d = b->h_sets[di++];
        if (q.trust_dev && !d.fused) {
            // split of the keys this set appended: distinct[saved .. *n_distinct)
            e = kc::launch_classify(q.filter->F, q.distinct_dev, q.n_distinct_dev,
                                    b->B.saved + (di - 1), q.n_bases, q.distinct_cap, q.tau,
                                    q.trust_dev, q.n_trust_dev, q.err_dev, q.n_err_dev,
                                    q.class_cap, q.filter->status, b->W, s, prof);
            if (e != hipSuccess)
                st = KC_EDEVICE;
        }
    }
    // joined even after a failure, so that a capture ends with every stream
    for (uint32_t l = 0; side && l < b->lanes_used; l++)
        if (hipStreamWaitEvent(s, b->joined[l], 0) != hipSuccess)
            st = KC_EDEVICE;
    return st;
}

// The single-set pipeline's knobs tried by the tuner: counters per region
// (the region pass's LDS tile: 16384, one workgroup per CU, or 8192, two per
// CU) and positions per chunk (a pass over the countBF per chunk; larger
// chunks take more scratch) for a filter whose inserts take the partitioned
// path, or the single-level binned path.
struct SideKnobs {
    uint32_t counters;
    uint64_t chunk;
};
constexpr SideKnobs kPartCandidates[] = {{kc::kRegionCounters, kc::kPartChunk},
                                         {kc::kSmallRegionCounters, kc::kPartChunk},
                                         {kc::kRegionCounters, 1ull << 31},
                                         {kc::kSmallRegionCounters, 1ull << 31}};
constexpr SideKnobs kBinCandidates[] = {{kc::kRegionCounters, kc::kBinChunk},
                                        {kc::kSmallRegionCounters, kc::kBinChunk},
                                        {kc::kRegionCounters, 1ull << 27}};

// Tune each side-lane set's knobs on this input, timing its whole pipeline
// once per candidate (reset first, so only with KC_BATCH_RESET: the real run
// resets again); the handle keeps the fastest.
kc_status tune_side(kc_batch *b, const kc_set *sets, hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return KC_EDEVICE;
    kc_status st = KC_OK;
    if (hipStreamSynchronize(s) != hipSuccess)  // the ingest of the buffer is done
        st = KC_EDEVICE;
    for (size_t j = 0; j < b->big.size() && st == KC_OK; j++) {
        const kc_set &q = sets[b->big[j]];
        kc_filter *f = q.filter;
        if (q.n_bases == 0 || !takes_binned_path(f, q.n_bases))
            continue;
        kc::BinPlan bp{};
        if (!kc::bin_plan(f->F, q.n_bases < kc::kBinChunk ? q.n_bases : kc::kBinChunk, bp,
                          f->part_log, f->region_counters))
            continue;
        const bool parts = bp.n_parts > 0;
        const SideKnobs *cand = parts ? kPartCandidates : kBinCandidates;
        const int n_cand = parts ? 4 : 3;
        const int l = b->big_lane[j];
        kc::Workspace *own = f->W;
        f->W = &b->side_ws[l];
        f->last = b->side[l];
        uint64_t &chunk_knob = parts ? f->part_chunk : f->bin_chunk;
        const SideKnobs keep{f->region_counters, chunk_knob};
        SideKnobs best = keep;
        float best_ms = 1e30f;
        for (int c = 0; c < n_cand && st == KC_OK; c++) {
            f->region_counters = cand[c].counters;
            chunk_knob = cand[c].chunk;
            // a candidate whose plan is another path (or none) is skipped, and
            // chunks at or above the insert's size repeat the whole-insert plan
            if (cand[c].chunk >= q.n_bases && c > 0 && cand[c - 1].counters == cand[c].counters &&
                cand[c - 1].chunk >= q.n_bases)
                continue;
            if (!takes_binned_path(f, q.n_bases))
                continue;
            if ((st = prepare_range(f, q.n_bases)) != KC_OK)
                break;
            float ms = 0.f;
            if (hipEventRecord(e0, b->side[l]) != hipSuccess ||
                (st = insert_range(f, b->W, q.first_base, q.n_bases, q.k, true, false,
                                   q.distinct_dev, q.distinct_cap, q.n_distinct_dev,
                                   q.n_windows_dev, q.tau, q.trust_dev, q.n_trust_dev, q.err_dev,
                                   q.n_err_dev, q.class_cap, b->side[l], nullptr)) != KC_OK ||
                hipEventRecord(e1, b->side[l]) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                if (st == KC_OK)
                    st = KC_EDEVICE;
                break;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = cand[c];
            }
        }
        const SideKnobs use = st == KC_OK ? best : keep;
        f->region_counters = use.counters;
        chunk_knob = use.chunk;
        if (st == KC_OK)
            st = prepare_range(f, q.n_bases);
        f->W = own;
        f->last = s;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Fastest work-item size for this input, timed on the binning kernels only
// (they do not modify any countBF).
kc_status autotune(kc_batch *b, const kc_set *sets, uint32_t n_sets, const uint8_t *reads,
                   const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases, hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return KC_EDEVICE;
    kc_status st = KC_OK;
    if (kc::launch_ingest(reads, n_bases, offsets, n_reads, b->W, s, nullptr) != hipSuccess)
        st = KC_EDEVICE;
    float best = 1e30f;
    uint64_t best_tile = b->tile;
    kc::ReadsArgs R{b->W.codes, b->W.inv, b->W.rs, n_bases, 0, b->W.valid};
    for (uint64_t tile : kTileCandidates) {
        if (st != KC_OK)
            break;
        kc::BatchPlan P = make_plan(b, sets, n_sets, n_bases, tile);
        if ((st = ensure_batch(b, P, s)) != KC_OK || (st = upload(b, P, s)) != KC_OK)
            break;
        float t_min = 1e30f;
        for (int rep = 0; rep < 3 && st == KC_OK; rep++) {
            (void)hipEventRecord(e0, s);
            if (kc::launch_batch_bins(P, b->B, R, s, nullptr) != hipSuccess)
                st = KC_EDEVICE;
            (void)hipEventRecord(e1, s);
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = KC_EDEVICE;
            if (rep > 0)
                t_min = std::min(t_min, ms);
        }
        if (st == KC_OK && t_min < best) {
            best = t_min;
            best_tile = tile;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == KC_OK)
        b->tile = best_tile;
    return st;
}

// Every buffer address of a workspace (a captured graph bakes them in).
void workspace_pointers(const kc::Workspace &W, std::vector<uint64_t> &out) {
    const void *p[] = {W.codes, W.inv, W.rs, W.valid, W.flags8, W.tile_a, W.tile_b, W.tile_c,
                       W.off_a, W.off_b, W.off_c, W.tmask, W.partial64, W.matrix, W.matrix_t,
                       W.coarse, W.partial32, W.slots, W.bucketed, W.entries, W.pmat, W.pbounds,
                       W.pdesc, W.totals, W.n_entries, W.win_cursors, W.carry,
                       W.carry_off, W.carry_n};
    for (const void *x : p)
        out.push_back((uint64_t)(uintptr_t)x);
    out.insert(out.end(), {W.cap, W.tile_cap, W.matrix_cap, W.coarse_cap, W.slots_cap,
                           W.entries_cap, W.pmat_cap, W.carry_cap, W.carry_idx_cap});
}

// Everything a captured graph depends on: the arguments, the work-item size
// and the workspace addresses baked into its kernels.
std::vector<uint8_t> call_key(const kc_batch *b, const kc_set *sets, uint32_t n_sets,
                              const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads,
                              uint64_t n_bases, uint32_t flags, hipStream_t s) {
    const kc::Workspace &W = b->W;
    const uint64_t tail[] = {(uint64_t)(uintptr_t)reads, (uint64_t)(uintptr_t)offsets, n_reads,
                             n_bases, flags & ~(uint32_t)KC_BATCH_TUNE, (uint64_t)(uintptr_t)s,
                             b->tile, n_sets,
                             (uint64_t)(uintptr_t)W.codes, (uint64_t)(uintptr_t)W.inv,
                             (uint64_t)(uintptr_t)W.rs, (uint64_t)(uintptr_t)W.valid,
                             (uint64_t)(uintptr_t)W.flags8,
                             (uint64_t)(uintptr_t)W.tile_a, (uint64_t)(uintptr_t)W.off_a,
                             (uint64_t)(uintptr_t)W.partial64, (uint64_t)(uintptr_t)W.totals,
                             (uint64_t)(uintptr_t)W.tmask};
    // each set's filter by its generation (a destroyed handle's host address
    // can be reused), the device state and plan its launches bake in, and
    // the side lanes' workspaces
    std::vector<uint64_t> filt;
    for (uint32_t i = 0; i < n_sets; i++) {
        const kc_filter *f = sets[i].filter;
        filt.insert(filt.end(), {f->generation, (uint64_t)(uintptr_t)f->F.words,
                                 (uint64_t)(uintptr_t)f->status, (uint64_t)(uintptr_t)f->F.aux,
                                 f->layout.X, f->layout.Y, f->layout.alpha, f->layout.k_h,
                                 f->chunk, f->bin_chunk, f->part_chunk, f->part_log,
                                 f->region_counters, (uint64_t)f->path});
    }
    for (uint32_t l = 0; l < b->lanes_used; l++)
        workspace_pointers(b->side_ws[l], filt);
    filt.insert(filt.end(), b->big.begin(), b->big.end());
    filt.insert(filt.end(), b->big_lane.begin(), b->big_lane.end());
    const size_t nf = filt.size() * sizeof(uint64_t);
    std::vector<uint8_t> k(n_sets * sizeof(kc_set) + sizeof tail + nf);
    std::memcpy(k.data(), sets, n_sets * sizeof(kc_set));
    std::memcpy(k.data() + n_sets * sizeof(kc_set), tail, sizeof tail);
    if (nf)
        std::memcpy(k.data() + n_sets * sizeof(kc_set) + sizeof tail, filt.data(), nf);
    return k;
}

kc_status validate(const kc_set *sets, uint32_t n_sets, const uint8_t *reads,
                   const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases, int device) {
    if (!sets || n_sets == 0)
        return KC_EINVAL;
    if (n_bases > 0 && (!reads || !offsets || n_reads == 0))
        return KC_EINVAL;
    uint64_t end = 0, entries = 0;
    for (uint32_t i = 0; i < n_sets; i++) {
        const kc_set &q = sets[i];
        kc_filter *f = q.filter;
        if (!f || f->device != device || q.k < 1 || q.k > 64 || !q.n_distinct_dev)
            return KC_EINVAL;
        if (f->k != 0 && f->k != q.k)
            return KC_ESTATE;
        if (q.first_base % kc::kSetAlign != 0 || q.first_base < end ||
            q.first_base + q.n_bases > n_bases)
            return KC_EINVAL;  // sets must be aligned, sorted and disjoint
        if (q.distinct_cap > 0 && !q.distinct_dev)
            return KC_EINVAL;
        if (q.trust_dev && (!q.n_trust_dev || !q.err_dev || !q.n_err_dev))
            return KC_EINVAL;
        for (uint32_t j = 0; j < i; j++)
            if (sets[j].filter == f)
                return KC_EINVAL;  // one filter per set
        if (q.n_bases > 0 && fused_form(q)) {
            entries += q.n_bases * f->F.k_h;
        } else {
            const kc_status st = check_range(f, q.n_bases, q.k);
            if (st != KC_OK)
                return st;
        }
        end = q.first_base + q.n_bases;
    }
    if (entries >= (1ull << 32))
        return KC_EINVAL;
    return KC_OK;
}

}  // namespace

bool kcapi::batchable(const kc_filter *f) {
    kc::BinPlan bp{};
    return kc::bin_plan(f->F, kc::kBinChunk, bp) && bp.n_regions <= kc::kBatchMaxRegions;
}

extern "C" {

kc_status kc_batch_create(kc_batch **out) {
    if (!out)
        return KC_EINVAL;
    *out = nullptr;
    kc_batch *b = new (std::nothrow) kc_batch();
    if (!b)
        return KC_ENOMEM;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return KC_EDEVICE;
    }
    b->B.W = &b->W;
    *out = b;
    return KC_OK;
}

void kc_batch_destroy(kc_batch *b) {
    if (!b)
        return;
    DeviceGuard g(b->device);
    (void)hipDeviceSynchronize();
    drop_graph(b);
    b->prof.release();
    free_batch_buffers(b);
    free_workspace(b->W);
    for (int l = 0; l < kSideLanes; l++) {
        free_workspace(b->side_ws[l]);
        if (b->side[l])
            (void)hipStreamDestroy(b->side[l]);
        if (b->joined[l])
            (void)hipEventDestroy(b->joined[l]);
    }
    if (b->forked)
        (void)hipEventDestroy(b->forked);
    if (b->staged)
        (void)hipEventDestroy(b->staged);
    if (b->stage)
        (void)hipHostFree(b->stage);
    delete b;
}

kc_status kc_batch_insert(kc_batch *b, const kc_set *sets, uint32_t n_sets,
                          const uint8_t *reads_dev, const uint64_t *offsets_dev, uint64_t n_reads,
                          uint64_t n_bases, uint32_t flags, void *stream) {
    if (!b)
        return KC_EINVAL;
    kc_status st = validate(sets, n_sets, reads_dev, offsets_dev, n_reads, n_bases, b->device);
    if (st != KC_OK)
        return st;
    DeviceGuard g(b->device);
    if (!g.ok)
        return KC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const bool graph = (flags & KC_BATCH_GRAPH) != 0;
    const bool reset = (flags & KC_BATCH_RESET) != 0;
    if (graph && !s)
        return KC_EINVAL;  // the null stream cannot be captured
    b->last = s;
    if ((st = ensure_scalars(b->W)) != KC_OK || (st = ensure_positions(b->W, s, n_bases, true)) != KC_OK ||
        (st = ensure_tiles(b->W, s, n_bases)) != KC_OK)
        return st;
    if ((st = plan_side(b, sets, n_sets)) != KC_OK)
        return st;
    if (flags & KC_BATCH_TUNE) {
        drop_graph(b);  // tuning rewrites the device descriptor table
        if (b->big.size() < n_sets &&
            (st = autotune(b, sets, n_sets, reads_dev, offsets_dev, n_reads, n_bases, s)) != KC_OK)
            return st;
        if (reset && !b->big.empty()) {
            if (kc::launch_ingest(reads_dev, n_bases, offsets_dev, n_reads, b->W, s, nullptr) !=
                hipSuccess)
                return KC_EDEVICE;
            if ((st = tune_side(b, sets, s)) != KC_OK)
                return st;
        }
    }
    std::vector<uint8_t> key;
    if (graph) {
        key = call_key(b, sets, n_sets, reads_dev, offsets_dev, n_reads, n_bases, flags, s);
        if (b->exec && key == b->graph_key) {
            if (hipGraphLaunch(b->exec, s) != hipSuccess)
                return KC_EDEVICE;
            for (uint32_t i = 0; i < n_sets; i++) {  // as after the captured call
                sets[i].filter->zero = false;
                sets[i].filter->k = sets[i].k;
                sets[i].filter->last = s;
            }
            return KC_OK;
        }
    }
    // a new descriptor table invalidates any captured graph
    drop_graph(b);
    kc::BatchPlan P = make_plan(b, sets, n_sets, n_bases, b->tile);
    if ((st = ensure_batch(b, P, s)) != KC_OK || (st = upload(b, P, s)) != KC_OK)
        return st;
    if (graph) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess)
            return KC_EDEVICE;
        st = launch_all(b, P, sets, n_sets, reads_dev, offsets_dev, n_reads, n_bases, reset, true,
                        s, nullptr);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(s, &gr);
        if (st != KC_OK || e != hipSuccess) {
            if (gr)
                (void)hipGraphDestroy(gr);
            return st != KC_OK ? st : KC_EDEVICE;
        }
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiateWithFlags(&ex, gr, 0) != hipSuccess) {
            (void)hipGraphDestroy(gr);
            return KC_EDEVICE;
        }
        b->graph = gr;
        b->exec = ex;
        b->graph_key = key;
        if (hipGraphLaunch(ex, s) != hipSuccess)
            return KC_EDEVICE;
    } else {
        st = launch_all(b, P, sets, n_sets, reads_dev, offsets_dev, n_reads, n_bases, reset, false,
                        s, &b->prof);
        if (st != KC_OK)
            return st;
    }
    for (uint32_t i = 0; i < n_sets; i++) {
        sets[i].filter->zero = false;
        sets[i].filter->k = sets[i].k;
        sets[i].filter->last = s;
    }
    return KC_OK;
}

kc_status kc_batch_get_tile(const kc_batch *b, uint64_t *tile) {
    if (!b || !tile)
        return KC_EINVAL;
    *tile = b->tile;
    return KC_OK;
}

kc_status kc_batch_set_tile(kc_batch *b, uint64_t tile) {
    if (!b || tile < (uint64_t)kc::kBinWG || tile % kc::kBinWG != 0 || tile > kc::kBinChunk)
        return KC_EINVAL;
    b->tile = tile;
    return KC_OK;
}

kc_status kc_batch_profile(kc_batch *b, int enable) {
    if (!b)
        return KC_EINVAL;
    b->prof.collect(nullptr, nullptr, 0);
    b->prof.on = enable != 0;
    return KC_OK;
}

kc_status kc_batch_profile_read(kc_batch *b, double *ms, uint64_t *launches, uint32_t n_phases) {
    if (!b || (n_phases > 0 && (!ms || !launches)))
        return KC_EINVAL;
    DeviceGuard g(b->device);
    if (!g.ok)
        return KC_EDEVICE;
    b->prof.collect(ms, launches, n_phases);
    return KC_OK;
}

kc_status kc_batch_sync(kc_batch *b) {
    if (!b)
        return KC_EINVAL;
    DeviceGuard g(b->device);
    if (!g.ok)
        return KC_EDEVICE;
    return hipStreamSynchronize(b->last) == hipSuccess ? KC_OK : KC_EDEVICE;
}

}  // extern "C"
