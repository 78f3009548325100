// Handle of a countBF (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "kc_kernels.hpp"
#include "kmerco.h"

enum class KcPath { Auto, Direct, Binned };

struct kc_filter {
    kc_layout layout;
    kc::FilterArgs F;
    kc::Workspace own;     // scratch of this handle's calls (library-allocated, or
                           // carved from the caller's scratch: own.fixed)
    kc::Workspace *W;      // &own, or a workspace shared by handles whose calls
                           // are all ordered on one stream

    int device;
    bool zero;             // every counter of the filter is zero
    uint32_t k;            // k of the first insert, 0 before it
    uint32_t *status;      // device: sticky status bits (kc::kStatus*)
    hipStream_t last;      // stream of the last enqueued call
    uint64_t chunk;        // direct path: positions per first-seen chunk
    uint64_t bin_chunk;    // binned path: positions per chunk
    uint64_t part_chunk;   // partitioned binned path: positions per chunk
    uint32_t part_log;     // partitioned binned path: log2(regions per partition)
    uint32_t region_counters;  // binned paths: counters per region (the region pass's LDS)
    bool carry;            // multi-chunk inserts classify in the last region pass
    KcPath path;
    kc::Profiler prof;     // optional per-kernel timing
    bool caller_scratch;   // status word and workspace live in the caller's buffer
    uint64_t generation;   // unique per handle of the process (graph keys)
};

// helpers shared by the single-set and batch entry points (kc_api.hip)
namespace kcapi {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

// Device allocations of the library go through dev_alloc, which has three
// modes:
//  - sizing (kc_scratch_bytes): while g_size_only is set, dev_alloc adds the
//    bytes it would allocate there and hands out a placeholder that is never
//    dereferenced; dev_free and the workspace waits do nothing;
//  - carving (caller-owned scratch): while g_carve is set, dev_alloc hands
//    out consecutive pieces of the caller's buffer and fails when it is
//    exhausted; dev_free does nothing;
//  - otherwise hipMalloc / hipFree.
// Every piece is a multiple of kAllocAlign bytes in the first two modes, so
// that a size counted in the first is exactly what the second carves.
constexpr uint64_t kAllocAlign = 256;

struct Carve {
    uint8_t *base = nullptr;
    uint64_t size = 0, used = 0;
};

extern thread_local uint64_t *g_size_only;
extern thread_local Carve *g_carve;

inline uint64_t alloc_round(uint64_t bytes) {
    return (bytes + kAllocAlign - 1) / kAllocAlign * kAllocAlign;
}

template <typename T>
bool dev_alloc(T **p, uint64_t count) {
    const uint64_t bytes = (count ? count : 1) * sizeof(T);
    if (g_size_only) {
        *g_size_only += alloc_round(bytes);
        *p = reinterpret_cast<T *>((uintptr_t)256);
        return true;
    }
    if (g_carve) {
        const uint64_t need = alloc_round(bytes);
        if (need > g_carve->size - g_carve->used)
            return false;
        *p = reinterpret_cast<T *>(g_carve->base + g_carve->used);
        g_carve->used += need;
        return true;
    }
    return hipMalloc((void **)p, bytes) == hipSuccess;
}

template <typename T>
void dev_free(T *&p) {
    if (!g_size_only && !g_carve)
        (void)hipFree(p);
    p = nullptr;
}

// Sets a mode of dev_alloc for the lifetime of the object.
struct SizeOnly {
    explicit SizeOnly(uint64_t *bytes) { g_size_only = bytes; }
    ~SizeOnly() { g_size_only = nullptr; }
};
struct Carving {
    explicit Carving(Carve *c) { g_carve = c; }
    ~Carving() { g_carve = nullptr; }
};

bool valid_layout(const kc_layout *L);
// A number no other handle of the process has had (keys of captured graphs
// name handles by it, not by their reusable host addresses).
uint64_t next_generation();
kc_status ensure_positions(kc::Workspace &W, hipStream_t wait_on, uint64_t n, bool valid_bitmap);
kc_status ensure_tiles(kc::Workspace &W, hipStream_t wait_on, uint64_t n);
kc_status ensure_scalars(kc::Workspace &W);
void free_workspace(kc::Workspace &W);

// Use W (owned by the caller, outliving f) instead of the handle's own
// scratch.  Every call on every handle sharing W must be enqueued on one
// stream, which is then also the stream waited on before W grows.
void share_workspace(kc_filter *f, kc::Workspace *W);
// Device bytes a handle of this layout allocates for itself on first insert
// besides the shared scratch (the direct path's per-counter first-seen
// entries), 0 for layouts that take the binned path.
uint64_t filter_private_bytes(const kc_layout &layout);
// Whether a handle can be a set of a kc_batch_insert call.
bool batchable(const kc_filter *f);
// Every buffer inserts of up to max_bases bases need, in the current
// dev_alloc mode, in f->W.
kc_status reserve_all(kc_filter *f, uint64_t max_bases);
// Whether inserts of n_bases into f take a binned path (else the direct
// path, which keeps per-counter state of its own).
bool takes_binned_path(const kc_filter *f, uint64_t n_bases);
// One read set of a larger ingested buffer (the batched form's sets that its
// fused kernels do not take): check_range validates it against f,
// prepare_range sizes f->W for it (may allocate and wait on f->last), and
// insert_range enqueues its insertion (and split, when trust != nullptr) on
// s, kernels only, reading the set's positions [base, base + n_bases) from
// pos's codes, bitmaps and flag bytes (base a multiple of kc::kTile) and
// using f->W for everything else.  reset: clear the countBF and the
// distinct / window counters first.  replayed: the launches are captured
// into a graph (the direct path then never assumes an empty filter unless
// reset).
kc_status check_range(const kc_filter *f, uint64_t n_bases, uint32_t k);
kc_status prepare_range(kc_filter *f, uint64_t n_bases);
kc_status insert_range(kc_filter *f, const kc::Workspace &pos, uint64_t base, uint64_t n_bases,
                       uint32_t k, bool reset, bool replayed, uint64_t *distinct,
                       uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows, uint32_t tau,
                       uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                       uint64_t cap_te, hipStream_t s, kc::Profiler *P);
// kc_insert / kc_insert_classify after the argument checks (trust ==
// nullptr: insertion only), with f's device current, in f->W.
kc_status insert_impl(kc_filter *f, const uint8_t *reads, const uint64_t *offsets,
                      uint64_t n_reads, uint64_t n_bases, uint32_t k, uint64_t *distinct,
                      uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows, uint32_t tau,
                      uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                      uint64_t cap_te, hipStream_t s);

}  // namespace kcapi
