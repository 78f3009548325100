// Handle of a countBF (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "kc_kernels.hpp"
#include "kmerco.h"

enum class KcPath { Auto, Direct, Binned };

struct kc_filter {
    kc_layout layout;
    kc::FilterArgs F;
    kc::Workspace W;
    int device;
    bool zero;             // every counter of the filter is zero
    uint32_t k;            // k of the first insert, 0 before it
    uint32_t *status;      // device: sticky status bits (kc::kStatus*)
    hipStream_t last;      // stream of the last enqueued call
    uint64_t chunk;        // direct path: positions per first-seen chunk
    uint64_t bin_chunk;    // binned path: positions per chunk
    KcPath path;
    kc::Profiler prof;     // optional per-kernel timing
};

// helpers shared by the single-set and batch entry points (kc_api.hip)
namespace kcapi {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

template <typename T>
bool dev_alloc(T **p, uint64_t count) {
    return hipMalloc((void **)p, (count ? count : 1) * sizeof(T)) == hipSuccess;
}

template <typename T>
void dev_free(T *&p) {
    (void)hipFree(p);
    p = nullptr;
}

kc_status ensure_positions(kc::Workspace &W, hipStream_t wait_on, uint64_t n);
kc_status ensure_tiles(kc::Workspace &W, hipStream_t wait_on, uint64_t n);
kc_status ensure_scalars(kc::Workspace &W);
void free_workspace(kc::Workspace &W);

}  // namespace kcapi
