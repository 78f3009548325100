// kc_insert_classify_noalloc: the insertion and classification phases of one
// read batch with every scratch buffer in a fixed device array of this file,
// so that the call allocates no device memory (declared in include/kmerco.h).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kc_handle.hpp"
#include "kc_kernels.hpp"
#include "kmerco.h"

namespace {

// The scratch of kc_insert_classify_noalloc: one copy per device, held from
// the library's load until the process ends.
constexpr uint64_t kNoallocScratchBytes = KC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (the current device
// must be `dev`); null when the runtime cannot name it.  Host code never
// uses the array's own name: in host code it is a stand-in, not a device
// address.
uint8_t *scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return nullptr;
        g_scratch[dev] = p;
    }
    return static_cast<uint8_t *>(g_scratch[dev]);
}

}  // namespace

extern "C" {

kc_status kc_insert_classify_noalloc(kc_filter *f, const uint8_t *reads_dev,
                                     const uint64_t *offsets_dev, uint64_t n_reads,
                                     uint64_t n_bases, uint32_t k, uint32_t tau,
                                     uint64_t *distinct_dev, uint64_t distinct_cap,
                                     uint64_t *n_distinct_dev, uint64_t *n_windows_dev,
                                     uint64_t *trust_dev, uint64_t *n_trust_dev, uint64_t *err_dev,
                                     uint64_t *n_err_dev, uint64_t class_cap, void *stream) {
    using namespace kcapi;
    if (!f || k < 1 || k > 64 || !n_distinct_dev || !n_trust_dev || !n_err_dev)
        return KC_EINVAL;
    if (n_bases > 0 && (!reads_dev || !offsets_dev))
        return KC_EINVAL;
    if ((distinct_cap > 0 && !distinct_dev) || (class_cap > 0 && (!trust_dev || !err_dev)))
        return KC_EINVAL;
    if (f->k != 0 && f->k != k)
        return KC_ESTATE;
    // the direct path keeps per-counter first-seen state beside the filter,
    // which this call has no room for
    if (!takes_binned_path(f, n_bases))
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    uint8_t *base = scratch_of(f->device);
    if (!base)
        return KC_EDEVICE;
    // this call's buffers, laid out from the start of the array (the layout
    // depends only on the filter's layout and n_bases; no contents carry
    // over between calls: every buffer is written before it is read)
    kc::Workspace W{};
    kc::Workspace *own = f->W;
    f->W = &W;
    Carve c;
    c.base = base;
    c.size = kNoallocScratchBytes;
    kc_status st;
    {
        Carving mode(&c);
        st = reserve_all(f, n_bases);
    }
    W.fixed = true;
    if (st == KC_ENOMEM)
        st = KC_ERANGE;  // the insert needs more than kNoallocScratchBytes
    if (st == KC_OK) {
        uint64_t *trust = trust_dev ? trust_dev : n_trust_dev;
        uint64_t *err = err_dev ? err_dev : n_err_dev;
        st = insert_impl(f, reads_dev, offsets_dev, n_reads, n_bases, k, distinct_dev,
                         distinct_cap, n_distinct_dev, n_windows_dev, tau, trust, n_trust_dev, err,
                         n_err_dev, class_cap, (hipStream_t)stream);
    }
    f->W = own;
    return st;
}

}  // extern "C"
