// C ABI of the gfx950 KmerCo library (declared in include/kmerco.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>

#include "kc_kernels.hpp"
#include "kmerco.h"

struct kc_filter {
    kc_layout layout;
    kc::FilterArgs F;
    kc::Workspace W;
    int device;
    bool zero;             // every counter of the filter is zero
    uint32_t k;            // k of the first insert, 0 before it
    uint32_t *status;      // device: sticky status bits (kc::kStatus*)
    hipStream_t last;      // stream of the last enqueued call
    uint64_t chunk;        // positions resolved per first-seen chunk
    kc::Profiler prof;     // optional per-kernel timing
};

namespace {

// Make the handle's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess)
            ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

bool valid_layout(const kc_layout *L) {
    if (!L)
        return false;
    if (L->X < 1 || L->Y < 1 || L->alpha < 1 || L->alpha > 32 || L->k_h < 1 || L->k_h > 8)
        return false;
    // X*Y*eta counters must be addressable with 64-bit indices
    if (L->X > (UINT64_MAX / 64) / L->Y)
        return false;
    return true;
}

void free_workspace(kc::Workspace &W) {
    (void)hipFree(W.codes);
    (void)hipFree(W.inv);
    (void)hipFree(W.rs);
    (void)hipFree(W.flags);
    (void)hipFree(W.tile_a);
    (void)hipFree(W.tile_b);
    (void)hipFree(W.tile_off);
    (void)hipFree(W.totals);
    W = kc::Workspace{};
}

template <typename T>
bool dev_alloc(T **p, uint64_t count) {
    return hipMalloc((void **)p, (count ? count : 1) * sizeof(T)) == hipSuccess;
}

// Grow the per-call workspace to hold `n` positions.  Waits for the
// handle's outstanding work before releasing old buffers.
kc_status ensure_workspace(kc_filter *f, uint64_t n) {
    if (n <= f->W.cap && f->W.codes)
        return KC_OK;
    if (f->W.codes)
        (void)hipStreamSynchronize(f->last);
    free_workspace(f->W);
    uint64_t cap = n < 65536 ? 65536 : n + n / 8;  // headroom for slowly growing calls
    kc::Workspace W;
    W.cap = cap;
    bool ok = dev_alloc(&W.codes, kc::code_words(cap)) && dev_alloc(&W.inv, kc::mask_words(cap)) &&
              dev_alloc(&W.rs, kc::mask_words(cap)) && dev_alloc(&W.flags, kc::flag_words(cap)) &&
              dev_alloc(&W.tile_a, kc::tiles(cap)) && dev_alloc(&W.tile_b, kc::tiles(cap)) &&
              dev_alloc(&W.tile_off, kc::tiles(cap)) && dev_alloc(&W.totals, 2);
    if (!ok) {
        free_workspace(W);
        return KC_ENOMEM;
    }
    f->W = W;
    return KC_OK;
}

// Positions per first-seen chunk: kc::kChunk, or KMERCO_CHUNK_POSITIONS
// (rounded down to a multiple of kc::kTile, at least one tile) so that small
// inputs can exercise the multi-chunk path.
uint64_t chunk_from_env() {
    const char *e = std::getenv("KMERCO_CHUNK_POSITIONS");
    if (!e || !*e)
        return kc::kChunk;
    char *end = nullptr;
    unsigned long long v = std::strtoull(e, &end, 10);
    if (end == e)
        return kc::kChunk;
    uint64_t c = (uint64_t)v / kc::kTile * kc::kTile;
    if (c < (uint64_t)kc::kTile)
        c = kc::kTile;
    return c > kc::kChunk ? kc::kChunk : c;
}

uint64_t next_prime_after(uint64_t n) {
    for (uint64_t p = n + 1;; p++) {
        if (p < 2)
            continue;
        bool prime = true;
        for (uint64_t d = 2; d * d <= p; d++)
            if (p % d == 0) {
                prime = false;
                break;
            }
        if (prime)
            return p;
    }
}

}  // namespace

extern "C" {

const char *kc_strerror(int status) {
    switch (status) {
    case KC_OK: return "ok";
    case KC_EINVAL: return "invalid argument";
    case KC_ENOMEM: return "device memory allocation failed";
    case KC_ERANGE: return "output capacity too small";
    case KC_EDEVICE: return "HIP runtime error";
    case KC_ESTATE: return "call not allowed in the filter's state";
    default: return "unknown status";
    }
}

int kc_version(void) { return 1; }

uint32_t kc_eta(uint32_t alpha) { return (alpha >= 1 && alpha <= 64) ? 64u / alpha : 0u; }

kc_status kc_dims(double n_items, double fpp, uint64_t *X, uint64_t *Y) {
    if (!X || !Y || !(n_items > 0) || !(fpp > 0) || !(fpp < 1))
        return KC_EINVAL;
    double m = -n_items * std::log(fpp) / (std::log(2.0) * std::log(2.0));
    double v = std::sqrt(m / 128.0);
    if (!(v < 1e15))
        return KC_EINVAL;
    uint64_t x = next_prime_after((uint64_t)std::floor(v));
    uint64_t y = x;
    for (int i = 0; i < 3; i++)
        y = next_prime_after(y);
    *X = x;
    *Y = y;
    return KC_OK;
}

kc_status kc_create(const kc_layout *layout, uint64_t *words_dev, int zero, void *stream,
                    kc_filter **out) {
    if (!out || !words_dev || !valid_layout(layout))
        return KC_EINVAL;
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return KC_EDEVICE;
    kc_filter *f = new (std::nothrow) kc_filter();
    if (!f)
        return KC_ENOMEM;
    f->layout = *layout;
    f->device = dev;
    f->zero = zero != 0;
    f->k = 0;
    f->last = (hipStream_t)stream;
    f->chunk = chunk_from_env();
    kc::FilterArgs &F = f->F;
    F.words = words_dev;
    F.X = layout->X;
    F.Y = layout->Y;
    F.mX = UINT64_MAX / layout->X;
    F.mY = UINT64_MAX / layout->Y;
    F.alpha = layout->alpha;
    F.eta = 64u / layout->alpha;
    F.mEta = UINT64_MAX / F.eta;
    F.eta_pow2 = (F.eta & (F.eta - 1)) == 0;
    F.k_h = layout->k_h;
    F.field_max = (layout->alpha >= 64) ? ~0ull : ((1ull << layout->alpha) - 1ull);
    uint64_t n_words = layout->X * layout->Y;
    uint64_t n_aux = n_words * F.eta;
    hipStream_t s = (hipStream_t)stream;
    if (!dev_alloc(&F.aux, n_aux) || !dev_alloc(&f->status, 1)) {
        (void)hipFree(F.aux);
        (void)hipFree(f->status);
        delete f;
        return KC_ENOMEM;
    }
    hipError_t e = kc::fill_u32(F.aux, n_aux, kc::kIdle, s);
    if (e == hipSuccess)
        e = kc::fill_u32(f->status, 1, 0u, s);
    if (e == hipSuccess && zero)
        e = kc::fill_u64(words_dev, n_words, 0ull, s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(F.aux);
        (void)hipFree(f->status);
        delete f;
        return KC_EDEVICE;
    }
    *out = f;
    return KC_OK;
}

void kc_destroy(kc_filter *f) {
    if (!f)
        return;
    DeviceGuard g(f->device);
    (void)hipDeviceSynchronize();
    f->prof.release();
    free_workspace(f->W);
    (void)hipFree(f->F.aux);
    (void)hipFree(f->status);
    delete f;
}

kc_status kc_reserve(kc_filter *f, uint64_t max_bases) {
    if (!f)
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    return ensure_workspace(f, max_bases);
}

kc_status kc_get_layout(const kc_filter *f, kc_layout *out) {
    if (!f || !out)
        return KC_EINVAL;
    *out = f->layout;
    return KC_OK;
}

kc_status kc_insert(kc_filter *f, const uint8_t *reads_dev, const uint64_t *offsets_dev,
                    uint64_t n_reads, uint64_t n_bases, uint32_t k, uint64_t *distinct_dev,
                    uint64_t distinct_cap, uint64_t *n_distinct_dev, uint64_t *n_windows_dev,
                    void *stream) {
    if (!f || k < 1 || k > 32 || !n_distinct_dev)
        return KC_EINVAL;
    if (n_bases > 0 && (!reads_dev || !offsets_dev))
        return KC_EINVAL;
    if (distinct_cap > 0 && !distinct_dev)
        return KC_EINVAL;
    if (f->k != 0 && f->k != k)
        return KC_ESTATE;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    f->last = s;
    f->k = k;
    if (n_bases == 0)
        return KC_OK;
    kc_status st = ensure_workspace(f, n_bases);
    if (st != KC_OK)
        return st;
    hipError_t e = kc::launch_ingest(reads_dev, n_bases, offsets_dev, n_reads, f->W, s, &f->prof);
    if (e != hipSuccess)
        return KC_EDEVICE;
    kc::ReadsArgs R{f->W.codes, f->W.inv, f->W.rs, n_bases, k};
    for (uint64_t c0 = 0; c0 < n_bases; c0 += f->chunk) {
        uint64_t c1 = c0 + f->chunk < n_bases ? c0 + f->chunk : n_bases;
        e = kc::launch_insert_chunk(f->F, R, c0, c1, f->zero, f->W, s, &f->prof);
        if (e != hipSuccess)
            return KC_EDEVICE;
        f->zero = false;
    }
    e = kc::launch_distinct(R, f->W, distinct_dev, distinct_cap, n_distinct_dev, n_windows_dev,
                            f->status, s, &f->prof);
    return e == hipSuccess ? KC_OK : KC_EDEVICE;
}

kc_status kc_classify(kc_filter *f, const uint64_t *keys_dev, const uint64_t *n_keys_dev,
                      uint64_t keys_cap, uint32_t tau, uint64_t *trust_dev, uint64_t *n_trust_dev,
                      uint64_t *err_dev, uint64_t *n_err_dev, void *stream) {
    if (!f || !n_keys_dev || !n_trust_dev || !n_err_dev)
        return KC_EINVAL;
    if (keys_cap > 0 && (!keys_dev || !trust_dev || !err_dev))
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    f->last = s;
    kc_status st = ensure_workspace(f, keys_cap);
    if (st != KC_OK)
        return st;
    hipError_t e = kc::launch_classify(f->F, keys_dev, n_keys_dev, keys_cap, tau, trust_dev,
                                       n_trust_dev, err_dev, n_err_dev, f->W, s, &f->prof);
    return e == hipSuccess ? KC_OK : KC_EDEVICE;
}

kc_status kc_query(kc_filter *f, const uint64_t *keys_dev, uint64_t n, uint32_t *freq_dev,
                   void *stream) {
    if (!f || (n > 0 && (!keys_dev || !freq_dev)))
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    f->last = s;
    return kc::launch_query(f->F, keys_dev, n, freq_dev, s, &f->prof) == hipSuccess ? KC_OK : KC_EDEVICE;
}

kc_status kc_sync(kc_filter *f) {
    if (!f)
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    if (hipStreamSynchronize(f->last) != hipSuccess)
        return KC_EDEVICE;
    uint32_t st = 0;
    if (hipMemcpy(&st, f->status, sizeof st, hipMemcpyDeviceToHost) != hipSuccess)
        return KC_EDEVICE;
    if (st) {
        uint32_t zero = 0;
        if (hipMemcpy(f->status, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
            return KC_EDEVICE;
        return KC_ERANGE;
    }
    return KC_OK;
}

kc_status kc_reset(kc_filter *f, void *stream) {
    if (!f)
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    f->last = s;
    f->prof.begin(kc::kPhReset, s);
    hipError_t e = kc::fill_u64(f->F.words, f->layout.X * f->layout.Y, 0ull, s);
    f->prof.end(s);
    if (e != hipSuccess)
        return KC_EDEVICE;
    // the first-seen workspace is back to idle after every insert
    f->zero = true;
    f->k = 0;
    return KC_OK;
}

kc_status kc_profile(kc_filter *f, int enable) {
    if (!f)
        return KC_EINVAL;
    f->prof.collect(nullptr, nullptr, 0);
    f->prof.on = enable != 0;
    return KC_OK;
}

kc_status kc_profile_read(kc_filter *f, double *ms, uint64_t *launches, uint32_t n_phases) {
    if (!f || (n_phases > 0 && (!ms || !launches)))
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    f->prof.collect(ms, launches, n_phases);
    return KC_OK;
}

const char *kc_phase_name(uint32_t phase) {
    static const char *names[kc::kPhCount] = {
        "ingest", "claim", "increment", "claim_increment", "resolve", "scan", "scatter",
        "classify_mark", "classify_scatter", "query", "reset"};
    return phase < (uint32_t)kc::kPhCount ? names[phase] : "unknown";
}

}  // extern "C"
