// C ABI of the gfx950 KmerCo library (declared in include/kmerco.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <new>

#include "kc_kernels.hpp"
#include "kmerco.h"

#include "kc_handle.hpp"

namespace kcapi {

// Make the handle's device current for the duration of a call.
DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
        ok = false;
        return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess)
        ok = false;
}

DeviceGuard::~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
        (void)hipSetDevice(prev);
}

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

thread_local uint64_t *g_size_only = nullptr;
thread_local Carve *g_carve = nullptr;

uint64_t next_generation() {
    static std::atomic<uint64_t> counter{1};
    return counter.fetch_add(1);
}

void wait_idle(kc_filter *f) {
    if (!g_size_only && !g_carve)
        (void)hipStreamSynchronize(f->last);
}

// per-position buffers for inserts of up to n bases (waits for `wait_on`
// before releasing smaller ones); valid_bitmap: with the valid-window bitmap
// of the binned paths
kc_status ensure_positions(kc::Workspace &W, hipStream_t wait_on, uint64_t n, bool valid_bitmap) {
    if (W.codes && n <= W.cap && (W.valid || !valid_bitmap))
        return KC_OK;
    if (W.fixed)
        return KC_ERANGE;  // larger than the caller's scratch was sized for
    if (!g_size_only && !g_carve)
        (void)hipStreamSynchronize(wait_on);
    dev_free(W.codes);
    dev_free(W.inv);
    dev_free(W.rs);
    dev_free(W.valid);
    dev_free(W.flags8);
    uint64_t cap = n < 65536 ? 65536 : n + n / 8;
    W.cap = 0;
    if (!dev_alloc(&W.codes, kc::code_words(cap)) || !dev_alloc(&W.inv, kc::mask_words(cap)) ||
        !dev_alloc(&W.rs, kc::mask_words(cap)) ||
        (valid_bitmap && !dev_alloc(&W.valid, kc::mask_words(cap))) ||
        !dev_alloc(&W.flags8, kc::tiles(cap) * kc::kTile))
        return KC_ENOMEM;
    W.cap = cap;
    return KC_OK;
}

// per-tile buffers for n positions or keys
kc_status ensure_tiles(kc::Workspace &W, hipStream_t wait_on, uint64_t n) {
    uint64_t nt = kc::tiles(n) + 1;
    if (W.tile_a && nt <= W.tile_cap)
        return KC_OK;
    if (W.fixed)
        return KC_ERANGE;
    if (!g_size_only && !g_carve)
        (void)hipStreamSynchronize(wait_on);
    dev_free(W.tile_a);
    dev_free(W.tile_b);
    dev_free(W.tile_c);
    dev_free(W.off_a);
    dev_free(W.off_b);
    dev_free(W.off_c);
    dev_free(W.tmask);
    dev_free(W.partial64);
    uint64_t cap = nt < 64 ? 64 : nt + nt / 8;
    W.tile_cap = 0;
    if (!dev_alloc(&W.tile_a, cap) || !dev_alloc(&W.tile_b, cap) || !dev_alloc(&W.tile_c, cap) ||
        !dev_alloc(&W.off_a, cap) || !dev_alloc(&W.off_b, cap) || !dev_alloc(&W.off_c, cap) ||
        !dev_alloc(&W.tmask, cap * (kc::kTile / 64)) ||
        !dev_alloc(&W.partial64, kc::scan_partials(cap)))
        return KC_ENOMEM;
    W.tile_cap = cap;
    return KC_OK;
}

kc_status ensure_positions(kc_filter *f, uint64_t n) {
    return ensure_positions(*f->W, f->last, n, true);
}
kc_status ensure_tiles(kc_filter *f, uint64_t n) { return ensure_tiles(*f->W, f->last, n); }

// binned-path buffers for one chunk of the given plan
kc_status ensure_binned(kc_filter *f, const kc::BinPlan &B, uint64_t chunk_positions) {
    kc::Workspace &W = *f->W;
    // smaller chunks of the same countBF make at most kBinSpread workgroups:
    // room for them too, so that a reservation covers every smaller insert
    const uint64_t g = B.G > kc::kBinSpread ? B.G : kc::kBinSpread;
    const uint64_t n_mat = (uint64_t)B.n_regions * g;
    const uint64_t n_coarse = (uint64_t)B.n_buckets * g;
    const uint64_t n_slots = chunk_positions * f->layout.k_h;
    const uint64_t n_ent = n_slots;
    if (W.matrix && n_mat <= W.matrix_cap && n_coarse <= W.coarse_cap && n_slots <= W.slots_cap &&
        n_ent <= W.entries_cap)
        return KC_OK;
    if (W.fixed)
        return KC_ERANGE;
    wait_idle(f);
    if (!W.matrix || n_mat > W.matrix_cap || n_coarse > W.coarse_cap) {
        dev_free(W.matrix);
        dev_free(W.matrix_t);
        dev_free(W.coarse);
        dev_free(W.partial32);
        W.matrix_cap = W.coarse_cap = 0;
        if (!dev_alloc(&W.matrix, n_mat) || !dev_alloc(&W.matrix_t, n_mat) ||
            !dev_alloc(&W.coarse, n_coarse) || !dev_alloc(&W.partial32, kc::scan_partials(n_mat)))
            return KC_ENOMEM;
        W.matrix_cap = n_mat;
        W.coarse_cap = n_coarse;
    }
    if (!W.slots || n_slots > W.slots_cap) {
        dev_free(W.slots);
        W.slots_cap = 0;
        if (!dev_alloc(&W.slots, n_slots))
            return KC_ENOMEM;
        W.slots_cap = n_slots;
    }
    if (!W.entries || n_ent > W.entries_cap) {
        dev_free(W.entries);
        dev_free(W.bucketed);
        W.entries_cap = 0;
        if (!dev_alloc(&W.entries, n_ent) || !dev_alloc(&W.bucketed, n_ent))
            return KC_ENOMEM;
        W.entries_cap = n_ent;
    }
    return KC_OK;
}

// partitioned binned-path buffers for one chunk of the given plan.  The
// path needs two entry-sized buffers besides its count matrices, each used
// twice (kernels of one stream, in this order):
//   bucketed: slot ids and partition bytes (hashing -> partition scatter),
//             then the bucket lists (list binning -> region binning);
//   entries:  the partition lists (partition scatter -> list binning), then
//             the region lists (region binning -> region pass).
kc_status ensure_parts(kc_filter *f, const kc::BinPlan &B, uint64_t chunk_positions) {
    kc::Workspace &W = *f->W;
    const uint64_t n_slots = chunk_positions * f->layout.k_h;
    const uint64_t n_pmat = (uint64_t)B.n_parts * B.G;
    const uint64_t n_fine = (uint64_t)B.n_regions * B.list_g;
    const uint64_t nbp = (1ull << B.part_log) >> B.bucket_shift;
    const uint64_t n_coarse = (uint64_t)B.n_parts * nbp * B.list_g;
    // the scans share partial32; the list workgroups' rows (matrix_t) are
    // 2^part_log counts long in every partition
    const uint64_t n_rows = (uint64_t)B.n_parts * B.list_g << B.part_log;
    uint64_t n_mat = n_fine > n_pmat ? n_fine : n_pmat;
    if (n_rows > n_mat)
        n_mat = n_rows;
    if (W.entries && W.pbounds && W.pdesc && n_slots <= W.entries_cap && n_pmat <= W.pmat_cap &&
        n_mat <= W.matrix_cap && n_coarse <= W.coarse_cap)
        return KC_OK;
    if (W.fixed)
        return KC_ERANGE;
    wait_idle(f);
    if (!W.pbounds && !dev_alloc(&W.pbounds, kc::kMaxParts + 1))
        return KC_ENOMEM;
    if (!W.pdesc && !dev_alloc(&W.pdesc, 3ull * kc::kMaxParts))
        return KC_ENOMEM;
    if (!W.matrix || n_mat > W.matrix_cap || n_coarse > W.coarse_cap) {
        const uint64_t m = n_mat > W.matrix_cap ? n_mat : W.matrix_cap;
        const uint64_t c = n_coarse > W.coarse_cap ? n_coarse : W.coarse_cap;
        dev_free(W.matrix);
        dev_free(W.matrix_t);
        dev_free(W.coarse);
        dev_free(W.partial32);
        W.matrix_cap = W.coarse_cap = 0;
        if (!dev_alloc(&W.matrix, m) || !dev_alloc(&W.matrix_t, m) || !dev_alloc(&W.coarse, c) ||
            !dev_alloc(&W.partial32, kc::scan_partials(m > c ? m : c)))
            return KC_ENOMEM;
        W.matrix_cap = m;
        W.coarse_cap = c;
    }
    if (!W.pmat || n_pmat > W.pmat_cap) {
        dev_free(W.pmat);
        W.pmat_cap = 0;
        if (!dev_alloc(&W.pmat, n_pmat))
            return KC_ENOMEM;
        W.pmat_cap = n_pmat;
    }
    if (!W.entries || n_slots > W.entries_cap) {
        dev_free(W.entries);
        dev_free(W.bucketed);
        W.entries_cap = 0;
        if (!dev_alloc(&W.entries, n_slots) || !dev_alloc(&W.bucketed, n_slots))
            return KC_ENOMEM;
        W.entries_cap = n_slots;
    }
    return KC_OK;
}

kc_status ensure_scalars(kc::Workspace &W) {
    if (W.totals)
        return KC_OK;
    if (W.fixed)
        return KC_ERANGE;
    if (!dev_alloc(&W.totals, 8) || !dev_alloc(&W.n_entries, 4) ||
        !dev_alloc(&W.win_cursors, kc::kWinCursors))
        return KC_ENOMEM;
    return KC_OK;
}

kc_status ensure_scalars(kc_filter *f) { return ensure_scalars(*f->W); }

// first-seen workspace of the direct path: one entry per counter
kc_status ensure_aux(kc_filter *f, hipStream_t s) {
    if (f->F.aux)
        return KC_OK;
    if (f->W->fixed)
        return KC_ERANGE;
    uint64_t n_aux = f->layout.X * f->layout.Y * f->F.eta;
    if (!dev_alloc(&f->F.aux, n_aux))
        return KC_ENOMEM;
    if (g_size_only)
        return KC_OK;
    return kc::fill_u32(f->F.aux, n_aux, kc::kIdle, s) == hipSuccess ? KC_OK : KC_EDEVICE;
}

void free_workspace(kc::Workspace &W) {
    dev_free(W.codes);
    dev_free(W.inv);
    dev_free(W.rs);
    dev_free(W.valid);
    dev_free(W.flags8);
    dev_free(W.tile_a);
    dev_free(W.tile_b);
    dev_free(W.tile_c);
    dev_free(W.off_a);
    dev_free(W.off_b);
    dev_free(W.off_c);
    dev_free(W.tmask);
    dev_free(W.partial64);
    dev_free(W.matrix);
    dev_free(W.matrix_t);
    dev_free(W.coarse);
    dev_free(W.partial32);
    dev_free(W.slots);
    dev_free(W.bucketed);
    dev_free(W.entries);
    dev_free(W.pmat);
    dev_free(W.pbounds);
    dev_free(W.pdesc);
    W.slots_cap = W.entries_cap = W.matrix_cap = W.coarse_cap = W.pmat_cap = 0;
    dev_free(W.carry);
    dev_free(W.carry_off);
    dev_free(W.carry_n);
    W.carry_cap = W.carry_idx_cap = 0;
    dev_free(W.totals);
    dev_free(W.n_entries);
    dev_free(W.win_cursors);
}

void free_all(kc_filter *f) {
    if (f->caller_scratch) {  // every buffer is a piece of the caller's scratch
        f->own = kc::Workspace{};
        f->F.aux = nullptr;
        f->status = nullptr;
        return;
    }
    free_workspace(f->own);
    dev_free(f->F.aux);
    dev_free(f->status);
}

uint64_t env_u64(const char *name, uint64_t dflt) {
    const char *e = std::getenv(name);
    if (!e || !*e)
        return dflt;
    char *end = nullptr;
    unsigned long long v = std::strtoull(e, &end, 10);
    return end == e ? dflt : (uint64_t)v;
}

// Chunk sizes: the defaults, or KMERCO_CHUNK_POSITIONS (rounded down to a
// multiple of kc::kTile, at least one tile) so that small inputs can
// exercise the multi-chunk paths.
uint64_t chunk_size(uint64_t dflt) {
    uint64_t c = env_u64("KMERCO_CHUNK_POSITIONS", dflt) / kc::kTile * kc::kTile;
    if (c < (uint64_t)kc::kTile)
        c = kc::kTile;
    return c > dflt ? dflt : c;
}

// Insertion path: binned unless the filter is too large for one level of
// regions; KMERCO_PATH=direct|binned forces one (tests compare both).
KcPath path_from_env() {
    const char *e = std::getenv("KMERCO_PATH");
    if (e && std::strcmp(e, "direct") == 0)
        return KcPath::Direct;
    if (e && std::strcmp(e, "binned") == 0)
        return KcPath::Binned;
    return KcPath::Auto;
}

// Partition size of the partitioned binned path: kc::kPartLog regions, or
// fewer with KMERCO_PART_LOG (so that small countBFs can exercise it).
uint32_t part_log_from_env() {
    uint64_t v = env_u64("KMERCO_PART_LOG", kc::kPartLog);
    return v > kc::kPartLog ? kc::kPartLog : (uint32_t)v;
}

// Counters per region of the binned paths: KMERCO_REGION_COUNTERS (8192 or
// 16384) when set, else 16384.
uint32_t region_counters_from_env() {
    const uint64_t v = env_u64("KMERCO_REGION_COUNTERS", kc::kRegionCounters);
    return v == (uint64_t)kc::kSmallRegionCounters ? kc::kSmallRegionCounters
                                                   : kc::kRegionCounters;
}

// The binned plan and chunk size for an insert of n_bases positions; false
// when the direct path is taken.
bool choose_plan(const kc_filter *f, uint64_t n_bases, kc::BinPlan &plan, uint64_t &chunk) {
    if (f->path == KcPath::Direct)
        return false;
    chunk = n_bases < f->bin_chunk ? n_bases : f->bin_chunk;
    if (!kc::bin_plan(f->F, chunk, plan, f->part_log, f->region_counters))
        return false;
    if (plan.n_parts) {
        // entries of a chunk (positions x hash functions) index 32-bit offsets
        const uint64_t most = ((1ull << 32) - 1) / f->layout.k_h / kc::kTile * kc::kTile;
        const uint64_t pc = f->part_chunk < most ? f->part_chunk : most;
        chunk = n_bases < pc ? n_bases : pc;
        return kc::bin_plan(f->F, chunk, plan, f->part_log, f->region_counters);
    }
    return true;
}

kc_status ensure_plan(kc_filter *f, const kc::BinPlan &plan, uint64_t chunk) {
    return plan.n_parts ? ensure_parts(f, plan, chunk) : ensure_binned(f, plan, chunk);
}

// Whether an insert of n_bases in chunks of `chunk` takes the carried
// classification (with a split: the last chunk's region pass classifies
// the earlier chunks' first-seen k-mers).
bool carries(const kc_filter *f, const kc::BinPlan &plan, uint64_t chunk, uint64_t n_bases) {
    return f->carry && f->layout.k_h == 1 && n_bases > chunk && kc::carry_fits(plan);
}

// Its buffers: (chunks - 1) x chunk records of 6 bytes, (chunks - 1) x
// regions offsets and counts.  A workspace carved from caller memory that
// lacks them takes the classification pass instead.
kc_status ensure_carry(kc_filter *f, const kc::BinPlan &plan, uint64_t chunk, uint64_t n_bases) {
    if (!carries(f, plan, chunk, n_bases))
        return KC_OK;
    kc::Workspace &W = *f->W;
    const uint64_t prev = (n_bases + chunk - 1) / chunk - 1;
    const uint64_t cap = prev * chunk;
    const uint64_t idx = prev * plan.n_regions;
    if ((W.carry && cap <= W.carry_cap && idx <= W.carry_idx_cap) || W.fixed)
        return KC_OK;
    wait_idle(f);
    dev_free(W.carry);
    dev_free(W.carry_off);
    dev_free(W.carry_n);
    W.carry_cap = W.carry_idx_cap = 0;
    if (!dev_alloc(&W.carry, 3 * cap) || !dev_alloc(&W.carry_off, idx) ||
        !dev_alloc(&W.carry_n, idx))
        return KC_ENOMEM;
    W.carry_cap = cap;
    W.carry_idx_cap = idx;
    return KC_OK;
}

// Every binned-path buffer of an insert of n_bases.
kc_status ensure_insert(kc_filter *f, const kc::BinPlan &plan, uint64_t chunk, uint64_t n_bases) {
    kc_status st = ensure_plan(f, plan, chunk);
    return st == KC_OK ? ensure_carry(f, plan, chunk, n_bases) : st;
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

// Every buffer inserts of up to max_bases bases (and classifications of up
// to max_bases keys) need, in the current dev_alloc mode: kc_reserve
// allocates them, kc_scratch_bytes counts them, kc_create_in carves them.
kc_status reserve_all(kc_filter *f, uint64_t max_bases) {
    kc_status st = ensure_scalars(f);
    if (st == KC_OK)
        st = ensure_positions(f, max_bases);
    if (st == KC_OK)
        st = ensure_tiles(f, max_bases);
    if (st != KC_OK || max_bases == 0)
        return st;
    kc::BinPlan plan{};
    uint64_t bchunk = 0;
    if (choose_plan(f, max_bases, plan, bchunk))
        return ensure_insert(f, plan, bchunk, max_bases);
    return ensure_aux(f, f->last);
}

bool takes_binned_path(const kc_filter *f, uint64_t n_bases) {
    kc::BinPlan plan{};
    uint64_t chunk = 0;
    return n_bases == 0 || choose_plan(f, n_bases, plan, chunk);
}

void share_workspace(kc_filter *f, kc::Workspace *W) { f->W = W ? W : &f->own; }

uint64_t filter_private_bytes(const kc_layout &layout) {
    kc::FilterArgs F{};
    F.X = layout.X;
    F.Y = layout.Y;
    F.eta = 64u / layout.alpha;
    kc::BinPlan plan{};
    if (path_from_env() != KcPath::Direct &&
        kc::bin_plan(F, 1u << 16, plan, part_log_from_env(), region_counters_from_env()))
        return 0;
    return layout.X * layout.Y * F.eta * sizeof(uint32_t);
}

// The layout-derived state of a handle: dimensions and reduction constants,
// chunk sizes and path choices (no device state).
void init_filter(kc_filter *f, const kc_layout *layout) {
    f->layout = *layout;
    f->W = &f->own;
    f->k = 0;
    f->chunk = chunk_size(kc::kChunk);
    f->bin_chunk = chunk_size(kc::kBinChunk);
    f->part_chunk = chunk_size(kc::kPartChunk);
    f->part_log = part_log_from_env();
    f->region_counters = region_counters_from_env();
    f->carry = env_u64("KMERCO_CARRY", 1) != 0;
    f->path = path_from_env();
    kc::FilterArgs &F = f->F;
    F.words = nullptr;
    F.aux = nullptr;
    F.X = layout->X;
    F.Y = layout->Y;
    F.mX = UINT64_MAX / layout->X;
    F.mY = UINT64_MAX / layout->Y;
    F.alpha = layout->alpha;
    F.eta = 64u / layout->alpha;
    F.mEta = UINT64_MAX / F.eta;
    F.eta_pow2 = (F.eta & (F.eta - 1)) == 0;
    F.small_dims = layout->X <= kc::kSmallDivisor && layout->Y <= kc::kSmallDivisor;
    F.k_h = layout->k_h;
    F.field_max = (layout->alpha >= 64) ? ~0ull : ((1ull << layout->alpha) - 1ull);
}

// Everything of an insert after its reads are ingested into W's
// per-position buffers (codes, bitmaps and flag bytes of positions
// 0..n_bases): the valid-window bitmap, the chunks, the distinct output and
// the split; W's other buffers are prepared for n_bases.  Kernels only.
kc_status insert_core(kc_filter *f, const kc::Workspace &W, uint64_t n_bases, uint32_t k,
                      bool binned, const kc::BinPlan &plan, uint64_t bchunk, uint64_t *distinct,
                      uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows, uint32_t tau,
                      uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                      uint64_t cap_te, hipStream_t s, kc::Profiler *P) {
    const bool split = trust != nullptr;
    hipError_t e = hipSuccess;
    if (binned)
        e = kc::launch_valid_windows(n_bases, k, W, s, P);
    if (e == hipSuccess && binned)  // valid windows, accumulated by the bin passes
        e = kc::fill_u64(W.totals + 5, 1, 0ull, s);
    if (e != hipSuccess)
        return KC_EDEVICE;
    kc::ReadsArgs R{W.codes, W.inv, W.rs, n_bases, k, W.valid};
    const uint64_t chunk = binned ? bchunk : f->chunk;
    // The split is taken from marks on the distinct flags: the region pass
    // of the last chunk marks the k-mers first seen in it (one hash function:
    // their one counter's final value is known there); the flags of earlier
    // chunks (and every flag with several hash functions or on the direct
    // path) are marked afterwards against the final countBF.
    const bool region_marks = split && binned && f->F.k_h == 1;
    // With several chunks, the earlier chunks' first-seen k-mers either wait
    // as records for the last chunk's region pass (carried) or are marked
    // afterwards by a pass that rereads their counters.
    const uint64_t n_chunks = (n_bases + chunk - 1) / chunk;
    kc::Carry carry{};
    if (region_marks && carries(f, plan, chunk, n_bases))
        carry = kc::carry_of(W, plan, chunk, n_chunks);
    uint64_t last_c0 = 0;
    uint32_t j = 0;
    for (uint64_t c0 = 0; c0 < n_bases; c0 += chunk, j++) {
        uint64_t c1 = c0 + chunk < n_bases ? c0 + chunk : n_bases;
        last_c0 = c0;
        if (binned) {
            kc::Carry cj = carry;
            if (carry.n_prev) {
                cj.mode = c1 == n_bases ? kc::Carry::kIn : kc::Carry::kOut;
                cj.chunk = j;
            }
            e = kc::launch_binned_chunk(f->F, R, c0, c1, plan, W, region_marks && c1 == n_bases,
                                        tau, cj, s, P);
        } else {
            e = kc::launch_insert_chunk(f->F, R, c0, c1, f->zero, W, s, P);
        }
        if (e != hipSuccess)
            return KC_EDEVICE;
        f->zero = false;
    }
    for (uint32_t c = 0; c < carry.n_prev; c++)
        if (kc::launch_carried_winners(plan, carry, c, (uint64_t)c * chunk, chunk, W, s, P) !=
            hipSuccess)
            return KC_EDEVICE;
    if (split && !carry.n_prev) {
        const uint64_t unmarked = region_marks ? last_c0 : n_bases;
        if (kc::launch_classify_flags(f->F, R, W, unmarked, tau, s, P) != hipSuccess)
            return KC_EDEVICE;
    }
    e = kc::launch_distinct(R, W, distinct, cap_d, n_distinct, n_windows, trust, n_trust, err,
                            n_err, cap_te, f->status, binned, s, P);
    return e == hipSuccess ? KC_OK : KC_EDEVICE;
}

// Both phases for one call.  trust == nullptr: insertion only.
kc_status insert_impl(kc_filter *f, const uint8_t *reads, const uint64_t *offsets,
                      uint64_t n_reads, uint64_t n_bases, uint32_t k, uint64_t *distinct,
                      uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows, uint32_t tau,
                      uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                      uint64_t cap_te, hipStream_t s) {
    const bool split = trust != nullptr;
    f->last = s;
    kc_status st = ensure_scalars(f);
    if (st != KC_OK)
        return st;
    if (n_bases == 0) {
        if (split && (kc::fill_u64(n_trust, 1, 0, s) != hipSuccess ||
                      kc::fill_u64(n_err, 1, 0, s) != hipSuccess))
            return KC_EDEVICE;
        f->k = k;
        return KC_OK;
    }
    if ((st = ensure_positions(f, n_bases)) != KC_OK || (st = ensure_tiles(f, n_bases)) != KC_OK)
        return st;
    kc::BinPlan plan{};
    uint64_t bchunk = 0;
    const bool binned = choose_plan(f, n_bases, plan, bchunk);
    if (f->path == KcPath::Binned && !binned)
        return KC_EINVAL;  // forced binned path but the filter does not fit it
    if (k > 32 && !binned)
        return KC_EINVAL;  // k-mers of 33..64 bases take the binned paths only
    if (binned) {
        if ((st = ensure_insert(f, plan, bchunk, n_bases)) != KC_OK)
            return st;
    } else if ((st = ensure_aux(f, s)) != KC_OK) {
        return st;
    }
    f->k = k;  // every check passed: the filter now holds k-mers of this length
    if (kc::launch_ingest(reads, n_bases, offsets, n_reads, *f->W, s, &f->prof) != hipSuccess)
        return KC_EDEVICE;
    return insert_core(f, *f->W, n_bases, k, binned, plan, bchunk, distinct, cap_d, n_distinct,
                       n_windows, tau, trust, n_trust, err, n_err, cap_te, s, &f->prof);
}

kc_status check_range(const kc_filter *f, uint64_t n_bases, uint32_t k) {
    if (k < 1 || k > 64)
        return KC_EINVAL;
    if (f->k != 0 && f->k != k)
        return KC_ESTATE;
    kc::BinPlan plan{};
    uint64_t bchunk = 0;
    const bool binned = n_bases == 0 || choose_plan(f, n_bases, plan, bchunk);
    if ((f->path == KcPath::Binned || k > 32) && !binned)
        return KC_EINVAL;
    return KC_OK;
}

kc_status prepare_range(kc_filter *f, uint64_t n_bases) {
    kc_status st = ensure_scalars(f);
    if (st == KC_OK)
        st = ensure_tiles(f, n_bases);
    if (st != KC_OK || n_bases == 0)
        return st;
    kc::BinPlan plan{};
    uint64_t bchunk = 0;
    if (choose_plan(f, n_bases, plan, bchunk))
        return ensure_insert(f, plan, bchunk, n_bases);
    return ensure_aux(f, f->last);
}

kc_status insert_range(kc_filter *f, const kc::Workspace &pos, uint64_t base, uint64_t n_bases,
                       uint32_t k, bool reset, bool replayed, uint64_t *distinct,
                       uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows, uint32_t tau,
                       uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                       uint64_t cap_te, hipStream_t s, kc::Profiler *P) {
    if (base % kc::kTile != 0)
        return KC_EINVAL;
    hipError_t e = hipSuccess;
    if (reset) {
        if (P)
            P->begin(kc::kPhReset, s);
        e = kc::fill_u64(f->F.words, f->layout.X * f->layout.Y, 0ull, s);
        if (P)
            P->end(s);
        if (e == hipSuccess)
            e = kc::fill_u64(n_distinct, 1, 0ull, s);
        if (e == hipSuccess && n_windows)
            e = kc::fill_u64(n_windows, 1, 0ull, s);
        if (e != hipSuccess)
            return KC_EDEVICE;
    }
    // the direct path's empty-filter variant only when the filter is known
    // to be empty whenever these launches run (a graph replays them later)
    f->zero = reset || (f->zero && !replayed);
    if (n_bases == 0) {
        if (trust && (kc::fill_u64(n_trust, 1, 0, s) != hipSuccess ||
                      kc::fill_u64(n_err, 1, 0, s) != hipSuccess))
            return KC_EDEVICE;
        f->k = k;
        return KC_OK;
    }
    kc::BinPlan plan{};
    uint64_t bchunk = 0;
    const bool binned = choose_plan(f, n_bases, plan, bchunk);
    f->k = k;
    // the set's positions in the shared per-position buffers (base is a
    // multiple of the 1024-position tile: whole bitmap words, code words and
    // flag tiles); every other buffer is f's
    kc::Workspace V = *f->W;
    V.codes = pos.codes + base / 16;
    V.inv = pos.inv + base / 32;
    V.rs = pos.rs + base / 32;
    V.valid = pos.valid + base / 32;
    V.flags8 = pos.flags8 + base;
    return insert_core(f, V, n_bases, k, binned, plan, bchunk, distinct, cap_d, n_distinct,
                       n_windows, tau, trust, n_trust, err, n_err, cap_te, s, P);
}

}  // namespace kcapi

using namespace kcapi;

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

int kc_version(void) { return 2; }

uint32_t kc_eta(uint32_t alpha) { return (alpha >= 1 && alpha <= 64) ? 64u / alpha : 0u; }

uint64_t kc_filter_bytes(const kc_layout *layout) {
    return valid_layout(layout) ? layout->X * layout->Y * sizeof(uint64_t) : 0u;
}

uint64_t kc_scratch_bytes(const kc_layout *layout, uint64_t max_bases) {
    if (!valid_layout(layout))
        return 0;
    // the status word and kc_reserve's allocations on a handle of this
    // layout, counted, not made (the order kc_create_in carves them in)
    kc_filter f{};
    init_filter(&f, layout);
    uint64_t bytes = 0;
    kc_status st = KC_OK;
    {
        SizeOnly mode(&bytes);
        st = dev_alloc(&f.status, 1) ? reserve_all(&f, max_bases) : KC_ENOMEM;
    }
    f.own = kc::Workspace{};  // placeholders only
    f.F.aux = nullptr;
    f.status = nullptr;
    return st == KC_OK ? bytes : 0u;
}

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

kc_status kc_create_in(const kc_layout *layout, uint64_t *words_dev, int zero, uint32_t k,
                       void *scratch_dev, uint64_t scratch_bytes, uint64_t max_bases,
                       void *stream, kc_filter **out) {
    if (!out)
        return KC_EINVAL;
    *out = nullptr;
    if (!words_dev || !valid_layout(layout) || k > 64)
        return KC_EINVAL;
    if (scratch_dev && (uintptr_t)scratch_dev % kAllocAlign != 0)
        return KC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return KC_EDEVICE;
    kc_filter *f = new (std::nothrow) kc_filter();
    if (!f)
        return KC_ENOMEM;
    init_filter(f, layout);
    f->device = dev;
    f->zero = zero != 0;
    f->k = k;
    f->last = (hipStream_t)stream;
    f->F.words = words_dev;
    f->generation = next_generation();
    hipStream_t s = (hipStream_t)stream;
    kc_status st = KC_OK;
    if (scratch_dev) {
        // every device buffer of the handle is a piece of the caller's
        // scratch, laid out once here in the order kc_scratch_bytes counts
        f->caller_scratch = true;
        Carve c;
        c.base = (uint8_t *)scratch_dev;
        c.size = scratch_bytes;
        {
            Carving mode(&c);
            st = dev_alloc(&f->status, 1) ? reserve_all(f, max_bases) : KC_ENOMEM;
        }
        if (st == KC_ENOMEM)
            st = KC_ERANGE;  // smaller than kc_scratch_bytes(layout, max_bases)
        f->own.fixed = true;
    } else {
        st = dev_alloc(&f->status, 1) ? KC_OK : KC_ENOMEM;
        if (st == KC_OK && max_bases > 0)
            st = reserve_all(f, max_bases);
    }
    if (st != KC_OK) {
        (void)hipStreamSynchronize(s);
        free_all(f);
        delete f;
        return st;
    }
    hipError_t e = kc::fill_u32(f->status, 1, 0u, s);
    if (e == hipSuccess && zero)
        e = kc::fill_u64(words_dev, layout->X * layout->Y, 0ull, s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        free_all(f);
        delete f;
        return KC_EDEVICE;
    }
    *out = f;
    return KC_OK;
}

kc_status kc_create(const kc_layout *layout, uint64_t *words_dev, int zero, void *stream,
                    kc_filter **out) {
    return kc_create_in(layout, words_dev, zero, 0, nullptr, 0, 0, stream, out);
}

void kc_destroy(kc_filter *f) {
    if (!f)
        return;
    DeviceGuard g(f->device);
    (void)hipDeviceSynchronize();
    f->prof.release();
    free_all(f);
    delete f;
}

kc_status kc_reserve(kc_filter *f, uint64_t max_bases) {
    if (!f)
        return KC_EINVAL;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    return reserve_all(f, max_bases);
}

kc_status kc_get_plan(const kc_filter *f, uint64_t n_bases, kc_plan *out) {
    if (!f || !out)
        return KC_EINVAL;
    *out = kc_plan{};
    kc::BinPlan plan{};
    uint64_t chunk = 0;
    if (n_bases > 0 && choose_plan(f, n_bases, plan, chunk)) {
        out->path = plan.n_parts ? KC_PATH_PARTITIONED : KC_PATH_BINNED;
        out->region_cells = 1u << plan.region_shift;
        out->n_regions = plan.n_regions;
        out->n_parts = plan.n_parts;
        out->chunk = chunk;
    } else {
        out->path = n_bases > 0 ? KC_PATH_DIRECT : KC_PATH_BINNED;
        out->chunk = n_bases > 0 ? f->chunk : 0;
    }
    out->n_chunks = out->chunk ? (n_bases + out->chunk - 1) / out->chunk : 0;
    if (out->path != KC_PATH_DIRECT && n_bases > 0 && carries(f, plan, chunk, n_bases)) {
        // the insert allocates the records unless the workspace is fixed
        const kc::Carry c = kc::carry_of(*f->W, plan, chunk, out->n_chunks);
        out->carried = (c.n_prev || !f->W->fixed) ? 1u : 0u;
    }
    return KC_OK;
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
    if (!f || k < 1 || k > 64 || !n_distinct_dev)
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
    return insert_impl(f, reads_dev, offsets_dev, n_reads, n_bases, k, distinct_dev, distinct_cap,
                       n_distinct_dev, n_windows_dev, 0, nullptr, nullptr, nullptr, nullptr, 0,
                       (hipStream_t)stream);
}

kc_status kc_insert_classify(kc_filter *f, const uint8_t *reads_dev, const uint64_t *offsets_dev,
                             uint64_t n_reads, uint64_t n_bases, uint32_t k, uint32_t tau,
                             uint64_t *distinct_dev, uint64_t distinct_cap,
                             uint64_t *n_distinct_dev, uint64_t *n_windows_dev,
                             uint64_t *trust_dev, uint64_t *n_trust_dev, uint64_t *err_dev,
                             uint64_t *n_err_dev, uint64_t class_cap, void *stream) {
    if (!f || k < 1 || k > 64 || !n_distinct_dev || !n_trust_dev || !n_err_dev)
        return KC_EINVAL;
    if (n_bases > 0 && (!reads_dev || !offsets_dev))
        return KC_EINVAL;
    if ((distinct_cap > 0 && !distinct_dev) || (class_cap > 0 && (!trust_dev || !err_dev)))
        return KC_EINVAL;
    if (f->k != 0 && f->k != k)
        return KC_ESTATE;
    DeviceGuard g(f->device);
    if (!g.ok)
        return KC_EDEVICE;
    // a non-null marker selects the classification outputs even at capacity 0
    uint64_t *trust = trust_dev ? trust_dev : n_trust_dev;
    uint64_t *err = err_dev ? err_dev : n_err_dev;
    return insert_impl(f, reads_dev, offsets_dev, n_reads, n_bases, k, distinct_dev, distinct_cap,
                       n_distinct_dev, n_windows_dev, tau, trust, n_trust_dev, err, n_err_dev,
                       class_cap, (hipStream_t)stream);
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
    kc_status st = ensure_scalars(f);
    if (st == KC_OK)
        st = ensure_tiles(f, keys_cap);
    if (st != KC_OK)
        return st;
    hipError_t e = kc::launch_classify(f->F, keys_dev, n_keys_dev, nullptr, keys_cap, keys_cap,
                                       tau, trust_dev, n_trust_dev, err_dev, n_err_dev, keys_cap,
                                       nullptr, *f->W, s, &f->prof, f->k > 32);
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
    return kc::launch_query(f->F, keys_dev, n, freq_dev, s, &f->prof, f->k > 32) == hipSuccess
               ? KC_OK
               : KC_EDEVICE;
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
    // the direct path's first-seen workspace is idle again after every insert
    f->zero = true;
    f->k = 0;
    return KC_OK;
}

kc_status kc_profile(kc_filter *f, int enable) {
    if (!f)
        return KC_EINVAL;
    f->prof.collect(nullptr, nullptr, 0);
    f->prof.on = enable != 0;
    f->prof.mask = ~0u;
    return KC_OK;
}

kc_status kc_profile_phases(kc_filter *f, uint32_t mask) {
    if (!f)
        return KC_EINVAL;
    f->prof.collect(nullptr, nullptr, 0);
    f->prof.on = mask != 0;
    f->prof.mask = mask;
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
        "classify_mark", "classify_scatter", "query", "reset", "bin_count", "bin_bucket",
        "region", "tile_count", "bin_region", "bin_part", "part_count", "valid_windows",
        "winners"};
    return phase < (uint32_t)kc::kPhCount ? names[phase] : "unknown";
}

}  // extern "C"
