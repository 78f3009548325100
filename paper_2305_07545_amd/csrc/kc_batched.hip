// Batched insertion: many independent read sets, each with its own countBF,
// k and tau, processed by one launch per phase.
//
// The sets' reads sit in one buffer; set s owns positions
// [base_s, base_s + n_s) with base_s a multiple of kSetAlign, so no tile of
// the shared per-position kernels straddles two sets.  Work items are
// (set, tile of T positions).  Every set's filter is cut into regions as on
// the single-set binned path; the sets' region-major count blocks are laid
// end to end and scanned once, which gives every (set, region, item) its
// segment of one shared entry list.  Entries are counting-sorted by region
// in LDS per batch (a set's filter has at most kBatchMaxRegions regions),
// one workgroup per region of every set counts hits and first occurrences
// in LDS, and a single compaction writes each set's distinct (and
// trustworthy / erroneous) k-mers to that set's outputs.
#include <hip/hip_runtime.h>

#include "kc_batched.hpp"
#include "kc_bin_hash.hpp"
#include "kc_device.hpp"
#include "kc_kernels.hpp"

namespace kc {

namespace {

// Positions of work item i: set s, tile j of the set.
struct Item {
    uint32_t s;
    uint64_t g0, g1;  // absolute positions
    uint32_t j;
};

__device__ __forceinline__ Item item_of(const SetDesc *__restrict__ sets,
                                        const uint32_t *__restrict__ item_set, uint32_t i,
                                        uint64_t tile) {
    Item it;
    it.s = item_set[i];
    const SetDesc &S = sets[it.s];
    it.j = i - S.item_base;
    it.g0 = S.base + (uint64_t)it.j * tile;
    const uint64_t end = S.base + S.n_bases;
    it.g1 = it.g0 + tile < end ? it.g0 + tile : end;
    return it;
}

}  // namespace

// Clear the countBFs and the call counters of every set (batch reset).
__global__ void kb_reset(const SetDesc *__restrict__ sets, uint32_t n_sets) {
    const uint32_t s = blockIdx.y;
    if (s >= n_sets)
        return;
    const SetDesc &S = sets[s];
    const uint64_t n = S.F.X * S.F.Y;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        S.F.words[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *S.n_distinct = 0;
        if (S.n_windows)
            *S.n_windows = 0;
    }
}

__global__ void kb_zero_valid(unsigned long long *__restrict__ valid, uint32_t n_sets) {
    for (uint32_t s = threadIdx.x; s < n_sets; s += blockDim.x)
        valid[s] = 0;
}

// The valid-window bitmap words of an item's positions, for its set's k
// (items start at multiples of 64 positions, so that no word spans two).
__global__ void __launch_bounds__(256) kb_valid(const SetDesc *__restrict__ sets,
                                                const uint32_t *__restrict__ item_set,
                                                ReadsArgs R, uint64_t tile, uint64_t n_words,
                                                uint32_t *__restrict__ valid) {
    const Item it = item_of(sets, item_set, blockIdx.x, tile);
    const SetDesc &S = sets[it.s];
    const uint64_t w1 = (it.g1 + 31u) / 32u;
    for (uint64_t w = it.g0 / 32u + threadIdx.x; w < w1 && w < n_words; w += 256u)
        valid[w] = valid_word(R.inv, R.rs, n_words, w, S.k, S.base + S.n_bases);
}

// Slot ids of an item's windows and its per-region counts, hashed as in the
// single-set bin pass (walk_windows, window_counters); kFast: every set has
// the fast layout (checked by the planner).
template <bool kFast>
__global__ void __launch_bounds__(kBinWG) kb_bin_count(const SetDesc *__restrict__ sets,
                                                       const uint32_t *__restrict__ item_set,
                                                       ReadsArgs R, uint64_t tile,
                                                       uint32_t *__restrict__ slots,
                                                       uint32_t *__restrict__ matrix,
                                                       unsigned long long *__restrict__ valid) {
    __shared__ uint32_t s_hist[kBatchMaxRegions];
    __shared__ uint32_t s_ring[kBinWG / 64][kWindowRing];
    __shared__ uint32_t s_valid;
    const Item it = item_of(sets, item_set, blockIdx.x, tile);
    const SetDesc &S = sets[it.s];
    const FilterArgs F = S.F;
    for (uint32_t i = threadIdx.x; i < S.n_regions; i += kBinWG)
        s_hist[i] = 0;
    if (threadIdx.x == 0)
        s_valid = 0;
    __syncthreads();
    R.k = S.k;
    // set-relative 32-bit positions (sets start at multiples of 4096)
    const uint32_t *__restrict__ codes = R.codes + (S.base >> 4);
    uint32_t *__restrict__ sl = slots + S.slot_base;
    const uint64_t nb = S.n_bases;
    const uint32_t K = S.k, shift = S.region_shift, k_h = kFast ? 1u : F.k_h;
    const uint32_t nv = walk_windows(
        R, it.g0, it.g1, S.base, s_ring[wave_id()],
        [&](uint32_t q) {
            for (uint32_t a = 0; a < k_h; a++)
                sl[(uint64_t)a * nb + q] = kNoSlot;
        },
        [&](uint32_t q) {
            window_counters<kFast, false>(F, codes, q, K, shift, [&](uint32_t a, uint32_t r,
                                                                       uint32_t local) {
                sl[(uint64_t)(a - 1) * nb + q] = (r << kLocalBits) | local;
                atomicAdd(&s_hist[r], 1u);
            });
        });
    if ((threadIdx.x & 63u) == 0)
        atomicAdd(&s_valid, nv);
    __syncthreads();
    // the item's counts as one contiguous row of the set's block (kb_transpose
    // makes the block region-major)
    for (uint32_t r = threadIdx.x; r < S.n_regions; r += kBinWG)
        matrix[S.mat_base + (uint64_t)it.j * S.n_regions + r] = s_hist[r];
    if (threadIdx.x == 0)
        atomicAdd(&valid[it.s], (unsigned long long)s_valid);
}

// Each set's G x n_regions block of item rows -> its n_regions x G
// region-major block (blockIdx.z = set; 64 x 64 LDS tiles, tiles outside
// the set's block return at once).
__global__ void __launch_bounds__(256) kb_transpose(const SetDesc *__restrict__ sets,
                                                    const uint32_t *__restrict__ in,
                                                    uint32_t *__restrict__ out) {
    __shared__ uint32_t t[64][65];
    const SetDesc &S = sets[blockIdx.z];
    const uint32_t rows = S.G, cols = S.n_regions;
    const uint32_t c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    if (c0 >= cols || r0 >= rows)
        return;
    const uint32_t *__restrict__ src = in + S.mat_base;
    uint32_t *__restrict__ dst = out + S.mat_base;
    const uint32_t tx = threadIdx.x & 63u, ty = threadIdx.x >> 6;
    for (uint32_t j = ty; j < 64; j += 4) {
        const uint32_t r = r0 + j, c = c0 + tx;
        if (r < rows && c < cols)
            t[j][tx] = src[(uint64_t)r * cols + c];
    }
    __syncthreads();
    for (uint32_t j = ty; j < 64; j += 4) {
        const uint32_t c = c0 + j, r = r0 + tx;
        if (c < cols && r < rows)
            dst[(uint64_t)c * rows + r] = t[tx][j];
    }
}

// Slot ids of an item -> its segments of the entry list, counting-sorted by
// region in LDS per batch of kWriteStage entries.  The large batch keeps the
// runs written per region long even for sets of 2048 regions (runs of the
// smaller level-1 batches of the single-set path would be 2 entries there).
constexpr int kWriteStage = 16384;  // 128 KiB of staged entries
constexpr uint32_t kWriteStageLog = 14;
static_assert(kWriteStage == (1 << kWriteStageLog), "stage size");

__global__ void __launch_bounds__(kBinWG) kb_bin_write(const SetDesc *__restrict__ sets,
                                                       const uint32_t *__restrict__ item_set,
                                                       uint64_t tile,
                                                       const uint32_t *__restrict__ slots,
                                                       const uint32_t *__restrict__ offsets,
                                                       uint64_t *__restrict__ entries,
                                                       uint64_t cap) {
    constexpr int kPer = kWriteStage / kBinWG;
    constexpr int kScanPer = kBatchMaxRegions / kBinWG;
    __shared__ uint64_t s_stage[kWriteStage];
    __shared__ uint32_t s_cnt[kBatchMaxRegions];
    __shared__ uint16_t s_start[kBatchMaxRegions];  // < kWriteStage
    __shared__ uint32_t s_cursor[kBatchMaxRegions];
    __shared__ uint32_t s_wave[kBinWG / 64];
    __shared__ uint32_t s_total;
    const Item it = item_of(sets, item_set, blockIdx.x, tile);
    const SetDesc &S = sets[it.s];
    const uint32_t nr = S.n_regions;
    const uint32_t k_h = S.F.k_h;
    for (uint32_t r = threadIdx.x; r < kBatchMaxRegions; r += kBinWG) {
        s_cursor[r] = r < nr ? offsets[S.mat_base + (uint64_t)r * S.G + it.j] : 0u;
        s_cnt[r] = 0;
    }
    __syncthreads();
    uint32_t bl = 0;
    while ((1u << bl) < k_h)
        bl++;
    const uint32_t batch_log = kWriteStageLog - bl;
    const uint32_t batch = 1u << batch_log;
    // set-relative positions and slot offsets fit 32 bits (sets hold at most
    // 2^28 bases, k_h <= 8)
    const uint32_t q_lo = (uint32_t)(it.g0 - S.base), q_hi = (uint32_t)(it.g1 - S.base);
    const uint32_t nb = (uint32_t)S.n_bases;
    const uint32_t *__restrict__ sl = slots + S.slot_base;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    // A full batch of one hash function is loaded 16 bytes per lane (slot
    // bases are multiples of 4 and q0 of 512: a thread's entries 4v .. 4v + 3
    // are consecutive positions); other batches one slot id per lane.
    // pos_of: the batch index of a thread's entry u.
    static_assert(kPer % 4 == 0, "whole 16-byte loads per thread");
    auto pos_of = [&](bool vec, int u) -> uint32_t {
        return vec ? (uint32_t)(u >> 2) * (4u * kBinWG) + 4u * threadIdx.x + (uint32_t)(u & 3)
                   : threadIdx.x + (uint32_t)u * kBinWG;
    };
    for (uint32_t q0 = q_lo; q0 < q_hi; q0 += batch) {
        const uint32_t nq = (q_hi - q0 < batch ? q_hi - q0 : batch);
        const bool vec = k_h == 1u && nq == batch;
        uint32_t id[kPer];
        if (vec) {
            const uint4 *p4 = reinterpret_cast<const uint4 *>(sl + q0);
#pragma unroll
            for (int v = 0; v < kPer / 4; v++) {
                const uint4 x = p4[(uint32_t)v * kBinWG + threadIdx.x];
                id[4 * v] = x.x;
                id[4 * v + 1] = x.y;
                id[4 * v + 2] = x.z;
                id[4 * v + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int u = 0; u < kPer; u++) {
                const uint32_t i = threadIdx.x + (uint32_t)u * kBinWG;
                const uint32_t a = i >> batch_log;
                const uint32_t qq = i & (batch - 1u);
                id[u] = (a < k_h && qq < nq) ? sl[a * nb + q0 + qq] : kNoSlot;
            }
        }
        uint32_t rk[kPer];  // entry u's rank among its region's in the batch
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (id[u] != kNoSlot)
                rk[u] = atomicAdd(&s_cnt[id[u] >> kLocalBits], 1u);
        __syncthreads();
        {  // exclusive scan of the region counts: kScanPer per thread
            uint32_t v[kScanPer];
            uint32_t sum = 0;
#pragma unroll
            for (int u = 0; u < kScanPer; u++) {
                v[u] = s_cnt[threadIdx.x * kScanPer + u];
                sum += v[u];
            }
            uint32_t incl = sum;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d)
                    incl += o;
            }
            if (lane == 63)
                s_wave[wave] = incl;
            __syncthreads();
            uint32_t run = incl - sum;
            for (uint32_t w = 0; w < wave; w++)
                run += s_wave[w];
#pragma unroll
            for (int u = 0; u < kScanPer; u++) {
                s_start[threadIdx.x * kScanPer + u] = (uint16_t)run;
                run += v[u];
            }
            if (threadIdx.x == kBinWG - 1)
                s_total = run;  // staged entries of this batch (<= kWriteStage)
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (id[u] != kNoSlot) {
                const uint32_t i = pos_of(vec, u);
                const uint32_t q = q0 + (i & (batch - 1u));
                const uint32_t r = id[u] >> kLocalBits;
                const uint32_t j = s_start[r] + rk[u];
                s_stage[j] = ((uint64_t)q << 32) | id[u];
            }
        __syncthreads();
        const uint32_t n_stage = s_total;
        for (uint32_t j = threadIdx.x; j < n_stage; j += kBinWG) {
            const uint64_t e = s_stage[j];
            const uint32_t r = (uint32_t)e >> kLocalBits;
            const uint64_t dst = (uint64_t)s_cursor[r] + (j - s_start[r]);
            if (dst < cap)
                entries[dst] = e;
        }
        __syncthreads();
        for (uint32_t r = threadIdx.x; r < kBatchMaxRegions; r += kBinWG) {
            s_cursor[r] += s_cnt[r];
            s_cnt[r] = 0;
        }
        __syncthreads();
    }
}

// One workgroup per region of every set (as the single-set region kernel).
__global__ void __launch_bounds__(kRegionWG) kb_region(const SetDesc *__restrict__ sets,
                                                       uint32_t n_sets,
                                                       const uint32_t *__restrict__ region_set,
                                                       const uint32_t *__restrict__ offsets,
                                                       const uint32_t *__restrict__ n_entries,
                                                       const uint64_t *__restrict__ entries,
                                                       uint64_t cap,
                                                       uint8_t *__restrict__ flags) {
    __shared__ uint32_t hits[kRegionCounters];
    __shared__ uint32_t first[kRegionCounters];
    const uint32_t s = region_set[blockIdx.x];
    const SetDesc &S = sets[s];
    const FilterArgs F = S.F;
    const uint32_t r = blockIdx.x - S.region_base;
    const uint32_t shift = S.region_shift;
    const uint32_t Sw = 1u << shift;
    for (uint32_t i = threadIdx.x; i < Sw * F.eta; i += kRegionWG) {
        hits[i] = 0;
        first[i] = kIdle;
    }
    __syncthreads();
    const uint64_t e0 = offsets[S.mat_base + (uint64_t)r * S.G];
    uint64_t e1;
    if (r + 1 < S.n_regions)
        e1 = offsets[S.mat_base + (uint64_t)(r + 1) * S.G];
    else
        e1 = s + 1 < n_sets ? offsets[sets[s + 1].mat_base] : *n_entries;
    if (e1 > cap)
        e1 = cap;
    constexpr int kUnroll = 8;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += (uint64_t)kUnroll * kRegionWG) {
        uint64_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const uint64_t x = e + (uint64_t)u * kRegionWG;
            v[u] = x < e1 ? entries[x] : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            if (v[u] == ~0ull)
                continue;
            const uint32_t local = (uint32_t)v[u] & (kRegionCounters - 1);
            atomicAdd(&hits[local], 1u);
            atomicMin(&first[local], (uint32_t)(v[u] >> 32));
        }
    }
    __syncthreads();
    const uint64_t wbase = (uint64_t)r << shift;
    const uint64_t n_words = F.X * F.Y;
    const uint32_t nw = wbase + Sw <= n_words ? Sw : (uint32_t)(n_words - wbase);
    for (uint32_t w = threadIdx.x; w < nw; w += kRegionWG) {
        const uint64_t pre = F.words[wbase + w];
        uint64_t next = pre;
        for (uint32_t l = 0; l < F.eta; l++) {
            const uint32_t idx = (l << shift) | w;
            const uint64_t h = hits[idx];
            if (h == 0)
                continue;
            const uint32_t sh = F.alpha * l;
            const uint64_t pf = (pre >> sh) & F.field_max;
            const uint64_t room = F.field_max - pf;
            const uint64_t nf = pf + (h < room ? h : room);
            next = (next & ~(F.field_max << sh)) | (nf << sh);
            if (pf == 0) {
                uint8_t flag = 1;
                if (S.fused && nf > (uint64_t)S.tau)
                    flag = 3;
                flags[S.base + first[idx]] = flag;
            }
        }
        if (next != pre)
            F.words[wbase + w] = next;
    }
}

// Per tile of every set, one wavefront per tile: the set's ordered outputs
// (as k_compact).  Sets start at multiples of 4096 positions, so a tile
// belongs to one set.
__global__ void __launch_bounds__(kWG) kb_compact(const SetDesc *__restrict__ sets,
                                                  const uint32_t *__restrict__ tile_set,
                                                  ReadsArgs R, const uint8_t *__restrict__ flags,
                                                  uint64_t n_tiles,
                                                  const uint64_t *__restrict__ off_d,
                                                  const uint64_t *__restrict__ off_t) {
    static_assert(kTile == 64 * 16, "16 flag bytes per lane and tile");
    __shared__ uint16_t s_pos[kWG / 64][kTile];
    __shared__ uint16_t s_tb[kWG / 64][kTile];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * (kWG / 64);
    const uint4 *f128 = reinterpret_cast<const uint4 *>(flags);
    uint16_t *lpos = s_pos[wave];
    uint16_t *ltb = s_tb[wave];
    for (uint64_t tile = (uint64_t)blockIdx.x * (kWG / 64) + wave; tile < n_tiles;
         tile += n_waves) {
        const uint32_t sidx = tile_set[tile];
        if (sidx == kNoSet)
            continue;
        const uint4 x4 = f128[tile * 64 + lane];
        const uint32_t x[4] = {x4.x, x4.y, x4.z, x4.w};
        uint32_t cd = 0, ct = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            cd += (uint32_t)__popc(x[u] & 0x01010101u);
            ct += (uint32_t)__popc(x[u] & 0x02020202u);
        }
        uint32_t tot_d, tot_t;
        uint32_t rd = wave_exclusive(cd, lane, tot_d);
        uint32_t rt = wave_exclusive(ct, lane, tot_t);
        if (tot_d == 0)
            continue;
        list_flags(x, lane, rd, rt, lpos, ltb);
        __builtin_amdgcn_wave_barrier();
        const SetDesc &S = sets[sidx];
        const uint64_t first_tile = S.base / kTile;
        const uint64_t pos0 = tile * kTile;
        // this set's distinct / trustworthy keys before the tile
        const uint64_t dd = off_d[tile] - off_d[first_tile];
        const uint64_t tt = off_t[tile] - off_t[first_tile];
        const uint64_t od = *S.n_distinct + dd;
        for (uint32_t i = lane; i < tot_d; i += 64) {
            const uint64_t p = pos0 + lpos[i];
            const uint64_t key = canonical_fast(window_key(R.codes, p, S.k), S.k).key;
            const uint64_t d = od + i;
            if (d < S.cap_d)
                S.distinct[d] = key;
            if (S.fused) {
                const uint32_t tb = ltb[i];
                const uint64_t ti = tt + (tb & 0x7FFFu);
                if (tb & 0x8000u) {
                    if (ti < S.cap_te)
                        S.trust[ti] = key;
                } else {
                    const uint64_t ei = dd + i - ti;
                    if (ei < S.cap_te)
                        S.err[ei] = key;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();  // the list is rewritten by the next tile
    }
}

__global__ void kb_save_bases(const SetDesc *__restrict__ sets, uint32_t n_sets,
                              uint64_t *__restrict__ saved) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_sets)
        saved[s] = *sets[s].n_distinct;
}

hipError_t launch_save_bases(const BatchBuffers &Bf, uint32_t n_sets, hipStream_t s) {
    hipLaunchKernelGGL(kb_save_bases, dim3((n_sets + 63) / 64), dim3(64), 0, s, Bf.sets, n_sets,
                       Bf.saved);
    return hipGetLastError();
}

// Per set: advance the counters, write the split counts, flag overflows.
__global__ void kb_finish(const SetDesc *__restrict__ sets, uint32_t n_sets,
                          const uint64_t *__restrict__ off_d, const uint64_t *__restrict__ off_t,
                          const uint64_t *__restrict__ totals, uint64_t n_tiles,
                          const unsigned long long *__restrict__ valid) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets)
        return;
    const SetDesc &S = sets[s];
    const uint64_t t0 = S.base / kTile;
    const uint64_t t1 = (S.base + S.n_bases + kTile - 1) / kTile;
    const uint64_t d = (t1 < n_tiles ? off_d[t1] : totals[0]) - off_d[t0];
    const uint64_t t = (t1 < n_tiles ? off_t[t1] : totals[1]) - off_t[t0];
    const uint64_t nd = *S.n_distinct + d;
    *S.n_distinct = nd;
    if (S.n_windows)
        *S.n_windows += valid[s];
    bool over = nd > S.cap_d;
    if (S.fused) {
        *S.n_trust = t;
        *S.n_err = d - t;
        over = over || t > S.cap_te || d - t > S.cap_te;
    }
    if (over)
        atomicOr(S.status, kStatusRange);
}

// ---------------------------------------------------------------------------
// launch sequence
// ---------------------------------------------------------------------------
hipError_t launch_batch_bins(const BatchPlan &bp, const BatchBuffers &Bf, const ReadsArgs &R,
                             hipStream_t s, Profiler *P) {
    if (!R.valid || (bp.tile & 63u))
        return hipErrorInvalidValue;  // items must start at multiples of 64 positions
    if (P)
        P->begin(kPhValid, s);
    hipLaunchKernelGGL(kb_valid, dim3(bp.n_items), dim3(256), 0, s, Bf.sets, Bf.item_set, R,
                       bp.tile, mask_words(R.n_bases), (uint32_t *)R.valid);
    if (P)
        P->end(s);
    const hipError_t ev = hipGetLastError();
    if (ev != hipSuccess)
        return ev;
    if (P)
        P->begin(kPhBinCount, s);
    hipLaunchKernelGGL((bp.fast ? kb_bin_count<true> : kb_bin_count<false>), dim3(bp.n_items),
                       dim3(kBinWG), 0, s, Bf.sets, Bf.item_set, R, bp.tile, Bf.slots,
                       Bf.matrix_t, Bf.valid);
    if (P)
        P->end(s);
    hipError_t e = hipGetLastError();
    if (P)
        P->begin(kPhScan, s);
    if (e == hipSuccess && bp.n_sets) {
        const uint32_t gx = (bp.max_regions + 63) / 64, gy = (bp.max_G + 63) / 64;
        if (gy > 65535 || bp.n_sets > 65535) {
            e = hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL(kb_transpose, dim3(gx, gy, bp.n_sets), dim3(256), 0, s, Bf.sets,
                               (const uint32_t *)Bf.matrix_t, Bf.matrix);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess)
        e = scan_u32_u32(Bf.matrix, Bf.matrix, bp.n_matrix, Bf.n_entries, Bf.partial32, s);
    if (P)
        P->end(s);
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhBinBucket, s);
    hipLaunchKernelGGL(kb_bin_write, dim3(bp.n_items), dim3(kBinWG), 0, s, Bf.sets, Bf.item_set,
                       bp.tile, (const uint32_t *)Bf.slots, (const uint32_t *)Bf.matrix,
                       Bf.entries, bp.entries_cap);
    if (P)
        P->end(s);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchPlan &bp, const BatchBuffers &Bf, const ReadsArgs &R,
                        bool reset, hipStream_t s, Profiler *P) {
    hipError_t e = hipSuccess;
    if (reset) {
        if (P)
            P->begin(kPhReset, s);
        hipLaunchKernelGGL(kb_reset, dim3(64, bp.n_sets), dim3(256), 0, s, Bf.sets, bp.n_sets);
        if (P)
            P->end(s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kb_zero_valid, dim3(1), dim3(256), 0, s, Bf.valid, bp.n_sets);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = launch_batch_bins(bp, Bf, R, s, P);
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhRegion, s);
    hipLaunchKernelGGL(kb_region, dim3(bp.n_regions), dim3(kRegionWG), 0, s, Bf.sets, bp.n_sets,
                       Bf.region_set, (const uint32_t *)Bf.matrix, (const uint32_t *)Bf.n_entries,
                       (const uint64_t *)Bf.entries, bp.entries_cap, Bf.W->flags8);
    if (P)
        P->end(s);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    const Workspace &W = *Bf.W;
    const dim3 grid((unsigned)(bp.n_tiles < (uint64_t)kTileGrid ? bp.n_tiles : kTileGrid));
    if (P)
        P->begin(kPhTileCount, s);
    e = launch_tile_count(R, W, bp.n_tiles, s);
    if (P)
        P->end(s);
    if (P)
        P->begin(kPhScan, s);
    if (e == hipSuccess)
        e = scan_u32_u64(W.tile_a, W.off_a, bp.n_tiles, nullptr, W.totals + 0, W.partial64, s);
    if (e == hipSuccess)
        e = scan_u32_u64(W.tile_b, W.off_b, bp.n_tiles, nullptr, W.totals + 1, W.partial64, s);
    if (P)
        P->end(s);
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhScatter, s);
    hipLaunchKernelGGL(kb_compact, grid, dim3(kWG), 0, s, Bf.sets, Bf.tile_set, R,
                       (const uint8_t *)W.flags8, bp.n_tiles, (const uint64_t *)W.off_a,
                       (const uint64_t *)W.off_b);
    if (P)
        P->end(s);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = launch_save_bases(Bf, bp.n_sets, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(kb_finish, dim3((bp.n_sets + 63) / 64), dim3(64), 0, s, Bf.sets, bp.n_sets,
                       (const uint64_t *)W.off_a, (const uint64_t *)W.off_b,
                       (const uint64_t *)W.totals, bp.n_tiles,
                       (const unsigned long long *)Bf.valid);
    return hipGetLastError();
}

}  // namespace kc
