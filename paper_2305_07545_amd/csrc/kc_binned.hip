// Binned insertion: the countBF update and the first-seen resolution done in
// LDS, one workgroup per filter region, with no global atomics on counters.
//
// A filter region is 2^shift consecutive cells whose eta*2^shift counters fit
// the LDS arrays; a bucket is 2^bshift consecutive regions (at most 64
// buckets).  For one chunk of positions [c0, c1) (t = p - c0):
//   bin_count   hash every valid window once; store its slot id
//               (region << 14 | local counter) per (position, hash function);
//               per-workgroup LDS histograms of regions and of buckets
//   (scans)     region-major scan of the region counts -> the offset of every
//               (region, bin workgroup) segment of the final entry list;
//               bucket-major scan of the bucket counts -> the same for the
//               intermediate bucket list
//   bin_bucket  read the slot ids; batches are counting-sorted by bucket in
//               LDS and written as contiguous runs: entry = t << 32 | slot id
//   bin_region  one workgroup per (bucket, slice of bin workgroups): move the
//               slice's entries to their regions' segments
//   region      each region by one workgroup of a persistent grid: in LDS, hits[c] += 1 and
//               first[c] = min(first[c], t) over the region's entries; then
//               counter = min(2^alpha - 1, old + hits) per counter, and the
//               occurrence first[c] is distinct when the counter was zero
//               before the chunk (the sequential Query-I result)
// Entry order inside a segment never matters: sums and minima are order-
// independent, so the outputs are deterministic.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "kc_bin_hash.hpp"
#include "kc_device.hpp"
#include "kc_kernels.hpp"

namespace kc {

namespace {

// coarse[b * G + g] = sum of the region counts s_hist[r] over the regions r
// of bucket b (after the histogram is complete in LDS), for n_regions
// regions in buckets of 2^bshift, for every one of the n_rows buckets
// (buckets past the last region get 0: every row of a scanned matrix must be
// written).  kBinWG threads: 8 per bucket, each summing every 8th region,
// then a shuffle reduction.
__device__ __forceinline__ void write_bucket_sums(const uint32_t *s_hist, uint32_t n_regions,
                                                  uint32_t n_rows, uint32_t bshift, uint64_t G,
                                                  uint32_t *__restrict__ coarse, uint32_t g) {
    static_assert(kBinWG == 8 * kMaxBuckets, "8 threads per bucket");
    const uint32_t n_buckets = n_rows;
    const uint32_t b = threadIdx.x >> 3, sub = threadIdx.x & 7u;
    uint32_t sum = 0;
    if (b < n_buckets) {
        const uint32_t r0 = b << bshift;
        const uint32_t r1 = r0 + (1u << bshift) < n_regions ? r0 + (1u << bshift) : n_regions;
        for (uint32_t r = r0 + sub; r < r1; r += 8)  // empty when r0 >= n_regions
            sum += s_hist[r];
    }
    sum += __shfl_xor(sum, 1, 64);
    sum += __shfl_xor(sum, 2, 64);
    sum += __shfl_xor(sum, 4, 64);
    if (b < n_buckets && sub == 0)
        coarse[(uint64_t)b * G + g] = sum;
}

// Entries of the single-level binned path take 6 bytes, a 32-bit word and a
// 16-bit half held in two arrays (the words, then the halves, in the space
// of the 8-byte entries):
//   level 1 (bucket lists): word = id within the bucket (region within the
//     bucket << kLocalBits | counter) | low bits of ts << 22, half = the
//     high bits, where ts = t - start of the slice of bin workgroups that
//     level 2 reads the entry in (the workgroup's rank in the slice x tile
//     + t - tile start);
//   level 2 (region lists): word = counter | low bits of t << kLocalBits,
//     half = the high bits (t chunk-relative).
constexpr uint32_t kBucketIdBits = 22;
constexpr uint32_t kMaxSliceLog = (32 - kBucketIdBits) + 16;  // ts: 26 bits
static_assert((1u << (kBucketIdBits - kLocalBits)) == kMaxRegionsPerBucket, "bucket ids");
static_assert((32 - kLocalBits) + 16 >= 32, "level-2 entries hold any 32-bit t");

// An entry as loaded, either format (hi = ~0u: no entry)
struct RawEntry {
    uint32_t lo, hi;
};

// Element at a 32-bit byte offset from a wavefront-uniform base: the address
// is the base's scalar registers plus one 32-bit vector register, not a
// 64-bit address per thread.
template <typename T>
__device__ __forceinline__ T &at_byte(T *base, uint32_t byte_off) {
    return *(T *)((char *)base + byte_off);
}
static_assert(kStage == (1 << kStageLog), "stage size");
static_assert(kRegionCounters == (1 << kLocalBits), "region size");
static_assert(kMaxRegions == (1u << kPartLog), "partition size");
static_assert(kMaxParts <= 256, "partition ids are bytes");

}  // namespace

// kParts: the partitioned path; the slot id holds the region within its
// partition, parts[] the partition, and the histogram counts partitions.
// kFast: the fast layout (fast_layout); kWide: k-mers of 33..64 bases.
// Every valid window of the workgroup's tile is hashed once (walk_windows);
// slot ids are stored per (hash function, chunk-relative position), kNoSlot
// for invalid windows.
template <bool kParts, bool kFast, bool kWide>
__global__ void __launch_bounds__(kBinWG) k_bin_count(FilterArgs F, ReadsArgs R, uint64_t c0,
                                                      uint64_t c1, BinPlan B,
                                                      uint32_t *__restrict__ slots,
                                                      uint8_t *__restrict__ parts,
                                                      uint32_t *__restrict__ fine,
                                                      uint32_t *__restrict__ coarse,
                                                      unsigned long long *__restrict__ n_valid) {
    extern __shared__ uint32_t s_hist[];  // n_regions region (n_parts partition) counts
    __shared__ uint32_t s_ring[kBinWG / 64][kWindowRing];
    __shared__ uint32_t s_valid;
    const uint32_t n_keys = kParts ? B.n_parts : B.n_regions;
    for (uint32_t i = threadIdx.x; i < n_keys; i += kBinWG)
        s_hist[i] = 0;
    if (threadIdx.x == 0)
        s_valid = 0;
    __syncthreads();
    const uint64_t len = c1 - c0;
    const uint64_t g0 = c0 + (uint64_t)blockIdx.x * B.tile;
    const uint64_t g1 = g0 + B.tile < c1 ? g0 + B.tile : c1;
    // chunk-relative 32-bit positions (a chunk is < 2^32 positions; c0 is a
    // multiple of 64, so the chunk's code words start at c0 / 16)
    const uint32_t *__restrict__ codes = R.codes + (c0 >> 4);
    const uint32_t K = R.k, shift = B.region_shift, k_h = kFast ? 1u : F.k_h;
    const uint32_t nv = walk_windows(
        R, g0, g1, c0, s_ring[wave_id()],
        [&](uint32_t q) {
            for (uint32_t a = 0; a < k_h; a++)
                slots[(uint64_t)a * len + q] = kNoSlot;
        },
        [&](uint32_t q) {
            window_counters<kFast, kWide>(F, codes, q, K, shift, [&](uint32_t a, uint32_t r,
                                                                       uint32_t local) {
                const uint64_t at = (uint64_t)(a - 1) * len + q;
                if (kParts) {
                    slots[at] = ((r & ((1u << B.part_log) - 1u)) << kLocalBits) | local;
                    parts[at] = (uint8_t)(r >> B.part_log);
                    atomicAdd(&s_hist[r >> B.part_log], 1u);
                } else {
                    slots[at] = (r << kLocalBits) | local;
                    atomicAdd(&s_hist[r], 1u);
                }
            });
        });
    if ((threadIdx.x & 63u) == 0)
        atomicAdd(&s_valid, nv);
    __syncthreads();
    // binned path: the workgroup's region counts as one contiguous row
    // (transposed to region-major afterwards); partitioned path: partition
    // counts, few per workgroup, written partition-major directly
    for (uint32_t i = threadIdx.x; i < n_keys; i += kBinWG)
        fine[kParts ? (uint64_t)i * B.G + blockIdx.x : (uint64_t)blockIdx.x * n_keys + i] =
            s_hist[i];
    if (!kParts)
        write_bucket_sums(s_hist, B.n_regions, B.n_buckets, B.bucket_shift, B.G, coarse,
                          blockIdx.x);
    if (threadIdx.x == 0)
        atomicAdd(n_valid, (unsigned long long)s_valid);
}

// Level 1: slot ids of this workgroup's positions -> runs of the bucket list.
// A batch holds kStage1 entries: the thread's kPer entries stay in registers
// between counting, staging and writing.  The pass runs one workgroup per
// CU (the launch reserves kLevel1Reserve bytes of LDS beside the 64 KiB
// batch): with fewer workgroups writing runs at once it moved the bacterial
// step's 1.6 GB in 0.376 ms, against 0.388 ms at two per CU and 0.430 ms at
// three (4096-entry batches).
constexpr int kStage1 = 8192;
constexpr uint32_t kStage1Log = 13;
constexpr size_t kLevel1Reserve = 20u << 10;
static_assert(kStage1 == (1 << kStage1Log), "level-1 batch size");
static_assert(kStage1 * sizeof(uint64_t) + kLevel1Reserve > (160u << 10) / 2,
              "one level-1 workgroup per CU (160 KiB of LDS)");
static_assert(kStage1 * sizeof(uint64_t) + kLevel1Reserve + 1024 <= (160u << 10),
              "the level-1 workgroup fits the LDS");
__global__ void __launch_bounds__(kBinWG) k_bin_bucket(uint64_t c0, uint64_t c1, uint32_t k_h,
                                                       BinPlan B,
                                                       const uint32_t *__restrict__ slots,
                                                       const uint32_t *__restrict__ coarse_off,
                                                       uint32_t *__restrict__ out_word,
                                                       uint16_t *__restrict__ out_half) {
    // 32-bit indices: a chunk of this path holds at most kBinChunk positions
    // and (positions x hash functions) < 2^32 slot ids and entries
    constexpr int kPer = kStage1 / kBinWG;
    __shared__ uint64_t s_stage[kStage1];
    __shared__ uint32_t s_cnt[kMaxBuckets];
    __shared__ uint32_t s_start[kMaxBuckets];
    __shared__ uint32_t s_cursor[kMaxBuckets];
    const uint32_t bshift = B.bucket_shift + kLocalBits;
    const uint32_t len = (uint32_t)(c1 - c0);
    const uint32_t g0 = blockIdx.x * (uint32_t)B.tile;  // chunk-relative
    const uint32_t g1 = g0 + (uint32_t)B.tile < len ? g0 + (uint32_t)B.tile : len;
    const uint32_t s0 = (blockIdx.x & ~(B.slice - 1u)) * (uint32_t)B.tile;  // its slice's start
    // positions per batch: a power of two with batch * k_h <= kStage1
    uint32_t bl = 0;
    while ((1u << bl) < k_h)
        bl++;
    const uint32_t batch_log = kStage1Log - bl;
    const uint32_t batch = 1u << batch_log;
    const uint32_t cap = B.entries_cap < 0xFFFFFFFFull ? (uint32_t)B.entries_cap : 0xFFFFFFFFu;
    for (uint32_t i = threadIdx.x; i < kMaxBuckets; i += kBinWG) {
        s_cursor[i] = i < B.n_buckets ? coarse_off[(uint64_t)i * B.G + blockIdx.x] : 0u;
        s_cnt[i] = 0;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    // the slot ids of the batch at q0 (entry i: hash function i / batch,
    // position i % batch); the next batch's are requested before this one
    // is sorted, so that their latency overlaps the LDS work
    // A full batch of one hash function is loaded 16 bytes per lane (a
    // thread's entries 4v .. 4v + 3 are consecutive positions); other batches
    // one slot id per lane.  pos_of: the batch index of a thread's entry u.
    auto full = [&](uint32_t q0) { return k_h == 1u && q0 + batch <= g1; };
    auto pos_of = [&](bool vec, int u) -> uint32_t {
        return vec ? (uint32_t)(u >> 2) * (4u * kBinWG) + 4u * threadIdx.x + (uint32_t)(u & 3)
                   : threadIdx.x + (uint32_t)u * kBinWG;
    };
    static_assert(kPer % 4 == 0, "whole 16-byte loads per thread");
    auto load = [&](uint32_t q0, uint32_t(&id)[kPer]) {
        if (full(q0)) {
            const uint4 *p4 = reinterpret_cast<const uint4 *>(slots + q0);  // q0 % 4 == 0
#pragma unroll
            for (int v = 0; v < kPer / 4; v++) {
                const uint4 x = p4[(uint32_t)v * kBinWG + threadIdx.x];
                id[4 * v] = x.x;
                id[4 * v + 1] = x.y;
                id[4 * v + 2] = x.z;
                id[4 * v + 3] = x.w;
            }
            return;
        }
        const uint32_t nq = (q0 + batch < g1 ? q0 + batch : g1) - q0;
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const uint32_t i = threadIdx.x + (uint32_t)u * kBinWG;
            const uint32_t a = i >> batch_log;
            const uint32_t dq = i & (batch - 1u);
            id[u] = (a < k_h && dq < nq) ? slots[a * len + q0 + dq] : kNoSlot;
        }
    };
    uint32_t next[kPer];
    if (g0 < g1)
        load(g0, next);
    for (uint32_t q0 = g0; q0 < g1; q0 += batch) {
        const bool vec = full(q0);
        uint32_t id[kPer];
#pragma unroll
        for (int u = 0; u < kPer; u++)
            id[u] = next[u];
        if (q0 + batch < g1)
            load(q0 + batch, next);
        uint32_t rk[kPer];  // entry u's rank among its destination's in the batch
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (id[u] != kNoSlot)
                rk[u] = atomicAdd(&s_cnt[id[u] >> bshift], 1u);
        __syncthreads();
        if (threadIdx.x < 64) {  // one wavefront scans the 64 bucket counts
            uint32_t v = s_cnt[lane];
            uint32_t incl = v;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d)
                    incl += o;
            }
            s_start[lane] = incl - v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (id[u] != kNoSlot) {
                const uint32_t i = pos_of(vec, u);
                const uint32_t q = q0 - s0 + (i & (batch - 1u));  // ts: within the slice
                const uint32_t b = id[u] >> bshift;
                const uint32_t j = s_start[b] + rk[u];
                s_stage[j] = ((uint64_t)q << 32) | id[u];
            }
        __syncthreads();
        const uint32_t n_stage = s_start[kMaxBuckets - 1] + s_cnt[kMaxBuckets - 1];
        for (uint32_t j = threadIdx.x; j < n_stage; j += kBinWG) {
            const uint64_t e = s_stage[j];
            const uint32_t b = (uint32_t)e >> bshift;
            const uint32_t dst = s_cursor[b] + (j - s_start[b]);
            const uint32_t q = (uint32_t)(e >> 32);
            if (dst < cap) {
                out_word[dst] = ((uint32_t)e & ((1u << bshift) - 1u)) | (q << kBucketIdBits);
                out_half[dst] = (uint16_t)(q >> (32 - kBucketIdBits));
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kMaxBuckets; i += kBinWG) {
            s_cursor[i] += s_cnt[i];
            s_cnt[i] = 0;
        }
        __syncthreads();
    }
}

// Level 2: the entries of bucket b written by bin workgroups [s*slice,
// (s+1)*slice) -> their regions' segments for those workgroups.  Batches of
// kStage2 entries are counting-sorted by region in LDS and written as runs
// (twice the level-1 batch: runs of 2 x 4096 / regions per bucket entries).
// kCompact: 6-byte entries in (single-level path), else 8-byte entries
// (t << 32 | slot id: the partitioned path's list binning); the region
// lists are written as 6-byte entries either way.
// kThreads: the workgroup (16 entries per thread and batch): 512 threads,
// batches of 8192 entries, two workgroups per CU; or 1024 threads, batches of
// 16384 (runs twice as long per region), one per CU.
template <bool kCompact, int kThreads>
__global__ void __launch_bounds__(kThreads) k_bin_region(BinPlan B,
                                                       const uint32_t *__restrict__ coarse_off,
                                                       const uint32_t *__restrict__ n_entries,
                                                       const uint32_t *__restrict__ fine_off,
                                                       const uint64_t *__restrict__ bucketed,
                                                       uint64_t *__restrict__ entries) {
    constexpr int kStage2 = 16 * kThreads;
    constexpr int kPer = kStage2 / kThreads;
    __shared__ uint64_t s_stage[kStage2];
    __shared__ uint32_t s_cursor[kMaxRegionsPerBucket];
    __shared__ uint32_t s_cnt[kMaxRegionsPerBucket];
    __shared__ uint32_t s_start[kMaxRegionsPerBucket];
    __shared__ uint32_t s_fill[kMaxRegionsPerBucket];
    __shared__ uint32_t s_delta[kMaxRegionsPerBucket];  // output index - staged index, per region
    __shared__ uint32_t s_wave[kThreads / 64];
    const uint32_t b = blockIdx.x / B.n_slices;
    const uint32_t s = blockIdx.x % B.n_slices;
    const uint32_t gs0 = s * B.slice;
    if (gs0 >= B.G)
        return;
    const uint32_t gs1 = gs0 + B.slice < B.G ? gs0 + B.slice : B.G;
    const uint32_t r0 = b << B.bucket_shift;
    const uint32_t nr = (r0 + (1u << B.bucket_shift) <= B.n_regions) ? (1u << B.bucket_shift)
                                                                      : B.n_regions - r0;
    // slot ids name the region within its partition (buckets never straddle
    // partitions)
    const uint32_t r0l = B.n_parts ? (r0 & ((1u << B.part_log) - 1u)) : r0;
    for (uint32_t i = threadIdx.x; i < kMaxRegionsPerBucket; i += kThreads) {
        s_cursor[i] = i < nr ? fine_off[(uint64_t)(r0 + i) * B.G + gs0] : 0u;
        s_cnt[i] = 0;
        s_fill[i] = 0;
    }
    __syncthreads();
    // entry indices are 32-bit: a chunk's entries (positions x hash
    // functions) number less than 2^32 on both paths
    const uint32_t e0 = coarse_off[(uint64_t)b * B.G + gs0];
    uint32_t e1;
    if (gs1 < B.G)
        e1 = coarse_off[(uint64_t)b * B.G + gs1];
    else
        e1 = b + 1 < B.n_buckets ? coarse_off[(uint64_t)(b + 1) * B.G] : *n_entries;
    const uint64_t cap = B.entries_cap;
    const uint32_t cap32 = cap < 0xFFFFFFFFull ? (uint32_t)cap : 0xFFFFFFFFu;
    if (e1 > cap32)
        e1 = cap32;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t *in_word = (const uint32_t *)bucketed;
    const uint16_t *in_half = (const uint16_t *)(in_word + cap);
    uint32_t *out_word = (uint32_t *)entries;
    uint16_t *out_half = (uint16_t *)(out_word + cap);
    const uint32_t slice0 = gs0 * (uint32_t)B.tile;  // chunk-relative start of the slice
    // entries of the batch at q0 as loaded (lo, hi: the 8-byte entry's
    // words, or the 6-byte entry's word and half; hi = ~0u past the end);
    // the next batch's are requested before this one is sorted and decoded
    // only then, so that their loads stay in flight meanwhile
    auto load = [&](uint32_t q0, RawEntry(&v)[kPer]) {
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const uint32_t x = q0 + threadIdx.x + (uint32_t)u * kThreads;
            v[u] = RawEntry{~0u, ~0u};
            if (x < e1) {
                if (kCompact) {
                    v[u].lo = in_word[x];
                    v[u].hi = in_half[x];
                } else {
                    const uint2 p = ((const uint2 *)bucketed)[x];
                    v[u].lo = p.x;
                    v[u].hi = p.y;
                }
            }
        }
    };
    RawEntry next[kPer];
    if (e0 < e1)
        load(e0, next);
    for (uint32_t q0 = e0; q0 < e1; q0 += kStage2) {
        uint64_t v[kPer];
        uint32_t ri[kPer];
        RawEntry raw[kPer];
#pragma unroll
        for (int u = 0; u < kPer; u++)
            raw[u] = next[u];
        if (e1 - q0 > (uint32_t)kStage2)
            load(q0 + kStage2, next);
        // kCompact: t << 32 | region within the bucket << kLocalBits | counter
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            if (raw[u].hi == ~0u)
                v[u] = ~0ull;
            else if (kCompact)
                v[u] = ((uint64_t)(slice0 + ((raw[u].lo >> kBucketIdBits) |
                                             (raw[u].hi << (32 - kBucketIdBits))))
                        << 32) |
                       (raw[u].lo & ((1u << kBucketIdBits) - 1u));
            else
                v[u] = ((uint64_t)raw[u].hi << 32) | raw[u].lo;
        }
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            if (kCompact) {
                const uint32_t r = (uint32_t)v[u] >> kLocalBits;
                ri[u] = (v[u] != ~0ull && r < nr) ? r : 0xFFFFFFFFu;
            } else {
                const uint32_t r = ((uint32_t)v[u] >> kLocalBits) & ((1u << kLocalBits) - 1u);
                ri[u] = (v[u] != ~0ull && r - r0l < nr) ? r - r0l : 0xFFFFFFFFu;
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (ri[u] != 0xFFFFFFFFu)
                atomicAdd(&s_cnt[ri[u]], 1u);
        __syncthreads();
        // exclusive scan of the region counts (kMaxRegionsPerBucket <= kThreads)
        {
            const uint32_t c = threadIdx.x < kMaxRegionsPerBucket ? s_cnt[threadIdx.x] : 0u;
            uint32_t incl = c;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d)
                    incl += o;
            }
            if (lane == 63)
                s_wave[wave] = incl;
            __syncthreads();
            uint32_t before = 0;
            for (uint32_t w = 0; w < wave; w++)
                before += s_wave[w];
            if (threadIdx.x < kMaxRegionsPerBucket) {
                s_start[threadIdx.x] = before + incl - c;
                s_delta[threadIdx.x] = s_cursor[threadIdx.x] - (before + incl - c);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (ri[u] != 0xFFFFFFFFu) {
                const uint32_t j = s_start[ri[u]] + atomicAdd(&s_fill[ri[u]], 1u);
                s_stage[j] = v[u];
            }
        __syncthreads();
        const uint32_t n_stage =
            s_start[kMaxRegionsPerBucket - 1] + s_cnt[kMaxRegionsPerBucket - 1];
        for (uint32_t j = threadIdx.x; j < n_stage; j += kThreads) {
            const uint64_t e = s_stage[j];
            const uint32_t r = kCompact
                                   ? (uint32_t)e >> kLocalBits
                                   : (((uint32_t)e >> kLocalBits) & ((1u << kLocalBits) - 1u)) - r0l;
            const uint32_t dst = s_delta[r] + j;
            const uint32_t t = (uint32_t)(e >> 32);  // chunk-relative: < 2^32 - 1
            if (dst < cap32) {
                out_word[dst] = ((uint32_t)e & (kRegionCounters - 1u)) | (t << kLocalBits);
                out_half[dst] = (uint16_t)(t >> (32 - kLocalBits));
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kMaxRegionsPerBucket; i += kThreads) {
            s_cursor[i] += s_cnt[i];
            s_cnt[i] = 0;
            s_fill[i] = 0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// partitioned path: countBFs of more than kMaxRegions regions
// ---------------------------------------------------------------------------

// bounds[p] = start of partition p in the partition list (the scanned
// partition-major matrix), bounds[n_parts] = total
__global__ void k_part_bounds(const uint32_t *__restrict__ pmat, uint32_t G, uint32_t n_parts,
                              const uint32_t *__restrict__ total, uint32_t *__restrict__ bounds) {
    for (uint32_t p = threadIdx.x; p <= n_parts; p += blockDim.x)
        bounds[p] = p < n_parts ? pmat[(uint64_t)p * G] : *total;
}

// Slot ids of this workgroup's positions -> runs of the partition list
// (entry = t << 32 | slot id), counting-sorted by partition in LDS batches of
// kStage entries like the level-1 pass.  The next batch's slot ids and
// partition bytes are requested before the current one is sorted; a full
// batch of one hash function is loaded 16 bytes of slot ids and 4 partition
// bytes per lane (a thread's entries 4v .. 4v + 3 are consecutive positions).
template <int kThreads>
__global__ void __launch_bounds__(kThreads) k_part_scatter(uint64_t c0, uint64_t c1, uint32_t k_h,
                                                         BinPlan B,
                                                         const uint32_t *__restrict__ slots,
                                                         const uint8_t *__restrict__ parts,
                                                         const uint32_t *__restrict__ pmat_off,
                                                         uint64_t *__restrict__ plist) {
    constexpr int kBatch = 8 * kThreads;
    constexpr int kPer = kBatch / kThreads;
    static_assert(kPer % 4 == 0, "whole 16-byte loads per thread");
    __shared__ uint64_t s_stage[kBatch];
    __shared__ uint8_t s_tag[kBatch];  // partition of each staged entry
    __shared__ uint32_t s_cnt[kMaxParts];
    __shared__ uint32_t s_start[kMaxParts];
    __shared__ uint32_t s_fill[kMaxParts];
    __shared__ uint32_t s_cursor[kMaxParts];
    __shared__ uint32_t s_wave[kThreads / 64];
    static_assert(kMaxParts <= kThreads, "one thread per partition count");
    const uint64_t len = c1 - c0;
    const uint64_t g0 = (uint64_t)blockIdx.x * B.tile;
    const uint64_t g1 = g0 + B.tile < len ? g0 + B.tile : len;
    uint32_t bl = 0;
    while ((1u << bl) < k_h)
        bl++;
    const uint32_t batch_log = (kThreads == 1024 ? 13u : kStageLog) - bl;
    const uint64_t batch = 1ull << batch_log;
    const uint64_t cap = B.entries_cap;
    for (uint32_t i = threadIdx.x; i < kMaxParts; i += kThreads) {
        s_cursor[i] = i < B.n_parts ? pmat_off[(uint64_t)i * B.G + blockIdx.x] : 0u;
        s_cnt[i] = 0;
        s_fill[i] = 0;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    // tiles and batches start at multiples of 4 positions, the slot and
    // partition arrays at 16- and 4-byte boundaries
    auto full = [&](uint64_t q0) { return k_h == 1u && q0 + batch <= g1; };
    // the batch offset of a thread's entry u
    auto pos_of = [&](bool vec, int u) -> uint64_t {
        return vec ? (uint64_t)(u >> 2) * (4u * kThreads) + 4u * threadIdx.x + (uint32_t)(u & 3)
                   : (((uint64_t)threadIdx.x + (uint64_t)u * kThreads) & (batch - 1));
    };
    auto load = [&](uint64_t q0, uint32_t(&id)[kPer], uint32_t(&pt)[kPer]) {
        if (full(q0)) {
            const uint4 *s4 = reinterpret_cast<const uint4 *>(slots + q0);
            const uint32_t *p4 = reinterpret_cast<const uint32_t *>(parts + q0);
#pragma unroll
            for (int v = 0; v < kPer / 4; v++) {
                const uint32_t at = (uint32_t)v * kThreads + threadIdx.x;
                const uint4 x = s4[at];
                const uint32_t pp = p4[at];
                id[4 * v] = x.x;
                id[4 * v + 1] = x.y;
                id[4 * v + 2] = x.z;
                id[4 * v + 3] = x.w;
#pragma unroll
                for (int j = 0; j < 4; j++)
                    pt[4 * v + j] = (pp >> (8 * j)) & 0xFFu;
            }
            return;
        }
        const uint64_t nq = (q0 + batch < g1 ? q0 + batch : g1) - q0;
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const uint64_t i = (uint64_t)threadIdx.x + (uint64_t)u * kThreads;
            const uint64_t a = i >> batch_log;
            const uint64_t q = q0 + (i & (batch - 1));
            const bool ok = a < k_h && q - q0 < nq;
            id[u] = ok ? slots[a * len + q] : kNoSlot;
            pt[u] = (id[u] != kNoSlot) ? (uint32_t)parts[a * len + q] : 0u;
        }
    };
    uint32_t nid[kPer], npt[kPer];
    if (g0 < g1)
        load(g0, nid, npt);
    for (uint64_t q0 = g0; q0 < g1; q0 += batch) {
        const bool vec = full(q0);
        uint32_t id[kPer], pt[kPer];
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            id[u] = nid[u];
            pt[u] = npt[u];
        }
        if (q0 + batch < g1)
            load(q0 + batch, nid, npt);
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (id[u] != kNoSlot)
                atomicAdd(&s_cnt[pt[u]], 1u);
        __syncthreads();
        {
            const uint32_t c = threadIdx.x < kMaxParts ? s_cnt[threadIdx.x] : 0u;
            uint32_t incl = c;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d)
                    incl += o;
            }
            if (lane == 63)
                s_wave[wave] = incl;
            __syncthreads();
            uint32_t before = 0;
            for (uint32_t w = 0; w < wave; w++)
                before += s_wave[w];
            if (threadIdx.x < kMaxParts)
                s_start[threadIdx.x] = before + incl - c;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (id[u] != kNoSlot) {
                const uint64_t q = q0 + pos_of(vec, u);
                const uint32_t j = s_start[pt[u]] + atomicAdd(&s_fill[pt[u]], 1u);
                s_stage[j] = (q << 32) | id[u];
                s_tag[j] = (uint8_t)pt[u];
            }
        __syncthreads();
        const uint32_t n_stage = s_start[kMaxParts - 1] + s_cnt[kMaxParts - 1];
        for (uint32_t j = threadIdx.x; j < n_stage; j += kThreads) {
            const uint32_t pj = s_tag[j];
            const uint64_t dst = (uint64_t)s_cursor[pj] + (j - s_start[pj]);
            if (dst < cap)
                plist[dst] = s_stage[j];
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kMaxParts; i += kThreads) {
            s_cursor[i] += s_cnt[i];
            s_cnt[i] = 0;
            s_fill[i] = 0;
        }
        __syncthreads();
    }
}

// The list slice of partition p handled by its list workgroup g: tiles of
// pdesc[p].tile entries from pdesc[p].lo (the tile size comes from the
// partition sizes on the device, so no host round trip is needed).
struct ListTile {
    uint64_t lo, n;  // first entry in the partition list, entries
};

__device__ __forceinline__ ListTile list_tile(const uint64_t *__restrict__ pdesc, uint32_t p,
                                              uint32_t g) {
    const uint64_t lo = pdesc[3 * p], n = pdesc[3 * p + 1], tile = pdesc[3 * p + 2];
    const uint64_t a = (uint64_t)g * tile;
    ListTile t;
    t.lo = lo + (a < n ? a : n);
    t.n = a < n ? (n - a < tile ? n - a : tile) : 0;
    return t;
}

// pdesc[p] = (start, entries, list tile) of each partition's list.
__global__ void k_pass_plan(const uint32_t *__restrict__ bounds, uint32_t n_parts, uint32_t list_g,
                            uint64_t cap, uint64_t *__restrict__ pdesc) {
    for (uint32_t p = threadIdx.x; p < n_parts; p += blockDim.x) {
        const uint64_t lo = bounds[p];
        uint64_t hi = bounds[p + 1];
        if (hi > cap)
            hi = cap;
        const uint64_t n = hi > lo ? hi - lo : 0;
        pdesc[3 * p] = lo;
        pdesc[3 * p + 1] = n;
        pdesc[3 * p + 2] = (n + list_g - 1) / list_g;
    }
}

// Region counts per list workgroup of every partition's list, one
// contiguous row per workgroup: fine_t[((p * list_g) + g) * 2^part_log + i]
// (transposed afterwards, partition by partition, to the region-major layout
// the single-level path uses), and the bucket sums into
// coarse[(p * buckets per partition + b) x list_g + g].
__global__ void __launch_bounds__(kBinWG) k_list_count(const uint64_t *__restrict__ plist,
                                                       const uint64_t *__restrict__ pdesc,
                                                       BinPlan B, uint32_t *__restrict__ fine,
                                                       uint32_t *__restrict__ coarse) {
    extern __shared__ uint32_t s_hist[];
    const uint32_t p = blockIdx.x / B.list_g, g = blockIdx.x % B.list_g;
    const uint32_t per = 1u << B.part_log;
    const uint32_t rp0 = p << B.part_log;
    const uint32_t nrp = B.n_regions - rp0 < per ? B.n_regions - rp0 : per;
    for (uint32_t i = threadIdx.x; i < nrp; i += kBinWG)
        s_hist[i] = 0;
    __syncthreads();
    const ListTile t = list_tile(pdesc, p, g);
    const uint64_t *__restrict__ list = plist + t.lo;
    constexpr int kUnroll = 8;
    for (uint64_t e = threadIdx.x; e < t.n; e += (uint64_t)kUnroll * kBinWG) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const uint64_t x = e + (uint64_t)u * kBinWG;
            v[u] = x < t.n ? (uint32_t)list[x] : kNoSlot;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++)
            if (v[u] != kNoSlot)
                atomicAdd(&s_hist[(v[u] >> kLocalBits) & (per - 1u)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nrp; i += kBinWG)
        fine[((uint64_t)p * B.list_g + g) * per + i] = s_hist[i];
    const uint32_t nbp = per >> B.bucket_shift;  // bucket rows per partition
    write_bucket_sums(s_hist, nrp, nbp, B.bucket_shift, B.list_g,
                      coarse + (uint64_t)p * nbp * B.list_g, g);
}

// Level 1 over every partition's list: the entries of list workgroup g of
// partition p -> runs of the partition's bucket segments.
template <int kThreads>
__global__ void __launch_bounds__(kThreads) k_bin_bucket_list(const uint64_t *__restrict__ plist,
                                                            const uint64_t *__restrict__ pdesc,
                                                            BinPlan B,
                                                            const uint32_t *__restrict__ coarse_off,
                                                            uint64_t *__restrict__ bucketed) {
    constexpr int kBatch = 8 * kThreads;
    constexpr int kPer = kBatch / kThreads;
    __shared__ uint64_t s_stage[kBatch];
    __shared__ uint32_t s_cnt[kMaxBuckets];
    __shared__ uint32_t s_start[kMaxBuckets];
    __shared__ uint32_t s_cursor[kMaxBuckets];
    const uint32_t p = blockIdx.x / B.list_g, g = blockIdx.x % B.list_g;
    const uint32_t per = 1u << B.part_log;
    const uint32_t nbp = per >> B.bucket_shift;
    const uint32_t bshift = B.bucket_shift + kLocalBits;
    const ListTile t = list_tile(pdesc, p, g);
    const uint64_t *__restrict__ list = plist + t.lo;
    const uint64_t cap = B.entries_cap;
    for (uint32_t i = threadIdx.x; i < kMaxBuckets; i += kThreads) {
        s_cursor[i] = i < nbp ? coarse_off[((uint64_t)p * nbp + i) * B.list_g + g] : 0u;
        s_cnt[i] = 0;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    // the next batch is requested before the current one is sorted
    auto load = [&](uint64_t q0, uint64_t(&v)[kPer]) {
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const uint64_t x = q0 + threadIdx.x + (uint64_t)u * kThreads;
            v[u] = x < t.n ? list[x] : ~0ull;
        }
    };
    uint64_t nv[kPer];
    if (t.n > 0)
        load(0, nv);
    for (uint64_t q0 = 0; q0 < t.n; q0 += kBatch) {
        uint64_t v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; u++)
            v[u] = nv[u];
        if (q0 + kBatch < t.n)
            load(q0 + kBatch, nv);
        uint32_t rk[kPer];  // entry u's rank among its destination's in the batch
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (v[u] != ~0ull)
                rk[u] = atomicAdd(&s_cnt[((uint32_t)v[u] >> bshift) & (kMaxBuckets - 1u)], 1u);
        __syncthreads();
        if (threadIdx.x < 64) {
            uint32_t c = s_cnt[lane];
            uint32_t incl = c;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d)
                    incl += o;
            }
            s_start[lane] = incl - c;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; u++)
            if (v[u] != ~0ull) {
                const uint32_t b = ((uint32_t)v[u] >> bshift) & (kMaxBuckets - 1u);
                const uint32_t j = s_start[b] + rk[u];
                s_stage[j] = v[u];
            }
        __syncthreads();
        const uint32_t n_stage = s_start[kMaxBuckets - 1] + s_cnt[kMaxBuckets - 1];
        for (uint32_t j = threadIdx.x; j < n_stage; j += kThreads) {
            const uint64_t e = s_stage[j];
            const uint32_t b = ((uint32_t)e >> bshift) & (kMaxBuckets - 1u);
            const uint64_t dst = (uint64_t)s_cursor[b] + (j - s_start[b]);
            if (dst < cap)
                bucketed[dst] = e;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kMaxBuckets; i += kThreads) {
            s_cursor[i] += s_cnt[i];
            s_cnt[i] = 0;
        }
        __syncthreads();
    }
}

// Where the region pass puts a first-seen occurrence (chunk-relative t and
// its mark: 1 distinct, 3 distinct and trustworthy): its flag byte, or, in
// records mode, a record in the region's own entry segment (whose entries
// the workgroup has read by then: every winner is one of them), which the
// winner passes below turn into flag bytes written in whole 16-byte groups.
struct WinnerSink {
    uint8_t *flags;
    uint64_t c0;
    uint32_t *rec_t;  // records or carry mode: the records' word array (null: flag mode)
    uint16_t *rec_m;  // ... and half array: the mark, or in carry mode the local counter
    uint64_t e0;      // the region's first record
    uint32_t *count;  // LDS: records written so far
    bool carry;       // carry mode: the half is the local counter id
};

__device__ __forceinline__ void put_winner(const WinnerSink &o, uint32_t t, uint32_t mark,
                                           uint32_t local) {
    if (!o.rec_t) {
        o.flags[o.c0 + t] = (uint8_t)mark;
        return;
    }
    const uint32_t i = atomicAdd(o.count, 1u);  // < the region's entries
    at_byte(o.rec_t + o.e0, 4u * i) = t;
    at_byte(o.rec_m + o.e0, 2u * i) = (uint16_t)(o.carry ? local : mark);
}

// Counter update of cell w of the region (pre = its value before the
// chunk); returns the cell's new value.  Leaves the cell's counters clean
// (hits 0, first kIdle) for the next region.
__device__ __forceinline__ uint64_t region_cell(const FilterArgs &F, const BinPlan &B,
                                                uint64_t wbase, uint32_t w, uint64_t pre,
                                                uint32_t *hits, uint32_t *first,
                                                const WinnerSink &out, int classify,
                                                uint32_t tau) {
    // counters are at most 32 bits wide: the field arithmetic is 32-bit
    const uint32_t fm = (uint32_t)F.field_max;
    uint64_t next = pre;
    for (uint32_t l = 0; l < F.eta; l++) {
        const uint32_t idx = (l << B.region_shift) | w;
        const uint32_t h = hits[idx];
        if (h == 0)
            continue;
        const uint32_t t = first[idx];
        hits[idx] = 0;
        first[idx] = kIdle;
        const uint32_t sh = F.alpha * l;
        const uint32_t pf = (uint32_t)(pre >> sh) & fm;
        const uint32_t room = fm - pf;
        const uint32_t nf = pf + (h < room ? h : room);
        next += (uint64_t)(nf - pf) << sh;  // the field grows without carrying out
        if (pf == 0)
            put_winner(out, t, (classify && nf > tau) ? 3u : 1u, idx);
    }
    if (next != pre)
        F.words[wbase + w] = next;
    return next;
}

// s_waitcnt vmcnt(0) in the gfx9 encoding, with expcnt and lgkmcnt left
// open: a wavefront's vector loads and stores all complete.
constexpr int kWaitVmem = 0x0F70;

// Region lists of 6-byte entries (both binned paths).  kCounters: the LDS
// arrays' size, the plan's counters per region (16384: 144 KiB of LDS, one
// workgroup per CU; 8192: 72 KiB, two per CU).  kHold: cells per thread held
// in registers; regions of up to kHold x kRegionWG cells take the held paths
// (the launcher picks the fewest that hold the plan's regions, which leaves
// registers for the prefetch).
//
// The grid is persistent: workgroup g takes regions g, g + gridDim.x, ....
// A workgroup that holds the CU's LDS alone has nobody else to hide its
// memory latency, so the next region's first batch of entries and cells
// (and first carried records) are requested before the current region is
// worked on, and the bounds that give their addresses one region earlier
// still.  A wavefront's loads and stores share one completion counter, and
// the wait for loads issued before a store must wait for the store too: the
// region's own stores (cell write-back, winner count) are therefore issued
// after the next region's requests, and the only wait for memory is where
// the next region's data moves into the current one's registers.
template <int kCounters, int kHold>
__global__ void __launch_bounds__(kRegionWG) k_region(FilterArgs F, uint64_t c0, BinPlan B,
                                                      const uint32_t *__restrict__ offsets,
                                                      const uint32_t *__restrict__ n_entries,
                                                      uint64_t *__restrict__ entries,
                                                      uint8_t *__restrict__ flags, int classify,
                                                      uint32_t tau, uint32_t *__restrict__ n_win,
                                                      Carry C) {
    constexpr int kUnroll = 8;
    constexpr uint32_t kSparseCells = kCounters / 8;  // cells of a region the sparse path stages
    static_assert(kSparseCells <= (uint32_t)kHold * kRegionWG, "sparse cells are held");
    static_assert(kCounters <= kRegionCounters, "local counter ids are 14-bit");
    __shared__ uint32_t hits[kCounters];
    __shared__ uint32_t first[kCounters];
    __shared__ unsigned long long s_cell[kSparseCells];
    __shared__ uint32_t s_nwin;
    const uint32_t S = 1u << B.region_shift;
    const uint64_t n_words = F.X * F.Y;
    uint32_t *e_word = (uint32_t *)entries;
    uint16_t *e_half = (uint16_t *)(e_word + B.entries_cap);
    // a region's work: entries [e0, e0 + n), cells [wbase, wbase + nw);
    // entry indices are 32-bit (a chunk's entries number less than 2^32)
    struct Region {
        uint32_t e0, n;
        uint64_t wbase;
        uint32_t nw;
        uint32_t c_off, c_n;  // carried chunk 0's records of the region
    };
    // entry ob + threadIdx.x (ob uniform) of a region of n entries from e0,
    // as loaded (hi = ~0u past its end); decoded where it is used, so that
    // prefetched loads stay in flight until then
    auto fetch = [&](uint32_t e0, uint32_t ob, uint32_t n) -> RawEntry {
        RawEntry e{~0u, ~0u};
        if (ob + threadIdx.x < n) {
            e.lo = at_byte(e_word + e0 + ob, 4u * threadIdx.x);
            e.hi = at_byte(e_half + e0 + ob, 2u * threadIdx.x);
        }
        return e;
    };
    auto t_of = [](RawEntry e) -> uint32_t {
        return (e.lo >> kLocalBits) | (e.hi << (32 - kLocalBits));
    };
    auto hold_of = [&](const Region &R) { return R.nw <= (uint32_t)kHold * kRegionWG; };
    // Carried records are classified only where the regions fit the sparse
    // tile (the launcher rejects a carry otherwise): in the instance that
    // holds the tile's cells.
    constexpr bool kTile = (uint32_t)kHold * kRegionWG == kSparseCells;
    const bool carry_in = kTile && C.mode == Carry::kIn && C.n_prev > 0;
    struct Bounds {
        uint32_t e0, e1;      // the region's entries
        uint32_t c_off, c_n;  // carried chunk 0's records of the region
    };
    // region r's bounds, requested as vector loads by lanes 0 (entry start)
    // and 1 (entry end) of every wavefront, and with carried records by
    // lanes 2 (record offset) and 3 (record count); bounds_of reads them out
    auto bounds = [&](uint32_t r) -> uint32_t {
        const uint32_t lane = threadIdx.x & 63u;
        uint32_t x = 0;
        if (r < B.n_regions && lane < 2u) {
            const uint32_t rr = r + lane;
            x = rr < B.n_regions ? offsets[(uint64_t)rr * B.G] : *n_entries;
        } else if (r < B.n_regions && carry_in && lane < 4u) {
            x = lane == 2u ? C.off[r] : C.n[r];
        }
        return x;
    };
    auto bounds_of = [](uint32_t x) -> Bounds {
        return Bounds{(uint32_t)__builtin_amdgcn_readlane((int)x, 0),
                      (uint32_t)__builtin_amdgcn_readlane((int)x, 1),
                      (uint32_t)__builtin_amdgcn_readlane((int)x, 2),
                      (uint32_t)__builtin_amdgcn_readlane((int)x, 3)};
    };
    // region r's first batch of entries and (when held) cells
    auto request = [&](uint32_t r, Bounds b, Region &R, RawEntry(&v)[kUnroll],
                       uint64_t(&cell)[kHold], uint32_t &ch) {
        const uint32_t cap = B.entries_cap < 0xFFFFFFFFull ? (uint32_t)B.entries_cap : 0xFFFFFFFFu;
        const uint32_t e0 = b.e0;
        uint32_t e1 = b.e1;
        if (e1 > cap)
            e1 = cap;
        R.e0 = e0;
        R.n = e1 > e0 ? e1 - e0 : 0u;
        R.wbase = (uint64_t)(B.region0 + r) << B.region_shift;
        R.nw = R.wbase + S <= n_words ? S : (uint32_t)(n_words - R.wbase);
        R.c_off = b.c_off;
        R.c_n = carry_in ? b.c_n : 0u;
        // the first carried record of each thread
        ch = threadIdx.x < R.c_n ? C.half[(uint64_t)R.c_off + threadIdx.x] : 0u;
#pragma unroll
        for (int u = 0; u < kUnroll; u++)
            v[u] = fetch(R.e0, (uint32_t)u * kRegionWG, R.n);
        const bool hold = hold_of(R);
#pragma unroll
        for (int k = 0; k < kHold; k++) {
            const uint32_t w = threadIdx.x + (uint32_t)k * kRegionWG;
            cell[k] = (hold && w < R.nw)
                          ? at_byte(F.words + R.wbase + (uint32_t)k * kRegionWG, 8u * threadIdx.x)
                          : 0ull;
        }
    };
    uint32_t r = blockIdx.x;
    if (r >= B.n_regions)
        return;
    Region R;
    RawEntry v[kUnroll];
    uint64_t cell[kHold];
    uint32_t ch;
    request(r, bounds_of(bounds(r)), R, v, cell, ch);
    uint32_t bn = bounds(r + gridDim.x);
    // the first region's data in place before the loop, so that no path
    // into the loop head has loads in flight
    __builtin_amdgcn_s_waitcnt(kWaitVmem);
    // Counters start every region clean (hits 0, first kIdle): cleared once
    // here, and each region leaves the counters it touched clean (the entry
    // that updates a counter resets it), so no region clears its own.
    for (uint32_t i = threadIdx.x; i < (uint32_t)kCounters; i += kRegionWG) {
        hits[i] = 0;
        first[i] = kIdle;
    }
    __syncthreads();
    // stores deferred from the previous region to just after the next
    // region's requests: its changed cells (sparse path) and its winner
    // count
    constexpr int kSparseHold = (int)(kSparseCells / kRegionWG);
    static_assert(kSparseHold >= 1 && kSparseHold <= kHold, "sparse cells per thread");
    uint64_t pc[kSparseHold];
    uint32_t pmask = 0;  // bit k: pc[k] is to be written (per thread)
    uint64_t pbase = 0;
    uint32_t p_r = ~0u, p_e0 = 0, p_n = 0;  // region, first entry, winner count
    const bool carry_out = C.mode == Carry::kOut;
    auto flush = [&]() {
#pragma unroll
        for (int k = 0; k < kSparseHold; k++)
            if (pmask & (1u << k))
                at_byte(F.words + pbase + (uint32_t)k * kRegionWG, 8u * threadIdx.x) = pc[k];
        pmask = 0;
        if (threadIdx.x == 0 && p_r != ~0u) {
            if (carry_out) {
                C.off[(uint64_t)C.chunk * C.stride + p_r] = p_e0;
                C.n[(uint64_t)C.chunk * C.stride + p_r] = p_n;
            } else if (n_win) {
                n_win[p_r] = p_n;
            }
        }
        p_r = ~0u;
    };
    for (;;) {
        const uint32_t rn = r + gridDim.x;
        Region Rn{};
        RawEntry vn[kUnroll];
        uint64_t celln[kHold];
        uint32_t chn = 0;
        if (rn < B.n_regions)
            request(rn, bounds_of(bn), Rn, vn, celln, chn);
        const uint32_t bn2 = bounds(rn + gridDim.x);
        flush();
        if (threadIdx.x == 0)
            s_nwin = 0;
        const WinnerSink out{flags,
                             c0,
                             carry_out ? C.word + (uint64_t)C.chunk * C.cap
                                       : (n_win ? e_word : nullptr),
                             carry_out ? C.half + (uint64_t)C.chunk * C.cap : e_half,
                             R.e0,
                             &s_nwin,
                             carry_out};
        if (R.n <= (uint32_t)(kUnroll * kRegionWG) && R.nw <= kSparseCells) {
            // Sparse region: every entry is in the register batch, and
            // counters are updated per entry, not by a pass over all of
            // them: the entry whose t is the counter's minimum applies
            // min(2^alpha - 1, old + hits) to the staged cell (a 64-bit LDS
            // add of the field's increase, which cannot carry into the next
            // field), flags its occurrence when the counter was zero and
            // resets the counter.  atomicCAS(first, t, kIdle) succeeds for
            // exactly one entry holding the minimum (with k_h > 1 one window
            // can put two entries on one counter).  The staged cells are
            // first read after the barrier that follows the atomics.
#pragma unroll
            for (int k = 0; k < kHold; k++) {
                const uint32_t w = threadIdx.x + (uint32_t)k * kRegionWG;
                if (w < R.nw)
                    s_cell[w] = cell[k];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; u++)
                if (v[u].hi != ~0u) {
                    const uint32_t local = v[u].lo & (kRegionCounters - 1);
                    atomicAdd(&hits[local], 1u);
                    atomicMin(&first[local], t_of(v[u]));
                }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kUnroll; u++)
                if (v[u].hi != ~0u) {
                    const uint32_t local = v[u].lo & (kRegionCounters - 1);
                    const uint32_t t = t_of(v[u]);
                    if (atomicCAS(&first[local], t, kIdle) != t)
                        continue;
                    const uint32_t w = local & (S - 1u);
                    const uint32_t sh = F.alpha * (local >> B.region_shift);
                    const uint32_t fm = (uint32_t)F.field_max;  // counters <= 32 bits
                    const uint32_t pf = (uint32_t)(s_cell[w] >> sh) & fm;
                    const uint32_t h = hits[local];
                    hits[local] = 0;
                    const uint32_t room = fm - pf;
                    const uint32_t inc = h < room ? h : room;
                    if (inc)
                        atomicAdd(&s_cell[w], (unsigned long long)inc << sh);
                    if (pf == 0)
                        put_winner(out, t, (classify && pf + inc > tau) ? 3u : 1u, local);
                }
            __syncthreads();
            pbase = R.wbase;
#pragma unroll
            for (int k = 0; k < kSparseHold; k++) {
                const uint32_t w = threadIdx.x + (uint32_t)k * kRegionWG;
                pc[k] = s_cell[w];
                if (w < R.nw && pc[k] != cell[k])
                    pmask |= 1u << k;
            }
        } else {
            for (uint32_t ob = 0;;) {  // the batch's first entry (uniform)
                // the next entries are requested before this batch's LDS atomics
                const uint32_t on = ob + (uint32_t)(kUnroll * kRegionWG);
                RawEntry w[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; u++)
                    w[u] = fetch(R.e0, on + (uint32_t)u * kRegionWG, R.n);
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
                    if (v[u].hi == ~0u)
                        continue;
                    const uint32_t local = v[u].lo & (kRegionCounters - 1);
                    atomicAdd(&hits[local], 1u);
                    atomicMin(&first[local], t_of(v[u]));
                }
                if (on >= R.n)
                    break;
                ob = on;
#pragma unroll
                for (int u = 0; u < kUnroll; u++)
                    v[u] = w[u];
            }
            // none of this path's loads in flight where it joins the sparse
            // path, whose registers it shares: the compiler would otherwise
            // wait for every load and store there, the next region's too
            __builtin_amdgcn_s_waitcnt(kWaitVmem);
            __syncthreads();
            if (hold_of(R)) {
#pragma unroll
                for (int k = 0; k < kHold; k++) {
                    const uint32_t w = threadIdx.x + (uint32_t)k * kRegionWG;
                    if (w < R.nw) {
                        const uint64_t next =
                            region_cell(F, B, R.wbase, w, cell[k], hits, first, out, classify, tau);
                        if (kTile && C.mode == Carry::kIn)
                            s_cell[w] = next;
                    }
                }
            } else {
                for (uint32_t w = threadIdx.x; w < R.nw; w += kRegionWG)
                    region_cell(F, B, R.wbase, w, F.words[R.wbase + w], hits, first, out,
                                classify, tau);
            }
        }
        __syncthreads();  // the region's LDS work and its winner count are complete
        if (kTile && C.mode == Carry::kIn) {
            // the carried records of this region: trustworthy (3) when the
            // counter's final value, now staged in s_cell, is above tau.
            // Chunk 0's records were requested with the region (the first
            // per thread) and its offset and count a region earlier, so that
            // in the common case nothing here waits for memory.
            auto mark = [&](uint32_t local) -> uint16_t {
                const uint64_t cv = s_cell[local & (S - 1u)];
                const uint32_t f =
                    (uint32_t)(cv >> (F.alpha * (local >> B.region_shift))) & (uint32_t)F.field_max;
                return f > tau ? 3u : 1u;
            };
            if (threadIdx.x < R.c_n)
                C.half[(uint64_t)R.c_off + threadIdx.x] = mark(ch);
            for (uint32_t i = threadIdx.x + kRegionWG; i < R.c_n; i += kRegionWG)
                C.half[(uint64_t)R.c_off + i] = mark(C.half[(uint64_t)R.c_off + i]);
            for (uint32_t j = 1; j < C.n_prev; j++) {
                const uint64_t at = (uint64_t)j * C.stride + r;
                const uint64_t x0 = (uint64_t)j * C.cap + C.off[at];
                const uint32_t n = C.n[at];
                for (uint32_t i = threadIdx.x; i < n; i += kRegionWG)
                    C.half[x0 + i] = mark(C.half[x0 + i]);
            }
            __syncthreads();  // s_cell is rewritten by the next region
        }
        // the region's winner count (wavefront-uniform; thread 0 writes it)
        p_r = r;
        p_e0 = R.e0;
        p_n = __builtin_amdgcn_readfirstlane(s_nwin);
        // the next region's data moves in on every path (also past the last
        // region): a path that skipped it would leave loads in flight at the
        // loop head, and the compiler would wait for them (and for every
        // store) at the head of the next region
        r = rn;
        R = Rn;
        bn = bn2;
#pragma unroll
        for (int u = 0; u < kUnroll; u++)
            v[u] = vn[u];
#pragma unroll
        for (int k = 0; k < kHold; k++)
            cell[k] = celln[k];
        ch = chn;
        if (r >= B.n_regions)
            break;
    }
    flush();
}

// The region pass's instance for a plan: the plan's counters per region,
// and two cells per thread (one with 8192 counters) where the regions fit the
// sparse tile, else four.
using RegionKernel = void (*)(FilterArgs, uint64_t, BinPlan, const uint32_t *, const uint32_t *,
                              uint64_t *, uint8_t *, int, uint32_t, uint32_t *, Carry);
RegionKernel region_kernel(const BinPlan &B) {
    const bool sparse_tile = carry_fits(B);
    if (B.region_counters == kSmallRegionCounters)
        return sparse_tile ? k_region<kSmallRegionCounters, kSmallRegionCounters / 8 / kRegionWG>
                           : k_region<kSmallRegionCounters, 4>;
    return sparse_tile ? k_region<kRegionCounters, kRegionCounters / 8 / kRegionWG>
                       : k_region<kRegionCounters, 4>;
}

// Workgroups of the persistent region pass: as many as the CUs hold at once
// (one per CU with the 144 KiB arrays, two with the 72 KiB ones), at most one
// per region.
uint32_t region_grid(uint32_t n_regions, uint32_t counters) {
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
            n_cu = v;
        else
            n_cu = 256;
    }
    const uint32_t g = (uint32_t)n_cu * (counters == (uint32_t)kSmallRegionCounters ? 2u : 1u);
    return n_regions < g ? n_regions : g;
}

// ---------------------------------------------------------------------------
// winner passes (records mode): the region pass's first-seen records, grouped
// by region, become flag bytes written in whole 16-byte groups.  Records are
// distributed by position in two counting-sort passes (by t >> 24, then by
// the next 5 bits) into blocks of 2^19 positions, whose flags are built in
// LDS bitmaps.  Runs are appended to each bucket at an atomic cursor (the
// order of records inside a bucket does not matter: a bitmap is built from
// them), in areas of the two entry buffers sized by the positions they
// cover, so that they always fit.
// ---------------------------------------------------------------------------
constexpr uint32_t kWinA = 24;             // level-A digit: t >> 24 (256 buckets)
constexpr uint32_t kWinB = 19;             // level-B digit: (t >> 19) & 31 (2^19 positions)
constexpr int kWinThreads = 1024;
constexpr int kWinBatch = 8192;            // records per LDS batch
constexpr uint32_t kWinRegions = 64;       // regions per level-A workgroup
constexpr uint32_t kWinSlices = 64;        // level-B workgroups per level-A bucket
constexpr uint32_t kWinBuckets = 256;
constexpr uint32_t kWinBlocksPerBucket = 1u << (kWinA - kWinB);

constexpr int kWinPer = kWinBatch / kWinThreads;  // records per thread and batch
static_assert(kWinBuckets <= 256 && kWinBlocksPerBucket <= 256, "digits are staged as bytes");

// A batch of records appended to buckets by digit d = (rec >> shift) & (nd
// - 1): record u of this thread is v[u] (present where bit u of ok is set).
// The records are ranked within their digit by LDS atomics, the digit
// counts scanned and each digit's run reserved at its bucket's cursor; the
// kept records (keep(rec)) are then staged in LDS in digit order and written
// out in that order, consecutive threads to consecutive addresses of a run
// (the order of records inside a run does not matter).  Ends with a barrier.
template <typename Rec, typename Keep>
__device__ void win_append(const Rec (&v)[kWinPer], uint32_t ok, uint32_t n, uint32_t shift,
                           uint32_t nd, uint32_t bucket0, uint32_t area_log, uint32_t *s_cnt,
                           uint32_t *s_start, uint32_t *s_base, uint32_t *s_wave,
                           uint32_t *s_stage, uint8_t *s_tag, uint32_t *__restrict__ cursor,
                           uint32_t *__restrict__ out, Keep keep) {
    for (uint32_t i = threadIdx.x; i < nd; i += kWinThreads)
        s_cnt[i] = 0;
    __syncthreads();
    uint32_t rk[kWinPer];
#pragma unroll
    for (int u = 0; u < kWinPer; u++)
        if (ok & (1u << u))
            rk[u] = atomicAdd(&s_cnt[(uint32_t)(v[u] >> shift) & (nd - 1u)], 1u);
    __syncthreads();
    // exclusive scan of the nd (<= 256) counts, 64 per wavefront
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t c = threadIdx.x < nd ? s_cnt[threadIdx.x] : 0u;
    uint32_t incl = c;
    if (threadIdx.x < nd) {
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (lane >= d)
                incl += o;
        }
        if (lane == 63 || threadIdx.x == nd - 1)
            s_wave[wave] = incl;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        uint32_t before = 0;
        for (uint32_t w = 0; w < wave; w++)
            before += s_wave[w];
        s_start[threadIdx.x] = before + incl - c;
        s_base[threadIdx.x] = c ? atomicAdd(&cursor[bucket0 + threadIdx.x], c) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kWinPer; u++)
        if (ok & (1u << u)) {
            const uint32_t d = (uint32_t)(v[u] >> shift) & (nd - 1u);
            const uint32_t j = s_start[d] + rk[u];
            s_stage[j] = keep(v[u]);
            s_tag[j] = (uint8_t)d;
        }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < n; j += kWinThreads) {
        const uint32_t d = s_tag[j];
        out[((uint64_t)(bucket0 + d) << area_log) + s_base[d] + (j - s_start[d])] = s_stage[j];
    }
    __syncthreads();
}

// Level A: the records of regions [kWinRegions * blockIdx.x, ...) (region r's
// n_win[r] records start at its first entry) -> bucket t >> 24, record
// (t & (2^24 - 1)) | mark << 24.  The regions' record counts are scanned in
// LDS first, so that the workgroup's records are one index range whose
// batches are filled by all threads at once (record i is found in its
// region by a binary search of the scan), not region after region.
__global__ void __launch_bounds__(kWinThreads) k_win_a(uint32_t n_regions,
                                                       const uint32_t *__restrict__ offsets,
                                                       uint64_t off_stride,
                                                       const uint32_t *__restrict__ n_win,
                                                       const uint32_t *__restrict__ e_word,
                                                       const uint16_t *__restrict__ e_half,
                                                       uint32_t *__restrict__ cursor,
                                                       uint32_t *__restrict__ out) {
    static_assert(kWinRegions == 64, "one wavefront scans the regions' counts");
    __shared__ uint32_t s_stage[kWinBatch];
    __shared__ uint8_t s_tag[kWinBatch];
    __shared__ uint32_t s_cnt[kWinBuckets], s_start[kWinBuckets], s_base[kWinBuckets];
    __shared__ uint32_t s_wave[kWinThreads / 64];
    __shared__ uint32_t s_first[kWinRegions];    // each region's first entry
    __shared__ uint32_t s_pre[kWinRegions + 1];  // records before each region
    const uint32_t r0 = blockIdx.x * kWinRegions;
    const uint32_t nr = r0 + kWinRegions < n_regions ? kWinRegions : n_regions - r0;
    if (threadIdx.x < 64) {
        const uint32_t i = threadIdx.x;
        const uint32_t n = i < nr ? n_win[r0 + i] : 0u;
        s_first[i] = i < nr ? offsets[(uint64_t)(r0 + i) * off_stride] : 0u;
        uint32_t incl = n;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (i >= d)
                incl += o;
        }
        s_pre[i + 1] = incl;
        if (i == 0)
            s_pre[0] = 0;
    }
    __syncthreads();
    const uint32_t total = s_pre[kWinRegions];
    auto keep = [](uint64_t r) -> uint32_t {
        return ((uint32_t)r & ((1u << kWinA) - 1u)) | ((uint32_t)(r >> 32) << kWinA);
    };
    for (uint32_t q = 0; q < total; q += kWinBatch) {
        const uint32_t m = total - q < (uint32_t)kWinBatch ? total - q : (uint32_t)kWinBatch;
        uint64_t v[kWinPer];
        uint32_t ok = 0;
#pragma unroll
        for (int u = 0; u < kWinPer; u++) {
            const uint32_t i = threadIdx.x + (uint32_t)u * kWinThreads;
            v[u] = 0;
            if (i < m) {
                const uint32_t idx = q + i;
                uint32_t j = 0;  // the last region with s_pre[j] <= idx
#pragma unroll
                for (uint32_t step = kWinRegions / 2; step; step >>= 1)
                    if (s_pre[j + step] <= idx)
                        j += step;
                const uint64_t x = (uint64_t)s_first[j] + (idx - s_pre[j]);
                v[u] = ((uint64_t)e_half[x] << 32) | e_word[x];
                ok |= 1u << u;
            }
        }
        win_append(v, ok, m, kWinA, kWinBuckets, 0, kWinA, s_cnt, s_start, s_base, s_wave,
                   s_stage, s_tag, cursor, out, keep);
    }
}

// Level B: slice blockIdx.y of level-A bucket a = blockIdx.x -> block
// (a << 5) | ((t24 >> 19) & 31), record (t & (2^19 - 1)) | mark << 19.
__global__ void __launch_bounds__(kWinThreads) k_win_b(const uint32_t *__restrict__ in,
                                                       const uint32_t *__restrict__ cursor_a,
                                                       uint32_t *__restrict__ cursor_b,
                                                       uint32_t *__restrict__ out) {
    __shared__ uint32_t s_stage[kWinBatch];
    __shared__ uint8_t s_tag[kWinBatch];
    __shared__ uint32_t s_cnt[kWinBlocksPerBucket], s_start[kWinBlocksPerBucket],
        s_base[kWinBlocksPerBucket];
    __shared__ uint32_t s_wave[kWinThreads / 64];
    const uint32_t a = blockIdx.x;
    const uint32_t n = cursor_a[a];
    const uint32_t per = ((1u << kWinA) + kWinSlices - 1) / kWinSlices;
    const uint32_t q0 = blockIdx.y * per;
    const uint32_t q1 = q0 + per < n ? q0 + per : n;
    const uint32_t *src = in + ((uint64_t)a << kWinA);
    auto keep = [](uint32_t v) -> uint32_t {
        return (v & ((1u << kWinB) - 1u)) | ((v >> kWinA) << kWinB);
    };
    for (uint32_t q = q0; q < q1; q += kWinBatch) {
        const uint32_t m = q1 - q < (uint32_t)kWinBatch ? q1 - q : (uint32_t)kWinBatch;
        uint32_t v[kWinPer];
        uint32_t ok = 0;
#pragma unroll
        for (int u = 0; u < kWinPer; u++) {
            const uint32_t i = threadIdx.x + (uint32_t)u * kWinThreads;
            v[u] = i < m ? src[q + i] : 0u;
            if (i < m)
                ok |= 1u << u;
        }
        // digit (t24 >> 19) & 31 of the record (t24 | mark << 24)
        win_append(v, ok, m, kWinB, kWinBlocksPerBucket, a * kWinBlocksPerBucket, kWinB, s_cnt,
                   s_start, s_base, s_wave, s_stage, s_tag, cursor_b, out, keep);
    }
}

// The flag bytes of block g = blockIdx.x (positions [g << 19, ...) of the
// chunk, flags at c0 + those) from its records: distinct and trustworthy
// bitmaps in LDS, then every 16-position group with a mark written whole
// (the others keep the zeros the ingest wrote).
__global__ void __launch_bounds__(kWinThreads) k_win_flags(const uint32_t *__restrict__ in,
                                                           const uint32_t *__restrict__ cursor_b,
                                                           uint64_t c0, uint64_t len,
                                                           uint8_t *__restrict__ flags) {
    constexpr uint32_t kWords = (1u << kWinB) / 32;
    __shared__ uint32_t s_d[kWords];
    __shared__ uint32_t s_t[kWords];
    const uint32_t g = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < kWords; i += kWinThreads) {
        s_d[i] = 0;
        s_t[i] = 0;
    }
    __syncthreads();
    const uint32_t n = cursor_b[g];
    const uint32_t *src = in + ((uint64_t)g << kWinB);
    for (uint32_t i = threadIdx.x; i < n; i += kWinThreads) {
        const uint32_t v = src[i];
        const uint32_t p = v & ((1u << kWinB) - 1u);
        atomicOr(&s_d[p >> 5], 1u << (p & 31u));
        if ((v >> kWinB) & 2u)
            atomicOr(&s_t[p >> 5], 1u << (p & 31u));
    }
    __syncthreads();
    const uint64_t p0 = (uint64_t)g << kWinB;
    uint4 *f128 = reinterpret_cast<uint4 *>(flags + c0 + p0);
    const uint32_t groups = (uint32_t)((len - p0 < (1u << kWinB) ? len - p0 : (1u << kWinB)) + 15) / 16;
    for (uint32_t q = threadIdx.x; q < groups; q += kWinThreads) {
        const uint32_t d16 = (s_d[q >> 1] >> ((q & 1u) * 16)) & 0xFFFFu;
        if (!d16)
            continue;
        const uint32_t t16 = (s_t[q >> 1] >> ((q & 1u) * 16)) & 0xFFFFu;
        uint32_t w[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            uint32_t x = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t b = 4 * u + j;
                x |= (((d16 >> b) & 1u) | (((t16 >> b) & 1u) << 1)) << (8 * j);
            }
            w[u] = x;
        }
        f128[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Records mode when a chunk's flag bytes are larger than the Infinity
// Cache (256 MB): random single-byte flag stores into HBM-resident flags
// cost the 8 Gbase insert's region pass about 20 ms; KMERCO_WINNER_RECORDS=1
// forces records mode for every chunk (tests), 0 turns it off.
bool records_mode(uint64_t len) {
    const char *e = std::getenv("KMERCO_WINNER_RECORDS");
    if (e && *e)
        return std::atoi(e) != 0;
    return len > (1ull << 28);
}

// The winner passes of one chunk [c0, c0 + len): its records, region r's
// n_win[r] of them at offsets[r * off_stride] of the word and half arrays.
hipError_t winner_passes(uint32_t n_regions, const uint32_t *offsets, uint64_t off_stride,
                         const uint32_t *n_win, const uint32_t *rec_word,
                         const uint16_t *rec_half, uint64_t c0, uint64_t len, const Workspace &W,
                         hipStream_t s, Profiler *P) {
    uint32_t *cursors = W.win_cursors;  // kWinBuckets level-A, then the blocks' level-B cursors
    const uint32_t n_a = (uint32_t)((len + (1ull << kWinA) - 1) >> kWinA);
    const uint32_t n_blocks = (uint32_t)((len + (1ull << kWinB) - 1) >> kWinB);
    if (P)
        P->begin(kPhWinners, s);
    static_assert(kWinBuckets + kWinBuckets * kWinBlocksPerBucket == kWinCursors, "cursors");
    hipError_t e = fill_u32(cursors, kWinCursors, 0u, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_win_a, dim3((n_regions + kWinRegions - 1) / kWinRegions),
                           dim3(kWinThreads), 0, s, n_regions, offsets, off_stride, n_win,
                           rec_word, rec_half, cursors, (uint32_t *)W.bucketed);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_win_b, dim3(n_a, kWinSlices), dim3(kWinThreads), 0, s,
                           (const uint32_t *)W.bucketed, (const uint32_t *)cursors,
                           cursors + kWinBuckets, (uint32_t *)W.entries);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_win_flags, dim3(n_blocks), dim3(kWinThreads), 0, s,
                           (const uint32_t *)W.entries, (const uint32_t *)(cursors + kWinBuckets),
                           c0, len, W.flags8);
        e = hipGetLastError();
    }
    if (P)
        P->end(s);
    return e;
}

// The winner passes of one chunk after its region pass in records mode: the
// records sit in the region lists' entry segments.
hipError_t launch_winner_passes(const BinPlan &Q, uint64_t c0, uint64_t len, const Workspace &W,
                                const uint32_t *n_win, hipStream_t s, Profiler *P) {
    const uint32_t *e_word = (const uint32_t *)W.entries;
    return winner_passes(Q.n_regions, (const uint32_t *)W.matrix, Q.G, n_win, e_word,
                         (const uint16_t *)(e_word + Q.entries_cap), c0, len, W, s, P);
}

bool carry_fits(const BinPlan &plan) {
    // the region's cells are staged in the region pass's s_cell array
    // (kSparseCells = counters / 8 entries)
    return (1u << plan.region_shift) <= plan.region_counters / 8u;
}

Carry carry_of(const Workspace &W, const BinPlan &plan, uint64_t chunk_positions,
               uint64_t n_chunks) {
    Carry c{};
    if (n_chunks < 2 || !carry_fits(plan))
        return c;
    const uint64_t prev = n_chunks - 1;
    if (!W.carry || W.carry_cap < prev * chunk_positions ||
        W.carry_idx_cap < prev * plan.n_regions)
        return c;
    c.n_prev = (uint32_t)prev;
    c.stride = plan.n_regions;
    c.cap = chunk_positions;
    c.word = (uint32_t *)W.carry;
    c.half = W.carry + 2 * W.carry_cap;
    c.off = W.carry_off;
    c.n = W.carry_n;
    return c;
}

hipError_t launch_carried_winners(const BinPlan &plan, const Carry &carry, uint32_t j, uint64_t c0,
                                  uint64_t len, const Workspace &W, hipStream_t s, Profiler *P) {
    const uint64_t at = (uint64_t)j * carry.stride;
    return winner_passes(plan.n_regions, carry.off + at, 1, carry.n + at,
                         carry.word + (uint64_t)j * carry.cap, carry.half + (uint64_t)j * carry.cap,
                         c0, len, W, s, P);
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
bool bin_plan(const FilterArgs &F, uint64_t chunk_positions, BinPlan &B, uint32_t part_log,
              uint32_t region_counters) {
    if (region_counters != kRegionCounters && region_counters != kSmallRegionCounters)
        return false;
    // largest power-of-two cell count whose eta counters fit the LDS arrays
    uint32_t shift = 0;
    while (((2ull << shift) * F.eta) <= (uint64_t)region_counters)
        shift++;
    if (((1ull << shift) * F.eta) > (uint64_t)region_counters)
        return false;
    if (part_log > kPartLog)
        part_log = kPartLog;
    const uint64_t n_words = F.X * F.Y;
    const uint64_t n_regions = (n_words + (1ull << shift) - 1) >> shift;
    B = BinPlan{};
    B.region_shift = shift;
    B.region_counters = region_counters;
    B.slice = kSlice;
    if (n_regions > (1ull << part_log)) {
        // partitioned: bin workgroups count partitions, passes over each
        // partition's list bin its regions as the single-level path does
        const uint64_t np = (n_regions + (1ull << part_log) - 1) >> part_log;
        if (np > kMaxParts)
            return false;
        B.n_regions = (uint32_t)n_regions;
        B.n_parts = (uint32_t)np;
        B.part_log = part_log;
        // 64 buckets per partition (fewer for tiny test partitions), so that
        // global bucket b holds regions [b << bshift, (b + 1) << bshift)
        B.bucket_shift = part_log >= 6 ? part_log - 6 : 0;
        B.n_buckets = (uint32_t)((n_regions + (1ull << B.bucket_shift) - 1) >> B.bucket_shift);
        // list workgroups per partition: about kListWGs in all, and region /
        // bucket count matrices of bounded size
        uint64_t lg = (kListWGs + np - 1) / np;
        if (lg > kMaxListG)
            lg = kMaxListG;
        if (lg * n_regions > kMaxMatrix)
            lg = kMaxMatrix / n_regions;
        const uint64_t nbp = (1ull << part_log) >> B.bucket_shift;
        if (lg * np * nbp > kMaxCoarse)
            lg = kMaxCoarse / (np * nbp);
        if (lg == 0)
            return false;
        B.list_g = (uint32_t)lg;
        uint64_t tile = kBinTileMin;
        while ((chunk_positions + tile - 1) / tile * np > kMaxMatrix)
            tile *= 2;
        B.tile = tile;
        B.G = (uint32_t)((chunk_positions + tile - 1) / tile);
        B.n_slices = (B.G + B.slice - 1) / B.slice;
        return true;
    }
    B.n_regions = (uint32_t)n_regions;
    uint32_t bshift = 0;
    while (((n_regions + (1ull << bshift) - 1) >> bshift) > kMaxBuckets)
        bshift++;
    B.bucket_shift = bshift;
    B.n_buckets = (uint32_t)((n_regions + (1ull << bshift) - 1) >> bshift);
    // positions per bin workgroup: kBinTileMin, enough to amortise the
    // histograms (small chunks: fewer, down to kBinTileFloor, so that about
    // kBinSpread workgroups still spread over the chip), and a region matrix
    // of at most kMaxMatrix counts
    uint64_t tile = (chunk_positions + kBinSpread - 1) / kBinSpread;
    tile = (tile + kBinWG - 1) / kBinWG * kBinWG;
    tile = tile < kBinTileFloor ? kBinTileFloor : (tile > kBinTileMin ? kBinTileMin : tile);
    while ((chunk_positions + tile - 1) / tile * n_regions > kMaxMatrix)
        tile *= 2;
    B.tile = tile;
    B.G = (uint32_t)((chunk_positions + tile - 1) / tile);
    B.n_slices = (B.G + B.slice - 1) / B.slice;
    return true;
}

namespace {

// Workgroup size of a partitioned-path scatter pass (its batches hold 8 or
// 16 entries per thread): the environment variable `name` (512 or 1024) when
// set, else dflt.  Levels 1 and 2 (KMERCO_L1_THREADS, KMERCO_L2_THREADS)
// take 1024 by default: with batches twice as large their runs are twice as
// long (per 8 Gbase step, level 1 26.8 against 30.2 ms, level 2 31.7 against
// 37.2 ms); the partition scatter (KMERCO_L0_THREADS) keeps 512 (22.2 against
// 24.6 ms).
int pass_threads(const char *name, int dflt) {
    const char *e = std::getenv(name);
    if (!e || !*e)
        return dflt;
    return std::atoi(e) == 1024 ? 1024 : kBinWG;
}

// The hashing kernel for a filter layout and k (partitioned or not).
template <bool kParts>
auto bin_count_kernel(const FilterArgs &F, uint32_t k) {
    const bool fast = fast_layout(F);
    if (k > 32)
        return fast ? k_bin_count<kParts, true, true> : k_bin_count<kParts, false, true>;
    return fast ? k_bin_count<kParts, true, false> : k_bin_count<kParts, false, false>;
}

// Partitioned chunk: hash + partition counts, partition lists, then the
// per-partition binning for all partitions at once (list workgroups size
// their slices from the partition sizes on the device), level 2 and the
// region pass over every region of the countBF.
hipError_t launch_parts_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                              const BinPlan &plan, const Workspace &W, bool classify,
                              uint32_t tau, const Carry &carry, hipStream_t s, Profiler *P) {
    BinPlan B = plan;
    B.G = (uint32_t)((c1 - c0 + B.tile - 1) / B.tile);
    B.n_slices = (B.G + B.slice - 1) / B.slice;
    B.entries_cap = W.entries_cap;
    const uint64_t n_pmat = (uint64_t)B.n_parts * B.G;
    // slot ids (positions x hash functions) and their partition bytes live
    // in `bucketed` until the partition scatter has read them; the partition
    // lists in `entries` until the list binning has read them
    uint32_t *slots = (uint32_t *)W.bucketed;
    uint8_t *parts = (uint8_t *)(slots + W.entries_cap);
    uint64_t *plist = W.entries;
    if (P)
        P->begin(kPhBinCount, s);
    hipLaunchKernelGGL(bin_count_kernel<true>(F, R.k), dim3(B.G), dim3(kBinWG),
                       (size_t)B.n_parts * sizeof(uint32_t), s, F, R, c0, c1, B, slots, parts,
                       W.pmat, nullptr, (unsigned long long *)(W.totals + 5));
    if (P)
        P->end(s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhScan, s);
        e = scan_u32_u32(W.pmat, W.pmat, n_pmat, W.n_entries + 2, W.partial32, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_part_bounds, dim3(1), dim3(256), 0, s, (const uint32_t *)W.pmat,
                               B.G, B.n_parts, (const uint32_t *)(W.n_entries + 2), W.pbounds);
            e = hipGetLastError();
        }
        if (P)
            P->end(s);
    }
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhBinPart, s);
        if (pass_threads("KMERCO_L0_THREADS", kBinWG) == 1024)
            hipLaunchKernelGGL(k_part_scatter<1024>, dim3(B.G), dim3(1024), 0, s, c0, c1, F.k_h,
                               B, (const uint32_t *)slots, (const uint8_t *)parts,
                               (const uint32_t *)W.pmat, plist);
        else
            hipLaunchKernelGGL(k_part_scatter<kBinWG>, dim3(B.G), dim3(kBinWG), 0, s, c0, c1,
                               F.k_h, B, (const uint32_t *)slots, (const uint8_t *)parts,
                               (const uint32_t *)W.pmat, plist);
        if (P)
            P->end(s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pass_plan, dim3(1), dim3(256), 0, s, (const uint32_t *)W.pbounds,
                           B.n_parts, B.list_g, W.entries_cap, W.pdesc);
        e = hipGetLastError();
    }
    if (e != hipSuccess)
        return e;
    // the plan of the list passes, level 2 and the region pass: every region
    // of the countBF, list_g workgroup columns
    BinPlan Q = B;
    Q.G = B.list_g;
    Q.n_slices = (Q.G + Q.slice - 1) / Q.slice;
    Q.region0 = 0;
    const uint32_t per = 1u << B.part_log;
    const uint64_t nbp = per >> B.bucket_shift;
    const uint64_t n_fine = (uint64_t)B.n_regions * Q.G;
    const uint64_t n_coarse = (uint64_t)B.n_parts * nbp * Q.G;
    const uint32_t n_list = B.n_parts * B.list_g;
    const uint32_t hist = B.n_regions < per ? B.n_regions : per;
    if (P)
        P->begin(kPhPartCount, s);
    hipLaunchKernelGGL(k_list_count, dim3(n_list), dim3(kBinWG), (size_t)hist * sizeof(uint32_t),
                       s, (const uint64_t *)plist, (const uint64_t *)W.pdesc, Q, W.matrix_t,
                       W.coarse);
    if (P)
        P->end(s);
    e = hipGetLastError();
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhScan, s);
        e = transpose_u32_blocks(W.matrix_t, W.matrix, B.list_g, per, B.n_regions, s);
        if (e == hipSuccess)
            e = scan_u32_u32(W.matrix, W.matrix, n_fine, W.n_entries, W.partial32, s);
        if (e == hipSuccess)
            e = scan_u32_u32(W.coarse, W.coarse, n_coarse, W.n_entries + 1, W.partial32, s);
        if (P)
            P->end(s);
    }
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhBinBucket, s);
        if (pass_threads("KMERCO_L1_THREADS", 1024) == 1024)
            hipLaunchKernelGGL(k_bin_bucket_list<1024>, dim3(n_list), dim3(1024), 0, s,
                               (const uint64_t *)plist, (const uint64_t *)W.pdesc, Q,
                               (const uint32_t *)W.coarse, W.bucketed);
        else
            hipLaunchKernelGGL(k_bin_bucket_list<kBinWG>, dim3(n_list), dim3(kBinWG), 0, s,
                               (const uint64_t *)plist, (const uint64_t *)W.pdesc, Q,
                               (const uint32_t *)W.coarse, W.bucketed);
        if (P)
            P->end(s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhBinRegion, s);
        if (pass_threads("KMERCO_L2_THREADS", 1024) == 1024)
            hipLaunchKernelGGL((k_bin_region<false, 1024>), dim3(Q.n_buckets * Q.n_slices),
                               dim3(1024), 0, s, Q, (const uint32_t *)W.coarse,
                               (const uint32_t *)(W.n_entries + 1), (const uint32_t *)W.matrix,
                               (const uint64_t *)W.bucketed, W.entries);
        else
            hipLaunchKernelGGL((k_bin_region<false, kBinWG>), dim3(Q.n_buckets * Q.n_slices),
                               dim3(kBinWG), 0, s, Q, (const uint32_t *)W.coarse,
                               (const uint32_t *)(W.n_entries + 1), (const uint32_t *)W.matrix,
                               (const uint64_t *)W.bucketed, W.entries);
        if (P)
            P->end(s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhRegion, s);
        const bool rec = carry.mode != Carry::kOut && records_mode(c1 - c0);
        hipLaunchKernelGGL(region_kernel(Q),
                           dim3(region_grid(Q.n_regions, Q.region_counters)), dim3(kRegionWG),
                           0, s, F, c0, Q,
                           (const uint32_t *)W.matrix, (const uint32_t *)W.n_entries, W.entries,
                           W.flags8, classify ? 1 : 0, tau, rec ? W.matrix_t : nullptr, carry);
        if (P)
            P->end(s);
        e = hipGetLastError();
        if (e == hipSuccess && rec)
            e = launch_winner_passes(Q, c0, c1 - c0, W, W.matrix_t, s, P);
    }
    return e;
}

}  // namespace

hipError_t launch_binned_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                               const BinPlan &plan, const Workspace &W, bool classify,
                               uint32_t tau, const Carry &carry, hipStream_t s, Profiler *P) {
    if ((c0 & 63u) || !R.valid)
        return hipErrorInvalidValue;  // waves read 64 bits of the valid-window bitmap
    if (carry.mode != Carry::kNone && (!carry_fits(plan) || carry.stride != plan.n_regions))
        return hipErrorInvalidValue;  // the region pass stages the cells it classifies against
    if (plan.n_parts)
        return launch_parts_chunk(F, R, c0, c1, plan, W, classify, tau, carry, s, P);
    if (c1 - c0 > kBinChunk || (c1 - c0) * F.k_h >= (1ull << 32))
        return hipErrorInvalidValue;  // the level-1 pass indexes in 32 bits
    BinPlan B = plan;
    B.G = (uint32_t)((c1 - c0 + B.tile - 1) / B.tile);
    B.n_slices = (B.G + B.slice - 1) / B.slice;
    B.entries_cap = W.entries_cap;
    // the 6-byte entries' fields (bucket ids, t - slice start)
    if ((B.slice & (B.slice - 1)) || B.tile * B.slice > (1ull << kMaxSliceLog) ||
        B.bucket_shift + kLocalBits > kBucketIdBits)
        return hipErrorInvalidValue;
    uint32_t *bucket_word = (uint32_t *)W.bucketed;
    uint16_t *bucket_half = (uint16_t *)(bucket_word + W.entries_cap);
    const size_t lds = (size_t)B.n_regions * sizeof(uint32_t);
    const uint64_t n_fine = (uint64_t)B.n_regions * B.G;
    const uint64_t n_coarse = (uint64_t)B.n_buckets * B.G;
    if (P)
        P->begin(kPhBinCount, s);
    hipLaunchKernelGGL(bin_count_kernel<false>(F, R.k), dim3(B.G), dim3(kBinWG), lds, s, F, R,
                       c0, c1, B, W.slots, nullptr, W.matrix_t, W.coarse,
                       (unsigned long long *)(W.totals + 5));
    if (P)
        P->end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhScan, s);
    e = transpose_u32(W.matrix_t, W.matrix, B.G, B.n_regions, s);
    if (e == hipSuccess)
        e = scan_u32_u32(W.matrix, W.matrix, n_fine, W.n_entries, W.partial32, s);
    if (e == hipSuccess)
        e = scan_u32_u32(W.coarse, W.coarse, n_coarse, W.n_entries + 1, W.partial32, s);
    if (P)
        P->end(s);
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhBinBucket, s);
    hipLaunchKernelGGL(k_bin_bucket, dim3(B.G), dim3(kBinWG), kLevel1Reserve, s, c0, c1, F.k_h, B,
                       (const uint32_t *)W.slots, (const uint32_t *)W.coarse, bucket_word,
                       bucket_half);
    if (P)
        P->end(s);
    e = hipGetLastError();
    if (e == hipSuccess) {
        if (P)
            P->begin(kPhBinRegion, s);
        hipLaunchKernelGGL((k_bin_region<true, kBinWG>), dim3(B.n_buckets * B.n_slices), dim3(kBinWG), 0, s, B,
                           (const uint32_t *)W.coarse, (const uint32_t *)(W.n_entries + 1),
                           (const uint32_t *)W.matrix, (const uint64_t *)W.bucketed, W.entries);
        if (P)
            P->end(s);
        e = hipGetLastError();
    }
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhRegion, s);
    const bool rec = carry.mode != Carry::kOut && records_mode(c1 - c0);
    hipLaunchKernelGGL(region_kernel(B),
                       dim3(region_grid(B.n_regions, B.region_counters)), dim3(kRegionWG), 0,
                       s, F, c0, B,
                       (const uint32_t *)W.matrix, (const uint32_t *)W.n_entries, W.entries,
                       W.flags8, classify ? 1 : 0, tau, rec ? W.matrix_t : nullptr, carry);
    if (P)
        P->end(s);
    e = hipGetLastError();
    if (e == hipSuccess && rec)
        e = launch_winner_passes(B, c0, c1 - c0, W, W.matrix_t, s, P);
    return e;
}

}  // namespace kc
