// Binned insertion: the countBF update and the first-seen resolution done in
// LDS, one workgroup per filter region, with no global atomics.
//
// For one chunk of positions [c0, c1) (t = p - c0):
//   bin_count   hash every valid window; per-workgroup LDS histogram of the
//               regions its slots fall in -> count matrix [region][workgroup]
//   (scan)      exclusive scan of the matrix in region-major order: the
//               offset of every (region, workgroup) segment of the entry list
//   bin_write   hash again; append (t, local counter) entries to the segments
//   region      one workgroup per region: in LDS, hits[c] += 1 and
//               first[c] = min(first[c], t) over the region's entries; then
//               counter = min(2^alpha - 1, old + hits) per counter, and the
//               occurrence first[c] is distinct when the counter was zero
//               before the chunk (the sequential Query-I result)
// The order of entries inside a segment does not matter: sums and minima
// are order-independent, so the outputs are deterministic.
#include <hip/hip_runtime.h>

#include "kc_device.hpp"
#include "kc_kernels.hpp"

namespace kc {

namespace {

__device__ __forceinline__ uint32_t wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

}  // namespace

__global__ void __launch_bounds__(kBinWG) k_bin_count(FilterArgs F, ReadsArgs R, uint64_t c0,
                                                      uint64_t c1, BinPlan B,
                                                      uint32_t *__restrict__ matrix) {
    extern __shared__ uint32_t hist[];
    for (uint32_t i = threadIdx.x; i < B.n_regions; i += kBinWG)
        hist[i] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t shift = B.region_shift;
    const uint64_t g0 = c0 + (uint64_t)blockIdx.x * B.tile;
    const uint64_t g1 = g0 + B.tile < c1 ? g0 + B.tile : c1;
    for (uint64_t pb = g0 + 64u * wave_id(); pb < g1; pb += kBinWG) {
        WaveWords w;
        wave_load(R, pb, w);
        uint64_t fwd;
        bool valid = wave_window(w, pb, lane, R.k, R.n_bases, fwd) && pb + lane < g1;
        if (valid) {
            const Canon c = canonical_fast(fwd, R.k);
            for (uint32_t a = 1; a <= F.k_h; a++) {
                uint64_t word;
                uint32_t l;
                slot_of(F, a == 1 ? c.h1 : hash_a(c.b0, c.b1, a), word, l);
                atomicAdd(&hist[(uint32_t)(word >> shift)], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < B.n_regions; i += kBinWG)
        matrix[(uint64_t)i * B.G + blockIdx.x] = hist[i];
}

__global__ void __launch_bounds__(kBinWG) k_bin_write(FilterArgs F, ReadsArgs R, uint64_t c0,
                                                      uint64_t c1, BinPlan B,
                                                      const uint32_t *__restrict__ offsets,
                                                      uint64_t *__restrict__ entries) {
    extern __shared__ uint32_t cursor[];
    for (uint32_t i = threadIdx.x; i < B.n_regions; i += kBinWG)
        cursor[i] = offsets[(uint64_t)i * B.G + blockIdx.x];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g0 = c0 + (uint64_t)blockIdx.x * B.tile;
    const uint64_t g1 = g0 + B.tile < c1 ? g0 + B.tile : c1;
    const uint32_t shift = B.region_shift;
    const uint64_t smask = (1ull << shift) - 1ull;
    const uint64_t cap = B.entries_cap;
    for (uint64_t pb = g0 + 64u * wave_id(); pb < g1; pb += kBinWG) {
        WaveWords w;
        wave_load(R, pb, w);
        uint64_t fwd;
        bool valid = wave_window(w, pb, lane, R.k, R.n_bases, fwd) && pb + lane < g1;
        if (valid) {
            const Canon c = canonical_fast(fwd, R.k);
            const uint64_t t = pb + lane - c0;
            for (uint32_t a = 1; a <= F.k_h; a++) {
                uint64_t word;
                uint32_t l;
                slot_of(F, a == 1 ? c.h1 : hash_a(c.b0, c.b1, a), word, l);
                uint32_t r = (uint32_t)(word >> shift);
                uint32_t local = (l << shift) | (uint32_t)(word & smask);
                uint32_t pos = atomicAdd(&cursor[r], 1u);
                if (pos < cap)
                    entries[pos] = (t << 32) | local;
            }
        }
    }
}

__global__ void __launch_bounds__(kRegionWG) k_region(FilterArgs F, uint64_t c0, BinPlan B,
                                                      const uint32_t *__restrict__ offsets,
                                                      const uint32_t *__restrict__ n_entries,
                                                      const uint64_t *__restrict__ entries,
                                                      uint8_t *__restrict__ flags, int classify,
                                                      uint32_t tau) {
    __shared__ uint32_t hits[kRegionCounters];
    __shared__ uint32_t first[kRegionCounters];
    const uint32_t r = blockIdx.x;
    const uint32_t S = 1u << B.region_shift;
    const uint32_t n_ctr = S * F.eta;
    for (uint32_t i = threadIdx.x; i < n_ctr; i += kRegionWG) {
        hits[i] = 0;
        first[i] = kIdle;
    }
    __syncthreads();
    const uint64_t e0 = offsets[(uint64_t)r * B.G];
    uint64_t e1 = r + 1 < B.n_regions ? offsets[(uint64_t)(r + 1) * B.G] : *n_entries;
    if (e1 > B.entries_cap)
        e1 = B.entries_cap;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += kRegionWG) {
        uint64_t v = entries[e];
        uint32_t local = (uint32_t)v & (kRegionCounters - 1);
        atomicAdd(&hits[local], 1u);
        atomicMin(&first[local], (uint32_t)(v >> 32));
    }
    __syncthreads();
    const uint64_t wbase = (uint64_t)r << B.region_shift;
    const uint64_t n_words = F.X * F.Y;
    const uint32_t nw = wbase + S <= n_words ? S : (uint32_t)(n_words - wbase);
    for (uint32_t w = threadIdx.x; w < nw; w += kRegionWG) {
        const uint64_t pre = F.words[wbase + w];
        uint64_t next = pre;
        for (uint32_t l = 0; l < F.eta; l++) {
            const uint32_t idx = (l << B.region_shift) | w;
            const uint64_t h = hits[idx];
            if (h == 0)
                continue;
            const uint32_t shift = F.alpha * l;
            const uint64_t pf = (pre >> shift) & F.field_max;
            const uint64_t room = F.field_max - pf;
            const uint64_t nf = pf + (h < room ? h : room);
            next = (next & ~(F.field_max << shift)) | (nf << shift);
            if (pf == 0) {
                uint8_t flag = 1;
                if (classify && nf > (uint64_t)tau)
                    flag = 3;
                flags[c0 + first[idx]] = flag;
            }
        }
        if (next != pre)
            F.words[wbase + w] = next;
    }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
bool bin_plan(const FilterArgs &F, uint64_t chunk_positions, BinPlan &B) {
    // largest power-of-two word count whose eta counters fit the LDS arrays
    uint32_t shift = 0;
    while (((2ull << shift) * F.eta) <= (uint64_t)kRegionCounters)
        shift++;
    if (((1ull << shift) * F.eta) > (uint64_t)kRegionCounters)
        return false;
    uint64_t n_words = F.X * F.Y;
    uint64_t n_regions = (n_words + (1ull << shift) - 1) >> shift;
    if (n_regions > kMaxRegions)
        return false;
    B.region_shift = shift;
    B.n_regions = (uint32_t)n_regions;
    // positions per bin workgroup: enough to amortise the histogram, and a
    // matrix of at most kMaxMatrix counts
    uint64_t tile = kBinTileMin;
    while ((chunk_positions + tile - 1) / tile * n_regions > kMaxMatrix)
        tile *= 2;
    B.tile = tile;
    B.G = (uint32_t)((chunk_positions + tile - 1) / tile);
    return true;
}

hipError_t launch_binned_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                               const BinPlan &plan, const Workspace &W, bool classify,
                               uint32_t tau, hipStream_t s, Profiler *P) {
    BinPlan B = plan;
    B.G = (uint32_t)((c1 - c0 + B.tile - 1) / B.tile);
    B.entries_cap = W.entries_cap;
    const size_t lds = (size_t)B.n_regions * sizeof(uint32_t);
    const uint64_t n_mat = (uint64_t)B.n_regions * B.G;
    if (P)
        P->begin(kPhBinCount, s);
    hipLaunchKernelGGL(k_bin_count, dim3(B.G), dim3(kBinWG), lds, s, F, R, c0, c1, B, W.matrix);
    if (P)
        P->end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhScan, s);
    e = scan_u32_u32(W.matrix, W.matrix, n_mat, W.n_entries, W.partial32, s);
    if (P)
        P->end(s);
    if (e != hipSuccess)
        return e;
    if (P)
        P->begin(kPhBinWrite, s);
    hipLaunchKernelGGL(k_bin_write, dim3(B.G), dim3(kBinWG), lds, s, F, R, c0, c1, B,
                       (const uint32_t *)W.matrix, W.entries);
    if (P)
        P->end(s);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (P)
        P->begin(kPhRegion, s);
    hipLaunchKernelGGL(k_region, dim3(B.n_regions), dim3(kRegionWG), 0, s, F, c0, B,
                       (const uint32_t *)W.matrix, (const uint32_t *)W.n_entries,
                       (const uint64_t *)W.entries, W.flags8, classify ? 1 : 0, tau);
    if (P)
        P->end(s);
    return hipGetLastError();
}

}  // namespace kc
