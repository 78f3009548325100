// gfx950 kernels of the KmerCo insertion and classification phases.
//
// Insertion (Algorithm 1) for one call, positions p = window start offsets in
// the concatenated read buffer (an occurrence's place in the sequential visit
// order is its p):
//   ingest        ASCII -> 2-bit codes + invalid-base bitmap       (streaming)
//   read_starts   read-start bitmap from the CSR offsets
//   per chunk of positions [c0, c1) with t = p - c0 < 2^32:
//     claim       for each slot of each occurrence whose counter is zero
//                 before the chunk: atomicMin(first[slot], t)
//     increment   saturating counter increments (Algorithm 3)
//     resolve     occurrence t is distinct iff first[slot] == t for one of
//                 its slots; the winner resets the entry; per-position flag
//                 bits and per-tile counts
//   (claim and increment are one kernel while the whole filter is zero)
//   scan          exclusive scan of per-tile distinct counts
//   scatter       distinct canonical keys written in position order
//
// Query-I before insert (Algorithm 4, then Algorithm 3) in the sequential
// algorithm returns 0 for occurrence t exactly when some slot of t was never
// touched by an earlier occurrence; the claim/resolve pair computes that set
// for all occurrences of a chunk at once, so the distinct list equals the
// sequential one even when distinct k-mers share slots.
#include <hip/hip_runtime.h>

#include "kc_device.hpp"
#include "kc_kernels.hpp"

namespace kc {

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, uint64_t n, uint64_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// ingest: one thread per 32 bases -> codes[2i], codes[2i+1], inv[i]
// ---------------------------------------------------------------------------
__global__ void k_ingest(const uint8_t *__restrict__ reads, uint64_t n_bases,
                         uint32_t *__restrict__ codes, uint32_t *__restrict__ inv,
                         uint64_t n_mask_words, int aligned16) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_mask_words)
        return;
    uint64_t p0 = i * 32u;
    uint32_t bytes[8];
    if (aligned16 && p0 + 32u <= n_bases) {
        const uint4 *v = reinterpret_cast<const uint4 *>(reads + p0);
        uint4 a = v[0], b = v[1];
        bytes[0] = a.x; bytes[1] = a.y; bytes[2] = a.z; bytes[3] = a.w;
        bytes[4] = b.x; bytes[5] = b.y; bytes[6] = b.z; bytes[7] = b.w;
    } else {
        for (int w = 0; w < 8; w++) {
            uint32_t x = 0;
            for (int c = 0; c < 4; c++) {
                uint64_t q = p0 + 4u * w + c;
                uint32_t b = q < n_bases ? reads[q] : 0u;  // 0 = invalid
                x |= b << (8 * c);
            }
            bytes[w] = x;
        }
    }
    uint32_t c_hi = 0, c_lo = 0, bad = 0;
#pragma unroll
    for (int q = 0; q < 32; q++) {
        uint32_t b = (bytes[q >> 2] >> (8 * (q & 3))) & 0xFFu;
        uint32_t c = base_code(b);
        uint32_t ok = base_valid(b, c);
        c = ok ? c : 0u;
        bad |= (ok ? 0u : 1u) << q;
        if (q < 16)
            c_hi |= c << (30 - 2 * q);
        else
            c_lo |= c << (30 - 2 * (q - 16));
    }
    codes[2 * i] = c_hi;
    codes[2 * i + 1] = c_lo;
    inv[i] = bad;
}

__global__ void k_read_starts(const uint64_t *__restrict__ offsets, uint64_t n_reads,
                              uint64_t n_bases, uint32_t *__restrict__ rs) {
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_reads)
        return;
    uint64_t o = offsets[r];
    if (o < n_bases)
        atomicOr(&rs[o >> 5], 1u << (o & 31u));
}

// ---------------------------------------------------------------------------
// insertion phases.  One workgroup per tile of kTile positions; thread tid
// visits p = tile0 + kWG*j + tid, so a wavefront always covers 64 aligned
// consecutive positions (one flag word).
// ---------------------------------------------------------------------------
template <int MODE>  // 0: claim only, 1: increment only, 2: claim + increment (zero filter)
__global__ void __launch_bounds__(kWG) k_insert_phase(FilterArgs F, ReadsArgs R, uint64_t c0,
                                                      uint64_t c1) {
    const uint64_t tile0 = c0 + (uint64_t)blockIdx.x * kTile;
#pragma unroll 1
    for (int j = 0; j < kTile / kWG; j++) {
        uint64_t p = tile0 + (uint64_t)j * kWG + threadIdx.x;
        if (p >= c1 || !window_valid(R, p))
            continue;
        uint64_t fwd = window_key(R.codes, p, R.k);
        Canon c = canonical(fwd, R.k);
        uint32_t t = (uint32_t)(p - c0);
        for (uint32_t a = 1; a <= F.k_h; a++) {
            uint64_t h = (a == 1) ? c.h1 : hash_a(c.b0, c.b1, a);
            uint64_t word;
            uint32_t l;
            slot_of(F, h, word, l);
            uint64_t idx = word * F.eta + l;
            if (MODE == 0) {
                if (read_counter(F, word, l) == 0)
                    atomicMin(&F.aux[idx], t);
            } else {
                if (MODE == 2)
                    atomicMin(&F.aux[idx], t);
                saturating_increment(&F.words[word], F.alpha * l, F.field_max);
            }
        }
    }
}

__global__ void __launch_bounds__(kWG) k_resolve(FilterArgs F, ReadsArgs R, uint64_t c0,
                                                 uint64_t c1, uint64_t *__restrict__ flags,
                                                 uint32_t *__restrict__ tile_distinct,
                                                 uint32_t *__restrict__ tile_valid) {
    __shared__ uint32_t s_cnt[2][kWG / 64];
    const uint64_t tile = c0 / kTile + blockIdx.x;
    const uint64_t tile0 = tile * kTile;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    uint32_t n_dist = 0, n_valid = 0;
#pragma unroll 1
    for (int j = 0; j < kTile / kWG; j++) {
        uint64_t p = tile0 + (uint64_t)j * kWG + threadIdx.x;
        bool valid = p < c1 && window_valid(R, p);
        bool win = false;
        if (valid) {
            uint64_t fwd = window_key(R.codes, p, R.k);
            Canon c = canonical(fwd, R.k);
            uint32_t t = (uint32_t)(p - c0);
            for (uint32_t a = 1; a <= F.k_h; a++) {
                uint64_t h = (a == 1) ? c.h1 : hash_a(c.b0, c.b1, a);
                uint64_t word;
                uint32_t l;
                slot_of(F, h, word, l);
                uint64_t idx = word * F.eta + l;
                if (F.aux[idx] == t) {
                    win = true;
                    F.aux[idx] = kIdle;
                }
            }
        }
        uint64_t wmask = __ballot(win);
        uint64_t vmask = __ballot(valid);
        if (lane == 0) {
            flags[(tile0 + (uint64_t)j * kWG) / 64 + wave] = wmask;
            n_dist += (uint32_t)__popcll(wmask);
            n_valid += (uint32_t)__popcll(vmask);
        }
    }
    if (lane == 0) {
        s_cnt[0][wave] = n_dist;
        s_cnt[1][wave] = n_valid;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int w = 0; w < kWG / 64; w++) {
            a += s_cnt[0][w];
            b += s_cnt[1][w];
        }
        tile_distinct[tile] = a;
        tile_valid[tile] = b;
    }
}

// ---------------------------------------------------------------------------
// single-workgroup exclusive scan of per-block counts
//   off[i] = (base ? *base : 0) + sum(cnt[0..i)),  totals[0] = sum(cnt),
//   totals[1] = sum(cnt2) when cnt2 is given
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kScanWG) k_scan(const uint32_t *__restrict__ cnt,
                                                  const uint32_t *__restrict__ cnt2, uint64_t nb,
                                                  uint64_t *__restrict__ off,
                                                  const uint64_t *__restrict__ base,
                                                  uint64_t *__restrict__ totals) {
    __shared__ uint64_t s_sum[kScanWG];
    __shared__ uint64_t s_sum2[kScanWG];
    const uint64_t per = (nb + kScanWG - 1) / kScanWG;
    const uint64_t lo = per * threadIdx.x;
    const uint64_t hi = lo + per < nb ? lo + per : nb;
    uint64_t sum = 0, sum2 = 0;
    for (uint64_t i = lo; i < hi; i++) {
        sum += cnt[i];
        if (cnt2)
            sum2 += cnt2[i];
    }
    s_sum[threadIdx.x] = sum;
    s_sum2[threadIdx.x] = sum2;
    __syncthreads();
    // Hillis-Steele inclusive scan over the per-thread sums
    for (int d = 1; d < kScanWG; d <<= 1) {
        uint64_t v = threadIdx.x >= (unsigned)d ? s_sum[threadIdx.x - d] : 0;
        uint64_t v2 = threadIdx.x >= (unsigned)d ? s_sum2[threadIdx.x - d] : 0;
        __syncthreads();
        s_sum[threadIdx.x] += v;
        s_sum2[threadIdx.x] += v2;
        __syncthreads();
    }
    uint64_t run = (base ? *base : 0) + s_sum[threadIdx.x] - sum;
    for (uint64_t i = lo; i < hi; i++) {
        off[i] = run;
        run += cnt[i];
    }
    if (threadIdx.x == kScanWG - 1) {
        totals[0] = s_sum[kScanWG - 1];
        totals[1] = s_sum2[kScanWG - 1];
    }
}

// ---------------------------------------------------------------------------
// ordered scatter of the distinct keys
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kWG) k_scatter_distinct(ReadsArgs R, uint64_t first_tile,
                                                          const uint64_t *__restrict__ flags,
                                                          const uint64_t *__restrict__ tile_off,
                                                          uint64_t *__restrict__ out,
                                                          uint64_t cap) {
    const uint64_t tile = first_tile + blockIdx.x;
    const uint64_t tile0 = tile * kTile;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    constexpr int kWords = kTile / 64;
    const uint64_t *fw = flags + tile0 / 64;
    uint64_t base = tile_off[tile];
#pragma unroll 1
    for (int j = 0; j < kTile / kWG; j++) {
        int widx = j * (kWG / 64) + wave;
        uint64_t word = fw[widx];
        if (((word >> lane) & 1ull) == 0)
            continue;
        uint64_t before = 0;
        for (int w = 0; w < widx; w++)
            before += (uint64_t)__popcll(fw[w]);
        before += (uint64_t)__popcll(word & ((1ull << lane) - 1ull));
        uint64_t p = tile0 + (uint64_t)j * kWG + threadIdx.x;
        uint64_t fwd = window_key(R.codes, p, R.k);
        uint64_t key = canonical(fwd, R.k).key;
        uint64_t dst = base + before;
        if (dst < cap)
            out[dst] = key;
    }
    (void)kWords;
}

__global__ void k_finish_insert(uint64_t *__restrict__ n_distinct, uint64_t *__restrict__ n_windows,
                                const uint64_t *__restrict__ totals, uint64_t cap,
                                uint32_t *__restrict__ status) {
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    uint64_t nd = *n_distinct + totals[0];
    *n_distinct = nd;
    if (n_windows)
        *n_windows += totals[1];
    if (nd > cap)
        atomicOr(status, kStatusRange);
}

// ---------------------------------------------------------------------------
// classification / query
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t query_key(const FilterArgs &F, uint64_t key) {
    uint32_t b0, b1;
    key_blocks(key, b0, b1);
    uint64_t best = 0;
    for (uint32_t a = 1; a <= F.k_h; a++) {
        uint64_t word;
        uint32_t l;
        slot_of(F, hash_a(b0, b1, a), word, l);
        uint64_t v = read_counter(F, word, l);
        if (v == 0)
            return 0;
        best = (a == 1 || v < best) ? v : best;
    }
    return best;
}

__global__ void __launch_bounds__(kWG) k_classify_mark(FilterArgs F, const uint64_t *__restrict__ keys,
                                                       const uint64_t *__restrict__ n_keys,
                                                       uint64_t cap, uint32_t tau,
                                                       uint64_t *__restrict__ tmask,
                                                       uint32_t *__restrict__ tile_trust) {
    __shared__ uint32_t s_cnt[kWG / 64];
    const uint64_t n = *n_keys < cap ? *n_keys : cap;
    const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    uint32_t cnt = 0;
    if (tile0 >= n) {
        if (threadIdx.x == 0)
            tile_trust[blockIdx.x] = 0;
        return;
    }
#pragma unroll 1
    for (int j = 0; j < kTile / kWG; j++) {
        uint64_t i = tile0 + (uint64_t)j * kWG + threadIdx.x;
        bool trust = false;
        if (i < n)
            trust = query_key(F, keys[i]) > (uint64_t)tau;
        uint64_t m = __ballot(trust);
        if (lane == 0) {
            tmask[(tile0 + (uint64_t)j * kWG) / 64 + wave] = m;
            cnt += (uint32_t)__popcll(m);
        }
    }
    if (lane == 0)
        s_cnt[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int w = 0; w < kWG / 64; w++)
            a += s_cnt[w];
        tile_trust[blockIdx.x] = a;
    }
}

__global__ void __launch_bounds__(kWG) k_classify_scatter(const uint64_t *__restrict__ keys,
                                                          const uint64_t *__restrict__ n_keys,
                                                          uint64_t cap,
                                                          const uint64_t *__restrict__ tmask,
                                                          const uint64_t *__restrict__ tile_off,
                                                          uint64_t *__restrict__ trust,
                                                          uint64_t *__restrict__ err) {
    const uint64_t n = *n_keys < cap ? *n_keys : cap;
    const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
    if (tile0 >= n)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t *fw = tmask + tile0 / 64;
    const uint64_t base = tile_off[blockIdx.x];
#pragma unroll 1
    for (int j = 0; j < kTile / kWG; j++) {
        uint64_t i = tile0 + (uint64_t)j * kWG + threadIdx.x;
        if (i >= n)
            break;
        int widx = j * (kWG / 64) + wave;
        uint64_t word = fw[widx];
        uint64_t before = 0;
        for (int w = 0; w < widx; w++)
            before += (uint64_t)__popcll(fw[w]);
        before += (uint64_t)__popcll(word & ((1ull << lane) - 1ull));
        uint64_t t_idx = base + before;  // trustworthy keys before i
        if ((word >> lane) & 1ull)
            trust[t_idx] = keys[i];
        else
            err[i - t_idx] = keys[i];
    }
}

__global__ void k_finish_classify(const uint64_t *__restrict__ n_keys, uint64_t cap,
                                  const uint64_t *__restrict__ totals,
                                  uint64_t *__restrict__ n_trust, uint64_t *__restrict__ n_err) {
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const uint64_t n = *n_keys < cap ? *n_keys : cap;
    *n_trust = totals[0];
    *n_err = n - totals[0];
}

__global__ void k_query(FilterArgs F, const uint64_t *__restrict__ keys, uint64_t n,
                        uint32_t *__restrict__ freq) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        freq[i] = (uint32_t)query_key(F, keys[i]);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(uint64_t n, unsigned per) {
    uint64_t g = (n + per - 1) / per;
    return (unsigned)(g ? g : 1);
}

hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Launch `kernel` bracketed by profiler events for `phase`.
template <typename K, typename... A>
static hipError_t launch(Profiler *P, int phase, K kernel, dim3 grid, dim3 block, hipStream_t s,
                         A... args) {
    if (P)
        P->begin(phase, s);
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    if (P)
        P->end(s);
    return hipGetLastError();
}

hipError_t launch_ingest(const uint8_t *reads, uint64_t n_bases, const uint64_t *offsets,
                         uint64_t n_reads, const Workspace &W, hipStream_t s, Profiler *P) {
    uint64_t n_mask = mask_words(n_bases);
    if (P)
        P->begin(kPhIngest, s);
    hipError_t e = fill_u32(W.rs, n_mask, 0u, s);
    if (e == hipSuccess) {
        int aligned = ((uintptr_t)reads & 15u) == 0;
        hipLaunchKernelGGL(k_ingest, dim3(grid_for(n_mask, 256)), dim3(256), 0, s, reads,
                           n_bases, W.codes, W.inv, n_mask, aligned);
        e = hipGetLastError();
    }
    if (e == hipSuccess && n_reads > 0) {
        hipLaunchKernelGGL(k_read_starts, dim3(grid_for(n_reads, 256)), dim3(256), 0, s, offsets,
                           n_reads, n_bases, W.rs);
        e = hipGetLastError();
    }
    if (P)
        P->end(s);
    return e;
}

hipError_t launch_insert_chunk(const FilterArgs &F, const ReadsArgs &R, uint64_t c0, uint64_t c1,
                               bool zero_filter, const Workspace &W, hipStream_t s, Profiler *P) {
    dim3 grid(grid_for(c1 - c0, kTile)), block(kWG);
    hipError_t e;
    if (zero_filter) {
        e = launch(P, kPhClaimIncrement, k_insert_phase<2>, grid, block, s, F, R, c0, c1);
    } else {
        e = launch(P, kPhClaim, k_insert_phase<0>, grid, block, s, F, R, c0, c1);
        if (e == hipSuccess)
            e = launch(P, kPhIncrement, k_insert_phase<1>, grid, block, s, F, R, c0, c1);
    }
    if (e != hipSuccess)
        return e;
    return launch(P, kPhResolve, k_resolve, grid, block, s, F, R, c0, c1, W.flags, W.tile_a,
                  W.tile_b);
}

hipError_t launch_distinct(const ReadsArgs &R, const Workspace &W, uint64_t *distinct,
                           uint64_t cap, uint64_t *n_distinct, uint64_t *n_windows,
                           uint32_t *status, hipStream_t s, Profiler *P) {
    uint64_t n_tiles = (R.n_bases + kTile - 1) / kTile;
    hipError_t e = launch(P, kPhScan, k_scan, dim3(1), dim3(kScanWG), s,
                          (const uint32_t *)W.tile_a, (const uint32_t *)W.tile_b, n_tiles,
                          W.tile_off, (const uint64_t *)n_distinct, W.totals);
    if (e == hipSuccess)
        e = launch(P, kPhScatter, k_scatter_distinct, dim3((unsigned)n_tiles), dim3(kWG), s, R,
                   (uint64_t)0, (const uint64_t *)W.flags, (const uint64_t *)W.tile_off, distinct,
                   cap);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_finish_insert, dim3(1), dim3(64), 0, s, n_distinct, n_windows,
                           (const uint64_t *)W.totals, cap, status);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_classify(const FilterArgs &F, const uint64_t *keys, const uint64_t *n_keys,
                           uint64_t cap, uint32_t tau, uint64_t *trust, uint64_t *n_trust,
                           uint64_t *err, uint64_t *n_err, const Workspace &W, hipStream_t s,
                           Profiler *P) {
    uint64_t n_tiles = (cap + kTile - 1) / kTile;
    if (n_tiles == 0)
        n_tiles = 1;
    hipError_t e = launch(P, kPhClassifyMark, k_classify_mark, dim3((unsigned)n_tiles), dim3(kWG),
                          s, F, keys, n_keys, cap, tau, W.flags, W.tile_a);
    if (e == hipSuccess)
        e = launch(P, kPhScan, k_scan, dim3(1), dim3(kScanWG), s, (const uint32_t *)W.tile_a,
                   (const uint32_t *)nullptr, n_tiles, W.tile_off, (const uint64_t *)nullptr,
                   W.totals);
    if (e == hipSuccess)
        e = launch(P, kPhClassifyScatter, k_classify_scatter, dim3((unsigned)n_tiles), dim3(kWG),
                   s, keys, n_keys, cap, (const uint64_t *)W.flags,
                   (const uint64_t *)W.tile_off, trust, err);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_finish_classify, dim3(1), dim3(64), 0, s, n_keys, cap,
                           (const uint64_t *)W.totals, n_trust, n_err);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_query(const FilterArgs &F, const uint64_t *keys, uint64_t n, uint32_t *freq,
                        hipStream_t s, Profiler *P) {
    if (n == 0)
        return hipSuccess;
    return launch(P, kPhQuery, k_query, dim3(grid_for(n, 256)), dim3(256), s, F, keys, n, freq);
}

}  // namespace kc
