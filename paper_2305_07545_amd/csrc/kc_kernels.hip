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
                         uint32_t *__restrict__ rs, uint8_t *__restrict__ flags,
                         uint64_t n_mask_words, uint64_t n_flag_words, int aligned16) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_mask_words)
        return;
    // clear this word's read-start bits (set afterwards by k_read_starts) and
    // its 32 flag bytes
    rs[i] = 0;
    if (i < n_flag_words) {
        uint4 *f = reinterpret_cast<uint4 *>(flags + 32u * i);
        f[0] = make_uint4(0u, 0u, 0u, 0u);
        f[1] = make_uint4(0u, 0u, 0u, 0u);
    }
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
    uint32_t c_hi = 0, c_lo = 0, good = 0;
#pragma unroll
    for (int w = 0; w < 8; w++) {
        uint32_t v4;
        const uint32_t c8 = codes4(bytes[w], v4);
        good |= v4 << (4 * w);
        if (w < 4)
            c_hi |= c8 << (24 - 8 * w);
        else
            c_lo |= c8 << (24 - 8 * (w - 4));
    }
    codes[2 * i] = c_hi;
    codes[2 * i + 1] = c_lo;
    inv[i] = ~good;
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
                                                 uint64_t c1, uint8_t *__restrict__ flags) {
    const uint64_t tile0 = c0 + (uint64_t)blockIdx.x * kTile;
#pragma unroll 1
    for (int j = 0; j < kTile / kWG; j++) {
        uint64_t p = tile0 + (uint64_t)j * kWG + threadIdx.x;
        if (p >= c1 || !window_valid(R, p))
            continue;
        uint64_t fwd = window_key(R.codes, p, R.k);
        Canon c = canonical(fwd, R.k);
        uint32_t t = (uint32_t)(p - c0);
        bool win = false;
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
        if (win)
            flags[p] = 1;
    }
}

// ---------------------------------------------------------------------------
// ordered output of the distinct k-mers (and optionally of their
// trustworthy / erroneous split): flag byte per position, 1 = distinct,
// 3 = distinct and trustworthy
// ---------------------------------------------------------------------------
// Per tile: distinct flags (bit 0 of a flag byte), trustworthy flags (bit 1)
// and, when asked, valid windows.  kSuper tiles per iteration; one 32-bit
// word (4 flag bytes) per thread and tile.
__global__ void __launch_bounds__(kWG) k_tile_count(ReadsArgs R, const uint8_t *__restrict__ flags,
                                                    uint64_t n_tiles, int count_valid,
                                                    uint32_t *__restrict__ tile_d,
                                                    uint32_t *__restrict__ tile_t,
                                                    uint32_t *__restrict__ tile_v) {
    // one wavefront per tile: 16 flag bytes per lane, counts reduced by
    // shuffles, no LDS and no barriers
    static_assert(kTile == 64 * 16, "16 flag bytes per lane and tile");
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * (kWG / 64);
    const uint4 *f128 = reinterpret_cast<const uint4 *>(flags);
    for (uint64_t tile = (uint64_t)blockIdx.x * (kWG / 64) + wave; tile < n_tiles;
         tile += n_waves) {
        const uint4 x = f128[tile * 64 + lane];
        uint32_t nd = (uint32_t)(__popc(x.x & 0x01010101u) + __popc(x.y & 0x01010101u) +
                                 __popc(x.z & 0x01010101u) + __popc(x.w & 0x01010101u));
        uint32_t nt = (uint32_t)(__popc(x.x & 0x02020202u) + __popc(x.y & 0x02020202u) +
                                 __popc(x.z & 0x02020202u) + __popc(x.w & 0x02020202u));
        uint32_t nv = 0;  // the same on every lane
        if (count_valid) {
#pragma unroll 1
            for (int j = 0; j < kTile / 64; j++) {
                const uint64_t pb = tile * kTile + 64u * (uint64_t)j;
                WaveWords w;
                wave_load(R, pb, w);
                uint64_t fwd;
                nv += (uint32_t)__popcll(__ballot(wave_window(w, pb, lane, R.k, R.n_bases, fwd)));
            }
        }
        for (uint32_t d = 32; d >= 1; d >>= 1) {
            nd += __shfl_down(nd, d, 64);
            nt += __shfl_down(nt, d, 64);
        }
        if (lane == 0) {
            tile_d[tile] = nd;
            tile_t[tile] = nt;
            tile_v[tile] = nv;
        }
    }
}

// Ordered output, one wavefront per tile.  The tile's flagged positions are
// first gathered into a wavefront-private list in position order (so that
// only they are hashed), then each listed window's canonical key goes to the
// distinct list and, when split, to the trustworthy or erroneous list.
// kWide: k-mers of 33..64 bases, written as (low, high) word pairs.
template <bool kWide>
__global__ void __launch_bounds__(kWG) k_compact(ReadsArgs R, const uint8_t *__restrict__ flags,
                                                 uint64_t n_tiles,
                                                 const uint64_t *__restrict__ off_d,
                                                 const uint64_t *__restrict__ off_t,
                                                 const uint64_t *__restrict__ call_base,
                                                 uint64_t *__restrict__ distinct, uint64_t cap_d,
                                                 uint64_t *__restrict__ trust,
                                                 uint64_t *__restrict__ err, uint64_t cap_te,
                                                 int split) {
    static_assert(kTile == 64 * 16, "16 flag bytes per lane and tile");
    static_assert(kTile <= 32768, "list entries are 15-bit");
    __shared__ uint16_t s_pos[kWG / 64][kTile];  // tile position of the i-th flagged window
    __shared__ uint16_t s_tb[kWG / 64][kTile];   // trustworthy windows before it; bit 15: it is one
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * (kWG / 64);
    const uint4 *f128 = reinterpret_cast<const uint4 *>(flags);
    const uint64_t base = split ? *call_base : 0;
    uint16_t *lpos = s_pos[wave];
    uint16_t *ltb = s_tb[wave];
    // each wavefront's next tile: its flags and offsets are requested before
    // the current tile's keys are written
    uint64_t tile = (uint64_t)blockIdx.x * (kWG / 64) + wave;
    uint4 nx = make_uint4(0u, 0u, 0u, 0u);
    uint64_t nd = 0, nt = 0;
    if (tile < n_tiles) {
        nx = f128[tile * 64 + lane];
        nd = off_d[tile];
        nt = split ? off_t[tile] : 0;
    }
    for (; tile < n_tiles; tile += n_waves) {
        const uint4 x4 = nx;
        const uint64_t od = nd;
        const uint64_t ot = nt;
        const uint64_t next = tile + n_waves;
        if (next < n_tiles) {
            nx = f128[next * 64 + lane];
            nd = off_d[next];
            nt = split ? off_t[next] : 0;
        }
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
        list_flags(x, lane, rd, rt, lpos, ltb);
        __builtin_amdgcn_wave_barrier();
        const uint64_t pos0 = tile * kTile;
        for (uint32_t i = lane; i < tot_d; i += 64) {
            const uint64_t p = pos0 + lpos[i];
            uint64_t key, key_hi = 0;
            if (kWide) {
                const Key128 c = canonical_wide(window_key_wide(R.codes, p, R.k), R.k).key;
                key = c.lo;
                key_hi = c.hi;
            } else {
                key = canonical_fast(window_key(R.codes, p, R.k), R.k).key;
            }
            auto put = [&](uint64_t *out, uint64_t at) {
                if (kWide) {
                    out[2 * at] = key;
                    out[2 * at + 1] = key_hi;
                } else {
                    out[at] = key;
                }
            };
            const uint64_t d = od + i;
            if (d < cap_d)
                put(distinct, d);
            if (split) {
                const uint32_t tb = ltb[i];
                const uint64_t ti = ot + (tb & 0x7FFFu);  // trustworthy keys before this one
                if (tb & 0x8000u) {
                    if (ti < cap_te)
                        put(trust, ti);
                } else {
                    const uint64_t ei = (d - base) - ti;  // erroneous keys before this one
                    if (ei < cap_te)
                        put(err, ei);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();  // the list is rewritten by the next tile
    }
}

// totals[0] distinct, [1] trustworthy, [2] valid windows counted by the tile
// pass, [5] valid windows counted by the insert passes
__global__ void k_finish_insert(uint64_t *__restrict__ n_distinct, uint64_t *__restrict__ n_windows,
                                uint64_t *__restrict__ n_trust, uint64_t *__restrict__ n_err,
                                const uint64_t *__restrict__ totals, int windows_counted,
                                uint64_t cap_d, uint64_t cap_te, uint32_t *__restrict__ status) {
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const uint64_t nd = *n_distinct + totals[0];
    *n_distinct = nd;
    if (n_windows)
        *n_windows += windows_counted ? totals[5] : totals[2];
    bool over = nd > cap_d;
    if (n_trust) {
        *n_trust = totals[1];
        *n_err = totals[0] - totals[1];
        over = over || totals[1] > cap_te || totals[0] - totals[1] > cap_te;
    }
    if (over)
        atomicOr(status, kStatusRange);
}

// copies *src to *dst (device scalars), so that a later kernel sees a value
// as it was at this point of the stream
__global__ void k_copy_u64(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dst = *src;
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

// Query-II of a 33..64-base key (Algorithm 5 with the 16-byte hash)
__device__ __forceinline__ uint64_t query_key_wide(const FilterArgs &F, Key128 key) {
    uint32_t b[4];
    key_blocks_wide(key, b);
    uint64_t best = 0;
    for (uint32_t a = 1; a <= F.k_h; a++) {
        uint64_t word;
        uint32_t l;
        slot_of(F, hash_a_wide(b, a), word, l);
        uint64_t v = read_counter(F, word, l);
        if (v == 0)
            return 0;
        best = (a == 1 || v < best) ? v : best;
    }
    return best;
}

// Query-II of a canonical key from its H_1 and MM3 blocks (as the hashing
// passes compute them): H_1 is not recomputed.
__device__ __forceinline__ uint64_t query_canon(const FilterArgs &F, const Canon &c) {
    uint64_t best = 0;
    for (uint32_t a = 1; a <= F.k_h; a++) {
        uint64_t word;
        uint32_t l;
        slot_of(F, a == 1 ? c.h1 : hash_a(c.b0, c.b1, a), word, l);
        const uint64_t v = read_counter(F, word, l);
        if (v == 0)
            return 0;
        best = (a == 1 || v < best) ? v : best;
    }
    return best;
}

__device__ __forceinline__ uint64_t query_canon_wide(const FilterArgs &F, const CanonWide &c) {
    uint64_t best = 0;
    for (uint32_t a = 1; a <= F.k_h; a++) {
        uint64_t word;
        uint32_t l;
        slot_of(F, a == 1 ? c.h1 : hash_a_wide(c.b, a), word, l);
        const uint64_t v = read_counter(F, word, l);
        if (v == 0)
            return 0;
        best = (a == 1 || v < best) ? v : best;
    }
    return best;
}

// Classification in the position domain (Algorithm 2 with Query-II): every
// position of [0, n_tiles * kTile) flagged distinct (1) whose k-mer's
// frequency in the countBF as it stands is above tau becomes 3 (distinct
// and trustworthy), the mark the region pass gives the first-seen k-mers
// whose final counter it knows; the ordered compaction then splits the
// distinct list by the marks.  One wavefront per tile of 1024 flag bytes
// (16 per lane): the flagged positions are listed in LDS, then each lane
// takes one, rebuilds its canonical k-mer from the packed codes and reads
// its k_h counters.  The marks go into an LDS copy of the tile, and a lane
// whose 16 bytes changed writes them back as one 16-byte store (no single-
// byte stores at scattered positions).
template <bool kWide>
__global__ void __launch_bounds__(kWG) k_classify_flags(FilterArgs F, ReadsArgs R,
                                                        uint8_t *__restrict__ flags,
                                                        uint64_t n_tiles, uint32_t tau) {
    static_assert(kTile == 64 * 16, "16 flag bytes per lane and tile");
    __shared__ uint16_t s_pos[kWG / 64][kTile];
    __shared__ uint16_t s_tb[kWG / 64][kTile];  // list_flags' second list (unused here)
    __shared__ uint4 s_tile[kWG / 64][64];      // the tile's flag bytes, marked
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * (kWG / 64);
    uint4 *f128 = reinterpret_cast<uint4 *>(flags);
    uint16_t *lpos = s_pos[wave];
    uint16_t *ltb = s_tb[wave];
    uint8_t *lmark = reinterpret_cast<uint8_t *>(s_tile[wave]);
    for (uint64_t tile = (uint64_t)blockIdx.x * (kWG / 64) + wave; tile < n_tiles;
         tile += n_waves) {
        const uint4 x4 = f128[tile * 64 + lane];
        const uint32_t x[4] = {x4.x, x4.y, x4.z, x4.w};
        uint32_t cd = 0;
#pragma unroll
        for (int u = 0; u < 4; u++)
            cd += (uint32_t)__popc(x[u] & 0x01010101u);
        uint32_t tot_d;
        const uint32_t rd = wave_exclusive(cd, lane, tot_d);
        if (tot_d == 0)
            continue;
        list_flags(x, lane, rd, 0, lpos, ltb);
        s_tile[wave][lane] = x4;
        __builtin_amdgcn_wave_barrier();
        const uint64_t pos0 = tile * kTile;
        for (uint32_t i = lane; i < tot_d; i += 64) {
            const uint32_t q = lpos[i];
            const uint64_t p = pos0 + q;
            const uint64_t f =
                kWide ? query_canon_wide(F, canonical_wide(window_key_wide(R.codes, p, R.k), R.k))
                      : query_canon(F, canonical_fast(window_key(R.codes, p, R.k), R.k));
            if (f > (uint64_t)tau)
                lmark[q] = 3;
        }
        __builtin_amdgcn_wave_barrier();
        const uint4 y4 = s_tile[wave][lane];
        if (y4.x != x4.x || y4.y != x4.y || y4.z != x4.z || y4.w != x4.w)
            f128[tile * 64 + lane] = y4;
        __builtin_amdgcn_wave_barrier();  // the list and the tile are rewritten by the next tile
    }
}

// Query-II of key i of a list: one uint64 per key, or (low, high) pairs.
template <bool kWide>
__device__ __forceinline__ uint64_t query_list(const FilterArgs &F, const uint64_t *keys,
                                               uint64_t i) {
    return kWide ? query_key_wide(F, Key128{keys[2 * i], keys[2 * i + 1]})
                 : query_key(F, keys[i]);
}

// keys used: keys[b .. e), b = *key_base (0 when null), e = min(*n_keys, limit)
__device__ __forceinline__ uint64_t key_count(const uint64_t *n_keys, const uint64_t *key_base,
                                              uint64_t limit, uint64_t &b) {
    b = key_base ? *key_base : 0;
    const uint64_t e = *n_keys < limit ? *n_keys : limit;
    return e > b ? e - b : 0;
}

template <bool kWide>
__global__ void __launch_bounds__(kWG) k_classify_mark(FilterArgs F, const uint64_t *__restrict__ keys,
                                                       const uint64_t *__restrict__ n_keys,
                                                       const uint64_t *__restrict__ key_base,
                                                       uint64_t cap, uint32_t tau,
                                                       uint64_t *__restrict__ tmask,
                                                       uint32_t *__restrict__ tile_trust) {
    __shared__ uint32_t s_cnt[kWG / 64];
    uint64_t b;
    const uint64_t n = key_count(n_keys, key_base, cap, b);
    keys += kWide ? 2 * b : b;
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
            trust = query_list<kWide>(F, keys, i) > (uint64_t)tau;
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

template <bool kWide>
__global__ void __launch_bounds__(kWG) k_classify_scatter(const uint64_t *__restrict__ keys,
                                                          const uint64_t *__restrict__ n_keys,
                                                          const uint64_t *__restrict__ key_base,
                                                          uint64_t cap,
                                                          const uint64_t *__restrict__ tmask,
                                                          const uint64_t *__restrict__ tile_off,
                                                          uint64_t *__restrict__ trust,
                                                          uint64_t *__restrict__ err,
                                                          uint64_t cap_out) {
    uint64_t b;
    const uint64_t n = key_count(n_keys, key_base, cap, b);
    keys += kWide ? 2 * b : b;
    const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
    if (tile0 >= n)
        return;
    auto copy = [&](uint64_t *out, uint64_t at, uint64_t i) {
        if (kWide) {
            out[2 * at] = keys[2 * i];
            out[2 * at + 1] = keys[2 * i + 1];
        } else {
            out[at] = keys[i];
        }
    };
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
        if ((word >> lane) & 1ull) {
            if (t_idx < cap_out)
                copy(trust, t_idx, i);
        } else if (i - t_idx < cap_out) {
            copy(err, i - t_idx, i);
        }
    }
}

__global__ void k_finish_classify(const uint64_t *__restrict__ n_keys,
                                  const uint64_t *__restrict__ key_base, uint64_t cap,
                                  const uint64_t *__restrict__ totals,
                                  uint64_t *__restrict__ n_trust, uint64_t *__restrict__ n_err,
                                  uint64_t cap_out, uint32_t *__restrict__ status) {
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    uint64_t b;
    const uint64_t n = key_count(n_keys, key_base, cap, b);
    *n_trust = totals[0];
    *n_err = n - totals[0];
    if (status && (totals[0] > cap_out || n - totals[0] > cap_out))
        atomicOr(status, kStatusRange);
}

template <bool kWide>
__global__ void k_query(FilterArgs F, const uint64_t *__restrict__ keys, uint64_t n,
                        uint32_t *__restrict__ freq) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        freq[i] = (uint32_t)query_list<kWide>(F, keys, i);
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

// The valid-window bitmap of K-base windows (valid_word), one mask word per
// thread.  Only the words of the call's tiles are written (n_out), so that a
// read set inside a larger buffer leaves its neighbours' words alone; the
// bin passes read no word past them.
__global__ void __launch_bounds__(256) k_valid_windows(const uint32_t *__restrict__ inv,
                                                       const uint32_t *__restrict__ rs,
                                                       uint64_t n_words, uint64_t n_out,
                                                       uint64_t n_bases, uint32_t K,
                                                       uint32_t *__restrict__ valid) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += stride)
        valid[i] = valid_word(inv, rs, n_words, i, K, n_bases);
}

hipError_t launch_valid_windows(uint64_t n_bases, uint32_t k, const Workspace &W, hipStream_t s,
                                Profiler *P) {
    const uint64_t n_mask = mask_words(n_bases);
    const uint64_t n_out = tiles(n_bases) * (kTile / 32);
    if (P)
        P->begin(kPhValid, s);
    hipLaunchKernelGGL(k_valid_windows, dim3(grid_for(n_out, 256)), dim3(256), 0, s,
                       (const uint32_t *)W.inv, (const uint32_t *)W.rs, n_mask, n_out, n_bases,
                       k, W.valid);
    if (P)
        P->end(s);
    return hipGetLastError();
}

hipError_t launch_ingest(const uint8_t *reads, uint64_t n_bases, const uint64_t *offsets,
                         uint64_t n_reads, const Workspace &W, hipStream_t s, Profiler *P) {
    uint64_t n_mask = mask_words(n_bases);
    if (P)
        P->begin(kPhIngest, s);
    // k_ingest also clears the read-start words and the flag bytes of every
    // tile of the call (n_mask * 32 positions cover them)
    int aligned = ((uintptr_t)reads & 15u) == 0;
    hipLaunchKernelGGL(k_ingest, dim3(grid_for(n_mask, 256)), dim3(256), 0, s, reads, n_bases,
                       W.codes, W.inv, W.rs, W.flags8, n_mask, tiles(n_bases) * (kTile / 32),
                       aligned);
    hipError_t e = hipGetLastError();
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
    return launch(P, kPhResolve, k_resolve, grid, block, s, F, R, c0, c1, W.flags8);
}

hipError_t launch_tile_count(const ReadsArgs &R, const Workspace &W, uint64_t n_tiles,
                             hipStream_t s) {
    const dim3 grid((unsigned)(n_tiles < (uint64_t)kTileGrid ? n_tiles : kTileGrid));
    hipLaunchKernelGGL(k_tile_count, grid, dim3(kWG), 0, s, R, (const uint8_t *)W.flags8, n_tiles,
                       0, W.tile_a, W.tile_b, W.tile_c);
    return hipGetLastError();
}

hipError_t launch_distinct(const ReadsArgs &R, const Workspace &W, uint64_t *distinct,
                           uint64_t cap_d, uint64_t *n_distinct, uint64_t *n_windows,
                           uint64_t *trust, uint64_t *n_trust, uint64_t *err, uint64_t *n_err,
                           uint64_t cap_te, uint32_t *status, bool windows_counted,
                           hipStream_t s, Profiler *P) {
    const uint64_t n_tiles = tiles(R.n_bases);
    const bool split = trust != nullptr;
    const dim3 grid((unsigned)(n_tiles < (uint64_t)kTileGrid ? n_tiles : kTileGrid));
    hipError_t e = launch(P, kPhTileCount, k_tile_count, grid, dim3(kWG), s, R,
                          (const uint8_t *)W.flags8, n_tiles, windows_counted ? 0 : 1, W.tile_a,
                          W.tile_b, W.tile_c);
    if (P)
        P->begin(kPhScan, s);
    if (e == hipSuccess)
        e = scan_u32_u64(W.tile_a, W.off_a, n_tiles, n_distinct, W.totals + 0, W.partial64, s);
    if (e == hipSuccess && split)
        e = scan_u32_u64(W.tile_b, W.off_b, n_tiles, nullptr, W.totals + 1, W.partial64, s);
    if (e == hipSuccess && !windows_counted)
        e = scan_u32_u64(W.tile_c, W.off_c, n_tiles, nullptr, W.totals + 2, W.partial64, s);
    if (e == hipSuccess) {  // the call's first distinct index, before k_finish_insert moves it
        hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, s, (const uint64_t *)n_distinct,
                           W.totals + 3);
        e = hipGetLastError();
    }
    if (P)
        P->end(s);
    if (e == hipSuccess && R.k > 32)
        e = launch(P, kPhScatter, k_compact<true>, grid, dim3(kWG), s, R,
                   (const uint8_t *)W.flags8, n_tiles, (const uint64_t *)W.off_a,
                   (const uint64_t *)W.off_b, (const uint64_t *)(W.totals + 3), distinct, cap_d,
                   trust, err, cap_te, split ? 1 : 0);
    else if (e == hipSuccess)
        e = launch(P, kPhScatter, k_compact<false>, grid, dim3(kWG), s, R,
                   (const uint8_t *)W.flags8, n_tiles, (const uint64_t *)W.off_a,
                   (const uint64_t *)W.off_b, (const uint64_t *)(W.totals + 3), distinct, cap_d,
                   trust, err, cap_te, split ? 1 : 0);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_finish_insert, dim3(1), dim3(64), 0, s, n_distinct, n_windows,
                           split ? n_trust : (uint64_t *)nullptr, n_err,
                           (const uint64_t *)W.totals, windows_counted ? 1 : 0, cap_d, cap_te,
                           status);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_classify(const FilterArgs &F, const uint64_t *keys, const uint64_t *n_keys,
                           const uint64_t *key_base, uint64_t grid_cap, uint64_t cap,
                           uint32_t tau, uint64_t *trust, uint64_t *n_trust, uint64_t *err,
                           uint64_t *n_err, uint64_t cap_out, uint32_t *status,
                           const Workspace &W, hipStream_t s, Profiler *P, bool wide) {
    // `cap` bounds the key buffer (keys[.. cap)); grid_cap >= the number of
    // keys classified sizes the grid
    uint64_t n_tiles = (grid_cap + kTile - 1) / kTile;
    if (n_tiles == 0)
        n_tiles = 1;
    hipError_t e = wide ? launch(P, kPhClassifyMark, k_classify_mark<true>,
                                 dim3((unsigned)n_tiles), dim3(kWG), s, F, keys, n_keys, key_base,
                                 cap, tau, W.tmask, W.tile_a)
                        : launch(P, kPhClassifyMark, k_classify_mark<false>,
                                 dim3((unsigned)n_tiles), dim3(kWG), s, F, keys, n_keys, key_base,
                                 cap, tau, W.tmask, W.tile_a);
    if (P)
        P->begin(kPhScan, s);
    if (e == hipSuccess)
        e = scan_u32_u64(W.tile_a, W.off_a, n_tiles, nullptr, W.totals + 4, W.partial64, s);
    if (P)
        P->end(s);
    if (e == hipSuccess && wide)
        e = launch(P, kPhClassifyScatter, k_classify_scatter<true>, dim3((unsigned)n_tiles),
                   dim3(kWG), s, keys, n_keys, key_base, cap, (const uint64_t *)W.tmask,
                   (const uint64_t *)W.off_a, trust, err, cap_out);
    else if (e == hipSuccess)
        e = launch(P, kPhClassifyScatter, k_classify_scatter<false>, dim3((unsigned)n_tiles),
                   dim3(kWG), s, keys, n_keys, key_base, cap, (const uint64_t *)W.tmask,
                   (const uint64_t *)W.off_a, trust, err, cap_out);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_finish_classify, dim3(1), dim3(64), 0, s, n_keys, key_base, cap,
                           (const uint64_t *)(W.totals + 4), n_trust, n_err, cap_out, status);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_classify_flags(const FilterArgs &F, const ReadsArgs &R, const Workspace &W,
                                 uint64_t n_positions, uint32_t tau, hipStream_t s,
                                 Profiler *P) {
    const uint64_t n_tiles = tiles(n_positions);
    if (n_tiles == 0)
        return hipSuccess;
    const dim3 grid((unsigned)(n_tiles < (uint64_t)kTileGrid ? n_tiles : kTileGrid));
    return R.k > 32 ? launch(P, kPhClassifyMark, k_classify_flags<true>, grid, dim3(kWG), s, F, R,
                             W.flags8, n_tiles, tau)
                    : launch(P, kPhClassifyMark, k_classify_flags<false>, grid, dim3(kWG), s, F,
                             R, W.flags8, n_tiles, tau);
}

hipError_t launch_query(const FilterArgs &F, const uint64_t *keys, uint64_t n, uint32_t *freq,
                        hipStream_t s, Profiler *P, bool wide) {
    if (n == 0)
        return hipSuccess;
    return wide ? launch(P, kPhQuery, k_query<true>, dim3(grid_for(n, 256)), dim3(256), s, F, keys,
                         n, freq)
                : launch(P, kPhQuery, k_query<false>, dim3(grid_for(n, 256)), dim3(256), s, F,
                         keys, n, freq);
}

}  // namespace kc
