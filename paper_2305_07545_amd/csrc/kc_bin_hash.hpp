// The hashing pass of the binned insertion, shared by the single-set and the
// batched bin kernels: which windows are hashed, and the slot id each valid
// window yields for every hash function (Sec. 2.3: canonical k-mer, H_a,
// cell (h mod X, h mod Y), counter h mod eta).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc_device.hpp"
#include "kc_kernels.hpp"

namespace kc {

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;  // slot id of an invalid window
constexpr uint32_t kLocalBits = 14;        // a slot id: region << kLocalBits | local counter
constexpr uint32_t kWindowRing = 128;      // queued window positions per wavefront (< 64 + 64)

// The fast layout: one hash function, eta a power of two, X and Y below 2^24
// and X*Y at most 2^32 (countBFs up to 32 GB), so that the counter is the
// low bits of h, the cell index i*Y + j a 32-bit value from one 24-bit
// multiply-add, and the hash-function loop and the layout branches go.
inline bool fast_layout(const FilterArgs &F) {
    return F.k_h == 1 && F.eta_pow2 && F.X < (1ull << 24) && F.Y < (1ull << 24) &&
           F.X * F.Y <= (1ull << 32);
}

__device__ __forceinline__ uint32_t wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Forward key of the K-base window at 32-bit position q of codes (q % 16
// bases into word q / 16; needs words q/16 .. q/16 + 2), as window_key: the
// 64 bits from bit s = 2 (q % 16) of (w0:w1:w2) on are two funnel shifts
// right by 32 - s (alignbit takes the shift mod 32, so s = 0 selects the
// words themselves), then right-aligned.
__device__ __forceinline__ uint64_t window_key32(const uint32_t *__restrict__ codes, uint32_t q,
                                                 uint32_t K) {
    const uint32_t m = q >> 4;
    const uint32_t s = 2u * (q & 15u);
    const uint32_t w0 = codes[m], w1 = codes[m + 1], w2 = codes[m + 2];
    const uint32_t hi = s ? __builtin_amdgcn_alignbit(w0, w1, 32u - s) : w0;
    const uint32_t lo = s ? __builtin_amdgcn_alignbit(w1, w2, 32u - s) : w1;
    return (((uint64_t)hi << 32) | lo) >> (64u - 2u * K);
}

// The counter of hash value h, as (region r, local id) for regions of
// 2^shift cells: r = cell >> shift, local = l << shift | cell offset.
template <bool kFast>
__device__ __forceinline__ void counter_of(const FilterArgs &F, uint64_t h, uint32_t shift,
                                           uint32_t &r, uint32_t &local) {
    if (kFast) {
        const uint32_t l = (uint32_t)h & (F.eta - 1u);
        const uint32_t cell = __umul24(mod_small(h, (uint32_t)F.X, F.mX), (uint32_t)F.Y) +
                              mod_small(h, (uint32_t)F.Y, F.mY);
        r = cell >> shift;
        local = (l << shift) | (cell & ((1u << shift) - 1u));
    } else {
        uint64_t cell;
        uint32_t l;
        slot_of(F, h, cell, l);
        r = (uint32_t)(cell >> shift);
        local = (l << shift) | (uint32_t)(cell & ((1ull << shift) - 1ull));
    }
}

// The counters of the window at position q of codes (K bases, 128-bit keys
// when kWide): emit(a, r, local) for hash functions a = 1 .. k_h.
template <bool kFast, bool kWide, typename Emit>
__device__ __forceinline__ void window_counters(const FilterArgs &F,
                                                const uint32_t *__restrict__ codes, uint32_t q,
                                                uint32_t K, uint32_t shift, Emit emit) {
    const uint32_t k_h = kFast ? 1u : F.k_h;
    uint32_t r, local;
    if (kWide) {
        const CanonWide c = canonical_wide(window_key_wide(codes, q, K), K);
        for (uint32_t a = 1; a <= k_h; a++) {
            counter_of<kFast>(F, a == 1 ? c.h1 : hash_a_wide(c.b, a), shift, r, local);
            emit(a, r, local);
        }
    } else {
        const Canon c = canonical_fast(window_key32(codes, q, K), K);
        for (uint32_t a = 1; a <= k_h; a++) {
            counter_of<kFast>(F, a == 1 ? c.h1 : hash_a(c.b0, c.b1, a), shift, r, local);
            emit(a, r, local);
        }
    }
}

// The windows of positions [g0, g1) (g0 a multiple of 64), 64 positions
// per wavefront at a time (wave w takes g0 + 64 w, then every kBinWG
// positions).  Validity comes from the valid-window bitmap (R.valid, one
// 64-bit word per wavefront step); skip(q) runs for every invalid position,
// and valid positions are queued, as 32-bit offsets q = p - base, in the
// wavefront's LDS ring (kWindowRing entries), so that hash(q) always runs
// with all 64 lanes on valid windows, but for the last call.  No lane hashes
// an invalid window (the last K-1 positions of every read, windows over
// 'N').  Returns the wavefront's number of valid windows (uniform).
template <typename Skip, typename Hash>
__device__ __forceinline__ uint32_t walk_windows(const ReadsArgs &R, uint64_t g0, uint64_t g1,
                                                 uint64_t base, uint32_t *ring, Skip skip,
                                                 Hash hash) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n = (uint32_t)(g1 - g0);       // a tile is < 2^32 positions
    const uint32_t q0 = (uint32_t)(g0 - base) + lane;
    uint32_t head = 0, queued = 0, n_valid = 0;  // wavefront-uniform
    for (uint32_t o = 64u * wave_id(); o < n; o += kBinWG) {
        const uint64_t m_in = n - o < 64u ? (1ull << (n - o)) - 1ull : ~0ull;
        const uint64_t m = wave_valid(R, g0 + o) & m_in;
        const uint32_t q = q0 + o;
        // the lane's bit of a uniform mask, taken as the execution mask
        if (__builtin_amdgcn_inverse_ballot_w64(m_in & ~m))
            skip(q);
        if (__builtin_amdgcn_inverse_ballot_w64(m)) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            ring[(head + queued + rank) & (kWindowRing - 1u)] = q;
        }
        const uint32_t c = (uint32_t)__popcll(m);
        queued += c;
        n_valid += c;
        __builtin_amdgcn_wave_barrier();
        if (queued >= 64u) {
            const uint32_t qq = ring[(head + lane) & (kWindowRing - 1u)];
            __builtin_amdgcn_wave_barrier();
            head = (head + 64u) & (kWindowRing - 1u);
            queued -= 64u;
            hash(qq);
        }
    }
    if (lane < queued)
        hash(ring[(head + lane) & (kWindowRing - 1u)]);
    return n_valid;
}

}  // namespace kc
