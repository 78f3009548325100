// Device-side building blocks of the gfx950 KmerCo kernels.
//
// Packed read layout produced by the ingest kernel (one per insert call):
//   codes[m]  uint32, bases 16m .. 16m+15 as 2-bit codes, base 16m in bits
//             31..30 (A=0 C=1 G=2 T=3; invalid bases stored as 0)
//   inv[b]    uint32, bit q%32 of word q/32 set when base q is not A/C/G/T;
//             positions past the end of the reads are set (invalid)
//   rs[b]     uint32, bit set at every read start offset
// A window of K bases starting at p is valid iff bases p..p+K-1 are valid
// and no read starts at p+1..p+K-1 (Algorithm 1 visits windows inside one
// read; windows holding a non-ACGT byte are skipped).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kc {

constexpr uint32_t kIdle = 0xFFFFFFFFu;  // first-seen scratch entry with no claimant

// Filter parameters handed to every kernel by value.
struct FilterArgs {
    uint64_t *words;      // X*Y cells
    uint32_t *aux;        // X*Y*eta first-seen entries (kIdle when unused)
    uint64_t X, Y;
    uint64_t mX, mY;      // floor((2^64-1)/X), floor((2^64-1)/Y)
    uint64_t mEta;        // floor((2^64-1)/eta)
    uint32_t eta;
    uint32_t alpha;
    uint32_t k_h;
    uint32_t eta_pow2;    // eta is a power of two (then l = h & (eta-1))
    uint32_t small_dims;  // X, Y <= kSmallDivisor (then mod_small applies)
    uint64_t field_max;   // 2^alpha - 1
};

// Packed reads of one insert call.
struct ReadsArgs {
    const uint32_t *codes;
    const uint32_t *inv;
    const uint32_t *rs;
    uint64_t n_bases;
    uint32_t k;
    const uint32_t *valid;  // valid-window bitmap of k (valid_word), where computed
};

// ----------------------------------------------------------------------------
// MurmurHash3_x86_32 of an 8-byte little-endian key, split so that the two
// block mixes (which do not depend on the seed) are shared between seeds.
// ----------------------------------------------------------------------------
// The arithmetic helpers below are __host__ __device__ so that host-side
// tests can check them on the CPU; only two primitives differ by side.
#define KC_HD __host__ __device__ __forceinline__

KC_HD uint32_t rotl32(uint32_t x, uint32_t r) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(x, x, 32u - r);
#else
    return (x << r) | (x >> (32u - r));
#endif
}

KC_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

KC_HD uint32_t mm3_block(uint32_t k) {
    k *= 0xcc9e2d51u;
    k = rotl32(k, 15);
    return k * 0x1b873593u;
}

KC_HD uint32_t mm3_seeded(uint32_t b0, uint32_t b1, uint32_t seed) {
    uint32_t h = seed ^ b0;
    h = rotl32(h, 13) * 5u + 0xe6546b64u;
    h ^= b1;
    h = rotl32(h, 13) * 5u + 0xe6546b64u;
    h ^= 8u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// H_a(key) for a = 1..8: seeds 2a-2 (high word) and 2a-1 (low word).
KC_HD uint64_t hash_a(uint32_t b0, uint32_t b1, uint32_t a) {
    uint32_t hi = mm3_seeded(b0, b1, 2u * a - 2u);
    uint32_t lo = mm3_seeded(b0, b1, 2u * a - 1u);
    return ((uint64_t)hi << 32) | lo;
}

KC_HD void key_blocks(uint64_t key, uint32_t &b0, uint32_t &b1) {
    b0 = mm3_block((uint32_t)key);
    b1 = mm3_block((uint32_t)(key >> 32));
}

// ----------------------------------------------------------------------------
// Exact h mod d with a precomputed reciprocal m = floor((2^64-1)/d):
// q = floor(h*m / 2^64) is floor(h/d) or one less, so one correction step
// gives the exact remainder for every 64-bit h and every d >= 1.
// ----------------------------------------------------------------------------
KC_HD uint64_t mod_by(uint64_t h, uint64_t d, uint64_t m) {
    uint64_t q = mulhi64(h, m);
    uint64_t r = h - q * d;
    return r >= d ? r - d : r;
}

// The same remainder for divisors d <= kSmallDivisor, in 32-bit arithmetic.
// Dropping the low partial product h_lo*m_lo from the 128-bit product h*m
// lowers the quotient estimate by at most one more, so q is floor(h/d),
// one or two less, and r = h - q*d lies in [0, 3d).  3d < 2^32, so r is
// exact from the low words alone (r = h_lo - q_lo*d mod 2^32), and only the
// low word of q is needed: the low word of h_hi*m_hi plus bits 32..63 of
// the middle products' sum (its carry out of bit 63 only changes q's high
// word).  Two conditional subtractions finish; min(r, r - d) is one, since
// r - d wraps above r exactly when r < d.
constexpr uint64_t kSmallDivisor = 0x55555555ull;  // floor((2^32 - 1) / 3)

KC_HD uint32_t mod_small(uint64_t h, uint32_t d, uint64_t m) {
    const uint32_t hl = (uint32_t)h, hh = (uint32_t)(h >> 32);
    const uint32_t ml = (uint32_t)m, mh = (uint32_t)(m >> 32);
    const uint64_t mid = (uint64_t)hh * ml + (uint64_t)hl * mh;
    const uint32_t q = hh * mh + (uint32_t)(mid >> 32);
    uint32_t r = hl - q * d;
    uint32_t t = r - d;
    r = t < r ? t : r;
    t = r - d;
    return t < r ? t : r;
}

// Counter index (word * eta + l) of hash value h.
KC_HD void slot_of(const FilterArgs &F, uint64_t h, uint64_t &word,
                                        uint32_t &l) {
    l = F.eta_pow2 ? (uint32_t)(h & (uint64_t)(F.eta - 1)) : (uint32_t)mod_by(h, F.eta, F.mEta);
    if (F.small_dims) {
        const uint32_t i = mod_small(h, (uint32_t)F.X, F.mX);
        const uint32_t j = mod_small(h, (uint32_t)F.Y, F.mY);
        word = (uint64_t)i * (uint32_t)F.Y + j;
        return;
    }
    uint64_t i = mod_by(h, F.X, F.mX);
    uint64_t j = mod_by(h, F.Y, F.mY);
    word = i * F.Y + j;
}

// ----------------------------------------------------------------------------
// Base codes: A=0x41 C=0x43 G=0x47 T=0x54 -> 0 1 2 3; any other byte invalid
// ----------------------------------------------------------------------------
KC_HD uint32_t base_code(uint32_t b) { return ((b >> 1) ^ (b >> 2)) & 3u; }

KC_HD bool base_valid(uint32_t b, uint32_t code) {
    return b == ((0x54474341u >> (8u * code)) & 0xFFu);
}

// Four bases at once: x holds 4 bytes (base i in bits 8i..8i+7).  Returns
// their codes packed in 8 bits (base 0 in bits 7..6, an invalid base as 0)
// and sets bit i of valid4 when base i is A, C, G or T.  Per byte: the code
// as base_code; the expected letter of that code picked from "ACGT" (one
// byte permute on the device); an exact zero-byte test of x ^ expected; the
// byte flags and the 2-bit codes gathered by multiplications whose partial
// products land on distinct bits (no carries).
KC_HD uint32_t codes4(uint32_t x, uint32_t &valid4) {
    const uint32_t c4 = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t e = __builtin_amdgcn_perm(0u, 0x54474341u, c4);
#else
    uint32_t e = 0;
    for (int i = 0; i < 4; i++)
        e |= ((0x54474341u >> (8 * ((c4 >> (8 * i)) & 3u))) & 0xFFu) << (8 * i);
#endif
    const uint32_t d = x ^ e;
    const uint32_t z = ~(((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d | 0x7F7F7F7Fu);  // 0x80: equal
    valid4 = (((z >> 7) * 0x00204081u) >> 21) & 0xFu;
    const uint32_t c = c4 & ((z >> 6) | (z >> 7));
    return (c * 0x40100401u) >> 24;
}

// ----------------------------------------------------------------------------
// Window extraction from the packed layout
// ----------------------------------------------------------------------------

// The 16 2-bit groups of x in reverse order, each code complemented.  A
// full bit reversal (one instruction) reverses the group order but also
// swaps the two bits inside every group; a shift each way and a bitwise
// select swap them back, and complementing every bit complements every code
// (c ^ 3 == ~c on 2 bits).  The select and the complement are one
// three-input bitwise instruction on gfx950.
KC_HD uint32_t revcomp16(uint32_t x) {
    const uint32_t y = __builtin_bitreverse32(x);
#if defined(__HIP_DEVICE_COMPILE__)
    // bit i of the table is the result for (M, a, b) = bits of i (M high):
    // ~(M ? a : b)
    return __builtin_amdgcn_bitop3_b32(0x55555555u, y >> 1, y << 1, 0x35);
#else
    return ~(((y >> 1) & 0x55555555u) | ((y << 1) & 0xAAAAAAAAu));
#endif
}

// 2-bit reverse complement of a K-base key (K <= 32): the reverse
// complement of all 32 groups, then the 32-K groups that came from the
// unused high end dropped.
KC_HD uint64_t revcomp_key(uint64_t x, uint32_t K) {
    const uint64_t r = ((uint64_t)revcomp16((uint32_t)x) << 32) | revcomp16((uint32_t)(x >> 32));
    return r >> (64u - 2u * K);
}

// Forward key of the K-base window starting at p (first base most
// significant).  Needs codes[p/16 + 2] to exist.  The 64 bits from base
// p % 16 of codes[p/16] on are the high word of (w0:w1) << s and the low word
// of (w1:w2) >> (32 - s), s = 2 (p % 16); both shifts stay below 64.
KC_HD uint64_t window_key(const uint32_t *__restrict__ codes, uint64_t p,
                                               uint32_t K) {
    const uint64_t m = p >> 4;
    const uint32_t s = 2u * (uint32_t)(p & 15u);
    const uint32_t w0 = codes[m], w1 = codes[m + 1], w2 = codes[m + 2];
    const uint32_t top_hi = (uint32_t)(((((uint64_t)w0 << 32) | w1) << s) >> 32);
    const uint32_t top_lo = (uint32_t)((((uint64_t)w1 << 32) | w2) >> (32u - s));
    return (((uint64_t)top_hi << 32) | top_lo) >> (64u - 2u * K);
}

// Window validity (see the layout note above).  Needs inv/rs[p/32 + 1].
KC_HD bool window_valid(const ReadsArgs &R, uint64_t p) {
    if (p + R.k > R.n_bases)
        return false;
    uint64_t b = p >> 5;
    uint32_t o = (uint32_t)(p & 31u);
    uint64_t kmask = (R.k >= 64u) ? ~0ull : ((1ull << R.k) - 1ull);
    uint64_t iv = ((((uint64_t)R.inv[b + 1]) << 32) | R.inv[b]) >> o;
    uint64_t st = ((((uint64_t)R.rs[b + 1]) << 32) | R.rs[b]) >> o;
    return ((iv & kmask) | (st & kmask & ~1ull)) == 0;
}

// OR of the L consecutive bits of x starting at every bit (L = 0..64): the
// runs are doubled up to the largest power of two c <= L, then two runs of
// c that overlap cover L.
KC_HD unsigned __int128 window_or(unsigned __int128 x, uint32_t L) {
    if (L == 0)
        return 0;
    uint32_t c = 1;
    while (2u * c <= L) {
        x |= x >> c;
        c *= 2u;
    }
    return x | (x >> (L - c));
}

// Bits of the valid-window bitmap for mask word i (positions 32 i + j):
// bit j is set when the window of K bases there is valid (as window_valid:
// inside the data, no invalid base, no read starting after its first base).
// inv, rs: the mask words, n_words of them.
KC_HD uint32_t valid_word(const uint32_t *inv, const uint32_t *rs, uint64_t n_words, uint64_t i,
                          uint32_t K, uint64_t n_bases) {
    const uint64_t p0 = i * 32u;
    if (p0 + K > n_bases)
        return 0;
    unsigned __int128 xi = 0, xr = 0;
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (i + d < n_words) {
            xi |= (unsigned __int128)inv[i + d] << (32 * d);
            xr |= (unsigned __int128)rs[i + d] << (32 * d);
        }
    const unsigned __int128 bad = window_or(xi, K) | window_or(xr >> 1, K - 1u);
    uint32_t v = ~(uint32_t)bad;
    const uint64_t last = n_bases - K - p0;  // windows j <= last end inside the data
    if (last < 31u)
        v &= (2u << last) - 1u;
    return v;
}

// Canonical key and its H_1 value (Sec. 2.3: the strand with the smaller
// hash; a tie keeps the reverse complement), plus the key's MM3 blocks for
// the remaining hash functions.
struct Canon {
    uint64_t key;
    uint64_t h1;
    uint32_t b0, b1;
};

KC_HD Canon canonical(uint64_t fwd, uint32_t K) {
    uint64_t rc = revcomp_key(fwd, K);
    uint32_t f0, f1, r0, r1;
    key_blocks(fwd, f0, f1);
    key_blocks(rc, r0, r1);
    uint64_t hf = hash_a(f0, f1, 1);
    uint64_t hr = hash_a(r0, r1, 1);
    Canon c;
    if (hf < hr) {
        c.key = fwd; c.h1 = hf; c.b0 = f0; c.b1 = f1;
    } else {
        c.key = rc; c.h1 = hr; c.b0 = r0; c.b1 = r1;
    }
    return c;
}

// Same choice with one MurmurHash3 call fewer: the high words (seed 0) of
// both strands decide unless they are equal; only the chosen strand's low
// word (seed 1) is then needed.  Identical result to canonical().
KC_HD Canon canonical_fast(uint64_t fwd, uint32_t K) {
    uint64_t rc = revcomp_key(fwd, K);
    uint32_t f0, f1, r0, r1;
    key_blocks(fwd, f0, f1);
    key_blocks(rc, r0, r1);
    uint32_t hf = mm3_seeded(f0, f1, 0u);
    uint32_t hr = mm3_seeded(r0, r1, 0u);
    Canon c;
    if (hf != hr) {
        bool take_fwd = hf < hr;
        c.key = take_fwd ? fwd : rc;
        c.b0 = take_fwd ? f0 : r0;
        c.b1 = take_fwd ? f1 : r1;
        c.h1 = ((uint64_t)(take_fwd ? hf : hr) << 32) | mm3_seeded(c.b0, c.b1, 1u);
    } else {
        uint64_t Hf = ((uint64_t)hf << 32) | mm3_seeded(f0, f1, 1u);
        uint64_t Hr = ((uint64_t)hr << 32) | mm3_seeded(r0, r1, 1u);
        bool take_fwd = Hf < Hr;
        c.key = take_fwd ? fwd : rc;
        c.b0 = take_fwd ? f0 : r0;
        c.b1 = take_fwd ? f1 : r1;
        c.h1 = take_fwd ? Hf : Hr;
    }
    return c;
}

// ----------------------------------------------------------------------------
// Wavefront-level window extraction.  A wavefront handles 64 consecutive
// positions pb .. pb+63 (pb a multiple of 64).  The packed words they need
// (6 code words, 3 invalid-base words, 3 read-start words) are the same for
// every lane, so they are loaded once per wavefront (scalar loads when pb is
// wave-uniform) and each lane selects its own.
// ----------------------------------------------------------------------------
struct WaveWords {
    uint32_t c[6];
    uint32_t iv[3];
    uint32_t st[3];
};

KC_HD void wave_load(const ReadsArgs &R, uint64_t pb, WaveWords &w) {
    const uint32_t *cp = R.codes + (pb >> 4);
    const uint32_t *ip = R.inv + (pb >> 5);
    const uint32_t *sp = R.rs + (pb >> 5);
#pragma unroll
    for (int i = 0; i < 6; i++)
        w.c[i] = cp[i];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        w.iv[i] = ip[i];
        w.st[i] = sp[i];
    }
}

// Valid-window bits of positions pb .. pb + 63 (pb a multiple of 64).  On
// the device the two words are read through a constant-address-space view
// (they are wavefront-uniform and not written while a kernel reads them),
// so that they come by a scalar load and stay in scalar registers.
KC_HD uint64_t wave_valid(const ReadsArgs &R, uint64_t pb) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) uint32_t ConstWord;
    ConstWord *vp = (ConstWord *)(R.valid + (pb >> 5));
#else
    const uint32_t *vp = R.valid + (pb >> 5);
#endif
    return ((uint64_t)vp[1] << 32) | vp[0];
}

KC_HD uint32_t pick4(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t i) {
    uint32_t lo = (i & 1u) ? a1 : a0;
    uint32_t hi = (i & 1u) ? a3 : a2;
    return (i & 2u) ? hi : lo;
}

// low 32 bits of (hi:lo) >> s, s in [0, 31]
KC_HD uint32_t funnel32(uint32_t hi, uint32_t lo, uint32_t s) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, s);
#else
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
#endif
}

// Forward key of the window at position pb + lane (lane < 64, K <= 32)
// from the wave's code words.
KC_HD uint64_t wave_key(const WaveWords &w, uint32_t lane, uint32_t K) {
    const uint32_t mo = lane >> 4;
    const uint32_t w0 = pick4(w.c[0], w.c[1], w.c[2], w.c[3], mo);
    const uint32_t w1 = pick4(w.c[1], w.c[2], w.c[3], w.c[4], mo);
    const uint32_t w2 = pick4(w.c[2], w.c[3], w.c[4], w.c[5], mo);
    const uint32_t s = 2u * (lane & 15u);
    // 64 bits starting at base (lane & 15) of w0: (w0:w1:w2) << s, as in
    // window_key
    const uint32_t top_hi = (uint32_t)(((((uint64_t)w0 << 32) | w1) << s) >> 32);
    const uint32_t top_lo = (uint32_t)((((uint64_t)w1 << 32) | w2) >> (32u - s));
    return (((uint64_t)top_hi << 32) | top_lo) >> (64u - 2u * K);
}

// Window at position pb + lane (lane < 64): validity and forward key.
KC_HD bool wave_window(const WaveWords &w, uint64_t pb, uint32_t lane, uint32_t K,
                       uint64_t n_bases, uint64_t &fwd) {
    fwd = wave_key(w, lane, K);
    // 32 mask bits starting at the window's first base
    const bool upper = (lane & 32u) != 0;
    const uint32_t o = lane & 31u;
    const uint32_t iv = funnel32(upper ? w.iv[2] : w.iv[1], upper ? w.iv[1] : w.iv[0], o);
    const uint32_t st = funnel32(upper ? w.st[2] : w.st[1], upper ? w.st[1] : w.st[0], o);
    const uint32_t kmask = K >= 32u ? 0xFFFFFFFFu : ((1u << K) - 1u);
    return (pb + lane + K <= n_bases) && ((iv & kmask) | (st & kmask & ~1u)) == 0;
}

// ----------------------------------------------------------------------------
// K-mers of 33..64 bases: the 2-bit key is a 128-bit integer (first base most
// significant), held as (lo, hi) and hashed as its 16 little-endian bytes,
// low word first.
// ----------------------------------------------------------------------------
struct Key128 {
    uint64_t lo, hi;
};

// (hi:lo) >> sh for 0 <= sh < 64
KC_HD Key128 shr128(uint64_t hi, uint64_t lo, uint32_t sh) {
    Key128 k;
    k.hi = hi >> sh;
    k.lo = sh ? ((lo >> sh) | (hi << (64u - sh))) : lo;
    return k;
}

// Reverse complement of a K-base key, 33 <= K <= 64: the 64 groups reversed
// and complemented (revcomp16 per 32-bit word, words in reverse order), the
// K groups that came from the key kept.
KC_HD Key128 revcomp_wide(Key128 x, uint32_t K) {
    const uint64_t hi = ((uint64_t)revcomp16((uint32_t)x.lo) << 32) |
                        revcomp16((uint32_t)(x.lo >> 32));
    const uint64_t lo = ((uint64_t)revcomp16((uint32_t)x.hi) << 32) |
                        revcomp16((uint32_t)(x.hi >> 32));
    return shr128(hi, lo, 128u - 2u * K);
}

// Forward key of the K-base window at p (33 <= K <= 64): the 128 bits from
// base p % 16 of codes[p/16] on, built from word pairs as in window_key, then
// right-aligned.  Needs codes[p/16 + 4] to exist.
KC_HD Key128 window_key_wide(const uint32_t *__restrict__ codes, uint64_t p, uint32_t K) {
    const uint64_t m = p >> 4;
    const uint32_t s = 2u * (uint32_t)(p & 15u);
    const uint32_t w0 = codes[m], w1 = codes[m + 1], w2 = codes[m + 2], w3 = codes[m + 3],
                   w4 = codes[m + 4];
    const uint64_t t0 = ((((((uint64_t)w0 << 32) | w1) << s) >> 32) << 32) |
                        (uint32_t)((((uint64_t)w1 << 32) | w2) >> (32u - s));
    const uint64_t t1 = ((((((uint64_t)w2 << 32) | w3) << s) >> 32) << 32) |
                        (uint32_t)((((uint64_t)w3 << 32) | w4) >> (32u - s));
    return shr128(t0, t1, 128u - 2u * K);
}

// MurmurHash3_x86_32 of a 16-byte key from its four block mixes.
KC_HD uint32_t mm3_seeded4(const uint32_t b[4], uint32_t seed) {
    uint32_t h = seed;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        h ^= b[i];
        h = rotl32(h, 13) * 5u + 0xe6546b64u;
    }
    h ^= 16u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

KC_HD void key_blocks_wide(Key128 k, uint32_t b[4]) {
    b[0] = mm3_block((uint32_t)k.lo);
    b[1] = mm3_block((uint32_t)(k.lo >> 32));
    b[2] = mm3_block((uint32_t)k.hi);
    b[3] = mm3_block((uint32_t)(k.hi >> 32));
}

KC_HD uint64_t hash_a_wide(const uint32_t b[4], uint32_t a) {
    return ((uint64_t)mm3_seeded4(b, 2u * a - 2u) << 32) | mm3_seeded4(b, 2u * a - 1u);
}

// Canonical 128-bit key and its H_1, as canonical_fast: the high words
// (seed 0) of both strands decide unless equal; a tie of the full H_1 keeps
// the reverse complement.
struct CanonWide {
    Key128 key;
    uint64_t h1;
    uint32_t b[4];
};

KC_HD CanonWide canonical_wide(Key128 fwd, uint32_t K) {
    const Key128 rc = revcomp_wide(fwd, K);
    uint32_t f[4], r[4];
    key_blocks_wide(fwd, f);
    key_blocks_wide(rc, r);
    const uint32_t hf = mm3_seeded4(f, 0u), hr = mm3_seeded4(r, 0u);
    bool take_fwd;
    uint64_t Hf = 0, Hr = 0;
    if (hf != hr) {
        take_fwd = hf < hr;
    } else {
        Hf = ((uint64_t)hf << 32) | mm3_seeded4(f, 1u);
        Hr = ((uint64_t)hr << 32) | mm3_seeded4(r, 1u);
        take_fwd = Hf < Hr;
    }
    CanonWide c;
    c.key = take_fwd ? fwd : rc;
#pragma unroll
    for (int i = 0; i < 4; i++)
        c.b[i] = take_fwd ? f[i] : r[i];
    c.h1 = hf != hr ? (((uint64_t)(take_fwd ? hf : hr) << 32) | mm3_seeded4(c.b, 1u))
                    : (take_fwd ? Hf : Hr);
    return c;
}

// Saturating increment of counter l of a cell (64-bit CAS loop).  Returns
// nothing; a saturated counter is left unchanged.
__device__ __forceinline__ void saturating_increment(uint64_t *cell, uint32_t shift,
                                                     uint64_t field_max) {
    const uint64_t fmask = field_max << shift;
    const uint64_t inc = 1ull << shift;
    uint64_t old = __hip_atomic_load(cell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((old & fmask) != fmask) {
        uint64_t assumed = old;
        old = atomicCAS((unsigned long long *)cell, (unsigned long long)assumed,
                        (unsigned long long)(assumed + inc));
        if (old == assumed)
            break;
    }
}

__device__ __forceinline__ uint64_t read_counter(const FilterArgs &F, uint64_t word, uint32_t l) {
    return (F.words[word] >> (F.alpha * l)) & F.field_max;
}

}  // namespace kc
