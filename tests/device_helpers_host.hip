// Host build of the GPU path's arithmetic helpers, for CPU tests (no kernel
// is launched).  Exposes them through a small C interface for ctypes.
#include <stdint.h>

#include "kc_device.hpp"

extern "C" {

uint64_t kch_mod_by(uint64_t h, uint64_t d) { return kc::mod_by(h, d, UINT64_MAX / d); }

uint64_t kch_mod_small(uint64_t h, uint32_t d) {
    return kc::mod_small(h, d, UINT64_MAX / d);
}

// Counts the h (n pseudo-random values, half of them within 2 of a multiple
// of d) where mod_small differs from h % d.  The generator is splitmix64.
uint64_t kch_mod_small_mismatches(uint32_t d, uint64_t n, uint64_t seed) {
    const uint64_t m = UINT64_MAX / d;
    uint64_t x = seed, bad = 0;
    for (uint64_t i = 0; i < n; i++) {
        x += 0x9e3779b97f4a7c15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        uint64_t h = z;
        if (i & 1)
            h = (z % (UINT64_MAX / d)) * d + (i >> 1) % 5 - 2;
        bad += kc::mod_small(h, d, m) != h % d;
    }
    return bad;
}

uint32_t kch_codes4(uint32_t x, uint32_t *valid4) { return kc::codes4(x, *valid4); }

uint64_t kch_revcomp(uint64_t x, uint32_t K) { return kc::revcomp_key(x, K); }

uint64_t kch_window_key(const uint32_t *codes, uint64_t p, uint32_t K) {
    return kc::window_key(codes, p, K);
}

int kch_window_valid(const uint32_t *codes, const uint32_t *inv, const uint32_t *rs,
                     uint64_t n_bases, uint32_t k, uint64_t p) {
    kc::ReadsArgs R{codes, inv, rs, n_bases, k};
    return kc::window_valid(R, p) ? 1 : 0;
}

uint32_t kch_valid_word(const uint32_t *inv, const uint32_t *rs, uint64_t n_words, uint64_t i,
                        uint32_t k, uint64_t n_bases) {
    return kc::valid_word(inv, rs, n_words, i, k, n_bases);
}

uint64_t kch_wave_valid(const uint32_t *valid, uint64_t pb) {
    kc::ReadsArgs R{nullptr, nullptr, nullptr, 0, 0, valid};
    return kc::wave_valid(R, pb);
}

uint64_t kch_hash(uint64_t key, uint32_t a) {
    uint32_t b0, b1;
    kc::key_blocks(key, b0, b1);
    return kc::hash_a(b0, b1, a);
}

uint64_t kch_canonical(uint64_t fwd, uint32_t K, uint64_t *h1) {
    kc::Canon c = kc::canonical(fwd, K);
    *h1 = c.h1;
    return c.key;
}

void kch_slot(uint64_t X, uint64_t Y, uint32_t alpha, uint64_t h, uint64_t *word, uint32_t *l) {
    kc::FilterArgs F{};
    F.X = X;
    F.Y = Y;
    F.mX = UINT64_MAX / X;
    F.mY = UINT64_MAX / Y;
    F.alpha = alpha;
    F.eta = 64u / alpha;
    F.mEta = UINT64_MAX / F.eta;
    F.eta_pow2 = (F.eta & (F.eta - 1)) == 0;
    F.small_dims = X <= kc::kSmallDivisor && Y <= kc::kSmallDivisor;
    kc::slot_of(F, h, *word, *l);
}

int kch_base(uint32_t b, uint32_t *code) {
    *code = kc::base_code(b);
    return kc::base_valid(b, *code) ? 1 : 0;
}
}

extern "C" {

int kch_wave_window(const uint32_t *codes, const uint32_t *inv, const uint32_t *rs,
                    uint64_t n_bases, uint32_t k, uint64_t p, uint64_t *fwd) {
    kc::ReadsArgs R{codes, inv, rs, n_bases, k};
    const uint64_t pb = p & ~63ull;
    kc::WaveWords w;
    kc::wave_load(R, pb, w);
    return kc::wave_window(w, pb, (uint32_t)(p - pb), k, n_bases, *fwd) ? 1 : 0;
}

uint64_t kch_canonical_fast(uint64_t fwd, uint32_t K, uint64_t *h1) {
    kc::Canon c = kc::canonical_fast(fwd, K);
    *h1 = c.h1;
    return c.key;
}
}

extern "C" {

void kch_window_key_wide(const uint32_t *codes, uint64_t p, uint32_t K, uint64_t *lo,
                         uint64_t *hi) {
    kc::Key128 k = kc::window_key_wide(codes, p, K);
    *lo = k.lo;
    *hi = k.hi;
}

void kch_revcomp_wide(uint64_t lo, uint64_t hi, uint32_t K, uint64_t *olo, uint64_t *ohi) {
    kc::Key128 k = kc::revcomp_wide(kc::Key128{lo, hi}, K);
    *olo = k.lo;
    *ohi = k.hi;
}

uint64_t kch_hash_wide(uint64_t lo, uint64_t hi, uint32_t a) {
    uint32_t b[4];
    kc::key_blocks_wide(kc::Key128{lo, hi}, b);
    return kc::hash_a_wide(b, a);
}

void kch_canonical_wide(uint64_t lo, uint64_t hi, uint32_t K, uint64_t *clo, uint64_t *chi,
                        uint64_t *h1) {
    kc::CanonWide c = kc::canonical_wide(kc::Key128{lo, hi}, K);
    *clo = c.key.lo;
    *chi = c.key.hi;
    *h1 = c.h1;
}
}
