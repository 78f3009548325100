/*
 * KmerCo CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of KmerCo's insertion and
 * classification phases, written from the paper (Nayak & Patgiri, "KmerCo: A
 * lightweight K-mer counting technique with a tiny memory footprint",
 * arXiv 2305.07545).  It exists to check the GPU library: only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code with the GPU path.
 *
 * Every step follows the paper's order and notation:
 *   - k-mer windows of a sequence: Sec. 1.1 (L-K+1 consecutive substrings);
 *   - reverse complement: Sec. 2.2 (A<->T, C<->G, then reversed);
 *   - canonical k-mer = strand with the smaller hash: Sec. 2.3 equation;
 *   - countBF layout, masks and sizing: Sec. 2.1 and Eq. (1);
 *   - insertion phase: Algorithm 1, calling Query-I (Algorithm 4) before
 *     the countBF insert (Algorithm 3);
 *   - classification phase: Algorithm 2 with Query-II (Algorithm 5).
 *
 * Readings taken where the paper is silent or inconsistent (each one is a
 * numbered reading listed in the design notes):
 *   R1  hash: H_a(x) = (MM3(x, 2a-2) << 32) | MM3(x, 2a-1), where MM3 is
 *       MurmurHash3_x86_32 over the 8-byte little-endian 2-bit key x;
 *   R2  what is hashed: the 2-bit key (A=0 C=1 G=2 T=3, first base most
 *       significant), K <= 32;
 *   R3  windows containing any byte other than 'A','C','G','T' are skipped;
 *       windows never span two reads;
 *   R4  canonical strand chosen once with H_1; a tie goes to the reverse
 *       complement (Algorithm 4's else-branch); all H_a hash that strand;
 *   R5  a counter saturates at 2^alpha - 1 (the increment that would reach
 *       2^alpha is dropped); each of the k_h counters saturates on its own;
 *   R6  Algorithm 5's "l <- h % tau" is read as "l <- h % eta";
 *   R7  cell (i, j) is word i*Y + j of a row-major uint64 array; counter l
 *       occupies bits [alpha*l, alpha*l + alpha) (the paper's first extract
 *       mask 0x00000000000000FF);
 *   R8  eta = floor(64 / alpha) counters per 64-bit cell (supplement table);
 *   R9  trustworthy iff frequency > tau, erroneous otherwise (Sec. 3);
 *   R15 K-mers of 33..64 bases (the paper's 55-mers, Sec. 4): the 2-bit key
 *       is a 128-bit integer (first base most significant), hashed as its 16
 *       little-endian bytes (R1 with a 16-byte key), and stored as two
 *       uint64 words, low word first.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KCO_OK 0
#define KCO_EINVAL (-1)
#define KCO_ERANGE (-3)

typedef struct {
    uint64_t X, Y;     /* countBF dimensions (primes) */
    uint32_t alpha;    /* counter length in bits */
    uint32_t k_h;      /* number of hash functions */
} kco_layout;

/* ------------------------------------------------------------------------
 * MurmurHash3_x86_32, written from Austin Appleby's published description of
 * the algorithm: 4-byte little-endian blocks mixed into the state, then the
 * 1..3 byte tail, then the length and the final avalanche ("fmix32").
 * ---------------------------------------------------------------------- */
static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

uint32_t kco_mm3_32(const uint8_t *data, uint64_t len, uint32_t seed)
{
    const uint32_t c1 = 0xcc9e2d51u;
    const uint32_t c2 = 0x1b873593u;
    uint32_t h = seed;
    uint64_t nblocks = len / 4;
    for (uint64_t b = 0; b < nblocks; b++) {
        const uint8_t *p = data + 4 * b;
        uint32_t k = (uint32_t)p[0] | ((uint32_t)p[1] << 8) |
                     ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xe6546b64u;
    }
    const uint8_t *tail = data + 4 * nblocks;
    uint32_t k = 0;
    switch (len & 3) {
    case 3: k ^= (uint32_t)tail[2] << 16; /* fall through */
    case 2: k ^= (uint32_t)tail[1] << 8;  /* fall through */
    case 1:
        k ^= (uint32_t)tail[0];
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
    }
    h ^= (uint32_t)len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* H_a of a 2-bit key (reading R1), a = 1..k_h. */
uint64_t kco_hash(uint64_t key, uint32_t a)
{
    uint8_t bytes[8];
    for (int i = 0; i < 8; i++)
        bytes[i] = (uint8_t)(key >> (8 * i));
    uint64_t hi = kco_mm3_32(bytes, 8, 2u * a - 2u);
    uint64_t lo = kco_mm3_32(bytes, 8, 2u * a - 1u);
    return (hi << 32) | lo;
}

/* ------------------------------------------------------------------------
 * Sequences (Sec. 2.2, reading R2)
 * ---------------------------------------------------------------------- */
static int base_code(uint8_t c)
{
    switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
    }
}

/* Complement table of Sec. 2.2: A<->T, C<->G, N stays N. */
static uint8_t complement(uint8_t c)
{
    switch (c) {
    case 'A': return 'T';
    case 'T': return 'A';
    case 'C': return 'G';
    case 'G': return 'C';
    default: return c;
    }
}

/* Reverse complement of a string: complement every base, then reverse. */
void kco_revcomp(const uint8_t *s, uint64_t len, uint8_t *out)
{
    for (uint64_t i = 0; i < len; i++)
        out[len - 1 - i] = complement(s[i]);
}

/* 2-bit key of a K-character string, first base most significant.
 * Returns 0 and sets *key, or -1 when a byte is not A/C/G/T. */
int kco_encode(const uint8_t *s, uint32_t K, uint64_t *key)
{
    uint64_t v = 0;
    for (uint32_t i = 0; i < K; i++) {
        int c = base_code(s[i]);
        if (c < 0)
            return -1;
        v = v * 4u + (uint64_t)c;
    }
    *key = v;
    return 0;
}

/* ------------------------------------------------------------------------
 * countBF (Sec. 2.1, readings R7, R8)
 * ---------------------------------------------------------------------- */
uint32_t kco_eta(uint32_t alpha) { return alpha == 0 ? 0 : 64u / alpha; }

/* extract mask M^e_l: alpha ones at bit alpha*l */
static uint64_t extract_mask(uint32_t alpha, uint32_t l)
{
    uint64_t ones = (alpha >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << alpha) - 1u);
    return ones << (alpha * l);
}

/* Slot of hash value h: cell (i, j) and counter l (Algorithm 3, line
 * "i <- h%x, j <- h%y, l <- h%eta"). */
void kco_slot(const kco_layout *L, uint64_t h, uint64_t *word, uint32_t *l)
{
    uint64_t i = h % L->X;
    uint64_t j = h % L->Y;
    *l = (uint32_t)(h % kco_eta(L->alpha));
    *word = i * L->Y + j;
}

static uint64_t read_counter(const kco_layout *L, const uint64_t *C, uint64_t word, uint32_t l)
{
    return (C[word] & extract_mask(L->alpha, l)) >> (L->alpha * l);
}

/* Algorithm 3 (IcountBF) for one k-mer: for every hash function, extract
 * the counter with the extract mask, add one, and write it back through the
 * reset mask unless that would overflow the counter (reading R5). */
static void icountbf(const kco_layout *L, uint64_t *C, uint64_t kmer)
{
    uint64_t maxv = (L->alpha >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << L->alpha) - 1u);
    for (uint32_t a = 1; a <= L->k_h; a++) {
        uint64_t h = kco_hash(kmer, a);
        uint64_t word;
        uint32_t l;
        kco_slot(L, h, &word, &l);
        uint64_t value = read_counter(L, C, word, l);
        if (value == maxv)
            continue; /* counter overflow: leave this counter as it is */
        value = value + 1u;
        uint64_t reset = ~extract_mask(L->alpha, l);
        C[word] = (C[word] & reset) | (value << (L->alpha * l));
    }
}

/* Algorithm 5 (QcountBF-II): 0 if any counter is 0, else the minimum. */
uint64_t kco_query(const kco_layout *L, const uint64_t *C, uint64_t kmer)
{
    uint64_t best = 0;
    for (uint32_t a = 1; a <= L->k_h; a++) {
        uint64_t h = kco_hash(kmer, a);
        uint64_t word;
        uint32_t l;
        kco_slot(L, h, &word, &l);
        uint64_t value = read_counter(L, C, word, l);
        if (value == 0)
            return 0;
        if (a == 1 || value < best)
            best = value;
    }
    return best;
}

/* Canonical choice of Algorithm 4 / Sec. 2.3 (reading R4): Result 0 keeps
 * the read, Result 1 takes the reverse complement. */
static int choose_strand(uint64_t fwd, uint64_t rc)
{
    uint64_t h = kco_hash(fwd, 1);
    uint64_t h1 = kco_hash(rc, 1);
    return (h < h1) ? 0 : 1;
}

uint64_t kco_canonical(uint64_t fwd, uint64_t rc)
{
    return choose_strand(fwd, rc) == 0 ? fwd : rc;
}

/* Algorithm 4 (QcountBF-I) restricted to the strand chosen once (R4). */
static uint64_t qcountbf_1(const kco_layout *L, const uint64_t *C, uint64_t fwd,
                           uint64_t rc, int *result)
{
    *result = choose_strand(fwd, rc);
    return kco_query(L, C, *result == 0 ? fwd : rc);
}

static int check_layout(const kco_layout *L)
{
    if (!L || L->X == 0 || L->Y == 0 || L->alpha < 1 || L->alpha > 64 ||
        L->k_h < 1 || L->k_h > 8)
        return KCO_EINVAL;
    return KCO_OK;
}

/* ------------------------------------------------------------------------
 * Algorithm 1 (InsertKmerCo).  Reads are processed in input order; in each
 * read every window start p = 0..len-K is visited in increasing order.  For
 * each valid window: build the read and its reverse complement (as strings),
 * encode both, query the countBF with Query-I; a zero answer appends the
 * canonical k-mer to the distinct list; then insert it with Algorithm 3.
 *
 * words:     countBF, X*Y uint64, modified in place
 * distinct:  receives this call's distinct k-mers (first-seen order)
 * n_windows: number of k-mers inserted (valid windows)
 * ---------------------------------------------------------------------- */
int kco_insert(const kco_layout *L, uint64_t *words, const uint8_t *reads,
               const uint64_t *offsets, uint64_t n_reads, uint32_t K,
               uint64_t *distinct, uint64_t distinct_cap, uint64_t *n_distinct,
               uint64_t *n_windows)
{
    if (check_layout(L) != KCO_OK || K < 1 || K > 32)
        return KCO_EINVAL;
    uint8_t read[32], read_rc[32];
    uint64_t nd = 0, nw = 0;
    int overflow = 0;
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t start = offsets[r], end = offsets[r + 1];
        if (end < start)
            return KCO_EINVAL;
        if (end - start < K)
            continue;
        for (uint64_t p = start; p + K <= end; p++) {
            memcpy(read, reads + p, K);                 /* Read <- K-mer */
            kco_revcomp(read, K, read_rc);              /* Read_RC */
            uint64_t fwd, rc;
            if (kco_encode(read, K, &fwd) != 0)
                continue;                               /* R3: skip */
            kco_encode(read_rc, K, &rc);
            int result;
            uint64_t freq = qcountbf_1(L, words, fwd, rc, &result);
            uint64_t kmer = (result == 0) ? fwd : rc;
            if (freq == 0) {
                if (nd < distinct_cap)
                    distinct[nd] = kmer;
                else
                    overflow = 1;
                nd++;
            }
            icountbf(L, words, kmer);
            nw++;
        }
    }
    *n_distinct = nd;
    *n_windows = nw;
    return overflow ? KCO_ERANGE : KCO_OK;
}

/* Algorithm 2 (QueryKmerCo): split the distinct list, in its order, into
 * trustworthy (frequency > tau) and erroneous k-mers. */
int kco_classify(const kco_layout *L, const uint64_t *words, const uint64_t *distinct,
                 uint64_t n, uint64_t tau, uint64_t *trust, uint64_t *n_trust,
                 uint64_t *err, uint64_t *n_err)
{
    if (check_layout(L) != KCO_OK)
        return KCO_EINVAL;
    uint64_t nt = 0, ne = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (kco_query(L, words, distinct[i]) > tau)
            trust[nt++] = distinct[i];
        else
            err[ne++] = distinct[i];
    }
    *n_trust = nt;
    *n_err = ne;
    return KCO_OK;
}

/* Query-II over an array of k-mers. */
int kco_query_many(const kco_layout *L, const uint64_t *words, const uint64_t *keys,
                   uint64_t n, uint64_t *freq)
{
    if (check_layout(L) != KCO_OK)
        return KCO_EINVAL;
    for (uint64_t i = 0; i < n; i++)
        freq[i] = kco_query(L, words, keys[i]);
    return KCO_OK;
}

/* Test helper: the canonical k-mer and its k_h slots for every valid window,
 * in Algorithm 1's visiting order (slot id = word * eta + l). */
int kco_occurrences(const kco_layout *L, const uint8_t *reads, const uint64_t *offsets,
                    uint64_t n_reads, uint32_t K, uint64_t *kmers, uint64_t *slot_ids,
                    uint64_t cap, uint64_t *n_out)
{
    if (check_layout(L) != KCO_OK || K < 1 || K > 32)
        return KCO_EINVAL;
    uint8_t read[32], read_rc[32];
    uint64_t n = 0;
    uint32_t eta = kco_eta(L->alpha);
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t start = offsets[r], end = offsets[r + 1];
        if (end - start < K)
            continue;
        for (uint64_t p = start; p + K <= end; p++) {
            memcpy(read, reads + p, K);
            kco_revcomp(read, K, read_rc);
            uint64_t fwd, rc;
            if (kco_encode(read, K, &fwd) != 0)
                continue;
            kco_encode(read_rc, K, &rc);
            uint64_t kmer = kco_canonical(fwd, rc);
            if (n < cap) {
                kmers[n] = kmer;
                for (uint32_t a = 1; a <= L->k_h; a++) {
                    uint64_t word;
                    uint32_t l;
                    kco_slot(L, kco_hash(kmer, a), &word, &l);
                    slot_ids[n * L->k_h + (a - 1)] = word * eta + l;
                }
            }
            n++;
        }
    }
    *n_out = n;
    return n > cap ? KCO_ERANGE : KCO_OK;
}

/* ------------------------------------------------------------------------
 * K-mers of 33..64 bases (reading R15).  The same steps as above -- window
 * visiting order, reverse complement, canonical strand by H_1, Query-I
 * before the insert, Algorithm 3's saturating increments, Algorithm 2's
 * split -- on 128-bit keys.
 * ---------------------------------------------------------------------- */
typedef unsigned __int128 kco_u128;

/* H_a of a 128-bit key given as (low, high) words: MM3 over its 16
 * little-endian bytes, low word first. */
uint64_t kco_hash_wide(uint64_t lo, uint64_t hi, uint32_t a)
{
    uint8_t bytes[16];
    for (int i = 0; i < 8; i++) {
        bytes[i] = (uint8_t)(lo >> (8 * i));
        bytes[8 + i] = (uint8_t)(hi >> (8 * i));
    }
    uint64_t h_hi = kco_mm3_32(bytes, 16, 2u * a - 2u);
    uint64_t h_lo = kco_mm3_32(bytes, 16, 2u * a - 1u);
    return (h_hi << 32) | h_lo;
}

static uint64_t hash_u128(kco_u128 key, uint32_t a)
{
    return kco_hash_wide((uint64_t)key, (uint64_t)(key >> 64), a);
}

/* 2-bit key of a K-character string (K <= 64), first base most significant. */
static int encode_wide(const uint8_t *s, uint32_t K, kco_u128 *key)
{
    kco_u128 v = 0;
    for (uint32_t i = 0; i < K; i++) {
        int c = base_code(s[i]);
        if (c < 0)
            return -1;
        v = v * 4u + (kco_u128)c;
    }
    *key = v;
    return 0;
}

/* Algorithm 3 for a 128-bit key. */
static void icountbf_wide(const kco_layout *L, uint64_t *C, kco_u128 kmer)
{
    uint64_t maxv = (L->alpha >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << L->alpha) - 1u);
    for (uint32_t a = 1; a <= L->k_h; a++) {
        uint64_t word;
        uint32_t l;
        kco_slot(L, hash_u128(kmer, a), &word, &l);
        uint64_t value = read_counter(L, C, word, l);
        if (value == maxv)
            continue;
        value = value + 1u;
        uint64_t reset = ~extract_mask(L->alpha, l);
        C[word] = (C[word] & reset) | (value << (L->alpha * l));
    }
}

/* Algorithm 5 for a 128-bit key: 0 if any counter is 0, else the minimum. */
static uint64_t query_u128(const kco_layout *L, const uint64_t *C, kco_u128 kmer)
{
    uint64_t best = 0;
    for (uint32_t a = 1; a <= L->k_h; a++) {
        uint64_t word;
        uint32_t l;
        kco_slot(L, hash_u128(kmer, a), &word, &l);
        uint64_t value = read_counter(L, C, word, l);
        if (value == 0)
            return 0;
        if (a == 1 || value < best)
            best = value;
    }
    return best;
}

uint64_t kco_query_wide(const kco_layout *L, const uint64_t *C, uint64_t lo, uint64_t hi)
{
    return query_u128(L, C, ((kco_u128)hi << 64) | lo);
}

/* Sec. 2.3 / Algorithm 4 for 128-bit keys (reading R4). */
static kco_u128 canonical_wide(kco_u128 fwd, kco_u128 rc)
{
    return hash_u128(fwd, 1) < hash_u128(rc, 1) ? fwd : rc;
}

/* Algorithm 1 for K = 33..64; distinct receives (low, high) pairs. */
int kco_insert_wide(const kco_layout *L, uint64_t *words, const uint8_t *reads,
                    const uint64_t *offsets, uint64_t n_reads, uint32_t K,
                    uint64_t *distinct, uint64_t distinct_cap, uint64_t *n_distinct,
                    uint64_t *n_windows)
{
    if (check_layout(L) != KCO_OK || K < 33 || K > 64)
        return KCO_EINVAL;
    uint8_t read[64], read_rc[64];
    uint64_t nd = 0, nw = 0;
    int overflow = 0;
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t start = offsets[r], end = offsets[r + 1];
        if (end < start)
            return KCO_EINVAL;
        if (end - start < K)
            continue;
        for (uint64_t p = start; p + K <= end; p++) {
            memcpy(read, reads + p, K);
            kco_revcomp(read, K, read_rc);
            kco_u128 fwd, rc = 0;
            if (encode_wide(read, K, &fwd) != 0)
                continue;
            encode_wide(read_rc, K, &rc);
            kco_u128 kmer = canonical_wide(fwd, rc);
            if (query_u128(L, words, kmer) == 0) {
                if (nd < distinct_cap) {
                    distinct[2 * nd] = (uint64_t)kmer;
                    distinct[2 * nd + 1] = (uint64_t)(kmer >> 64);
                } else {
                    overflow = 1;
                }
                nd++;
            }
            icountbf_wide(L, words, kmer);
            nw++;
        }
    }
    *n_distinct = nd;
    *n_windows = nw;
    return overflow ? KCO_ERANGE : KCO_OK;
}

/* Algorithm 2 for (low, high) key pairs. */
int kco_classify_wide(const kco_layout *L, const uint64_t *words, const uint64_t *distinct,
                      uint64_t n, uint64_t tau, uint64_t *trust, uint64_t *n_trust,
                      uint64_t *err, uint64_t *n_err)
{
    if (check_layout(L) != KCO_OK)
        return KCO_EINVAL;
    uint64_t nt = 0, ne = 0;
    for (uint64_t i = 0; i < n; i++) {
        kco_u128 kmer = ((kco_u128)distinct[2 * i + 1] << 64) | distinct[2 * i];
        uint64_t *out = query_u128(L, words, kmer) > tau ? trust + 2 * nt++ : err + 2 * ne++;
        out[0] = distinct[2 * i];
        out[1] = distinct[2 * i + 1];
    }
    *n_trust = nt;
    *n_err = ne;
    return KCO_OK;
}

/* Test helper for K = 33..64: canonical keys as (low, high) pairs and the
 * k_h slot ids of every valid window. */
int kco_occurrences_wide(const kco_layout *L, const uint8_t *reads, const uint64_t *offsets,
                         uint64_t n_reads, uint32_t K, uint64_t *kmers, uint64_t *slot_ids,
                         uint64_t cap, uint64_t *n_out)
{
    if (check_layout(L) != KCO_OK || K < 33 || K > 64)
        return KCO_EINVAL;
    uint8_t read[64], read_rc[64];
    uint64_t n = 0;
    uint32_t eta = kco_eta(L->alpha);
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t start = offsets[r], end = offsets[r + 1];
        if (end - start < K)
            continue;
        for (uint64_t p = start; p + K <= end; p++) {
            memcpy(read, reads + p, K);
            kco_revcomp(read, K, read_rc);
            kco_u128 fwd, rc = 0;
            if (encode_wide(read, K, &fwd) != 0)
                continue;
            encode_wide(read_rc, K, &rc);
            kco_u128 kmer = canonical_wide(fwd, rc);
            if (n < cap) {
                kmers[2 * n] = (uint64_t)kmer;
                kmers[2 * n + 1] = (uint64_t)(kmer >> 64);
                for (uint32_t a = 1; a <= L->k_h; a++) {
                    uint64_t word;
                    uint32_t l;
                    kco_slot(L, hash_u128(kmer, a), &word, &l);
                    slot_ids[n * L->k_h + (a - 1)] = word * eta + l;
                }
            }
            n++;
        }
    }
    *n_out = n;
    return n > cap ? KCO_ERANGE : KCO_OK;
}

/* ------------------------------------------------------------------------
 * Eq. (1): m = -n ln(FPP) / (ln 2)^2, v = sqrt(m / 128), X = smallest prime
 * greater than v, Y = the third prime after X.  The countBF holds X*Y cells
 * of beta = 64 bits.
 * ---------------------------------------------------------------------- */
static int is_prime(uint64_t n)
{
    if (n < 2)
        return 0;
    for (uint64_t d = 2; d * d <= n; d++)
        if (n % d == 0)
            return 0;
    return 1;
}

static uint64_t next_prime_after(uint64_t n)
{
    uint64_t p = n + 1;
    while (!is_prime(p))
        p++;
    return p;
}

int kco_is_prime(uint64_t n) { return is_prime(n); }

int kco_dims(double n_items, double fpp, uint64_t *X, uint64_t *Y)
{
    if (!(n_items > 0) || !(fpp > 0) || !(fpp < 1))
        return KCO_EINVAL;
    double m = -n_items * log(fpp) / (log(2.0) * log(2.0));
    double v = sqrt(m / 128.0);
    uint64_t x = next_prime_after((uint64_t)floor(v));
    uint64_t y = x;
    for (int i = 0; i < 3; i++)
        y = next_prime_after(y);
    *X = x;
    *Y = y;
    return KCO_OK;
}
