/*
 * kmerco.h -- C ABI of the MI355X (gfx950) KmerCo library.
 *
 * KmerCo (Nayak & Patgiri, arXiv 2305.07545) counts k-mers with a countBF:
 * an X x Y array of 64-bit cells, each holding eta = floor(64/alpha) packed
 * alpha-bit counters (Sec. 2.1, Eq. (1)).  Its insertion phase (Algorithm 1)
 * inserts every k-mer of the input reads and lists the distinct ones in
 * first-seen order; its classification phase (Algorithm 2) splits the
 * distinct k-mers into trustworthy (frequency > tau) and erroneous ones.
 *
 * Conventions shared by every entry point
 *  - Pointers named *_dev are device (HBM) pointers owned by the caller; the
 *    library never frees them.  Host pointers are named without the suffix.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls marked "async" only enqueue work on that stream; results are
 *    valid once the stream has reached them.
 *  - k-mers are 2-bit keys in a uint64: A=0, C=1, G=2, T=3, first base most
 *    significant, K <= 32.  Reads are ASCII bytes; any byte other than
 *    'A','C','G','T' (upper case) is an invalid base and every window that
 *    contains one is skipped.  Windows never span two reads.
 *  - Hash functions: H_a(x) = (MM3(x, 2a-2) << 32) | MM3(x, 2a-1), with MM3
 *    = MurmurHash3_x86_32 over the 8-byte little-endian key (the paper names
 *    the murmur hash, Sec. 3).  Canonical k-mer = the strand with the smaller
 *    H_1 (Sec. 2.3 equation; a tie keeps the reverse complement).
 *  - Slot of a k-mer for hash function a (Algorithm 3): h = H_a(canonical),
 *    cell (i, j) = (h mod X, h mod Y) stored row-major at word i*Y + j,
 *    counter l = h mod eta at bits [alpha*l, alpha*l + alpha).
 *  - A counter saturates at 2^alpha - 1; each of the k_h counters saturates
 *    on its own.
 *  - Errors are returned as kc_status codes; nothing is thrown across the
 *    ABI.  Asynchronous device-side errors (an output buffer too small) are
 *    sticky in the filter handle and reported by kc_sync().
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef KMERCO_H
#define KMERCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KC_OK = 0,
    KC_EINVAL = -1,   /* bad argument (layout, k, sizes, null pointer) */
    KC_ENOMEM = -2,   /* device workspace allocation failed */
    KC_ERANGE = -3,   /* an output capacity was too small (counts still report the need) */
    KC_EDEVICE = -4,  /* a HIP runtime call failed */
    KC_ESTATE = -5    /* call not allowed in the handle's state (e.g. k differs from the first insert) */
} kc_status;

typedef struct kc_filter kc_filter;

/* countBF layout (Sec. 2.1).  X, Y: dimensions (the paper uses primes from
 * Eq. (1); any X, Y >= 1 with X*Y*8 bytes addressable are accepted).
 * alpha: counter length in bits, 1..32.  k_h: hash functions, 1..8. */
typedef struct {
    uint64_t X, Y;
    uint32_t alpha;
    uint32_t k_h;
} kc_layout;

/* Text for a status code (static string). */
const char *kc_strerror(int status);

/* Library ABI version (incremented on incompatible changes). */
int kc_version(void);

/* Eq. (1), host only, pure: m = -n ln(fpp) / (ln 2)^2, v = sqrt(m / 128),
 * X = smallest prime > v, Y = third prime after X.
 * n_items > 0, 0 < fpp < 1, else KC_EINVAL. */
kc_status kc_dims(double n_items, double fpp, uint64_t *X, uint64_t *Y);

/* Counters per 64-bit cell: floor(64 / alpha) (supplement counter table). */
uint32_t kc_eta(uint32_t alpha);

/* Create a countBF over caller-owned device memory `words_dev` (X*Y uint64,
 * 8-byte aligned).  zero != 0: the library clears the words (async on
 * `stream`) and the filter starts empty; zero == 0: the words are taken as
 * they are (resuming an existing countBF).  The handle owns a first-seen
 * workspace of 4 bytes per counter (X*Y*eta*4 bytes of device memory),
 * allocated here.  Returns KC_EINVAL for a bad layout, KC_ENOMEM when the
 * workspace cannot be allocated. */
kc_status kc_create(const kc_layout *layout, uint64_t *words_dev, int zero, void *stream,
                    kc_filter **out);

/* Release the handle and its workspace (not the caller's words).  Waits for
 * the handle's outstanding work first.  NULL is ignored. */
void kc_destroy(kc_filter *f);

/* Pre-size the per-call workspace for inserts of up to `max_bases` bases
 * (about max_bases/2 bytes + 256 B per 1024 bases) so that later kc_insert
 * calls of that size allocate nothing.  Synchronous. */
kc_status kc_reserve(kc_filter *f, uint64_t max_bases);

/* Insertion phase (Algorithm 1 with Query-I / Algorithm 4 before the
 * countBF insert / Algorithm 3), async on `stream`.
 *
 * reads_dev    n_bases ASCII bytes, all reads concatenated.
 * offsets_dev  n_reads + 1 uint64 CSR offsets: read r is
 *              reads_dev[offsets[r] .. offsets[r+1]); offsets[0] must be 0,
 *              offsets must be non-decreasing and offsets[n_reads] must equal
 *              n_bases (not checked on the device; offsets outside the read
 *              buffer only change results, never the memory touched).
 * k            k-mer length, 1..32; every insert into one filter must use the
 *              same k (else KC_ESTATE).
 * distinct_dev receives this call's distinct k-mers (canonical keys) in
 *              first-seen order (reads in input order, windows by start
 *              position), appended at index *n_distinct_dev.
 * distinct_cap capacity of distinct_dev in keys.  Keys that do not fit are
 *              dropped, *n_distinct_dev still counts them and the handle
 *              records KC_ERANGE (returned by kc_sync).
 * n_distinct_dev  device uint64, in/out: running distinct count.
 * n_windows_dev   device uint64 or NULL, in/out: += number of k-mers inserted
 *              (valid windows) by this call.
 *
 * Several calls are equivalent to one call on the concatenated reads.  The
 * result is bit-identical to the sequential algorithm, hash collisions
 * included. */
kc_status kc_insert(kc_filter *f, const uint8_t *reads_dev, const uint64_t *offsets_dev,
                    uint64_t n_reads, uint64_t n_bases, uint32_t k,
                    uint64_t *distinct_dev, uint64_t distinct_cap, uint64_t *n_distinct_dev,
                    uint64_t *n_windows_dev, void *stream);

/* Both phases of KmerCo for one read batch (the pipeline of Sec. 3: insert
 * every k-mer, then classify the distinct ones), async on `stream`.
 * Insertion is exactly kc_insert (same arguments, same distinct output).
 * This call's distinct k-mers are then split by Query-II against the countBF
 * as it stands after the call: frequency > tau -> trust_dev, else err_dev,
 * both in distinct order, class_cap keys of room each; *n_trust_dev and
 * *n_err_dev are overwritten with the counts (a count above class_cap drops
 * the excess and records KC_ERANGE, returned by kc_sync).  Identical to
 * kc_insert followed by kc_classify of the keys the insert appended. */
kc_status kc_insert_classify(kc_filter *f, const uint8_t *reads_dev, const uint64_t *offsets_dev,
                             uint64_t n_reads, uint64_t n_bases, uint32_t k, uint32_t tau,
                             uint64_t *distinct_dev, uint64_t distinct_cap,
                             uint64_t *n_distinct_dev, uint64_t *n_windows_dev,
                             uint64_t *trust_dev, uint64_t *n_trust_dev, uint64_t *err_dev,
                             uint64_t *n_err_dev, uint64_t class_cap, void *stream);

/* Classification phase (Algorithm 2 with Query-II / Algorithm 5), async.
 * keys_dev / n_keys_dev: the k-mers to classify (typically the distinct list
 * and its device count); n = min(*n_keys_dev, keys_cap) keys are used.
 * trust_dev, err_dev: outputs with room for n keys each; the order of
 * keys_dev is kept in both.  *n_trust_dev, *n_err_dev are overwritten with
 * the counts.  frequency > tau -> trustworthy, else erroneous. */
kc_status kc_classify(kc_filter *f, const uint64_t *keys_dev, const uint64_t *n_keys_dev,
                      uint64_t keys_cap, uint32_t tau, uint64_t *trust_dev,
                      uint64_t *n_trust_dev, uint64_t *err_dev, uint64_t *n_err_dev,
                      void *stream);

/* Query-II (Algorithm 5) for n canonical keys, async: freq_dev[i] = 0 if any
 * of the key's k_h counters is 0, else their minimum. */
kc_status kc_query(kc_filter *f, const uint64_t *keys_dev, uint64_t n, uint32_t *freq_dev,
                   void *stream);

/* Wait for the handle's last stream and return (and clear) the sticky
 * device-side status: KC_OK or KC_ERANGE; KC_EDEVICE if the runtime failed. */
kc_status kc_sync(kc_filter *f);

/* Layout of a handle (host copy). */
kc_status kc_get_layout(const kc_filter *f, kc_layout *out);

/* Clear the countBF (async on `stream`): every counter back to zero, the
 * filter empty again and its k unset, as after kc_create with zero != 0
 * (the sequential algorithm's initial state, Sec. 2.1: all slots 0). */
kc_status kc_reset(kc_filter *f, void *stream);

/* ------------------------------------------------------------------------
 * Kernel timing.  When enabled, the library brackets each of its kernels
 * with HIP events recorded on the launch stream; kc_profile_read waits for
 * them and adds the elapsed milliseconds and launch counts per phase into
 * the caller's arrays (n_phases entries each, indexed by kc_phase), then
 * forgets the records.  Not for use under stream capture.
 * ---------------------------------------------------------------------- */
typedef enum {
    KC_PHASE_INGEST = 0,          /* ASCII -> 2-bit codes + base/read-start bitmaps */
    KC_PHASE_CLAIM = 1,           /* direct path: first-seen claims (filter not empty) */
    KC_PHASE_INCREMENT = 2,       /* direct path: saturating counter increments */
    KC_PHASE_CLAIM_INCREMENT = 3, /* direct path: claims + increments (filter empty) */
    KC_PHASE_RESOLVE = 4,         /* direct path: first-seen winners -> distinct flags */
    KC_PHASE_SCAN = 5,            /* per-tile offsets (insert and classify) */
    KC_PHASE_SCATTER = 6,         /* ordered distinct-key output */
    KC_PHASE_CLASSIFY_MARK = 7,   /* Query-II + threshold per key */
    KC_PHASE_CLASSIFY_SCATTER = 8,/* ordered trustworthy / erroneous output */
    KC_PHASE_QUERY = 9,           /* kc_query */
    KC_PHASE_RESET = 10,          /* kc_reset / kc_create clears */
    KC_PHASE_BIN_COUNT = 11,      /* binned path: per-region entry counts */
    KC_PHASE_BIN_BUCKET = 12,     /* binned path: entries grouped by bucket of regions */
    KC_PHASE_REGION = 13,         /* binned path: LDS counting + first-seen per region */
    KC_PHASE_TILE_COUNT = 14,     /* per-tile distinct / trustworthy / window counts */
    KC_PHASE_BIN_REGION = 15,     /* binned path: bucket slices -> region segments */
    KC_PHASE_COUNT = 16
} kc_phase;

kc_status kc_profile(kc_filter *f, int enable);
kc_status kc_profile_read(kc_filter *f, double *ms, uint64_t *launches, uint32_t n_phases);
const char *kc_phase_name(uint32_t phase);

/* ------------------------------------------------------------------------
 * Batched form: many independent read sets, each with its own countBF, k and
 * tau, inserted (and classified) together by one launch per phase.  The
 * result for every set is identical to kc_insert_classify (or kc_insert when
 * trust_dev is NULL) on that set's reads alone.
 *
 * All sets' reads live in one buffer (reads_dev, offsets_dev as for
 * kc_insert, n_bases bytes in total).  Set i owns bases
 * [first_base, first_base + n_bases) of it, which must hold whole reads:
 * first_base a multiple of 4096, sets sorted by first_base and disjoint
 * (padding between sets must be reads of invalid bases, e.g. 'N', which add
 * no k-mer).  Each set has its own filter handle (at most one set per
 * handle), created on the batch's device; its countBF may span at most 2048
 * regions of 16384 counters (about 16 MB at alpha = 8) and hold at most
 * 2^28 bases; larger sets go through kc_insert.  The total number of
 * (base, hash function) pairs must stay below 2^32.  Outputs per set have the
 * meaning of kc_insert_classify; distinct capacity overflows are sticky in
 * the set's filter (kc_sync on it).
 * ---------------------------------------------------------------------- */
typedef struct kc_batch kc_batch;

typedef struct {
    kc_filter *filter;
    uint64_t first_base, n_bases;
    uint32_t k, tau;
    uint64_t *distinct_dev;
    uint64_t distinct_cap;
    uint64_t *n_distinct_dev;   /* in/out, appended at */
    uint64_t *n_windows_dev;    /* in/out, may be NULL */
    uint64_t *trust_dev;        /* NULL: insertion only */
    uint64_t *n_trust_dev;
    uint64_t *err_dev;
    uint64_t *n_err_dev;
    uint64_t class_cap;
} kc_set;

/* kc_batch_insert flags */
#define KC_BATCH_RESET 1u  /* first clear every set's countBF and zero its distinct/window counters */
#define KC_BATCH_GRAPH 2u  /* capture the launches into a HIP graph; a later call with the same
                              arguments replays it (stream must not be the null stream) */
#define KC_BATCH_TUNE 4u   /* time the candidate work-item sizes on this input, keep the fastest */

kc_status kc_batch_create(kc_batch **out);
void kc_batch_destroy(kc_batch *b);
kc_status kc_batch_insert(kc_batch *b, const kc_set *sets, uint32_t n_sets,
                          const uint8_t *reads_dev, const uint64_t *offsets_dev, uint64_t n_reads,
                          uint64_t n_bases, uint32_t flags, void *stream);
/* work-item size (positions per binning workgroup) in use / to use */
kc_status kc_batch_get_tile(const kc_batch *b, uint64_t *tile);
kc_status kc_batch_set_tile(kc_batch *b, uint64_t tile);
kc_status kc_batch_profile(kc_batch *b, int enable);
kc_status kc_batch_profile_read(kc_batch *b, double *ms, uint64_t *launches, uint32_t n_phases);
kc_status kc_batch_sync(kc_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* KMERCO_H */
