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
 *  - k-mers are 2-bit keys: A=0, C=1, G=2, T=3, first base most significant.
 *    For K <= 32 a key is one uint64.  For K = 33..64 (the paper's 55-mers,
 *    Sec. 4) it is a 128-bit integer stored as two uint64 words, low word
 *    first, in every key array (capacities still count keys); such keys are
 *    taken by the binned insertion paths (also inside the batched form and
 *    the server), kc_classify and kc_query, not by the direct path
 *    (KC_EINVAL).
 *    Reads are ASCII bytes; any byte other than
 *    'A','C','G','T' (upper case) is an invalid base and every window that
 *    contains one is skipped.  Windows never span two reads.
 *  - Hash functions: H_a(x) = (MM3(x, 2a-2) << 32) | MM3(x, 2a-1), with MM3
 *    = MurmurHash3_x86_32 over the 8-byte little-endian key (16 bytes, low
 *    word first, for K > 32; the paper names the murmur hash, Sec. 3).  Canonical k-mer = the strand with the smaller
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

/* ------------------------------------------------------------------------
 * Input front end (host only).  The paper inserts the k-mers of sequencing
 * data sets read from files (Sec. 4.1); kc_parse_fastx turns FASTA or FASTQ text
 * in host memory into the read layout the insert calls take.
 *
 * text[0..len): FASTA ('>' header lines, the sequence lines up to the next
 * header; ';' lines are comments) or FASTQ ('@' header, sequence lines, a
 * '+' line, quality lines of the same total length), the format taken from
 * the first line that is neither blank nor a comment; blank lines are
 * skipped.  Each record's sequence
 * lines are concatenated, their line ends (LF or CR LF) removed and bytes
 * kept as they are (so 'N' and lower case stay invalid bases), into
 * seq[0..*n_bases), and offsets[0..*n_reads] receives the CSR offsets
 * (offsets[0] = 0): one read per record, records with no bases included.
 * flags: KC_FASTX_ONE_SEQUENCE makes all records one read, so windows span
 * record boundaries: the paper counts L - K + 1 windows per data set (its
 * 28-mer and 55-mer totals differ by 27 for every data set, Sec. 4.2).
 * All buffers are the caller's host memory.  *n_bases and *n_reads are
 * always set to the sizes needed; KC_ERANGE when seq_cap < *n_bases or
 * off_cap < *n_reads + 1, with nothing written past either capacity (call
 * with capacities 0 to size the buffers, then again).  KC_EINVAL: null
 * pointers (text with len > 0, outputs with non-zero capacities, the
 * counts), unknown flags, a first line starting with neither '>' nor '@', a
 * FASTQ record not starting with '@', without its '+' line, or whose
 * quality lines do not add up to its sequence length.
 * ---------------------------------------------------------------------- */
#define KC_FASTX_ONE_SEQUENCE 1u
kc_status kc_parse_fastx(const char *text, uint64_t len, uint32_t flags, uint8_t *seq,
                         uint64_t seq_cap, uint64_t *offsets, uint64_t off_cap,
                         uint64_t *n_bases, uint64_t *n_reads);

/* Eq. (1), host only, pure: m = -n ln(fpp) / (ln 2)^2, v = sqrt(m / 128),
 * X = smallest prime > v, Y = third prime after X.
 * n_items > 0, 0 < fpp < 1, else KC_EINVAL. */
kc_status kc_dims(double n_items, double fpp, uint64_t *X, uint64_t *Y);

/* Counters per 64-bit cell: floor(64 / alpha) (supplement counter table). */
uint32_t kc_eta(uint32_t alpha);

/* Bytes of the countBF words of a layout: X * Y * 8 (the caller allocates
 * them, Sec. 2.1: X x Y cells of 64 bits).  0 for an invalid layout.  Host
 * only, pure. */
uint64_t kc_filter_bytes(const kc_layout *layout);

/* Device bytes a handle of this layout needs for inserts of up to max_bases
 * bases and classifications of up to max_bases keys: its status word and
 * what kc_reserve(max_bases) allocates on a new handle (the per-position and
 * per-tile buffers and the binned, partitioned or direct path's scratch, as
 * kc_insert would size them, and, for an insert of several chunks with one
 * hash function, the carried first-seen records of kc_insert_classify: 6
 * bytes per position before the last chunk, see kc_get_plan), each piece
 * rounded up to 256 bytes.  It is the
 * scratch_bytes kc_create_in needs for that max_bases, and lets callers
 * budget HBM before creating handles.  0 for an invalid layout.  Host only,
 * pure: it counts the allocations without making them and touches no
 * device. */
uint64_t kc_scratch_bytes(const kc_layout *layout, uint64_t max_bases);

/* Create a countBF over caller-owned device memory `words_dev` (X*Y uint64,
 * 8-byte aligned).  zero != 0: the library clears the words (async on
 * `stream`) and the filter starts empty; zero == 0: the words are taken as
 * they are (resuming an existing countBF).  The handle's scratch is
 * allocated on first use (see kc_reserve).  Returns KC_EINVAL for a bad
 * layout, KC_ENOMEM when the handle cannot be allocated. */
kc_status kc_create(const kc_layout *layout, uint64_t *words_dev, int zero, void *stream,
                    kc_filter **out);

/* kc_create with the handle's device state in caller memory and/or its k
 * fixed from the start (the countBF of Sec. 2.1 over caller-owned words, as
 * for kc_create; zero as for kc_create).
 *
 * k            0: no k-mer length yet (set by the first insert).  1..64: the
 *              handle's k-mer length (for zero == 0, that of the k-mers the
 *              words already hold: a resumed countBF): inserts must use it
 *              (else KC_ESTATE) and kc_classify / kc_query read keys of its
 *              width from the start.
 * scratch_dev  NULL: the library allocates the handle's scratch (as
 *              kc_create; max_bases > 0 reserves it at once, as kc_reserve).
 *              Otherwise a caller-owned device buffer of scratch_bytes
 *              bytes, 256-byte aligned, at least kc_scratch_bytes(layout,
 *              max_bases): the handle's status word and every buffer its
 *              calls use are laid out in it here, once.  The library then
 *              never allocates device memory for the handle and its insert,
 *              classify and query calls never wait on the host, so they may
 *              be captured into a HIP graph by the caller; an insert of more
 *              than max_bases bases or a classification of more than
 *              max_bases keys returns KC_ERANGE and enqueues nothing.  The
 *              buffer must outlive the handle; kc_destroy does not free it,
 *              and its contents between calls are the library's.
 * Errors: KC_EINVAL (bad layout, k > 64, a misaligned scratch_dev),
 * KC_ERANGE (scratch_bytes below the need), KC_ENOMEM. */
kc_status kc_create_in(const kc_layout *layout, uint64_t *words_dev, int zero, uint32_t k,
                       void *scratch_dev, uint64_t scratch_bytes, uint64_t max_bases,
                       void *stream, kc_filter **out);

/* Release the handle and its workspace (not the caller's words).  Waits for
 * the handle's outstanding work first.  NULL is ignored. */
void kc_destroy(kc_filter *f);

/* Pre-size the handle's scratch for inserts of up to `max_bases` bases so
 * that later kc_insert calls of that size allocate nothing.  Synchronous.
 * KC_ERANGE on a handle whose scratch is the caller's (kc_create_in) when
 * max_bases exceeds what it was laid out for.
 * Sizes, k_h = 1: countBFs of up to 16384 regions (256 MB at alpha = 8) take
 * the binned path, about 22 bytes per base (packed codes and bitmaps, a flag
 * byte, slot ids, two entry lists); larger countBFs take the partitioned
 * path, about 19 bytes per base of a chunk of up to 2^32 - 2^16 bases (two
 * 8-byte entry lists, each holding two kinds of data in turn); the direct
 * path (forced, or beyond 256 partitions) takes 4 bytes per counter plus
 * about 2 bytes per base.  Scratch grows, and is never shrunk, by calls
 * larger than the reservation. */
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
 * k            k-mer length, 1..64 (33..64: two-word keys, binned paths only);
 *              every insert into one filter must use the same k (else
 *              KC_ESTATE).
 * distinct_dev receives this call's distinct k-mers (canonical keys) in
 *              first-seen order (reads in input order, windows by start
 *              position), appended at index *n_distinct_dev.  This is the
 *              listing of distinct k-mers the insertion phase produces
 *              (Algorithm 1): the list is the caller's buffer, so there is
 *              no separate call to fetch it.
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

/* kc_insert_classify for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same outputs, but every scratch buffer of the
 * call is a piece of one fixed device array of KC_NOALLOC_SCRATCH_BYTES
 * bytes that the library holds per device from its load until the process
 * ends, so the call allocates nothing (the handle's own scratch is not
 * used).  The inputs and outputs are still the caller's.
 * Limits: the call's scratch (about kc_scratch_bytes(layout, n_bases)) must
 * fit the array, else KC_ERANGE and nothing is enqueued: about 2.5 M bases
 * for countBFs of up to a few hundred regions; filters that take the direct
 * path (KMERCO_PATH=direct) are refused with KC_EINVAL.
 * Every call on one device uses that device's one array: calls that overlap
 * on a device (other host threads, other streams not ordered with this
 * one) race and give wrong results; calls ordered on one stream are safe. */
#define KC_NOALLOC_SCRATCH_BYTES (64ull << 20)
kc_status kc_insert_classify_noalloc(kc_filter *f, const uint8_t *reads_dev,
                                     const uint64_t *offsets_dev, uint64_t n_reads,
                                     uint64_t n_bases, uint32_t k, uint32_t tau,
                                     uint64_t *distinct_dev, uint64_t distinct_cap,
                                     uint64_t *n_distinct_dev, uint64_t *n_windows_dev,
                                     uint64_t *trust_dev, uint64_t *n_trust_dev, uint64_t *err_dev,
                                     uint64_t *n_err_dev, uint64_t class_cap, void *stream);

/* Classification phase (Algorithm 2 with Query-II / Algorithm 5), async.
 * keys_dev / n_keys_dev: the k-mers to classify (typically the distinct list
 * and its device count); n = min(*n_keys_dev, keys_cap) keys are used.
 * trust_dev, err_dev: outputs with room for n keys each; the order of
 * keys_dev is kept in both.  *n_trust_dev, *n_err_dev are overwritten with
 * the counts.  frequency > tau -> trustworthy, else erroneous.  Keys take
 * two words each when the filter's inserts used k > 32. */
kc_status kc_classify(kc_filter *f, const uint64_t *keys_dev, const uint64_t *n_keys_dev,
                      uint64_t keys_cap, uint32_t tau, uint64_t *trust_dev,
                      uint64_t *n_trust_dev, uint64_t *err_dev, uint64_t *n_err_dev,
                      void *stream);

/* Query-II (Algorithm 5) for n canonical keys, async: freq_dev[i] = 0 if any
 * of the key's k_h counters is 0, else their minimum.  Keys take two words
 * each (2n words) when the filter's inserts used k > 32. */
kc_status kc_query(kc_filter *f, const uint64_t *keys_dev, uint64_t n, uint32_t *freq_dev,
                   void *stream);

/* Wait for the handle's last stream and return (and clear) the sticky
 * device-side status: KC_OK or KC_ERANGE; KC_EDEVICE if the runtime failed. */
kc_status kc_sync(kc_filter *f);

/* The insertion plan of a handle for an insert of n_bases bases (host only,
 * touches no device): the path (the single-level binned path for countBFs
 * of up to 16384 regions, the partitioned one for larger ones, the direct
 * path when forced or beyond 256 partitions), cells per region and the
 * number of regions and partitions of the binned paths, and the positions
 * per chunk (the countBF's cells are read and written once per chunk) with
 * the chunks of this insert.  The batched form's tuner may change a
 * handle's chunk size; this reports the one in use.  carried = 1: a split
 * insert of this size (kc_insert_classify) classifies the first-seen k-mers
 * of the chunks before the last in the last chunk's region pass, from the
 * counters it holds (one hash function, at least 8 counters per cell, and
 * the handle's workspace holds the carried records: 6 bytes per position
 * before the last chunk, allocated by kc_reserve or the insert itself);
 * 0: they are classified by a pass over their flags that rereads their
 * counters. */
#define KC_PATH_DIRECT 0u
#define KC_PATH_BINNED 1u
#define KC_PATH_PARTITIONED 2u
typedef struct {
    uint32_t path;
    uint32_t region_cells;
    uint32_t n_regions;
    uint32_t n_parts;
    uint64_t chunk;
    uint64_t n_chunks;
    uint32_t carried;
    uint32_t reserved;
} kc_plan;
kc_status kc_get_plan(const kc_filter *f, uint64_t n_bases, kc_plan *out);

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
    KC_PHASE_BIN_PART = 16,       /* partitioned path: entries grouped by partition */
    KC_PHASE_PART_COUNT = 17,     /* partitioned path: per-partition region counts */
    KC_PHASE_VALID = 18,          /* binned paths: valid-window bitmap of the call's k */
    KC_PHASE_WINNERS = 19,        /* binned paths, chunks beyond 2^28 positions: first-seen
                                     records -> flag bytes */
    KC_PHASE_COUNT = 20
} kc_phase;

kc_status kc_profile(kc_filter *f, int enable);
/* Time only the phases whose bit (1u << kc_phase) is set in mask; 0 turns
 * timing off.  Fewer events per call: two per timed kernel launch. */
kc_status kc_profile_phases(kc_filter *f, uint32_t mask);
kc_status kc_profile_read(kc_filter *f, double *ms, uint64_t *launches, uint32_t n_phases);
const char *kc_phase_name(uint32_t phase);

/* ------------------------------------------------------------------------
 * Batched form: many independent read sets, each with its own countBF, k and
 * tau, inserted (and classified) together by one call.  The result for every
 * set is identical to kc_insert_classify (or kc_insert when trust_dev is
 * NULL) on that set's reads alone.
 *
 * All sets' reads live in one buffer (reads_dev, offsets_dev as for
 * kc_insert, n_bases bytes in total).  Set i owns bases
 * [first_base, first_base + n_bases) of it, which must hold whole reads:
 * first_base a multiple of 4096, sets sorted by first_base and disjoint
 * (padding between sets must be reads of invalid bases, e.g. 'N', which add
 * no k-mer).  Each set has its own filter handle (at most one set per
 * handle), created on the batch's device.  The whole buffer is ingested once;
 * sets whose countBF spans at most 2048 regions (a region is the largest
 * power-of-two number of cells whose counters number at most 16384: 2048
 * cells at alpha = 8, so at most 32 MB of countBF), that hold at most 2^28
 * bases and use k <= 32 then go through one launch per phase for all of
 * them (the total number of their (base, hash function) pairs must stay
 * below 2^32); every other set (up to k = 64, any countBF kc_insert takes)
 * runs the single-set pipeline over its range of the buffer on one of up to
 * three side streams the call forks from `stream` after the ingest and joins
 * before it returns, each side lane with scratch of its own (held by the
 * batch), so that such sets overlap one another and the fused phases.
 * Outputs per set have the meaning of kc_insert_classify; distinct capacity
 * overflows are sticky in the set's filter (kc_sync on it).
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
#define KC_BATCH_TUNE 4u   /* time the candidate work-item sizes of the fused phases on this
                              input and keep the fastest; with KC_BATCH_RESET also time each
                              side-lane set's whole pipeline at several chunk sizes (positions
                              per pass over its countBF, kc_get_plan) and keep the fastest in
                              its handle */

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

/* ------------------------------------------------------------------------
 * Serving form: a request loop over device-resident countBFs.
 *
 * A session is one countBF with its k and its distinct list, kept on the
 * device across requests; a request inserts a read set into a session
 * (continuing the session's sequential order, so that a session's requests
 * together equal one kc_insert of their concatenated reads) and/or
 * classifies the session's whole distinct list at a threshold (Algorithm 2
 * with Query-II).  Sessions are admitted by device memory: a session opened
 * while the budget is spent waits, with its requests, until closed sessions
 * have released enough; admission is in order of kc_server_open.
 *
 * kc_server_pump() runs the loop once without blocking: it retires finished
 * batches, admits waiting sessions, and issues new batches while a lane is
 * free.  A lane is a slot for one batch in flight with its own staging,
 * copy and compute streams and batched-form scratch; lanes run concurrently
 * on the device.  A batch takes queued requests in arrival order, at most
 * one per session, copies their reads to the lane on its copy stream and
 * runs them on its compute stream: every insert of the batch goes through
 * one kc_batch_insert call (large countBFs and requests on its side lanes),
 * then the classify requests through kc_classify.  A session's requests run
 * in submission order: a lane that takes a request of a session whose
 * previous request is still in flight on another lane waits for it on the
 * device.  Requests that arrive while batches run are copied in and issued
 * as soon as a lane is free, and overlap the batches already running.  A
 * request's outputs do not depend on which other requests share its batch
 * or run beside it.
 *
 * Memory: the server allocates, and frees on close/destroy, each session's
 * countBF (8*X*Y bytes), distinct list (8*distinct_cap bytes, twice that for
 * k > 32), its classification scratch (about 0.17 bytes per key of room) and
 * the per-counter first-seen entries of countBFs too large for the binned
 * path (4 bytes per counter); these count against memory_budget.  The
 * lanes' staging and insert scratch are the server's own and do not.
 * Host memory passed in a request (reads, offsets) must stay valid and
 * unchanged until the request is done; pinned memory lets the copies run
 * asynchronously.  Not thread-safe: one host thread drives a server.
 * ---------------------------------------------------------------------- */
typedef struct kc_server kc_server;

typedef struct {
    uint64_t memory_budget;  /* device bytes for admitted sessions */
    uint64_t lane_bases;     /* staging room of one lane in bases: the largest request */
    uint64_t lane_reads;     /* staging room of one lane in reads */
    uint32_t lane_requests;  /* most requests in one batch (1..4096) */
    uint32_t lanes;          /* batches in flight, 1..8 */
} kc_server_config;

/* request operations (bit set) */
#define KC_OP_INSERT 1u
#define KC_OP_CLASSIFY 2u

typedef struct {
    uint32_t session;
    uint32_t op;                   /* KC_OP_INSERT, KC_OP_CLASSIFY or both (insert first) */
    uint32_t tau;                  /* classification threshold: frequency > tau -> trustworthy */
    uint32_t reserved;             /* 0 */
    const uint8_t *reads_host;     /* ASCII bases; host memory */
    const uint64_t *offsets_host;  /* n_reads + 1 CSR offsets, offsets[0] == 0, non-decreasing */
    uint64_t n_reads;
    uint64_t *trust_dev;           /* classify: device outputs, class_cap keys of room each */
    uint64_t *err_dev;
    uint64_t class_cap;
} kc_request;

typedef struct {
    int32_t status;          /* KC_OK, or KC_ERANGE when the session's distinct list or
                                class_cap overflowed, KC_ENOMEM when the session could not be
                                allocated, KC_EDEVICE on a device error */
    uint32_t done;           /* 1 once the outputs are final */
    uint64_t n_windows;      /* k-mers inserted (valid windows) */
    uint64_t distinct_first; /* this request's first-seen k-mers are the session's distinct */
    uint64_t n_new;          /* keys [distinct_first, distinct_first + n_new) */
    uint64_t n_trust, n_err; /* classify: counts written to trust_dev / err_dev */
    double t_submit, t_issue, t_done;  /* seconds since kc_server_create */
} kc_result;

typedef struct {
    uint64_t session_bytes;      /* admitted sessions' device bytes */
    uint64_t staging_bytes;      /* the lanes' device staging */
    uint32_t sessions_open;      /* admitted */
    uint32_t sessions_waiting;   /* opened, waiting for memory */
    uint64_t requests_done;
    uint64_t batches;            /* lanes issued */
    uint64_t batched_requests;   /* requests inserted through kc_batch_insert (all inserts) */
    uint64_t plain_requests;     /* requests inserted through kc_insert (none since every
                                    insert goes through the batched call) */
    uint32_t max_batch;          /* most requests in one issued lane */
    uint32_t lanes_in_flight_max;  /* most lanes with work on the device at once */
} kc_server_stats;

/* Create a server on the current device.  KC_EINVAL for a bad config. */
kc_status kc_server_create(const kc_server_config *cfg, kc_server **out);
/* Wait for all work, free every session and the staging. */
void kc_server_destroy(kc_server *s);
/* Open a session for a countBF of this layout and k-mer length k (1..64),
 * with room for distinct_cap distinct k-mers; *session receives its id at once, and
 * the session is admitted when its bytes fit the budget.  KC_ENOMEM if they
 * exceed the whole budget, KC_EINVAL for a bad layout or k. */
kc_status kc_server_open(kc_server *s, const kc_layout *layout, uint32_t k,
                         uint64_t distinct_cap, uint32_t *session);
/* Close a session: after its submitted requests are done its memory is
 * released; further submits to it fail with KC_ESTATE. */
kc_status kc_server_close(kc_server *s, uint32_t session);
/* Queue a request; *ticket identifies it.  Validates the request on the host
 * (offsets monotone and within the staging room, outputs present) and
 * returns KC_EINVAL / KC_ERANGE without queuing it otherwise. */
kc_status kc_server_submit(kc_server *s, const kc_request *req, uint64_t *ticket);
/* Run the loop once without blocking; *n_done (may be NULL) receives the
 * number of requests retired by this call. */
kc_status kc_server_pump(kc_server *s, uint32_t *n_done);
/* Pump until the ticket's request is done (ticket 0: until all are). */
kc_status kc_server_wait(kc_server *s, uint64_t ticket);
/* The ticket's result so far (done == 0 while queued or running).  Results
 * are kept until kc_server_release or kc_server_destroy. */
kc_status kc_server_result(const kc_server *s, uint64_t ticket, kc_result *out);
/* Forget a done request's result; its ticket becomes unknown.  KC_ESTATE
 * while the request is not done, KC_EINVAL for an unknown ticket. */
kc_status kc_server_release(kc_server *s, uint64_t ticket);
/* Copy n keys of a session's distinct list, from index first, to host
 * memory (waits for the server's issued work); keys of k > 32 take two words
 * each (2n words).  KC_ERANGE past the end. */
kc_status kc_server_read_distinct(kc_server *s, uint32_t session, uint64_t first, uint64_t n,
                                  uint64_t *dst_host);
/* Copy a session's countBF cells (8*X*Y bytes) to host memory (waits). */
kc_status kc_server_read_words(kc_server *s, uint32_t session, uint64_t *dst_host);
kc_status kc_server_stats_get(const kc_server *s, kc_server_stats *out);
/* Seconds since kc_server_create on the server's clock. */
double kc_server_now(const kc_server *s);

#ifdef __cplusplus
}
#endif

#endif /* KMERCO_H */
