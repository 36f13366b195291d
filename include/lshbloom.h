/*
 * lshbloom.h — C ABI of the MI355X (gfx950) LSHBloom hot path.
 *
 * LSHBloom ("LSHBloom: Internet-Scale Text Deduplication", arXiv 2411.04257)
 * answers the streaming question of Section 2.1: for each document d_i of a
 * stream, is some earlier document d_j (j < i) similar to it?  The hot path
 * has three steps, all run by hand-written HIP kernels behind this ABI:
 *
 *   1. MinHash (Section 2.2): a document is the set of its w-token shingles;
 *      signature row i is min over shingles of h_i(shingle hash).
 *   2. Band keys (Sections 2.3, 4.1): rows are grouped in b bands of r rows
 *      and each band is reduced to one 64-bit key by a sum of per-row hashes
 *      mod N, N = 2^64.
 *   3. One Bloom filter per band (Sections 2.4, 4, 4.2): a document is flagged
 *      when, in some band, all k filter bits of its key are already set; then
 *      its bits are set in every band.  Flags are exactly those of processing
 *      the documents one at a time in stream order (Section 4.4.2).
 *
 * Exact definitions (bit-for-bit; every GPU result equals the sequential
 * definition below, including the final filter bits):
 *   - shingles of a document of L tokens: tokens[t..t+w-1] for t = 0..L-w when
 *     L >= w; one shingle of all L tokens when 1 <= L < w; none when L = 0.
 *   - shingle hash x: SHA-1 (FIPS 180-4) of the shingle's tokens as
 *     little-endian uint32 bytes; x = first four digest bytes, little-endian.
 *   - h_i(x) = ((a_i * x + b_i) mod (2^61 - 1)) mod 2^32, exact; an empty
 *     document has the all-0xFFFFFFFF signature.
 *   - coefficients: SplitMix64 stream from `seed` (state += 0x9E3779B97F4A7C15,
 *     output = the standard SplitMix64 finalizer of the state); a_0..a_{P-1}
 *     are successive outputs >> 3, redrawn while 0 or >= 2^61-1; then
 *     b_0..b_{P-1} the same, redrawn while >= 2^61-1; then salt_M, salt_1,
 *     salt_2 are three raw outputs.
 *   - band key K_j = sum_{t<r} fmix64((sig[j*r+t] | t << 32) ^ salt_M)
 *     mod 2^64, where fmix64 is the SplitMix64 finalizer.  Rows from b*r to
 *     P-1 are not used.
 *   - positions: h1 = fmix64(K_j ^ salt_1), h2 = fmix64(K_j ^ salt_2) | 1,
 *     g_l = floor(((h1 + l*h2) mod 2^64) * m / 2^64), l = 0..k-1.
 *   - filter of band j: m bits in m/64 little-endian uint64 words; bit g is
 *     bit (g & 63) of word g >> 6.
 *   - sizing (Section 4.5): m = 64 * ceil((-(n * ln p) / (ln 2 * ln 2)) / 64)
 *     evaluated in IEEE double in that order, with n = expected_n and
 *     p = fp_rate, the per-band false-positive rate; k = max(1,
 *     floor(-log2(p) + 0.5)).  The effective rate over b bands is
 *     p_eff = 1 - (1 - p)^b (Section 4.3).
 *
 * Memory: every pointer argument named d_* is a device pointer in the
 * caller's ownership (for example a torch CUDA tensor's data_ptr()).  The
 * library owns its filters and workspace, allocates them once in create and
 * frees them in destroy; the hot-path calls allocate nothing.
 *
 * Streams: every call is asynchronous on `stream` (a hipStream_t; NULL is the
 * null stream).  Calls that read or change the filters of one handle are
 * serialised in host call order whatever stream they use: each waits for the
 * previous one (an event kept in the handle).  Document order is therefore
 * host call order, then index within a call.  lshbloom_minhash touches no
 * handle state and may run concurrently on any stream.
 *
 * Errors: functions returning int give LSHBLOOM_OK (0) or a negative code;
 * lshbloom_last_error() returns a message for the calling thread's last
 * failure.  Invalid arguments are rejected before anything is launched.  A
 * device error inside a filter-changing call poisons the handle (its filters
 * may be half-written): every later call on it returns LSHBLOOM_EPOISONED.
 * The kernels also check their own bookkeeping (record totals, table
 * capacities, that every probed clear bit was registered) and raise bits of
 * a device status word when it fails; each filter-changing call ends with an
 * asynchronous copy of that word to host memory.  The first call on the
 * handle that finds it nonzero (at the latest, the first one made after the
 * host has waited for the failing call: lshbloom_sync, lshbloom_pipeline_wait
 * or _poll, lshbloom_count_set_bits, lshbloom_save, or a read_filters into
 * pageable memory) poisons the handle and returns LSHBLOOM_EDEVICE; the
 * flags of calls from the failing one on are not to be trusted.
 * Device-side data (offsets, tokens) is trusted: offsets must be
 * non-decreasing and in bounds of d_tokens.
 *
 * Thread safety: one handle may be used from several host threads; calls are
 * serialised internally.
 */
#ifndef LSHBLOOM_H
#define LSHBLOOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lshbloom lshbloom_t;
typedef void *lshbloom_stream_t; /* a hipStream_t */

enum {
  LSHBLOOM_OK = 0,
  LSHBLOOM_EINVAL = -1,    /* bad argument; nothing was launched */
  LSHBLOOM_ENOMEM = -2,    /* device memory (or the HBM budget) exhausted */
  LSHBLOOM_EHIP = -3,      /* HIP runtime error; message in last_error */
  LSHBLOOM_EPOISONED = -4, /* an earlier device error left the filters indeterminate */
  LSHBLOOM_EIO = -5,       /* a file could not be opened, read or written */
  LSHBLOOM_EDEVICE = -6,   /* a kernel reported an internal inconsistency; the handle is poisoned */
};

/* Limits of this implementation. */
#define LSHBLOOM_MAX_NUM_PERM 512u        /* signature width P */
#define LSHBLOOM_MAX_BANDS 64u            /* b */
#define LSHBLOOM_MAX_SHINGLE_WIDTH 13u    /* w: one shingle fits one SHA-1 block */
#define LSHBLOOM_MAX_M_BITS 0xFFFFFFFFC0ull /* m < 2^40 bits per band */

typedef struct lshbloom_params {
  uint32_t num_perm;      /* P >= 1, <= LSHBLOOM_MAX_NUM_PERM */
  uint32_t bands;         /* b >= 1, <= LSHBLOOM_MAX_BANDS */
  uint32_t rows;          /* r >= 1, b * r <= P */
  uint64_t expected_n;    /* n >= 1: documents the filters are sized for */
  double fp_rate;         /* per-band false-positive rate p, 0 < p < 1 */
  uint64_t seed;          /* coefficient and salt stream seed */
  uint32_t shingle_width; /* w, 1..LSHBLOOM_MAX_SHINGLE_WIDTH; 0 means 5 */
  uint64_t hbm_budget;    /* bytes the handle may allocate; 0 = no limit */
  uint64_t chunk_docs;    /* documents per in-order query-insert chunk; 0 = automatic */
  uint32_t qi_mode;       /* query-insert algorithm: 0 automatic, 1 direct (first-setter hash table
                             with device atomics), 2 binned (probes partitioned by bit range; one
                             workgroup owns each range); results are identical */
  uint64_t workspace_budget; /* bytes for the binned query-insert's workspace; 0 = 4 GiB */
} lshbloom_params_t;

typedef struct lshbloom_info {
  uint32_t num_perm, bands, rows, shingle_width;
  uint32_t k;               /* probes per band */
  uint64_t m_bits;          /* bits per band */
  uint64_t words_per_band;  /* m_bits / 64 */
  uint64_t filter_bytes;    /* bands * m_bits / 8 */
  uint64_t workspace_bytes; /* device bytes besides the filters */
  uint64_t chunk_docs;      /* documents per direct query-insert chunk */
  uint64_t binned_chunk_docs; /* documents per binned query-insert chunk */
  double fp_rate;           /* per-band p */
  double p_eff;             /* 1 - (1 - p)^bands (Section 4.3) */
  uint64_t docs_inserted;   /* documents inserted so far (host count of calls) */
  uint64_t seed;
  int poisoned;
  uint32_t device_status; /* 0 unless a kernel detected an internal inconsistency */
  uint64_t general_path_bins; /* binned query-insert: bins whose records or bits outgrew the
                                 one-wave LDS tables and took the global-memory path, summed
                                 over the handle's calls (a diagnostic; results are the same) */
} lshbloom_info_t;

/* Create an index of `bands` empty Bloom filters (Section 4: one per band)
 * sized for expected_n documents at per-band rate fp_rate (Section 4.5), with
 * shingle width 5.  Allocates the filters and workspace on the current HIP
 * device.  Returns NULL on error (message in lshbloom_last_error). */
lshbloom_t *lshbloom_create(uint32_t num_perm, uint32_t bands, uint32_t rows, uint64_t expected_n, double fp_rate,
                            uint64_t seed);

/* As lshbloom_create, with every parameter of lshbloom_params_t. */
lshbloom_t *lshbloom_create_ex(const lshbloom_params_t *params);

/* Free the filters and workspace (after synchronising the handle's last
 * call).  NULL is a no-op. */
void lshbloom_destroy(lshbloom_t *h);

/* MinHash signatures of a CSR batch (Section 2.2).
 *   d_offsets: int64 [n_docs + 1], non-decreasing; document d owns
 *              d_tokens[d_offsets[d] .. d_offsets[d+1]).
 *   d_tokens:  uint32 token ids.
 *   d_sigs:    uint32 [n_docs][num_perm] row-major output.
 * n_docs = 0 is a no-op.  Stateless: runs concurrently with other calls. */
int lshbloom_minhash(lshbloom_t *h, const int64_t *d_offsets, const uint32_t *d_tokens, int64_t n_docs,
                     uint32_t *d_sigs, lshbloom_stream_t stream);

/* Query then insert a batch of signatures in stream order (Sections 2.1, 4.1,
 * 4.2, 4.4.2): d_flags[i] = 1 iff, for some band, all k bits of document i's
 * key were set by the filters' earlier contents or by documents 0..i-1 of
 * this batch; then every band's bits of every document are set.
 *   d_sigs:  uint32 [n_docs][num_perm] (for example lshbloom_minhash output).
 *   d_flags: uint8 [n_docs] output, 0 or 1.
 * n_docs = 0 is a no-op. */
int lshbloom_query_insert(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                          lshbloom_stream_t stream);

/* Allocation-free lshbloom_query_insert, for callers that cannot allocate
 * device memory while they run (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result, ordering
 * and errors as lshbloom_query_insert; it runs the direct (first-setter
 * table) algorithm with its table and per-pair arrays in a fixed
 * device array of the library (33 MiB per GPU, held until the process ends),
 * not in the handle's workspace, and calls no allocating routine.  At most
 * LSHBLOOM_NOALLOC_MAX_DOCS documents per call (LSHBLOOM_EINVAL beyond);
 * larger calls are processed in chunks that fit the array.  Every call of
 * this function on one GPU uses the same array: calls of it that overlap
 * on one GPU (two handles driven from different streams without ordering
 * between them) race and give wrong flags; calls on one handle are ordered
 * by the handle. */
#define LSHBLOOM_NOALLOC_MAX_DOCS 65536u
int lshbloom_query_insert_noalloc(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                                  lshbloom_stream_t stream);

/* Query only (Section 4.2): flags against the filters as they are; nothing is
 * inserted and documents of the batch do not see each other. */
int lshbloom_query(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                   lshbloom_stream_t stream);

/* Insert only (Section 4.1): set every band's bits of every document. */
int lshbloom_insert(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, lshbloom_stream_t stream);

/* Query then insert from band keys (Section 4.1 reduces each band of a
 * signature to one integer, the key; the filters see only keys):
 *   d_keys:  uint64 [n_docs][bands], e.g. lshbloom_band_keys or
 *            lshbloom_band_keys61 output.
 *   d_flags: uint8 [n_docs] output.
 * Same order, ordering and errors as lshbloom_query_insert, which equals
 * this call on lshbloom_band_keys of its signatures. */
int lshbloom_query_insert_keys(lshbloom_t *h, const uint64_t *d_keys, int64_t n_docs, uint8_t *d_flags,
                               lshbloom_stream_t stream);

/* Wide-value MinHash (Section 4.5: the index size does not depend on the
 * width of the MinHash values): d_sigs uint64 [n_docs][num_perm], each value
 * the whole permutation value (a_i x + b_i) mod (2^61 - 1) minimised over the
 * document's shingles (x the same 32-bit shingle hash); an empty document
 * gives 2^64 - 1 throughout.  Same CSR input and ordering as lshbloom_minhash. */
int lshbloom_minhash61(lshbloom_t *h, const int64_t *d_offsets, const uint32_t *d_tokens, int64_t n_docs,
                       uint64_t *d_sigs, lshbloom_stream_t stream);

/* Band keys of wide signatures, uint64 [n_docs][bands]: per band the sum
 * mod 2^64 over its rows t of fmix64((v + t * 0x9E3779B97F4A7C15) ^ salt_M). */
int lshbloom_band_keys61(lshbloom_t *h, const uint64_t *d_sigs, int64_t n_docs, uint64_t *d_keys,
                         lshbloom_stream_t stream);

/* Band keys K_j of each document (Section 4.1), uint64 [n_docs][bands]. */
int lshbloom_band_keys(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint64_t *d_keys,
                       lshbloom_stream_t stream);

/* Copy nbytes of the filter words, starting at byte `offset` of the
 * band-major array (band j's words start at byte j * m_bits / 8), to `dst`
 * (host or device memory), ordered after the handle's previous calls.
 * Synchronous when dst is pageable host memory. */
int lshbloom_read_filters(lshbloom_t *h, void *dst, uint64_t offset, uint64_t nbytes, lshbloom_stream_t stream);

/* Overwrite filter bytes from `src` (host or device memory); sets
 * docs_inserted to `docs_inserted` when it is not UINT64_MAX.  Used to load a
 * saved index or a preloaded state. */
int lshbloom_write_filters(lshbloom_t *h, const void *src, uint64_t offset, uint64_t nbytes,
                           uint64_t docs_inserted, lshbloom_stream_t stream);

/* Save the index to a file (Section 4.5: the index is a persistent bit
 * array): an 80-byte little-endian header
 *   "LSHBLM01", num_perm, bands, rows, shingle_width (u32 each),
 *   expected_n (u64), fp_rate (f64), seed, m_bits (u64), k, 0 (u32 each),
 *   docs_inserted, words_per_band (u64 each)
 * then the band-major filter words (u64 each), after the handle's previous
 * calls.  The words pass through a 64 MB pinned host buffer, so filters far
 * larger than host memory can be saved.  Synchronous.  LSHBLOOM_EIO if the
 * file cannot be created or written (a partial file may remain). */
int lshbloom_save(lshbloom_t *h, const char *path, lshbloom_stream_t stream);

/* Load a file written by lshbloom_save into a handle created with the same
 * num_perm, bands, rows, shingle_width, seed, m_bits and k (LSHBLOOM_EINVAL
 * otherwise, filters untouched); replaces the filters and docs_inserted.
 * Synchronous.  LSHBLOOM_EIO if the file is missing or short (the filters may
 * then be partly overwritten: the handle is poisoned). */
int lshbloom_load(lshbloom_t *h, const char *path, lshbloom_stream_t stream);

/* Number of set bits of each band's filter, written to out[bands] (host
 * memory), counted after the handle's previous calls; synchronous.  At the
 * k of Section 4.5's sizing about half of a filter's bits are set after
 * expected_n documents, so the count tracks how full the index is; the
 * difference over a call is the number of bits that call set. */
int lshbloom_count_set_bits(lshbloom_t *h, uint64_t *out, lshbloom_stream_t stream);

/* Parameters, sizes and counters of the handle. */
int lshbloom_info(const lshbloom_t *h, lshbloom_info_t *out);

/* Wait for the handle's outstanding calls, then report their outcome:
 * LSHBLOOM_OK, LSHBLOOM_EDEVICE if a kernel raised the device status word
 * (the handle is then poisoned), LSHBLOOM_EPOISONED if it already was, or
 * LSHBLOOM_EHIP for a runtime error. */
int lshbloom_sync(lshbloom_t *h);

/* Per-band rate p that gives an effective rate p_eff over `bands` bands,
 * p = 1 - (1 - p_eff)^(1/bands) (Section 4.3). */
double lshbloom_p_band_from_eff(double p_eff, uint32_t bands);

/* (b, r) minimising w_fp * FP_lsh + w_fn * FN_lsh (Section 4.3, Eq. 1-2) over
 * b * r <= num_perm; returns LSHBLOOM_EINVAL for bad arguments. */
int lshbloom_optimal_bands(double threshold, uint32_t num_perm, double w_fp, double w_fn, uint32_t *bands,
                           uint32_t *rows);

/* ------------------------------------------------------------------------ */
/* Batched form: a host-to-host pipeline around one handle.                  */
/* ------------------------------------------------------------------------ */

typedef struct lshbloom_pipeline lshbloom_pipeline_t;

typedef struct lshbloom_pipeline_params {
  uint64_t max_docs;          /* capacity: documents per submitted batch */
  uint64_t max_tokens;        /* capacity: tokens per submitted batch */
  uint32_t n_buckets;         /* 1..4 MinHash length buckets; 0 = chosen by the autotuner (or 1) */
  uint64_t bucket_edges[3];   /* token-length edges: bucket b holds lengths in [edge[b-1], edge[b]) */
  uint32_t waves_per_cu[4];   /* persistent MinHash waves per compute unit, per bucket; 0 = sized by the
                                 bucket's tokens (one wave per ~2,048, 16 to 256 per compute unit) */
  uint32_t use_graph;         /* 1: capture each slot's device work in a hipGraph and replay it */
  uint32_t autotune;          /* 1: on the first batch, time candidate bucket edges and grid sizes */
  const char *tune_cache;     /* text file for autotuned choices (read, then appended); NULL = none */
} lshbloom_pipeline_params_t;

typedef struct lshbloom_pipeline_info {
  uint32_t n_buckets;
  uint64_t bucket_edges[3];
  uint32_t waves_per_cu[4];
  int tuned;
  float tune_best_ms;          /* MinHash time of the chosen configuration on the tuning batch */
  uint64_t batches;
  uint64_t graph_launches, graph_updates, graph_instantiations;
  uint64_t timed_batches;      /* non-empty batches collected so far */
  double minhash_ms_total;     /* their MinHash stages (pre-fill + MinHash launches), summed, in ms */
  double qi_ms_total;          /* their query-insert kernels, summed, in ms (HIP events on the query-insert stream) */
} lshbloom_pipeline_info_t;

/* Create a pipeline that feeds `h` (which must outlive it).  It owns two
 * slots of pinned host staging and device buffers sized by the capacities,
 * and two streams of its own.  NULL on error. */
lshbloom_pipeline_t *lshbloom_pipeline_create(lshbloom_t *h, const lshbloom_pipeline_params_t *params);

/* Submit one CSR batch from host memory: offsets int64 [n_docs + 1] index
 * h_tokens (checked on the host: non-decreasing, within max_tokens); the
 * batch's flags (Section 2.1 decisions, uint8) are written to h_flags by
 * lshbloom_pipeline_wait of the returned ticket (>= 0), or when the slot is
 * reused two submissions later.  h_tokens and h_flags must stay valid and
 * unmodified until then.  Documents are ordered by submission, then index;
 * the call returns once the batch is enqueued (the host work of the next
 * batch overlaps this one's GPU work).  Negative return = error code. */
int64_t lshbloom_pipeline_submit(lshbloom_pipeline_t *pl, const int64_t *h_offsets, const uint32_t *h_tokens,
                                 int64_t n_docs, uint8_t *h_flags);

/* Block until the batch of `ticket` is done and its flags are in its h_flags.
 * Returns LSHBLOOM_EDEVICE (flags delivered but not to be trusted; the handle
 * is poisoned) when a kernel of the handle reported an inconsistency. */
int lshbloom_pipeline_wait(lshbloom_pipeline_t *pl, int64_t ticket);

/* Non-blocking: 1 if the batch of `ticket` is done (its flags are then in
 * its h_flags), 0 if not yet, negative on error. */
int lshbloom_pipeline_poll(lshbloom_pipeline_t *pl, int64_t ticket);

/* Chosen buckets, grid sizes, graph counters and stage times. */
int lshbloom_pipeline_info(const lshbloom_pipeline_t *pl, lshbloom_pipeline_info_t *out);

/* Finish outstanding batches (delivering their flags) and free the pipeline. */
void lshbloom_pipeline_destroy(lshbloom_pipeline_t *pl);

/* ---- Exact MinHashLSH band index (the comparison baseline) ----------------
 *
 * The traditional index that LSHBloom replaces (Section 2.3, "MinHashLSH
 * for Text Deduplication"; Section 4): per band, a hash table keyed by the band's
 * r signature values, compared exactly.  Document i is flagged iff, for some
 * band j, its r values of band j equal those of an earlier document (of an
 * earlier call, or 0..i-1 of this call); every document is then inserted.
 * On the same stream LSHBloom's flags contain these flags (equal band values
 * give equal band keys); the difference is the Bloom filters' false positives
 * and band-key collisions (Section 4.3, Eq. 3).  Device memory, allocated by create:
 * per band 2^ceil(log2(2 capacity)) slots of 12 + 4 r bytes. */
typedef struct lshbloom_exact lshbloom_exact_t;

/* capacity_docs: documents the index can hold over its life, 1..2^30 (a call
 * that would exceed it returns LSHBLOOM_EINVAL with nothing launched).
 * fp_bits: bits of the 64-bit fingerprint of a band's values that pick its
 * slot and prefilter comparisons (0 = 64); fewer bits only make different
 * values share fingerprints more often, which stays exact but slower (for
 * tests).  NULL on error (message in lshbloom_last_error). */
lshbloom_exact_t *lshbloom_exact_create(uint32_t num_perm, uint32_t bands, uint32_t rows, uint64_t capacity_docs,
                                        uint32_t fp_bits);

/* Frees the tables after the index's outstanding work.  NULL is a no-op. */
void lshbloom_exact_destroy(lshbloom_exact_t *x);

/* Query then insert in stream order, as lshbloom_query_insert: d_sigs uint32
 * [n_docs][num_perm] and d_flags uint8 [n_docs] are device pointers owned by
 * the caller; asynchronous on stream; calls on one index are ordered by host
 * call order.  n_docs = 0 is a no-op. */
int lshbloom_exact_query_insert(lshbloom_exact_t *x, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                                lshbloom_stream_t stream);

/* Host outputs (each may be NULL): documents inserted, bytes of the tables,
 * and the number of (document, band) pairs so far whose fingerprint was
 * shared with different band values (placed exactly by full comparison).
 * Synchronous when fp_shared is requested. */
int lshbloom_exact_stats(lshbloom_exact_t *x, uint64_t *docs_inserted, uint64_t *table_bytes, uint64_t *fp_shared);

/* Message for the calling thread's last failure ("" if none). */
const char *lshbloom_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LSHBLOOM_H */
