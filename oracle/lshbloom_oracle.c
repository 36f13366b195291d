/*
 * LSHBloom CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential reference of the LSHBloom hot path (MinHash
 * signatures over shingles, band keys, one Bloom filter per band, query then
 * insert in stream order).  It exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can check the GPU library against an
 * independently written definition.  Nothing in the product path may call it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Paper: "LSHBloom: Internet-Scale Text Deduplication" (arXiv 2411.04257).
 *   §2.1   stream semantics: F(d_i) = 1 iff some earlier document is similar.
 *   §2.2   shingle sets and MinHash: P[min-hash equal] = Jaccard.
 *   §2.3   banding of the signature matrix into b bands of r rows.
 *   §2.4   Bloom filter: m-bit array, k hash positions, insert sets bits,
 *          query = all k bits set, no false negatives.
 *   §4.1   insertion: one Bloom filter per band; a band of r values is
 *          reduced to one integer by a sum of per-row hashes mod N.
 *   §4.2   querying: a hit in any band marks the document a duplicate.
 *   §4.3   error rate: p_eff = 1-(1-p)^b; FP/FN integrals (Eq. 1-2).
 *   §4.4.2 filter writes are sequential in stream order.
 *   §4.5   filter size m = -n ln p / (ln 2)^2 bits.
 *
 * Where the paper leaves a choice open, the reading taken here is the one the
 * design notes list (shingle width w, SHA-1 shingle hash truncated to its
 * first four digest bytes read little-endian, exact (a*x+b) mod 2^61-1
 * permutations truncated to 32 bits, SplitMix64 coefficient stream, 64-bit
 * mixed per-row band-key summands with N = 2^64, per-band fp_rate, double
 * hashing with multiply-high range reduction, little-endian 64-bit filter
 * words, every document inserted).
 *
 * Every function below states the passage or published definition it follows.
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_P61 ((uint64_t)0x1FFFFFFFFFFFFFFFull) /* 2^61 - 1 */

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* SHA-1 exactly as FIPS 180-4 §5.1.1 (padding), §6.1.2 (computation).       */
/* The paper's universal hash for shingles is SHA-1 (§4.1).                  */
/* ------------------------------------------------------------------------ */
static uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

void ora_sha1(const uint8_t *msg, uint64_t len, uint8_t digest[20]) {
  uint32_t H[5] = {0x67452301u, 0xEFCDAB89u, 0x98BADCFEu, 0x10325476u, 0xC3D2E1F0u};
  /* padded length: smallest multiple of 64 bytes holding msg, 0x80 and the
     64-bit big-endian bit length */
  uint64_t total = ((len + 8) / 64 + 1) * 64;
  uint64_t bitlen = len * 8;
  for (uint64_t off = 0; off < total; off += 64) {
    uint8_t block[64];
    for (int i = 0; i < 64; ++i) {
      uint64_t p = off + (uint64_t)i;
      uint8_t byte;
      if (p < len)
        byte = msg[p];
      else if (p == len)
        byte = 0x80;
      else if (p >= total - 8)
        byte = (uint8_t)(bitlen >> (8 * (total - 1 - p)));
      else
        byte = 0;
      block[i] = byte;
    }
    uint32_t W[80];
    for (int t = 0; t < 16; ++t)
      W[t] = ((uint32_t)block[4 * t] << 24) | ((uint32_t)block[4 * t + 1] << 16) |
             ((uint32_t)block[4 * t + 2] << 8) | (uint32_t)block[4 * t + 3];
    for (int t = 16; t < 80; ++t) W[t] = rotl32(W[t - 3] ^ W[t - 8] ^ W[t - 14] ^ W[t - 16], 1);
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4];
    for (int t = 0; t < 80; ++t) {
      uint32_t f, K;
      if (t < 20) {
        f = (b & c) ^ (~b & d); /* Ch */
        K = 0x5A827999u;
      } else if (t < 40) {
        f = b ^ c ^ d; /* Parity */
        K = 0x6ED9EBA1u;
      } else if (t < 60) {
        f = (b & c) ^ (b & d) ^ (c & d); /* Maj */
        K = 0x8F1BBCDCu;
      } else {
        f = b ^ c ^ d; /* Parity */
        K = 0xCA62C1D6u;
      }
      uint32_t T = rotl32(a, 5) + f + e + K + W[t];
      e = d;
      d = c;
      c = rotl32(b, 30);
      b = a;
      a = T;
    }
    H[0] += a;
    H[1] += b;
    H[2] += c;
    H[3] += d;
    H[4] += e;
  }
  for (int i = 0; i < 5; ++i) {
    digest[4 * i] = (uint8_t)(H[i] >> 24);
    digest[4 * i + 1] = (uint8_t)(H[i] >> 16);
    digest[4 * i + 2] = (uint8_t)(H[i] >> 8);
    digest[4 * i + 3] = (uint8_t)H[i];
  }
}

/* Shingle hash (§4.1 names SHA-1; §4.3 uses 32-bit hash values): the shingle's
   tokens as little-endian uint32 bytes, SHA-1, first four digest bytes read
   as a little-endian uint32. */
uint32_t ora_shingle_hash(const uint32_t *tok, uint32_t len) {
  uint8_t buf[4 * 64];
  uint8_t *bytes = len <= 64 ? buf : (uint8_t *)malloc(4 * (size_t)len);
  for (uint32_t i = 0; i < len; ++i) {
    bytes[4 * i] = (uint8_t)tok[i];
    bytes[4 * i + 1] = (uint8_t)(tok[i] >> 8);
    bytes[4 * i + 2] = (uint8_t)(tok[i] >> 16);
    bytes[4 * i + 3] = (uint8_t)(tok[i] >> 24);
  }
  uint8_t dg[20];
  ora_sha1(bytes, 4 * (uint64_t)len, dg);
  if (bytes != buf) free(bytes);
  return (uint32_t)dg[0] | ((uint32_t)dg[1] << 8) | ((uint32_t)dg[2] << 16) | ((uint32_t)dg[3] << 24);
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014): state += golden gamma, output is the */
/* state passed through the variant-13 finalizer.                            */
/* ------------------------------------------------------------------------ */
uint64_t ora_fmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t ora_splitmix64_next(uint64_t *state) {
  *state += 0x9E3779B97F4A7C15ull;
  return ora_fmix64(*state);
}

/* ------------------------------------------------------------------------ */
/* MinHash permutation (§2.2, §4.1): h_i(x) = ((a_i x + b_i) mod (2^61-1))    */
/* mod 2^32, computed exactly in 128-bit arithmetic.                         */
/* ------------------------------------------------------------------------ */
uint32_t ora_perm(uint64_t a, uint64_t b, uint32_t x) {
  u128 v = (u128)a * (u128)x + (u128)b;
  return (uint32_t)(uint64_t)(v % (u128)ORA_P61);
}

/* MinHash signature of one document (§2.2): sig[i] = min over the document's
   shingle set of h_i(shingle hash).  A document of L >= w tokens has the
   shingles tokens[t..t+w-1], t = 0..L-w; 1 <= L < w gives one shingle of all
   L tokens; L = 0 gives the empty set and the signature of all 0xFFFFFFFF. */
void ora_minhash_doc(const uint32_t *tok, int64_t L, uint32_t w, uint32_t num_perm,
                     const uint64_t *a, const uint64_t *b, uint32_t *sig) {
  for (uint32_t i = 0; i < num_perm; ++i) sig[i] = 0xFFFFFFFFu;
  if (L <= 0) return;
  int64_t n_sh = L >= (int64_t)w ? L - (int64_t)w + 1 : 1;
  uint32_t sh_len = L >= (int64_t)w ? w : (uint32_t)L;
  for (int64_t t = 0; t < n_sh; ++t) {
    uint32_t x = ora_shingle_hash(tok + t, sh_len);
    for (uint32_t i = 0; i < num_perm; ++i) {
      uint32_t v = ora_perm(a[i], b[i], x);
      if (v < sig[i]) sig[i] = v;
    }
  }
}

/* Band key (§4.1, band hash equation): K_j = sum over the r rows of band j of
   h(row value, row index) mod N with N = 2^64, where the per-row summand is
   the SplitMix64 finalizer of (value | row << 32) xor salt_M. */
uint64_t ora_band_key(const uint32_t *sig, uint32_t band, uint32_t rows, uint64_t salt_m) {
  uint64_t K = 0;
  for (uint32_t t = 0; t < rows; ++t) {
    uint64_t v = (uint64_t)sig[(uint64_t)band * rows + t] | ((uint64_t)t << 32);
    K += ora_fmix64(v ^ salt_m);
  }
  return K;
}

/* Bloom positions for one key (§2.4: k hash functions into the m-bit array):
   double hashing g_l = h1 + l*h2 (Kirsch & Mitzenmacher 2006) mapped to
   [0, m) by the exact multiply-high floor(g * m / 2^64) (Lemire 2019). */
void ora_positions(uint64_t key, uint64_t salt1, uint64_t salt2, uint64_t m, uint32_t k, uint64_t *g) {
  uint64_t h1 = ora_fmix64(key ^ salt1);
  uint64_t h2 = ora_fmix64(key ^ salt2) | 1ull;
  for (uint32_t l = 0; l < k; ++l) {
    uint64_t h = h1 + (uint64_t)l * h2;
    g[l] = (uint64_t)(((u128)h * (u128)m) >> 64);
  }
}

/* Filter sizing (§4.5): m = -n ln p / (ln 2)^2 bits, rounded up to a whole
   number of 64-bit words; k = max(1, round(-log2 p)) probes (the optimum
   (m/n) ln 2 for this m).  p is the per-band false-positive rate. */
int ora_params(uint64_t n, double p, uint64_t *m_bits, uint32_t *k) {
  if (n == 0 || !(p > 0.0) || !(p < 1.0)) return -1;
  double bits = -((double)n * log(p)) / (log(2.0) * log(2.0));
  double words = ceil(bits / 64.0);
  *m_bits = (uint64_t)words * 64ull;
  double kk = floor(-log2(p) + 0.5);
  *k = kk < 1.0 ? 1u : (uint32_t)kk;
  return 0;
}

/* §4.3: the per-band rate p that gives an effective rate p_eff over b bands,
   p = 1 - (1 - p_eff)^(1/b), and its inverse p_eff = 1 - (1 - p)^b; written
   with expm1/log1p so that rates near 1e-10 keep full double precision. */
double ora_p_band_from_eff(double p_eff, uint32_t bands) { return -expm1(log1p(-p_eff) / (double)bands); }
double ora_p_eff_from_band(double p, uint32_t bands) { return -expm1((double)bands * log1p(-p)); }

/* §4.3 Eq. 1-2: FP_lsh = int_0^T 1-(1-t^r)^b dt, FN_lsh = int_T^1 (1-t^r)^b dt,
   by composite Simpson's rule on 2*1000 panels. */
static double curve(double t, uint32_t b, uint32_t r) { return 1.0 - pow(1.0 - pow(t, (double)r), (double)b); }

static double simpson(double lo, double hi, uint32_t b, uint32_t r, int false_neg) {
  const int n = 2000;
  double h = (hi - lo) / n, s = 0.0;
  for (int i = 0; i <= n; ++i) {
    double t = lo + h * i;
    double y = false_neg ? 1.0 - curve(t, b, r) : curve(t, b, r);
    double wgt = (i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0);
    s += wgt * y;
  }
  return s * h / 3.0;
}

double ora_fp_lsh(double T, uint32_t b, uint32_t r) { return simpson(0.0, T, b, r, 0); }
double ora_fn_lsh(double T, uint32_t b, uint32_t r) { return simpson(T, 1.0, b, r, 1); }

/* (b, r) choice (§4.3, following the cited LSH Ensemble tuning): over all
   b, r >= 1 with b*r <= num_perm, minimise w_fp*FP_lsh + w_fn*FN_lsh; ties
   keep the first (smallest b) found. */
void ora_optimal_br(double T, uint32_t num_perm, double w_fp, double w_fn, uint32_t *best_b, uint32_t *best_r) {
  double best = INFINITY;
  *best_b = 1;
  *best_r = 1;
  for (uint32_t b = 1; b <= num_perm; ++b) {
    for (uint32_t r = 1; b * r <= num_perm; ++r) {
      double err = w_fp * ora_fp_lsh(T, b, r) + w_fn * ora_fn_lsh(T, b, r);
      if (err < best) {
        best = err;
        *best_b = b;
        *best_r = r;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* The index: b Bloom filters, one per band (§4, §4.1), processed in stream   */
/* order (§2.1, §4.4.2).                                                     */
/* ------------------------------------------------------------------------ */
typedef struct ora_index {
  uint32_t num_perm, bands, rows, w;
  uint64_t expected_n;
  double fp_rate;
  uint64_t seed;
  uint64_t m_bits;
  uint32_t k;
  uint64_t *a, *b;
  uint64_t salt_m, salt1, salt2;
  uint64_t words_per_band;
  uint64_t *filters; /* bands * words_per_band little-endian uint64 words */
  uint64_t docs_inserted;
} ora_index;

/* Coefficient stream: SplitMix64 from `seed`; a_0..a_{P-1} take the top 61
   bits of successive outputs, rejecting 0 and values >= 2^61-1; then
   b_0..b_{P-1} the same, rejecting only values >= 2^61-1; then salt_M,
   salt_1, salt_2 as three raw outputs. */
static void ora_coefficients(ora_index *h) {
  uint64_t s = h->seed;
  for (uint32_t i = 0; i < h->num_perm; ++i) {
    uint64_t u;
    do {
      u = ora_splitmix64_next(&s) >> 3;
    } while (u == 0 || u >= ORA_P61);
    h->a[i] = u;
  }
  for (uint32_t i = 0; i < h->num_perm; ++i) {
    uint64_t u;
    do {
      u = ora_splitmix64_next(&s) >> 3;
    } while (u >= ORA_P61);
    h->b[i] = u;
  }
  h->salt_m = ora_splitmix64_next(&s);
  h->salt1 = ora_splitmix64_next(&s);
  h->salt2 = ora_splitmix64_next(&s);
}

void ora_destroy(ora_index *h) {
  if (!h) return;
  free(h->a);
  free(h->b);
  free(h->filters);
  free(h);
}

ora_index *ora_create(uint32_t num_perm, uint32_t bands, uint32_t rows, uint64_t expected_n, double fp_rate,
                      uint64_t seed, uint32_t w) {
  if (num_perm == 0 || bands == 0 || rows == 0 || w == 0) return NULL;
  if ((uint64_t)bands * rows > num_perm) return NULL;
  ora_index *h = (ora_index *)calloc(1, sizeof(ora_index));
  if (!h) return NULL;
  h->num_perm = num_perm;
  h->bands = bands;
  h->rows = rows;
  h->w = w;
  h->expected_n = expected_n;
  h->fp_rate = fp_rate;
  h->seed = seed;
  if (ora_params(expected_n, fp_rate, &h->m_bits, &h->k) != 0) {
    free(h);
    return NULL;
  }
  h->words_per_band = h->m_bits / 64;
  h->a = (uint64_t *)malloc(sizeof(uint64_t) * num_perm);
  h->b = (uint64_t *)malloc(sizeof(uint64_t) * num_perm);
  h->filters = (uint64_t *)calloc((size_t)(h->words_per_band * bands), sizeof(uint64_t));
  if (!h->a || !h->b || !h->filters) {
    ora_destroy(h);
    return NULL;
  }
  ora_coefficients(h);
  return h;
}

/* MinHash of a CSR batch: documents d = 0..n_docs-1 own tokens
   [offsets[d], offsets[d+1]); sigs is row-major [n_docs][num_perm]. */
int ora_minhash(const ora_index *h, const int64_t *offsets, const uint32_t *tokens, int64_t n_docs, uint32_t *sigs) {
  if (n_docs < 0) return -1;
  for (int64_t d = 0; d < n_docs; ++d) {
    if (offsets[d + 1] < offsets[d]) return -1;
    ora_minhash_doc(tokens + offsets[d], offsets[d + 1] - offsets[d], h->w, h->num_perm, h->a, h->b,
                    sigs + (uint64_t)d * h->num_perm);
  }
  return 0;
}

/* The same MinHash with documents shared out over `threads` host threads:
   every document is still the sequential per-document definition above
   (ora_minhash_doc), and documents are independent (§2.2), so the output
   equals ora_minhash's.  It exists to time the CPU path the way the paper's
   own system runs it (MinHash parallel over documents, the filters
   sequential, §4.4.2); ora_query_insert stays sequential. */
typedef struct {
  const ora_index *h;
  const int64_t *offsets;
  const uint32_t *tokens;
  int64_t n_docs;
  uint32_t *sigs;
  atomic_llong next;
} ora_mh_job;

static void *ora_mh_worker(void *arg) {
  ora_mh_job *j = (ora_mh_job *)arg;
  for (;;) {
    const int64_t d0 = (int64_t)atomic_fetch_add(&j->next, 16);
    if (d0 >= j->n_docs) break;
    const int64_t d1 = d0 + 16 < j->n_docs ? d0 + 16 : j->n_docs;
    for (int64_t d = d0; d < d1; ++d)
      ora_minhash_doc(j->tokens + j->offsets[d], j->offsets[d + 1] - j->offsets[d], j->h->w, j->h->num_perm,
                      j->h->a, j->h->b, j->sigs + (uint64_t)d * j->h->num_perm);
  }
  return NULL;
}

int ora_minhash_threads(const ora_index *h, const int64_t *offsets, const uint32_t *tokens, int64_t n_docs,
                        uint32_t *sigs, int threads) {
  if (n_docs < 0 || threads < 1 || threads > 1024) return -1;
  for (int64_t d = 0; d < n_docs; ++d)
    if (offsets[d + 1] < offsets[d]) return -1;
  ora_mh_job job = {h, offsets, tokens, n_docs, sigs, 0};
  pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
  if (!tid) return -1;
  int started = 0;
  for (int t = 1; t < threads; ++t) {
    if (pthread_create(&tid[t], NULL, ora_mh_worker, &job) != 0) break;
    ++started;
  }
  ora_mh_worker(&job);
  for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
  free(tid);
  return 0;
}

static int ora_test_bit(const ora_index *h, uint32_t band, uint64_t g) {
  uint64_t word = h->filters[(uint64_t)band * h->words_per_band + (g >> 6)];
  return (int)((word >> (g & 63)) & 1ull);
}

static void ora_set_bit(ora_index *h, uint32_t band, uint64_t g) {
  h->filters[(uint64_t)band * h->words_per_band + (g >> 6)] |= 1ull << (g & 63);
}

/* Stream query-then-insert (§2.1, §4.1, §4.2, §4.4.2): for each document in
   order, flag = 1 iff in some band all k bits of its band key are already
   set; then the document's k bits are set in every band. */
int ora_query_insert(ora_index *h, const uint32_t *sigs, int64_t n_docs, uint8_t *flags) {
  if (n_docs < 0) return -1;
  uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * h->k);
  if (!g) return -1;
  for (int64_t i = 0; i < n_docs; ++i) {
    const uint32_t *sig = sigs + (uint64_t)i * h->num_perm;
    int hit = 0;
    for (uint32_t j = 0; j < h->bands; ++j) {
      uint64_t K = ora_band_key(sig, j, h->rows, h->salt_m);
      ora_positions(K, h->salt1, h->salt2, h->m_bits, h->k, g);
      int all = 1;
      for (uint32_t l = 0; l < h->k; ++l)
        if (!ora_test_bit(h, j, g[l])) all = 0;
      if (all) hit = 1;
    }
    flags[i] = (uint8_t)hit;
    for (uint32_t j = 0; j < h->bands; ++j) {
      uint64_t K = ora_band_key(sig, j, h->rows, h->salt_m);
      ora_positions(K, h->salt1, h->salt2, h->m_bits, h->k, g);
      for (uint32_t l = 0; l < h->k; ++l) ora_set_bit(h, j, g[l]);
    }
    h->docs_inserted += 1;
  }
  free(g);
  return 0;
}

/* Query only (§4.2): flags as above, filters untouched. */
int ora_query(const ora_index *h, const uint32_t *sigs, int64_t n_docs, uint8_t *flags) {
  if (n_docs < 0) return -1;
  uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * h->k);
  if (!g) return -1;
  for (int64_t i = 0; i < n_docs; ++i) {
    const uint32_t *sig = sigs + (uint64_t)i * h->num_perm;
    int hit = 0;
    for (uint32_t j = 0; j < h->bands; ++j) {
      uint64_t K = ora_band_key(sig, j, h->rows, h->salt_m);
      ora_positions(K, h->salt1, h->salt2, h->m_bits, h->k, g);
      int all = 1;
      for (uint32_t l = 0; l < h->k; ++l)
        if (!ora_test_bit(h, j, g[l])) all = 0;
      if (all) hit = 1;
    }
    flags[i] = (uint8_t)hit;
  }
  free(g);
  return 0;
}

/* Insert only (§4.1): every document's k bits in every band are set. */
int ora_insert(ora_index *h, const uint32_t *sigs, int64_t n_docs) {
  if (n_docs < 0) return -1;
  uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * h->k);
  if (!g) return -1;
  for (int64_t i = 0; i < n_docs; ++i) {
    const uint32_t *sig = sigs + (uint64_t)i * h->num_perm;
    for (uint32_t j = 0; j < h->bands; ++j) {
      uint64_t K = ora_band_key(sig, j, h->rows, h->salt_m);
      ora_positions(K, h->salt1, h->salt2, h->m_bits, h->k, g);
      for (uint32_t l = 0; l < h->k; ++l) ora_set_bit(h, j, g[l]);
    }
    h->docs_inserted += 1;
  }
  free(g);
  return 0;
}

/* Band keys of a batch (§4.1), row-major [n_docs][bands]. */
void ora_band_keys(const ora_index *h, const uint32_t *sigs, int64_t n_docs, uint64_t *keys) {
  for (int64_t i = 0; i < n_docs; ++i)
    for (uint32_t j = 0; j < h->bands; ++j)
      keys[(uint64_t)i * h->bands + j] = ora_band_key(sigs + (uint64_t)i * h->num_perm, j, h->rows, h->salt_m);
}

/* ------------------------------------------------------------------------ */
/* Wide-value variant (§4.5: the index size does not depend on the width of  */
/* the MinHash values, so they may be widened at no cost in index space).    */
/* The permutation value is kept whole, h_i(x) = (a_i x + b_i) mod (2^61-1), */
/* 61 bits, instead of its low 32 bits; the shingle hash x is unchanged.     */
/* ------------------------------------------------------------------------ */
uint64_t ora_perm61(uint64_t a, uint64_t b, uint32_t x) {
  u128 v = (u128)a * (u128)x + (u128)b;
  return (uint64_t)(v % (u128)ORA_P61);
}

/* Wide signature of one document: sig[i] = min over the shingle set of
   h_i; the empty set gives all ones (2^64 - 1, above every value). */
void ora_minhash_doc61(const uint32_t *tok, int64_t L, uint32_t w, uint32_t num_perm,
                       const uint64_t *a, const uint64_t *b, uint64_t *sig) {
  for (uint32_t i = 0; i < num_perm; ++i) sig[i] = ~0ull;
  if (L <= 0) return;
  int64_t n_sh = L >= (int64_t)w ? L - (int64_t)w + 1 : 1;
  uint32_t sh_len = L >= (int64_t)w ? w : (uint32_t)L;
  for (int64_t t = 0; t < n_sh; ++t) {
    uint32_t x = ora_shingle_hash(tok + t, sh_len);
    for (uint32_t i = 0; i < num_perm; ++i) {
      uint64_t v = ora_perm61(a[i], b[i], x);
      if (v < sig[i]) sig[i] = v;
    }
  }
}

int ora_minhash61(const ora_index *h, const int64_t *offsets, const uint32_t *tokens, int64_t n_docs,
                  uint64_t *sigs) {
  if (n_docs < 0) return -1;
  for (int64_t d = 0; d < n_docs; ++d) {
    if (offsets[d + 1] < offsets[d]) return -1;
    ora_minhash_doc61(tokens + offsets[d], offsets[d + 1] - offsets[d], h->w, h->num_perm, h->a, h->b,
                      sigs + (uint64_t)d * h->num_perm);
  }
  return 0;
}

/* Band key of a band of wide values (§4.1, band hash equation): the same sum
   mod 2^64 of per-row finalizer terms; the value fills the word, so the row
   index enters as an offset of t times the golden-ratio constant before the
   salt: term = fmix64((v + t * 0x9E3779B97F4A7C15) xor salt_M). */
uint64_t ora_band_key61(const uint64_t *sig, uint32_t band, uint32_t rows, uint64_t salt_m) {
  uint64_t K = 0;
  for (uint32_t t = 0; t < rows; ++t) {
    uint64_t v = sig[(uint64_t)band * rows + t] + (uint64_t)t * 0x9E3779B97F4A7C15ull;
    K += ora_fmix64(v ^ salt_m);
  }
  return K;
}

void ora_band_keys61(const ora_index *h, const uint64_t *sigs, int64_t n_docs, uint64_t *keys) {
  for (int64_t i = 0; i < n_docs; ++i)
    for (uint32_t j = 0; j < h->bands; ++j)
      keys[(uint64_t)i * h->bands + j] = ora_band_key61(sigs + (uint64_t)i * h->num_perm, j, h->rows, h->salt_m);
}

/* Stream query-then-insert from band keys [n_docs][bands] (§4.1 reduces
   each band to one integer; from there on the steps are those of
   ora_query_insert). */
int ora_query_insert_keys(ora_index *h, const uint64_t *keys, int64_t n_docs, uint8_t *flags) {
  if (n_docs < 0) return -1;
  uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * h->k);
  if (!g) return -1;
  for (int64_t i = 0; i < n_docs; ++i) {
    const uint64_t *K = keys + (uint64_t)i * h->bands;
    int hit = 0;
    for (uint32_t j = 0; j < h->bands; ++j) {
      ora_positions(K[j], h->salt1, h->salt2, h->m_bits, h->k, g);
      int all = 1;
      for (uint32_t l = 0; l < h->k; ++l)
        if (!ora_test_bit(h, j, g[l])) all = 0;
      if (all) hit = 1;
    }
    flags[i] = (uint8_t)hit;
    for (uint32_t j = 0; j < h->bands; ++j) {
      ora_positions(K[j], h->salt1, h->salt2, h->m_bits, h->k, g);
      for (uint32_t l = 0; l < h->k; ++l) ora_set_bit(h, j, g[l]);
    }
    h->docs_inserted += 1;
  }
  free(g);
  return 0;
}

/* One band's share of the stream (§4.1, §4.2): band j has a Bloom filter of
   its own that only band j's keys ever reach, so over the stream that filter
   is itself queried then inserted in document order; hits[i] = 1 iff all k
   bits of document i's band-j key were set just before document i.  A
   document's flag is the OR of its bands' hits (§4.2), which is what
   ora_query_insert computes band by band inside its document loop.  Calls for
   different bands touch different filters and may run at the same time;
   docs_inserted is not changed (the caller counts documents once). */
int ora_query_insert_band(ora_index *h, const uint32_t *sigs, int64_t n_docs, uint32_t band, uint8_t *hits) {
  if (n_docs < 0 || band >= h->bands) return -1;
  uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * h->k);
  if (!g) return -1;
  for (int64_t i = 0; i < n_docs; ++i) {
    const uint64_t K = ora_band_key(sigs + (uint64_t)i * h->num_perm, band, h->rows, h->salt_m);
    ora_positions(K, h->salt1, h->salt2, h->m_bits, h->k, g);
    int all = 1;
    for (uint32_t l = 0; l < h->k; ++l)
      if (!ora_test_bit(h, band, g[l])) all = 0;
    hits[i] = (uint8_t)all;
    for (uint32_t l = 0; l < h->k; ++l) ora_set_bit(h, band, g[l]);
  }
  free(g);
  return 0;
}

/* Add n documents to the inserted count (after ora_query_insert_band calls). */
void ora_count_docs(ora_index *h, uint64_t n) { h->docs_inserted += n; }

/* Accessors for tests. */
uint64_t ora_m_bits(const ora_index *h) { return h->m_bits; }
uint32_t ora_k(const ora_index *h) { return h->k; }
uint64_t ora_words_per_band(const ora_index *h) { return h->words_per_band; }
uint64_t *ora_filters(ora_index *h) { return h->filters; }
uint64_t ora_docs_inserted(const ora_index *h) { return h->docs_inserted; }
void ora_coeffs(const ora_index *h, uint64_t *a, uint64_t *b, uint64_t salts[3]) {
  memcpy(a, h->a, sizeof(uint64_t) * h->num_perm);
  memcpy(b, h->b, sizeof(uint64_t) * h->num_perm);
  salts[0] = h->salt_m;
  salts[1] = h->salt1;
  salts[2] = h->salt2;
}
