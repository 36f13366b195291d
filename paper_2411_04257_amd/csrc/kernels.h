// Host-side launchers of the LSHBloom HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lb {

// Permutation coefficients as 32-bit halves: {a_lo, a_hi, b_lo, b_hi}.
struct PermCoef {
  uint32_t a_lo, a_hi, b_lo, b_hi;
};

struct MinhashLaunch {
  // Document boundaries in the position space the persistent grid splits:
  // document d covers positions [offsets[d], offsets[d+1]).
  const int64_t *offsets;
  const uint32_t *tokens;
  int64_t n_docs;
  const PermCoef *coef;
  uint32_t *sigs;
  // wide-value variant: when set, signatures are the whole 61-bit
  // permutation values written here (and sigs is unused)
  uint64_t *sigs64;
  uint32_t num_perm;
  uint32_t w;
  int waves;  // total waves of the persistent grid (multiple of 4)
  // Optional indirection (length buckets): the token of position p of
  // document d is tokens[p + tok_shift[d]] and its signature row is
  // row_ids[d]; both null means identity.
  const int64_t *tok_shift;
  const int64_t *row_ids;
};

struct BloomLaunch {
  const uint32_t *sigs;  // [n][num_perm]
  const uint64_t *keys_in;   // [n][bands] band keys given by the caller (instead of sigs), or null
  const uint64_t *sigs64;    // [n][num_perm] wide signatures (k_band_keys61 only)
  int64_t n;
  uint32_t num_perm, bands, rows, k;
  uint64_t m_bits, words_per_band;
  uint64_t salt_m, salt1, salt2;
  uint64_t *filters;
  uint64_t *table;  // first-setter table, power-of-two slots
  uint64_t table_mask;
  uint64_t *keys;   // [n][bands]
  uint64_t *masks;  // [n][bands]
  uint8_t *hitb;    // [n][bands]
  uint8_t *flags;   // [n]
  uint32_t *status;  // device status word (nonzero = internal inconsistency)
};

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_minhash(const MinhashLaunch &a, hipStream_t s);
hipError_t launch_band_keys(const BloomLaunch &a, hipStream_t s);
// Band keys of wide signatures (a.sigs64) into a.keys [n][bands].
hipError_t launch_band_keys61(const BloomLaunch &a, hipStream_t s);
// One in-order chunk: clear table, probe, resolve + insert, flags.
hipError_t launch_query_insert_chunk(const BloomLaunch &a, uint64_t table_slots, hipStream_t s);
hipError_t launch_query(const BloomLaunch &a, hipStream_t s);
hipError_t launch_insert(const BloomLaunch &a, hipStream_t s);
// out[j] += set bits of words[j * words_per_band .. (j + 1) * words_per_band).
hipError_t launch_popcount(const uint64_t *words, uint64_t words_per_band, uint32_t bands, uint64_t *out,
                           hipStream_t s);

// Size of the persistent MinHash grid.  Waves own equal token ranges; many
// more waves than fit at once (up to 256 per compute unit) let the hardware
// balance the tail, and one wave per ~2,048 tokens keeps each range long
// enough to amortise its start.  When only the document count is known on the
// host, four waves per document stand in for the token count.
inline int minhash_waves_for_tokens(int cus, uint64_t tokens) {
  uint64_t w = tokens / 2048;
  const uint64_t lo = 16ull * (uint64_t)cus, hi = 256ull * (uint64_t)cus;
  w = w < lo ? lo : (w > hi ? hi : w);
  return (int)(w < 4 ? 4 : w / 4 * 4);
}
inline int minhash_waves_for_docs(int cus, uint64_t n_docs) { return minhash_waves_for_tokens(cus, n_docs * 4 * 2048); }

constexpr uint64_t kTableEmpty = ~0ull;
constexpr int kIdxBits = 18;  // doc index within a chunk
constexpr uint64_t kMaxChunkDocs = (1ull << kIdxBits) - 1;

}  // namespace lb
