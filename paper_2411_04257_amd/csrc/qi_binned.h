// Binned in-order query-insert (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lb {

// Documents per pass-1 block (a power of two: a block's probe slots are
// enumerated l-major, slot = l * kTileDocs + document).
#ifndef LB_TILE_LOG
#define LB_TILE_LOG 10
#endif
constexpr uint32_t kTileLog = LB_TILE_LOG;
constexpr uint32_t kTileDocs = 1u << kTileLog;
// Largest chunk the 64-bit record format holds: document index in 23 bits.
constexpr uint64_t kBinnedMaxDocs = (1ull << 23) - 1;
// Records per chunk must stay below 2^31 (32-bit record offsets and table caps).
constexpr uint64_t kBinnedMaxRecords = (1ull << 31) - 1;

// Bin geometry of one chunk.  Bits of band j are cut into bins of 2^bin_bits
// bits (one workgroup owns a bin); bins are grouped into buckets of
// bins_per_bucket consecutive bins (2^bucket_bits bits), the unit of the
// first partition pass.
struct BinnedGeometry {
  uint32_t bin_bits;
  uint64_t bins_per_band;
  uint32_t bucket_bits;
  uint32_t buckets_per_band;  // F1: fan-out of pass 1 within a band
  uint32_t bins_per_bucket;   // F2: fan-out of pass 2
  uint32_t n_tiles;           // pass-1 blocks per band
  bool direct_words;          // a bin's filter words fit in LDS (bin_bits <= 15)
};

struct BinnedLaunch {
  const uint32_t *sigs;  // [n][num_perm]
  const uint64_t *keys_in;  // [n][bands] band keys given by the caller (instead of sigs), or null
  int64_t n;
  uint32_t num_perm, bands, rows, k;
  uint64_t m_bits, words_per_band;
  uint64_t salt_m, salt1, salt2;
  uint64_t *filters;
  BinnedGeometry G;
  uint32_t n_records;  // n * bands * k (< 2^31)
  // workspace
  uint64_t *keys;      // [bands][n] band keys
  uint32_t *counts;    // [bands][F1][n_tiles] per-block bucket counts, then offsets
  uint32_t *bstart;    // [bands * F1 + 1] bucket totals, then starts
  uint64_t *rec1;      // pass-1 records (bucket order); then the published tables (2 slots per rec2 slot)
  uint64_t *rec2;      // records in bin order: bucket q's region starts at bstart[q] + q (slice_slack + 1) F2
  uint32_t *off2;      // [bands * bins_per_band] first record of every bin in rec2
  uint32_t *end2;      // [bands * bins_per_band] end of every bin's records in rec2
  uint32_t slice_slack; // spare slots per bin of pass 2's slices (0: counted, compact layout)
  uint64_t *dir;       // [bands * bins_per_band] published table of a bin: first record << 32 | slots
  uint32_t *ovf;       // [1 + bands * bins_per_band] count, then the bins left to the general path
  unsigned long long *ovf_total;  // bins left to the general path, summed over chunks (a diagnostic)
  uint8_t *res0;       // [bands][n] probe 0 of (document, band) was set before the document
  uint8_t *flags;      // [n]
  uint32_t *status;
  uint32_t cus;        // compute units of the device (sizes persistent grids)
  bool shared_device;  // other kernels run beside this call's (the batched form's next MinHash)
};

// Spare slots per bin for pass 2's single-read layout: about five standard
// deviations of a bin's record count (records / bins on average) plus 16.
inline uint32_t binned_slice_slack(uint64_t records, uint64_t bins) {
  const double mean = bins ? (double)records / (double)bins : 0.0;
  uint32_t sd5 = 0;
  while ((double)sd5 * sd5 < 25.0 * mean) ++sd5;
  return sd5 + 16;
}
// Pass 2 reads a bucket once (into slices) when buckets average at least
// this many records; below it counting first and a compact layout are faster
// (2M-document chunks of the 10M-document workload: 118,000 records per
// bucket, 9.4 -> 7.2 ms per chunk; the filter-scale stream's 46,000: 4.6 ->
// 4.7 ms).
constexpr uint64_t kSliceMinBucket = 65536;
// Binned-record slots pass 2's single-read layout needs for a geometry.
inline uint64_t binned_slice_slots(const BinnedGeometry &G, uint32_t bands, uint64_t records) {
  const uint32_t slack = binned_slice_slack(records, (uint64_t)bands * G.bins_per_band);
  return records + (uint64_t)bands * G.buckets_per_band * G.bins_per_bucket * (slack + 1);
}

// Records per bin aimed at (a sparse bin's wave holds up to 320).
constexpr uint32_t kBinTarget = 192;
// Dense bins (at most 2^15 bits) are widened while they average at most this
// many records (a dense bin's wave holds up to 576): fewer, fuller bins
// spread each bin's fixed work (reading, claiming and writing back its
// words) over more records.
constexpr uint32_t kDenseFill = 480;

BinnedGeometry binned_geometry(uint64_t n_docs, uint32_t bands, uint32_t k, uint64_t m_bits,
                               uint32_t target_per_bin = kBinTarget);
// Workspace entries of a geometry (for sizing and checks).
inline uint64_t binned_counts_entries(const BinnedGeometry &G, uint32_t bands) {
  return (uint64_t)bands * G.buckets_per_band * G.n_tiles;
}
inline uint64_t binned_bucket_entries(const BinnedGeometry &G, uint32_t bands) {
  return (uint64_t)bands * G.buckets_per_band + 1;
}
inline uint64_t binned_bin_entries(const BinnedGeometry &G, uint32_t bands) {
  return (uint64_t)bands * G.bins_per_band + 1;
}
// part 0: the whole chunk; part 1: up to and including the partition passes
// (keys, pass 1, pass 2); part 2: the rest (bins, resolve).  Parts 1 then 2
// on one stream are the whole chunk.
hipError_t launch_query_insert_binned(const BinnedLaunch &a, hipStream_t s, int part = 0);

}  // namespace lb
