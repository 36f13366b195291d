// Binned in-order query-insert (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lb {

// Bin geometry of one chunk: bins of 2^bin_bits bits within a band, grouped
// into super bins of bins_per_super consecutive bins of one band.
struct BinnedGeometry {
  uint32_t bin_bits;
  uint64_t bins_per_band;
  uint32_t bins_per_super;
  uint32_t supers_per_band;
  uint32_t n_supers;
  uint32_t items_per_block;  // (document, band) items per pass-1 block
  uint32_t n_blocks1;
};

struct BinnedLaunch {
  const uint32_t *sigs;  // [n][num_perm]
  int64_t n;
  uint32_t num_perm, bands, rows, k;
  uint64_t m_bits, words_per_band;
  uint64_t salt_m, salt1, salt2;
  uint64_t *filters;
  // geometry
  uint32_t bin_bits;
  uint64_t bins_per_band;
  uint32_t bins_per_super, supers_per_band, n_supers;
  uint32_t items_per_block, n_blocks1;
  uint32_t n_records;  // n * bands * k (< 2^32)
  // workspace
  uint32_t *counts1;  // [n_supers][n_blocks1]
  uint32_t *offs1;    // [n_supers][n_blocks1] absolute record offsets
  uint32_t *super_tot;  // [n_supers] records per super bin, then their starts
  uint64_t *rec1;     // pass-1 records; reused as the published bit tables (2 slots per record)
  uint64_t *rec2;     // records grouped by bin
  uint64_t *table;    // == rec1
  uint32_t *off2;     // [bands * bins_per_band + 1] record offsets of every bin
  uint8_t *hitb;      // [n][bands]
  uint8_t *flags;     // [n]
  uint32_t *status;
};

// Records per bin aimed at (the LDS path handles up to 1024).
constexpr uint32_t kBinTarget = 512;

BinnedGeometry binned_geometry(uint64_t n_docs, uint32_t bands, uint32_t k, uint64_t m_bits,
                               uint32_t target_per_bin = kBinTarget);
hipError_t launch_query_insert_binned(const BinnedLaunch &a, hipStream_t s);

}  // namespace lb
