// Internal definition of the LSHBloom handle, shared by the C-ABI entry
// points and the batched pipeline.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "../../include/lshbloom.h"
#include "kernels.h"
#include "qi_binned.h"

struct lshbloom {
  lshbloom_params_t prm;
  uint64_t m_bits = 0, words_per_band = 0;
  uint32_t k = 0;
  uint64_t salt_m = 0, salt1 = 0, salt2 = 0;
  int device = 0;
  lb::PermCoef *d_coef = nullptr;
  uint64_t *d_filters = nullptr;
  uint64_t *d_table = nullptr;
  uint64_t table_slots_max = 0;
  uint64_t *d_keys = nullptr;
  uint64_t *d_masks = nullptr;
  uint8_t *d_hitb = nullptr;
  uint32_t *d_status = nullptr;  // [0]: consistency word; bytes 8..15: bins left to the binned path's general path
  uint32_t *h_status = nullptr;  // pinned host copy of d_status, refreshed at the end of every query-insert call
  uint64_t *d_count = nullptr;  // per-band set-bit counts [bands]
  uint64_t chunk_docs = 0;
  uint64_t workspace_bytes = 0;
  // binned query-insert workspace
  uint32_t qi_mode = 0;
  uint64_t bin_chunk = 0;
  uint64_t bin_counts_cap = 0;  // entries of the pass-1 count/offset array
  uint64_t bin_buckets_cap = 0; // bucket starts
  uint64_t bin_bins_cap = 0;    // bin offsets / directory
  uint64_t bin_rec2_cap = 0;    // binned-record slots (records plus pass 2's spare slices)
  uint32_t *d_counts1 = nullptr, *d_bstart = nullptr, *d_off2 = nullptr, *d_end2 = nullptr;
  uint64_t *d_rec1 = nullptr, *d_rec2 = nullptr, *d_bkeys = nullptr, *d_dir = nullptr;
  uint32_t *d_ovf = nullptr;  // bins left to the general path (count, then bins)
  uint8_t *d_res0 = nullptr;
  int minhash_waves = 0;  // persistent MinHash grid; 0 = sized per call
  int cus = 0;            // compute units of the device
  hipEvent_t last = nullptr;
  bool has_last = false;
  std::atomic<bool> poisoned{false};
  uint64_t docs_inserted = 0;
  uint64_t calls = 0;
  int64_t fault_at = -1;  // host-forced failure of the n-th filter call (testing)
  uint64_t qi_calls = 0;
  int64_t status_at = -1;  // host-forced device status report by the n-th query-insert call (testing)
  std::mutex mu;
};

namespace lbh {

void set_err(const char *fmt, ...);
int fail_hip(lshbloom *h, hipError_t e, const char *what);
// Order the work enqueued next on s after the handle's previous filter call,
// and record the end of that work as the handle's new last call.
hipError_t begin_ordered(lshbloom *h, hipStream_t s);
hipError_t end_ordered(lshbloom *h, hipStream_t s);
// LSHBLOOM_OK, or the error a call on h must return: EDEVICE the first time
// the host copy of the device status word is seen nonzero (the handle is
// then poisoned), EPOISONED afterwards.
int check_ready(lshbloom *h);
// End of a query-insert call on s: the device status word's copy to host
// memory (and, for testing, a host-forced status report).
hipError_t finish_qi(lshbloom *h, hipStream_t s);
// Enqueue the in-order query-insert of n signatures on s (no locking, no
// ordering events, no counters); the algorithm follows the handle's mode.
// Returns LSHBLOOM_OK or an error code (message set, handle poisoned on a
// HIP error).
// With d_keys (band keys [n][bands]) the keys are taken as given and d_sigs
// is not read.
// part 0 enqueues the whole query-insert; when qi_splits(h, n), part 1
// enqueues its partition passes and part 2 the rest (1 then 2 on one stream
// is the whole call); otherwise part 1 enqueues everything and part 2 nothing.
// Parts 1 and 2 are the batched form's, whose next MinHash runs beside them:
// they size the dense bins' persistent grid to leave it room.
int qi_enqueue(lshbloom *h, const uint32_t *d_sigs, int64_t n, uint8_t *d_flags, hipStream_t s,
               const uint64_t *d_keys = nullptr, int part = 0);
// The query-insert of n documents is one binned chunk (so it splits in two).
bool qi_splits(const lshbloom *h, int64_t n);

}  // namespace lbh
