// C ABI of the LSHBloom hot path (declared in include/lshbloom.h).
//
// Host side only: argument checks, sizing (Section 4.5), the coefficient
// stream, device memory, stream ordering between calls, chunking of the
// in-order query-insert, and error reporting.  All per-document work runs in
// the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"

namespace {
thread_local std::string g_err;
}  // namespace

namespace lbh {
void set_err(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}
}  // namespace lbh

namespace {
using lbh::set_err;

// SplitMix64 stream (Steele, Lea & Flood 2014).
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

constexpr uint64_t kP61 = 0x1FFFFFFFFFFFFFFFull;
constexpr uint64_t kDefaultTableBytes = 128ull << 20;
// Calls with at least this many documents use the binned query-insert when
// the mode is automatic (its fixed cost of ~10 launches pays off there).
constexpr int64_t kBinnedMinDocs = 4096;

uint64_t next_pow2(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Scratch of lshbloom_query_insert_noalloc: the direct algorithm's
// first-setter table (kNaTableSlots 8-byte slots), then the band keys (8 B),
// found-bit masks (8 B) and hit bytes (1 B) of up to kNaPairs (document,
// band) pairs of one chunk.  One copy per device, in the code object; its
// device address is looked up once per device (na_scratch_ptr) and only that
// address is handed to kernels.
constexpr uint64_t kNaTableSlots = 1ull << 21;  // 16 MiB
constexpr uint64_t kNaPairs = 1ull << 20;       // 17 MiB of keys, masks and hit bytes
constexpr uint64_t kNaBytes = kNaTableSlots * 8 + kNaPairs * (8 + 8) + kNaPairs;
constexpr int kNaMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kNaBytes];

std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices] = {};
bool g_na_done[kNaMaxDevices] = {};
hipError_t g_na_err[kNaMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// on the first call for that device.
hipError_t na_scratch_ptr(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kNaMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_done[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_na_err[device] = e;
    g_na_ptr[device] = e == hipSuccess ? p : nullptr;
    g_na_done[device] = true;
  }
  *out = g_na_ptr[device];
  return g_na_err[device];
}

}  // namespace



namespace lbh {

int fail_hip(lshbloom *h, hipError_t e, const char *what) {
  set_err("%s: %s", what, hipGetErrorString(e));
  if (h) h->poisoned = true;
  return LSHBLOOM_EHIP;
}

}  // namespace lbh

namespace {
using lbh::fail_hip;

void free_all(lshbloom *h) {
  if (!h) return;
  if (h->d_coef) (void)hipFree(h->d_coef);
  if (h->d_filters) (void)hipFree(h->d_filters);
  if (h->d_table) (void)hipFree(h->d_table);
  if (h->d_keys) (void)hipFree(h->d_keys);
  if (h->d_masks) (void)hipFree(h->d_masks);
  if (h->d_hitb) (void)hipFree(h->d_hitb);
  if (h->d_status) (void)hipFree(h->d_status);
  if (h->h_status) (void)hipHostFree(h->h_status);
  if (h->d_count) (void)hipFree(h->d_count);
  if (h->d_counts1) (void)hipFree(h->d_counts1);
  if (h->d_bstart) (void)hipFree(h->d_bstart);
  if (h->d_off2) (void)hipFree(h->d_off2);
  if (h->d_end2) (void)hipFree(h->d_end2);
  if (h->d_dir) (void)hipFree(h->d_dir);
  if (h->d_ovf) (void)hipFree(h->d_ovf);
  if (h->d_rec1) (void)hipFree(h->d_rec1);
  if (h->d_rec2) (void)hipFree(h->d_rec2);
  if (h->d_bkeys) (void)hipFree(h->d_bkeys);
  if (h->d_res0) (void)hipFree(h->d_res0);
  if (h->last) (void)hipEventDestroy(h->last);
}

}  // namespace

namespace lbh {
// Order this call after the handle's previous filter call.
hipError_t begin_ordered(lshbloom *h, hipStream_t s) {
  if (h->has_last) return hipStreamWaitEvent(s, h->last, 0);
  return hipSuccess;
}

hipError_t end_ordered(lshbloom *h, hipStream_t s) {
  hipError_t e = hipEventRecord(h->last, s);
  if (e == hipSuccess) h->has_last = true;
  return e;
}

int check_ready(lshbloom *h) {
  if (!h) {
    set_err("null handle");
    return LSHBLOOM_EINVAL;
  }
  const uint32_t st = h->h_status ? __atomic_load_n(h->h_status, __ATOMIC_ACQUIRE) : 0u;
  if (st != 0 && !h->poisoned.exchange(true)) {
    set_err("a kernel reported an internal inconsistency (device status 0x%x); the handle is poisoned", st);
    return LSHBLOOM_EDEVICE;
  }
  if (h->poisoned) {
    set_err("handle poisoned by an earlier device error; filters are indeterminate");
    return LSHBLOOM_EPOISONED;
  }
  return LSHBLOOM_OK;
}

hipError_t finish_qi(lshbloom *h, hipStream_t s) {
  h->qi_calls += 1;
  if (h->status_at >= 0 && (int64_t)h->qi_calls == h->status_at) {
    const hipError_t e = lb::launch_fill_u32(h->d_status, 1, 16u, s);
    if (e != hipSuccess) return e;
  }
  return hipMemcpyAsync(h->h_status, h->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
}

}  // namespace lbh

namespace {
using lbh::begin_ordered;
using lbh::check_ready;
using lbh::end_ordered;

bool forced_fault(lshbloom *h) {
  h->calls += 1;
  if (h->fault_at >= 0 && (int64_t)h->calls == h->fault_at) {
    set_err("injected device failure at filter call %llu (LSHBLOOM_FAULT_AT)", (unsigned long long)h->calls);
    h->poisoned = true;
    return true;
  }
  return false;
}

lb::BloomLaunch bloom_args(lshbloom *h, const uint32_t *sigs, int64_t n) {
  lb::BloomLaunch a{};
  a.sigs = sigs;
  a.n = n;
  a.num_perm = h->prm.num_perm;
  a.bands = h->prm.bands;
  a.rows = h->prm.rows;
  a.k = h->k;
  a.m_bits = h->m_bits;
  a.words_per_band = h->words_per_band;
  a.salt_m = h->salt_m;
  a.salt1 = h->salt1;
  a.salt2 = h->salt2;
  a.filters = h->d_filters;
  a.table = h->d_table;
  a.table_mask = h->table_slots_max - 1;
  a.keys = h->d_keys;
  a.masks = h->d_masks;
  a.hitb = h->d_hitb;
  a.status = h->d_status;
  return a;
}

}  // namespace

namespace lbh {

bool qi_splits(const lshbloom *h, int64_t n_docs) {
  const bool binned = h->bin_chunk && (h->qi_mode == 2 || (h->qi_mode == 0 && n_docs >= kBinnedMinDocs));
  return binned && n_docs > 0 && (uint64_t)n_docs <= h->bin_chunk;
}

int qi_enqueue(lshbloom *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags, hipStream_t s,
               const uint64_t *d_keys, int part) {
  hipError_t e;
  const uint64_t pd = (uint64_t)h->prm.bands * h->k;
  const bool binned = h->bin_chunk && (h->qi_mode == 2 || (h->qi_mode == 0 && n_docs >= kBinnedMinDocs));
  // parts are enqueued by the batched form, whose next MinHash runs beside them
  const bool shared_device = part != 0;
  if (part != 0 && !qi_splits(h, n_docs)) {
    if (part == 2) return LSHBLOOM_OK;
    part = 0;
  }
  if (binned) {
    for (int64_t c0 = 0; c0 < n_docs; c0 += (int64_t)h->bin_chunk) {
      const int64_t cn = std::min<int64_t>((int64_t)h->bin_chunk, n_docs - c0);
      const lb::BinnedGeometry G = lb::binned_geometry((uint64_t)cn, h->prm.bands, h->k, h->m_bits);
      lb::BinnedLaunch a{};
      a.sigs = d_keys ? nullptr : d_sigs + c0 * (int64_t)h->prm.num_perm;
      a.keys_in = d_keys ? d_keys + c0 * (int64_t)h->prm.bands : nullptr;
      a.n = cn;
      a.num_perm = h->prm.num_perm;
      a.bands = h->prm.bands;
      a.rows = h->prm.rows;
      a.k = h->k;
      a.m_bits = h->m_bits;
      a.words_per_band = h->words_per_band;
      a.salt_m = h->salt_m;
      a.salt1 = h->salt1;
      a.salt2 = h->salt2;
      a.filters = h->d_filters;
      a.G = G;
      a.n_records = (uint32_t)((uint64_t)cn * pd);
      a.keys = h->d_bkeys;
      a.counts = h->d_counts1;
      a.bstart = h->d_bstart;
      a.rec1 = h->d_rec1;
      a.rec2 = h->d_rec2;
      a.off2 = h->d_off2;
      a.end2 = h->d_end2;
      {
        // pass 2 reads each bucket once when buckets are large and the
        // workspace holds their spare slices; otherwise it counts first (the
        // same result)
        const uint64_t slots = lb::binned_slice_slots(G, h->prm.bands, a.n_records);
        const uint64_t buckets = (uint64_t)h->prm.bands * G.buckets_per_band;
        a.slice_slack = slots <= h->bin_rec2_cap && slots < (1ull << 32) && a.n_records >= buckets * lb::kSliceMinBucket
                            ? lb::binned_slice_slack(a.n_records, (uint64_t)h->prm.bands * G.bins_per_band)
                            : 0u;
      }
      a.dir = h->d_dir;
      a.ovf = h->d_ovf;
      a.ovf_total = reinterpret_cast<unsigned long long *>(h->d_status + 2);
      a.res0 = h->d_res0;
      a.flags = d_flags + c0;
      a.status = h->d_status;
      a.cus = (uint32_t)h->cus;
      a.shared_device = shared_device;
      if (lb::binned_counts_entries(G, h->prm.bands) > h->bin_counts_cap ||
          lb::binned_bucket_entries(G, h->prm.bands) > h->bin_buckets_cap ||
          lb::binned_bin_entries(G, h->prm.bands) > h->bin_bins_cap) {
        set_err("query_insert: binned geometry exceeds the workspace (internal error)");
        h->poisoned = true;
        return LSHBLOOM_EHIP;
      }
      e = lb::launch_query_insert_binned(a, s, part);
      if (e != hipSuccess) return fail_hip(h, e, "query_insert: binned launch");
    }
    return LSHBLOOM_OK;
  }
  for (int64_t c0 = 0; c0 < n_docs; c0 += (int64_t)h->chunk_docs) {
    const int64_t cn = std::min<int64_t>((int64_t)h->chunk_docs, n_docs - c0);
    lb::BloomLaunch a = bloom_args(h, d_keys ? nullptr : d_sigs + c0 * (int64_t)h->prm.num_perm, cn);
    a.keys_in = d_keys ? d_keys + c0 * (int64_t)h->prm.bands : nullptr;
    a.flags = d_flags + c0;
    const uint64_t slots = std::min<uint64_t>(h->table_slots_max, next_pow2(std::max<uint64_t>(1024, 2 * cn * pd)));
    a.table_mask = slots - 1;
    e = lb::launch_query_insert_chunk(a, slots, s);
    if (e != hipSuccess) return fail_hip(h, e, "query_insert: launch");
  }
  return LSHBLOOM_OK;
}

}  // namespace lbh

extern "C" {

const char *lshbloom_last_error(void) { return g_err.c_str(); }

double lshbloom_p_band_from_eff(double p_eff, uint32_t bands) {
  if (!(p_eff > 0.0 && p_eff < 1.0) || bands == 0) return NAN;
  return -std::expm1(std::log1p(-p_eff) / (double)bands);
}

int lshbloom_optimal_bands(double threshold, uint32_t num_perm, double w_fp, double w_fn, uint32_t *bands,
                           uint32_t *rows) {
  if (!(threshold > 0.0 && threshold < 1.0) || num_perm == 0 || !bands || !rows || !(w_fp >= 0) || !(w_fn >= 0)) {
    set_err("optimal_bands: threshold must be in (0,1), num_perm >= 1, weights >= 0");
    return LSHBLOOM_EINVAL;
  }
  // FP_lsh = int_0^T 1-(1-t^r)^b dt, FN_lsh = int_T^1 (1-t^r)^b dt (Section 4.3,
  // Eq. 1-2), by 16-point Gauss-Legendre on 64 equal panels of each interval.
  static const double gx[8] = {0.0950125098376374, 0.2816035507792589, 0.4580167776572274, 0.6178762444026438,
                               0.7554044083550030, 0.8656312023878318, 0.9445750230732326, 0.9894009349916499};
  static const double gw[8] = {0.1894506104550685, 0.1826034150449236, 0.1691565193950025, 0.1495959888165767,
                               0.1246289712555339, 0.0951585116824928, 0.0622535239386479, 0.0271524594117541};
  auto integrate = [&](double lo, double hi, uint32_t b, uint32_t r, bool fn) {
    const int panels = 64;
    const double h = (hi - lo) / panels;
    double s = 0.0;
    for (int q = 0; q < panels; ++q) {
      const double c = lo + (q + 0.5) * h, half = 0.5 * h;
      for (int u = 0; u < 8; ++u) {
        for (int sg = -1; sg <= 1; sg += 2) {
          const double t = c + sg * gx[u] * half;
          const double miss = std::pow(1.0 - std::pow(t, (double)r), (double)b);
          s += gw[u] * half * (fn ? miss : 1.0 - miss);
        }
      }
    }
    return s;
  };
  double best = INFINITY;
  uint32_t bb = 1, br = 1;
  for (uint32_t b = 1; b <= num_perm; ++b) {
    for (uint32_t r = 1; (uint64_t)b * r <= num_perm; ++r) {
      const double err = w_fp * integrate(0.0, threshold, b, r, false) + w_fn * integrate(threshold, 1.0, b, r, true);
      if (err < best) {
        best = err;
        bb = b;
        br = r;
      }
    }
  }
  *bands = bb;
  *rows = br;
  return LSHBLOOM_OK;
}

lshbloom_t *lshbloom_create_ex(const lshbloom_params_t *p) {
  if (!p) {
    set_err("create: null params");
    return nullptr;
  }
  lshbloom_params_t prm = *p;
  if (prm.shingle_width == 0) prm.shingle_width = 5;
  if (prm.num_perm == 0 || prm.num_perm > LSHBLOOM_MAX_NUM_PERM) {
    set_err("create: num_perm must be in [1, %u]", LSHBLOOM_MAX_NUM_PERM);
    return nullptr;
  }
  if (prm.bands == 0 || prm.bands > LSHBLOOM_MAX_BANDS || prm.rows == 0 ||
      (uint64_t)prm.bands * prm.rows > prm.num_perm) {
    set_err("create: need 1 <= bands <= %u, rows >= 1 and bands * rows <= num_perm", LSHBLOOM_MAX_BANDS);
    return nullptr;
  }
  if (prm.shingle_width > LSHBLOOM_MAX_SHINGLE_WIDTH) {
    set_err("create: shingle_width must be in [1, %u]", LSHBLOOM_MAX_SHINGLE_WIDTH);
    return nullptr;
  }
  if (prm.expected_n == 0 || !(prm.fp_rate > 0.0) || !(prm.fp_rate < 1.0)) {
    set_err("create: need expected_n >= 1 and 0 < fp_rate < 1");
    return nullptr;
  }
  // Section 4.5 sizing, evaluated exactly as documented in the header.
  const double bits = -((double)prm.expected_n * std::log(prm.fp_rate)) / (std::log(2.0) * std::log(2.0));
  const double words = std::ceil(bits / 64.0);
  if (!(words >= 1.0) || words * 64.0 > (double)LSHBLOOM_MAX_M_BITS) {
    set_err("create: filter of %.3e bits per band exceeds the %llu-bit limit", words * 64.0,
            (unsigned long long)LSHBLOOM_MAX_M_BITS);
    return nullptr;
  }
  const double kk = std::floor(-std::log2(prm.fp_rate) + 0.5);
  const uint32_t k = kk < 1.0 ? 1u : (uint32_t)kk;
  if (k > 64) {
    set_err("create: fp_rate %.3g needs %u probes per band (limit 64)", prm.fp_rate, k);
    return nullptr;
  }

  lshbloom *h = new (std::nothrow) lshbloom();
  if (!h) {
    set_err("create: out of host memory");
    return nullptr;
  }
  h->prm = prm;
  h->m_bits = (uint64_t)words * 64ull;
  h->words_per_band = h->m_bits / 64;
  h->k = k;
  if (const char *fa = std::getenv("LSHBLOOM_FAULT_AT")) h->fault_at = std::atoll(fa);
  if (const char *sa = std::getenv("LSHBLOOM_STATUS_AT")) h->status_at = std::atoll(sa);

  // Coefficient stream.
  SplitMix64 rng{prm.seed};
  std::vector<uint64_t> a(prm.num_perm), b(prm.num_perm);
  for (auto &v : a) {
    do v = rng.next() >> 3;
    while (v == 0 || v >= kP61);
  }
  for (auto &v : b) {
    do v = rng.next() >> 3;
    while (v >= kP61);
  }
  h->salt_m = rng.next();
  h->salt1 = rng.next();
  h->salt2 = rng.next();
  std::vector<lb::PermCoef> coef(prm.num_perm);
  for (uint32_t i = 0; i < prm.num_perm; ++i)
    coef[i] = {(uint32_t)a[i], (uint32_t)(a[i] >> 32), (uint32_t)b[i], (uint32_t)(b[i] >> 32)};

  // Chunk size of the in-order query-insert: the first-setter table holds at
  // least twice the probes of a chunk.
  const uint64_t probes_per_doc = (uint64_t)prm.bands * k;
  uint64_t table_bytes = kDefaultTableBytes;
  // A caller's chunk size applies to the direct algorithm only when it is
  // selected explicitly; otherwise the direct path (small calls) keeps a
  // 128 MB table.
  uint64_t chunk = prm.qi_mode == 1 ? prm.chunk_docs : 0;
  if (chunk == 0) chunk = table_bytes / 8 / (2 * probes_per_doc);
  if (chunk > lb::kMaxChunkDocs) chunk = lb::kMaxChunkDocs;
  if (chunk < 1) chunk = 1;
  const uint64_t slots = next_pow2(std::max<uint64_t>(1024, 2 * chunk * probes_per_doc));
  h->chunk_docs = chunk;
  h->table_slots_max = slots;

  // Binned query-insert: 24 bytes per binned-record slot (pass-1 records,
  // 8 B per probe, whose space then holds the published tables, 2 x 8 B per
  // slot, and the binned records, 8 B per slot) plus 9 bytes per (document,
  // band) (band keys and probe-0 answers) and the count, bucket and bin
  // arrays.  A slot per probe, plus the spare slices that let pass 2 read
  // each bucket once (about a quarter more); a chunk sized from the budget
  // leaves room for them.
  h->qi_mode = prm.qi_mode;
  if (const char *qm = std::getenv("LSHBLOOM_QI_MODE")) {
    if (!std::strcmp(qm, "direct")) h->qi_mode = 1;
    if (!std::strcmp(qm, "binned")) h->qi_mode = 2;
  }
  uint64_t bin_chunk = 0, bin_ws = 0;
  if (h->qi_mode != 1) {
    const uint64_t budget = prm.workspace_budget ? prm.workspace_budget : (4ull << 30);
    const uint64_t per_doc = 32 * probes_per_doc + 9ull * prm.bands;
    bin_chunk = prm.chunk_docs ? prm.chunk_docs : budget / per_doc;
    if (!prm.chunk_docs) bin_chunk = std::min<uint64_t>(bin_chunk, std::max<uint64_t>(prm.expected_n, 65536));
    bin_chunk = std::min<uint64_t>(bin_chunk, lb::kBinnedMaxDocs);                       // document field
    bin_chunk = std::min<uint64_t>(bin_chunk, lb::kBinnedMaxRecords / probes_per_doc);   // record offsets
    if (bin_chunk < 1) bin_chunk = 1;
    // the arrays grow with the chunk (fewer records per band mean wider bins)
    const lb::BinnedGeometry g = lb::binned_geometry(bin_chunk, prm.bands, k, h->m_bits);
    h->bin_counts_cap = lb::binned_counts_entries(g, prm.bands);
    h->bin_buckets_cap = lb::binned_bucket_entries(g, prm.bands);
    h->bin_bins_cap = lb::binned_bin_entries(g, prm.bands);
    const uint64_t records = bin_chunk * probes_per_doc;
    const uint64_t sliced = lb::binned_slice_slots(g, prm.bands, records);
    const bool room = prm.chunk_docs || (sliced - records) * 24 + bin_chunk * (24 * probes_per_doc + 9ull * prm.bands) <= budget;
    h->bin_rec2_cap = room && sliced < (1ull << 32) ? sliced : records;
    bin_ws = h->bin_rec2_cap * 24 + bin_chunk * 9ull * prm.bands + h->bin_counts_cap * 4 + h->bin_buckets_cap * 4 +
             h->bin_bins_cap * 20;
  }
  h->bin_chunk = bin_chunk;
  const uint64_t hitb_docs = chunk;

  const uint64_t filter_bytes = h->m_bits / 8 * prm.bands;
  const uint64_t ws = slots * 8 + chunk * prm.bands * (8 + 8) + hitb_docs * prm.bands +
                      prm.num_perm * sizeof(lb::PermCoef) + 256 + bin_ws;
  h->workspace_bytes = ws;
  if (prm.hbm_budget && filter_bytes + ws > prm.hbm_budget) {
    set_err("create: filters (%llu B) + workspace (%llu B) exceed the HBM budget (%llu B)",
            (unsigned long long)filter_bytes, (unsigned long long)ws, (unsigned long long)prm.hbm_budget);
    delete h;
    return nullptr;
  }

  hipError_t e;
  if ((e = hipGetDevice(&h->device)) != hipSuccess) {
    fail_hip(nullptr, e, "create: hipGetDevice");
    delete h;
    return nullptr;
  }
  hipDeviceProp_t dp;
  if ((e = hipGetDeviceProperties(&dp, h->device)) != hipSuccess) {
    fail_hip(nullptr, e, "create: hipGetDeviceProperties");
    delete h;
    return nullptr;
  }
  // The allocation-free query-insert's scratch address on this device (its
  // failure is reported by that call only).
  {
    void *na = nullptr;
    (void)na_scratch_ptr(h->device, &na);
  }
  // Persistent MinHash grid: sized per call (minhash_waves_for_docs) unless
  // fixed by the environment.
  h->cus = dp.multiProcessorCount;
  h->minhash_waves = 0;
  if (const char *mw = std::getenv("LSHBLOOM_MINHASH_WAVES")) {
    int v = std::atoi(mw);
    if (v >= 4) h->minhash_waves = (v / 4) * 4;
  }

#define LB_ALLOC(ptr, bytes)                                               \
  do {                                                                     \
    if ((e = hipMalloc((void **)&(ptr), (bytes))) != hipSuccess) {         \
      set_err("create: hipMalloc of %llu bytes failed: %s",                \
              (unsigned long long)(bytes), hipGetErrorString(e));          \
      free_all(h);                                                         \
      delete h;                                                            \
      return nullptr;                                                      \
    }                                                                      \
  } while (0)
  LB_ALLOC(h->d_filters, filter_bytes);
  LB_ALLOC(h->d_table, slots * 8);
  LB_ALLOC(h->d_keys, chunk * prm.bands * 8);
  LB_ALLOC(h->d_masks, chunk * prm.bands * 8);
  LB_ALLOC(h->d_hitb, hitb_docs * prm.bands);
  if (bin_chunk) {
    LB_ALLOC(h->d_counts1, h->bin_counts_cap * 4);
    LB_ALLOC(h->d_bstart, h->bin_buckets_cap * 4);
    LB_ALLOC(h->d_off2, h->bin_bins_cap * 4);
    LB_ALLOC(h->d_end2, h->bin_bins_cap * 4);
    LB_ALLOC(h->d_dir, h->bin_bins_cap * 8);
    LB_ALLOC(h->d_ovf, h->bin_bins_cap * 4);
    LB_ALLOC(h->d_rec1, h->bin_rec2_cap * 16);
    LB_ALLOC(h->d_rec2, h->bin_rec2_cap * 8);
    LB_ALLOC(h->d_bkeys, bin_chunk * prm.bands * 8);
    LB_ALLOC(h->d_res0, (bin_chunk * prm.bands + 15) & ~15ull);  // zeroed as 32-bit words
  }
  LB_ALLOC(h->d_coef, prm.num_perm * sizeof(lb::PermCoef));
  LB_ALLOC(h->d_status, 256);
  if ((e = hipHostMalloc((void **)&h->h_status, 64, hipHostMallocDefault)) != hipSuccess) {
    fail_hip(nullptr, e, "create: pinned status word");
    free_all(h);
    delete h;
    return nullptr;
  }
  *h->h_status = 0;
  LB_ALLOC(h->d_count, (size_t)prm.bands * 8);
#undef LB_ALLOC
  if ((e = hipMemcpy(h->d_coef, coef.data(), coef.size() * sizeof(lb::PermCoef), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemset(h->d_filters, 0, filter_bytes)) != hipSuccess ||
      (e = hipMemset(h->d_status, 0, 256)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&h->last, hipEventDisableTiming)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    fail_hip(nullptr, e, "create: initialisation");
    free_all(h);
    delete h;
    return nullptr;
  }
  return h;
}

lshbloom_t *lshbloom_create(uint32_t num_perm, uint32_t bands, uint32_t rows, uint64_t expected_n, double fp_rate,
                            uint64_t seed) {
  lshbloom_params_t p{};
  p.num_perm = num_perm;
  p.bands = bands;
  p.rows = rows;
  p.expected_n = expected_n;
  p.fp_rate = fp_rate;
  p.seed = seed;
  p.shingle_width = 5;
  return lshbloom_create_ex(&p);
}

void lshbloom_destroy(lshbloom_t *h) {
  if (!h) return;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->has_last) (void)hipEventSynchronize(h->last);
    free_all(h);
  }
  delete h;
}

int lshbloom_minhash(lshbloom_t *h, const int64_t *d_offsets, const uint32_t *d_tokens, int64_t n_docs,
                     uint32_t *d_sigs, lshbloom_stream_t stream) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_offsets || !d_sigs || !d_tokens))) {
    set_err("minhash: need n_docs >= 0 and non-null offsets, tokens and sigs");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = lb::launch_fill_u32(d_sigs, (uint64_t)n_docs * h->prm.num_perm, 0xFFFFFFFFu, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "minhash: fill");
  lb::MinhashLaunch a{};
  a.offsets = d_offsets;
  a.tokens = d_tokens;
  a.n_docs = n_docs;
  a.coef = h->d_coef;
  a.sigs = d_sigs;
  a.num_perm = h->prm.num_perm;
  a.w = h->prm.shingle_width;
  a.waves = h->minhash_waves ? h->minhash_waves : lb::minhash_waves_for_docs(h->cus, (uint64_t)n_docs);
  e = lb::launch_minhash(a, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "minhash: launch");
  return LSHBLOOM_OK;
}

int lshbloom_query_insert(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                          lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_sigs || !d_flags))) {
    set_err("query_insert: need n_docs >= 0 and non-null sigs and flags");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  if (forced_fault(h)) return LSHBLOOM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query_insert: stream wait");
  rc = lbh::qi_enqueue(h, d_sigs, n_docs, d_flags, s);
  if (rc) return rc;
  e = lbh::finish_qi(h, s);
  if (e == hipSuccess) e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query_insert: event");
  h->docs_inserted += (uint64_t)n_docs;
  return LSHBLOOM_OK;
}

int lshbloom_query_insert_noalloc(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                                  lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_sigs || !d_flags))) {
    set_err("query_insert_noalloc: need n_docs >= 0 and non-null sigs and flags");
    return LSHBLOOM_EINVAL;
  }
  if ((uint64_t)n_docs > LSHBLOOM_NOALLOC_MAX_DOCS) {
    set_err("query_insert_noalloc: %lld documents exceed the limit of %llu per call", (long long)n_docs,
            (unsigned long long)LSHBLOOM_NOALLOC_MAX_DOCS);
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  void *na = nullptr;
  hipError_t e = na_scratch_ptr(h->device, &na);
  if (e != hipSuccess || !na) return fail_hip(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                              "query_insert_noalloc: scratch address");
  // Chunk so that the table holds at least twice the chunk's probes and the
  // pair arrays its (document, band) pairs.
  const uint64_t pd = (uint64_t)h->prm.bands * h->k;
  uint64_t chunk = std::min<uint64_t>(kNaTableSlots / (2 * pd), kNaPairs / h->prm.bands);
  chunk = std::min<uint64_t>(chunk, lb::kMaxChunkDocs);
  if (chunk < 1) {
    set_err("query_insert_noalloc: %llu probes per document exceed the scratch", (unsigned long long)pd);
    return LSHBLOOM_EINVAL;
  }
  if (forced_fault(h)) return LSHBLOOM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query_insert_noalloc: stream wait");
  uint8_t *base = static_cast<uint8_t *>(na);
  for (int64_t c0 = 0; c0 < n_docs; c0 += (int64_t)chunk) {
    const int64_t cn = std::min<int64_t>((int64_t)chunk, n_docs - c0);
    lb::BloomLaunch a = bloom_args(h, d_sigs + c0 * (int64_t)h->prm.num_perm, cn);
    const uint64_t slots = std::min<uint64_t>(kNaTableSlots, next_pow2(std::max<uint64_t>(1024, 2 * cn * pd)));
    a.table = reinterpret_cast<uint64_t *>(base);
    a.table_mask = slots - 1;
    a.keys = reinterpret_cast<uint64_t *>(base + kNaTableSlots * 8);
    a.masks = reinterpret_cast<uint64_t *>(base + kNaTableSlots * 8 + kNaPairs * 8);
    a.hitb = base + kNaTableSlots * 8 + kNaPairs * 16;
    a.flags = d_flags + c0;
    e = lb::launch_query_insert_chunk(a, slots, s);
    if (e != hipSuccess) return fail_hip(h, e, "query_insert_noalloc: launch");
  }
  e = lbh::finish_qi(h, s);
  if (e == hipSuccess) e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query_insert_noalloc: event");
  h->docs_inserted += (uint64_t)n_docs;
  return LSHBLOOM_OK;
}

int lshbloom_query(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                   lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_sigs || !d_flags))) {
    set_err("query: need n_docs >= 0 and non-null sigs and flags");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query: stream wait");
  for (int64_t c0 = 0; c0 < n_docs; c0 += (int64_t)h->chunk_docs) {
    const int64_t cn = std::min<int64_t>((int64_t)h->chunk_docs, n_docs - c0);
    lb::BloomLaunch a = bloom_args(h, d_sigs + c0 * (int64_t)h->prm.num_perm, cn);
    a.flags = d_flags + c0;
    e = lb::launch_query(a, s);
    if (e != hipSuccess) return fail_hip(h, e, "query: launch");
  }
  e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query: event");
  return LSHBLOOM_OK;
}

int lshbloom_insert(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && !d_sigs)) {
    set_err("insert: need n_docs >= 0 and non-null sigs");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  if (forced_fault(h)) return LSHBLOOM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "insert: stream wait");
  lb::BloomLaunch a = bloom_args(h, d_sigs, n_docs);
  e = lb::launch_insert(a, s);
  if (e != hipSuccess) return fail_hip(h, e, "insert: launch");
  e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "insert: event");
  h->docs_inserted += (uint64_t)n_docs;
  return LSHBLOOM_OK;
}

int lshbloom_band_keys(lshbloom_t *h, const uint32_t *d_sigs, int64_t n_docs, uint64_t *d_keys,
                       lshbloom_stream_t stream) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_sigs || !d_keys))) {
    set_err("band_keys: need n_docs >= 0 and non-null sigs and keys");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  lb::BloomLaunch a = bloom_args(h, d_sigs, n_docs);
  a.keys = d_keys;
  hipError_t e = lb::launch_band_keys(a, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "band_keys: launch");
  return LSHBLOOM_OK;
}

int lshbloom_minhash61(lshbloom_t *h, const int64_t *d_offsets, const uint32_t *d_tokens, int64_t n_docs,
                       uint64_t *d_sigs, lshbloom_stream_t stream) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_offsets || !d_sigs || !d_tokens))) {
    set_err("minhash61: need n_docs >= 0 and non-null offsets, tokens and sigs");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = lb::launch_fill_u64(d_sigs, (uint64_t)n_docs * h->prm.num_perm, ~0ull, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "minhash61: fill");
  lb::MinhashLaunch a{};
  a.offsets = d_offsets;
  a.tokens = d_tokens;
  a.n_docs = n_docs;
  a.coef = h->d_coef;
  a.sigs64 = d_sigs;
  a.num_perm = h->prm.num_perm;
  a.w = h->prm.shingle_width;
  a.waves = h->minhash_waves ? h->minhash_waves : lb::minhash_waves_for_docs(h->cus, (uint64_t)n_docs);
  e = lb::launch_minhash(a, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "minhash61: launch");
  return LSHBLOOM_OK;
}

int lshbloom_band_keys61(lshbloom_t *h, const uint64_t *d_sigs, int64_t n_docs, uint64_t *d_keys,
                         lshbloom_stream_t stream) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_sigs || !d_keys))) {
    set_err("band_keys61: need n_docs >= 0 and non-null sigs and keys");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  lb::BloomLaunch a = bloom_args(h, nullptr, n_docs);
  a.sigs64 = d_sigs;
  a.keys = d_keys;
  hipError_t e = lb::launch_band_keys61(a, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "band_keys61: launch");
  return LSHBLOOM_OK;
}

int lshbloom_query_insert_keys(lshbloom_t *h, const uint64_t *d_keys, int64_t n_docs, uint8_t *d_flags,
                               lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  if (n_docs < 0 || (n_docs > 0 && (!d_keys || !d_flags))) {
    set_err("query_insert_keys: need n_docs >= 0 and non-null keys and flags");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  if (forced_fault(h)) return LSHBLOOM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query_insert_keys: stream wait");
  rc = lbh::qi_enqueue(h, nullptr, n_docs, d_flags, s, d_keys);
  if (rc) return rc;
  e = lbh::finish_qi(h, s);
  if (e == hipSuccess) e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "query_insert_keys: event");
  h->docs_inserted += (uint64_t)n_docs;
  return LSHBLOOM_OK;
}

int lshbloom_read_filters(lshbloom_t *h, void *dst, uint64_t offset, uint64_t nbytes, lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  const uint64_t total = h->m_bits / 8 * h->prm.bands;
  if (!dst || offset > total || nbytes > total - offset) {
    set_err("read_filters: range [%llu, +%llu) outside the %llu filter bytes", (unsigned long long)offset,
            (unsigned long long)nbytes, (unsigned long long)total);
    return LSHBLOOM_EINVAL;
  }
  if (nbytes == 0) return LSHBLOOM_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "read_filters: stream wait");
  e = hipMemcpyAsync(dst, (const char *)h->d_filters + offset, nbytes, hipMemcpyDefault, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "read_filters: copy");
  e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "read_filters: event");
  return LSHBLOOM_OK;
}

namespace {

struct FileHeader {
  char magic[8];
  uint32_t num_perm, bands, rows, shingle_width;
  uint64_t expected_n;
  double fp_rate;
  uint64_t seed, m_bits;
  uint32_t k, reserved;
  uint64_t docs_inserted, words_per_band;
};
static_assert(sizeof(FileHeader) == 80, "file header layout");
constexpr char kMagic[8] = {'L', 'S', 'H', 'B', 'L', 'M', '0', '1'};
constexpr size_t kStageBytes = 64ull << 20;

struct PinnedStage {
  void *p = nullptr;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
};

}  // namespace

int lshbloom_save(lshbloom_t *h, const char *path, lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  if (!path) {
    set_err("save: path is NULL");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  PinnedStage st;
  hipError_t e = hipHostMalloc(&st.p, kStageBytes, hipHostMallocDefault);
  if (e != hipSuccess) return fail_hip(nullptr, e, "save: pinned staging");
  FILE *f = std::fopen(path, "wb");
  if (!f) {
    set_err("save: cannot create %s", path);
    return LSHBLOOM_EIO;
  }
  FileHeader hd{};
  std::memcpy(hd.magic, kMagic, 8);
  hd.num_perm = h->prm.num_perm;
  hd.bands = h->prm.bands;
  hd.rows = h->prm.rows;
  hd.shingle_width = h->prm.shingle_width;
  hd.expected_n = h->prm.expected_n;
  hd.fp_rate = h->prm.fp_rate;
  hd.seed = h->prm.seed;
  hd.m_bits = h->m_bits;
  hd.k = h->k;
  hd.docs_inserted = h->docs_inserted;
  hd.words_per_band = h->words_per_band;
  bool ok = std::fwrite(&hd, sizeof hd, 1, f) == 1;
  e = begin_ordered(h, s);
  const uint64_t total = h->m_bits / 8 * h->prm.bands;
  for (uint64_t off = 0; ok && e == hipSuccess && off < total; off += kStageBytes) {
    const size_t nb = (size_t)std::min<uint64_t>(kStageBytes, total - off);
    e = hipMemcpyAsync(st.p, (const char *)h->d_filters + off, nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) ok = std::fwrite(st.p, 1, nb, f) == nb;
  }
  if (e == hipSuccess) e = end_ordered(h, s);
  ok = (std::fclose(f) == 0) && ok;
  if (e != hipSuccess) return fail_hip(nullptr, e, "save: copy");
  if (!ok) {
    set_err("save: writing %s failed", path);
    return LSHBLOOM_EIO;
  }
  return LSHBLOOM_OK;
}

int lshbloom_load(lshbloom_t *h, const char *path, lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  if (!path) {
    set_err("load: path is NULL");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    set_err("load: cannot open %s", path);
    return LSHBLOOM_EIO;
  }
  FileHeader hd{};
  if (std::fread(&hd, sizeof hd, 1, f) != 1 || std::memcmp(hd.magic, kMagic, 8) != 0) {
    std::fclose(f);
    set_err("load: %s is not an index file", path);
    return LSHBLOOM_EIO;
  }
  if (hd.num_perm != h->prm.num_perm || hd.bands != h->prm.bands || hd.rows != h->prm.rows ||
      hd.shingle_width != h->prm.shingle_width || hd.seed != h->prm.seed || hd.m_bits != h->m_bits ||
      hd.k != h->k || hd.words_per_band != h->words_per_band) {
    std::fclose(f);
    set_err("load: %s holds an index of other parameters (P %u, b %u, r %u, w %u, seed %llu, m %llu, k %u)", path,
            hd.num_perm, hd.bands, hd.rows, hd.shingle_width, (unsigned long long)hd.seed,
            (unsigned long long)hd.m_bits, hd.k);
    return LSHBLOOM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  PinnedStage st;
  hipError_t e = hipHostMalloc(&st.p, kStageBytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    std::fclose(f);
    return fail_hip(nullptr, e, "load: pinned staging");
  }
  e = begin_ordered(h, s);
  const uint64_t total = h->m_bits / 8 * h->prm.bands;
  bool ok = true;
  for (uint64_t off = 0; ok && e == hipSuccess && off < total; off += kStageBytes) {
    const size_t nb = (size_t)std::min<uint64_t>(kStageBytes, total - off);
    e = hipStreamSynchronize(s);  // the staging buffer is free again
    if (e == hipSuccess) ok = std::fread(st.p, 1, nb, f) == nb;
    if (e == hipSuccess && ok) e = hipMemcpyAsync((char *)h->d_filters + off, st.p, nb, hipMemcpyHostToDevice, s);
  }
  std::fclose(f);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "load: copy");
  if (!ok) {
    h->poisoned = true;
    set_err("load: %s is shorter than its header says; the filters are partly overwritten", path);
    return LSHBLOOM_EIO;
  }
  h->docs_inserted = hd.docs_inserted;
  return LSHBLOOM_OK;
}

int lshbloom_count_set_bits(lshbloom_t *h, uint64_t *out, lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  if (!out) {
    set_err("count_set_bits: out is NULL");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "count_set_bits: stream wait");
  if ((e = lb::launch_fill_u64(h->d_count, h->prm.bands, 0, s)) != hipSuccess ||
      (e = lb::launch_popcount(h->d_filters, h->words_per_band, h->prm.bands, h->d_count, s)) != hipSuccess)
    return fail_hip(h, e, "count_set_bits: launch");
  e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "count_set_bits: event");
  if ((e = hipMemcpyAsync(out, h->d_count, (size_t)h->prm.bands * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return fail_hip(h, e, "count_set_bits: copy");
  return LSHBLOOM_OK;
}

int lshbloom_write_filters(lshbloom_t *h, const void *src, uint64_t offset, uint64_t nbytes, uint64_t docs_inserted,
                           lshbloom_stream_t stream) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = check_ready(h);
  if (rc) return rc;
  const uint64_t total = h->m_bits / 8 * h->prm.bands;
  if (!src || offset > total || nbytes > total - offset) {
    set_err("write_filters: range [%llu, +%llu) outside the %llu filter bytes", (unsigned long long)offset,
            (unsigned long long)nbytes, (unsigned long long)total);
    return LSHBLOOM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = begin_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "write_filters: stream wait");
  if (nbytes) {
    e = hipMemcpyAsync((char *)h->d_filters + offset, src, nbytes, hipMemcpyDefault, s);
    if (e != hipSuccess) return fail_hip(h, e, "write_filters: copy");
  }
  e = end_ordered(h, s);
  if (e != hipSuccess) return fail_hip(h, e, "write_filters: event");
  if (docs_inserted != UINT64_MAX) h->docs_inserted = docs_inserted;
  return LSHBLOOM_OK;
}

int lshbloom_sync(lshbloom_t *h) {
  if (!h) return check_ready(h);
  std::lock_guard<std::mutex> lk(h->mu);
  if (h->has_last) {
    const hipError_t e = hipEventSynchronize(h->last);
    if (e != hipSuccess) return fail_hip(h, e, "sync");
  }
  return check_ready(h);
}

int lshbloom_info(const lshbloom_t *hc, lshbloom_info_t *out) {
  if (!hc || !out) {
    set_err("info: null argument");
    return LSHBLOOM_EINVAL;
  }
  const lshbloom *h = hc;
  std::memset(out, 0, sizeof *out);
  out->num_perm = h->prm.num_perm;
  out->bands = h->prm.bands;
  out->rows = h->prm.rows;
  out->shingle_width = h->prm.shingle_width;
  out->k = h->k;
  out->m_bits = h->m_bits;
  out->words_per_band = h->words_per_band;
  out->filter_bytes = h->m_bits / 8 * h->prm.bands;
  out->workspace_bytes = h->workspace_bytes;
  out->chunk_docs = h->chunk_docs;
  out->binned_chunk_docs = h->bin_chunk;
  out->fp_rate = h->prm.fp_rate;
  out->p_eff = -std::expm1((double)h->prm.bands * std::log1p(-h->prm.fp_rate));
  out->docs_inserted = h->docs_inserted;
  out->seed = h->prm.seed;
  out->poisoned = h->poisoned ? 1 : 0;
  // Internal consistency word written by the kernels (0 = consistent); read
  // after the handle's last call.
  lshbloom *hm = const_cast<lshbloom *>(h);
  std::lock_guard<std::mutex> lk(hm->mu);
  if (hm->has_last) (void)hipEventSynchronize(hm->last);
  uint32_t st = 0;
  if (hipMemcpy(&st, hm->d_status, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) st = 0xFFFFFFFFu;
  out->device_status = st;
  uint64_t gp = 0;
  if (hipMemcpy(&gp, hm->d_status + 2, sizeof gp, hipMemcpyDeviceToHost) != hipSuccess) gp = ~0ull;
  out->general_path_bins = gp;
  return LSHBLOOM_OK;
}

}  // extern "C"
