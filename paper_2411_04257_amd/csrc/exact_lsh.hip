// Exact MinHashLSH band index: the traditional index LSHBloom replaces
// (Section 2.3, "MinHashLSH for Text Deduplication"; Section 4), kept on the
// device as the comparison baseline.
//
// Per band an open-addressing table of 2^t slots (load <= 1/2 at capacity):
// a fingerprint of the band's r values (0 = empty), the band's r values
// themselves, and the least stream index of a document holding them.  A
// 64-bit hash of the values gives the first slot (high bits) and the
// fingerprint (low bits).
// A call is processed in chunks; per chunk, with one thread per (document,
// band) item:
//
//   claim   (k_ex_claim): probe from the fingerprint's slot; an empty slot is
//           claimed by compare-and-swap of the fingerprint and the claimer
//           writes its r values; a slot holding the same fingerprint is the
//           item's tentative slot;
//   verify  (k_ex_verify): the r values are compared with the slot's (all
//           written by the previous kernel); equal -> atomicMin of the
//           document index into the slot; different (another band's values
//           with the same fingerprint) -> the item joins a list;
//   settle  (k_ex_settle): one thread places the listed items by full
//           comparison of the r values, creating slots as needed;
//   flags   (k_ex_flags): document i is flagged iff some band's slot holds
//           a document index below its own.
//
// So a band equal to an earlier document's band (of an earlier call or
// earlier in the chunk) is found whatever the fingerprints do: the result is
// the exact sequential definition for every chunking.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_math.h"
#include "handle.h"

namespace {

constexpr uint32_t kT = 256;
constexpr uint32_t kNoDoc = 0xFFFFFFFFu;
constexpr uint32_t kOwner = 0x80000000u;  // slot claimed by this item
constexpr uint64_t kChunkDocs = 1ull << 20;
constexpr uint64_t kMaxCapacity = 1ull << 30;  // slot indices < 2^31

struct ExLaunch {
  const uint32_t *sigs;
  int64_t n;
  uint32_t num_perm, bands, rows;
  uint64_t slots, mask, fp_mask;
  uint64_t *fp;       // [bands][slots]
  uint32_t *first;    // [bands][slots]
  uint32_t *vals;     // [bands][slots][rows]
  uint32_t *slot;     // [n][bands]: slot | kOwner
  uint32_t *list;     // [n * bands] items to settle
  uint32_t *count;    // [1] list length (cleared by k_ex_settle)
  uint64_t *shared;   // [1] total items settled so far
  uint32_t base;      // stream index of the chunk's first document
  uint8_t *flags;
};

// 64-bit hash of a band's values: its high bits pick the first slot, its
// low fp_bits (0 mapped to 1: 0 marks an empty slot) are the fingerprint.
__device__ __forceinline__ uint64_t band_hash(const uint32_t *v, uint32_t rows) {
  uint64_t h = 0x243F6A8885A308D3ull;
  for (uint32_t t = 0; t < rows; ++t) h = lb::fmix64(h + ((uint64_t)t << 32 | v[t]));
  return h;
}
__device__ __forceinline__ uint64_t fp_of(uint64_t h, uint64_t fp_mask) { return (h & fp_mask) ? (h & fp_mask) : 1; }

__device__ __forceinline__ bool same_vals(const uint32_t *a, const uint32_t *b, uint32_t rows) {
  bool eq = true;
  for (uint32_t t = 0; t < rows; ++t) eq &= a[t] == b[t];
  return eq;
}

__global__ __launch_bounds__(kT) void k_ex_claim(ExLaunch A) {
  const int64_t it = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (it >= A.n * A.bands) return;
  const int64_t i = it / A.bands;
  const uint32_t j = (uint32_t)(it - i * A.bands);
  const uint32_t *v = A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows;
  const uint64_t hv = band_hash(v, A.rows), f = fp_of(hv, A.fp_mask);
  uint64_t *F = A.fp + (uint64_t)j * A.slots;
  uint64_t s = (hv >> 33) & A.mask;
  uint32_t res = kNoDoc;
  for (uint64_t probe = 0; probe < A.slots; ++probe) {
    uint64_t cur = __hip_atomic_load(&F[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == 0) {
      cur = atomicCAS((unsigned long long *)&F[s], 0ull, (unsigned long long)f);
      if (cur == 0) {
        uint32_t *dst = A.vals + ((uint64_t)j * A.slots + s) * A.rows;
        for (uint32_t t = 0; t < A.rows; ++t) dst[t] = v[t];
        res = (uint32_t)s | kOwner;
        break;
      }
    }
    if (cur == f) {
      res = (uint32_t)s;
      break;
    }
    s = (s + 1) & A.mask;
  }
  A.slot[it] = res;  // kNoDoc cannot happen: the table is at most half full
}

__global__ __launch_bounds__(kT) void k_ex_verify(ExLaunch A) {
  const int64_t it = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (it >= A.n * A.bands) return;
  const int64_t i = it / A.bands;
  const uint32_t j = (uint32_t)(it - i * A.bands);
  const uint32_t r = A.slot[it];
  const uint32_t doc = A.base + (uint32_t)i;
  const uint64_t s = r & ~kOwner;
  bool match = (r & kOwner) != 0;
  if (!match && r != kNoDoc) {
    const uint32_t *v = A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows;
    match = same_vals(v, A.vals + ((uint64_t)j * A.slots + s) * A.rows, A.rows);
  }
  if (match) {
    atomicMin(&A.first[(uint64_t)j * A.slots + s], doc);
  } else {
    A.list[atomicAdd(A.count, 1u)] = (uint32_t)it;
    A.slot[it] = kNoDoc;
  }
}

// One thread: exact placement of the listed items (fingerprint shared by
// different band values; none in practice with 64-bit fingerprints).
__global__ void k_ex_settle(ExLaunch A) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t cnt = *A.count;
  for (uint32_t q = 0; q < cnt; ++q) {
    const uint32_t it = A.list[q];
    const int64_t i = it / A.bands;
    const uint32_t j = (uint32_t)(it - i * A.bands);
    const uint32_t *v = A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows;
    const uint32_t doc = A.base + (uint32_t)i;
    const uint64_t hv = band_hash(v, A.rows), f = fp_of(hv, A.fp_mask);
    uint64_t *F = A.fp + (uint64_t)j * A.slots;
    uint64_t s = (hv >> 33) & A.mask;
    for (uint64_t probe = 0; probe < A.slots; ++probe) {
      uint32_t *sv = A.vals + ((uint64_t)j * A.slots + s) * A.rows;
      uint32_t *fs = &A.first[(uint64_t)j * A.slots + s];
      if (F[s] == 0) {
        F[s] = f;
        for (uint32_t t = 0; t < A.rows; ++t) sv[t] = v[t];
        *fs = doc;
        A.slot[it] = (uint32_t)s;
        break;
      }
      if (F[s] == f && same_vals(v, sv, A.rows)) {
        *fs = min(*fs, doc);
        A.slot[it] = (uint32_t)s;
        break;
      }
      s = (s + 1) & A.mask;
    }
  }
  *A.shared += cnt;
  *A.count = 0;
}

__global__ __launch_bounds__(kT) void k_ex_flags(ExLaunch A) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= A.n) return;
  const uint32_t doc = A.base + (uint32_t)i;
  uint8_t hit = 0;
  for (uint32_t j = 0; j < A.bands; ++j) {
    const uint32_t s = A.slot[i * A.bands + j] & ~kOwner;
    // every item has a slot (the tables are at most half full); the bound
    // keeps a broken invariant from reading outside them
    if (s < A.slots) hit |= A.first[(uint64_t)j * A.slots + s] < doc ? 1 : 0;
  }
  A.flags[i] = hit;
}

template <typename T>
__global__ void k_ex_fill(T *p, uint64_t n, T v) {
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (uint64_t)gridDim.x * blockDim.x)
    p[q] = v;
}

unsigned grid_of(uint64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

struct lshbloom_exact {
  uint32_t num_perm = 0, bands = 0, rows = 0;
  uint64_t capacity = 0, slots = 0, fp_mask = 0, chunk = 0;
  uint64_t *fp = nullptr, *shared = nullptr;
  uint32_t *first = nullptr, *vals = nullptr, *slot = nullptr, *list = nullptr, *count = nullptr;
  uint64_t table_bytes = 0;
  uint64_t docs_inserted = 0;
  int device = 0;
  hipEvent_t last = nullptr;
  bool has_last = false;
  bool poisoned = false;
  std::mutex mu;
};

namespace {

void ex_free(lshbloom_exact *x) {
  (void)hipFree(x->fp);
  (void)hipFree(x->shared);
  (void)hipFree(x->first);
  (void)hipFree(x->vals);
  (void)hipFree(x->slot);
  (void)hipFree(x->list);
  (void)hipFree(x->count);
  if (x->last) (void)hipEventDestroy(x->last);
  delete x;
}

int ex_hip(lshbloom_exact *x, hipError_t e, const char *what) {
  lbh::set_err("exact %s: %s", what, hipGetErrorString(e));
  if (x) x->poisoned = true;
  return LSHBLOOM_EHIP;
}

}  // namespace

extern "C" {

lshbloom_exact_t *lshbloom_exact_create(uint32_t num_perm, uint32_t bands, uint32_t rows, uint64_t capacity_docs,
                                        uint32_t fp_bits) {
  if (num_perm == 0 || num_perm > LSHBLOOM_MAX_NUM_PERM || bands == 0 || bands > LSHBLOOM_MAX_BANDS || rows == 0 ||
      (uint64_t)bands * rows > num_perm) {
    lbh::set_err("exact_create: need 0 < bands <= %u, rows > 0, bands * rows <= num_perm <= %u", LSHBLOOM_MAX_BANDS,
                 LSHBLOOM_MAX_NUM_PERM);
    return nullptr;
  }
  if (capacity_docs == 0 || capacity_docs > kMaxCapacity) {
    lbh::set_err("exact_create: capacity_docs must be in [1, 2^30]");
    return nullptr;
  }
  if (fp_bits > 64) {
    lbh::set_err("exact_create: fp_bits must be in [0, 64]");
    return nullptr;
  }
  lshbloom_exact *x = new lshbloom_exact();
  x->num_perm = num_perm;
  x->bands = bands;
  x->rows = rows;
  x->capacity = capacity_docs;
  uint64_t slots = 2;
  while (slots < 2 * capacity_docs) slots <<= 1;
  x->slots = slots;
  x->fp_mask = (fp_bits == 0 || fp_bits == 64) ? ~0ull : ((1ull << fp_bits) - 1);
  x->chunk = capacity_docs < kChunkDocs ? capacity_docs : kChunkDocs;
  (void)hipGetDevice(&x->device);
  const uint64_t ns = slots * bands;
  const uint64_t items = x->chunk * bands;
  x->table_bytes = ns * (8 + 4 + 4ull * rows);
  hipError_t e = hipSuccess;
  auto alloc = [&](void **p, uint64_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void **)&x->fp, ns * 8);
  alloc((void **)&x->first, ns * 4);
  alloc((void **)&x->vals, ns * 4 * rows);
  alloc((void **)&x->slot, items * 4);
  alloc((void **)&x->list, items * 4);
  alloc((void **)&x->count, 4);
  alloc((void **)&x->shared, 8);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&x->last, hipEventDisableTiming);
  if (e != hipSuccess) {
    lbh::set_err("exact_create: %s (%llu bytes of tables)", hipGetErrorString(e), (unsigned long long)x->table_bytes);
    ex_free(x);
    return nullptr;
  }
  hipLaunchKernelGGL(k_ex_fill<uint64_t>, dim3(1024), dim3(kT), 0, 0, x->fp, ns, (uint64_t)0);
  hipLaunchKernelGGL(k_ex_fill<uint32_t>, dim3(1024), dim3(kT), 0, 0, x->first, ns, kNoDoc);
  hipLaunchKernelGGL(k_ex_fill<uint32_t>, dim3(1), dim3(kT), 0, 0, x->count, (uint64_t)1, 0u);
  hipLaunchKernelGGL(k_ex_fill<uint64_t>, dim3(1), dim3(kT), 0, 0, x->shared, (uint64_t)1, (uint64_t)0);
  e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    lbh::set_err("exact_create: %s", hipGetErrorString(e));
    ex_free(x);
    return nullptr;
  }
  return x;
}

void lshbloom_exact_destroy(lshbloom_exact_t *x) {
  if (!x) return;
  if (x->has_last) (void)hipEventSynchronize(x->last);
  ex_free(x);
}

int lshbloom_exact_query_insert(lshbloom_exact_t *x, const uint32_t *d_sigs, int64_t n_docs, uint8_t *d_flags,
                                lshbloom_stream_t stream) {
  if (!x) {
    lbh::set_err("null handle");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(x->mu);
  if (x->poisoned) {
    lbh::set_err("exact index poisoned by an earlier device error");
    return LSHBLOOM_EPOISONED;
  }
  if (n_docs < 0 || (n_docs > 0 && (!d_sigs || !d_flags))) {
    lbh::set_err("exact_query_insert: need n_docs >= 0 and non-null sigs and flags");
    return LSHBLOOM_EINVAL;
  }
  if (n_docs == 0) return LSHBLOOM_OK;
  if (x->docs_inserted + (uint64_t)n_docs > x->capacity) {
    lbh::set_err("exact_query_insert: %llu documents would exceed the capacity of %llu",
                 (unsigned long long)(x->docs_inserted + n_docs), (unsigned long long)x->capacity);
    return LSHBLOOM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (x->has_last) e = hipStreamWaitEvent(s, x->last, 0);
  if (e != hipSuccess) return ex_hip(x, e, "stream wait");
  for (int64_t c0 = 0; c0 < n_docs; c0 += (int64_t)x->chunk) {
    const int64_t cn = std::min<int64_t>((int64_t)x->chunk, n_docs - c0);
    ExLaunch a{};
    a.sigs = d_sigs + c0 * (int64_t)x->num_perm;
    a.n = cn;
    a.num_perm = x->num_perm;
    a.bands = x->bands;
    a.rows = x->rows;
    a.slots = x->slots;
    a.mask = x->slots - 1;
    a.fp_mask = x->fp_mask;
    a.fp = x->fp;
    a.first = x->first;
    a.vals = x->vals;
    a.slot = x->slot;
    a.list = x->list;
    a.count = x->count;
    a.shared = x->shared;
    a.base = (uint32_t)(x->docs_inserted + (uint64_t)c0);
    a.flags = d_flags + c0;
    const uint64_t items = (uint64_t)cn * x->bands;
    hipLaunchKernelGGL(k_ex_claim, dim3(grid_of(items)), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_ex_verify, dim3(grid_of(items)), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_ex_settle, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_ex_flags, dim3(grid_of((uint64_t)cn)), dim3(kT), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return ex_hip(x, e, "launch");
  }
  e = hipEventRecord(x->last, s);
  if (e != hipSuccess) return ex_hip(x, e, "event");
  x->has_last = true;
  x->docs_inserted += (uint64_t)n_docs;
  return LSHBLOOM_OK;
}

int lshbloom_exact_stats(lshbloom_exact_t *x, uint64_t *docs_inserted, uint64_t *table_bytes, uint64_t *fp_shared) {
  if (!x) {
    lbh::set_err("null handle");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(x->mu);
  if (docs_inserted) *docs_inserted = x->docs_inserted;
  if (table_bytes) *table_bytes = x->table_bytes;
  if (fp_shared) {
    hipError_t e = x->has_last ? hipEventSynchronize(x->last) : hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(fp_shared, x->shared, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ex_hip(x, e, "stats");
  }
  return LSHBLOOM_OK;
}

}  // extern "C"
