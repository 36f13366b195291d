// Batched form of the hot path: a host-to-host pipeline around one handle.
//
// Each submitted batch (host CSR in, host flags out) goes through
//   host:   CSR check, length bucketing (documents grouped by token count so
//           that each bucket runs its own persistent MinHash launch with its
//           own grid), bucket descriptors into pinned memory;
//   copy stream: H2D tokens + descriptors, one batch after another in
//           submission order (each copy gets the link to itself, so copies of
//           two batches do not share it and finish together);
//   MinHash stream (graph G1 of the batch's slot): after its batch's copy and
//           after the partition passes of the previous batch's query-insert,
//           signature pre-fill and one MinHash launch per non-empty bucket;
//   query-insert stream: after G1 of this batch and after every earlier
//           filter call of the handle, the partition passes (graph G2), an
//           event, the bins and resolve (graph G3), then the status word's
//           and the flags' copies to the host.
// Two slots of buffers alternate, so the copy of batch t+1 overlaps the
// query-insert of batch t, and the MinHash of batch t+1 runs beside the bins
// of batch t (the partition passes fill every compute unit; the bin kernel
// leaves room), while query-inserts stay in submission order.
// Per-batch device work is captured into a hipGraph per slot and stage and
// replayed (the executable graph is updated in place when only launch
// parameters change).  A small autotuner times candidate bucket edges and
// grid sizes for MinHash on the first batch (MinHash is stateless, so
// tuning changes no result) and can persist its choice in a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"

namespace {

constexpr int kSlots = 2;
constexpr uint32_t kMaxBuckets = 4;

struct Slot {
  hipEvent_t copied = nullptr, mh_done = nullptr, done = nullptr;
  // timing events around the batch's MinHash stage (MinHash stream) and its
  // query-insert kernels (query-insert stream)
  hipEvent_t mh_t0 = nullptr, mh_t1 = nullptr, qi_t0 = nullptr, qi_t1 = nullptr;
  int64_t *h_desc = nullptr;     // pinned bucket descriptors
  uint32_t *h_tokens = nullptr;  // pinned token staging (used when the caller's buffer is pageable)
  uint8_t *h_flags = nullptr;    // pinned flags
  uint32_t *d_tokens = nullptr;
  int64_t *d_desc = nullptr;
  uint32_t *d_sigs = nullptr;
  uint8_t *d_flags = nullptr;
  hipGraphExec_t g1 = nullptr, g2 = nullptr, g3 = nullptr;
  int64_t ticket = -1, n_docs = 0;
  uint8_t *user_flags = nullptr;
  bool pending = false;
};

struct Buckets {
  uint32_t n = 1;
  uint64_t edges[kMaxBuckets - 1] = {0, 0, 0};
  uint32_t waves_per_cu[kMaxBuckets] = {0, 0, 0, 0};  // 0: sized by the bucket's tokens
};

}  // namespace

struct lshbloom_pipeline {
  lshbloom *h = nullptr;
  lshbloom_pipeline_params_t prm{};
  Buckets bk;
  int cus = 256;
  // One stream per stage: the MinHash launches of every batch (one after the
  // other: each fills the device), the query-inserts in submission order, and
  // the host-to-device copies.  With the process's null stream that is four
  // streams, so under the runtime's default of four hardware queues each gets
  // a queue of its own (two streams that share a queue run one after the other).
  hipStream_t qi_stream = nullptr;
  hipStream_t mh_stream = nullptr;
  hipStream_t copy_stream = nullptr;
  // Recorded on the query-insert stream when the partition passes of the
  // latest enqueued query-insert are done: the next batch's MinHash waits for
  // it, so that it runs beside the memory-bound bin kernels rather than the
  // partition passes (whose one-workgroup-per-compute-unit launches leave no
  // room for MinHash waves).
  hipEvent_t qi_mid = nullptr;
  bool has_mid = false;
  Slot slot[kSlots];
  int64_t next_ticket = 0;
  bool tuned = false;
  uint64_t graph_launches = 0, graph_updates = 0, graph_instantiations = 0;
  float tune_best_ms = 0.f;
  uint64_t timed_batches = 0;
  double minhash_ms_total = 0.0, qi_ms_total = 0.0;
  std::mutex mu;
};

namespace {

using lbh::fail_hip;
using lbh::set_err;

// Descriptor layout for B buckets of a batch with n documents:
//   [0, B)                 counts
//   then per bucket b:     voff (count_b + 1), tok_shift (count_b), row (count_b)
uint64_t desc_words(uint64_t max_docs) { return kMaxBuckets + 3 * max_docs + kMaxBuckets; }

struct BucketView {
  int64_t count, tokens;
  uint64_t voff, shift, row;  // word offsets into the descriptor array
};

// Host bucketing: stable by document order within each bucket.
void build_buckets(const Buckets &bk, const int64_t *off, int64_t n, int64_t *desc, BucketView *views) {
  int64_t cnt[kMaxBuckets] = {0, 0, 0, 0};
  auto bucket_of = [&](int64_t L) {
    uint32_t b = 0;
    while (b + 1 < bk.n && (uint64_t)L >= bk.edges[b]) ++b;
    return b;
  };
  for (int64_t d = 0; d < n; ++d) cnt[bucket_of(off[d + 1] - off[d])]++;
  uint64_t pos = kMaxBuckets;
  for (uint32_t b = 0; b < kMaxBuckets; ++b) {
    desc[b] = b < bk.n ? cnt[b] : 0;
    views[b].count = b < bk.n ? cnt[b] : 0;
    views[b].voff = pos;
    pos += views[b].count + 1;
    views[b].shift = pos;
    pos += views[b].count;
    views[b].row = pos;
    pos += views[b].count;
  }
  int64_t fill[kMaxBuckets] = {0, 0, 0, 0};
  int64_t vsum[kMaxBuckets] = {0, 0, 0, 0};
  for (uint32_t b = 0; b < bk.n; ++b) desc[views[b].voff] = 0;
  const int64_t base = off[0];
  for (int64_t d = 0; d < n; ++d) {
    const int64_t L = off[d + 1] - off[d];
    const uint32_t b = bucket_of(L);
    const int64_t q = fill[b]++;
    desc[views[b].shift + q] = (off[d] - base) - vsum[b];
    desc[views[b].row + q] = d;
    vsum[b] += L;
    desc[views[b].voff + q + 1] = vsum[b];
  }
  for (uint32_t b = 0; b < kMaxBuckets; ++b) views[b].tokens = vsum[b];
}

hipError_t enqueue_minhash(lshbloom_pipeline *pl, Slot &S, const BucketView *views, int64_t n,
                           const Buckets &bk) {
  lshbloom *h = pl->h;
  hipError_t e = lb::launch_fill_u32(S.d_sigs, (uint64_t)n * h->prm.num_perm, 0xFFFFFFFFu, pl->mh_stream);
  if (e != hipSuccess) return e;
  for (uint32_t b = 0; b < bk.n; ++b) {
    if (views[b].count == 0) continue;
    lb::MinhashLaunch a{};
    a.offsets = S.d_desc + views[b].voff;
    a.tokens = S.d_tokens;
    a.n_docs = views[b].count;
    a.coef = h->d_coef;
    a.sigs = S.d_sigs;
    a.num_perm = h->prm.num_perm;
    a.w = h->prm.shingle_width;
    a.waves = bk.waves_per_cu[b] ? std::max(4, (int)(bk.waves_per_cu[b] * pl->cus) / 4 * 4)
                                 : lb::minhash_waves_for_tokens(pl->cus, (uint64_t)views[b].tokens);
    a.tok_shift = S.d_desc + views[b].shift;
    a.row_ids = S.d_desc + views[b].row;
    e = lb::launch_minhash(a, pl->mh_stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Capture what `body` enqueues on `s` into a graph and launch it, reusing the
// slot's executable graph when the topology is unchanged.
template <class F>
hipError_t run_graph(lshbloom_pipeline *pl, hipStream_t s, hipGraphExec_t &exec, F body) {
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t eb = body();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (eb != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return eb;
  }
  if (e != hipSuccess) return e;
  bool updated = false;
  if (exec) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      updated = true;
      pl->graph_updates++;
    } else {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
  }
  if (!updated) {
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return e;
    }
    pl->graph_instantiations++;
  }
  (void)hipGraphDestroy(g);
  pl->graph_launches++;
  return hipGraphLaunch(exec, s);
}

bool is_pinned(const void *p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeHost;
}

std::string tune_key(lshbloom_pipeline *pl, const int64_t *off, int64_t n) {
  std::vector<int64_t> L(n);
  for (int64_t d = 0; d < n; ++d) L[d] = off[d + 1] - off[d];
  std::sort(L.begin(), L.end());
  char buf[256];
  snprintf(buf, sizeof buf, "P%u_w%u_n%lld_p50_%lld_p99_%lld", pl->h->prm.num_perm, pl->h->prm.shingle_width,
           (long long)n, (long long)(n ? L[n / 2] : 0), (long long)(n ? L[(n * 99) / 100] : 0));
  return buf;
}

bool load_tuned(lshbloom_pipeline *pl, const std::string &key) {
  if (!pl->prm.tune_cache) return false;
  FILE *f = fopen(pl->prm.tune_cache, "r");
  if (!f) return false;
  char line[512];
  bool ok = false;
  while (fgets(line, sizeof line, f)) {
    char k[256];
    unsigned nb, w0, w1, w2, w3;
    unsigned long long e0, e1, e2;
    if (sscanf(line, "%255s %u %llu %llu %llu %u %u %u %u", k, &nb, &e0, &e1, &e2, &w0, &w1, &w2, &w3) == 9 &&
        key == k && nb >= 1 && nb <= kMaxBuckets) {
      pl->bk.n = nb;
      pl->bk.edges[0] = e0;
      pl->bk.edges[1] = e1;
      pl->bk.edges[2] = e2;
      pl->bk.waves_per_cu[0] = w0;
      pl->bk.waves_per_cu[1] = w1;
      pl->bk.waves_per_cu[2] = w2;
      pl->bk.waves_per_cu[3] = w3;
      ok = true;
    }
  }
  fclose(f);
  return ok;
}

void save_tuned(lshbloom_pipeline *pl, const std::string &key) {
  if (!pl->prm.tune_cache) return;
  FILE *f = fopen(pl->prm.tune_cache, "a");
  if (!f) return;
  fprintf(f, "%s %u %llu %llu %llu %u %u %u %u\n", key.c_str(), pl->bk.n, (unsigned long long)pl->bk.edges[0],
          (unsigned long long)pl->bk.edges[1], (unsigned long long)pl->bk.edges[2], pl->bk.waves_per_cu[0],
          pl->bk.waves_per_cu[1], pl->bk.waves_per_cu[2], pl->bk.waves_per_cu[3]);
  fclose(f);
}

// Time MinHash of the staged batch (tokens already on the device) under
// candidate bucketings and grid sizes; keep the fastest.
int autotune(lshbloom_pipeline *pl, Slot &S, const int64_t *off, int64_t n) {
  const std::string key = tune_key(pl, off, n);
  if (load_tuned(pl, key)) {
    pl->tuned = true;
    return LSHBLOOM_OK;
  }
  std::vector<Buckets> cands;
  const uint64_t edge_sets[][3] = {{0, 0, 0}, {512, 0, 0}, {256, 8192, 0}, {64, 1024, 16384}};
  const uint32_t nbs[] = {1, 2, 3, 4};
  // per compute unit; 0 = by the bucket's tokens.  Grids of at most about a
  // hundred waves per compute unit leave room for the query-insert's bin
  // kernel beside which the MinHash of the next batch runs.
  const uint32_t waves[] = {0, 32, 64};
  for (int es = 0; es < 4; ++es)
    for (uint32_t w : waves) {
      Buckets b;
      b.n = nbs[es];
      for (int q = 0; q < 3; ++q) b.edges[q] = edge_sets[es][q];
      for (uint32_t q = 0; q < kMaxBuckets; ++q) b.waves_per_cu[q] = w;
      cands.push_back(b);
    }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail_hip(nullptr, hipGetLastError(), "autotune: event");
  float best = 1e30f;
  Buckets best_b = pl->bk;
  BucketView views[kMaxBuckets];
  for (const Buckets &b : cands) {
    build_buckets(b, off, n, S.h_desc, views);
    hipError_t e = hipMemcpyAsync(S.d_desc, S.h_desc, desc_words(n) * 8, hipMemcpyHostToDevice, pl->mh_stream);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, pl->mh_stream);
      if (e == hipSuccess) e = enqueue_minhash(pl, S, views, n, b);
      if (e == hipSuccess) e = hipEventRecord(e1, pl->mh_stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail_hip(nullptr, e, "autotune: timing run");
    }
    if (ms < best) {
      best = ms;
      best_b = b;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pl->bk = best_b;
  pl->tune_best_ms = best;
  pl->tuned = true;
  save_tuned(pl, key);
  return LSHBLOOM_OK;
}

void free_pipeline(lshbloom_pipeline *pl) {
  if (pl->mh_stream) (void)hipStreamSynchronize(pl->mh_stream);
  for (Slot &S : pl->slot) {
    if (S.g1) (void)hipGraphExecDestroy(S.g1);
    if (S.g2) (void)hipGraphExecDestroy(S.g2);
    if (S.g3) (void)hipGraphExecDestroy(S.g3);
    if (S.copied) (void)hipEventDestroy(S.copied);
    if (S.mh_done) (void)hipEventDestroy(S.mh_done);
    if (S.done) (void)hipEventDestroy(S.done);
    for (hipEvent_t ev : {S.mh_t0, S.mh_t1, S.qi_t0, S.qi_t1})
      if (ev) (void)hipEventDestroy(ev);
    if (S.h_desc) (void)hipHostFree(S.h_desc);
    if (S.h_tokens) (void)hipHostFree(S.h_tokens);
    if (S.h_flags) (void)hipHostFree(S.h_flags);
    if (S.d_tokens) (void)hipFree(S.d_tokens);
    if (S.d_desc) (void)hipFree(S.d_desc);
    if (S.d_sigs) (void)hipFree(S.d_sigs);
    if (S.d_flags) (void)hipFree(S.d_flags);
  }
  if (pl->qi_stream) {
    (void)hipStreamSynchronize(pl->qi_stream);
    (void)hipStreamDestroy(pl->qi_stream);
  }
  if (pl->copy_stream) {
    (void)hipStreamSynchronize(pl->copy_stream);
    (void)hipStreamDestroy(pl->copy_stream);
  }
  if (pl->mh_stream) (void)hipStreamDestroy(pl->mh_stream);
  if (pl->qi_mid) (void)hipEventDestroy(pl->qi_mid);
}

// Copy a finished slot's flags to the caller (after its done event), add its
// stage times, and report a device status raised by its query-insert (or an
// earlier call of the handle).
int collect(lshbloom_pipeline *pl, Slot &S) {
  if (!S.pending) return LSHBLOOM_OK;
  hipError_t e = hipEventSynchronize(S.done);
  if (e != hipSuccess) return fail_hip(nullptr, e, "pipeline: wait");
  if (S.n_docs) std::memcpy(S.user_flags, S.h_flags, (size_t)S.n_docs);
  S.pending = false;
  float mh = 0.f, qi = 0.f;
  if (S.n_docs && hipEventElapsedTime(&mh, S.mh_t0, S.mh_t1) == hipSuccess &&
      hipEventElapsedTime(&qi, S.qi_t0, S.qi_t1) == hipSuccess) {
    pl->timed_batches += 1;
    pl->minhash_ms_total += mh;
    pl->qi_ms_total += qi;
  }
  (void)hipGetLastError();
  std::lock_guard<std::mutex> hk(pl->h->mu);
  return lbh::check_ready(pl->h);
}

}  // namespace

extern "C" {

lshbloom_pipeline_t *lshbloom_pipeline_create(lshbloom_t *h, const lshbloom_pipeline_params_t *p) {
  if (!h || !p || p->max_docs == 0 || p->max_tokens == 0) {
    set_err("pipeline_create: need a handle, max_docs >= 1 and max_tokens >= 1");
    return nullptr;
  }
  if (p->n_buckets > kMaxBuckets) {
    set_err("pipeline_create: at most %u length buckets", kMaxBuckets);
    return nullptr;
  }
  lshbloom_pipeline *pl = new (std::nothrow) lshbloom_pipeline();
  if (!pl) {
    set_err("pipeline_create: out of host memory");
    return nullptr;
  }
  pl->h = h;
  pl->prm = *p;
  if (p->n_buckets) {
    pl->bk.n = p->n_buckets;
    for (uint32_t q = 0; q + 1 < p->n_buckets; ++q) pl->bk.edges[q] = p->bucket_edges[q];
    pl->tuned = true;  // explicit buckets: no tuning of the edges
  }
  for (uint32_t q = 0; q < kMaxBuckets; ++q)
    if (p->waves_per_cu[q]) pl->bk.waves_per_cu[q] = p->waves_per_cu[q];
  if (!p->autotune) pl->tuned = true;
  hipDeviceProp_t dp;
  hipError_t e = hipGetDeviceProperties(&dp, h->device);
  if (e == hipSuccess) pl->cus = dp.multiProcessorCount;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->qi_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->mh_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->copy_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->qi_mid, hipEventDisableTiming);
  const uint64_t P = h->prm.num_perm;
  for (int q = 0; q < kSlots && e == hipSuccess; ++q) {
    Slot &S = pl->slot[q];
    e = hipEventCreateWithFlags(&S.copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S.mh_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S.done, hipEventDisableTiming);
    for (hipEvent_t *ev : {&S.mh_t0, &S.mh_t1, &S.qi_t0, &S.qi_t1})
      if (e == hipSuccess) e = hipEventCreate(ev);
    if (e == hipSuccess) e = hipHostMalloc((void **)&S.h_desc, desc_words(p->max_docs) * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&S.h_tokens, p->max_tokens * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&S.h_flags, p->max_docs, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void **)&S.d_tokens, p->max_tokens * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&S.d_desc, desc_words(p->max_docs) * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&S.d_sigs, p->max_docs * P * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&S.d_flags, p->max_docs);
  }
  if (e != hipSuccess) {
    set_err("pipeline_create: %s", hipGetErrorString(e));
    free_pipeline(pl);
    delete pl;
    return nullptr;
  }
  return pl;
}

void lshbloom_pipeline_destroy(lshbloom_pipeline_t *pl) {
  if (!pl) return;
  {
    std::lock_guard<std::mutex> lk(pl->mu);
    for (Slot &S : pl->slot) (void)collect(pl, S);
    free_pipeline(pl);
  }
  delete pl;
}

int64_t lshbloom_pipeline_submit(lshbloom_pipeline_t *pl, const int64_t *h_offsets, const uint32_t *h_tokens,
                                 int64_t n_docs, uint8_t *h_flags) {
  if (!pl) {
    set_err("pipeline_submit: null pipeline");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(pl->mu);
  lshbloom *h = pl->h;
  if (const int crc = lbh::check_ready(h)) return crc;
  if (n_docs < 0 || (uint64_t)n_docs > pl->prm.max_docs || (n_docs > 0 && (!h_offsets || !h_flags))) {
    set_err("pipeline_submit: need 0 <= n_docs <= max_docs and non-null offsets and flags");
    return LSHBLOOM_EINVAL;
  }
  // host-side CSR validation (the device path trusts its input)
  for (int64_t d = 0; d < n_docs; ++d)
    if (h_offsets[d + 1] < h_offsets[d]) {
      set_err("pipeline_submit: offsets decrease at document %lld", (long long)d);
      return LSHBLOOM_EINVAL;
    }
  const int64_t n_tok = n_docs ? h_offsets[n_docs] - h_offsets[0] : 0;
  if ((uint64_t)n_tok > pl->prm.max_tokens || (n_tok > 0 && !h_tokens)) {
    set_err("pipeline_submit: %lld tokens exceed max_tokens %llu", (long long)n_tok,
            (unsigned long long)pl->prm.max_tokens);
    return LSHBLOOM_EINVAL;
  }
  const int64_t ticket = pl->next_ticket;
  Slot &S = pl->slot[ticket % kSlots];
  int rc = collect(pl, S);  // the slot's previous batch must be done before its buffers are reused
  if (rc) return rc;
  pl->next_ticket++;
  S.ticket = ticket;
  S.n_docs = n_docs;
  S.user_flags = h_flags;
  if (n_docs == 0) return ticket;

  // tokens: DMA straight from a pinned caller buffer, else stage them
  const uint32_t *src = h_tokens + h_offsets[0];
  if (!is_pinned(src)) {
    std::memcpy(S.h_tokens, src, (size_t)n_tok * 4);
    src = S.h_tokens;
  }
  hipError_t e = hipSuccess;
  if (!pl->tuned) {
    e = hipMemcpyAsync(S.d_tokens, src, (size_t)n_tok * 4, hipMemcpyHostToDevice, pl->mh_stream);
    if (e != hipSuccess) return fail_hip(nullptr, e, "pipeline: token copy");
    rc = autotune(pl, S, h_offsets, n_docs);
    if (rc) return rc;
    // the slot's device buffers are rewritten on the copy stream below
    if ((e = hipStreamSynchronize(pl->mh_stream)) != hipSuccess) return fail_hip(nullptr, e, "pipeline: tuning");
  }
  BucketView views[kMaxBuckets];
  build_buckets(pl->bk, h_offsets, n_docs, S.h_desc, views);
  const Buckets bk = pl->bk;
  // inputs on the copy stream, in submission order (the slot's previous batch
  // is complete: collect() waited for it)
  e = hipMemcpyAsync(S.d_tokens, src, (size_t)n_tok * 4, hipMemcpyHostToDevice, pl->copy_stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S.d_desc, S.h_desc, desc_words(n_docs) * 8, hipMemcpyHostToDevice, pl->copy_stream);
  if (e == hipSuccess) e = hipEventRecord(S.copied, pl->copy_stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(pl->mh_stream, S.copied, 0);
  if (e == hipSuccess && pl->has_mid) e = hipStreamWaitEvent(pl->mh_stream, pl->qi_mid, 0);
  if (e == hipSuccess) e = hipEventRecord(S.mh_t0, pl->mh_stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "pipeline: input copy");
  auto g1_body = [&]() -> hipError_t { return enqueue_minhash(pl, S, views, n_docs, bk); };
  e = pl->prm.use_graph ? run_graph(pl, pl->mh_stream, S.g1, g1_body) : g1_body();
  if (e != hipSuccess) return fail_hip(nullptr, e, "pipeline: MinHash stage");
  e = hipEventRecord(S.mh_t1, pl->mh_stream);
  if (e == hipSuccess) e = hipEventRecord(S.mh_done, pl->mh_stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "pipeline: event");

  {
    std::lock_guard<std::mutex> hk(h->mu);
    if (const int crc = lbh::check_ready(h)) return crc;
    e = hipStreamWaitEvent(pl->qi_stream, S.mh_done, 0);
    if (e == hipSuccess) e = lbh::begin_ordered(h, pl->qi_stream);
    if (e == hipSuccess) e = hipEventRecord(S.qi_t0, pl->qi_stream);
    if (e != hipSuccess) return fail_hip(h, e, "pipeline: ordering");
    int qrc = LSHBLOOM_OK;
    // partition passes (G2), the event the next MinHash waits for, then the
    // bins and resolve (G3); a query-insert that does not split runs whole in G2
    const bool split = lbh::qi_splits(h, n_docs);
    auto g2_body = [&]() -> hipError_t {
      qrc = lbh::qi_enqueue(h, S.d_sigs, n_docs, S.d_flags, pl->qi_stream, nullptr, 1);
      return qrc ? hipErrorUnknown : hipSuccess;
    };
    auto g3_body = [&]() -> hipError_t {
      qrc = lbh::qi_enqueue(h, S.d_sigs, n_docs, S.d_flags, pl->qi_stream, nullptr, 2);
      return qrc ? hipErrorUnknown : hipSuccess;
    };
    e = pl->prm.use_graph ? run_graph(pl, pl->qi_stream, S.g2, g2_body) : g2_body();
    if (e == hipSuccess && !qrc && split) e = hipEventRecord(pl->qi_mid, pl->qi_stream);
    if (e == hipSuccess && !qrc && split)
      e = pl->prm.use_graph ? run_graph(pl, pl->qi_stream, S.g3, g3_body) : g3_body();
    if (qrc) return qrc;
    if (e != hipSuccess) return fail_hip(h, e, "pipeline: query-insert stage");
    // a query-insert that did not split has no partition boundary to wait
    // for: the next MinHash then overlaps it whole
    pl->has_mid = split;
    e = hipEventRecord(S.qi_t1, pl->qi_stream);
    if (e == hipSuccess) e = lbh::finish_qi(h, pl->qi_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S.h_flags, S.d_flags, (size_t)n_docs, hipMemcpyDeviceToHost, pl->qi_stream);
    if (e == hipSuccess) e = lbh::end_ordered(h, pl->qi_stream);
    if (e == hipSuccess) e = hipEventRecord(S.done, pl->qi_stream);
    if (e != hipSuccess) return fail_hip(h, e, "pipeline: event");
    h->docs_inserted += (uint64_t)n_docs;
  }
  S.pending = true;
  return ticket;
}

int lshbloom_pipeline_wait(lshbloom_pipeline_t *pl, int64_t ticket) {
  if (!pl) {
    set_err("pipeline_wait: null pipeline");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(pl->mu);
  if (ticket < 0 || ticket >= pl->next_ticket) {
    set_err("pipeline_wait: unknown ticket %lld", (long long)ticket);
    return LSHBLOOM_EINVAL;
  }
  Slot &S = pl->slot[ticket % kSlots];
  if (S.ticket != ticket) return LSHBLOOM_OK;  // an older batch: collected when its slot was reused
  return collect(pl, S);
}

int lshbloom_pipeline_poll(lshbloom_pipeline_t *pl, int64_t ticket) {
  if (!pl) {
    set_err("pipeline_poll: null pipeline");
    return LSHBLOOM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(pl->mu);
  if (ticket < 0 || ticket >= pl->next_ticket) {
    set_err("pipeline_poll: unknown ticket %lld", (long long)ticket);
    return LSHBLOOM_EINVAL;
  }
  Slot &S = pl->slot[ticket % kSlots];
  if (S.ticket != ticket || !S.pending) return 1;
  const hipError_t q = hipEventQuery(S.done);
  if (q == hipErrorNotReady) return 0;
  if (q != hipSuccess) return fail_hip(nullptr, q, "pipeline_poll: event");
  const int rc = collect(pl, S);
  return rc ? rc : 1;
}

int lshbloom_pipeline_info(const lshbloom_pipeline_t *plc, lshbloom_pipeline_info_t *out) {
  if (!plc || !out) {
    set_err("pipeline_info: null argument");
    return LSHBLOOM_EINVAL;
  }
  lshbloom_pipeline *pl = const_cast<lshbloom_pipeline *>(plc);
  std::lock_guard<std::mutex> lk(pl->mu);
  std::memset(out, 0, sizeof *out);
  out->n_buckets = pl->bk.n;
  for (int q = 0; q < 3; ++q) out->bucket_edges[q] = pl->bk.edges[q];
  for (uint32_t q = 0; q < kMaxBuckets; ++q) out->waves_per_cu[q] = pl->bk.waves_per_cu[q];
  out->tuned = pl->tuned ? 1 : 0;
  out->tune_best_ms = pl->tune_best_ms;
  out->batches = (uint64_t)pl->next_ticket;
  out->graph_launches = pl->graph_launches;
  out->graph_updates = pl->graph_updates;
  out->graph_instantiations = pl->graph_instantiations;
  out->timed_batches = pl->timed_batches;
  out->minhash_ms_total = pl->minhash_ms_total;
  out->qi_ms_total = pl->qi_ms_total;
  return LSHBLOOM_OK;
}

}  // extern "C"
