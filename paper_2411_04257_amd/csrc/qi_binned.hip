// Binned in-order query-insert for large batches (Sections 2.1, 2.4, 4.1,
// 4.2, 4.4.2), atomic-free on the filters.
//
// A chunk's probes are partitioned by (band, bit range) so that one
// workgroup owns every probe of a bin of 2^s filter bits and can settle the
// in-chunk order of its bits in LDS:
//
//   keys      (k_bq_keys): band key of every (document, band), band-major;
//   pass 1    (k_bq_count1, scans, k_bq_scatter1): one block per (band,
//             tile of 1024 documents) computes the k positions of its
//             documents and writes 64-bit records
//                 [probe-0 flag : 1][document : 23][bit position : 40]
//             into buckets of consecutive bins, staging each 16,384-record
//             sub-tile in LDS so that every bucket's records leave as one
//             contiguous run; each XCD takes a contiguous range of tiles;
//   pass 2    (k_bq_part2): one block per bucket splits it into its bins
//             the same way (large buckets straight into per-bin slices,
//             smaller ones after counting their bins) and publishes each
//             bin's record range;
//   bins      (k_bq_bin): one wave per bin reads the bin's filter words
//             (the state before the chunk), builds in LDS a table of its
//             distinct bits with the least document probing each and a
//             "probed by two documents or more" flag, ORs every probe into
//             the words and writes them back with plain stores (it is their
//             only writer; bins its LDS tables cannot hold are left to
//             bin_global, in k_bq_bin_overflow).  A bit
//             was set before document i iff it was set before the chunk or
//             its least document is < i.  The bin answers that at once for
//             the probe-0 records (res0), and publishes the bits a later
//             lookup can need: those set before the chunk and those probed
//             by more than one document.  A bit probed by one document only
//             was never set before that document, and no other document
//             looks it up;
//   resolve   (k_bq_resolve): per document and band, probe 0's answer
//             decides most pairs (a miss ends the band); otherwise probes
//             1..k-1 are looked up in the published tables with early exit.
//
// Every step is exact, so flags and final filter words equal the sequential
// definition for every chunking.  Bins with more records than the LDS
// tables hold take a slower path with their table in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "launch_order.h"
#include "qi_binned.h"

namespace lb {

namespace {

constexpr uint32_t kThreads = 256;
constexpr uint32_t kInit = 0xFFFFFFFFu;       // bit set before the chunk
constexpr uint32_t kNoFs = 0xFFFFFFFEu;       // no document recorded yet
constexpr uint64_t kMask40 = (1ull << 40) - 1;
constexpr uint32_t kDocMask = (1u << 23) - 1;
constexpr uint64_t kProbe0 = 1ull << 63;
constexpr uint32_t kMaxF1 = 1024;
constexpr uint32_t kKeysLds = 8192;           // signature words staged per keys block

__host__ __device__ inline uint32_t keys_tile_docs(uint32_t br) { return br >= kKeysLds ? 1u : kKeysLds / br; }
constexpr uint32_t kMaxF2 = 1024;

// Slot of a 32-bit key in a table of `cap` slots (multiply-high range reduction).
__device__ __forceinline__ uint32_t slot_of(uint32_t key, uint32_t cap) {
  const uint32_t h = key * 0x9E3779B1u;
  const uint32_t h2 = (h ^ (h >> 15)) * 0x85EBCA77u;
  return (uint32_t)(((uint64_t)(h2 ^ (h2 >> 13)) * cap) >> 32);
}

// Workgroup barrier for LDS only: waits for this wave's LDS operations, not
// for its global stores, which stay in flight across the barrier (no kernel
// here reads back global memory written by another wave of its workgroup
// except bin_global, which uses device-scope atomics and fences).
__device__ __forceinline__ void sync_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Exclusive scan of in[0..n) into out[0..n) (may alias) by a block of NT
// threads: each thread sums a run of consecutive entries, the
// runs are scanned within each wave by shuffles and across the waves through
// part[] (NT / 64 words of LDS).  Returns the total.  Every thread of the block must call
// it; it ends with a barrier.
template <uint32_t NT = kThreads>
__device__ uint32_t block_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *part) {
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t a = min(n, threadIdx.x * per), b = min(n, a + per);
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t s = 0;
  for (uint32_t q = a; q < b; ++q) s += in[q];
  uint32_t x = s;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) part[wave] = x;
  sync_lds();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < NT / 64; ++w) {
    const uint32_t t = part[w];
    if (w < wave) base += t;
    total += t;
  }
  uint32_t run = base + x - s;
  for (uint32_t q = a; q < b; ++q) {
    const uint32_t v = in[q];
    out[q] = run;
    run += v;
  }
  sync_lds();
  return total;
}

// ------------------------------------------------------------------ keys ----
// Band keys of a tile of documents: the tile's first b*r signature values per
// document are staged in LDS (coalesced reads, rows padded by one word), then
// every (band, document) key is written band-major.
__global__ __launch_bounds__(256) void k_bq_keys(BinnedLaunch A) {
  extern __shared__ uint32_t srow[];
  const uint32_t br = A.bands * A.rows, stride = br + 1;
  const uint32_t td = keys_tile_docs(br);
  const int64_t d0 = (int64_t)blockIdx.x * td;
  const uint32_t nd = (uint32_t)min((int64_t)td, A.n - d0);
  const uint32_t nq = nd * br;
  // Element q = d * br + c of the tile, walked in steps of kThreads: (d, c)
  // advance by (kThreads / br, kThreads % br) with one carry, instead of a
  // division per element.
  const uint32_t dstep = kThreads / br, cstep = kThreads - dstep * br;
  uint32_t d = threadIdx.x / br, c = threadIdx.x - d * br;
  for (uint32_t q0 = 0; q0 < nq; q0 += 8 * kThreads) {
    uint32_t v[8], dd[8], cc[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      const uint32_t q = q0 + u * kThreads + threadIdx.x;
      dd[u] = d;
      cc[u] = c;
      v[u] = q < nq ? A.sigs[(d0 + d) * (int64_t)A.num_perm + c] : 0u;
      d += dstep;
      c += cstep;
      if (c >= br) {
        c -= br;
        ++d;
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      const uint32_t q = q0 + u * kThreads + threadIdx.x;
      if (q < nq) srow[dd[u] * stride + cc[u]] = v[u];
    }
  }
  __syncthreads();
  // Key p = j * nd + dk: (j, dk) advance the same way.
  const uint32_t jstep = kThreads / nd, kstep = kThreads - jstep * nd;
  uint32_t j = threadIdx.x / nd, dk = threadIdx.x - j * nd;
  for (uint32_t p = threadIdx.x; p < nd * A.bands; p += kThreads) {
    A.keys[(int64_t)j * A.n + d0 + dk] = band_key(&srow[dk * stride + j * A.rows], A.rows, A.salt_m);
    j += jstep;
    dk += kstep;
    if (dk >= nd) {
      dk -= nd;
      ++j;
    }
  }
}

// Zero the probe-0 answers of a chunk (their bytes as 32-bit words).
__global__ __launch_bounds__(256) void k_bq_zero_res0(BinnedLaunch A, uint64_t words) {
  if (blockIdx.x == 0 && threadIdx.x == 0) A.ovf[0] = 0;  // no bin left to the general path yet
  uint32_t *w = reinterpret_cast<uint32_t *>(A.res0);
  for (uint64_t q = (uint64_t)blockIdx.x * kThreads + threadIdx.x; q < words; q += (uint64_t)gridDim.x * kThreads)
    w[q] = 0;
}

// Band keys given by the caller, [n][bands] -> band-major.
__global__ __launch_bounds__(256) void k_bq_keys_in(BinnedLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t d = t / A.bands;
  const uint32_t j = (uint32_t)(t - d * A.bands);
  A.keys[(int64_t)j * A.n + d] = A.keys_in[t];
}

// ---------------------------------------------------------------- pass 1 ----
// Block (tile of 1024 documents, band j).  k_bq_count1: per-bucket record
// counts of the block.  k_bq_scatter1 (1024 threads, one block per compute
// unit): the records, staged in LDS by bucket in sub-tiles of 16,384 so that
// each bucket's share leaves as one run, written at counts-derived offsets.
#ifndef LB_PER1
#define LB_PER1 16
#endif
constexpr uint32_t kT1 = kTileDocs;
constexpr uint32_t kPer1 = LB_PER1;
constexpr uint32_t kSub1 = kT1 * kPer1;

// Pass-1 blocks, renumbered so that each of the 8 XCDs works through a
// contiguous range of (band, tile) pairs: neighbouring tiles' writes to a
// bucket, whose ends share lines, then meet in one L2.
__device__ __forceinline__ void pass1_block(uint32_t n_tiles, uint32_t &tile, uint32_t &band) {
  const uint32_t P = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  tile = P % n_tiles;
  band = P / n_tiles;
}

__global__ __launch_bounds__(256) void k_bq_count1(BinnedLaunch A) {
  extern __shared__ uint32_t hist[];  // [F1]
  const BinnedGeometry &G = A.G;
  const uint32_t F1 = G.buckets_per_band;
  uint32_t tile, j;
  pass1_block(G.n_tiles, tile, j);
  const int64_t d0 = (int64_t)tile * kTileDocs;
  const uint32_t nd = (uint32_t)min((int64_t)kTileDocs, A.n - d0);
  for (uint32_t f = threadIdx.x; f < F1; f += kThreads) hist[f] = 0;
  sync_lds();
  // whole documents per thread: the pair of hashes stays in registers
  const uint64_t *K = A.keys + (int64_t)j * A.n + d0;
  for (uint32_t d = threadIdx.x; d < nd; d += kThreads) {
    const uint64_t key = K[d];
    const uint64_t h1 = fmix64(key ^ A.salt1), h2 = fmix64(key ^ A.salt2) | 1ull;
    for (uint32_t l = 0; l < A.k; ++l) {
      const uint64_t g = umulhi64(h1 + (uint64_t)l * h2, A.m_bits);
      atomicAdd(&hist[(uint32_t)(g >> G.bucket_bits)], 1u);
    }
  }
  sync_lds();
  const uint64_t row = ((uint64_t)j * F1) * G.n_tiles + tile;  // + f * n_tiles
  for (uint32_t f = threadIdx.x; f < F1; f += kThreads) A.counts[row + (uint64_t)f * G.n_tiles] = hist[f];
}

__global__ __launch_bounds__(kT1) void k_bq_scatter1(BinnedLaunch A) {
  extern __shared__ __align__(16) uint8_t smem[];
  const BinnedGeometry &G = A.G;
  const uint32_t F1 = G.buckets_per_band;
  const uint32_t F1r = (F1 + 3) & ~3u;
  uint64_t *stage = (uint64_t *)smem;              // [kSub1]
  uint32_t *hist = (uint32_t *)(stage + kSub1);    // [F1]
  uint32_t *lstart = hist + F1r;                   // [F1]
  uint32_t *cur = lstart + F1r;                    // [F1]
  uint32_t *part = cur + F1r;                      // [16]
  uint32_t *dl = part + 16;                        // [F1] where a bucket's run goes, less its stage start
  uint32_t tile, j;
  pass1_block(G.n_tiles, tile, j);
  const int64_t d0 = (int64_t)tile * kTileDocs;
  const uint32_t nd = (uint32_t)min((int64_t)kTileDocs, A.n - d0);
  const uint64_t row = ((uint64_t)j * F1) * G.n_tiles + tile;  // + f * n_tiles
  for (uint32_t f = threadIdx.x; f < F1; f += kT1) {
    hist[f] = 0;
    cur[f] = A.bstart[(uint64_t)j * F1 + f] + A.counts[row + (uint64_t)f * G.n_tiles];
  }
  sync_lds();
  const uint32_t total = kTileDocs * A.k;
  // slot q = l * kTileDocs + d with kT1 == kTileDocs: thread t always holds
  // document t, whose pair of hashes stays in registers
  static_assert(kT1 == kTileDocs, "one document per thread");
  const uint32_t d = threadIdx.x;
  uint64_t dh1 = 0, dh2 = 0;
  if (d < nd) {
    const uint64_t key = A.keys[(int64_t)j * A.n + d0 + d];
    dh1 = fmix64(key ^ A.salt1);
    dh2 = fmix64(key ^ A.salt2) | 1ull;
  }
  for (uint32_t q0 = 0; q0 < total; q0 += kSub1) {
    uint64_t rec[kPer1];
    uint32_t rk[kPer1];
#pragma unroll
    for (uint32_t u = 0; u < kPer1; ++u) {
      const uint32_t q = q0 + u * kT1 + threadIdx.x;
      const uint32_t l = q >> kTileLog;
      rec[u] = ~0ull;
      if (q < total && d < nd) {
        const uint64_t g = umulhi64(dh1 + (uint64_t)l * dh2, A.m_bits);
        rk[u] = atomicAdd(&hist[(uint32_t)(g >> G.bucket_bits)], 1u);
        rec[u] = (l == 0 ? kProbe0 : 0ull) | ((uint64_t)(d0 + d) << 40) | g;
      }
    }
    sync_lds();
    const uint32_t cnt = block_scan<kT1>(hist, lstart, F1, part);
#pragma unroll
    for (uint32_t u = 0; u < kPer1; ++u)
      if (rec[u] != ~0ull) stage[lstart[(uint32_t)((rec[u] & kMask40) >> G.bucket_bits)] + rk[u]] = rec[u];
    // stage slot p of bucket f goes to p + dl[f] (one LDS read per record);
    // the bucket's write position moves past this sub-tile's share
    for (uint32_t f = threadIdx.x; f < F1; f += kT1) {
      dl[f] = cur[f] - lstart[f];
      cur[f] += hist[f];
      hist[f] = 0;
    }
    sync_lds();
    for (uint32_t p = threadIdx.x; p < cnt; p += kT1) {
      const uint64_t r = stage[p];
      A.rec1[p + dl[(uint32_t)((r & kMask40) >> G.bucket_bits)]] = r;
    }
    sync_lds();
  }
}

// Exclusive scan of every (band, bucket) row of per-block counts; the row
// total goes to bstart.
__global__ __launch_bounds__(256) void k_bq_scan_tiles(BinnedLaunch A) {
  __shared__ uint32_t part[kThreads];
  uint32_t *row = A.counts + (uint64_t)blockIdx.x * A.G.n_tiles;
  const uint32_t t = block_scan(row, row, A.G.n_tiles, part);
  if (threadIdx.x == 0) A.bstart[blockIdx.x] = t;
}

// Exclusive scan of the bucket totals (one block): bucket starts, and the
// record count at the end.
__global__ __launch_bounds__(256) void k_bq_scan_buckets(BinnedLaunch A) {
  __shared__ uint32_t part[kThreads];
  const uint32_t nb = A.bands * A.G.buckets_per_band;
  const uint32_t t = block_scan(A.bstart, A.bstart, nb, part);
  if (threadIdx.x == 0) {
    A.bstart[nb] = t;
    if (t != A.n_records) atomicOr(A.status, 8u);
  }
}

// ---------------------------------------------------------------- pass 2 ----
// One 1024-thread block per bucket (one block fills a compute unit's LDS)
// splits the bucket into bins through LDS-staged sub-tiles of PER x 1024
// records (19 where LDS holds them beside the bins' arrays, up to 507 bins
// per bucket, else 16), so that each bin's share of a sub-tile leaves as one
// contiguous run, and publishes every bin's record range [start, end).
//
// Bucket q owns the binned-record region that starts at bstart[q] +
// q (slack + 1) F2 and holds its T records plus (slack + 1) F2 spare slots.
// With slack > 0 each bin first gets a slice of ceil(T / bins) + slack slots
// (slack is about five standard deviations of a bin's record count), so the
// bucket is read once; a bin that outgrows its slice (a skewed bucket) makes
// the block lay the bucket out again, compactly, from its exact bin counts.
// With slack = 0 (smaller buckets, where a second read costs less than the
// slices' partial-line writes, or no spare slots in the workspace) the block
// counts first, then splits compactly.
#ifndef LB_T2
#define LB_T2 1024
#endif
#ifndef LB_PER2
#define LB_PER2 16
#endif
#ifndef LB_PER2_BIG
#define LB_PER2_BIG 19
#endif
constexpr uint32_t kT2 = LB_T2;
constexpr uint32_t kPer2 = LB_PER2;
constexpr uint32_t kPer2Big = LB_PER2_BIG;
// LDS of a pass-2 block: the stage, four per-bin arrays, 17 more words
constexpr size_t part2_lds(uint32_t per, uint32_t bins) { return (size_t)per * kT2 * 8 + 4 * (size_t)bins * 4 + 17 * 4; }

template <uint32_t PER>
__global__ __launch_bounds__(kT2) void k_bq_part2(BinnedLaunch A) {
  constexpr uint32_t kSub2 = kT2 * PER;
  extern __shared__ __align__(16) uint8_t smem[];
  const BinnedGeometry &G = A.G;
  const uint32_t F2 = G.bins_per_bucket;
  uint64_t *stage = (uint64_t *)smem;            // [kSub2]
  uint32_t *cur = (uint32_t *)(stage + kSub2);   // [F2] next write position of each bin
  uint32_t *h = cur + F2;                        // [F2]
  uint32_t *lstart = h + F2;                     // [F2]
  uint32_t *part = lstart + F2;                  // [16]
  uint32_t *ovf = part + 16;                     // [1] a bin outgrew its slice
  uint32_t *dl = ovf + 1;                        // [F2] where a bin's run goes, less its stage start

  const uint32_t q = blockIdx.x;
  const uint32_t j = q / G.buckets_per_band, f = q - j * G.buckets_per_band;
  const uint32_t s0 = A.bstart[q], s1 = A.bstart[q + 1];
  const uint64_t first_bin = (uint64_t)f * F2;  // within the band
  const uint32_t nbins = (uint32_t)min((uint64_t)F2, G.bins_per_band - first_bin);
  const uint32_t slack = A.slice_slack;
  const uint32_t base2 = s0 + (slack ? q * (slack + 1) * F2 : 0u);
  const uint32_t capb = slack ? (s1 - s0 + nbins - 1) / nbins + slack : 0u;  // slice of each bin
  const uint32_t bmask = F2 - 1;
  uint32_t *start = A.off2 + (uint64_t)j * G.bins_per_band + first_bin;
  uint32_t *end = A.end2 + (uint64_t)j * G.bins_per_band + first_bin;

  // Split the bucket: every record goes to cur[bin] + its rank among the
  // bin's records so far; with `limit`, a position at or past the bin's
  // slice end is not written and raises *ovf.  rec[] holds the first
  // sub-tile (loaded here unless `loaded`); the next sub-tile's records are
  // loaded as soon as the current ones sit in LDS, so that their latency
  // overlaps the write-out and the barriers.
  uint64_t rec[PER];
  auto split = [&](bool limit, bool loaded) {
    if (!loaded) {
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u) {
        const uint32_t r = s0 + u * kT2 + threadIdx.x;
        rec[u] = r < s1 ? A.rec1[r] : ~0ull;
      }
    }
    for (uint32_t q0 = s0; q0 < s1; q0 += kSub2) {
      uint32_t rk[PER];
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u)
        if (rec[u] != ~0ull) rk[u] = atomicAdd(&h[((uint32_t)rec[u] >> G.bin_bits) & bmask], 1u);
      sync_lds();
      const uint32_t cnt = block_scan<kT2>(h, lstart, F2, part);
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u)
        if (rec[u] != ~0ull) stage[lstart[((uint32_t)rec[u] >> G.bin_bits) & bmask] + rk[u]] = rec[u];
      // stage slot p of bin b goes to p + dl[b]; the bin's write position
      // moves past this sub-tile's share
      for (uint32_t b = threadIdx.x; b < F2; b += kT2) {
        dl[b] = cur[b] - lstart[b];
        cur[b] += h[b];
        h[b] = 0;
      }
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u) {
        const uint32_t r = q0 + kSub2 + u * kT2 + threadIdx.x;
        rec[u] = r < s1 ? A.rec1[r] : ~0ull;
      }
      sync_lds();
      for (uint32_t p = threadIdx.x; p < cnt; p += kT2) {
        const uint64_t r = stage[p];
        const uint32_t b = ((uint32_t)r >> G.bin_bits) & bmask;
        const uint32_t w = p + dl[b];
        if (!limit || w < base2 + (b + 1) * capb)
          A.rec2[w] = r;
        else
          *ovf = 1u;
      }
      sync_lds();
    }
  };

  for (uint32_t b = threadIdx.x; b < F2; b += kT2) {
    cur[b] = slack ? base2 + b * capb : 0u;
    h[b] = 0;
  }
  if (threadIdx.x == 0) *ovf = 0u;
  sync_lds();
  bool loaded = false;
  if (slack) {
    split(true, false);
    if (*ovf == 0u) {
      for (uint32_t b = threadIdx.x; b < nbins; b += kT2) {
        start[b] = base2 + b * capb;
        end[b] = cur[b];
      }
      return;
    }
    // a bin outgrew its slice: its exact count is known; lay the bucket out
    // compactly in its region instead
    for (uint32_t b = threadIdx.x; b < F2; b += kT2) cur[b] -= base2 + b * capb;
  } else {
    // count the bins first.  The first sub-tile's records stay in registers
    // for the split, so that a bucket of at most kSub2 records is read once;
    // the counting pass needs only a record's bin within its bucket, bits
    // [bin_bits, bucket_bits) of its bit, all in the record's low 32 bits
    // (bucket_bits <= 32 is checked at launch), so the later sub-tiles load
    // only those
    const uint32_t *lo1 = reinterpret_cast<const uint32_t *>(A.rec1);
    uint32_t bi[PER];
#pragma unroll
    for (uint32_t u = 0; u < PER; ++u) {
      const uint32_t r = s0 + u * kT2 + threadIdx.x;
      rec[u] = r < s1 ? A.rec1[r] : ~0ull;
      bi[u] = r < s1 ? ((uint32_t)rec[u] >> G.bin_bits) & bmask : ~0u;
    }
    for (uint32_t q0 = s0; q0 < s1; q0 += kSub2) {
      uint32_t g[PER];
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u) {
        const uint32_t r = q0 + kSub2 + u * kT2 + threadIdx.x;
        g[u] = r < s1 ? lo1[2ull * r] : 0u;
      }
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u)
        if (bi[u] != ~0u) atomicAdd(&cur[bi[u]], 1u);
#pragma unroll
      for (uint32_t u = 0; u < PER; ++u)
        bi[u] = q0 + kSub2 + u * kT2 + threadIdx.x < s1 ? (g[u] >> G.bin_bits) & bmask : ~0u;
    }
    loaded = true;
  }
  sync_lds();
  block_scan<kT2>(cur, cur, F2, part);
  for (uint32_t b = threadIdx.x; b < F2; b += kT2) {
    cur[b] += base2;
    if (b < nbins) start[b] = cur[b];
  }
  sync_lds();
  split(false, loaded);
  for (uint32_t b = threadIdx.x; b < nbins; b += kT2) end[b] = cur[b];
}

// ------------------------------------------------------------------- bins ----
// One wave per bin (64-thread workgroups), so that a bin's steps need no
// workgroup barrier and several bins per SIMD overlap their memory latency.
// LDS holds, per wave, the bin's distinct bits (key = local bit + 1, bit 31
// marking "probed by two documents or more") with 0 for a bit set before the
// chunk or 1 + the least document probing it, and either the bin's filter
// words (direct mode) or a table of the words it touches with their OR masks;
// that space then holds the published table, whose entries carry kInit or
// the least document.
#ifndef LB_WCAP
#define LB_WCAP 320
#endif
constexpr uint32_t kWCap = LB_WCAP;           // records per bin on the sparse wave path
constexpr uint32_t kWPer = kWCap / 64;        // records per lane
#ifndef LB_BIN_TAB
#define LB_BIN_TAB (2 * kWCap)
#endif
constexpr uint32_t kWTab = LB_BIN_TAB;        // bit / word table slots (at most 2 per record)
static_assert(kWTab >= kWCap && kWTab % 64 == 0, "a table slot for every record of a wave-path bin");
constexpr uint32_t kWRegion = 512;            // direct mode: the bin's words (bin_bits <= 15)
constexpr uint32_t kMulti = 0x80000000u;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A bin with more records than the wave's LDS tables hold: its table (every
// distinct bit, 2 slots per record) is built in the bin's own slots of the
// table area with device atomics; filter bits are set after every record has
// read the state before the chunk.
__device__ void bin_global(const BinnedLaunch &A, uint32_t j, uint64_t bin, uint32_t r0, uint32_t r1, uint64_t b0,
                           uint64_t *F) {
  const uint32_t lane = threadIdx.x;
  const uint32_t nr = r1 - r0, cap = 2 * nr;
  unsigned long long *T = (unsigned long long *)(A.rec1 + 2ull * r0);
  for (uint32_t q = lane; q < cap; q += 64) T[q] = (unsigned long long)kNoFs;
  __threadfence();
  wave_sync();
  for (uint32_t r = r0 + lane; r < r1; r += 64) {
    const uint64_t rec = A.rec2[r];
    const uint32_t i = (uint32_t)(rec >> 40) & kDocMask;
    const uint32_t lb = (uint32_t)((rec & kMask40) - b0);
    const bool init = (F[lb >> 6] >> (lb & 63)) & 1ull;
    uint32_t h = slot_of(lb, cap);
    bool placed = false;
    for (uint32_t tries = 0; tries < cap && !placed;) {
      unsigned long long cur = __hip_atomic_load(&T[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (;;) {
        const uint32_t key = (uint32_t)(cur >> 32);
        if (key == lb + 1) {
          placed = true;
          break;
        }
        if (key != 0) break;
        const unsigned long long want = ((unsigned long long)(lb + 1) << 32) | kNoFs;
        const unsigned long long old = atomicCAS(&T[h], cur, want);
        if (old == cur) {
          placed = true;
          break;
        }
        cur = old;
      }
      if (!placed) {
        h = (h + 1 == cap) ? 0 : h + 1;
        ++tries;
      }
    }
    if (!placed) {
      atomicOr(A.status, 4u);
      continue;
    }
    if (init)
      atomicOr(&T[h], (unsigned long long)kInit);
    else
      atomicMin(&T[h], ((unsigned long long)(lb + 1) << 32) | i);
  }
  __threadfence();
  wave_sync();
  for (uint32_t r = r0 + lane; r < r1; r += 64) {
    const uint64_t rec = A.rec2[r];
    const uint32_t lb = (uint32_t)((rec & kMask40) - b0);
    atomicOr((unsigned long long *)&F[lb >> 6], (unsigned long long)(1ull << (lb & 63)));
    if (rec & kProbe0) {
      const uint32_t i = (uint32_t)(rec >> 40) & kDocMask;
      uint32_t h = slot_of(lb, cap);
      uint32_t v = kNoFs;
      for (uint32_t tries = 0; tries < cap; ++tries) {
        const unsigned long long e = __hip_atomic_load(&T[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(e >> 32) == lb + 1) {
          v = (uint32_t)e;
          break;
        }
        h = (h + 1 == cap) ? 0 : h + 1;
      }
      if (v == kInit || v < i) A.res0[(int64_t)j * A.n + i] = 1;  // res0 starts zeroed
    }
  }
  if (lane == 0) A.dir[bin] = ((uint64_t)r0 << 32) | cap;
  __threadfence();
  wave_sync();
}

// A bin the wave paths cannot take (more records, shared bits or published
// bits than their LDS tables hold) is listed for k_bq_bin_overflow, which
// runs it through bin_global once the bin kernel has ended.  Bins own
// disjoint filter bits, so the order does not matter; nothing of the bin
// has been written but probe-0 answers, which bin_global gives again.  Kept
// out of the bin kernels' loops, the general path leaves their loads and
// waits as the common path needs them.
__device__ __forceinline__ void defer_bin(const BinnedLaunch &A, uint64_t bin) {
  if (threadIdx.x == 0) A.ovf[1 + atomicAdd(&A.ovf[0], 1u)] = (uint32_t)bin;
}

__global__ __launch_bounds__(64) void k_bq_bin_overflow(BinnedLaunch A) {
  const BinnedGeometry &G = A.G;
  if (blockIdx.x == 0 && threadIdx.x == 0 && A.ovf[0]) atomicAdd(A.ovf_total, (unsigned long long)A.ovf[0]);
  for (uint32_t t = blockIdx.x; t < A.ovf[0]; t += gridDim.x) {
    const uint64_t bin = A.ovf[1 + t];
    const uint32_t j = (uint32_t)(bin / G.bins_per_band);
    const uint64_t b0 = (bin - (uint64_t)j * G.bins_per_band) << G.bin_bits;
    bin_global(A, j, bin, A.off2[bin], A.end2[bin], b0, A.filters + (uint64_t)j * A.words_per_band + (b0 >> 6));
  }
}

// Sparse bins (bin_bits > 15: the bin's words do not fit in LDS): one wave
// per bin (64-thread workgroups), so that a bin's steps need no workgroup
// barrier and several bins per SIMD overlap their memory latency.  LDS holds,
// per wave, the bin's distinct bits (key = local bit + 1, bit 31 marking
// "probed by two documents or more") with 0 for a bit set before the chunk or
// 1 + the least document probing it, and a table of the words the records
// touch with their OR masks; that space then holds the published table, whose
// entries carry kInit or the least document.  Each record reads its own word
// from HBM (the state before the chunk).
__global__ __launch_bounds__(64) void k_bq_bin_sparse(BinnedLaunch A) {
  // tmin[slot]: 0 if the bit was set before the chunk, else 1 + the least
  // document probing it (so one atomicMin serves both), kNoFs before any.
  __shared__ __align__(16) uint32_t tkey[kWTab];
  __shared__ __align__(16) uint32_t tmin[kWTab];
  __shared__ __align__(16) unsigned long long wv[kWTab];
  __shared__ uint32_t wk[kWTab];  // word keys

  const uint32_t lane = threadIdx.x;
  const BinnedGeometry &G = A.G;
  const uint64_t n_bins = (uint64_t)A.bands * G.bins_per_band;
  // A wave's bins are pipelined as in the dense kernel: the next bin's
  // records and the record range of the bin after it are loaded with the
  // bin's own words and taken in (settle) after its bit table is built,
  // before any of its stores; every lane loads, the selects come at settle.
  // A bin's records fill rows of 64; in its last row the lanes past the end
  // repeat the bin's first record (a repeated record changes nothing: it
  // finds its bit's slot taken by its twin, ORs the same bit and answers
  // the same probe 0), so that every lane of a row holds a record; rows
  // past the end, and every row of a bin above kWCap records, hold ~0.
  auto load_range = [&](uint64_t b) -> uint32_t {
    const uint32_t *p = lane == 0 ? A.off2 : A.end2;
    return p[b < n_bins ? b : 0];
  };
  auto range_of = [&](uint32_t v, uint64_t b, uint32_t &q0, uint32_t &q1) {
    q0 = b < n_bins ? (uint32_t)__builtin_amdgcn_readlane((int)v, 0) : 0u;
    q1 = b < n_bins ? (uint32_t)__builtin_amdgcn_readlane((int)v, 1) : 0u;
  };
  auto load_raw = [&](uint32_t q0, uint32_t q1, uint64_t *raw) {
    const uint32_t last = q1 > 0 ? q1 - 1 : 0;
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) {
      const uint32_t r = q0 + u * 64 + lane;
      raw[u] = A.rec2[min(r < q1 ? r : q0, last)];
    }
  };
  auto mask_recs = [&](uint32_t q0, uint32_t q1, const uint64_t *raw, uint64_t *out) {
    const uint32_t nrr = q1 - q0;
    const bool small = nrr <= kWCap;
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) out[u] = (small && u * 64 < nrr) ? raw[u] : ~0ull;
  };
  uint32_t r0, r1, n0, n1;  // the current and the next bin's record ranges
  uint64_t rec[kWPer];
  {
    const uint64_t b1 = (uint64_t)blockIdx.x + gridDim.x;
    range_of(load_range(blockIdx.x), blockIdx.x, r0, r1);
    uint64_t raw[kWPer];
    load_raw(r0, r1, raw);
    const uint32_t v1 = load_range(b1);
    mask_recs(r0, r1, raw, rec);
    range_of(v1, b1, n0, n1);
  }
  for (uint64_t bin = blockIdx.x; bin < n_bins; bin += gridDim.x) {
    const uint64_t b2 = bin + 2ull * gridDim.x;
    uint32_t m0, m1, mv;  // the range of the bin after next
    uint64_t nraw[kWPer], nrec[kWPer];
    auto prefetch = [&]() {
      load_raw(n0, n1, nraw);
      mv = load_range(b2);
    };
    auto settle = [&]() {
      mask_recs(n0, n1, nraw, nrec);
      range_of(mv, b2, m0, m1);
    };
    auto advance = [&]() {
      r0 = n0;
      r1 = n1;
      n0 = m0;
      n1 = m1;
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u) rec[u] = nrec[u];
    };
    const uint32_t nr = r1 - r0;
    if (nr == 0 || nr > kWCap) {
      if (nr > kWCap) defer_bin(A, bin);
      prefetch();
      settle();
      advance();
      continue;
    }
    const uint32_t nu = (nr + 63) >> 6;  // rows of records (uniform)
    const uint32_t j = (uint32_t)(bin / G.bins_per_band);
    const uint64_t lbin = bin - (uint64_t)j * G.bins_per_band;
    const uint64_t b0 = lbin << G.bin_bits;  // first bit of the bin (a multiple of 64)
    uint64_t *F = A.filters + (uint64_t)j * A.words_per_band + (b0 >> 6);
    const uint32_t cap = min(2 * nr, kWTab);
#pragma unroll
    for (uint32_t t = 0; t < kWTab / 64; ++t) {
      const uint32_t q = t * 64 + lane;
      if (q < cap) {
        tkey[q] = 0;
        tmin[q] = kNoFs;
        wk[q] = 0;
        wv[q] = 0;
      }
    }
    // this bin's loads first (each record's word; rows past the end re-read
    // the first record's), then the next bin's records
    uint64_t pre[kWPer];
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) pre[u] = F[(uint32_t)(((u < nu ? rec[u] : rec[0]) & kMask40) - b0) >> 6];
    prefetch();
    wave_sync();
    // phase A: insert every record's bit into the bit table.  A lane's
    // records probe in rounds (one compare-and-swap per record per round,
    // issued together), so their LDS round trips overlap.  The record whose
    // swap fills a slot owns the bit.
    uint32_t slot[kWPer], key1[kWPer];
    uint32_t init = 0, own = 0;  // init: the bit was set before the chunk
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) {
      slot[u] = 0;
      key1[u] = 0;
      if (u < nu) {
        const uint32_t lb = (uint32_t)((rec[u] & kMask40) - b0);
        init |= (uint32_t)(pre[u] >> (lb & 63) & 1ull) << u;
        key1[u] = lb + 1;
        slot[u] = slot_of(lb, cap);
      }
    }
    uint32_t pend = 0;
    {
      uint32_t old[kWPer];
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u)
        if (u < nu) old[u] = atomicCAS(&tkey[slot[u]], 0u, key1[u]);
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u) {
        if (u >= nu) continue;
        if (old[u] == 0u) own |= 1u << u;
        if (old[u] != 0u && old[u] != key1[u]) {
          pend |= 1u << u;
          slot[u] = (slot[u] + 1 == cap) ? 0 : slot[u] + 1;
        }
      }
    }
    for (uint32_t round = 1; pend && round < cap; ++round) {
      uint32_t old[kWPer];
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u)
        if (pend >> u & 1u) old[u] = atomicCAS(&tkey[slot[u]], 0u, key1[u]);
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u) {
        if (!(pend >> u & 1u)) continue;
        if (old[u] == 0u) own |= 1u << u;
        if (old[u] == 0u || old[u] == key1[u])
          pend &= ~(1u << u);
        else
          slot[u] = (slot[u] + 1 == cap) ? 0 : slot[u] + 1;
      }
    }
    if (pend) atomicOr(A.status, 4u);  // cannot happen: cap >= distinct bits
    wave_sync();
    settle();
    // least document (+1) probing each clear bit, 0 for bits set before the
    // chunk (every record of a bit sees the same state)
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u)
      if (u < nu) atomicMin(&tmin[slot[u]], (init >> u & 1u) ? 0u : ((uint32_t)(rec[u] >> 40) & kDocMask) + 1);
    wave_sync();
    // phase B: probe 0 of every (document, band) is answered here (its bit
    // was set before document i iff tmin <= i); a clear bit whose least
    // document is not the reader's was probed by two documents or more; the
    // newly set bits are ORed into the words
    uint32_t owner = 0, wslot[kWPer], wpend = 0;
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) {
      if (u >= nu) continue;
      const uint32_t i = (uint32_t)(rec[u] >> 40) & kDocMask;
      const uint32_t v = tmin[slot[u]];
      // res0 starts zeroed: only the set-before answers are written
      if ((rec[u] & kProbe0) && v <= i) A.res0[(int64_t)j * A.n + i] = 1;
      const bool clr = !(init >> u & 1u);
      if (clr && v != i + 1) atomicOr(&tkey[slot[u]], kMulti);  // rare: skipped by most rows
      if (clr) {
        wslot[u] = slot_of((key1[u] - 1) >> 6, cap);
        wpend |= 1u << u;
      }
    }
    // the word table, in rounds like the bit table; the record that claims a
    // word's slot writes the word back
    for (uint32_t round = 0; wpend && round < cap; ++round) {
      uint32_t old[kWPer];
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u)
        if (wpend >> u & 1u) old[u] = atomicCAS(&wk[wslot[u]], 0u, ((key1[u] - 1) >> 6) + 1);
#pragma unroll
      for (uint32_t u = 0; u < kWPer; ++u) {
        if (!(wpend >> u & 1u)) continue;
        const uint32_t want = ((key1[u] - 1) >> 6) + 1;
        if (old[u] == 0u) owner |= 1u << u;
        if (old[u] == 0u || old[u] == want)
          wpend &= ~(1u << u);
        else
          wslot[u] = (wslot[u] + 1 == cap) ? 0 : wslot[u] + 1;
      }
    }
    if (wpend) atomicOr(A.status, 4u);
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u)
      if (u < nu && !(init >> u & 1u)) atomicOr(&wv[wslot[u]], 1ull << ((key1[u] - 1) & 63));
    wave_sync();
    // changed words (this wave is their only writer in the chunk)
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u)
      if (owner >> u & 1u) F[(key1[u] - 1) >> 6] = pre[u] | wv[wslot[u]];
    // publish the bits a lookup can need (set before the chunk, or probed by
    // two documents or more), each by the record owning its slot, as
    // (local bit + 1) << 32 | (kInit, or the least document)
    uint32_t ib = 0;
    unsigned long long ent[kWPer];
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) {
      ent[u] = 0;
      if (own >> u & 1u) {
        const uint32_t k = tkey[slot[u]], v = tmin[slot[u]];
        if (v == 0 || (k & kMulti)) {
          ib |= 1u << u;
          ent[u] = ((unsigned long long)(k & ~kMulti) << 32) | (v == 0 ? kInit : v - 1);
        }
      }
    }
    // entries of the whole wave: one ballot per record row (scalar work, no
    // cross-lane shuffles)
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) mine += (uint32_t)__popcll(__ballot((ib >> u) & 1u));
    const uint32_t pcap = min(2 * mine, kWTab);
    wave_sync();
#pragma unroll
    for (uint32_t t = 0; t < kWTab / 64; ++t) {
      const uint32_t q = t * 64 + lane;
      if (q < pcap) wv[q] = 0;
    }
    wave_sync();
#pragma unroll
    for (uint32_t u = 0; u < kWPer; ++u) {
      if (!(ib >> u & 1u)) continue;
      uint32_t h = slot_of((uint32_t)(ent[u] >> 32) - 1, pcap);
      for (uint32_t tries = 0; tries < pcap; ++tries) {
        if (atomicCAS(&wv[h], 0ull, ent[u]) == 0ull) break;
        h = (h + 1 == pcap) ? 0 : h + 1;
      }
    }
    wave_sync();
    uint64_t *T = A.rec1 + 2ull * r0;
    for (uint32_t q = lane; q < pcap; q += 64) T[q] = wv[q];
    if (lane == 0) A.dir[bin] = ((uint64_t)r0 << 32) | pcap;
    wave_sync();
    advance();
  }
}

// Dense bins (bin_bits <= 15: the bin's 512 words fit in LDS): one wave per
// bin, without a per-record hash table.  Every record sets its bit in an LDS
// claim bitmap with one atomicOr; the one that finds the bit clear is the
// bit's first claimer, and every later claimer appends the bit to a short
// list of shared bits (a few per bin: 231 or 462 records over 32,768 bits).
// Only the records of listed bits then take the least and greatest document
// probing the bit.  A bit was set before document i iff it was set before
// the chunk or its least document is below i; it is published for the
// resolve step (by its first claimer) iff it was set before the chunk or two
// different documents probe it.  The new words are the old words ORed with
// the claim bitmap.  A list longer than kListCap leaves the bin to the
// general path (nothing of it has been written yet).
#ifndef LB_LIST_CAP
#define LB_LIST_CAP 96
#endif
constexpr uint32_t kListCap = LB_LIST_CAP;
// Records per bin on the dense path (kDPer per lane): binned_geometry widens
// dense bins while they average at most kDenseFill records.
constexpr uint32_t kDPer = 9;
constexpr uint32_t kDCap = kDPer * 64;
static_assert(kDPer <= 32, "per-lane record masks are 32-bit");
// Persistent grid of the dense bin kernel, waves per compute unit: 16 when
// the call has the device to itself (LDS holds 17 waves of 9.1 KB), 12 when
// other kernels run beside it (the batched form's next MinHash), which keeps
// room on every SIMD for one of their waves.
#ifndef LB_DENSE_WPC
#define LB_DENSE_WPC 16
#endif
#ifndef LB_DENSE_WPC_SHARED
#define LB_DENSE_WPC_SHARED 12
#endif
constexpr uint32_t kDenseWavesPerCu = LB_DENSE_WPC;
constexpr uint32_t kDenseWavesPerCuShared = LB_DENSE_WPC_SHARED;

__global__ __launch_bounds__(64) void k_bq_bin_dense(BinnedLaunch A) {
  __shared__ __align__(16) unsigned long long wv[kWRegion];  // the bin's words; then its published table
  __shared__ __align__(16) unsigned long long cb[kWRegion];  // claim bitmap (the chunk's bits)
  __shared__ uint32_t lk[kListCap], lmin[kListCap], lmax[kListCap];
  __shared__ uint32_t ln;

  const uint32_t lane = threadIdx.x;
  const BinnedGeometry &G = A.G;
  const uint64_t n_bins = (uint64_t)A.bands * G.bins_per_band;
  // A wave's bins are pipelined: the next bin's records and the record
  // range of the bin after it are loaded with the bin's own words, and taken
  // in (settle) after its claims, before any of its stores.  The waits are
  // then for this bin's loads only: a load behind a branch, or a value used
  // as soon as it is loaded, would make the wave wait for the words and the
  // records one after the other.  So every lane loads (lanes past a bin's
  // end re-read a valid slot) and the selects come at settle, where lanes
  // past the end get ~0 (not a record: document indices stay below
  // 2^23 - 1), as does every lane of a bin too large for the dense path.
  // A range is loaded per lane (its start by lane 0, its end by the others)
  // so that it stays in a vector register until it is read.
  auto load_range = [&](uint64_t b) -> uint32_t {
    const uint32_t *p = lane == 0 ? A.off2 : A.end2;
    return p[b < n_bins ? b : 0];
  };
  auto range_of = [&](uint32_t v, uint64_t b, uint32_t &q0, uint32_t &q1) {
    q0 = b < n_bins ? (uint32_t)__builtin_amdgcn_readlane((int)v, 0) : 0u;
    q1 = b < n_bins ? (uint32_t)__builtin_amdgcn_readlane((int)v, 1) : 0u;
  };
  auto load_raw = [&](uint32_t q0, uint32_t q1, uint64_t *raw) {
    const uint32_t last = q1 > 0 ? q1 - 1 : 0;
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) raw[u] = A.rec2[min(q0 + u * 64 + lane, last)];
  };
  auto mask_recs = [&](uint32_t q0, uint32_t q1, const uint64_t *raw, uint64_t *out) {
    const bool small = q1 - q0 <= kDCap;
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) {
      const uint32_t r = q0 + u * 64 + lane;
      out[u] = (small && r < q1) ? raw[u] : ~0ull;
    }
  };
  uint32_t r0, r1, n0, n1;  // the current and the next bin's record ranges
  uint64_t rec[kDPer];
  {
    const uint64_t b1 = (uint64_t)blockIdx.x + gridDim.x;
    range_of(load_range(blockIdx.x), blockIdx.x, r0, r1);
    uint64_t raw[kDPer];
    load_raw(r0, r1, raw);
    const uint32_t v1 = load_range(b1);
    mask_recs(r0, r1, raw, rec);
    range_of(v1, b1, n0, n1);
  }
  for (uint64_t bin = blockIdx.x; bin < n_bins; bin += gridDim.x) {
    const uint64_t b2 = bin + 2ull * gridDim.x;
    uint32_t m0, m1, mv;  // the range of the bin after next
    uint64_t nraw[kDPer], nrec[kDPer];
    auto prefetch = [&]() {
      load_raw(n0, n1, nraw);
      mv = load_range(b2);
    };
    auto settle = [&]() {
      mask_recs(n0, n1, nraw, nrec);
      range_of(mv, b2, m0, m1);
    };
    auto advance = [&]() {
      r0 = n0;
      r1 = n1;
      n0 = m0;
      n1 = m1;
#pragma unroll
      for (uint32_t u = 0; u < kDPer; ++u) rec[u] = nrec[u];
    };
    const uint32_t nr = r1 - r0;
    const uint32_t j = (uint32_t)(bin / G.bins_per_band);
    const uint64_t b0 = (bin - (uint64_t)j * G.bins_per_band) << G.bin_bits;  // a multiple of 64
    uint64_t *F = A.filters + (uint64_t)j * A.words_per_band + (b0 >> 6);
    if (nr == 0 || nr > kDCap) {
      if (nr > kDCap) defer_bin(A, bin);
      prefetch();
      settle();
      advance();
      continue;
    }
    // the bin's words: 2^(bin_bits - 6) <= kWRegion, fewer in a band's last bin
    const uint32_t W = (uint32_t)min((uint64_t)1 << (G.bin_bits - 6), A.words_per_band - (b0 >> 6));
    const bool full = W == kWRegion;
    // clear the claim bitmap and the list; read the bin's words
    {
      uint4 *c4 = reinterpret_cast<uint4 *>(cb);
      const uint4 z = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (uint32_t t = 0; t < kWRegion / 128; ++t) c4[t * 64 + lane] = z;
      if (lane == 0) ln = 0;
      uint64_t reg[kWRegion / 64];
#pragma unroll
      for (uint32_t u = 0; u < kWRegion / 64; ++u) {
        const uint32_t w = u * 64 + lane;
        reg[u] = F[full ? w : min(w, W - 1)];
      }
      prefetch();
#pragma unroll
      for (uint32_t u = 0; u < kWRegion / 64; ++u) {
        const uint32_t w = u * 64 + lane;
        wv[w] = (full || w < W) ? reg[u] : 0ull;
      }
    }
    wave_sync();
    // claims: one atomicOr per record; later claimers list their bit
    uint32_t lbv[kDPer];
    uint32_t initm = 0, dupm = 0;
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) {
      lbv[u] = ~0u;
      if (rec[u] == ~0ull) continue;
      const uint32_t lb = (uint32_t)((rec[u] & kMask40) - b0);
      lbv[u] = lb;
      initm |= (uint32_t)(wv[lb >> 6] >> (lb & 63) & 1ull) << u;
      const unsigned long long bit = 1ull << (lb & 63);
      const unsigned long long old = atomicOr(&cb[lb >> 6], bit);
      if (old & bit) dupm |= 1u << u;
    }
    if (dupm) {
#pragma unroll
      for (uint32_t u = 0; u < kDPer; ++u) {
        if (!(dupm >> u & 1u)) continue;
        const uint32_t k = atomicAdd(&ln, 1u);
        if (k < kListCap) {
          lk[k] = lbv[u];
          lmin[k] = ~0u;
          lmax[k] = 0u;
        }
      }
    }
    wave_sync();
    settle();
    const uint32_t nl = ln;
    if (nl > kListCap) {
      // more shared bits than the list holds: the general path
      defer_bin(A, bin);
      advance();
      continue;
    }
    // records of listed bits: the first list entry of their bit, and the
    // least and greatest document probing it
    uint32_t kix[kDPer];
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) kix[u] = ~0u;
    if (nl) {
      for (uint32_t k = 0; k < nl; ++k) {
        const uint32_t key = lk[k];
#pragma unroll
        for (uint32_t u = 0; u < kDPer; ++u)
          if (kix[u] == ~0u && lbv[u] == key) kix[u] = k;
      }
#pragma unroll
      for (uint32_t u = 0; u < kDPer; ++u) {
        if (kix[u] == ~0u) continue;
        const uint32_t i = (uint32_t)(rec[u] >> 40) & kDocMask;
        atomicMin(&lmin[kix[u]], i);
        atomicMax(&lmax[kix[u]], i);
      }
      wave_sync();
    }
    // probe-0 answers and the entries to publish
    uint32_t pubm = 0;
    unsigned long long ent[kDPer];
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) {
      ent[u] = 0;
      if (lbv[u] == ~0u) continue;
      const uint32_t i = (uint32_t)(rec[u] >> 40) & kDocMask;
      const bool init = initm >> u & 1u;
      uint32_t mn = i;
      bool multi = false;
      if (kix[u] != ~0u) {
        mn = lmin[kix[u]];
        multi = mn != lmax[kix[u]];
      }
      // res0 starts zeroed: only the set-before answers are written
      if ((rec[u] & kProbe0) && (init || mn < i)) A.res0[(int64_t)j * A.n + i] = 1;
      if (!(dupm >> u & 1u) && (init || multi)) {
        pubm |= 1u << u;
        ent[u] = ((unsigned long long)(lbv[u] + 1) << 32) | (init ? kInit : mn);
      }
    }
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) mine += (uint32_t)__popcll(__ballot((pubm >> u) & 1u));
    if (mine > kWRegion) {
      // more bits to publish than the LDS table holds (a filter nearly full):
      // the general path; nothing of the bin but probe-0 answers, which it
      // gives again, has been written
      defer_bin(A, bin);
      advance();
      continue;
    }
    const uint32_t pcap = min(2 * mine, kWRegion);
    // the words after the chunk (this wave is their only writer)
#pragma unroll
    for (uint32_t u = 0; u < kWRegion / 64; ++u) {
      const uint32_t w = u * 64 + lane;
      if (full || w < W) F[w] = wv[w] | cb[w];
    }
    wave_sync();
    {
      uint4 *w4 = reinterpret_cast<uint4 *>(wv);
      const uint4 z = make_uint4(0u, 0u, 0u, 0u);
      for (uint32_t q = lane; 2 * q < pcap; q += 64) w4[q] = z;
    }
    wave_sync();
#pragma unroll
    for (uint32_t u = 0; u < kDPer; ++u) {
      if (!(pubm >> u & 1u)) continue;
      uint32_t h = slot_of(lbv[u], pcap);
      for (uint32_t tries = 0; tries < pcap; ++tries) {
        if (atomicCAS(&wv[h], 0ull, ent[u]) == 0ull) break;
        h = (h + 1 == pcap) ? 0 : h + 1;
      }
    }
    wave_sync();
    uint64_t *T = A.rec1 + 2ull * r0;
    for (uint32_t q = lane; q < pcap; q += 64) T[q] = wv[q];
    if (lane == 0) A.dir[bin] = ((uint64_t)r0 << 32) | pcap;
    wave_sync();
    advance();
  }
}

// --------------------------------------------------------------- resolve ----
// A document's bands are cut into S slices (S a power of two dividing the
// block, chosen so that a chunk of few documents still fills the device);
// thread (slice, document) walks its slice's bands in order and stops at the
// first match, and the slices' answers meet in LDS.
#ifndef LB_RES_GROUP
#define LB_RES_GROUP 4
#endif
constexpr uint32_t kResGroup = LB_RES_GROUP;  // probes whose lookups are issued together

__global__ __launch_bounds__(256) void k_bq_resolve(BinnedLaunch A, uint32_t slice_log) {
  __shared__ uint32_t fl[kThreads];
  const uint32_t per = kThreads >> slice_log;          // documents per block
  const uint32_t sl = threadIdx.x / per, t = threadIdx.x - sl * per;
  const int64_t i = (int64_t)blockIdx.x * per + t;
  const uint32_t bps = (A.bands + (1u << slice_log) - 1) >> slice_log;  // bands per slice
  const uint32_t j0 = sl * bps, j1 = min(A.bands, j0 + bps);
  const BinnedGeometry &G = A.G;
  if (threadIdx.x < per) fl[threadIdx.x] = 0;
  __syncthreads();
  uint32_t flag = 0;
  for (uint32_t j = j0; i < A.n && j < j1 && !flag; ++j) {
    if (!A.res0[(int64_t)j * A.n + i]) continue;
    const uint64_t key = A.keys[(int64_t)j * A.n + i];
    const uint64_t h1 = fmix64(key ^ A.salt1), h2 = fmix64(key ^ A.salt2) | 1ull;
    bool hit = true;
    // Probes 1..k-1 in groups of kResGroup (four): the group's directory
    // entries and first table slots are loaded before any is examined, so that a
    // band whose probes all hit waits for k/4 rounds of dependent loads, not
    // k.  The answer is the same conjunction; the extra reads of a group
    // after a miss are reads of valid tables.
    for (uint32_t l0 = 1; l0 < A.k && hit; l0 += kResGroup) {
      const uint32_t nl = min(kResGroup, A.k - l0);
      uint32_t lb[kResGroup], pcap[kResGroup], h[kResGroup];
      const uint64_t *T[kResGroup];
      uint64_t e[kResGroup];
#pragma unroll
      for (uint32_t u = 0; u < kResGroup; ++u) {
        pcap[u] = 0;
        if (u < nl) {
          const uint64_t g = umulhi64(h1 + (uint64_t)(l0 + u) * h2, A.m_bits);
          const uint64_t lbin = g >> G.bin_bits;
          const uint64_t d = A.dir[(uint64_t)j * G.bins_per_band + lbin];
          pcap[u] = (uint32_t)d;
          T[u] = A.rec1 + 2ull * (d >> 32);
          lb[u] = (uint32_t)(g - (lbin << G.bin_bits));
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < kResGroup; ++u) {
        h[u] = pcap[u] ? slot_of(lb[u], pcap[u]) : 0;
        e[u] = pcap[u] ? T[u][h[u]] : 0;
      }
#pragma unroll
      for (uint32_t u = 0; u < kResGroup; ++u) {
        if (u >= nl || !hit) break;
        bool found = false;
        uint32_t v = 0;
        for (uint32_t tries = 0; tries < pcap[u]; ++tries) {
          const uint32_t ek = (uint32_t)(e[u] >> 32);
          if (ek == lb[u] + 1) {
            v = (uint32_t)e[u];
            found = true;
            break;
          }
          if (ek == 0) break;
          h[u] = (h[u] + 1 == pcap[u]) ? 0 : h[u] + 1;
          e[u] = T[u][h[u]];
        }
        // not published: the only document probing the bit is this one
        hit = found && (v == kInit || v < (uint32_t)i);
      }
    }
    if (hit) flag = 1;
  }
  if (flag) atomicOr(&fl[t], 1u);
  __syncthreads();
  if (threadIdx.x < per && i < A.n) A.flags[i] = (uint8_t)fl[threadIdx.x];
}

inline unsigned grid1(uint64_t n, unsigned bs) {
  const uint64_t g = (n + bs - 1) / bs;
  return (unsigned)(g == 0 ? 1 : g);
}

inline uint32_t ceil_log2(uint64_t x) {
  uint32_t s = 0;
  while (s < 63 && (1ull << s) < x) ++s;
  return s;
}

}  // namespace

BinnedGeometry binned_geometry(uint64_t n_docs, uint32_t bands, uint32_t k, uint64_t m_bits, uint32_t target_per_bin) {
  (void)bands;
  BinnedGeometry G{};
  const double probes_per_band = (double)n_docs * k;
  // bits per bin so that a bin receives about target_per_bin records
  const double want = (double)m_bits * target_per_bin / (probes_per_band > 0 ? probes_per_band : 1.0);
  uint32_t s = 6;  // nearest power of two
  while (s < 24 && (double)(1ull << s) * 1.4142135623730951 <= want) ++s;
  while (s < 15 && probes_per_band * (double)(1ull << (s + 1)) <= (double)kDenseFill * (double)m_bits) ++s;
  G.bin_bits = s;
  G.bins_per_band = (m_bits + (1ull << s) - 1) >> s;
  // at most 2^20 bins per band (1024 x 1024 over the two passes): wider bins
  // beyond that (only for chunks of more than ~1.9e8 probes per band)
  while (s < 39 && ceil_log2(G.bins_per_band) > 20) {
    ++s;
    G.bin_bits = s;
    G.bins_per_band = (m_bits + (1ull << s) - 1) >> s;
  }
  // split the bins of a band between the two passes, pass 1 taking one bit
  // more than half (at most 1024 buckets and 1024 bins per bucket): smaller
  // pass-2 buckets are re-read less between counting and splitting, which
  // outweighs pass 1's shorter runs (1M-document chunks over 117,006 bins
  // per band: 18.8 ms per chunk against 19.8 with an even split)
  const uint32_t t = ceil_log2(G.bins_per_band);
  uint32_t f1 = t / 2 + 1;
  if (f1 > t) f1 = t;
  if (f1 > 10) f1 = 10;
  if (t > 10 && t - 10 > f1) f1 = t - 10;
  G.bucket_bits = s + (t - f1);
  G.bins_per_bucket = 1u << (t - f1);
  G.buckets_per_band = (uint32_t)((m_bits + (1ull << G.bucket_bits) - 1) >> G.bucket_bits);
  G.n_tiles = (uint32_t)((n_docs + kTileDocs - 1) / kTileDocs);
  if (G.n_tiles == 0) G.n_tiles = 1;
  G.direct_words = s <= 15;
  return G;
}

namespace {

// Keys, pass 1 and pass 2 of a chunk.
hipError_t launch_partition(const BinnedLaunch &a, hipStream_t s) {
  const BinnedGeometry &G = a.G;
  hipError_t e;
  const uint32_t td = keys_tile_docs(a.bands * a.rows);
  const size_t ldsk = (size_t)td * (a.bands * a.rows + 1) * 4;
  {
    const uint64_t words = ((uint64_t)a.n * a.bands + 3) / 4;  // the allocation is padded to 16 bytes
    const uint64_t g = std::min<uint64_t>((words + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_bq_zero_res0, dim3((unsigned)std::max<uint64_t>(g, 1)), dim3(kThreads), 0, s, a, words);
  }
  if (a.keys_in)
    hipLaunchKernelGGL(k_bq_keys_in, dim3(grid1((uint64_t)a.n * a.bands, kThreads)), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_bq_keys, dim3(grid1((uint64_t)a.n, td)), dim3(kThreads), ldsk, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_count1, dim3(G.n_tiles, a.bands), dim3(kThreads), (size_t)G.buckets_per_band * 4, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t nb = a.bands * G.buckets_per_band;
  hipLaunchKernelGGL(k_bq_scan_tiles, dim3(nb), dim3(kThreads), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_scan_buckets, dim3(1), dim3(kThreads), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds1 = kSub1 * 8 + 4 * (size_t)((G.buckets_per_band + 3) & ~3u) * 4 + 16 * 4;
  hipLaunchKernelGGL(k_bq_scatter1, dim3(G.n_tiles, a.bands), dim3(kT1), lds1, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the larger sub-tile where LDS holds it (c3: 118,000-record buckets in 7
  // sub-tiles instead of 8; c4: a larger first sub-tile kept in registers)
  if (part2_lds(kPer2Big, G.bins_per_bucket) <= 163840)
    hipLaunchKernelGGL(k_bq_part2<kPer2Big>, dim3(nb), dim3(kT2), part2_lds(kPer2Big, G.bins_per_bucket), s, a);
  else
    hipLaunchKernelGGL(k_bq_part2<kPer2>, dim3(nb), dim3(kT2), part2_lds(kPer2, G.bins_per_bucket), s, a);
  return hipGetLastError();
}

// Bins and resolve of a chunk (after its partition).
hipError_t launch_bins(const BinnedLaunch &a, hipStream_t s) {
  const BinnedGeometry &G = a.G;
  hipError_t e;
  const uint64_t n_bins = (uint64_t)a.bands * G.bins_per_band;
  // dense bins: a persistent grid of kDenseWavesPerCu waves per compute unit,
  // or of kDenseWavesPerCuShared beside other work, which leaves room on every
  // compute unit for the waves of a MinHash launch; sparse bins: one
  // workgroup per bin (at most 262,144), as many waves as fit, to cover the
  // random reads' latency
  const uint32_t wpc = a.shared_device ? kDenseWavesPerCuShared : kDenseWavesPerCu;
  const uint64_t cap = G.direct_words ? (uint64_t)wpc * (a.cus ? a.cus : 256) : 262144;
  const unsigned gb = (unsigned)(n_bins < cap ? n_bins : cap);
  if (G.direct_words)
    hipLaunchKernelGGL(k_bq_bin_dense, dim3(gb), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_bq_bin_sparse, dim3(gb), dim3(64), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the bins left to the general path (usually none: then every wave reads
  // the count and ends)
  hipLaunchKernelGGL(k_bq_bin_overflow, dim3((unsigned)kDenseWavesPerCu * (a.cus ? a.cus : 256)), dim3(64), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // slices of bands per document: enough threads for about 2^18 (document,
  // slice) pairs, at most one band per slice and 256 slices
  uint32_t slice_log = 0;
  while (slice_log < 8 && ((uint64_t)a.n << slice_log) < (1ull << 18) && (1u << (slice_log + 1)) <= a.bands) ++slice_log;
  hipLaunchKernelGGL(k_bq_resolve, dim3(grid1((uint64_t)a.n, kThreads >> slice_log)), dim3(kThreads), 0, s, a, slice_log);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_query_insert_binned(const BinnedLaunch &a, hipStream_t s, int part) {
  if (a.n == 0) return hipSuccess;
  const BinnedGeometry &G = a.G;
  if (G.buckets_per_band > kMaxF1 || G.bins_per_bucket > kMaxF2 || G.bucket_bits > 32) return hipErrorInvalidValue;
  if (part != 2) {
    const hipError_t e = launch_partition(a, s);
    if (e != hipSuccess || part == 1) return e;
  }
  return launch_bins(a, s);
}

}  // namespace lb
