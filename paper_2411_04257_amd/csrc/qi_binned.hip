// Binned, atomic-free (on global memory) in-order query-insert for large
// batches (Sections 2.1, 2.4, 4.1, 4.2, 4.4.2).
//
// The direct query-insert of kernels.hip spends one device-scope atomic per
// probe on the first-setter table and another on the filter word; on MI355X
// those run near 2e10/s whatever the locality.  Here one chunk's probes are
// partitioned by (band, bit range) so that one workgroup owns every probe of
// a bin of 2^s filter bits:
//
//   pass 1 (k_bq_count1 / scan / k_bq_scatter1): per (document, band) item,
//       the k Bloom positions, bucketed into "super bins" (ranges of bins of
//       one band) with per-block LDS histograms, written as 64-bit records
//       (document index << 40 | bit position);
//   pass 2 (k_bq_part2): one block per super bin splits its records into bins
//       and writes every bin's record range;
//   bin   (k_bq_bin): one workgroup per bin reads the filter word of every
//       record (the state before the chunk), builds in LDS a table of the
//       bin's distinct bits with their first setter (minimum document index,
//       or a marker when the bit was already set) and a table of OR masks per
//       word, then writes the changed words back with plain stores (it is the
//       only writer of its bit range) and publishes its bit table to global
//       memory, in the same slot layout;
//   resolve (k_bq_resolve): one thread per (document, band) looks its
//       positions up in the published tables: a bit was set before document i
//       iff it was set before the chunk or its first setter is < i; the band
//       hits iff all k were, and the scan stops at the first miss.
//
// Every step is exact, so flags and final filter words equal the sequential
// definition for every chunking; bins whose record count exceeds the LDS
// capacity take a slower path with global-memory tables owned by the bin.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "qi_binned.h"

namespace lb {

namespace {

constexpr uint32_t kInit = 0xFFFFFFFFu;   // bit set before the chunk
constexpr uint32_t kNoFs = 0xFFFFFFFEu;   // no setter recorded yet
constexpr uint64_t kMask40 = (1ull << 40) - 1;

// Slot of a 32-bit key in a table of `cap` slots (multiply-high range reduction).
__device__ __forceinline__ uint32_t slot_of(uint32_t key, uint32_t cap) {
  const uint32_t h = key * 0x9E3779B1u;
  const uint32_t h2 = (h ^ (h >> 15)) * 0x85EBCA77u;
  return (uint32_t)(((uint64_t)(h2 ^ (h2 >> 13)) * cap) >> 32);
}

struct ItemPos {
  uint64_t h1, h2;
};

__device__ __forceinline__ ItemPos item_hashes(const BinnedLaunch &A, int64_t i, uint32_t j) {
  const uint64_t K = band_key(A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows, A.rows, A.salt_m);
  return {fmix64(K ^ A.salt1), fmix64(K ^ A.salt2) | 1ull};
}

__device__ __forceinline__ uint32_t super_of(const BinnedLaunch &A, uint32_t j, uint64_t g) {
  const uint64_t lbin = g >> A.bin_bits;
  return j * A.supers_per_band + (uint32_t)(lbin / A.bins_per_super);
}

// ---------------------------------------------------------------- pass 1 ----
__global__ __launch_bounds__(1024) void k_bq_count1(BinnedLaunch A) {
  extern __shared__ uint32_t hist[];  // n_supers counters
  for (uint32_t s = threadIdx.x; s < A.n_supers; s += blockDim.x) hist[s] = 0;
  __syncthreads();
  const int64_t items = A.n * (int64_t)A.bands;
  const int64_t t0 = (int64_t)blockIdx.x * A.items_per_block;
  const int64_t t1 = min(items, t0 + (int64_t)A.items_per_block);
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int64_t i = t / A.bands;
    const uint32_t j = (uint32_t)(t - i * A.bands);
    const ItemPos hp = item_hashes(A, i, j);
    for (uint32_t l = 0; l < A.k; ++l) {
      const uint64_t g = umulhi64(hp.h1 + (uint64_t)l * hp.h2, A.m_bits);
      atomicAdd(&hist[super_of(A, j, g)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < A.n_supers; s += blockDim.x)
    A.counts1[(uint64_t)s * A.n_blocks1 + blockIdx.x] = hist[s];
}

__global__ __launch_bounds__(1024) void k_bq_scatter1(BinnedLaunch A) {
  extern __shared__ uint32_t cur[];  // n_supers cursors
  for (uint32_t s = threadIdx.x; s < A.n_supers; s += blockDim.x)
    cur[s] = A.offs1[(uint64_t)s * A.n_blocks1 + blockIdx.x];
  __syncthreads();
  const int64_t items = A.n * (int64_t)A.bands;
  const int64_t t0 = (int64_t)blockIdx.x * A.items_per_block;
  const int64_t t1 = min(items, t0 + (int64_t)A.items_per_block);
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int64_t i = t / A.bands;
    const uint32_t j = (uint32_t)(t - i * A.bands);
    const ItemPos hp = item_hashes(A, i, j);
    for (uint32_t l = 0; l < A.k; ++l) {
      const uint64_t g = umulhi64(hp.h1 + (uint64_t)l * hp.h2, A.m_bits);
      const uint32_t pos = atomicAdd(&cur[super_of(A, j, g)], 1u);
      A.rec1[pos] = ((uint64_t)i << 40) | g;
    }
  }
}

// Exclusive scan of every super bin's row of per-block counts (one block per
// super bin); the row total goes to super_tot.
__global__ __launch_bounds__(1024) void k_bq_rowscan(BinnedLaunch A) {
  __shared__ uint32_t buf[1024];
  __shared__ uint32_t carry;
  const uint32_t s = blockIdx.x;
  const uint32_t *in = A.counts1 + (uint64_t)s * A.n_blocks1;
  uint32_t *out = A.offs1 + (uint64_t)s * A.n_blocks1;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < A.n_blocks1; base += 1024) {
    const uint32_t idx = base + threadIdx.x;
    const uint32_t v = idx < A.n_blocks1 ? in[idx] : 0u;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
      const uint32_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0u;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    const uint32_t incl = buf[threadIdx.x];
    if (idx < A.n_blocks1) out[idx] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) A.super_tot[s] = carry;
}

// Exclusive scan of the super bins' totals (one block), then every row of
// offs1 is shifted by its super bin's start (grid over rows).
__global__ __launch_bounds__(1024) void k_bq_superscan(BinnedLaunch A) {
  __shared__ uint32_t buf[1024];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < A.n_supers; base += 1024) {
    const uint32_t idx = base + threadIdx.x;
    const uint32_t v = idx < A.n_supers ? A.super_tot[idx] : 0u;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
      const uint32_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0u;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    const uint32_t incl = buf[threadIdx.x];
    if (idx < A.n_supers) A.super_tot[idx] = carry + incl - v;  // now the super bin's start
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_bq_rowshift(BinnedLaunch A) {
  const uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (uint64_t)A.n_supers * A.n_blocks1) return;
  A.offs1[q] += A.super_tot[q / A.n_blocks1];
}

// ---------------------------------------------------------------- pass 2 ----
// One block per super bin: count its records per bin, scan in LDS, publish
// the bins' offsets and scatter the records by bin.
__global__ __launch_bounds__(1024) void k_bq_part2(BinnedLaunch A) {
  extern __shared__ uint32_t cnt[];  // bins_per_super counters
  const uint32_t s = blockIdx.x;
  const uint32_t j = s / A.supers_per_band;
  const uint64_t first_lbin = (uint64_t)(s % A.supers_per_band) * A.bins_per_super;
  const uint32_t r0 = A.super_tot[s];
  const uint32_t r1 = (s + 1 < A.n_supers) ? A.super_tot[s + 1] : A.n_records;
  const uint32_t fb = A.bins_per_super;
  for (uint32_t f = threadIdx.x; f < fb; f += blockDim.x) cnt[f] = 0;
  __syncthreads();
  for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const uint64_t g = A.rec1[r] & kMask40;
    atomicAdd(&cnt[(uint32_t)((g >> A.bin_bits) - first_lbin)], 1u);
  }
  __syncthreads();
  // exclusive scan of cnt[0..fb) by thread 0..: fb <= 4096, simple strided
  // two-level scan: each thread sums a run, then the runs are scanned.
  __shared__ uint32_t run[1024];
  const uint32_t per = (fb + blockDim.x - 1) / blockDim.x;
  const uint32_t f0 = threadIdx.x * per, f1 = min(fb, f0 + per);
  uint32_t sum = 0;
  for (uint32_t f = f0; f < f1; ++f) sum += cnt[f];
  run[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t q = 0; q < blockDim.x; ++q) {
      const uint32_t v = run[q];
      run[q] = acc;
      acc += v;
    }
  }
  __syncthreads();
  uint32_t acc = r0 + run[threadIdx.x];
  for (uint32_t f = f0; f < f1; ++f) {
    const uint32_t v = cnt[f];
    cnt[f] = acc;  // becomes the cursor
    const uint64_t lbin = first_lbin + f;
    if (lbin < A.bins_per_band) A.off2[(uint64_t)j * A.bins_per_band + lbin] = acc;
    acc += v;
  }
  __syncthreads();
  for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const uint64_t rec = A.rec1[r];
    const uint64_t g = rec & kMask40;
    const uint32_t pos = atomicAdd(&cnt[(uint32_t)((g >> A.bin_bits) - first_lbin)], 1u);
    A.rec2[pos] = rec;
  }
  if (s == A.n_supers - 1 && threadIdx.x == 0) A.off2[(uint64_t)A.bands * A.bins_per_band] = A.n_records;
}

// ------------------------------------------------------------------- bins ----
constexpr uint32_t kBinCap = 1024;       // records per bin handled in LDS
constexpr uint32_t kTab = 2 * kBinCap;   // LDS table slots

__global__ __launch_bounds__(256) void k_bq_bin(BinnedLaunch A) {
  __shared__ uint32_t tkey[kTab];  // bit table: local bit + 1 (0 = empty)
  __shared__ uint32_t tval[kTab];  // first setter, or kInit
  __shared__ uint32_t wkey[kTab];  // word table: local word + 1
  __shared__ unsigned long long wmask[kTab];

  const uint64_t n_bins = (uint64_t)A.bands * A.bins_per_band;
  for (uint64_t bin = blockIdx.x; bin < n_bins; bin += gridDim.x) {
    const uint32_t r0 = A.off2[bin], r1 = A.off2[bin + 1];
    const uint32_t nr = r1 - r0;
    if (nr == 0) continue;
    const uint32_t j = (uint32_t)(bin / A.bins_per_band);
    const uint64_t lbin = bin - (uint64_t)j * A.bins_per_band;
    const uint64_t b0 = lbin << A.bin_bits;  // first bit of the bin (multiple of 64)
    uint64_t *F = A.filters + (uint64_t)j * A.words_per_band + (b0 >> 6);
    uint64_t *T = A.table + 2ull * r0;
    const uint32_t cap = 2 * nr;
    if (nr <= kBinCap) {
      for (uint32_t q = threadIdx.x; q < cap; q += blockDim.x) {
        tkey[q] = 0;
        tval[q] = kNoFs;
        wkey[q] = 0;
        wmask[q] = 0;
      }
      __syncthreads();
      for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const uint64_t rec = A.rec2[r];
        const uint32_t i = (uint32_t)(rec >> 40);
        const uint32_t lb = (uint32_t)((rec & kMask40) - b0);
        const uint32_t lw = lb >> 6;
        const bool init = (F[lw] >> (lb & 63)) & 1ull;
        uint32_t h = slot_of(lb, cap);
        for (uint32_t tries = 0; tries < cap; ++tries) {
          const uint32_t old = atomicCAS(&tkey[h], 0u, lb + 1);
          if (old == 0u || old == lb + 1) break;
          h = (h + 1 == cap) ? 0 : h + 1;
        }
        if (init)
          tval[h] = kInit;
        else
          atomicMin(&tval[h], i);
        uint32_t hw = slot_of(lw, cap);
        for (uint32_t tries = 0; tries < cap; ++tries) {
          const uint32_t old = atomicCAS(&wkey[hw], 0u, lw + 1);
          if (old == 0u || old == lw + 1) break;
          hw = (hw + 1 == cap) ? 0 : hw + 1;
        }
        atomicOr(&wmask[hw], 1ull << (lb & 63));
      }
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < cap; q += blockDim.x) {
        const uint32_t wk = wkey[q];
        if (wk) {
          const uint64_t old = F[wk - 1];
          const uint64_t nw = old | wmask[q];
          if (nw != old) F[wk - 1] = nw;
        }
        const uint32_t key = tkey[q];
        T[q] = key ? (((uint64_t)key << 32) | tval[q]) : 0ull;
      }
      __syncthreads();
    } else {
      // Hot bin (many documents sharing bits): the same steps with the bit
      // table in the bin's own global segment; filter bits are set after every
      // record has read the state before the chunk.
      for (uint32_t q = threadIdx.x; q < cap; q += blockDim.x) T[q] = ((uint64_t)0 << 32) | kNoFs;
      __syncthreads();
      for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const uint64_t rec = A.rec2[r];
        const uint32_t i = (uint32_t)(rec >> 40);
        const uint32_t lb = (uint32_t)((rec & kMask40) - b0);
        const bool init = (F[lb >> 6] >> (lb & 63)) & 1ull;
        uint32_t h = slot_of(lb, cap);
        for (uint32_t tries = 0; tries < 4 * cap; ++tries) {
          unsigned long long *slot = (unsigned long long *)&T[h];
          const unsigned long long cur = *slot;
          const uint32_t key = (uint32_t)(cur >> 32);
          if (key == lb + 1) break;
          if (key == 0) {
            const unsigned long long want = ((unsigned long long)(lb + 1) << 32) | kNoFs;
            const unsigned long long old = atomicCAS(slot, cur, want);
            if (old == cur || (uint32_t)(old >> 32) == lb + 1) break;
            continue;  // another key took the slot: look at it again
          }
          h = (h + 1 == cap) ? 0 : h + 1;
        }
        unsigned long long *slot = (unsigned long long *)&T[h];
        if (init)
          atomicOr(slot, (unsigned long long)kInit);  // low word becomes all ones
        else
          atomicMin(slot, ((unsigned long long)(lb + 1) << 32) | i);
      }
      __syncthreads();
      for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const uint32_t lb = (uint32_t)((A.rec2[r] & kMask40) - b0);
        atomicOr((unsigned long long *)&F[lb >> 6], (unsigned long long)(1ull << (lb & 63)));
      }
      __syncthreads();
      // empty slots must read as key 0
      for (uint32_t q = threadIdx.x; q < cap; q += blockDim.x)
        if ((uint32_t)(T[q] >> 32) == 0) T[q] = 0;
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------- resolve ----
__global__ __launch_bounds__(256) void k_bq_resolve(BinnedLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  const ItemPos hp = item_hashes(A, i, j);
  bool hit = true;
  for (uint32_t l = 0; l < A.k && hit; ++l) {
    const uint64_t g = umulhi64(hp.h1 + (uint64_t)l * hp.h2, A.m_bits);
    const uint64_t lbin = g >> A.bin_bits;
    const uint64_t bin = (uint64_t)j * A.bins_per_band + lbin;
    const uint32_t r0 = A.off2[bin], r1 = A.off2[bin + 1];
    const uint32_t cap = 2 * (r1 - r0);
    const uint32_t lb = (uint32_t)(g - (lbin << A.bin_bits));
    const uint64_t *T = A.table + 2ull * r0;
    uint32_t h = slot_of(lb, cap);
    uint32_t val = kNoFs;
    bool found = false;
    for (uint32_t tries = 0; tries < cap; ++tries) {
      const uint64_t e = T[h];
      const uint32_t key = (uint32_t)(e >> 32);
      if (key == lb + 1) {
        val = (uint32_t)e;
        found = true;
        break;
      }
      if (key == 0) break;
      h = (h + 1 == cap) ? 0 : h + 1;
    }
    if (!found || val == kNoFs) {
      atomicOr(A.status, 2u);  // every probed bit was published by its bin
      hit = false;
      break;
    }
    if (val != kInit && val >= (uint32_t)i) hit = false;
  }
  A.hitb[t] = hit ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_bq_flags(BinnedLaunch A) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= A.n) return;
  const uint8_t *hb = A.hitb + i * (int64_t)A.bands;
  uint8_t f = 0;
  for (uint32_t j = 0; j < A.bands; ++j) f |= hb[j];
  A.flags[i] = f;
}

inline unsigned grid1(uint64_t n, unsigned bs) {
  const uint64_t g = (n + bs - 1) / bs;
  return (unsigned)(g == 0 ? 1 : g);
}

}  // namespace

BinnedGeometry binned_geometry(uint64_t n_docs, uint32_t bands, uint32_t k, uint64_t m_bits, uint32_t target_per_bin) {
  BinnedGeometry G{};
  const double probes_per_band = (double)n_docs * k;
  // bits per bin so that a bin receives about target_per_bin records
  const double want = (double)m_bits * target_per_bin / (probes_per_band > 0 ? probes_per_band : 1.0);
  uint32_t s = 6;
  while (s < 24 && (double)(1ull << (s + 1)) <= want) ++s;
  for (;; ++s) {
    G.bin_bits = s;
    G.bins_per_band = (m_bits + (1ull << s) - 1) >> s;
    uint64_t spb = 2048 / bands;
    if (spb < 1) spb = 1;
    if (spb > G.bins_per_band) spb = G.bins_per_band;
    uint64_t fb = (G.bins_per_band + spb - 1) / spb;
    while (fb > 4096) {  // a super bin's counters live in LDS
      spb *= 2;
      fb = (G.bins_per_band + spb - 1) / spb;
    }
    G.supers_per_band = (uint32_t)((G.bins_per_band + fb - 1) / fb);
    G.bins_per_super = (uint32_t)fb;
    G.n_supers = G.supers_per_band * bands;
    if (G.n_supers <= 8192 || s >= 31) break;  // local bits must fit 32-bit keys  // pass-1 histograms live in LDS too
  }
  const uint64_t items = n_docs * bands;
  uint64_t ipb = (items + 1535) / 1536;
  if (ipb < 1024) ipb = 1024;
  G.items_per_block = (uint32_t)ipb;
  G.n_blocks1 = (uint32_t)((items + ipb - 1) / ipb);
  if (G.n_blocks1 == 0) G.n_blocks1 = 1;
  return G;
}

hipError_t launch_query_insert_binned(const BinnedLaunch &a, hipStream_t s) {
  const uint64_t items = (uint64_t)a.n * a.bands;
  if (items == 0) return hipSuccess;
  const size_t lds1 = (size_t)a.n_supers * sizeof(uint32_t);
  hipLaunchKernelGGL(k_bq_count1, dim3(a.n_blocks1), dim3(1024), lds1, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_rowscan, dim3(a.n_supers), dim3(1024), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_superscan, dim3(1), dim3(1024), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_rowshift, dim3(grid1((uint64_t)a.n_supers * a.n_blocks1, 256)), dim3(256), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_scatter1, dim3(a.n_blocks1), dim3(1024), lds1, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_part2, dim3(a.n_supers), dim3(1024), (size_t)a.bins_per_super * sizeof(uint32_t), s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint64_t n_bins = (uint64_t)a.bands * a.bins_per_band;
  uint64_t gb = n_bins < 32768 ? n_bins : 32768;
  hipLaunchKernelGGL(k_bq_bin, dim3((unsigned)gb), dim3(256), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_resolve, dim3(grid1(items, 256)), dim3(256), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bq_flags, dim3(grid1((uint64_t)a.n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lb
