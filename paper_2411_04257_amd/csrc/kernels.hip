// LSHBloom hot-path kernels for gfx950 (wave64, VALU integer work, no MFMA).
//
//  k_minhash   : Section 2.2.  Persistent grid; each wave owns one contiguous
//                range of token positions of the whole CSR batch.  Per tile of
//                64 positions, lane l hashes the shingle starting at position
//                tile+l (SHA-1), then the wave walks the tile's valid shingles
//                with lanes = permutations, keeping running minima in VGPRs
//                across tiles while the document continues.  A document that
//                lies wholly in the wave's range is stored with plain
//                coalesced stores; one cut by a range boundary is merged with
//                atomicMin into a row pre-filled with 0xFFFFFFFF.
//  k_band_keys : Section 4.1 band keys (export for checking).
//  k_qi_probe  : Sections 2.4, 4.2.  One thread per (document, band) of a
//                chunk: band key, k positions, read the filter words; bits
//                already set are recorded in a mask, bits still clear are
//                registered in a first-setter table keyed by (band, bit)
//                whose value is the smallest document index probing it.
//  k_qi_resolve: the bit was set before document i iff it was set before the
//                chunk or its first setter is < i (Section 2.1 order); the
//                band hits iff all k bits were; the first setter of a clear bit
//                sets it with atomicOr (Section 4.1 insert).
//  k_qi_flags  : OR over bands (Section 4.2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.h"
#include "kernels.h"

namespace lb {

namespace {

constexpr int kBlock = 256;

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// First index i in [0, n) with a[i] > v, or n.
__device__ __forceinline__ int64_t upper_bound_i64(const int64_t *__restrict__ a, int64_t n, int64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) {
  const uint32_t lo = (uint32_t)(uint64_t)v, hi = (uint32_t)((uint64_t)v >> 32);
  const uint32_t rlo = (uint32_t)__shfl((int)lo, src, 64);
  const uint32_t rhi = (uint32_t)__shfl((int)hi, src, 64);
  return (int64_t)(((uint64_t)rhi << 32) | rlo);
}

// Orders one wave's LDS accesses around an exchange between its lanes: a
// wave's LDS operations complete in issue order, so only the compiler needs
// holding back.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane src's value of v in scalar registers: known wave-uniform, so that
// branches on it and values derived from it stay off the vector registers.
__device__ __forceinline__ int64_t readlane64(int64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Waves per SIMD the register budget must allow (97 VGPRs would give 4 at
// PPL = 2; 96 gives 5).
constexpr int minhash_min_waves(int ppl) { return ppl <= 2 ? 5 : (ppl <= 4 ? 4 : 3); }

// WIDE: the signature values are the whole 61-bit permutation values
// (uint64 rows in A.sigs64) instead of their low 32 bits.
template <int PPL, int WFIX, bool WIDE>
__global__ __launch_bounds__(kBlock, minhash_min_waves(PPL)) void k_minhash(MinhashLaunch A) {
  using V = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  constexpr V kEmpty = ~(V)0;
  const int lane = threadIdx.x & 63;
  // The wave's row of shingle hashes for the full-tile path.
  __shared__ __align__(16) uint32_t xs_block[kBlock];
  uint32_t *const xs = xs_block + (threadIdx.x & ~63u);
  // The wave's index, its token range and the tile positions derived from it
  // are wave-uniform: readfirstlane keeps them in scalar registers.
  const int64_t wave =
      (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t n_docs = A.n_docs;
  const int64_t base = A.offsets[0];
  const int64_t end = A.offsets[n_docs];
  const int64_t total = end - base;
  if (total <= 0) return;
  const int64_t r0 = base + (total * wave) / A.waves;
  const int64_t r1 = base + (total * (wave + 1)) / A.waves;
  if (r0 >= r1) return;

  const uint32_t P = A.num_perm;
  const int64_t w = WFIX ? WFIX : (int64_t)A.w;
  uint32_t al[PPL], ah[PPL], bl[PPL], bh[PPL];
  V mn[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const uint32_t i = (uint32_t)p * 64u + (uint32_t)lane;
    PermCoef c = {0, 0, 0, 0};
    if (i < P) c = A.coef[i];
    // The high words are kept times 8 (perm_lo32_flagged, perm_r_flagged).
    al[p] = c.a_lo;
    ah[p] = c.a_hi << 3;
    bl[p] = c.b_lo;
    bh[p] = c.b_hi << 3;
    mn[p] = kEmpty;
  }

  // Document containing the first position of the current tile.
  int64_t dcur = upper_bound_i64(A.offsets, n_docs + 1, r0) - 1;
  int64_t cur = -1;  // document whose partial minima are held in mn[]

  auto flush = [&](int64_t d) {
    const int64_t s0 = A.offsets[d], e0 = A.offsets[d + 1];
    const int64_t last = (e0 - s0 >= w) ? e0 - w : s0;
    const bool inside = s0 >= r0 && last < r1;
    if constexpr (WIDE) {
      uint64_t *row = A.sigs64 + (A.row_ids ? A.row_ids[d] : d) * (int64_t)P;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const uint32_t i = (uint32_t)p * 64u + (uint32_t)lane;
        if (i < P) {
          if (inside)
            row[i] = mn[p];
          else
            atomicMin((unsigned long long *)&row[i], (unsigned long long)mn[p]);
        }
        mn[p] = kEmpty;
      }
    } else {
      uint32_t *row = A.sigs + (A.row_ids ? A.row_ids[d] : d) * (int64_t)P;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const uint32_t i = (uint32_t)p * 64u + (uint32_t)lane;
        if (i < P) {
          if (inside)
            row[i] = mn[p];
          else
            atomicMin(&row[i], mn[p]);
        }
        mn[p] = kEmpty;
      }
    }
  };

  // A tile of 64 shingles of document d, lane i holding shingle i's hash.
  // The hashes go through the wave's LDS row and come back as uniform-address
  // 16-byte reads, broadcasts on the LDS pipe instead of one VALU readlane
  // per shingle.  The flag words of the whole tile fold into one maximum,
  // tested once; a flagged tile restarts from the minima saved at its start
  // and takes the exact form for all its evaluations.
  auto full_tile = [&](int64_t d, uint32_t x) {
    if (d != cur) {
      if (cur >= 0) flush(cur);
      cur = d;
    }
    wave_lds_sync();
    xs[lane] = x;
    wave_lds_sync();
    V saved[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) saved[p] = mn[p];
    uint32_t fmax = 0;
#pragma unroll 2
    for (int k = 0; k < 64; k += 4) {
      const uint4 q = *reinterpret_cast<const uint4 *>(xs + k);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        uint32_t f0, f1, f2, f3;
        if constexpr (WIDE) {
          // folded values not yet below p: a flag-free tile has them all < p
          const uint64_t c0 = perm_r_flagged(q.x, al[p], ah[p], bl[p], bh[p], f0);
          const uint64_t c1 = perm_r_flagged(q.y, al[p], ah[p], bl[p], bh[p], f1);
          const uint64_t c2 = perm_r_flagged(q.z, al[p], ah[p], bl[p], bh[p], f2);
          const uint64_t c3 = perm_r_flagged(q.w, al[p], ah[p], bl[p], bh[p], f3);
          mn[p] = min(min(min(min(mn[p], c0), c1), c2), c3);
        } else {
          const uint32_t v0 = perm_lo32_flagged(q.x, al[p], ah[p], bl[p], bh[p], f0);
          const uint32_t v1 = perm_lo32_flagged(q.y, al[p], ah[p], bl[p], bh[p], f1);
          const uint32_t v2 = perm_lo32_flagged(q.z, al[p], ah[p], bl[p], bh[p], f2);
          const uint32_t v3 = perm_lo32_flagged(q.w, al[p], ah[p], bl[p], bh[p], f3);
          // chains, so that each folds into two v_min3 / v_max3
          mn[p] = min(min(min(min(mn[p], v0), v1), v2), v3);
        }
        fmax = max(max(max(max(fmax, f0), f1), f2), f3);
      }
    }
    if (__ballot(fmax >= kPermFlag)) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) mn[p] = saved[p];
      for (int k = 0; k < 64; ++k) {
        const uint32_t xk = xs[k];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          if constexpr (WIDE) {
            uint32_t f;
            const uint64_t c = perm_r_flagged(xk, al[p], ah[p], bl[p], bh[p], f);
            mn[p] = min(mn[p], c >= kP61 ? c - kP61 : c);
          } else {
            mn[p] = min(mn[p], perm_lo32(xk, al[p], ah[p] >> 3, bl[p], bh[p] >> 3));
          }
        }
      }
    }
  };

  for (int64_t tb = r0; tb < r1; tb += 64) {
    const int64_t pos = tb + lane;
    int64_t doc, ds, de, dnext;
    bool valid;
    // Tile inside the current document: its end, one scalar load, covers the
    // last lane's shingle (and the next tile starts in it too), so every lane
    // holds a shingle of document dcur and the search is skipped.  ds = tb
    // stands in for the document's start (only L >= w is read from it).
    de = A.offsets[dcur + 1];
    const bool inside_doc = tb + 64 <= r1 && de >= tb + 63 + (w > 2 ? w : 2);
    if (inside_doc) {
      doc = dcur;
      ds = tb;
      dnext = dcur;
      valid = true;
    } else {
      const bool in_range = pos < r1;
      // Ends of documents dcur, dcur+1, ..., dcur+63.
      const int64_t jd = dcur + 1 + lane;
      const int64_t e = (jd <= n_docs) ? A.offsets[jd] : INT64_MAX;
      const int64_t e63 = readlane64(e, 63);
      if (e63 > tb + 64) {
        // The 64-document window covers the tile: count the ends <= pos.
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const int64_t v = shfl64(e, lo + step - 1);
          if (v <= pos) lo += step;
        }
        doc = dcur + lo;
        de = shfl64(e, lo);
        const int64_t prev = shfl64(e, lo > 0 ? lo - 1 : 0);
        ds = lo > 0 ? prev : A.offsets[dcur];
        dnext = dcur + __popcll(__ballot(e <= tb + 64));
      } else {
        // More than 63 documents end inside the tile (empty documents):
        // search the whole offsets array.
        doc = upper_bound_i64(A.offsets, n_docs + 1, pos) - 1;
        if (doc > n_docs - 1) doc = n_docs - 1;
        ds = A.offsets[doc];
        de = A.offsets[doc + 1];
        dnext = upper_bound_i64(A.offsets, n_docs + 1, tb + 64) - 1;
        if (dnext > n_docs) dnext = n_docs;
      }
      const int64_t L = de - ds;
      valid = in_range && pos >= ds && pos < de && L > 0 && ((L >= w) ? (pos <= de - w) : (pos == ds));
    }
    const int64_t L = de - ds;
    uint32_t x = 0;
    if (valid) {
      const uint32_t *tp = A.tokens + pos + (A.tok_shift ? A.tok_shift[doc] : 0);
      if (WFIX && L >= w)
        x = shingle_hash_fixed<(WFIX ? WFIX : 1)>(tp);
      else
        x = shingle_hash_var(tp, (uint32_t)(L >= w ? w : L));
    }
    if (inside_doc) {
      full_tile(dcur, x);
      continue;
    }
    const int32_t drel = (int32_t)(doc - dcur);

    uint64_t vm = __ballot(valid);
    // Full tile found by the search: 64 shingles of one document (documents
    // ascend with the lane, so the first and last lane decide).
    if (vm == ~0ull && __builtin_amdgcn_readlane(drel, 0) == __builtin_amdgcn_readlane(drel, 63)) {
      full_tile(dcur + __builtin_amdgcn_readlane(drel, 0), x);
      vm = 0;
    }
    while (vm) {
      const int s = __ffsll((unsigned long long)vm) - 1;
      const int32_t dr = __builtin_amdgcn_readlane(drel, s);
      const int64_t d = dcur + dr;
      if (d != cur) {
        if (cur >= 0) flush(cur);
        cur = d;
      }
      const uint64_t seg = __ballot(valid && drel == dr);
      vm &= ~seg;
      uint64_t sm = seg;
      while (sm) {
        // Two shingles per iteration (the second repeats the first when the
        // segment has an odd count: min is idempotent), so that the running
        // minimum takes one v_min3 per permutation for two evaluations.
        const int s0 = __ffsll((unsigned long long)sm) - 1;
        sm &= sm - 1;
        const int s1 = sm ? __ffsll((unsigned long long)sm) - 1 : s0;
        sm &= sm - 1;
        const uint32_t x0 = __builtin_amdgcn_readlane(x, s0);
        const uint32_t x1 = __builtin_amdgcn_readlane(x, s1);
        if constexpr (WIDE) {
          // the canonical value: R < 2p needs one conditional subtraction,
          // taken only when some lane's flag says R may be >= p
          uint64_t c0[PPL], c1[PPL];
          uint32_t fmax = 0;
#pragma unroll
          for (int p = 0; p < PPL; ++p) {
            uint32_t f0, f1;
            c0[p] = perm_r_flagged(x0, al[p], ah[p], bl[p], bh[p], f0);
            c1[p] = perm_r_flagged(x1, al[p], ah[p], bl[p], bh[p], f1);
            fmax = max(max(fmax, f0), f1);
          }
          if (__ballot(fmax >= kPermFlag)) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
              c0[p] = c0[p] >= kP61 ? c0[p] - kP61 : c0[p];
              c1[p] = c1[p] >= kP61 ? c1[p] - kP61 : c1[p];
            }
          }
#pragma unroll
          for (int p = 0; p < PPL; ++p) mn[p] = min(mn[p], min(c0[p], c1[p]));
          continue;
        }
        // 32-bit values: the low words of the Mersenne-folded R without the
        // canonical correction, and one flag word per evaluation whose
        // maximum is tested once per two shingles.  A flag at or above
        // kPermFlag (about 2^-28 per evaluation, a superset of R >= p) sends
        // the wave through the exact form for these evaluations.
        uint32_t v0[PPL], v1[PPL];
        uint32_t fmax = 0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          uint32_t f0, f1;
          v0[p] = perm_lo32_flagged(x0, al[p], ah[p], bl[p], bh[p], f0);
          v1[p] = perm_lo32_flagged(x1, al[p], ah[p], bl[p], bh[p], f1);
          fmax = max(fmax, max(f0, f1));
        }
        if (__ballot(fmax >= kPermFlag)) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) {
            v0[p] = perm_lo32(x0, al[p], ah[p] >> 3, bl[p], bh[p] >> 3);
            v1[p] = perm_lo32(x1, al[p], ah[p] >> 3, bl[p], bh[p] >> 3);
          }
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) mn[p] = min(mn[p], (V)min(v0[p], v1[p]));
      }
    }
    dcur = dnext;
  }
  if (cur >= 0) flush(cur);
}

// Set bits of a band's words; one block per (range of words, band).
__global__ __launch_bounds__(kBlock) void k_popcount(const uint64_t *words, uint64_t words_per_band,
                                                     uint64_t per_block, uint64_t *out) {
  __shared__ unsigned long long part[kBlock / 64];
  const uint64_t *W = words + (uint64_t)blockIdx.y * words_per_band;
  const uint64_t w0 = (uint64_t)blockIdx.x * per_block;
  const uint64_t w1 = min(words_per_band, w0 + per_block);
  unsigned long long c = 0;
  for (uint64_t w = w0 + threadIdx.x; w < w1; w += kBlock) c += __popcll(W[w]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < kBlock / 64; ++q) t += part[q];
    atomicAdd((unsigned long long *)&out[blockIdx.y], t);
  }
}

__device__ __forceinline__ uint64_t table_slot(uint64_t key, uint64_t mask) {
  return fmix64(key * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull) & mask;
}

__global__ __launch_bounds__(kBlock) void k_band_keys61(BloomLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  A.keys[t] = band_key61(A.sigs64 + i * (int64_t)A.num_perm + (int64_t)j * A.rows, A.rows, A.salt_m);
}

__global__ __launch_bounds__(kBlock) void k_band_keys(BloomLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  A.keys[t] = band_key(A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows, A.rows, A.salt_m);
}

constexpr int kProbeBatch = 8;

__global__ __launch_bounds__(kBlock) void k_qi_probe(BloomLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  const uint64_t K = A.keys_in ? A.keys_in[t]
                              : band_key(A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows, A.rows, A.salt_m);
  A.keys[t] = K;
  const uint64_t h1 = fmix64(K ^ A.salt1);
  const uint64_t h2 = fmix64(K ^ A.salt2) | 1ull;
  const uint64_t *F = A.filters + (uint64_t)j * A.words_per_band;
  uint64_t mask = 0;
  for (uint32_t l0 = 0; l0 < A.k; l0 += kProbeBatch) {
    uint64_t g[kProbeBatch], word[kProbeBatch];
#pragma unroll
    for (int u = 0; u < kProbeBatch; ++u) {
      const uint32_t l = l0 + u;
      g[u] = umulhi64(h1 + (uint64_t)l * h2, A.m_bits);
      word[u] = (l < A.k) ? F[g[u] >> 6] : ~0ull;
    }
#pragma unroll
    for (int u = 0; u < kProbeBatch; ++u) {
      const uint32_t l = l0 + u;
      if (l >= A.k) break;
      if ((word[u] >> (g[u] & 63)) & 1ull) {
        mask |= 1ull << l;
      } else {
        const uint64_t key = ((uint64_t)j << 40) | g[u];
        const uint64_t ent = (key << kIdxBits) | (uint64_t)i;
        uint64_t s = table_slot(key, A.table_mask);
        for (uint64_t tries = 0; tries <= A.table_mask; ++tries) {
          const uint64_t old = atomicCAS((unsigned long long *)&A.table[s], (unsigned long long)kTableEmpty,
                                         (unsigned long long)ent);
          if (old == kTableEmpty) break;
          if ((old >> kIdxBits) == key) {
            if ((old & kMaxChunkDocs) > (uint64_t)i) atomicMin((unsigned long long *)&A.table[s], (unsigned long long)ent);
            break;
          }
          s = (s + 1) & A.table_mask;
        }
      }
    }
  }
  A.masks[t] = mask;
}

__global__ __launch_bounds__(kBlock) void k_qi_resolve(BloomLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  const uint64_t K = A.keys[t];
  const uint64_t mask = A.masks[t];
  const uint64_t h1 = fmix64(K ^ A.salt1);
  const uint64_t h2 = fmix64(K ^ A.salt2) | 1ull;
  uint64_t *F = A.filters + (uint64_t)j * A.words_per_band;
  bool hit = true;
  for (uint32_t l = 0; l < A.k; ++l) {
    if ((mask >> l) & 1ull) continue;
    const uint64_t g = umulhi64(h1 + (uint64_t)l * h2, A.m_bits);
    const uint64_t key = ((uint64_t)j << 40) | g;
    uint64_t s = table_slot(key, A.table_mask);
    uint64_t ent = kTableEmpty;
    for (uint64_t tries = 0; tries <= A.table_mask; ++tries) {
      ent = A.table[s];
      if (ent == kTableEmpty || (ent >> kIdxBits) == key) break;
      s = (s + 1) & A.table_mask;
    }
    if (ent == kTableEmpty || (ent >> kIdxBits) != key) {
      atomicOr(A.status, 1u);  // every clear bit was registered by k_qi_probe
      hit = false;
      continue;
    }
    const uint64_t fs = ent & kMaxChunkDocs;
    if (fs >= (uint64_t)i) hit = false;
    if (fs == (uint64_t)i) atomicOr((unsigned long long *)&F[g >> 6], (unsigned long long)(1ull << (g & 63)));
  }
  A.hitb[t] = hit ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_qi_flags(BloomLaunch A) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= A.n) return;
  const uint8_t *hb = A.hitb + i * (int64_t)A.bands;
  uint8_t f = 0;
  for (uint32_t j = 0; j < A.bands; ++j) f |= hb[j];
  A.flags[i] = f;
}

__global__ __launch_bounds__(kBlock) void k_query(BloomLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  const uint64_t K = band_key(A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows, A.rows, A.salt_m);
  const uint64_t h1 = fmix64(K ^ A.salt1);
  const uint64_t h2 = fmix64(K ^ A.salt2) | 1ull;
  const uint64_t *F = A.filters + (uint64_t)j * A.words_per_band;
  bool hit = true;
  for (uint32_t l = 0; l < A.k && hit; ++l) {
    const uint64_t g = umulhi64(h1 + (uint64_t)l * h2, A.m_bits);
    if (!((F[g >> 6] >> (g & 63)) & 1ull)) hit = false;
  }
  A.hitb[t] = hit ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_insert(BloomLaunch A) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= A.n * (int64_t)A.bands) return;
  const int64_t i = t / A.bands;
  const uint32_t j = (uint32_t)(t - i * A.bands);
  const uint64_t K = band_key(A.sigs + i * (int64_t)A.num_perm + (int64_t)j * A.rows, A.rows, A.salt_m);
  const uint64_t h1 = fmix64(K ^ A.salt1);
  const uint64_t h2 = fmix64(K ^ A.salt2) | 1ull;
  uint64_t *F = A.filters + (uint64_t)j * A.words_per_band;
  for (uint32_t l = 0; l < A.k; ++l) {
    const uint64_t g = umulhi64(h1 + (uint64_t)l * h2, A.m_bits);
    atomicOr((unsigned long long *)&F[g >> 6], (unsigned long long)(1ull << (g & 63)));
  }
}

inline unsigned grid_for(uint64_t n) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  return (unsigned)(g == 0 ? 1 : g);
}

inline unsigned fill_grid(uint64_t n) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  return (unsigned)(g == 0 ? 1 : g);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_popcount(const uint64_t *words, uint64_t words_per_band, uint32_t bands, uint64_t *out,
                           hipStream_t s) {
  if (bands == 0 || words_per_band == 0) return hipSuccess;
  const uint64_t per_block = 64 * 1024;  // words per block
  const uint64_t gx = (words_per_band + per_block - 1) / per_block;
  hipLaunchKernelGGL(k_popcount, dim3((unsigned)gx, bands), dim3(kBlock), 0, s, words, words_per_band, per_block, out);
  return hipGetLastError();
}

hipError_t launch_minhash(const MinhashLaunch &a, hipStream_t s) {
  const unsigned blocks = (unsigned)(a.waves / (kBlock / 64));
  const int ppl = (int)((a.num_perm + 63) / 64);
  const bool w5 = a.w == 5;
  const bool wide = a.sigs64 != nullptr;
#define LB_MH(PPL_)                                                                              \
  do {                                                                                           \
    if (wide) {                                                                                  \
      if (w5)                                                                                    \
        hipLaunchKernelGGL((k_minhash<PPL_, 5, true>), dim3(blocks), dim3(kBlock), 0, s, a);     \
      else                                                                                       \
        hipLaunchKernelGGL((k_minhash<PPL_, 0, true>), dim3(blocks), dim3(kBlock), 0, s, a);     \
    } else if (w5) {                                                                             \
      hipLaunchKernelGGL((k_minhash<PPL_, 5, false>), dim3(blocks), dim3(kBlock), 0, s, a);      \
    } else {                                                                                     \
      hipLaunchKernelGGL((k_minhash<PPL_, 0, false>), dim3(blocks), dim3(kBlock), 0, s, a);      \
    }                                                                                            \
  } while (0)
  if (ppl <= 1)
    LB_MH(1);
  else if (ppl <= 2)
    LB_MH(2);
  else if (ppl <= 4)
    LB_MH(4);
  else
    LB_MH(8);
#undef LB_MH
  return hipGetLastError();
}

hipError_t launch_band_keys(const BloomLaunch &a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n * a.bands;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_band_keys61(const BloomLaunch &a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n * a.bands;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_keys61, dim3(grid_for(n)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_query_insert_chunk(const BloomLaunch &a, uint64_t table_slots, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n * a.bands;
  if (n == 0) return hipSuccess;
  hipError_t e = launch_fill_u64(a.table, table_slots, kTableEmpty, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_qi_probe, dim3(grid_for(n)), dim3(kBlock), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_qi_resolve, dim3(grid_for(n)), dim3(kBlock), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_qi_flags, dim3(grid_for((uint64_t)a.n)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_query(const BloomLaunch &a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n * a.bands;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_query, dim3(grid_for(n)), dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_qi_flags, dim3(grid_for((uint64_t)a.n)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_insert(const BloomLaunch &a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n * a.bands;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_insert, dim3(grid_for(n)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace lb
