// Integer building blocks of the LSHBloom hot path, written for gfx950 VALU.
//
// Everything here is exact integer arithmetic; the functions are also
// compiled for the host by the unit tests that check them exhaustively
// against big-integer definitions.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define LB_FN __host__ __device__ __forceinline__
#else
#define LB_FN static inline
#endif

namespace lb {

// 2^61 - 1, the Mersenne prime modulus of the MinHash permutations.
constexpr uint64_t kP61 = 0x1FFFFFFFFFFFFFFFull;

LB_FN uint32_t rotl32(uint32_t x, int n) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_alignbit(x, x, 32 - n);
#else
  return (x << n) | (x >> (32 - n));
#endif
}

LB_FN uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// SplitMix64 output finalizer (Steele, Lea & Flood 2014).
LB_FN uint64_t fmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// High 64 bits of the 128-bit product x * y.
LB_FN uint64_t umulhi64(uint64_t x, uint64_t y) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(x, y);
#else
  return (uint64_t)(((unsigned __int128)x * y) >> 64);
#endif
}

// Low 32 bits of ((a * x + b) mod (2^61 - 1)) for a, b < 2^61 - 1 and a
// 32-bit x, given a = a_hi * 2^32 + a_lo and b = b_hi * 2^32 + b_lo.
//
//   P = a_lo * x + b_lo                         < 2^64   (one v_mad_u64_u32)
//   Q = a_hi * x + b_hi + (P >> 32)              < 2^62   (one v_mad_u64_u32)
//   a*x + b = Q * 2^32 + (P mod 2^32)
// Since 2^61 = 1 (mod p), Q * 2^32 = (Q >> 29) + (Q mod 2^29) * 2^32, so
//   R = (Q mod 2^29) * 2^32 + (P mod 2^32) + (Q >> 29)   < 2^61 + 2^33 < 2p
// is congruent to a*x + b and one conditional subtraction of p makes it
// canonical.  R >= p exactly when R + 1 >= 2^61, and R - p has the low word
// of R plus one (2^61 has a zero low word), so the result is
//   low32(R) + ((R + 1) >> 61).
LB_FN uint32_t perm_lo32(uint32_t x, uint32_t a_lo, uint32_t a_hi, uint32_t b_lo, uint32_t b_hi) {
  const uint64_t P = (uint64_t)a_lo * x + b_lo;
  const uint64_t Q = (uint64_t)a_hi * x + ((P >> 32) + b_hi);
  const uint64_t R = ((Q & 0x1FFFFFFFull) << 32) + (uint32_t)P + (Q >> 29);
  return (uint32_t)R + (uint32_t)((R + 1) >> 61);
}

// SHA-1 (FIPS 180-4 §6.1.2) of one already-padded 64-byte block given as 16
// big-endian words, from the standard initial state; returns the first four
// digest bytes read as a little-endian uint32, i.e. bswap(H0).
LB_FN uint32_t sha1_block_h0_le(uint32_t W[16]) {
  uint32_t a = 0x67452301u, b = 0xEFCDAB89u, c = 0x98BADCFEu, d = 0x10325476u, e = 0xC3D2E1F0u;
#pragma unroll
  for (int t = 0; t < 80; ++t) {
    uint32_t wt;
    if (t < 16) {
      wt = W[t];
    } else {
      wt = rotl32(W[(t - 3) & 15] ^ W[(t - 8) & 15] ^ W[(t - 14) & 15] ^ W[t & 15], 1);
      W[t & 15] = wt;
    }
    uint32_t f, K;
    if (t < 20) {
      f = d ^ (b & (c ^ d));
      K = 0x5A827999u;
    } else if (t < 40) {
      f = b ^ c ^ d;
      K = 0x6ED9EBA1u;
    } else if (t < 60) {
      f = (b & c) | (d & (b | c));
      K = 0x8F1BBCDCu;
    } else {
      f = b ^ c ^ d;
      K = 0xCA62C1D6u;
    }
    const uint32_t T = rotl32(a, 5) + f + e + K + wt;
    e = d;
    d = c;
    c = rotl32(b, 30);
    b = a;
    a = T;
  }
  return bswap32(0x67452301u + a);
}

// Shingle hash of `len` (1..13) tokens: SHA-1 over their little-endian bytes.
// The message is 4*len bytes, so the padded block is: the tokens as
// big-endian words (byte-swapped), the 0x80 terminator word, zeros, and the
// bit length 32*len in the last word.
template <int LEN>
LB_FN uint32_t shingle_hash_fixed(const uint32_t *tok) {
  uint32_t W[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) W[i] = 0;
#pragma unroll
  for (int i = 0; i < LEN; ++i) W[i] = bswap32(tok[i]);
  W[LEN] = 0x80000000u;
  W[15] = 32u * LEN;
  return sha1_block_h0_le(W);
}

LB_FN uint32_t shingle_hash_var(const uint32_t *tok, uint32_t len) {
  uint32_t W[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    uint32_t v = 0;
    if ((uint32_t)i < len) v = bswap32(tok[i]);
    if ((uint32_t)i == len) v = 0x80000000u;
    W[i] = v;
  }
  W[15] = 32u * len;
  return sha1_block_h0_le(W);
}

// Band key of one band: sum over its r rows of fmix64((v | t << 32) ^ salt).
LB_FN uint64_t band_key(const uint32_t *row0, uint32_t rows, uint64_t salt_m) {
  uint64_t K = 0;
  for (uint32_t t = 0; t < rows; ++t) K += fmix64(((uint64_t)row0[t] | ((uint64_t)t << 32)) ^ salt_m);
  return K;
}

}  // namespace lb
