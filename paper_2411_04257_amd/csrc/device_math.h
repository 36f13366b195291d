// Integer building blocks of the LSHBloom hot path, written for gfx950 VALU.
//
// Everything here is exact integer arithmetic; the functions are also
// compiled for the host by the unit tests that check them exhaustively
// against big-integer definitions.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define LB_FN __host__ __device__ __forceinline__
#define LB_MEMBER __host__ __device__ __forceinline__
#else
#define LB_FN static inline
#define LB_MEMBER inline
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
// With a_hi, b_hi <= 2^29 - 1 and P >> 32 <= 2^32 - 1, Q <= 2^61 - 1, so in
// fact Q >> 29 < 2^32 and R < 2^61 + 2^32.
LB_FN uint64_t perm_r(uint32_t x, uint32_t a_lo, uint32_t a_hi, uint32_t b_lo, uint32_t b_hi) {
  const uint64_t P = (uint64_t)a_lo * x + b_lo;
  const uint64_t Q = (uint64_t)a_hi * x + b_hi + (P >> 32);
  // (Q mod 2^29) * 2^32 and P mod 2^32 occupy disjoint bits: one register pair.
  uint64_t pair = ((Q & 0x1FFFFFFFull) << 32) | (uint32_t)P;
#if defined(__HIP_DEVICE_COMPILE__)
  // Keep the pair as one 64-bit register value: without this barrier the
  // compiler re-associates the sum into two 64-bit adds and extra moves.
  asm("" : "+v"(pair));
#endif
  return pair + (Q >> 29);
}

LB_FN uint32_t perm_lo32(uint32_t x, uint32_t a_lo, uint32_t a_hi, uint32_t b_lo, uint32_t b_hi) {
  const uint64_t R = perm_r(x, a_lo, a_hi, b_lo, b_hi);
  return (uint32_t)R + (uint32_t)((R + 1) >> 61);
}

// The low word of R above, in three 32x32+64 multiply-adds, plus a word that
// flags the rare R >= p.  The high coefficient words come times 8
// (a_hi8 = 8 a_hi, b_hi8 = 8 b_hi, both below 2^32 as a_hi, b_hi < 2^29):
//   S = a_hi8 * x + b_hi8 + 8 * (P >> 32) = 8 Q   (< 2^64 as Q < 2^61),
// so S >> 32 = Q >> 29 and low32(S) = 8 (Q mod 2^29), and
//   low32(R) = low32(P) + (S >> 32).
// R >= p needs Q mod 2^29 >= 2^29 - 2, i.e. flag = low32(S) >= 2^32 - 16:
// otherwise R <= (2^29 - 3) 2^32 + 2 (2^32 - 1) < 2^61 - 1.  A caller that
// finds no flag at or above kPermFlag has the canonical low words; otherwise
// it recomputes with perm_lo32 (about 2^-28 of evaluations).
constexpr uint32_t kPermFlag = 0xFFFFFFF0u;

LB_FN uint32_t perm_lo32_flagged(uint32_t x, uint32_t a_lo, uint32_t a_hi8, uint32_t b_lo, uint32_t b_hi8,
                                 uint32_t &flag) {
  const uint64_t P = (uint64_t)a_lo * x + b_lo;
  uint32_t eight = 8;
#if defined(__HIP_DEVICE_COMPILE__)
  // An opaque 8 in a scalar register: the product below then stays one
  // v_mad_u64_u32 that reads the high word of P in place, where a constant
  // would become a 64-bit shift of a register pair built by an extra move.
  asm("" : "+s"(eight));
#endif
  const uint64_t S = (uint64_t)(uint32_t)(P >> 32) * eight + ((uint64_t)a_hi8 * x + b_hi8);
  flag = (uint32_t)S;
  return (uint32_t)P + (uint32_t)(S >> 32);
}

// The whole folded R of perm_r (not yet reduced below p) from the same three
// multiply-adds: Q mod 2^29 = low32(S) >> 3 and Q >> 29 = S >> 32, so
//   R = (low32(S) >> 3) * 2^32 + low32(P) + (S >> 32),
// with the same flag word: no flag at or above kPermFlag means R < p.
LB_FN uint64_t perm_r_flagged(uint32_t x, uint32_t a_lo, uint32_t a_hi8, uint32_t b_lo, uint32_t b_hi8,
                              uint32_t &flag) {
  const uint64_t P = (uint64_t)a_lo * x + b_lo;
  uint32_t eight = 8;
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+s"(eight));  // as in perm_lo32_flagged
#endif
  const uint64_t S = (uint64_t)(uint32_t)(P >> 32) * eight + ((uint64_t)a_hi8 * x + b_hi8);
  flag = (uint32_t)S;
  // two 32-bit halves with one carry, not a 64-bit sum of register pairs
  const uint32_t s_hi = (uint32_t)(S >> 32);
  const uint32_t r_lo = (uint32_t)P + s_hi;
  const uint32_t r_hi = ((uint32_t)S >> 3) + (r_lo < s_hi ? 1u : 0u);
  return ((uint64_t)r_hi << 32) | r_lo;
}

// Three-input bitwise functions of SHA-1 (FIPS 180-4 §4.1.1).  On gfx950 each
// is one v_bitop3_b32 (truth tables 0x96 = x^y^z, 0xE8 = majority; both are
// symmetric, so the operand order does not matter).
LB_FN uint32_t xor3(uint32_t x, uint32_t y, uint32_t z) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(x, y, z, 0x96);
#else
  return x ^ y ^ z;
#endif
}

LB_FN uint32_t maj3(uint32_t x, uint32_t y, uint32_t z) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(x, y, z, 0xE8);
#else
  return (x & y) | (z & (x | y));
#endif
}

LB_FN uint32_t ch3(uint32_t x, uint32_t y, uint32_t z) { return z ^ (x & (y ^ z)); }  // v_bfi_b32

// One SHA-1 round t (FIPS 180-4 §6.1.2 step 3) with message word wt.
template <int T>
LB_FN void sha1_round(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d, uint32_t &e, uint32_t wt) {
  uint32_t f, K;
  if constexpr (T < 20) {
    f = ch3(b, c, d);
    K = 0x5A827999u;
  } else if constexpr (T < 40) {
    f = xor3(b, c, d);
    K = 0x6ED9EBA1u;
  } else if constexpr (T < 60) {
    f = maj3(b, c, d);
    K = 0x8F1BBCDCu;
  } else {
    f = xor3(b, c, d);
    K = 0xCA62C1D6u;
  }
  const uint32_t tmp = rotl32(a, 5) + f + e + (K + wt);
  e = d;
  d = c;
  c = rotl32(b, 30);
  b = a;
  a = tmp;
}

// SHA-1 of one padded block whose words LEN..15 are the padding of a
// 4*LEN-byte message (0x80000000, zeros, bit length 32*LEN), unrolled at
// compile time so that schedule terms that are padding constants fold away
// (W_t = rotl1(W_{t-3} ^ W_{t-8} ^ W_{t-14} ^ W_{t-16}), §6.1.2 step 1).
template <int LEN>
struct Sha1Fixed {
  static constexpr bool is_pad(int i) { return i >= LEN && i < 16; }
  static constexpr uint32_t pad(int i) { return i == LEN ? 0x80000000u : (i == 15 ? 32u * LEN : 0u); }

  // Message word t: W holds the 16-word ring (initial words 0..LEN-1, then
  // computed words), written back for t >= 16.
  template <int T>
  static LB_MEMBER uint32_t word(uint32_t (&W)[16]) {
    if constexpr (T < 16) {
      if constexpr (is_pad(T)) return pad(T);
      else return W[T];
    } else {
      constexpr int i0 = T - 3, i1 = T - 8, i2 = T - 14, i3 = T - 16;
      // constant part of the XOR and the variable terms
      constexpr uint32_t cst = (i0 < 16 && is_pad(i0) ? pad(i0) : 0u) ^ (i1 < 16 && is_pad(i1) ? pad(i1) : 0u) ^
                               (i2 < 16 && is_pad(i2) ? pad(i2) : 0u) ^ (i3 < 16 && is_pad(i3) ? pad(i3) : 0u);
      constexpr bool v0 = !(i0 < 16 && is_pad(i0)), v1 = !(i1 < 16 && is_pad(i1));
      constexpr bool v2 = !(i2 < 16 && is_pad(i2)), v3 = !(i3 < 16 && is_pad(i3));
      constexpr int nv = (int)v0 + (int)v1 + (int)v2 + (int)v3;
      uint32_t t[4];
      int k = 0;
      if constexpr (v0) t[k++] = W[i0 & 15];
      if constexpr (v1) t[k++] = W[i1 & 15];
      if constexpr (v2) t[k++] = W[i2 & 15];
      if constexpr (v3) t[k++] = W[i3 & 15];
      uint32_t x;
      if constexpr (nv == 4) {
        x = xor3(t[0], t[1], t[2]) ^ t[3];
        if constexpr (cst != 0u) x ^= cst;
      } else if constexpr (nv == 3) {
        x = (cst != 0u) ? (xor3(t[0], t[1], t[2]) ^ cst) : xor3(t[0], t[1], t[2]);
      } else if constexpr (nv == 2) {
        x = (cst != 0u) ? xor3(t[0], t[1], cst) : (t[0] ^ t[1]);
      } else if constexpr (nv == 1) {
        x = t[0] ^ cst;
      } else {
        x = cst;
      }
      const uint32_t w = rotl32(x, 1);
      W[T & 15] = w;
      return w;
    }
  }

  template <int T>
  static LB_MEMBER void rounds(uint32_t (&W)[16], uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d, uint32_t &e) {
    if constexpr (T < 80) {
      const uint32_t wt = word<T>(W);
      sha1_round<T>(a, b, c, d, e, wt);
      rounds<T + 1>(W, a, b, c, d, e);
    }
  }

  // First four digest bytes read as a little-endian uint32, i.e. bswap(H0).
  static LB_MEMBER uint32_t h0_le(uint32_t (&W)[16]) {
    uint32_t a = 0x67452301u, b = 0xEFCDAB89u, c = 0x98BADCFEu, d = 0x10325476u, e = 0xC3D2E1F0u;
    rounds<0>(W, a, b, c, d, e);
    return bswap32(0x67452301u + a);
  }
};

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
      wt = rotl32(xor3(W[(t - 3) & 15], W[(t - 8) & 15], W[(t - 14) & 15]) ^ W[t & 15], 1);
      W[t & 15] = wt;
    }
    uint32_t f, K;
    if (t < 20) {
      f = ch3(b, c, d);
      K = 0x5A827999u;
    } else if (t < 40) {
      f = xor3(b, c, d);
      K = 0x6ED9EBA1u;
    } else if (t < 60) {
      f = maj3(b, c, d);
      K = 0x8F1BBCDCu;
    } else {
      f = xor3(b, c, d);
      K = 0xCA62C1D6u;
    }
    const uint32_t T = rotl32(a, 5) + f + e + (K + wt);
    e = d;
    d = c;
    c = rotl32(b, 30);
    b = a;
    a = T;
  }
  return bswap32(0x67452301u + a);
}

// Shingle hash of LEN (1..13) tokens: SHA-1 over their little-endian bytes.
// The message is 4*LEN bytes, so the padded block is: the tokens as
// big-endian words (byte-swapped), the 0x80 terminator word, zeros, and the
// bit length 32*LEN in the last word.
template <int LEN>
LB_FN uint32_t shingle_hash_fixed(const uint32_t *tok) {
  uint32_t W[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) W[i] = 0;
#pragma unroll
  for (int i = 0; i < LEN; ++i) W[i] = bswap32(tok[i]);
  return Sha1Fixed<LEN>::h0_le(W);
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

// Band key of one band of wide (61-bit) values: sum over its r rows of
// fmix64((v + t * 0x9E3779B97F4A7C15) ^ salt); the row enters as an offset
// since the value fills the word.
LB_FN uint64_t band_key61(const uint64_t *row0, uint32_t rows, uint64_t salt_m) {
  uint64_t K = 0;
  for (uint32_t t = 0; t < rows; ++t) K += fmix64((row0[t] + (uint64_t)t * 0x9E3779B97F4A7C15ull) ^ salt_m);
  return K;
}

// Band key of one band: sum over its r rows of fmix64((v | t << 32) ^ salt).
LB_FN uint64_t band_key(const uint32_t *row0, uint32_t rows, uint64_t salt_m) {
  uint64_t K = 0;
  for (uint32_t t = 0; t < rows; ++t) K += fmix64(((uint64_t)row0[t] | ((uint64_t)t << 32)) ^ salt_m);
  return K;
}

}  // namespace lb
