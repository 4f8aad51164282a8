// keccak_dev.hpp -- Keccak-f[1600] and the SHAKE256 tweakable hashes of the
// SHAKE parameter sets (FIPS 202; FIPS 205 Section 11.1) for gfx950.
//
// A 64-bit lane is held as two 32-bit halves; a rotate is two v_alignbit_b32
// (a swap of the halves for 32), the three-input XORs of theta and the
// a ^ (~b & c) of chi are each one v_bitop3_b32 per half.  Byte i of the
// sponge is byte i % 8 of lane i / 8, little-endian, while the library keeps
// values as big-endian 32-bit words: a word enters or leaves the state with
// one byte swap.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sha2_dev.hpp"

// Included by slh_dev.hpp after struct Adrs.

namespace slh {

struct KLane {
  uint32_t lo, hi;
};

template <int R>
__device__ __forceinline__ KLane krotl(KLane x) {
  if constexpr (R == 0) {
    return x;
  } else if constexpr (R < 32) {
    return KLane{__builtin_amdgcn_alignbit(x.lo, x.hi, 32 - R), __builtin_amdgcn_alignbit(x.hi, x.lo, 32 - R)};
  } else if constexpr (R == 32) {
    return KLane{x.hi, x.lo};
  } else {
    return KLane{__builtin_amdgcn_alignbit(x.hi, x.lo, 64 - R), __builtin_amdgcn_alignbit(x.lo, x.hi, 64 - R)};
  }
}
__device__ __forceinline__ KLane kxor3(KLane a, KLane b, KLane c) {
  return KLane{xor3(a.lo, b.lo, c.lo), xor3(a.hi, b.hi, c.hi)};
}
// a ^ (~b & c): truth table 0xD2 for index (a << 2) | (b << 1) | c
__device__ __forceinline__ KLane kchi(KLane a, KLane b, KLane c) {
  return KLane{uint32_t(__builtin_amdgcn_bitop3_b32(a.lo, b.lo, c.lo, 0xD2)),
               uint32_t(__builtin_amdgcn_bitop3_b32(a.hi, b.hi, c.hi, 0xD2))};
}

// Round constants RC[ir] of FIPS 202 Algorithm 6 (iota), as derived from
// the rc(t) LFSR of Algorithm 5; the rho offsets of Algorithm 2 are in
// keccak_round.
static __constant__ uint64_t kKeccakRC[24] = {
    0x0000000000000001ull, 0x0000000000008082ull, 0x800000000000808aull, 0x8000000080008000ull,
    0x000000000000808bull, 0x0000000080000001ull, 0x8000000080008081ull, 0x8000000000008009ull,
    0x000000000000008aull, 0x0000000000000088ull, 0x0000000080008009ull, 0x000000008000000aull,
    0x000000008000808bull, 0x800000000000008bull, 0x8000000000008089ull, 0x8000000000008003ull,
    0x8000000000008002ull, 0x8000000000000080ull, 0x000000000000800aull, 0x800000008000000aull,
    0x8000000080008081ull, 0x8000000000008080ull, 0x0000000080000001ull, 0x8000000080008008ull};

// One round: theta, rho and pi, chi, iota.  s[x + 5 y].
__device__ __forceinline__ void keccak_round(KLane s[25], uint64_t rc) {
  KLane C[5];
#pragma unroll
  for (int x = 0; x < 5; x++) {
    const KLane t = kxor3(s[x], s[x + 5], s[x + 10]);
    C[x] = kxor3(t, s[x + 15], s[x + 20]);
  }
  KLane D[5];
#pragma unroll
  for (int x = 0; x < 5; x++) D[x] = krotl<1>(C[(x + 1) % 5]);
  // rho offsets r[x + 5 y] (Algorithm 2) and pi: B[y + 5 ((2x + 3y) mod 5)] = rotl(A[x + 5y], r)
  KLane B[25];
#define SLH_KRP(x, y, r)                                                                          \
  B[(y) + 5 * ((2 * (x) + 3 * (y)) % 5)] = krotl<r>(kxor3(s[(x) + 5 * (y)], C[((x) + 4) % 5], D[x]));
  SLH_KRP(0, 0, 0) SLH_KRP(1, 0, 1) SLH_KRP(2, 0, 62) SLH_KRP(3, 0, 28) SLH_KRP(4, 0, 27)
  SLH_KRP(0, 1, 36) SLH_KRP(1, 1, 44) SLH_KRP(2, 1, 6) SLH_KRP(3, 1, 55) SLH_KRP(4, 1, 20)
  SLH_KRP(0, 2, 3) SLH_KRP(1, 2, 10) SLH_KRP(2, 2, 43) SLH_KRP(3, 2, 25) SLH_KRP(4, 2, 39)
  SLH_KRP(0, 3, 41) SLH_KRP(1, 3, 45) SLH_KRP(2, 3, 15) SLH_KRP(3, 3, 21) SLH_KRP(4, 3, 8)
  SLH_KRP(0, 4, 18) SLH_KRP(1, 4, 2) SLH_KRP(2, 4, 61) SLH_KRP(3, 4, 56) SLH_KRP(4, 4, 14)
#undef SLH_KRP
#pragma unroll
  for (int y = 0; y < 5; y++)
#pragma unroll
    for (int x = 0; x < 5; x++) s[x + 5 * y] = kchi(B[x + 5 * y], B[(x + 1) % 5 + 5 * y], B[(x + 2) % 5 + 5 * y]);
  s[0].lo ^= uint32_t(rc);
  s[0].hi ^= uint32_t(rc >> 32);
}

// Rounds 0 and 23 stand outside the loop: once a caller's absorb and
// squeeze are inlined around them, the zero and constant lanes of round 0
// fold away and round 23 computes only the lanes the caller reads.
__device__ __forceinline__ void keccak_f1600(KLane s[25]) {
  keccak_round(s, 0x0000000000000001ull);  // RC[0]
#pragma unroll 1
  for (int ir = 1; ir < 23; ir += 2) {
    keccak_round(s, kKeccakRC[ir]);
    keccak_round(s, kKeccakRC[ir + 1]);
  }
  keccak_round(s, 0x8000000080008008ull);  // RC[23]
}

// XOR big-endian message word q of a block into the state.
__device__ __forceinline__ void kabsorb_word(KLane s[25], int q, uint32_t w) {
  if (q & 1) s[q >> 1].hi ^= __builtin_bswap32(w);
  else s[q >> 1].lo ^= __builtin_bswap32(w);
}
// Big-endian output word q of the state.
__device__ __forceinline__ uint32_t ksqueeze_word(const KLane s[25], int q) {
  return __builtin_bswap32((q & 1) ? s[q >> 1].hi : s[q >> 1].lo);
}

constexpr int kShakeRateWords = 34;  // 136 bytes

// The full 32-byte address as big-endian words, from the compressed form
// kept in Adrs: layer(4) | tree(12) | type(4) | word1 | word2 | word3.
__device__ __forceinline__ void adrs_full(const Adrs& A, uint32_t f[8]) {
  f[0] = A.w[0] >> 24;
  f[1] = 0;
  f[2] = __builtin_amdgcn_alignbit(A.w[0], A.w[1], 24);
  f[3] = __builtin_amdgcn_alignbit(A.w[1], A.w[2], 24);
  f[4] = (A.w[2] >> 16) & 0xFFu;
  f[5] = __builtin_amdgcn_alignbit(A.w[2], A.w[3], 16);
  f[6] = __builtin_amdgcn_alignbit(A.w[3], A.w[4], 16);
  f[7] = __builtin_amdgcn_alignbit(A.w[4], A.tail, 16);
}

// SHAKE256(PK.seed | ADRS | x, 4 NOUT bytes) for inputs that fit one block
// (4 (NW + 8 + NX) < 136): PRF, F and H.
template <int NW, int NX, int NOUT>
__device__ __forceinline__ void thshake(const uint32_t* pk_seed, const Adrs& A, const uint32_t* x, uint32_t* out) {
  constexpr int Q = NW + 8 + NX;  // message words
  static_assert(Q < kShakeRateWords, "single block");
  KLane s[25];
#pragma unroll
  for (int i = 0; i < 25; i++) s[i] = KLane{0u, 0u};
  uint32_t f[8];
  adrs_full(A, f);
#pragma unroll
  for (int q = 0; q < NW; q++) kabsorb_word(s, q, pk_seed[q]);
#pragma unroll
  for (int q = 0; q < 8; q++) kabsorb_word(s, NW + q, f[q]);
#pragma unroll
  for (int q = 0; q < NX; q++) kabsorb_word(s, NW + 8 + q, x[q]);
  kabsorb_word(s, Q, 0x1F000000u);                      // domain bits and first pad bit
  kabsorb_word(s, kShakeRateWords - 1, 0x00000080u);    // last pad bit at byte 135
  keccak_f1600(s);
#pragma unroll
  for (int q = 0; q < NOUT; q++) out[q] = ksqueeze_word(s, q);
}

// SHAKE256(PK.seed | ADRS | values, n) over L n-byte values read through
// get(word): T_l of the SHAKE sets.
template <int NW, int L, class Get>
__device__ __forceinline__ void thshake_t(const uint32_t* pk_seed, const Adrs& A, Get get, uint32_t* out) {
  constexpr int Q = NW + 8 + L * NW;  // message words
  constexpr int NBLK = (4 * Q + 1 + 135) / 136;
  constexpr int R = kShakeRateWords;
  static_assert(NBLK >= 2, "T_l spans several blocks");
  uint32_t f[8];
  adrs_full(A, f);
  KLane s[25];
#pragma unroll
  for (int i = 0; i < 25; i++) s[i] = KLane{0u, 0u};
  // block 0: PK.seed, ADRS, then the first values
#pragma unroll
  for (int j = 0; j < R; j++)
    kabsorb_word(s, j, j < NW ? pk_seed[j] : j < NW + 8 ? f[j - NW] : get(j - NW - 8));
  keccak_f1600(s);
  // middle blocks: values only
#pragma unroll 1
  for (int b = 1; b < NBLK - 1; b++) {
    const int base = b * R - NW - 8;
#pragma unroll
    for (int j = 0; j < R; j++) kabsorb_word(s, j, get(base + j));
    keccak_f1600(s);
  }
  // last block: the remaining values and the padding
  constexpr int LB = (NBLK - 1) * R;
#pragma unroll
  for (int j = 0; j < R; j++) {
    const int q = LB + j;
    uint32_t w = q < Q ? get(q - NW - 8) : (q == Q ? 0x1F000000u : 0u);
    if (j == R - 1) w |= 0x00000080u;
    kabsorb_word(s, j, w);
  }
  keccak_f1600(s);
#pragma unroll
  for (int q = 0; q < NW; q++) out[q] = ksqueeze_word(s, q);
}

// Big-endian word of the message portion starting at byte p, with the SHAKE
// domain and first padding byte 0x1F at byte mlen (p >= 0).
__device__ __forceinline__ uint32_t kmsg_word(const uint8_t* msg, uint64_t mlen, int64_t p) {
  uint32_t w = 0;
#pragma unroll
  for (int t = 0; t < 4; t++) {
    const int64_t q = p + t;
    const uint32_t byte = (q < int64_t(mlen)) ? msg[q] : (q == int64_t(mlen) ? 0x1Fu : 0u);
    w = (w << 8) | byte;
  }
  return w;
}

// Byte string prefix (PW BE words) | msg (mlen bytes) absorbed into SHAKE256
// and NOUT BE words squeezed (PRF_msg, H_msg; NOUT <= 34).  A block that lies
// inside the message at a 4-byte aligned address is read as dwords; the
// first block (prefix) and the last (padding) word by word.
template <int PW, int NOUT>
__device__ void shake256_stream(const uint32_t* prefix, const uint8_t* msg, uint64_t mlen, uint32_t* out) {
  static_assert(PW < kShakeRateWords, "prefix fits the first block");
  const uint64_t total = 4 * PW + mlen;
  const uint64_t nblk = (total + 1 + 135) / 136;
  KLane s[25];
#pragma unroll
  for (int i = 0; i < 25; i++) s[i] = KLane{0u, 0u};
  for (uint64_t b = 0; b < nblk; b++) {
    uint32_t w[kShakeRateWords];
    const int64_t p0 = int64_t(b) * 136 - 4 * PW;  // message byte at the block's start
    if (b == 0) {
#pragma unroll
      for (int j = 0; j < kShakeRateWords; j++) w[j] = j < PW ? prefix[j] : kmsg_word(msg, mlen, 4 * j - 4 * PW);
    } else if (uint64_t(p0) + 136 <= mlen && (reinterpret_cast<uintptr_t>(msg + p0) & 3) == 0) {
      const uint32_t* q4 = reinterpret_cast<const uint32_t*>(msg + p0);
#pragma unroll
      for (int j = 0; j < kShakeRateWords; j++) w[j] = __builtin_bswap32(q4[j]);
    } else {
#pragma unroll
      for (int j = 0; j < kShakeRateWords; j++) w[j] = kmsg_word(msg, mlen, p0 + 4 * j);
    }
    if (b == nblk - 1) w[kShakeRateWords - 1] |= 0x00000080u;  // last padding bit at byte 135
#pragma unroll
    for (int j = 0; j < kShakeRateWords; j++) kabsorb_word(s, j, w[j]);
    keccak_f1600(s);
  }
#pragma unroll
  for (int q = 0; q < NOUT; q++) out[q] = ksqueeze_word(s, q);
}

}  // namespace slh
