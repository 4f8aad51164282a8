// sha2_dev.hpp -- register-resident SHA-256 / SHA-512 compression for gfx950.
//
// The paper (Section III-C, "selection of PTX-level instructions") finds SHA-2
// round arithmetic to be the bound of every kernel and tunes its instruction
// selection on NVIDIA hardware.  Here the same arithmetic (FIPS 180-4
// Sections 4.1.2, 4.1.3, 6.2.2, 6.4.2) is written for the CDNA4 vector ALU:
//   - 32-bit rotates are one v_alignbit_b32;
//   - the three-input XORs of the Sigma functions, Ch and Maj are each one
//     v_bitop3_b32 (gfx950 has no v_xor3_b32);
//   - sums of three terms become v_add3_u32.
// Message words are kept as big-endian-interpreted 32-bit words throughout
// the library, so no byte swap occurs inside the hash pipeline at all; the
// swap (v_perm_b32) happens only where bytes enter or leave the library.
//
// All loops are fully unrolled with compile-time indices so that W[] and the
// state stay in VGPRs.  Words of W that are compile-time constants (padding
// zeros, the length word) are folded away by the compiler, and words that do
// not change across the hash steps of one WOTS+ chain are hoisted out of the
// chain loop by the caller's loop structure.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slh {

// ---------------------------------------------------------------- SHA-256
__device__ __forceinline__ uint32_t rotr32(uint32_t x, uint32_t r) {
  return __builtin_amdgcn_alignbit(x, x, r);
}
// v_bitop3_b32 truth-table index is (S0 << 2) | (S1 << 1) | S2.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t ch32(uint32_t e, uint32_t f, uint32_t g) {
  return __builtin_amdgcn_bitop3_b32(e, f, g, 0xCA);  // e ? f : g
}
__device__ __forceinline__ uint32_t maj32(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);  // majority
}

// ---------------------------------------------------------------- variants
// Instruction variants of the SHA-2 arithmetic.  The paper compiles each
// hashing kernel twice, once from native code and once with hand-written
// PTX, profiles both and keeps the faster per kernel (Section III-C,
// "PTX Branch Selection at Kernel-Level", Table 5).  On gfx950 the same
// choice is between instruction forms of the round arithmetic; a kernel
// template takes the variant V and the autotuner picks V per kernel and
// parameter set:
//   V = 0            the library's forms: v_bitop3_b32 for the three-input
//                    XORs, Ch and Maj; v_add3_u32 for three-term sums;
//                    v_lshl_add_u64 for every SHA-512 64-bit add;
//   V & kIsaLogic    no three-input logic op: an XOR of three as two
//                    v_xor_b32, Ch as v_bfi_b32, Maj as v_xor_b32 + v_bfi_b32;
//   V & kIsaAdds     no fused adds: every sum of two run-time values as one
//                    v_add_u32 (no v_add3_u32), every 64-bit add as a
//                    v_add_co_u32 / v_addc_co_u32 carry pair.
// Operations whose operands are compile-time constants after inlining (the
// padding and length words, hoisted address words) fold in every variant,
// so the variants differ only where a kernel computes at run time.
enum : int { kIsaLogic = 1, kIsaAdds = 2 };

template <int V>
__device__ __forceinline__ uint32_t vxor3(uint32_t a, uint32_t b, uint32_t c) {
  if constexpr ((V & kIsaLogic) != 0) {
    if (__builtin_constant_p(a ^ b ^ c)) return a ^ b ^ c;
    uint32_t t, r;
    asm("v_xor_b32 %0, %1, %2" : "=v"(t) : "v"(a), "v"(b));
    asm("v_xor_b32 %0, %1, %2" : "=v"(r) : "v"(t), "v"(c));
    return r;
  } else {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
  }
}
template <int V>
__device__ __forceinline__ uint32_t vch(uint32_t e, uint32_t f, uint32_t g) {
  if constexpr ((V & kIsaLogic) != 0) {
    if (__builtin_constant_p((e & f) | (~e & g))) return (e & f) | (~e & g);
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(e), "v"(f), "v"(g));
    return r;
  } else {
    return __builtin_amdgcn_bitop3_b32(e, f, g, 0xCA);  // e ? f : g
  }
}
template <int V>
__device__ __forceinline__ uint32_t vmaj(uint32_t a, uint32_t b, uint32_t c) {
  if constexpr ((V & kIsaLogic) != 0) {
    if (__builtin_constant_p((a & b) | (a & c) | (b & c))) return (a & b) | (a & c) | (b & c);
    uint32_t t, r;  // majority = (a ^ b) ? c : b
    asm("v_xor_b32 %0, %1, %2" : "=v"(t) : "v"(a), "v"(b));
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(t), "v"(c), "v"(b));
    return r;
  } else {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);  // majority
  }
}
// a + b; in the kIsaAdds variant a sum of two run-time values is one
// v_add_u32 that the compiler cannot merge into a v_add3_u32.
template <int V>
__device__ __forceinline__ uint32_t vadd(uint32_t a, uint32_t b) {
  if constexpr ((V & kIsaAdds) != 0) {
    if (__builtin_constant_p(a) || __builtin_constant_p(b)) return a + b;
    uint32_t r;
    asm("v_add_u32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
  } else {
    return a + b;
  }
}

struct K256Table {
  uint32_t v[64];
};
__device__ __forceinline__ constexpr K256Table k256() {
  return K256Table{{
      0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u,
      0x923f82a4u, 0xab1c5ed5u, 0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u,
      0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u, 0xe49b69c1u, 0xefbe4786u,
      0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
      0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u,
      0x06ca6351u, 0x14292967u, 0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u,
      0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u, 0xa2bfe8a1u, 0xa81a664bu,
      0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
      0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au,
      0x5b9cca4fu, 0x682e6ff3u, 0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u,
      0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u}};
}

template <int V = 0>
__device__ __forceinline__ uint32_t bsig0_256(uint32_t a) {
  return vxor3<V>(rotr32(a, 2), rotr32(a, 13), rotr32(a, 22));
}
template <int V = 0>
__device__ __forceinline__ uint32_t bsig1_256(uint32_t e) {
  return vxor3<V>(rotr32(e, 6), rotr32(e, 11), rotr32(e, 25));
}
template <int V = 0>
__device__ __forceinline__ uint32_t ssig0_256(uint32_t x) {
  return vxor3<V>(rotr32(x, 7), rotr32(x, 18), x >> 3);
}
template <int V = 0>
__device__ __forceinline__ uint32_t ssig1_256(uint32_t x) {
  return vxor3<V>(rotr32(x, 17), rotr32(x, 19), x >> 10);
}

__device__ __forceinline__ void sha256_iv(uint32_t s[8]) {
  s[0] = 0x6a09e667u; s[1] = 0xbb67ae85u; s[2] = 0x3c6ef372u; s[3] = 0xa54ff53au;
  s[4] = 0x510e527fu; s[5] = 0x9b05688cu; s[6] = 0x1f83d9abu; s[7] = 0x5be0cd19u;
}

// Rounds R0..63 of one compression.  `st` holds the working variables
// a..h *after* round R0-1 (for R0 = 0: the chaining value), `w` the 16
// message words of the block.  On return `st` holds the working variables
// after round 63 (the caller adds the chaining value).  w[] is overwritten
// by the message schedule.
template <int R0 = 0, int V = 0>
__device__ __forceinline__ void sha256_rounds(uint32_t st[8], uint32_t w[16]) {
  constexpr K256Table K = k256();
  uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
  uint32_t e = st[4], f = st[5], g = st[6], h = st[7];
#pragma unroll
  for (int i = R0; i < 64; i++) {
    if (i >= 16) {
      // grouped so that the terms that are fixed for a chain come first
      w[i & 15] = vadd<V>(vadd<V>(vadd<V>(w[i & 15], ssig0_256<V>(w[(i + 1) & 15])), w[(i + 9) & 15]),
                          ssig1_256<V>(w[(i + 14) & 15]));
    }
    uint32_t t1 = vadd<V>(vadd<V>(vadd<V>(h, K.v[i] + w[i & 15]), bsig1_256<V>(e)), vch<V>(e, f, g));
    uint32_t t2 = vadd<V>(bsig0_256<V>(a), vmaj<V>(a, b, c));
    h = g; g = f; f = e; e = vadd<V>(d, t1); d = c; c = b; b = a; a = vadd<V>(t1, t2);
  }
  st[0] = a; st[1] = b; st[2] = c; st[3] = d; st[4] = e; st[5] = f; st[6] = g; st[7] = h;
}

// Full compression: st <- st + rounds(st, w).
template <int V = 0>
__device__ __forceinline__ void sha256_compress(uint32_t st[8], uint32_t w[16]) {
  uint32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = st[i];
  sha256_rounds<0, V>(x, w);
#pragma unroll
  for (int i = 0; i < 8; i++) st[i] += x[i];
}

// ---------------------------------------------------------------- SHA-512
// 64-bit words are handled as (hi, lo) pairs of 32-bit registers; a 64-bit
// rotate is two v_alignbit_b32, the XORs are v_bitop3_b32 per half.
struct u64p {
  uint32_t hi, lo;
};
__device__ __forceinline__ u64p mk64(uint64_t v) { return u64p{uint32_t(v >> 32), uint32_t(v)}; }
__device__ __forceinline__ uint64_t to64(u64p x) { return (uint64_t(x.hi) << 32) | x.lo; }
template <int R>
__device__ __forceinline__ u64p rotr64(u64p x) {
  if constexpr (R < 32) {
    return u64p{__builtin_amdgcn_alignbit(x.lo, x.hi, R), __builtin_amdgcn_alignbit(x.hi, x.lo, R)};
  } else if constexpr (R == 32) {
    return u64p{x.lo, x.hi};
  } else {
    return u64p{__builtin_amdgcn_alignbit(x.hi, x.lo, R - 32),
                __builtin_amdgcn_alignbit(x.lo, x.hi, R - 32)};
  }
}
template <int R>
__device__ __forceinline__ u64p shr64(u64p x) {
  static_assert(R < 32, "small shifts only");
  return u64p{x.hi >> R, __builtin_amdgcn_alignbit(x.hi, x.lo, R)};
}
__device__ __forceinline__ u64p xor3_64(u64p a, u64p b, u64p c) {
  return u64p{xor3(a.hi, b.hi, c.hi), xor3(a.lo, b.lo, c.lo)};
}
__device__ __forceinline__ u64p ch64(u64p e, u64p f, u64p g) {
  return u64p{ch32(e.hi, f.hi, g.hi), ch32(e.lo, f.lo, g.lo)};
}
__device__ __forceinline__ u64p maj64(u64p a, u64p b, u64p c) {
  return u64p{maj32(a.hi, b.hi, c.hi), maj32(a.lo, b.lo, c.lo)};
}
__device__ __forceinline__ u64p add64(u64p a, u64p b) { return mk64(to64(a) + to64(b)); }

// Round constants in constant memory: with the round loop unrolled every
// index is a compile-time constant, so they arrive through scalar loads into
// SGPRs (wave-uniform operands) instead of occupying vector registers.
static __constant__ uint64_t kK512[80] = {
      0x428a2f98d728ae22ull, 0x7137449123ef65cdull, 0xb5c0fbcfec4d3b2full, 0xe9b5dba58189dbbcull,
      0x3956c25bf348b538ull, 0x59f111f1b605d019ull, 0x923f82a4af194f9bull, 0xab1c5ed5da6d8118ull,
      0xd807aa98a3030242ull, 0x12835b0145706fbeull, 0x243185be4ee4b28cull, 0x550c7dc3d5ffb4e2ull,
      0x72be5d74f27b896full, 0x80deb1fe3b1696b1ull, 0x9bdc06a725c71235ull, 0xc19bf174cf692694ull,
      0xe49b69c19ef14ad2ull, 0xefbe4786384f25e3ull, 0x0fc19dc68b8cd5b5ull, 0x240ca1cc77ac9c65ull,
      0x2de92c6f592b0275ull, 0x4a7484aa6ea6e483ull, 0x5cb0a9dcbd41fbd4ull, 0x76f988da831153b5ull,
      0x983e5152ee66dfabull, 0xa831c66d2db43210ull, 0xb00327c898fb213full, 0xbf597fc7beef0ee4ull,
      0xc6e00bf33da88fc2ull, 0xd5a79147930aa725ull, 0x06ca6351e003826full, 0x142929670a0e6e70ull,
      0x27b70a8546d22ffcull, 0x2e1b21385c26c926ull, 0x4d2c6dfc5ac42aedull, 0x53380d139d95b3dfull,
      0x650a73548baf63deull, 0x766a0abb3c77b2a8ull, 0x81c2c92e47edaee6ull, 0x92722c851482353bull,
      0xa2bfe8a14cf10364ull, 0xa81a664bbc423001ull, 0xc24b8b70d0f89791ull, 0xc76c51a30654be30ull,
      0xd192e819d6ef5218ull, 0xd69906245565a910ull, 0xf40e35855771202aull, 0x106aa07032bbd1b8ull,
      0x19a4c116b8d2d0c8ull, 0x1e376c085141ab53ull, 0x2748774cdf8eeb99ull, 0x34b0bcb5e19b48a8ull,
      0x391c0cb3c5c95a63ull, 0x4ed8aa4ae3418acbull, 0x5b9cca4f7763e373ull, 0x682e6ff3d6b2b8a3ull,
      0x748f82ee5defb2fcull, 0x78a5636f43172f60ull, 0x84c87814a1f0ab72ull, 0x8cc702081a6439ecull,
      0x90befffa23631e28ull, 0xa4506cebde82bde9ull, 0xbef9a3f7b2c67915ull, 0xc67178f2e372532bull,
      0xca273eceea26619cull, 0xd186b8c721c0c207ull, 0xeada7dd6cde0eb1eull, 0xf57d4f7fee6ed178ull,
      0x06f067aa72176fbaull, 0x0a637dc5a2c898a6ull, 0x113f9804bef90daeull, 0x1b710b35131c471bull,
      0x28db77f523047d84ull, 0x32caab7b40c72493ull, 0x3c9ebe0a15c9bebcull, 0x431d67c49c100d4cull,
      0x4cc5d4becb3e42b6ull, 0x597f299cfc657e2aull, 0x5fcb6fab3ad6faecull, 0x6c44198c4a475817ull};

__device__ __forceinline__ void sha512_iv(u64p s[8]) {
  s[0] = mk64(0x6a09e667f3bcc908ull); s[1] = mk64(0xbb67ae8584caa73bull);
  s[2] = mk64(0x3c6ef372fe94f82bull); s[3] = mk64(0xa54ff53a5f1d36f1ull);
  s[4] = mk64(0x510e527fade682d1ull); s[5] = mk64(0x9b05688c2b3e6c1full);
  s[6] = mk64(0x1f83d9abfb41bd6bull); s[7] = mk64(0x5be0cd19137e2179ull);
}

// 64-bit helpers on native uint64_t values (kept in aligned register pairs,
// which v_lshl_add_u64 needs; building results as pairs avoids the register
// moves a (hi, lo) struct formulation costs).
__device__ __forceinline__ uint64_t pair64(uint32_t hi, uint32_t lo) { return (uint64_t(hi) << 32) | lo; }
// The value composed from two 32-bit halves, made opaque to the optimiser:
// otherwise the or of the halves is rewritten as an add and the 64-bit sums
// of a round are split into 32-bit partial sums plus zero-extension moves
// (about 25 % more instructions per compression than one v_lshl_add_u64 per
// 64-bit add).  The empty asm emits no instruction.
__device__ __forceinline__ uint64_t opaque64(uint64_t x) {
  asm("" : "+v"(x));
  return x;
}
template <int R>
__device__ __forceinline__ uint64_t rot64(uint64_t x) {
  const uint32_t hi = uint32_t(x >> 32), lo = uint32_t(x);
  if constexpr (R < 32) {
    return pair64(__builtin_amdgcn_alignbit(lo, hi, R), __builtin_amdgcn_alignbit(hi, lo, R));
  } else if constexpr (R == 32) {
    return pair64(lo, hi);
  } else {
    return pair64(__builtin_amdgcn_alignbit(hi, lo, R - 32), __builtin_amdgcn_alignbit(lo, hi, R - 32));
  }
}
template <int V = 0>
__device__ __forceinline__ uint64_t xor3_u64(uint64_t a, uint64_t b, uint64_t c) {
  return opaque64(pair64(vxor3<V>(uint32_t(a >> 32), uint32_t(b >> 32), uint32_t(c >> 32)),
                         vxor3<V>(uint32_t(a), uint32_t(b), uint32_t(c))));
}
template <int V = 0>
__device__ __forceinline__ uint64_t ch_u64(uint64_t e, uint64_t f, uint64_t g) {
  return opaque64(pair64(vch<V>(uint32_t(e >> 32), uint32_t(f >> 32), uint32_t(g >> 32)),
                         vch<V>(uint32_t(e), uint32_t(f), uint32_t(g))));
}
template <int V = 0>
__device__ __forceinline__ uint64_t maj_u64(uint64_t a, uint64_t b, uint64_t c) {
  return opaque64(pair64(vmaj<V>(uint32_t(a >> 32), uint32_t(b >> 32), uint32_t(c >> 32)),
                         vmaj<V>(uint32_t(a), uint32_t(b), uint32_t(c))));
}
// a + b on 64 bits: one v_lshl_add_u64, or (kIsaAdds, two run-time values)
// a v_add_co_u32 / v_addc_co_u32 carry pair.
template <int V = 0>
__device__ __forceinline__ uint64_t add_u64(uint64_t a, uint64_t b) {
  if constexpr ((V & kIsaAdds) != 0) {
    if (__builtin_constant_p(a) || __builtin_constant_p(b)) return a + b;
    uint32_t lo, hi;
    asm("v_add_co_u32 %0, vcc, %2, %3\n\tv_addc_co_u32 %1, vcc, %4, %5, vcc"
        : "=&v"(lo), "=v"(hi)
        : "v"(uint32_t(a)), "v"(uint32_t(b)), "v"(uint32_t(a >> 32)), "v"(uint32_t(b >> 32))
        : "vcc");
    return pair64(hi, lo);
  } else {
    return a + b;
  }
}

// Sixteen SHA-512 rounds with the message schedule extended in place (SCHED:
// rounds >= 16).  Ring-buffer indices are compile-time constants, so w[]
// stays in VGPRs; after sixteen rounds the working variables are back in
// their original registers.  kr: the sixteen round constants (read from
// constant memory into scalar registers, so K + W stays one add in every
// variant).
template <bool SCHED, int V = 0>
__device__ __forceinline__ void sha512_16rounds(uint64_t& a, uint64_t& b, uint64_t& c, uint64_t& d, uint64_t& e,
                                                uint64_t& f, uint64_t& g, uint64_t& h, uint64_t w[16],
                                                const uint64_t* kr) {
#pragma unroll
  for (int i = 0; i < 16; i++) {
    if (SCHED) {
      const uint64_t x15 = w[(i + 1) & 15], x2 = w[(i + 14) & 15];
      const uint64_t s0 = xor3_u64<V>(rot64<1>(x15), rot64<8>(x15), x15 >> 7);
      const uint64_t s1 = xor3_u64<V>(rot64<19>(x2), rot64<61>(x2), x2 >> 6);
      w[i] = add_u64<V>(add_u64<V>(add_u64<V>(w[i], s0), w[(i + 9) & 15]), s1);
    }
    const uint64_t S1 = xor3_u64<V>(rot64<14>(e), rot64<18>(e), rot64<41>(e));
    const uint64_t S0 = xor3_u64<V>(rot64<28>(a), rot64<34>(a), rot64<39>(a));
    const uint64_t t1 = add_u64<V>(add_u64<V>(add_u64<V>(h, kr[i] + w[i]), S1), ch_u64<V>(e, f, g));
    const uint64_t t2 = add_u64<V>(S0, maj_u64<V>(a, b, c));
    h = g; g = f; f = e; e = add_u64<V>(d, t1); d = c; c = b; b = a; a = add_u64<V>(t1, t2);
  }
}

// One SHA-512 compression: st <- st + rounds(st, w).  w[] is overwritten.
// Rounds 0-15 are peeled; rounds 16-79 run as a loop of four 16-round
// blocks, which keeps the code at two copies of sixteen rounds.
template <int V = 0>
__device__ __forceinline__ void sha512_compress(u64p st[8], u64p w16[16]) {
  uint64_t w[16];
#pragma unroll
  for (int i = 0; i < 16; i++) w[i] = to64(w16[i]);
  uint64_t a = to64(st[0]), b = to64(st[1]), c = to64(st[2]), d = to64(st[3]);
  uint64_t e = to64(st[4]), f = to64(st[5]), g = to64(st[6]), h = to64(st[7]);
  sha512_16rounds<false, V>(a, b, c, d, e, f, g, h, w, kK512);
#pragma unroll 1
  for (int r = 16; r < 80; r += 16) sha512_16rounds<true, V>(a, b, c, d, e, f, g, h, w, kK512 + r);
  st[0] = mk64(to64(st[0]) + a); st[1] = mk64(to64(st[1]) + b); st[2] = mk64(to64(st[2]) + c);
  st[3] = mk64(to64(st[3]) + d); st[4] = mk64(to64(st[4]) + e); st[5] = mk64(to64(st[5]) + f);
  st[6] = mk64(to64(st[6]) + g); st[7] = mk64(to64(st[7]) + h);
}

}  // namespace slh
