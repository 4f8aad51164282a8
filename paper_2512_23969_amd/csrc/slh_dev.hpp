// slh_dev.hpp -- SPHINCS+ device primitives for gfx950: parameter sets,
// compressed addresses, the tweakable hashes F / PRF / H / T_l and the
// byte-stream hashes of the message prelude.
//
// Definitions: the paper's Table 1 (parameter sets) and Section II-A (WOTS+,
// FORS, XMSS, hypertree); the SHA2 instantiation of the tweakable hashes is
// that of FIPS 205 Section 11.2 (PK.seed padded to one hash block, then the
// 22-byte compressed address, then the input).
//
// Representation: every n-byte value is held as n/4 32-bit words in
// big-endian interpretation ("BE words"), which is exactly the form SHA-2
// consumes and produces.  Because the compressed address is 22 bytes long,
// an input that follows it starts at byte 2 of a message word; each message
// word is then one v_alignbit_b32 of two neighbouring BE words.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sha2_dev.hpp"

namespace slh {

// ---------------------------------------------------------------- params
template <int ID>
struct Prm;
// SHA2-128f: n=16, h=66, d=22, h'=3, a=6, k=33, w=16 (paper Table 1)
template <>
struct Prm<1> {
  static constexpr int n = 16, h = 66, d = 22, hp = 3, a = 6, k = 33, len1 = 32, len2 = 3, m = 34;
  static constexpr bool wide = false;
  static constexpr bool shake = false;
};
// SHA2-192f: n=24, h=66, d=22, h'=3, a=8, k=33, w=16
template <>
struct Prm<2> {
  static constexpr int n = 24, h = 66, d = 22, hp = 3, a = 8, k = 33, len1 = 48, len2 = 3, m = 42;
  static constexpr bool wide = true;
  static constexpr bool shake = false;
};
// SHA2-256f: n=32, h=68, d=17, h'=4, a=9, k=35, w=16
template <>
struct Prm<3> {
  static constexpr int n = 32, h = 68, d = 17, hp = 4, a = 9, k = 35, len1 = 64, len2 = 3, m = 49;
  static constexpr bool wide = true;
  static constexpr bool shake = false;
};

// SHA2-128s: n=16, h=63, d=7, h'=9, a=12, k=14, w=16 (FIPS 205 Table 2)
template <>
struct Prm<4> {
  static constexpr int n = 16, h = 63, d = 7, hp = 9, a = 12, k = 14, len1 = 32, len2 = 3, m = 30;
  static constexpr bool wide = false;
  static constexpr bool shake = false;
};
// SHA2-192s: n=24, h=63, d=7, h'=9, a=14, k=17, w=16
template <>
struct Prm<5> {
  static constexpr int n = 24, h = 63, d = 7, hp = 9, a = 14, k = 17, len1 = 48, len2 = 3, m = 39;
  static constexpr bool wide = true;
  static constexpr bool shake = false;
};
// SHA2-256s: n=32, h=64, d=8, h'=8, a=14, k=22, w=16
template <>
struct Prm<6> {
  static constexpr int n = 32, h = 64, d = 8, hp = 8, a = 14, k = 22, len1 = 64, len2 = 3, m = 47;
  static constexpr bool wide = true;
  static constexpr bool shake = false;
};

// SHAKE-128f .. SHAKE-256s: the shapes of sets 1..6 with every hash SHAKE256
// (FIPS 205 Section 11.1).
template <int BASE>
struct PrmShake : Prm<BASE> {
  static constexpr bool wide = false;
  static constexpr bool shake = true;
};
template <> struct Prm<7> : PrmShake<1> {};
template <> struct Prm<8> : PrmShake<2> {};
template <> struct Prm<9> : PrmShake<3> {};
template <> struct Prm<10> : PrmShake<4> {};
template <> struct Prm<11> : PrmShake<5> {};
template <> struct Prm<12> : PrmShake<6> {};

template <int ID>
struct P : Prm<ID> {
  using B = Prm<ID>;
  static constexpr int NW = B::n / 4;                       // words per value
  static constexpr int len = B::len1 + B::len2;             // WOTS+ chains
  static constexpr int leaves = 1 << B::hp;                 // leaves per XMSS tree
  static constexpr int fors_bytes = B::k * (B::a + 1) * B::n;
  static constexpr int xmss_bytes = (len + B::hp) * B::n;
  static constexpr int ht_off = B::n + fors_bytes;          // offset of SIG_HT
  static constexpr int sig_bytes = B::n + fors_bytes + B::d * xmss_bytes;
  static constexpr int md_bytes = (B::k * B::a + 7) / 8;
  static constexpr int tree_bits = B::h - B::hp;
  static constexpr int tree_bytes = (tree_bits + 7) / 8;
  static constexpr int leaf_bytes = (B::hp + 7) / 8;
  // Trees taller than one wave's 64 leaves (the small sets) are built in
  // units of 64 leaves (height 6) whose roots a second step combines; FORS
  // trees above 2^12 leaves likewise in units of 2^12 leaves.
  static constexpr int unit_hp = B::hp < 6 ? B::hp : 6;          // height of a TREE unit
  static constexpr int tree_units = 1 << (B::hp - unit_hp);      // units per XMSS tree
  static constexpr int unit_a = B::a < 12 ? B::a : 12;           // height of a FORS unit
  static constexpr int fors_units = 1 << (B::a - unit_a);        // units per FORS tree
};

// Address types (FIPS 205 Section 4.2)
enum : uint32_t { A_WOTS_HASH = 0, A_WOTS_PK = 1, A_TREE = 2, A_FORS_TREE = 3, A_FORS_ROOTS = 4,
                  A_WOTS_PRF = 5, A_FORS_PRF = 6 };

// ---------------------------------------------------------------- tables in HBM
// Per-key record in the device key table (256 bytes).  All values are BE words.
struct DevKey {
  uint32_t param, n;
  uint32_t cache_layers;  // top hypertree layers whose tree nodes are cached (0: none)
  uint32_t pad1;
  uint32_t sk_seed[8];
  uint32_t sk_prf[8];
  uint32_t pk_seed[8];
  uint32_t pk_root[8];
  uint32_t mid256[8];   // SHA-256 chaining value after PK.seed || 0^(64-n)
  uint32_t mid512[16];  // SHA-512 chaining value after PK.seed || 0^(128-n), (hi, lo) pairs
  uint64_t cache_off;   // byte offset of this key's trees in the context's tree cache
  uint32_t pad2[2];
};
static_assert(sizeof(DevKey) == 256, "DevKey layout");

// One sign request as handed to the library (slh_item of slh.h plus the
// location of opt_rand for hedged signing).
struct DevItem {
  uint32_t param;
  uint32_t key_slot;
  uint64_t msg_off;
  uint64_t msg_len;
  uint64_t sig_off;
  uint64_t rnd_off;  // n bytes of opt_rand in the message buffer, or kNoRnd (opt_rand = PK.seed)
};
static_assert(sizeof(DevItem) == 40, "DevItem layout");
constexpr uint64_t kNoRnd = ~uint64_t(0);

// Per-message state shared by the kernels of one batch (1 KiB).
struct WorkRec {
  uint64_t idx_tree;
  uint32_t idx_leaf;
  uint32_t key_slot;
  uint64_t sig_off;
  uint32_t pad[2];
  uint16_t indices[64];   // FORS indices (k <= 35)
  uint32_t fors_pk[8];    // FORS public key = message of layer 0
  uint32_t roots[24][8];  // XMSS root of each layer = message of the next layer
  uint32_t pad2[16];
};
static_assert(sizeof(WorkRec) == 1024, "WorkRec layout");

// ---------------------------------------------------------------- byte order
__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// Write NW BE words as n bytes (4-byte aligned destination).
template <int NW>
__device__ __forceinline__ void store_be(uint8_t* dst, const uint32_t v[NW]) {
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
  for (int i = 0; i < NW; i++) d[i] = bswap32(v[i]);
}
template <int NW>
__device__ __forceinline__ void load_words(const uint32_t* src, uint32_t v[NW]) {
#pragma unroll
  for (int i = 0; i < NW; i++) v[i] = src[i];
}
template <int NW>
__device__ __forceinline__ void store_words(uint32_t* dst, const uint32_t v[NW]) {
#pragma unroll
  for (int i = 0; i < NW; i++) dst[i] = v[i];
}

// ---------------------------------------------------------------- addresses
// The 22-byte compressed address ADRSc = layer(1) | tree(8) | type(1) |
// word1(4) | word2(4) | word3(4) (FIPS 205 Section 11.2) as message words
// 0..4 plus the upper half of word 5 (the low 16 bits of word3).
struct Adrs {
  uint32_t w[5];
  uint32_t tail;  // low 16 bits of word3, already shifted to bits 31..16
};
__device__ __forceinline__ Adrs make_adrs(uint32_t layer, uint64_t tree, uint32_t type, uint32_t w1,
                                          uint32_t w2, uint32_t w3) {
  Adrs A;
  uint32_t thi = uint32_t(tree >> 32), tlo = uint32_t(tree);
  A.w[0] = (layer << 24) | (thi >> 8);
  A.w[1] = (thi << 24) | (tlo >> 8);
  A.w[2] = (tlo << 24) | ((type & 0xFF) << 16) | (w1 >> 16);
  A.w[3] = (w1 << 16) | (w2 >> 16);
  A.w[4] = (w2 << 16) | (w3 >> 16);
  A.tail = w3 << 16;
  return A;
}

}  // namespace slh
#include "keccak_dev.hpp"
namespace slh {

// Message words 0..15 of a block holding ADRSc | x (NX BE words) | padding,
// where the block follows one earlier block (the PK.seed block).
// For SHA-256: 22 + 4 NX + 9 <= 64, i.e. NX <= 8.
template <int NX>
__device__ __forceinline__ void th256_words(const Adrs& A, const uint32_t* x, uint32_t w[16]) {
  static_assert(NX <= 8, "single block");
#pragma unroll
  for (int i = 0; i < 5; i++) w[i] = A.w[i];
  w[5] = A.tail | (x[0] >> 16);
#pragma unroll
  for (int i = 1; i < NX; i++) w[5 + i] = __builtin_amdgcn_alignbit(x[i - 1], x[i], 16);
  w[5 + NX] = (x[NX - 1] << 16) | 0x8000u;
#pragma unroll
  for (int i = 6 + NX; i < 15; i++) w[i] = 0;
  w[15] = (64 + 22 + 4 * NX) * 8;
}

// Tweakable hash with SHA-256 over one block: out = first NOUT words of
// SHA-256(PK.seed || 0^(64-n) || ADRSc || x).
template <int NX, int NOUT, int V = 0>
__device__ __forceinline__ void th256(const uint32_t mid[8], const Adrs& A, const uint32_t* x,
                                      uint32_t* out) {
  uint32_t w[16], st[8];
  th256_words<NX>(A, x, w);
#pragma unroll
  for (int i = 0; i < 8; i++) st[i] = mid[i];
  sha256_rounds<0, V>(st, w);
#pragma unroll
  for (int i = 0; i < NOUT; i++) out[i] = mid[i] + st[i];
}

// Tweakable hash with SHA-512 over one block: out = first NOUT BE words of
// SHA-512(PK.seed || 0^(128-n) || ADRSc || x).  22 + 4 NX + 17 <= 128.
template <int NX, int NOUT, int V = 0>
__device__ __forceinline__ void th512(const uint32_t mid[16], const Adrs& A, const uint32_t* x,
                                      uint32_t* out) {
  static_assert(NX <= 22, "single block");
  uint32_t v[32];
#pragma unroll
  for (int i = 0; i < 5; i++) v[i] = A.w[i];
  v[5] = A.tail | (x[0] >> 16);
#pragma unroll
  for (int i = 1; i < NX; i++) v[5 + i] = __builtin_amdgcn_alignbit(x[i - 1], x[i], 16);
  v[5 + NX] = (x[NX - 1] << 16) | 0x8000u;
#pragma unroll
  for (int i = 6 + NX; i < 31; i++) v[i] = 0;
  v[31] = (128 + 22 + 4 * NX) * 8;
  u64p w[16], st[8];
#pragma unroll
  for (int i = 0; i < 16; i++) w[i] = u64p{v[2 * i], v[2 * i + 1]};
#pragma unroll
  for (int i = 0; i < 8; i++) st[i] = u64p{mid[2 * i], mid[2 * i + 1]};
  sha512_compress<V>(st, w);
#pragma unroll
  for (int i = 0; i < NOUT; i++) out[i] = (i & 1) ? st[i >> 1].lo : st[i >> 1].hi;
}

// For the SHAKE sets the key's mid256 slot holds PK.seed itself (there is
// no chaining value to precompute: PK.seed, ADRS and the input share one
// SHAKE256 block), so every tweakable hash below takes `mid256` as either.
//
// F and PRF: SHA-256 in every SHA2 category (FIPS 205 Sections 11.2.1 and
// 11.2.2), SHAKE256 in the SHAKE ones (Section 11.1).
// V: instruction variant of the SHA-2 arithmetic (sha2_dev.hpp); the SHAKE
// sets have one form.
template <int ID, int V = 0>
__device__ __forceinline__ void thF(const uint32_t mid256[8], const Adrs& A, const uint32_t* x,
                                    uint32_t* out) {
  if constexpr (P<ID>::shake)
    thshake<P<ID>::NW, P<ID>::NW, P<ID>::NW>(mid256, A, x, out);
  else
    th256<P<ID>::NW, P<ID>::NW, V>(mid256, A, x, out);
}
// H: SHA-256 for n = 16, SHA-512 for n = 24, 32; SHAKE256 for the SHAKE sets.
template <int ID, int V = 0>
__device__ __forceinline__ void thH(const DevKey& key, const Adrs& A, const uint32_t* lr,
                                    uint32_t* out) {
  if constexpr (P<ID>::shake)
    thshake<P<ID>::NW, 2 * P<ID>::NW, P<ID>::NW>(key.mid256, A, lr, out);
  else if constexpr (P<ID>::wide)
    th512<2 * P<ID>::NW, P<ID>::NW, V>(key.mid512, A, lr, out);
  else
    th256<2 * P<ID>::NW, P<ID>::NW, V>(key.mid256, A, lr, out);
}
template <int ID, int V = 0>
__device__ __forceinline__ void thH(const uint32_t* mid256, const uint32_t* mid512, const Adrs& A,
                                    const uint32_t* lr, uint32_t* out) {
  if constexpr (P<ID>::shake)
    thshake<P<ID>::NW, 2 * P<ID>::NW, P<ID>::NW>(mid256, A, lr, out);
  else if constexpr (P<ID>::wide)
    th512<2 * P<ID>::NW, P<ID>::NW, V>(mid512, A, lr, out);
  else
    th256<2 * P<ID>::NW, P<ID>::NW, V>(mid256, A, lr, out);
}

// ---------------------------------------------------------------- T_l
// T_l over l n-byte values read through a getter `get(word_index)` that
// returns BE word `word_index` of the concatenated values.  The message is
// ADRSc (22 bytes) | values, after the PK.seed block; SHA-256 for n = 16,
// SHA-512 for n >= 24.  Message word q >= 6 is alignbit(V[q-6], V[q-5], 16).
template <int ID, int L, int V, class Get>
__device__ __forceinline__ void thT_sha2(const uint32_t* mid256, const uint32_t* mid512, const Adrs& A,
                                         Get get, uint32_t* out) {
  constexpr int NW = P<ID>::NW;
  constexpr int NV = L * NW;                 // value words
  constexpr int MB = 22 + 4 * NV;            // message bytes after the seed block
  constexpr bool wide = P<ID>::wide;
  constexpr int BW = wide ? 32 : 16;         // 32-bit words per block
  constexpr int NBLK = (MB + (wide ? 17 : 9) + 4 * BW - 1) / (4 * BW);
  constexpr int LASTQ = 5 + NV;              // word holding the 0x80 byte
  constexpr uint32_t BITS = ((wide ? 128 : 64) + MB) * 8;
  // Message word q of the stream.  The first block is built with
  // compile-time indices (it holds the address words); later blocks only
  // hold value words, padding and the length.
  auto tail_word = [&](int q) -> uint32_t {
    if (q < LASTQ) return __builtin_amdgcn_alignbit(get(q - 6), get(q - 5), 16);
    if (q == LASTQ) return (get(NV - 1) << 16) | 0x8000u;
    if (q == NBLK * BW - 1) return BITS;
    return 0u;
  };
  auto first_word = [&](int q) -> uint32_t {
    if (q < 5) return A.w[q];
    if (q == 5) return A.tail | (get(0) >> 16);
    return tail_word(q);
  };
  if constexpr (!wide) {
    uint32_t st[8];
#pragma unroll
    for (int i = 0; i < 8; i++) st[i] = mid256[i];
    {
      uint32_t w[16];
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = first_word(j);
      sha256_compress<V>(st, w);
    }
    for (int b = 1; b < NBLK; b++) {
      uint32_t w[16];
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = tail_word(16 * b + j);
      sha256_compress<V>(st, w);
    }
#pragma unroll
    for (int i = 0; i < NW; i++) out[i] = st[i];
  } else {
    u64p st[8];
#pragma unroll
    for (int i = 0; i < 8; i++) st[i] = u64p{mid512[2 * i], mid512[2 * i + 1]};
    {
      u64p w[16];
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = u64p{first_word(2 * j), first_word(2 * j + 1)};
      sha512_compress<V>(st, w);
    }
    for (int b = 1; b < NBLK; b++) {
      u64p w[16];
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = u64p{tail_word(32 * b + 2 * j), tail_word(32 * b + 2 * j + 1)};
      sha512_compress<V>(st, w);
    }
#pragma unroll
    for (int i = 0; i < NW; i++) out[i] = (i & 1) ? st[i >> 1].lo : st[i >> 1].hi;
  }
}

// T_l: SHA-2 after the PK.seed block, or SHAKE256 for the SHAKE sets.
template <int ID, int L, int V = 0, class Get>
__device__ __forceinline__ void thT(const uint32_t* mid256, const uint32_t* mid512, const Adrs& A,
                                    Get get, uint32_t* out) {
  if constexpr (P<ID>::shake)
    thshake_t<P<ID>::NW, L>(mid256, A, get, out);
  else
    thT_sha2<ID, L, V>(mid256, mid512, A, get, out);
}

// ---------------------------------------------------------------- byte streams
// SHA-256 / SHA-512 over  prefix (PW BE words held by the caller, PW*4 bytes
// that fit in the first block) | msg (mlen bytes in global memory) with the
// standard padding; `pre` bytes were already absorbed into `st`.
__device__ __forceinline__ uint32_t msg_word(const uint8_t* msg, uint64_t mlen, int64_t p) {
  // 4 bytes of the padded message portion starting at byte p (p may be < 0
  // only for positions covered by the prefix, which callers never ask for)
  uint32_t w = 0;
#pragma unroll
  for (int t = 0; t < 4; t++) {
    int64_t q = p + t;
    uint32_t byte = (q < (int64_t)mlen) ? msg[q] : (q == (int64_t)mlen ? 0x80u : 0u);
    w = (w << 8) | byte;
  }
  return w;
}

// N words of the padded message portion starting at byte p0.  A range that
// lies entirely inside the message at a 4-byte aligned address is read as
// aligned dwords, without per-byte bounds checks (messages placed at 4-byte
// aligned offsets stream about twice as fast); anything else byte by byte.
template <int N>
__device__ __forceinline__ void msg_words(const uint8_t* msg, uint64_t mlen, int64_t p0, uint32_t* w) {
  const uint8_t* q = msg + p0;
  if (p0 >= 0 && uint64_t(p0) + 4 * N <= mlen && (reinterpret_cast<uintptr_t>(q) & 3) == 0) {
    const uint32_t* q4 = reinterpret_cast<const uint32_t*>(q);
#pragma unroll
    for (int j = 0; j < N; j++) w[j] = __builtin_bswap32(q4[j]);
  } else {
#pragma unroll
    for (int j = 0; j < N; j++) w[j] = msg_word(msg, mlen, p0 + 4 * j);
  }
}

template <int PW>
__device__ void sha256_stream(uint32_t st[8], const uint32_t* prefix, const uint8_t* msg,
                              uint64_t mlen, uint64_t pre) {
  static_assert(PW <= 13, "prefix plus padding start must fit the first block");
  const uint64_t total = PW * 4 + mlen;
  const uint64_t nblk = (total + 9 + 63) / 64;
  const uint64_t bits = (pre + total) * 8;
  for (uint64_t b = 0; b < nblk; b++) {
    uint32_t w[16];
    if (b == 0) {
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = j < PW ? prefix[j] : msg_word(msg, mlen, 4 * j - PW * 4);
    } else {
      msg_words<16>(msg, mlen, int64_t(b) * 64 - PW * 4, w);
    }
    if (b == nblk - 1) {
      w[14] = uint32_t(bits >> 32);
      w[15] = uint32_t(bits);
    }
    sha256_compress(st, w);
  }
}

template <int PW>
__device__ void sha512_stream(u64p st[8], const uint32_t* prefix, const uint8_t* msg,
                              uint64_t mlen, uint64_t pre) {
  static_assert(PW <= 27, "prefix plus padding start must fit the first block");
  const uint64_t total = PW * 4 + mlen;
  const uint64_t nblk = (total + 17 + 127) / 128;
  const uint64_t bits = (pre + total) * 8;
  for (uint64_t b = 0; b < nblk; b++) {
    uint32_t v[32];
    if (b == 0) {
#pragma unroll
      for (int j = 0; j < 32; j++) v[j] = j < PW ? prefix[j] : msg_word(msg, mlen, 4 * j - PW * 4);
    } else {
      msg_words<32>(msg, mlen, int64_t(b) * 128 - PW * 4, v);
    }
    if (b == nblk - 1) {
      v[28] = 0; v[29] = 0;
      v[30] = uint32_t(bits >> 32);
      v[31] = uint32_t(bits);
    }
    u64p w[16];
#pragma unroll
    for (int j = 0; j < 16; j++) w[j] = u64p{v[2 * j], v[2 * j + 1]};
    sha512_compress(st, w);
  }
}

// Hash of exactly NWORDS BE words held in registers (fixed layout, unrolled).
template <int NWORDS>
__device__ __forceinline__ void sha256_words(const uint32_t* in, uint32_t out[8]) {
  constexpr int total = NWORDS * 4;
  constexpr int nblk = (total + 9 + 63) / 64;
  uint32_t st[8];
  sha256_iv(st);
#pragma unroll
  for (int b = 0; b < nblk; b++) {
    uint32_t w[16];
#pragma unroll
    for (int j = 0; j < 16; j++) {
      int q = 16 * b + j;
      w[j] = q < NWORDS ? in[q] : (q == NWORDS ? 0x80000000u : 0u);
    }
    if (b == nblk - 1) w[15] = total * 8;
    sha256_compress(st, w);
  }
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = st[i];
}

template <int NWORDS>
__device__ __forceinline__ void sha512_words(const uint32_t* in, uint32_t out[16]) {
  constexpr int total = NWORDS * 4;
  constexpr int nblk = (total + 17 + 127) / 128;
  u64p st[8];
  sha512_iv(st);
#pragma unroll
  for (int b = 0; b < nblk; b++) {
    uint32_t v[32];
#pragma unroll
    for (int j = 0; j < 32; j++) {
      int q = 32 * b + j;
      v[j] = q < NWORDS ? in[q] : (q == NWORDS ? 0x80000000u : 0u);
    }
    if (b == nblk - 1) v[31] = total * 8;
    u64p w[16];
#pragma unroll
    for (int j = 0; j < 16; j++) w[j] = u64p{v[2 * j], v[2 * j + 1]};
    sha512_compress(st, w);
  }
#pragma unroll
  for (int i = 0; i < 8; i++) { out[2 * i] = st[i].hi; out[2 * i + 1] = st[i].lo; }
}

}  // namespace slh
