// kernels.hpp -- the HIP kernels of the batched signing path.
//
// One batch of messages of one parameter set is signed by four launches:
//   k_prelude : one lane per message.  R = PRF_msg, digest = H_msg, FORS
//               indices, idx_tree / idx_leaf  (FIPS 205 Algorithm 19 steps
//               before fors_sign; the paper's Fig. 2 hash_message and
//               message_to_indices).
//   k_fors    : one workgroup per message builds all k FORS trees, writes the
//               selected secret values and auth paths and the FORS public
//               key (paper Section II-A "FORS Signature", Section III-B).
//   k_tree    : one workgroup per 64 hypertree leaves (8 trees of 8 leaves or
//               4 trees of 16 leaves, across messages and layers).  Lanes
//               first run one WOTS+ chain each, then one lane per leaf runs
//               T_len, then the leaves are reduced to the root in registers
//               (paper Section III-A: every XMSS tree of every layer is
//               independent once idx_tree and idx_leaf are known).
//   k_wots    : one lane per WOTS+ chain of the signing leaves.  The TREE
//               kernel kept every intermediate value of those chains, so the
//               WOTS+ signature of layer j (a function of the FORS public key
//               or of root j-1) is a gather, with no hashing.
// The paper launches FORS_Sign and TREE_Sign concurrently and then
// WOTS+_Sign (Section III-F); here the same dependency holds.  The fused
// persistent kernel runs FORS and TREE work from one work counter, and the
// dedup kernels let messages that share an XMSS tree compute it once.
#pragma once
#include "slh_dev.hpp"

namespace slh {

constexpr int kTreeThreads = 256;   // 4 waves
constexpr int kLeavesPerBlock = 64; // one wave's worth of leaves
constexpr int kForsThreads = 256;

// ------------------------------------------------------------------ keys
// Chaining values after the PK.seed block, one lane per key.  Keys of the
// SHAKE sets (parameter ids 7..12) keep PK.seed itself in the mid256 slot.
static __global__ void k_key_midstates(DevKey* keys, uint32_t first, uint32_t count) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  DevKey& K = keys[first + i];
  const int nw = int(K.n) / 4;
  if (K.param >= 7) {
#pragma unroll
    for (int j = 0; j < 8; j++) K.mid256[j] = j < nw ? K.pk_seed[j] : 0u;
    return;
  }
  {
    uint32_t st[8], w[16];
    sha256_iv(st);
#pragma unroll
    for (int j = 0; j < 16; j++) w[j] = (j < 8 && j < nw) ? K.pk_seed[j] : 0u;
    sha256_compress(st, w);
#pragma unroll
    for (int j = 0; j < 8; j++) K.mid256[j] = st[j];
  }
  {
    u64p st[8], w[16];
    sha512_iv(st);
#pragma unroll
    for (int j = 0; j < 16; j++) {
      uint32_t hi = (2 * j < nw && 2 * j < 8) ? K.pk_seed[2 * j] : 0u;
      uint32_t lo = (2 * j + 1 < nw && 2 * j + 1 < 8) ? K.pk_seed[2 * j + 1] : 0u;
      w[j] = u64p{hi, lo};
    }
    sha512_compress(st, w);
#pragma unroll
    for (int j = 0; j < 8; j++) { K.mid512[2 * j] = st[j].hi; K.mid512[2 * j + 1] = st[j].lo; }
  }
}

// Cache placement of keys first .. first+count-1: `layers` cached layers,
// key i's trees at byte offset off0 + i * per_key.
static __global__ void k_set_cache(DevKey* keys, uint32_t first, uint32_t count, uint32_t layers, uint64_t off0,
                            uint64_t per_key) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  keys[first + i].cache_layers = layers;
  keys[first + i].cache_off = off0 + uint64_t(i) * per_key;
}

// ------------------------------------------------------------------ external interface
// Message encodings of FIPS 205 Section 10: pure SLH-DSA (Algorithm 22:
// M' = 0 | len(ctx) | ctx | M) and HashSLH-DSA (Algorithm 23: M' = 1 |
// len(ctx) | ctx | OID | PH(M), PH = SHA-256 or SHA-512).  One workgroup per
// request; the lanes copy bytes, lane 0 computes the pre-hash.  opt_rand (n
// bytes) is copied next to M' when given.
struct ExtJob {
  uint64_t msg_off, msg_len;  // M in the caller's buffer
  uint64_t ctx_off;           // ctx in the caller's buffer
  uint64_t rnd_in;            // opt_rand in the caller's buffer, or kNoRnd
  uint64_t out_off, out_len;  // M' in the encode buffer
  uint64_t rnd_out;           // opt_rand in the encode buffer
  uint32_t ctx_len, prehash, n, pad;
};
constexpr int kEncodeThreads = 256;

static __global__ __launch_bounds__(kEncodeThreads) void k_encode_ext(const ExtJob* __restrict__ jobs,
                                                               const uint8_t* __restrict__ in,
                                                               uint8_t* __restrict__ out) {
  const ExtJob J = jobs[blockIdx.x];
  const uint32_t t = threadIdx.x;
  uint8_t* o = out + J.out_off;
  if (t == 0) {
    o[0] = J.prehash ? 1 : 0;
    o[1] = uint8_t(J.ctx_len);
  }
  for (uint32_t b = t; b < J.ctx_len; b += kEncodeThreads) o[2 + b] = in[J.ctx_off + b];
  if (J.rnd_in != kNoRnd)
    for (uint32_t b = t; b < J.n; b += kEncodeThreads) out[J.rnd_out + b] = in[J.rnd_in + b];
  uint8_t* body = o + 2 + J.ctx_len;
  if (J.prehash == 0) {
    for (uint64_t b = t; b < J.msg_len; b += kEncodeThreads) body[b] = in[J.msg_off + b];
    return;
  }
  if (t != 0) return;
  // DER encodings of id-sha256 (2.16.840.1.101.3.4.2.1) and id-sha512 (...2.3)
  const uint8_t oid[11] = {0x06, 0x09, 0x60, 0x86, 0x48, 0x01, 0x65, 0x03, 0x04, 0x02,
                           uint8_t(J.prehash == 1 ? 0x01 : 0x03)};
  for (int b = 0; b < 11; b++) body[b] = oid[b];
  uint8_t* d = body + 11;
  if (J.prehash == 1) {
    uint32_t st[8];
    sha256_iv(st);
    sha256_stream<0>(st, nullptr, in + J.msg_off, J.msg_len, 0);
    for (int w = 0; w < 8; w++)
      for (int b = 0; b < 4; b++) d[4 * w + b] = uint8_t(st[w] >> (24 - 8 * b));
  } else {
    u64p st[8];
    sha512_iv(st);
    sha512_stream<0>(st, nullptr, in + J.msg_off, J.msg_len, 0);
    for (int w = 0; w < 8; w++)
      for (int b = 0; b < 8; b++) d[8 * w + b] = uint8_t((b < 4 ? st[w].hi : st[w].lo) >> (24 - 8 * (b & 3)));
  }
}

// ------------------------------------------------------------------ prelude
// Per-key values the message hashes need (a DevKey, or a verifier's copy).
struct KeyView {
  const uint32_t* sk_prf;
  const uint32_t* pk_seed;
  const uint32_t* pk_root;
  const uint32_t* opt_rand;  // PK.seed for deterministic signing
};

// R = PRF_msg(SK.prf, opt_rand, M) = Trunc_n(HMAC-SHA-X(SK.prf, opt_rand | M)),
// or SHAKE256(SK.prf | opt_rand | M, 8n) for the SHAKE sets
template <int ID>
__device__ void prf_msg(const KeyView& K, const uint8_t* msg, uint64_t mlen, uint32_t* R) {
  constexpr int NW = P<ID>::NW;
  if constexpr (P<ID>::shake) {
    uint32_t pre[2 * NW];
#pragma unroll
    for (int j = 0; j < NW; j++) { pre[j] = K.sk_prf[j]; pre[NW + j] = K.opt_rand[j]; }
    shake256_stream<2 * NW, NW>(pre, msg, mlen, R);
  } else if constexpr (!P<ID>::wide) {
    uint32_t st[8], blk[16];
    sha256_iv(st);
#pragma unroll
    for (int j = 0; j < 16; j++) blk[j] = (j < NW ? K.sk_prf[j] : 0u) ^ 0x36363636u;
    sha256_compress(st, blk);
    sha256_stream<NW>(st, K.opt_rand, msg, mlen, 64);
    uint32_t inner[8];
#pragma unroll
    for (int j = 0; j < 8; j++) inner[j] = st[j];
    sha256_iv(st);
#pragma unroll
    for (int j = 0; j < 16; j++) blk[j] = (j < NW ? K.sk_prf[j] : 0u) ^ 0x5c5c5c5cu;
    sha256_compress(st, blk);
    sha256_stream<8>(st, inner, nullptr, 0, 64);
#pragma unroll
    for (int j = 0; j < NW; j++) R[j] = st[j];
  } else {
    u64p st[8], w[16];
    sha512_iv(st);
#pragma unroll
    for (int j = 0; j < 16; j++)
      w[j] = u64p{(2 * j < NW ? K.sk_prf[2 * j] : 0u) ^ 0x36363636u,
                  (2 * j + 1 < NW ? K.sk_prf[2 * j + 1] : 0u) ^ 0x36363636u};
    sha512_compress(st, w);
    sha512_stream<NW>(st, K.opt_rand, msg, mlen, 128);
    uint32_t inner[16];
#pragma unroll
    for (int j = 0; j < 8; j++) { inner[2 * j] = st[j].hi; inner[2 * j + 1] = st[j].lo; }
    sha512_iv(st);
#pragma unroll
    for (int j = 0; j < 16; j++)
      w[j] = u64p{(2 * j < NW ? K.sk_prf[2 * j] : 0u) ^ 0x5c5c5c5cu,
                  (2 * j + 1 < NW ? K.sk_prf[2 * j + 1] : 0u) ^ 0x5c5c5c5cu};
    sha512_compress(st, w);
    sha512_stream<16>(st, inner, nullptr, 0, 128);
#pragma unroll
    for (int j = 0; j < NW; j++) R[j] = (j & 1) ? st[j >> 1].lo : st[j >> 1].hi;
  }
}

// digest = H_msg(R, PK.seed, PK.root, M)
//        = MGF1-SHA-X(R | PK.seed | SHA-X(R | PK.seed | PK.root | M), m)
//        (SHA2 sets) or SHAKE256(R | PK.seed | PK.root | M, 8m) (SHAKE sets)
// (16 BE words; the first m bytes are meaningful)
template <int ID>
__device__ void h_msg(const KeyView& K, const uint32_t* R, const uint8_t* msg, uint64_t mlen,
                      uint32_t digest[16]) {
  constexpr int NW = P<ID>::NW;
  uint32_t pre[3 * NW];
#pragma unroll
  for (int j = 0; j < NW; j++) { pre[j] = R[j]; pre[NW + j] = K.pk_seed[j]; pre[2 * NW + j] = K.pk_root[j]; }
  if constexpr (P<ID>::shake) {
    // SHAKE256(R | PK.seed | PK.root | M, 8m)
    shake256_stream<3 * NW, 16>(pre, msg, mlen, digest);
  } else if constexpr (!P<ID>::wide) {
    uint32_t st[8];
    sha256_iv(st);
    sha256_stream<3 * NW>(st, pre, msg, mlen, 0);
    uint32_t seed[2 * NW + 8 + 1];
#pragma unroll
    for (int j = 0; j < 2 * NW; j++) seed[j] = pre[j];
#pragma unroll
    for (int j = 0; j < 8; j++) seed[2 * NW + j] = st[j];
    // MGF1-SHA-256: m = 34 bytes needs counters 0 and 1
#pragma unroll
    for (int c = 0; c < 2; c++) {
      seed[2 * NW + 8] = uint32_t(c);
      uint32_t o[8];
      sha256_words<2 * NW + 9>(seed, o);
#pragma unroll
      for (int j = 0; j < 8; j++) digest[8 * c + j] = o[j];
    }
  } else {
    u64p st[8];
    sha512_iv(st);
    sha512_stream<3 * NW>(st, pre, msg, mlen, 0);
    uint32_t seed[2 * NW + 16 + 1];
#pragma unroll
    for (int j = 0; j < 2 * NW; j++) seed[j] = pre[j];
#pragma unroll
    for (int j = 0; j < 8; j++) { seed[2 * NW + 2 * j] = st[j].hi; seed[2 * NW + 2 * j + 1] = st[j].lo; }
    // MGF1-SHA-512: m <= 64 bytes needs counter 0 only
    seed[2 * NW + 16] = 0u;
    sha512_words<2 * NW + 17>(seed, digest);
  }
}

// Split of the digest (FIPS 205 Algorithm 19): md -> k FORS indices of a
// bits, most-significant bit first (base_2b); then idx_tree and idx_leaf.
template <int ID>
__device__ void split_digest(const uint32_t digest[16], uint16_t* indices, uint64_t* idx_tree,
                             uint32_t* idx_leaf) {
  using Q = P<ID>;
  auto dbyte = [&](int b) -> uint32_t { return (digest[b >> 2] >> (24 - 8 * (b & 3))) & 0xFFu; };
#pragma unroll
  for (int t = 0; t < Q::k; t++) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < Q::a; j++) {
      const int bit = t * Q::a + j;
      v = (v << 1) | ((dbyte(bit >> 3) >> (7 - (bit & 7))) & 1u);
    }
    indices[t] = uint16_t(v);
  }
  uint64_t tree = 0;
#pragma unroll
  for (int j = 0; j < Q::tree_bytes; j++) tree = (tree << 8) | dbyte(Q::md_bytes + j);
  if constexpr (Q::tree_bits < 64) tree &= (uint64_t(1) << Q::tree_bits) - 1;
  uint32_t leaf = 0;
#pragma unroll
  for (int j = 0; j < Q::leaf_bytes; j++) leaf = (leaf << 8) | dbyte(Q::md_bytes + Q::tree_bytes + j);
  *idx_tree = tree;
  *idx_leaf = leaf & ((1u << Q::hp) - 1);
}

// One lane per message: R (written as the first n signature bytes), the
// digest and its split into the message's work record.  The message is read
// as bytes, so any length and alignment is accepted.
template <int ID>
__global__ __launch_bounds__(64) void k_prelude(const DevKey* __restrict__ keys, const DevItem* __restrict__ items,
                          uint32_t count, const uint8_t* __restrict__ msgs, uint8_t* sigs,
                          WorkRec* __restrict__ recs, uint32_t* queue) {
  constexpr int NW = P<ID>::NW;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && queue) {
    queue[0] = 0u;  // work counter of the fused kernel of this batch
    queue[2] = 0u;  // its TREE block counter (chunk-scheduled kernel)
  }
  if (i >= count) return;
  const DevItem it = items[i];
  const DevKey& K = keys[it.key_slot];
  uint32_t rnd[NW];
  if (it.rnd_off != kNoRnd) {
#pragma unroll
    for (int j = 0; j < NW; j++) rnd[j] = msg_word(msgs + it.rnd_off, 4 * NW, 4 * j);
  }
  const KeyView kv{K.sk_prf, K.pk_seed, K.pk_root, it.rnd_off != kNoRnd ? rnd : K.pk_seed};
  const uint8_t* msg = msgs + it.msg_off;
  uint32_t R[NW], digest[16];
  prf_msg<ID>(kv, msg, it.msg_len, R);
  store_be<NW>(sigs + it.sig_off, R);
  h_msg<ID>(kv, R, msg, it.msg_len, digest);
  WorkRec& W = recs[i];
  uint64_t tree;
  uint32_t leaf;
  split_digest<ID>(digest, W.indices, &tree, &leaf);
  W.idx_tree = tree;
  W.idx_leaf = leaf;
  W.key_slot = it.key_slot;
  W.sig_off = it.sig_off;
}

// ------------------------------------------------------------------ FORS
// The k FORS trees of every message of the batch form one flat list of
// trees (tree id = message * k + t).  A workgroup takes FG consecutive trees,
// which may belong to different messages and keys.
//   pair phase : one lane per pair of sibling leaves computes PRF and F for
//                both (one SHA-256 code copy, run four times in a loop) and
//                their parent with H; parents go to LDS.
//   level phase: levels 2..a are reduced level by level in LDS, the node of
//                index q at level z written over its left child (slot
//                q << (z - 1)).
// The selected secret value and every auth node are written by the lane that
// computes them; the root of each tree goes to `roots` (n bytes per tree).
// The FORS public key T_k of a message is computed afterwards by k_fors_pk,
// once all its trees are done (paper Section II-A "FORS Signature"; the
// paper's FORS fusion, Section III-B, groups trees per thread block for the
// same reason: more independent nodes per synchronisation).
// A FORS unit is a whole tree (f sets) or a subtree of 2^12 leaves (192s,
// 256s); its root is a FORS root or a level-12 node for k_fors_top.
template <int ID>
struct ForsShape {
  static constexpr int PAIRS = 1 << (P<ID>::unit_a - 1);  // level-1 nodes per unit
  static constexpr int UNITS = P<ID>::fors_units;          // units per FORS tree
};

// One group of FG units (flat unit ids group*FG ...; unit u of tree ft is
// ft * UNITS + u), reduced by a workgroup of FT lanes.  LPL (leaves per
// lane, the paper's Relax-FORS per-thread buffer, Section III-B): each lane
// task builds LPL = 2 or 4 sibling leaves and reduces them in registers to
// one node of level log2(LPL); those nodes go to LDS.  `node` is LDS of
// FG * BASE * NW words.  All threads of the workgroup must call it.
template <int ID, int LPL>
struct ForsLeaves {
  static_assert(LPL == 2 || LPL == 4, "two or four leaves per lane");
  static constexpr int L0 = LPL == 4 ? 2 : 1;                 // level of the nodes that go to LDS
  static constexpr int BASE = 1 << (P<ID>::unit_a - L0);      // such nodes per unit
};

template <int ID, int FG, int LPL = 2, int FT = kForsThreads, int V = 0>
__device__ __forceinline__ void fors_group(const DevKey* __restrict__ keys, const WorkRec* __restrict__ recs,
                           uint32_t nunits, uint8_t* sigs, uint32_t* __restrict__ roots, uint32_t group,
                           uint32_t* node) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, A = Q::a, KT = Q::k, AU = Q::unit_a, UNITS = ForsShape<ID>::UNITS;
  constexpr int L0 = ForsLeaves<ID, LPL>::L0, BASE = ForsLeaves<ID, LPL>::BASE;
  const uint32_t fu0 = group * FG;

  // leaf phase: one task per level-L0 node
  for (int q = threadIdx.x; q < FG * BASE; q += FT) {
    const uint32_t fu = fu0 + q / BASE;
    if (fu >= nunits) break;  // q only grows, so the rest of this lane's tasks are out too
    const uint32_t ft = fu / UNITS, u = fu % UNITS;
    const uint32_t j = (u << (AU - L0)) + q % BASE;  // level-L0 node index within the tree
    const uint32_t msg = ft / KT, t = ft - msg * KT;
    const WorkRec& W = recs[msg];
    const DevKey& K = keys[W.key_slot];
    const uint64_t tree = W.idx_tree;
    const uint32_t kp = W.idx_leaf;
    const uint32_t idx = W.indices[t];
    uint8_t* tsig = sigs + W.sig_off + Q::n + t * (A + 1) * Q::n;
    uint32_t mid[8], sks[NW];
    load_words<8>(K.mid256, mid);
    load_words<NW>(K.sk_seed, sks);
    uint32_t lvl1[(LPL / 2) * NW];  // this task's level-1 nodes, left to right
#pragma unroll
    for (int pr = 0; pr < LPL / 2; pr++) {
      const uint32_t jp = j * (LPL / 2) + pr;  // level-1 node (leaf pair) index within the tree
      const uint32_t g0 = (t << A) + 2 * jp;
      uint32_t sk[NW], lr[2 * NW];
      // four hashes: PRF(leaf 2jp), F(leaf 2jp), PRF(leaf 2jp+1), F(leaf 2jp+1)
#pragma unroll 1
      for (int c = 0; c < 4; c++) {
        const uint32_t g = g0 + (c >> 1);
        const bool isF = c & 1;
        uint32_t in[NW], out[NW];
#pragma unroll
        for (int w = 0; w < NW; w++) in[w] = isF ? sk[w] : sks[w];
        thF<ID, V>(mid, make_adrs(0, tree, isF ? A_FORS_TREE : A_FORS_PRF, kp, 0, g), in, out);
        if (!isF) {
#pragma unroll
          for (int w = 0; w < NW; w++) sk[w] = out[w];
          if (g == (t << A) + idx) store_be<NW>(tsig, sk);  // the selected secret value
        } else {
#pragma unroll
          for (int w = 0; w < NW; w++) {
            if (c == 1) lr[w] = out[w]; else lr[NW + w] = out[w];
          }
        }
      }
      if ((idx >> 1) == jp) store_be<NW>(tsig + Q::n, (idx & 1) ? lr : lr + NW);  // auth[0]
      thH<ID, V>(K, make_adrs(0, tree, A_FORS_TREE, kp, 1, (t << (A - 1)) + jp), lr, &lvl1[pr * NW]);
      if (((idx >> 1) ^ 1u) == jp) store_be<NW>(tsig + 2 * Q::n, &lvl1[pr * NW]);  // auth[1]
    }
    if constexpr (L0 == 1) {
      store_words<NW>(&node[q * NW], lvl1);
    } else {
      uint32_t par[NW];
      thH<ID, V>(K, make_adrs(0, tree, A_FORS_TREE, kp, 2, (t << (A - 2)) + j), lvl1, par);
      if (((idx >> 2) ^ 1u) == j) store_be<NW>(tsig + 3 * Q::n, par);  // auth[2]
      store_words<NW>(&node[q * NW], par);
    }
  }
  __syncthreads();
  // level phase: levels L0+1 .. AU in LDS; node q of level z is written over
  // its left child (slot q << (z - L0))
#pragma unroll 1
  for (int z = L0 + 1; z <= AU; z++) {
    const int per = 1 << (AU - z);  // nodes of level z per unit
    for (int q = threadIdx.x; q < FG * per; q += FT) {
      const uint32_t fu = fu0 + q / per;
      if (fu >= nunits) break;
      const uint32_t ft = fu / UNITS, u = fu % UNITS;
      const uint32_t i = (u << (AU - z)) + q % per;  // node index within the tree's level z
      const uint32_t msg = ft / KT, t = ft - msg * KT;
      const WorkRec& W = recs[msg];
      const DevKey& K = keys[W.key_slot];
      const uint32_t idx = W.indices[t];
      const int ls = (2 * q) << (z - 1 - L0), rs = (2 * q + 1) << (z - 1 - L0);
      uint32_t lr[2 * NW];
      load_words<NW>(&node[ls * NW], lr);
      load_words<NW>(&node[rs * NW], lr + NW);
      uint32_t out[NW];
      thH<ID, V>(K, make_adrs(0, W.idx_tree, A_FORS_TREE, W.idx_leaf, z, (t << (A - z)) + i), lr, out);
      if (z < A && (((idx >> z) ^ 1u) == i))
        store_be<NW>(sigs + W.sig_off + Q::n + t * (A + 1) * Q::n + (1 + z) * Q::n, out);  // auth[z]
      if (z == AU) store_words<NW>(roots + size_t(fu) * NW, out);
      else store_words<NW>(&node[ls * NW], out);
    }
    __syncthreads();
  }
}

template <int ID, int FG, int LPL = 2, int FT = kForsThreads, int V = 0>
__global__ __launch_bounds__(FT) void k_fors(const DevKey* __restrict__ keys, const WorkRec* __restrict__ recs,
                                             uint32_t nunits, uint8_t* sigs, uint32_t* __restrict__ roots) {
  __shared__ uint32_t node[FG * ForsLeaves<ID, LPL>::BASE * P<ID>::NW];
  fors_group<ID, FG, LPL, FT, V>(keys, recs, nunits, sigs, roots, blockIdx.x, node);
}

// FORS trees built in units: one lane per tree combines its unit roots
// (level unit_a) up to the tree root, writing the authentication nodes of
// those upper levels; tree roots go to `troots` for k_fors_pk.
template <int ID>
__global__ void k_fors_top(const DevKey* __restrict__ keys, const WorkRec* __restrict__ recs, uint32_t ntrees,
                           uint8_t* sigs, const uint32_t* __restrict__ uroots, uint32_t* __restrict__ troots) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, A = Q::a, KT = Q::k, AU = Q::unit_a, UNITS = Q::fors_units;
  const uint32_t ft = blockIdx.x * blockDim.x + threadIdx.x;
  if (ft >= ntrees) return;
  const uint32_t msg = ft / KT, t = ft - msg * KT;
  const WorkRec& W = recs[msg];
  const DevKey& K = keys[W.key_slot];
  const uint32_t idx = W.indices[t];
  uint32_t lvl[UNITS * NW];
#pragma unroll
  for (int w = 0; w < UNITS * NW; w++) lvl[w] = uroots[size_t(ft) * UNITS * NW + w];
#pragma unroll
  for (int z = AU + 1; z <= A; z++) {
    const int cnt = 1 << (A - z);  // nodes of level z in this tree
#pragma unroll
    for (int i = 0; i < cnt; i++) {
      uint32_t out[NW];
      thH<ID>(K, make_adrs(0, W.idx_tree, A_FORS_TREE, W.idx_leaf, z, (t << (A - z)) + i), &lvl[2 * i * NW], out);
#pragma unroll
      for (int u = 0; u < NW; u++) lvl[i * NW + u] = out[u];
      if (z < A && (((idx >> z) ^ 1u) == uint32_t(i)))
        store_be<NW>(sigs + W.sig_off + Q::n + t * (A + 1) * Q::n + (1 + z) * Q::n, out);  // auth[z]
    }
  }
  store_words<NW>(troots + size_t(ft) * NW, lvl);
}

// FORS public key T_k(FORS_ROOTS address, roots) of each message, one lane
// per message, from the roots the FORS kernel left in HBM.
template <int ID>
__global__ void k_fors_pk(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs, uint32_t count,
                          const uint32_t* __restrict__ roots) {
  using Q = P<ID>;
  constexpr int NW = Q::NW;
  const uint32_t msg = blockIdx.x * blockDim.x + threadIdx.x;
  if (msg >= count) return;
  WorkRec& W = recs[msg];
  const DevKey& K = keys[W.key_slot];
  const uint32_t* r = roots + size_t(msg) * Q::k * NW;
  auto get = [&](int wi) -> uint32_t { return r[wi]; };
  uint32_t pk[NW];
  thT<ID, Q::k>(K.mid256, K.mid512, make_adrs(0, W.idx_tree, A_FORS_ROOTS, W.idx_leaf, 0, 0), get, pk);
  store_words<NW>(W.fors_pk, pk);
}

// ------------------------------------------------------------------ TREE
// Tree-job description: which XMSS tree a group of 2^h' leaves belongs to.
struct TreeJob {
  const DevKey* key;
  uint32_t layer;
  uint64_t tree;
  int32_t sign_leaf;   // leaf whose WOTS+ chains are kept, or -1
  uint8_t* sig_xmss;   // XMSS signature slot of this layer, or null
  uint32_t* root_out;  // where the root goes (BE words), or null
  uint32_t* spill;     // len * 16 * NW words for the signing leaf, or null
};

template <int ID>
__device__ __forceinline__ TreeJob sign_job(const DevKey* keys, WorkRec* recs, uint8_t* sigs,
                                            uint32_t* spill, uint32_t ftree) {
  using Q = P<ID>;
  const uint32_t msg = ftree / Q::d, layer = ftree - msg * Q::d;
  WorkRec& W = recs[msg];
  TreeJob J;
  J.key = &keys[W.key_slot];
  J.layer = layer;
  const uint32_t sh = Q::hp * layer;
  J.tree = sh >= 64 ? 0 : (W.idx_tree >> sh);
  if (layer == 0) {
    J.sign_leaf = int32_t(W.idx_leaf);
  } else {
    const uint32_t sh1 = Q::hp * (layer - 1);
    J.sign_leaf = int32_t((W.idx_tree >> sh1) & ((1u << Q::hp) - 1));
  }
  J.sig_xmss = sigs + W.sig_off + Q::ht_off + size_t(layer) * Q::xmss_bytes;
  J.root_out = (layer + 1 < uint32_t(Q::d)) ? W.roots[layer] : nullptr;
  J.spill = spill ? spill + size_t(ftree) * Q::len * 16 * Q::NW : nullptr;
  return J;
}

// Digit c of the WOTS+ message of layer `layer` of a signature: the base-16
// digits of that layer's message (FORS pk for layer 0, root of layer j-1
// otherwise) with the checksum digits appended (FIPS 205 Algorithm 7).
template <int ID>
__device__ __forceinline__ uint32_t wots_digit(const WorkRec& W, uint32_t layer, uint32_t c) {
  using Q = P<ID>;
  const uint32_t* M = layer == 0 ? W.fors_pk : W.roots[layer - 1];
  auto nib = [&](int i) -> uint32_t { return (M[i >> 3] >> (28 - 4 * (i & 7))) & 15u; };
  if (c < uint32_t(Q::len1)) return nib(c);
  uint32_t csum = 0;
  for (int i = 0; i < Q::len1; i++) csum += 15u - nib(i);
  csum <<= 4;  // (8 - (len2 * lg_w) mod 8) mod 8 = 4 for len2 = 3
  return (csum >> (12 - 4 * (c - Q::len1))) & 15u;
}

// One WOTS+ chain: PRF then 15 F steps.  If `keep` is set, every value of
// the chain (steps 0..15) is written to keep[step * NW ...].  CAP (layers
// signed in order): if `cap` is set, the value after `cap_step` steps is
// written there as signature bytes (FIPS 205 Algorithm 7: the WOTS+
// signature of chain c is the chain advanced by the message's digit c).
template <int ID, int V = 0, bool CAP = false>
__device__ __forceinline__ void wots_chain(const uint32_t mid[8], const uint32_t* sks, uint32_t layer,
                                           uint64_t tree, uint32_t kp, uint32_t c, uint32_t* keep,
                                           uint32_t x[P<ID>::NW], uint32_t cap_step = 0,
                                           uint8_t* cap = nullptr) {
  constexpr int NW = P<ID>::NW;
  thF<ID, V>(mid, make_adrs(layer, tree, A_WOTS_PRF, kp, c, 0), sks, x);
  if (keep) store_words<NW>(keep, x);
  if (CAP && cap && cap_step == 0) store_be<NW>(cap, x);
  const Adrs A0 = make_adrs(layer, tree, A_WOTS_HASH, kp, c, 0);
  for (uint32_t s = 0; s < 15; s++) {
    Adrs A = A0;
    A.tail = s << 16;
    uint32_t y[NW];
    thF<ID, V>(mid, A, x, y);
#pragma unroll
    for (int u = 0; u < NW; u++) x[u] = y[u];
    if (keep) store_words<NW>(keep + (s + 1) * NW, x);
    if (CAP && cap && cap_step == s + 1) store_be<NW>(cap, x);
  }
}

// Chain chunks of wave 0 in a TREE block.  Wave 0 also runs T_len and the
// XMSS levels of the block (10 + 3 SHA-256, 13 and 22 SHA-512 compressions,
// about 13, 37 and 62 chain-step equivalents at 2.8 SHA-256 per SHA-512), so
// it takes fewer of the len chunks of 16 compressions: w0 + extra / 16 =
// (len - w0) / 3 gives 8, 11 and 14.
// With NWAV waves per block the same balance w0 + extra / 16 =
// (len - w0) / (NWAV - 1) gives w0 = (len - (NWAV - 1) extra / 16) / NWAV:
// 17 / 24 / 31 chunks for two waves, 8 / 11 / 14 for four, 4 / 4 / 5 for
// eight.
template <int ID, int NWAV = 4>
struct TreeSplit {
  static_assert(NWAV == 2 || NWAV == 4 || NWAV == 8, "TREE blocks of 2, 4 or 8 waves");
  static constexpr int L = P<ID>::len;
  static constexpr int wave0 = NWAV == 4 ? (L == 35 ? 8 : (L == 51 ? 11 : 14))
                             : NWAV == 2 ? (L == 35 ? 17 : (L == 51 ? 24 : 31))
                                         : (L == 35 ? 4 : (L == 51 ? 4 : 5));
};

// What a TREE block works on: the trees of a batch's signatures, the top tree
// of a new key, or the cached upper layers of keys.
enum TreeKind : int { kSignTrees = 0, kKeygenTree = 1, kCacheTrees = 2 };

// Cached upper layers of a key: layer d-1-u (u = 0 .. L-1) has 2^(h' u) trees,
// stored top layer first, so its trees start at (2^(h' u) - 1) / (2^h' - 1).
template <int ID>
struct CacheShape {
  __host__ __device__ static constexpr uint64_t layer_first(uint32_t u) {
    return ((uint64_t(1) << (P<ID>::hp * u)) - 1) / ((uint64_t(1) << P<ID>::hp) - 1);
  }
  __host__ __device__ static constexpr uint64_t trees(uint32_t layers) { return layer_first(layers); }
};

// Number of nodes of one XMSS tree and the offset of level z in a node
// buffer: level z (2^(h'-z) nodes) starts at 2^(h'+1) - 2^(h'-z+1).
template <int ID>
struct TreeNodes {
  static constexpr int count = (2 << P<ID>::hp) - 1;
  __device__ static constexpr int off(int z) { return (2 << P<ID>::hp) - (2 << (P<ID>::hp - z)); }
};

// Phase 1 of a block of 64 leaves (TPB trees, flat tree ids block*TPB ...):
// the WOTS+ chains, one lane per chain, chain ends to `st` (len * 64 * NW
// words).  kKeygenTree: a single tree (layer d-1, tree 0) of key `key_slot`;
// kCacheTrees: tree i of the cached layers of keys key_slot, key_slot + 1,
// ... (all with the same cache_layers); kSignTrees: trees from the batch's
// work records.
template <int ID, int KIND>
__device__ __forceinline__ TreeJob tree_job(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs,
                                            uint8_t* sigs, uint32_t* spill, uint32_t key_slot,
                                            uint32_t* root_out, uint32_t ftree) {
  if constexpr (KIND == kSignTrees) {
    return sign_job<ID>(keys, recs, sigs, spill, ftree);
  } else {
    TreeJob J;
    J.sign_leaf = -1;
    J.sig_xmss = nullptr;
    J.spill = nullptr;
    if constexpr (KIND == kKeygenTree) {
      J.key = &keys[key_slot];
      J.layer = P<ID>::d - 1;
      J.tree = 0;
      J.root_out = root_out;
    } else {
      const uint32_t L = keys[key_slot].cache_layers;
      const uint64_t per = CacheShape<ID>::trees(L);
      const uint32_t k = uint32_t(ftree / per);
      const uint64_t local = ftree - uint64_t(k) * per;
      uint32_t u = 0;
      while (u + 1 < L && local >= CacheShape<ID>::layer_first(u + 1)) u++;
      J.key = &keys[key_slot + k];
      J.layer = P<ID>::d - 1 - u;
      J.tree = local - CacheShape<ID>::layer_first(u);
      J.root_out = nullptr;
    }
    return J;
  }
}

// Trees of a batch, optionally restricted to a list of distinct trees
// (within-batch dedup): tree slot i of the list is flat tree id ulist[i],
// and there are *ucount of them; without a list, slot i is tree i of ntrees.
// With dedup, lown[ft * leaves + leaf] names the (message, layer) pair whose
// kept-chain area receives the chains of that leaf of tree ft (~0: no pair
// signs with that leaf).
// Without a list, slot i is tree first + i.  For trees built in units
// (XMSS trees above 64 leaves), slots are units (unit u of tree ft is
// ft * tree_units + u) and each unit's root goes to uroots.
// Layers signed in order take the trees of one layer: slot i is tree
// first + i * stride (first = the layer, stride = d).
struct TreeList {
  const uint32_t* ulist;
  const uint32_t* ucount;
  const uint32_t* lown;
  uint32_t first;
  uint32_t* uroots = nullptr;
  uint32_t stride = 1;
  __device__ __forceinline__ uint32_t count(uint32_t ntrees) const { return ucount ? *ucount : ntrees; }
  __device__ __forceinline__ uint32_t at(uint32_t i) const { return ulist ? ulist[i] : first + i * stride; }
};

// NWAV: waves of the block (chunk split of TreeSplit); V: instruction
// variant; CAP: layers signed in order, the signing leaf's chains write the
// WOTS+ signature of the layer as they pass its digits.
// w0 > 0 overrides wave 0's share of the chunks (the fused kernel's tuning);
// cstep > 0 overrides the whole split: this wave runs chunks cbeg, cbeg +
// cstep, ... below cend (the fused kernel's items of several blocks).
template <int ID, int KIND, bool SPLIT = false, int NWAV = 4, int V = 0, bool CAP = false>
__device__ __forceinline__ void tree_chains(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs,
                                            uint32_t ntrees, uint8_t* sigs, uint32_t* __restrict__ st,
                                            uint32_t* __restrict__ spill, uint32_t key_slot, uint32_t* root_out,
                                            uint32_t block, TreeList tl = TreeList{nullptr, nullptr, nullptr, 0u},
                                            int w0 = 0, int cbeg = 0, int cend_ = 0, int cstep_ = 0) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len, LV = 1 << Q::unit_hp, UT = Q::tree_units;
  constexpr int TPB = kLeavesPerBlock / LV;
  const int W0 = w0 > 0 ? w0 : TreeSplit<ID, NWAV>::wave0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t tree0 = block * TPB;
  const uint32_t lt = lane / LV;
  if (tree0 + lt >= tl.count(ntrees)) return;
  const uint32_t fu = tl.at(tree0 + lt), ft = fu / UT;
  const uint32_t kp = ((fu % UT) << Q::unit_hp) + lane % LV;  // leaf within the tree
  const TreeJob J = tree_job<ID, KIND>(keys, recs, sigs, spill, key_slot, root_out, ft);
  uint32_t mid[8], sks[NW];
  load_words<8>(J.key->mid256, mid);
  load_words<NW>(J.key->sk_seed, sks);
  uint32_t* keep = nullptr;
  if (tl.lown) {
    const uint32_t o = tl.lown[size_t(ft) * Q::leaves + kp];
    if (spill && o != 0xffffffffu) keep = spill + size_t(o) * LEN * 16 * NW;
  } else if (J.spill && int32_t(kp) == J.sign_leaf) {
    keep = J.spill;
  }
  // a block of NWAV waves: wave 0 chunks 0 .. W0-1, waves 1..NWAV-1 chunks
  // W0 + (wave - 1) + (NWAV - 1) i; a split block (one wave per workgroup,
  // part blockIdx.y of gridDim.y): chunks part, part + parts, ...
  const int c0 = cstep_ > 0 ? cbeg : SPLIT ? int(blockIdx.y) : (wave == 0 ? 0 : W0 + wave - 1);
  const int cend = cstep_ > 0 ? cend_ : SPLIT ? LEN : (wave == 0 ? W0 : LEN);
  const int cstep = cstep_ > 0 ? cstep_ : SPLIT ? int(gridDim.y) : (wave == 0 ? 1 : NWAV - 1);
  const bool cap = CAP && int32_t(kp) == J.sign_leaf;
  for (int c = c0; c < cend; c += cstep) {
    uint32_t x[NW];
    if constexpr (CAP) {
      const uint32_t digit = cap ? wots_digit<ID>(recs[ft / Q::d], J.layer, uint32_t(c)) : 0u;
      wots_chain<ID, V, true>(mid, sks, J.layer, J.tree, kp, c, nullptr, x, digit,
                              cap ? J.sig_xmss + c * Q::n : nullptr);
    } else {
      wots_chain<ID, V>(mid, sks, J.layer, J.tree, kp, c, keep ? keep + c * 16 * NW : nullptr, x);
    }
    store_words<NW>(st + (c * kLeavesPerBlock + lane) * NW, x);
  }
}

// Phases 2 and 3 of a block, run by one wave: T_len of each leaf over its
// chain ends, then the XMSS levels inside the wave (the node of level z lives
// in the lanes with kp % 2^z == 0, its partner is 2^(z-1) lanes up); auth
// nodes and the root are written where they are computed.
// `nodes` (optional): every node of the tree is stored at
// nodes[(ft * TreeNodes::count + off(z) + i) * NW] for the dedup scatter.
template <int ID, int KIND, int V = 0>
__device__ __forceinline__ void tree_finish(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs,
                                            uint32_t ntrees, uint8_t* sigs, const uint32_t* __restrict__ st,
                                            uint32_t* __restrict__ spill, uint32_t key_slot, uint32_t* root_out,
                                            uint32_t block, TreeList tl = TreeList{nullptr, nullptr, nullptr, 0u},
                                            uint32_t* __restrict__ nodes = nullptr) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len, UH = Q::unit_hp, LV = 1 << UH, UT = Q::tree_units;
  constexpr int TPB = kLeavesPerBlock / LV;
  const int lane = threadIdx.x & 63;
  const uint32_t tree0 = block * TPB;
  const uint32_t lt = lane / LV, kl = lane % LV;  // leaf within the unit
  const bool valid = tree0 + lt < tl.count(ntrees);
  const uint32_t fu = valid ? tl.at(tree0 + lt) : 0u, ft = fu / UT;
  const uint32_t kp = ((fu % UT) << UH) + kl;  // leaf within the tree
  uint32_t* tn = (UT == 1 && nodes) ? nodes + size_t(ft) * TreeNodes<ID>::count * NW : nullptr;
  uint32_t v[NW];
  TreeJob J{};
  if (valid) {
    J = tree_job<ID, KIND>(keys, recs, sigs, spill, key_slot, root_out, ft);
    auto get = [&](int wi) -> uint32_t {
      const int c = wi / NW, u = wi - c * NW;
      return st[(c * kLeavesPerBlock + lane) * NW + u];
    };
    thT<ID, LEN, V>(J.key->mid256, J.key->mid512, make_adrs(J.layer, J.tree, A_WOTS_PK, kp, 0, 0), get, v);
  } else {
#pragma unroll
    for (int u = 0; u < NW; u++) v[u] = 0;
  }
#pragma unroll 1
  for (int z = 1; z <= UH; z++) {
    const uint32_t span = 1u << (z - 1);
    // auth node of level z-1
    if (valid && J.sig_xmss && (kl & (span - 1)) == 0) {
      const uint32_t i = kp >> (z - 1);
      if (i == ((uint32_t(J.sign_leaf) >> (z - 1)) ^ 1u))
        store_be<NW>(J.sig_xmss + (LEN + z - 1) * Q::n, v);
    }
    if (valid && tn && (kl & (span - 1)) == 0)
      store_words<NW>(tn + (TreeNodes<ID>::off(z - 1) + (kp >> (z - 1))) * NW, v);
    uint32_t lr[2 * NW];
#pragma unroll
    for (int u = 0; u < NW; u++) {
      lr[u] = v[u];
      lr[NW + u] = __shfl_down(v[u], span, 64);
    }
    if (valid && (kl & ((span << 1) - 1)) == 0) {
      thH<ID, V>(J.key->mid256, J.key->mid512, make_adrs(J.layer, J.tree, A_TREE, 0, z, kp >> z), lr, v);
    }
  }
  if constexpr (UT == 1) {
    if (valid && kl == 0 && J.root_out) store_words<NW>(J.root_out, v);
    if (valid && kl == 0 && tn) store_words<NW>(tn + TreeNodes<ID>::off(UH) * NW, v);
  } else {
    if (valid && kl == 0) store_words<NW>(tl.uroots + size_t(fu) * NW, v);  // level-UH node
  }
}

// A TREE block of NWAV waves (64 NWAV lanes; the workgroup-size knob), SHA-2
// variant V; CAP: one layer of the batch's trees (first = layer, stride = d)
// with the WOTS+ signature captured on the way (layers signed in order).
template <int ID, int KIND, int NWAV = 4, int V = 0, bool CAP = false>
__global__ __launch_bounds__(64 * NWAV) void k_tree(const DevKey* __restrict__ keys,
                                                    WorkRec* __restrict__ recs, uint32_t ntrees,
                                                    uint8_t* sigs, uint32_t* __restrict__ stage,
                                                    uint32_t* __restrict__ spill,
                                                    uint32_t key_slot, uint32_t* root_out,
                                                    const uint32_t* ulist, const uint32_t* ucount,
                                                    const uint32_t* lown, uint32_t* nodes, uint32_t first,
                                                    uint32_t* uroots, uint32_t stride) {
  TreeList tl{ulist, ucount, lown, first, uroots};
  tl.stride = stride;
  if (blockIdx.x * (kLeavesPerBlock >> P<ID>::unit_hp) >= tl.count(ntrees)) return;  // beyond the distinct trees
  uint32_t* st = stage + size_t(blockIdx.x) * P<ID>::len * kLeavesPerBlock * P<ID>::NW;
  tree_chains<ID, KIND, false, NWAV, V, CAP>(keys, recs, ntrees, sigs, st, spill, key_slot, root_out, blockIdx.x,
                                             tl);
  __syncthreads();
  if ((threadIdx.x >> 6) == 0)
    tree_finish<ID, KIND, V>(keys, recs, ntrees, sigs, st, spill, key_slot, root_out, blockIdx.x, tl, nodes);
}

// The two phases of k_tree as separate launches, for batches too small to
// spread their blocks over the CUs: k_tree_chains runs the chains of block
// blockIdx.x split over gridDim.y one-wave workgroups (part q takes chunks
// q, q + gridDim.y, ...), so one block's chains run on many CUs at once;
// k_tree_finish (one wave per block) then runs T_len and the XMSS levels.
template <int ID, int KIND>
__global__ __launch_bounds__(64) void k_tree_chains(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs,
                                                    uint32_t ntrees, uint8_t* sigs, uint32_t* __restrict__ stage,
                                                    uint32_t* __restrict__ spill, uint32_t key_slot,
                                                    uint32_t* root_out, const uint32_t* ulist,
                                                    const uint32_t* ucount, const uint32_t* lown, uint32_t first,
                                                    uint32_t* uroots) {
  const TreeList tl{ulist, ucount, lown, first, uroots};
  if (blockIdx.x * (kLeavesPerBlock >> P<ID>::unit_hp) >= tl.count(ntrees)) return;
  uint32_t* st = stage + size_t(blockIdx.x) * P<ID>::len * kLeavesPerBlock * P<ID>::NW;
  tree_chains<ID, KIND, true>(keys, recs, ntrees, sigs, st, spill, key_slot, root_out, blockIdx.x, tl);
}
template <int ID, int KIND>
__global__ __launch_bounds__(64) void k_tree_finish(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs,
                                                    uint32_t ntrees, uint8_t* sigs, uint32_t* __restrict__ stage,
                                                    uint32_t* __restrict__ spill, uint32_t key_slot,
                                                    uint32_t* root_out, const uint32_t* ulist,
                                                    const uint32_t* ucount, const uint32_t* lown, uint32_t* nodes,
                                                    uint32_t first, uint32_t* uroots) {
  const TreeList tl{ulist, ucount, lown, first, uroots};
  if (blockIdx.x * (kLeavesPerBlock >> P<ID>::unit_hp) >= tl.count(ntrees)) return;
  const uint32_t* st = stage + size_t(blockIdx.x) * P<ID>::len * kLeavesPerBlock * P<ID>::NW;
  tree_finish<ID, KIND>(keys, recs, ntrees, sigs, st, spill, key_slot, root_out, blockIdx.x, tl, nodes);
}

// XMSS trees built in units (the small sets): one lane per tree combines the
// unit roots (level unit_hp) up to the root, writing the authentication
// nodes of those levels for the signing leaf (FIPS 205 Algorithms 9-10).
template <int ID, int KIND>
__global__ void k_tree_top(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs, uint32_t ntrees,
                           uint8_t* sigs, uint32_t key_slot, uint32_t* root_out, uint32_t first,
                           const uint32_t* __restrict__ uroots) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len, UH = Q::unit_hp, HP = Q::hp, UT = Q::tree_units;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntrees) return;
  const uint32_t ft = first + i;
  const TreeJob J = tree_job<ID, KIND>(keys, recs, sigs, nullptr, key_slot, root_out, ft);
  uint32_t lvl[UT * NW];
#pragma unroll
  for (int w = 0; w < UT * NW; w++) lvl[w] = uroots[size_t(ft) * UT * NW + w];
#pragma unroll
  for (int z = UH + 1; z <= HP; z++) {
    const int cnt = 1 << (HP - z);  // nodes of level z
    // auth node of level z-1: the sibling of the signing leaf's ancestor
#pragma unroll
    for (int q = 0; q < 2 * cnt; q++)
      if (J.sig_xmss && uint32_t(q) == ((uint32_t(J.sign_leaf) >> (z - 1)) ^ 1u))
        store_be<NW>(J.sig_xmss + (LEN + z - 1) * Q::n, &lvl[q * NW]);
#pragma unroll
    for (int q = 0; q < cnt; q++) {
      uint32_t out[NW];
      thH<ID>(J.key->mid256, J.key->mid512, make_adrs(J.layer, J.tree, A_TREE, 0, z, q), &lvl[2 * q * NW], out);
#pragma unroll
      for (int u = 0; u < NW; u++) lvl[q * NW + u] = out[u];
    }
  }
  if (J.root_out) store_words<NW>(J.root_out, lvl);
}

// ------------------------------------------------------------------ fused
// Persistent kernel of one parameter set: workgroups take work items from a
// device counter until the list is exhausted.  Items [0, ntb) are TREE
// blocks, items [ntb, ntb + nfg) FORS groups; the long TREE blocks go first
// and the short FORS groups fill the tail.  TREE blocks are software
// pipelined: while all four waves run the chains of block i, wave 0 also
// finishes block i-1 (T_len and the XMSS levels) from the other half of the
// workgroup's double-buffered chain-end staging, so no wave waits for
// another between blocks.  Staging is indexed by the workgroup, so it scales
// with the grid, not the batch.  The counter is zeroed by k_prelude of the
// same batch; every workgroup leaves once the counter passes the end.
//
// wave0_chunks: chunks of an item's chains that wave 0 runs (it also
// finishes the previous item); 0 = TreeSplit's share per block, which
// balances instruction counts.  bpi: TREE blocks per work item (1 or 2):
// the chunks of both blocks of an item are dealt out together, so the
// waves' shares can be balanced more finely.
//
// Waves per SIMD the fused kernel is compiled for (bounds its VGPRs to 168).
// Three for every set: a four-wave build (128 VGPRs, a few spills) ran no
// faster, and the persistent grid gains nothing beyond three workgroups per
// CU.
template <int ID>
struct FusedOcc {
  static constexpr int waves = 3;
};

// NWAV: waves per workgroup, 4 or 2.  A TREE block's chains are dealt to
// the waves in whole chunks (one chain of all 64 leaves), and every item
// ends at a workgroup barrier, so the slowest wave sets an item's time:
// with four waves the three chunk waves share len - w0 chunks evenly only
// when that divides by three (192f: 14 + 13 + 13 against wave 0's 11 +
// finish); with two waves, wave 0's chunks plus the finish and wave 1's
// chunks can be balanced to within half a chunk.  FORS groups of the same
// workgroup use 64 NWAV lanes.
template <int ID, int FG, int LPL = 2, int NWAV = 4>
__global__ __launch_bounds__(64 * NWAV, FusedOcc<ID>::waves) void k_fused(
    const DevKey* __restrict__ keys, WorkRec* __restrict__ recs, uint32_t nmsg, uint8_t* sigs,
    uint32_t* __restrict__ stage, uint32_t* __restrict__ spill, uint32_t* __restrict__ roots, uint32_t* queue,
    uint32_t ntb, uint32_t nfg, const uint32_t* ulist, const uint32_t* ucount, const uint32_t* lown,
    uint32_t* nodes, uint32_t wave0_chunks, uint32_t bpi) {
  static_assert(NWAV == 2 || NWAV == 4, "fused workgroups of 2 or 4 waves");
  using Q = P<ID>;
  constexpr int LEN = Q::len;
  constexpr size_t SW = size_t(LEN) * kLeavesPerBlock * Q::NW;  // words of one block's staging
  __shared__ uint32_t node[FG * ForsLeaves<ID, LPL>::BASE * Q::NW];
  __shared__ uint32_t item;
  uint32_t* st0 = stage + size_t(blockIdx.x) * 2 * bpi * SW;
  const TreeList tl{ulist, ucount, lown, 0u};
  const uint32_t ntrees = nmsg * Q::d;
  constexpr uint32_t TPB = kLeavesPerBlock / Q::leaves;
  if (ucount) ntb = (*ucount + TPB - 1) / TPB;  // TREE blocks over the distinct trees only
  const uint32_t nti = (ntb + bpi - 1) / bpi;   // TREE items of bpi blocks
  const uint32_t total = nti + nfg;
  const int wave = int(threadIdx.x >> 6);
  const bool w0 = wave == 0;
  // this wave's chunks of an item: wave 0 takes 0 .. W0-1, wave k >= 1 takes
  // W0 + (k - 1) + (NWAV - 1) i, over the bpi * len chunks of the item
  const int W0 = wave0_chunks ? int(wave0_chunks) : int(bpi) * TreeSplit<ID, NWAV>::wave0;
  const int cc0 = w0 ? 0 : W0 + wave - 1, ccend = w0 ? W0 : int(bpi) * LEN, ccstep = w0 ? 1 : NWAV - 1;
  uint32_t pend = 0xffffffffu;  // TREE item waiting for its finish (uniform)
  uint32_t cur = 0;             // staging half of the next TREE item (uniform)
  auto finish = [&](uint32_t ti, uint32_t* st) {
    for (uint32_t b = 0; b < bpi && ti * bpi + b < ntb; b++)
      tree_finish<ID, kSignTrees>(keys, recs, ntrees, sigs, st + b * SW, spill, 0u, nullptr, ti * bpi + b, tl, nodes);
  };
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t it = item;
    __syncthreads();  // everyone holds `it` before thread 0 may overwrite `item`
    if (it >= total) break;
    if (pend != 0xffffffffu) {
      // finish the previous TREE item while the other waves start this item
      if (w0) finish(pend, st0 + (cur ^ 1) * bpi * SW);
      pend = 0xffffffffu;
    }
    if (it < nti) {
      uint32_t* st = st0 + cur * bpi * SW;
      for (uint32_t b = 0; b < bpi && it * bpi + b < ntb; b++) {
        // this wave's chunks inside block b: the part of its sequence in
        // [b len, (b + 1) len), shifted to the block's own chunk numbers
        const int lo = int(b) * LEN, hi = lo + LEN;
        const int first = cc0 >= lo ? cc0 : cc0 + ((lo - cc0 + ccstep - 1) / ccstep) * ccstep;
        const int end = ccend < hi ? ccend : hi;
        if (first < end)
          tree_chains<ID, kSignTrees, false, NWAV>(keys, recs, ntrees, sigs, st + b * SW, spill, 0u, nullptr,
                                                   it * bpi + b, tl, 0, first - lo, end - lo, ccstep);
      }
      pend = it;
      cur ^= 1;
    } else {
      fors_group<ID, FG, LPL, 64 * NWAV>(keys, recs, nmsg * Q::k, sigs, roots, it - nti, node);
    }
  }
  if (pend != 0xffffffffu && w0) finish(pend, st0 + (cur ^ 1) * bpi * SW);
}

// The fused kernel scheduled per chains chunk.  Workgroups take TREE blocks
// one at a time from a device counter (queue[2]); inside a block the four
// waves take its chains chunks one at a time from a counter in LDS, so a
// wave that is slower (it finished the previous block, or shares its SIMD
// with older waves, which the SIMD's arbiter serves first) simply takes
// fewer, and workgroups that run slower take fewer blocks.  A barrier ends
// each block; after it, one wave (rotating with the block) finishes that
// block (T_len and the XMSS levels) from its half of the workgroup's
// double-buffered staging while the other waves start the next block's
// chunks.  The FORS groups follow from the device counter queue[0].
template <int ID, int FG, int LPL = 2>
__global__ __launch_bounds__(256, FusedOcc<ID>::waves) void k_fused_chunks(
    const DevKey* __restrict__ keys, WorkRec* __restrict__ recs, uint32_t nmsg, uint8_t* sigs,
    uint32_t* __restrict__ stage, uint32_t* __restrict__ spill, uint32_t* __restrict__ roots, uint32_t* queue,
    uint32_t ntb, uint32_t nfg, const uint32_t* ulist, const uint32_t* ucount, const uint32_t* lown,
    uint32_t* nodes) {
  using Q = P<ID>;
  constexpr uint32_t LEN = Q::len;
  constexpr int NW = Q::NW, LV = Q::leaves;
  constexpr size_t SW = size_t(LEN) * kLeavesPerBlock * NW;  // words of one block's staging
  __shared__ uint32_t node[FG * ForsLeaves<ID, LPL>::BASE * NW];
  __shared__ uint32_t next, item;
  const TreeList tl{ulist, ucount, lown, 0u};
  const uint32_t ntrees = nmsg * Q::d;
  constexpr uint32_t TPB = kLeavesPerBlock / Q::leaves;
  if (ucount) ntb = (*ucount + TPB - 1) / TPB;  // TREE blocks over the distinct trees only
  const int lane = int(threadIdx.x & 63), wave = int(threadIdx.x >> 6);
  uint32_t* st0 = stage + size_t(blockIdx.x) * 2 * SW;
  auto take = [&]() -> uint32_t {
    uint32_t v = 0;
    if (lane == 0) v = atomicAdd(&next, 1u);
    return __shfl(v, 0, 64);
  };
  uint32_t prev = 0xffffffffu;  // the block finished after the next barrier
  uint32_t cur = 0;             // staging half of the next block
  for (;;) {
    if (threadIdx.x == 0) {
      item = atomicAdd(queue + 2, 1u);
      next = 0u;
    }
    __syncthreads();  // the new block is known, and every chunk of the previous one is written
    const uint32_t b = item;
    if (prev != 0xffffffffu && wave == int(prev & 3u))
      tree_finish<ID, kSignTrees>(keys, recs, ntrees, sigs, st0 + (cur ^ 1u) * SW, spill, 0u, nullptr, prev, tl,
                                  nodes);
    if (b >= ntb) break;
    uint32_t* st = st0 + cur * SW;
    uint32_t i = take();
    if (i < LEN) {
      // the lane's leaf of block b and its chain inputs, kept over this
      // wave's chunks of the block
      const uint32_t lt = uint32_t(lane) / LV, kp = uint32_t(lane) % LV;
      const bool valid = b * TPB + lt < tl.count(ntrees);
      const uint32_t ft = valid ? tl.at(b * TPB + lt) : 0u;
      const TreeJob J = sign_job<ID>(keys, recs, sigs, spill, ft);
      uint32_t mid[8], sks[NW];
      load_words<8>(J.key->mid256, mid);
      load_words<NW>(J.key->sk_seed, sks);
      uint32_t* keep = nullptr;
      if (lown) {
        const uint32_t o = lown[size_t(ft) * Q::leaves + kp];
        if (spill && o != 0xffffffffu) keep = spill + size_t(o) * LEN * 16 * NW;
      } else if (J.spill && int32_t(kp) == J.sign_leaf) {
        keep = J.spill;
      }
      do {
        if (valid) {
          uint32_t x[NW];
          wots_chain<ID>(mid, sks, J.layer, J.tree, kp, i, keep ? keep + i * 16 * NW : nullptr, x);
          store_words<NW>(st + (i * kLeavesPerBlock + lane) * NW, x);
        }
        i = take();
      } while (i < LEN);
    }
    prev = b;
    cur ^= 1u;
    __syncthreads();  // every chunk of b is written; everyone holds b before item changes
  }
  __syncthreads();
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t it = item;
    __syncthreads();  // everyone holds `it` before thread 0 may overwrite `item`
    if (it >= nfg) break;
    fors_group<ID, FG, LPL, 256>(keys, recs, nmsg * Q::k, sigs, roots, it, node);
  }
}

// ------------------------------------------------------------------ WOTS
// One lane per (message, layer, chain): digit of the layer's message (see
// wots_digit), then the chain value at that digit.

// Chain c of the signing leaf of job J advanced `digit` steps from its PRF
// secret (FIPS 205 Algorithms 5 and 7).
template <int ID>
__device__ __forceinline__ void wots_value(const TreeJob& J, uint32_t c, uint32_t digit, uint32_t x[P<ID>::NW]) {
  constexpr int NW = P<ID>::NW;
  uint32_t mid[8], sks[NW];
  load_words<8>(J.key->mid256, mid);
  load_words<NW>(J.key->sk_seed, sks);
  const uint32_t kp = uint32_t(J.sign_leaf);
  thF<ID>(mid, make_adrs(J.layer, J.tree, A_WOTS_PRF, kp, c, 0), sks, x);
  Adrs A = make_adrs(J.layer, J.tree, A_WOTS_HASH, kp, c, 0);
  for (uint32_t st = 0; st < digit; st++) {
    A.tail = st << 16;
    uint32_t y[NW];
    thF<ID>(mid, A, x, y);
#pragma unroll
    for (int u = 0; u < NW; u++) x[u] = y[u];
  }
}

// Gather from the kept chain values of the signing leaves.
template <int ID>
__global__ void k_wots(const WorkRec* __restrict__ recs, uint32_t count, uint8_t* sigs,
                       const uint32_t* __restrict__ spill) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t total = count * Q::d * LEN;
  if (gid >= total) return;
  const uint32_t ftree = gid / LEN, c = gid - ftree * LEN;
  const uint32_t msg = ftree / Q::d, layer = ftree - msg * Q::d;
  const WorkRec& W = recs[msg];
  const uint32_t digit = wots_digit<ID>(W, layer, c);
  const uint32_t* src = spill + ((size_t(ftree) * LEN + c) * 16 + digit) * NW;
  uint32_t v[NW];
  load_words<NW>(src, v);
  store_be<NW>(sigs + W.sig_off + Q::ht_off + size_t(layer) * Q::xmss_bytes + c * Q::n, v);
}

// WOTS+ signatures recomputed instead of gathered (for contexts that do not
// keep the chain values of the signing leaves): one lane per chain runs PRF
// and then `digit` F steps.
template <int ID>
__global__ void k_wots_recompute(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs,
                                 uint32_t count, uint8_t* sigs) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t total = count * Q::d * LEN;
  if (gid >= total) return;
  const uint32_t ftree = gid / LEN, c = gid - ftree * LEN;
  const TreeJob J = sign_job<ID>(keys, recs, sigs, nullptr, ftree);
  uint32_t x[NW];
  wots_value<ID>(J, c, wots_digit<ID>(recs[ftree / Q::d], J.layer, c), x);
  store_be<NW>(J.sig_xmss + c * Q::n, x);
}

// ------------------------------------------------------------------ dedup
// Within-batch dedup of XMSS trees.  Two (message, layer) pairs whose key,
// layer and tree address agree need the same tree; only the one with the
// smallest flat tree id (the representative) computes it.  Layers whose tree
// address has at most 35 bits are eligible, so that key slot (24 bits), layer
// (5 bits) and tree address form one exact 64-bit key; a repeat of a wider
// address within one batch has probability below 2^-10 per batch of 2^12.
// The map is an open-addressing table of 2^k >= 2 entries per tree.
struct DedupSlot {
  unsigned long long key;
  uint32_t owner;
  uint32_t pad;
};
constexpr unsigned long long kDedupEmpty = ~0ull;

static __global__ void k_dedup_init(DedupSlot* table, uint32_t size, uint32_t* lown, uint32_t nlown, uint32_t* ucount) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < size) {
    table[i].key = kDedupEmpty;
    table[i].owner = 0xffffffffu;
  }
  if (i < nlown) lown[i] = 0xffffffffu;
  if (i == 0) *ucount = 0;
}

__device__ __forceinline__ uint32_t dedup_hash(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return uint32_t(k);
}

// Marks a (message, layer) pair whose tree sits in its key's tree cache.
constexpr uint32_t kCachedTree = 0xfffffffeu;

// rep[ft] <- table slot of its triple, 0xffffffff when not eligible, or
// kCachedTree when the key caches the layer.
template <int ID>
__global__ void k_dedup_insert(const DevKey* __restrict__ keys, const WorkRec* __restrict__ recs, uint32_t nmsg,
                               DedupSlot* table, uint32_t size, uint32_t* rep) {
  using Q = P<ID>;
  const uint32_t ft = blockIdx.x * blockDim.x + threadIdx.x;
  if (ft >= nmsg * Q::d) return;
  const uint32_t msg = ft / Q::d, layer = ft - msg * Q::d;
  const WorkRec& W = recs[msg];
  if (layer + keys[W.key_slot].cache_layers >= uint32_t(Q::d)) {
    rep[ft] = kCachedTree;
    return;
  }
  const int bits = Q::tree_bits - int(Q::hp * layer);  // bits of this layer's tree address
  if (bits > 35 || W.key_slot >= (1u << 24)) {
    rep[ft] = 0xffffffffu;
    return;
  }
  const uint32_t sh = Q::hp * layer;
  const unsigned long long tree = sh >= 64 ? 0ull : (W.idx_tree >> sh);
  const unsigned long long key = (unsigned long long)W.key_slot << 40 | (unsigned long long)layer << 35 | tree;
  uint32_t h = dedup_hash(key) & (size - 1);
  for (uint32_t probe = 0; probe < size; probe++) {
    const unsigned long long prev = atomicCAS(&table[h].key, kDedupEmpty, key);
    if (prev == kDedupEmpty || prev == key) {
      atomicMin(&table[h].owner, ft);
      rep[ft] = h;
      return;
    }
    h = (h + 1) & (size - 1);
  }
  rep[ft] = 0xffffffffu;  // table full (cannot happen at 2 entries per tree): compute it alone
}

// rep[ft] <- representative flat tree id; representatives are appended to
// ulist (order irrelevant: every output position is fixed by the tree id);
// the smallest pair signing with each leaf of a representative becomes that
// leaf's owner in lown.
template <int ID>
__global__ void k_dedup_resolve(const WorkRec* __restrict__ recs, uint32_t nmsg, const DedupSlot* table,
                                uint32_t* rep, uint32_t* ulist, uint32_t* ucount, uint32_t* lown) {
  using Q = P<ID>;
  const uint32_t ft = blockIdx.x * blockDim.x + threadIdx.x;
  if (ft >= nmsg * Q::d) return;
  const uint32_t h = rep[ft];
  if (h == kCachedTree) return;
  const uint32_t r = h == 0xffffffffu ? ft : table[h].owner;
  rep[ft] = r;
  if (r == ft) ulist[atomicAdd(ucount, 1u)] = ft;
  const uint32_t msg = ft / Q::d, layer = ft - msg * Q::d;
  const WorkRec& W = recs[msg];
  const uint32_t leaf = layer == 0 ? W.idx_leaf
                                   : uint32_t((W.idx_tree >> (Q::hp * (layer - 1))) & ((1u << Q::hp) - 1));
  atomicMin(&lown[size_t(r) * Q::leaves + leaf], ft);
}

// Running totals of eligible-or-not trees and distinct trees computed (one
// lane; stream order makes plain adds safe).
static __global__ void k_dedup_stats(uint32_t trees, const uint32_t* ucount, unsigned long long* stats) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stats[0] += trees;
    stats[1] += *ucount;
  }
}

// Auth path and root of every non-representative (message, layer) from the
// representative's node buffer; one lane per pair.
// Cached pairs read the key's tree cache instead.
template <int ID>
__global__ void k_dedup_scatter(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs, uint32_t nmsg,
                                uint8_t* sigs, const uint32_t* __restrict__ rep, const uint32_t* __restrict__ nodes,
                                const uint8_t* __restrict__ cache) {
  using Q = P<ID>;
  constexpr int NW = Q::NW;
  const uint32_t ft = blockIdx.x * blockDim.x + threadIdx.x;
  if (ft >= nmsg * Q::d) return;
  const uint32_t r = rep[ft];
  if (r == ft) return;
  const TreeJob J = sign_job<ID>(keys, recs, sigs, nullptr, ft);
  const uint32_t leaf = uint32_t(J.sign_leaf);
  const uint32_t* tn;
  if (r == kCachedTree) {
    const uint64_t t = CacheShape<ID>::layer_first(Q::d - 1 - J.layer) + J.tree;
    tn = reinterpret_cast<const uint32_t*>(cache + J.key->cache_off) + t * TreeNodes<ID>::count * NW;
  } else {
    tn = nodes + size_t(r) * TreeNodes<ID>::count * NW;
  }
  uint8_t* xs = J.sig_xmss + Q::len * Q::n;
  for (int z = 0; z < Q::hp; z++) {
    uint32_t v[NW];
    load_words<NW>(tn + (TreeNodes<ID>::off(z) + ((leaf >> z) ^ 1u)) * NW, v);
    store_be<NW>(xs + z * Q::n, v);
  }
  if (J.root_out) {
    uint32_t v[NW];
    load_words<NW>(tn + TreeNodes<ID>::off(Q::hp) * NW, v);
    store_words<NW>(J.root_out, v);
  }
}

// WOTS+ signatures with dedup: the chains of every leaf some pair signs with
// were kept (in the area of that leaf's owner), so every computed pair
// gathers; pairs of cached layers recompute their chains.
template <int ID>
__global__ void k_wots_dedup(const DevKey* __restrict__ keys, WorkRec* __restrict__ recs, uint32_t count,
                             uint8_t* sigs, const uint32_t* __restrict__ spill, const uint32_t* __restrict__ rep,
                             const uint32_t* __restrict__ lown) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= count * Q::d * LEN) return;
  const uint32_t ftree = gid / LEN, c = gid - ftree * LEN;
  const TreeJob J = sign_job<ID>(keys, recs, sigs, nullptr, ftree);
  const uint32_t digit = wots_digit<ID>(recs[ftree / Q::d], J.layer, c);
  const uint32_t r = rep[ftree];
  uint32_t x[NW];
  if (r == kCachedTree) {
    wots_value<ID>(J, c, digit, x);
  } else {
    const uint32_t o = lown[size_t(r) * Q::leaves + uint32_t(J.sign_leaf)];
    load_words<NW>(spill + ((size_t(o) * LEN + c) * 16 + digit) * NW, x);
  }
  store_be<NW>(J.sig_xmss + c * Q::n, x);
}

// ------------------------------------------------------------------ verify
// Batched verification (FIPS 205 Algorithm 20).  A group of G lanes (16: a
// quarter of a wave; 32 for batches too small to give every SIMD a wave at
// 16) verifies one signature; a workgroup of 256 lanes holds 256 / G
// signatures:
//   setup   : the group's first lane derives the per-key chaining values,
//             recomputes the digest (H_msg) and splits it;
//   FORS    : one lane per FORS tree (trees g, g + G, ...) climbs from the
//             revealed secret value to the root; the first lane runs T_k;
//   layers  : per hypertree layer, the len WOTS+ chains are spread over the
//             G lanes, longest first in a snake order (rank r goes to lane
//             r mod G, reversed on odd rounds), so that every lane has about
//             the same number of F steps; each lane works through its chains
//             step by step; the first lane then runs T_len and climbs the
//             h' authentication levels to the layer's root.  The next
//             lanes load that layer's h' authentication nodes into LDS while
//             the chains start, so the climb does not wait for memory.
// A group never spans two waves, and its lanes share only LDS slots of
// their own group, so the phases are separated by wave-local ordering
// (wave_sync) rather than workgroup barriers: each wave moves on as soon as
// its own four (or two) signatures are done with a phase, instead of
// waiting for the slowest signature of the workgroup.
// The result (1 valid, 0 invalid) is written to results[res_idx].  V: the
// instruction variant of the chain, tree and T_l hashes (sha2_dev.hpp).
struct VerifyItem {
  uint64_t msg_off, msg_len, sig_off, pk_off, res_idx;
};
constexpr int kVerifyThreads = 256;
constexpr int kVerifyGroup = 16;      // lanes per signature for large batches
constexpr int kVerifyGroupWide = 32;  // lanes per signature up to kVerifyWideMax signatures
constexpr uint32_t kVerifyWideMax = 2048;

__device__ __forceinline__ uint32_t load_be32(const uint8_t* p) {
  return (uint32_t(p[0]) << 24) | (uint32_t(p[1]) << 16) | (uint32_t(p[2]) << 8) | uint32_t(p[3]);
}
template <int NW>
__device__ __forceinline__ void load_be(const uint8_t* p, uint32_t* v) {
#pragma unroll
  for (int i = 0; i < NW; i++) v[i] = load_be32(p + 4 * i);
}
// The same from a 4-byte aligned address as dword loads (`aligned`), else
// byte by byte.
template <int NW>
__device__ __forceinline__ void load_be_any(const uint8_t* p, bool aligned, uint32_t* v) {
  if (aligned) {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int i = 0; i < NW; i++) v[i] = __builtin_bswap32(q[i]);
  } else {
    load_be<NW>(p, v);
  }
}

// Orders the LDS accesses of one wave: the lanes of a wave execute in
// lockstep and a wave's LDS operations complete in issue order, so a
// compiler fence around the wave barrier is all that separates a phase's
// LDS writes from the next phase's reads by other lanes of the same wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Base-16 digit of WOTS+ chain c for message words M (len1 message digits,
// then the three checksum digits of csum << 4), FIPS 205 Algorithm 7.
template <int ID>
__device__ __forceinline__ uint32_t verify_digit(const uint32_t* M, uint32_t csum, uint32_t c) {
  if (c < uint32_t(P<ID>::len1)) return (M[c >> 3] >> (28 - 4 * (c & 7))) & 15u;
  return (csum >> (12 - 4 * (c - P<ID>::len1))) & 15u;
}

template <int ID, int G, int V = 0>
__global__ __launch_bounds__(kVerifyThreads) void k_verify(const VerifyItem* __restrict__ items,
                                                          uint32_t count, const uint8_t* msgs,
                                                          const uint8_t* sigs, const uint8_t* pks,
                                                          int* results) {
  using Q = P<ID>;
  constexpr int NW = Q::NW, LEN = Q::len, KT = Q::k, A = Q::a, HP = Q::hp, kVerifySigs = kVerifyThreads / G;
  constexpr int SLOTS = (LEN + G - 1) / G;
  static_assert(KT <= 64, "FORS indices per signature");
  static_assert(64 % G == 0, "a verify group lies inside one wave");
  static_assert(HP < G, "one loading lane per authentication node");
  __shared__ uint32_t s_vals[kVerifySigs][(LEN > KT ? LEN : KT) * NW];
  __shared__ uint32_t s_auth[kVerifySigs][HP * NW];
  __shared__ uint16_t s_order[kVerifySigs][SLOTS * G];
  __shared__ uint16_t s_idx[kVerifySigs][64];
  __shared__ uint32_t s_mid256[kVerifySigs][8], s_mid512[kVerifySigs][16], s_root[kVerifySigs][8];
  __shared__ uint32_t s_cur[kVerifySigs][8];
  __shared__ uint64_t s_tree[kVerifySigs];
  __shared__ uint32_t s_leaf[kVerifySigs];
  const int tid = threadIdx.x, grp = tid / G, g = tid % G;
  const uint32_t sidx = blockIdx.x * kVerifySigs + grp;
  const bool valid = sidx < count;
  const VerifyItem it = valid ? items[sidx] : VerifyItem{0, 0, 0, 0, 0};
  const uint8_t* sig = sigs + it.sig_off;
  const bool al = (reinterpret_cast<uintptr_t>(sig) & 3) == 0;  // every signature part is then aligned
  uint32_t* vals = s_vals[grp];
  // ---- setup
  if (valid && g == 0) {
    uint32_t pk_seed[8] = {0}, pk_root[8] = {0};
    load_be<NW>(pks + it.pk_off, pk_seed);
    load_be<NW>(pks + it.pk_off + Q::n, pk_root);
    if constexpr (Q::shake) {
#pragma unroll
      for (int j = 0; j < 8; j++) s_mid256[grp][j] = pk_seed[j];
    } else {
      uint32_t st[8], w[16];
      sha256_iv(st);
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = j < NW ? pk_seed[j] : 0u;
      sha256_compress(st, w);
#pragma unroll
      for (int j = 0; j < 8; j++) s_mid256[grp][j] = st[j];
    }
    if constexpr (Q::wide) {
      u64p s5[8], w5[16];
      sha512_iv(s5);
#pragma unroll
      for (int j = 0; j < 16; j++)
        w5[j] = u64p{2 * j < NW ? pk_seed[2 * j] : 0u, 2 * j + 1 < NW ? pk_seed[2 * j + 1] : 0u};
      sha512_compress(s5, w5);
#pragma unroll
      for (int j = 0; j < 8; j++) { s_mid512[grp][2 * j] = s5[j].hi; s_mid512[grp][2 * j + 1] = s5[j].lo; }
    }
#pragma unroll
    for (int j = 0; j < 8; j++) s_root[grp][j] = pk_root[j];
    uint32_t R[NW], digest[16];
    load_be_any<NW>(sig, al, R);
    const KeyView kv{nullptr, pk_seed, pk_root, nullptr};
    h_msg<ID>(kv, R, msgs + it.msg_off, it.msg_len, digest);
    uint64_t tree;
    uint32_t leaf;
    split_digest<ID>(digest, s_idx[grp], &tree, &leaf);
    s_tree[grp] = tree;
    s_leaf[grp] = leaf;
  }
  wave_sync();
  uint32_t mid256[8], mid512[16];
#pragma unroll
  for (int j = 0; j < 8; j++) mid256[j] = s_mid256[grp][j];
#pragma unroll
  for (int j = 0; j < 16; j++) mid512[j] = Q::wide ? s_mid512[grp][j] : 0u;
  uint64_t tree = s_tree[grp];
  uint32_t leaf = s_leaf[grp];
  // ---- FORS: roots of trees g, g + G, ...
  if (valid) {
    for (int t = g; t < KT; t += G) {
      const uint8_t* ts = sig + Q::n + t * (A + 1) * Q::n;
      const uint32_t idx = s_idx[grp][t];
      uint32_t x[NW], y[NW], lr[2 * NW];
      load_be_any<NW>(ts, al, x);
      uint32_t gi = (uint32_t(t) << A) + idx;
      thF<ID, V>(mid256, make_adrs(0, tree, A_FORS_TREE, leaf, 0, gi), x, y);
      for (int j = 0; j < A; j++) {
        uint32_t au[NW];
        load_be_any<NW>(ts + (1 + j) * Q::n, al, au);
        const bool even = ((idx >> j) & 1u) == 0;
#pragma unroll
        for (int u = 0; u < NW; u++) {
          lr[u] = even ? y[u] : au[u];
          lr[NW + u] = even ? au[u] : y[u];
        }
        gi >>= 1;
        thH<ID, V>(mid256, mid512, make_adrs(0, tree, A_FORS_TREE, leaf, j + 1, gi), lr, y);
      }
      store_words<NW>(&vals[t * NW], y);
    }
  }
  wave_sync();
  if (valid && g == 0) {
    auto get = [&](int wi) -> uint32_t { return vals[wi]; };
    uint32_t pk[NW];
    thT<ID, KT, V>(mid256, mid512, make_adrs(0, tree, A_FORS_ROOTS, leaf, 0, 0), get, pk);
    store_words<NW>(s_cur[grp], pk);
  }
  wave_sync();
  const uint8_t* ht = sig + Q::ht_off;
  for (int layer = 0; layer < Q::d; layer++) {
    const uint8_t* xs = ht + layer * Q::xmss_bytes;
    uint32_t M[NW];
#pragma unroll
    for (int u = 0; u < NW; u++) M[u] = s_cur[grp][u];
    uint32_t csum = 0;
#pragma unroll
    for (int i = 0; i < Q::len1; i++) csum += 15u - ((M[i >> 3] >> (28 - 4 * (i & 7))) & 15u);
    csum <<= 4;  // (8 - (len2 * lg_w) mod 8) mod 8 = 4 for len2 = 3
    if (valid) {
      // lanes 1..h' fetch the layer's authentication nodes for the climb
      if (g >= 1 && g <= HP) {
        uint32_t au[NW];
        load_be_any<NW>(xs + (LEN + g - 1) * Q::n, al, au);
        store_words<NW>(&s_auth[grp][(g - 1) * NW], au);
      }
      // chain start values (the signature's WOTS+ part) into LDS, and the
      // rank of each of this lane's home chains by descending step count
      for (int c = g; c < LEN; c += G) {
        uint32_t x[NW];
        load_be_any<NW>(xs + c * Q::n, al, x);
        store_words<NW>(&vals[c * NW], x);
        const uint32_t sc = 15u - verify_digit<ID>(s_cur[grp], csum, c);
        uint32_t rank = 0;
#pragma unroll
        for (int c2 = 0; c2 < LEN; c2++) {
          const uint32_t s2 = 15u - verify_digit<ID>(M, csum, c2);
          rank += (s2 > sc || (s2 == sc && c2 < c)) ? 1u : 0u;
        }
        s_order[grp][rank] = uint16_t(c);
      }
    }
    wave_sync();
    if (valid) {
      // this lane's chains: ranks g, 2G - 1 - g, 2G + g, ... (snake order)
      int slot = 0;
      int c = -1;
      uint32_t st = 15, x[NW];
      for (;;) {
        while (st == 15) {
          if (c >= 0) store_words<NW>(&vals[c * NW], x);
          c = -1;
          if (slot >= SLOTS) break;
          const int r = slot * G + ((slot & 1) ? G - 1 - g : g);
          slot++;
          if (r >= LEN) continue;
          c = s_order[grp][r];
          st = verify_digit<ID>(s_cur[grp], csum, uint32_t(c));
#pragma unroll
          for (int u = 0; u < NW; u++) x[u] = vals[c * NW + u];
        }
        if (c < 0) break;
        Adrs Ad = make_adrs(layer, tree, A_WOTS_HASH, leaf, uint32_t(c), 0);
        Ad.tail = st << 16;
        uint32_t y[NW];
        thF<ID, V>(mid256, Ad, x, y);
#pragma unroll
        for (int u = 0; u < NW; u++) x[u] = y[u];
        st++;
      }
    }
    wave_sync();
    if (valid && g == 0) {
      auto get = [&](int wi) -> uint32_t { return vals[wi]; };
      uint32_t node[NW], lr[2 * NW];
      thT<ID, LEN, V>(mid256, mid512, make_adrs(layer, tree, A_WOTS_PK, leaf, 0, 0), get, node);
      uint32_t ti = leaf;
      for (int j = 0; j < HP; j++) {
        uint32_t au[NW];
        load_words<NW>(&s_auth[grp][j * NW], au);
        const bool even = (ti & 1u) == 0;
#pragma unroll
        for (int u = 0; u < NW; u++) {
          lr[u] = even ? node[u] : au[u];
          lr[NW + u] = even ? au[u] : node[u];
        }
        ti >>= 1;
        thH<ID, V>(mid256, mid512, make_adrs(layer, tree, A_TREE, 0, j + 1, ti), lr, node);
      }
      store_words<NW>(s_cur[grp], node);
    }
    wave_sync();
    leaf = uint32_t(tree & ((1u << Q::hp) - 1));
    tree = Q::hp >= 64 ? 0 : (tree >> Q::hp);
  }
  if (valid && g == 0) {
    bool ok = true;
#pragma unroll
    for (int u = 0; u < NW; u++) ok = ok && (s_cur[grp][u] == s_root[grp][u]);
    results[it.res_idx] = ok ? 1 : 0;
  }
}

}  // namespace slh
