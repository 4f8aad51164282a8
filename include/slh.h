/*
 * slh.h -- C ABI of the MI355X (gfx950) batched SPHINCS+ signing library.
 *
 * What the library computes.  SPHINCS+ signature generation as accelerated by
 * the HERO-Sign paper (arXiv 2512.23969): its Section II-A describes the
 * scheme (WOTS+, FORS, XMSS trees, hypertree), Table 1 the -f parameter sets
 * and the Fig. 2 listing the signing flow.  The exact arithmetic is that of
 * FIPS 205 (SLH-DSA) with the SHA2 "simple" tweakable hashes (FIPS 205
 * Section 11.2): keygen is slh_keygen_internal (Algorithm 18), signing is
 * slh_sign_internal (Algorithm 19) with opt_rand = PK.seed (deterministic
 * signing, no context prefix: the raw message M is signed), verification is
 * slh_verify_internal (Algorithm 20).  The SHAKE sets (ids 7..12) use the
 * SHAKE256 instantiation of FIPS 205 Section 11.1 on the same trees.
 *
 * Parameter sets (the paper's Table 1; the small sets from FIPS 205 Table 2):
 *   SLH_SHA2_128F  n=16 h=66 d=22 a=6 k=33 w=16   signature 17088 bytes
 *   SLH_SHA2_192F  n=24 h=66 d=22 a=8 k=33 w=16   signature 35664 bytes
 *   SLH_SHA2_256F  n=32 h=68 d=17 a=9 k=35 w=16   signature 49856 bytes
 *   SLH_SHA2_128S  n=16 h=63 d=7  a=12 k=14 w=16  signature  7856 bytes
 *   SLH_SHA2_192S  n=24 h=63 d=7  a=14 k=17 w=16  signature 16224 bytes
 *   SLH_SHA2_256S  n=32 h=64 d=8  a=14 k=22 w=16  signature 29792 bytes
 *   SLH_SHAKE_*    the same six shapes and sizes with SHAKE256
 *
 * Byte encodings are those of FIPS 205:
 *   seed = SK.seed | SK.prf | PK.seed                 (3n bytes)
 *   pk   = PK.seed | PK.root                          (2n bytes)
 *   sk   = SK.seed | SK.prf | PK.seed | PK.root       (4n bytes)
 *   sig  = R | SIG_FORS | SIG_HT                      (sizes above)
 *
 * Conventions.
 *   - Return value: SLH_OK (0) or a negative error code.  Arguments are
 *     validated on the host before anything is launched; on SLH_EINVAL
 *     nothing has been written.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are device
 *     memory of the context's GPU (for example torch tensors' data_ptr()).
 *   - The caller owns every buffer it passes.  The library keeps no caller
 *     pointer after a call's work has completed on its stream.
 *   - Calls that take a stream enqueue their GPU work on it and return
 *     without waiting; results are ready when the stream has reached the
 *     point of the call.  Calls on one context are serialised by the
 *     library across streams.
 *   - A context is not thread safe: one host thread at a time per context.
 */
#ifndef SLH_H
#define SLH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameter sets: the SHA2 "fast" sets the paper evaluates (its Table 1)
 * and the SHA2 "small" sets (FIPS 205 Table 2; h' = 8-9, FORS trees of
 * 2^12-2^14 leaves, built on the GPU in units of 64 XMSS leaves and 2^12
 * FORS leaves), then the same six shapes with the SHAKE256 hashes of FIPS
 * 205 Section 11.1 (SLH_SHAKE_*: F, H, T_l, PRF = SHAKE256(PK.seed | ADRS |
 * ..., 8n) over the full 32-byte address; PRF_msg and H_msg are SHAKE256 of
 * the concatenated inputs).  SLH_MODE_FUSED, SLH_MODE_DEDUP and
 * slh_ctx_cache_keys apply to the fast sets (1-3, 7-9); small-set requests
 * always take the per-phase path. */
#define SLH_SHA2_128F 1u
#define SLH_SHA2_192F 2u
#define SLH_SHA2_256F 3u
#define SLH_SHA2_128S 4u
#define SLH_SHA2_192S 5u
#define SLH_SHA2_256S 6u
#define SLH_SHAKE_128F 7u
#define SLH_SHAKE_192F 8u
#define SLH_SHAKE_256F 9u
#define SLH_SHAKE_128S 10u
#define SLH_SHAKE_192S 11u
#define SLH_SHAKE_256S 12u

#define SLH_OK 0
#define SLH_EINVAL (-1)  /* bad parameter set, slot, size, offset or null pointer */
#define SLH_ENOMEM (-2)  /* device memory could not be obtained within the budget */
#define SLH_EDEVICE (-3) /* a HIP call failed; slh_last_error() has the text      */
#define SLH_EBUSY (-4)   /* admission refused (serving queue full)               */

/* Sizes of a parameter set. */
typedef struct {
    uint32_t n;          /* security parameter, bytes */
    uint32_t h, d, hp;   /* hypertree height, layers, XMSS tree height h/d */
    uint32_t a, k;       /* FORS tree height, number of FORS trees */
    uint32_t len;        /* WOTS+ chains per key (len1 + len2) */
    uint32_t m;          /* digest bytes taken from H_msg */
    uint32_t seed_bytes; /* 3n */
    uint32_t pk_bytes;   /* 2n */
    uint32_t sk_bytes;   /* 4n */
    uint32_t sig_bytes;  /* n (1 + k (a + 1) + h + d len) */
} slh_sizes;

/* One signing request of a batch (32 bytes, host memory).
 *   param     parameter set of the request; must equal the key slot's set
 *   key_slot  slot returned by slh_ctx_add_keys
 *   msg_off   byte offset of the message in the batch's message buffer
 *   msg_len   message length in bytes (any length, 0 allowed)
 *   sig_off   byte offset of the signature in the batch's signature buffer;
 *             must be a multiple of 16 */
typedef struct {
    uint32_t param;
    uint32_t key_slot;
    uint64_t msg_off;
    uint64_t msg_len;
    uint64_t sig_off;
} slh_item;

typedef struct slh_ctx slh_ctx;

/* Execution modes of slh_sign_batch (bit flags).  Every mode produces the
 * same bytes.
 *   SLH_MODE_PLAIN  per-phase kernels (prelude, FORS, TREE, FORS pk, WOTS)
 *                   launched one after another on the caller's stream.
 *   SLH_MODE_FUSED  FORS and TREE work of each parameter set in one
 *                   persistent kernel fed by a device work counter; the
 *                   parameter sets of a mixed batch run concurrently on
 *                   branch streams joined back into the caller's stream.
 *   SLH_MODE_GRAPH  the launch sequence is captured once into a hipGraph
 *                   (per batch shape, buffers and tuning) and replayed with a
 *                   single hipGraphLaunch; combine with SLH_MODE_FUSED for the
 *                   batched fused pipeline.  Per-phase timing is not recorded
 *                   inside graphs.  A context keeps up to 8 graphs and
 *                   drops them all when keys are added, tuning changes, or
 *                   its working memory, staging or tree cache is reallocated.
 *   SLH_MODE_DEDUP  within-batch dedup of XMSS trees (combines with the
 *                   others): messages of one key whose hypertree paths share
 *                   a tree at some layer (FIPS 205 Algorithm 12: the layer's
 *                   tree address idx_tree >> (j h')) compute that tree once;
 *                   the others take its authentication path and root from a
 *                   node buffer, and the chains of every leaf that some
 *                   message signs with are kept, so WOTS+ stays a gather.
 *                   Only layers whose tree address has at most 35 bits are
 *                   matched (wider addresses practically never repeat within
 *                   a batch).  Costs (2^(h'+1) - 1) n + 4 * 2^h' + 40 bytes
 *                   of working memory per tree or less. */
#define SLH_MODE_PLAIN 0u
#define SLH_MODE_FUSED 1u
#define SLH_MODE_GRAPH 2u
#define SLH_MODE_DEDUP 4u

/* Fill *out with the sizes of parameter set `param`.
 * Errors: SLH_EINVAL for an unknown set or a null pointer. */
int slh_params(uint32_t param, slh_sizes *out);

/* Create a signing context on GPU `device`.  `hbm_budget` caps the bytes of
 * working memory the context keeps on the device (0 = default of 8 GiB),
 * split evenly over the parameter sets it holds keys of; larger batches are
 * processed in chunks that fit.
 * Errors: SLH_EINVAL (null out, bad device), SLH_EDEVICE. */
int slh_ctx_create(int device, uint64_t hbm_budget, slh_ctx **out);

/* Release a context and all its device memory.  Waits for its pending work.
 * A null context is accepted and ignored. */
int slh_ctx_destroy(slh_ctx *ctx);

/* Text of the last error recorded on the context (never null; owned by the
 * context, valid until its next call).  A null context gives the text of
 * the last error of the context-free calls of the calling thread. */
const char *slh_last_error(const slh_ctx *ctx);

/* Key generation (Algorithm 18) on the current GPU.  Host pointers:
 *   seed  3n bytes SK.seed | SK.prf | PK.seed   (input)
 *   pk    2n bytes                               (output)
 *   sk    4n bytes                               (output)
 * Synchronous.  Errors: SLH_EINVAL, SLH_ENOMEM, SLH_EDEVICE. */
int slh_keygen(uint32_t param, const uint8_t *seed, uint8_t *pk, uint8_t *sk);

/* Copy `count` secret keys (host, count * 4n bytes, each SK.seed | SK.prf |
 * PK.seed | PK.root) of parameter set `param` into the context's device key
 * table and derive their per-key hash state.  Their slots are
 * *first_slot ... *first_slot + count - 1.  Synchronous.
 * Errors: SLH_EINVAL, SLH_ENOMEM, SLH_EDEVICE. */
int slh_ctx_add_keys(slh_ctx *ctx, uint32_t param, const uint8_t *sks, uint32_t count,
                     uint32_t *first_slot);

/* Allocate, now, the working memory and pinned staging that slh_sign_batch
 * needs for batches of up to `count` requests in `mode`, for every parameter
 * set the context holds keys of, so that such calls allocate nothing later
 * (an allocation or free in the middle of serving would wait for the whole
 * GPU).  Working memory is capped by the context's budget, split evenly over
 * those parameter sets.  Synchronous.  Errors: SLH_EINVAL, SLH_ENOMEM,
 * SLH_EDEVICE. */
int slh_ctx_reserve(slh_ctx *ctx, uint32_t count, uint32_t mode);

/* Keep on the device every node of the XMSS trees of the top `layers`
 * hypertree layers of keys first_slot .. first_slot + count - 1 (one
 * parameter set).  These trees depend only on the key: layer d-1-u has
 * 2^(h' u) of them, addressed by the tree index of FIPS 205 Algorithm 12.
 * slh_sign_batch in SLH_MODE_DEDUP then takes the authentication path and
 * root of those layers from the cache and only recomputes their WOTS+
 * chains (Algorithm 10 with the cached nodes).  Memory per key:
 * (2^(h' layers) - 1) / (2^h' - 1) trees of (2^(h'+1) - 1) n bytes, outside
 * the context's HBM budget.  layers: 1..6 (128f, 192f and their SHAKE
 * twins), 1..4 (256f, SHAKE-256f).
 * Synchronous.  Errors: SLH_EINVAL (range outside the table, mixed sets, a
 * key cached already, layers out of range), SLH_ENOMEM, SLH_EDEVICE. */
int slh_ctx_cache_keys(slh_ctx *ctx, uint32_t first_slot, uint32_t count, uint32_t layers);

/* Sign a batch (Algorithm 19 per request, deterministic).
 *   items       host array of `count` requests (any mix of parameter sets)
 *   msgs        device buffer holding the messages, msgs_bytes long
 *   sigs        device buffer receiving the signatures, sigs_bytes long,
 *               16-byte aligned
 *   mode        SLH_MODE_*
 *   stream      hipStream_t to enqueue on (null = the default stream)
 * Every item must satisfy msg_off + msg_len <= msgs_bytes and
 * sig_off + sig_bytes(param) <= sigs_bytes; signature ranges must not
 * overlap.  count == 0 is a no-op.  Messages may start at any byte; those
 * at 4-byte aligned addresses are hashed from dword loads (long messages
 * about twice as fast).
 * Errors: SLH_EINVAL, SLH_ENOMEM, SLH_EDEVICE. */
int slh_sign_batch(slh_ctx *ctx, const slh_item *items, uint32_t count, const uint8_t *msgs,
                   uint64_t msgs_bytes, uint8_t *sigs, uint64_t sigs_bytes, uint32_t mode,
                   void *stream);

/* slh_sign_batch for callers that cannot allocate memory: code that runs
 * while a HIP graph is being captured, tight serving loops, harnesses that
 * forbid hipMalloc.  The call allocates no device or pinned host memory and
 * frees none (no hipMalloc, hipHostMalloc, hipFree or library allocator),
 * and its host bookkeeping stays in buffers the context set up when it was
 * created.  It signs exactly what slh_sign_batch signs, with the same
 * kernels, and gives the same bytes.
 *   items, count, msgs, msgs_bytes, sigs, sigs_bytes, stream
 *               as in slh_sign_batch; count <= SLH_NOALLOC_MAX_ITEMS
 *   mode        SLH_MODE_PLAIN, SLH_MODE_FUSED and SLH_MODE_DEDUP (bit
 *               flags); SLH_MODE_GRAPH is refused (a graph is allocated)
 * Working memory: one library-owned device array of
 * SLH_NOALLOC_SCRATCH_BYTES on every GPU the library runs on (reserved when
 * the library's code is loaded onto that GPU, held until the process ends).
 * The batch's requests are copied into it, and each parameter set of the
 * batch is signed in turn in chunks that fit the rest of it, on `stream`.
 * With the default tuning a chunk holds up to about 900 / 410 / 230
 * requests of 128f / 192f / 256f in SLH_MODE_PLAIN (with keep_chains = 0
 * about 2700 / 1230 / 460); a set whose single request does not fit in the
 * chosen mode and tuning is refused with SLH_EINVAL before anything is
 * launched.
 * The array is shared by every call on that GPU, from any context or
 * stream, and keeps the previous call's contents (the kernels clear what
 * they need): calls that overlap in time on one GPU race, and the caller
 * must order them (one stream, or events).  Calls on one context are
 * ordered by the library as for slh_sign_batch.  The keys must already be
 * in the context (slh_ctx_add_keys allocates).
 * Errors: SLH_EINVAL (as slh_sign_batch, plus count above
 * SLH_NOALLOC_MAX_ITEMS, SLH_MODE_GRAPH, or a request too large for the
 * array), SLH_EDEVICE. */
#define SLH_NOALLOC_SCRATCH_BYTES (256ull << 20)
#define SLH_NOALLOC_MAX_ITEMS 4096u
int slh_sign_batch_noalloc(slh_ctx *ctx, const slh_item *items, uint32_t count,
                           const uint8_t *msgs, uint64_t msgs_bytes, uint8_t *sigs,
                           uint64_t sigs_bytes, uint32_t mode, void *stream);

/* One request of the external interface (FIPS 205 Section 10; host memory,
 * 56 bytes).  Offsets index the batch's device message buffer.
 *   param, key_slot, msg_off, msg_len, sig_off   as in slh_item
 *   ctx_off, ctx_len  context string, 0..255 bytes
 *   rnd_off    n bytes of fresh randomness for hedged signing (opt_rand of
 *              Algorithm 19), or SLH_RND_NONE for the deterministic variant
 *              (opt_rand = PK.seed)
 *   prehash    SLH_PREHASH_NONE: pure SLH-DSA, Algorithm 22, signs
 *              M' = 0 | len(ctx) | ctx | M;
 *              SLH_PREHASH_SHA256 / _SHA512: HashSLH-DSA, Algorithm 23,
 *              signs M' = 1 | len(ctx) | ctx | OID | SHA-256(M) / SHA-512(M) */
typedef struct {
    uint32_t param;
    uint32_t key_slot;
    uint64_t msg_off;
    uint64_t msg_len;
    uint64_t sig_off;
    uint64_t ctx_off;
    uint64_t rnd_off;
    uint32_t ctx_len;
    uint32_t prehash;
} slh_item_ext;

#define SLH_RND_NONE (~(uint64_t)0)
#define SLH_PREHASH_NONE 0u
#define SLH_PREHASH_SHA256 1u
#define SLH_PREHASH_SHA512 2u

/* Sign a batch through the external interface (Algorithms 22 and 23).  The
 * library encodes every M' on the GPU (one workgroup per request; the
 * pre-hash runs on one lane) into a buffer it owns, then signs as
 * slh_sign_batch does; arguments, modes and errors as there, plus
 * SLH_EINVAL for a context string over 255 bytes, an unknown pre-hash or an
 * opt_rand range outside the message buffer. */
int slh_sign_batch_ext(slh_ctx *ctx, const slh_item_ext *items, uint32_t count,
                       const uint8_t *msgs, uint64_t msgs_bytes, uint8_t *sigs,
                       uint64_t sigs_bytes, uint32_t mode, void *stream);

/* Verify one signature (Algorithm 20) on the current GPU.  Host pointers.
 * Returns 1 if valid, 0 if not (including a wrong sig_len), negative on
 * error (SLH_EINVAL, SLH_ENOMEM, SLH_EDEVICE).  Synchronous. */
int slh_verify(uint32_t param, const uint8_t *msg, size_t msg_len, const uint8_t *sig,
               size_t sig_len, const uint8_t *pk);

/* One verification request of a batch (host memory, 40 bytes).  Offsets
 * index the batch's device buffers of messages, signatures and public keys
 * (pk = PK.seed | PK.root, 2n bytes). */
typedef struct {
    uint32_t param;
    uint32_t pad;
    uint64_t msg_off;
    uint64_t msg_len;
    uint64_t sig_off;
    uint64_t pk_off;
} slh_verify_item;

/* Verify a batch (Algorithm 20 per item) on the context's GPU: 16 lanes per
 * signature (32 when a parameter set has at most 2048 items in the batch),
 * the WOTS+ chains of each layer balanced over the signature's lanes.
 * results (device, count int32) receives 1 for a
 * valid signature and 0 otherwise, in item order.  Asynchronous on `stream`
 * like slh_sign_batch.  Errors: SLH_EINVAL (nothing launched), SLH_ENOMEM,
 * SLH_EDEVICE. */
int slh_verify_batch(slh_ctx *ctx, const slh_verify_item *items, uint32_t count, const uint8_t *msgs,
                     uint64_t msgs_bytes, const uint8_t *sigs, uint64_t sigs_bytes, const uint8_t *pks,
                     uint64_t pks_bytes, int32_t *results, void *stream);

/* One verification request of the external interface (host memory, 56
 * bytes): slh_verify_item plus the context string (ctx_off, ctx_len <= 255)
 * and the encoding (prehash, as in slh_item_ext). */
typedef struct {
    uint32_t param;
    uint32_t prehash;
    uint64_t msg_off;
    uint64_t msg_len;
    uint64_t sig_off;
    uint64_t pk_off;
    uint64_t ctx_off;
    uint32_t ctx_len;
    uint32_t pad;
} slh_verify_item_ext;

/* Verify a batch through the external interface (slh_verify, Algorithm 24,
 * and hash_slh_verify, Algorithm 25): M' is encoded on the GPU as for
 * slh_sign_batch_ext, then verified as slh_verify_batch does; arguments and
 * errors as there. */
int slh_verify_batch_ext(slh_ctx *ctx, const slh_verify_item_ext *items, uint32_t count,
                         const uint8_t *msgs, uint64_t msgs_bytes, const uint8_t *sigs,
                         uint64_t sigs_bytes, const uint8_t *pks, uint64_t pks_bytes,
                         int32_t *results, void *stream);

/* Kernel phases of the signing path, for per-phase timing. */
#define SLH_PHASE_PRELUDE 0 /* PRF_msg, H_msg, index split                     */
#define SLH_PHASE_FORS 1    /* FORS trees and auth paths (plain mode)          */
#define SLH_PHASE_TREE 2    /* WOTS+ chains, leaves, XMSS roots/auth (plain)   */
#define SLH_PHASE_WOTS 3    /* FORS public key and WOTS+ signatures            */
#define SLH_PHASE_FUSED 4   /* FORS and TREE in the persistent kernel (fused)  */
#define SLH_NPHASES 5

/* Per-parameter-set knobs of the signing kernels (the autotuner's search
 * space: the paper tunes its FORS fusion per GPU with Algorithm 1 and the
 * Relax-FORS buffer, Section III-B, orders FORS_Sign, TREE_Sign and
 * WOTS+_Sign as a task graph, Section III-F, and picks native or PTX code
 * per kernel, Section III-C).  Every setting gives the same bytes.
 *   fors_trees_per_group  FORS trees reduced together by one workgroup:
 *                         4, 8 or 16 for 128f and 192f, 2, 4 or 8 for 256f
 *                         (0 = default: 8, 8, 4); 1 or 2 FORS units of 2^12
 *                         leaves for the small sets (0 = 1)
 *   wgs_per_cu            fused mode: persistent workgroups per compute unit
 *                         (0 = as many as fit, at most 64)
 *   keep_chains           1: the TREE phase keeps every value of the signing
 *                         leaves' WOTS+ chains and the WOTS phase gathers the
 *                         signature from them; 0: nothing is kept (less
 *                         memory) and the WOTS phase recomputes the chains
 *   split_max_blocks      a batch of this parameter set with at most this
 *                         many TREE blocks (64 hypertree leaves each) takes
 *                         the per-phase path with each block's WOTS+ chains
 *                         split over up to len one-wave workgroups, in every
 *                         mode: such a batch cannot fill the chip, and the
 *                         split cuts its latency (0 = default: 1.5 x the
 *                         number of compute units; SLH_SPLIT_NEVER = never)
 *   fors_leaves_per_lane  FORS leaves one lane builds and reduces in
 *                         registers before the LDS levels: 2 or 4 (0 = 2;
 *                         the fast sets; the small sets take 2)
 *   fors_threads          lanes of a FORS workgroup of the per-phase path:
 *                         128, 256 or 512 (0 = 256; the fused kernel's
 *                         workgroups have 256; fast sets only)
 *   tree_waves            waves of a TREE block of the per-phase path (64
 *                         hypertree leaves): 2, 4 or 8 (0 = 4; fast sets)
 *   layer_order           SLH_LAYERS_PARALLEL: every hypertree layer of every
 *                         signature in one TREE launch (the layers are
 *                         independent once idx_tree is known), WOTS+ then a
 *                         gather (keep_chains = 1) or a recomputation;
 *                         SLH_LAYERS_IN_ORDER: FORS first, then one TREE
 *                         launch per layer, whose signing leaves write their
 *                         WOTS+ signature while their chains pass the digits
 *                         of that layer's message (known once the layer
 *                         below is done): nothing kept, nothing recomputed,
 *                         no WOTS phase.  In-order signing takes the
 *                         per-phase path in every mode except the dedup
 *                         modes, which keep the parallel order (fast sets)
 *   variant_tree, variant_fors, variant_verify
 *                         instruction variant of the SHA-2 arithmetic in the
 *                         TREE, FORS and verification kernels of the SHA2
 *                         fast sets: SLH_VARIANT_DEFAULT (v_bitop3 logic,
 *                         three-input and fused 64-bit adds),
 *                         SLH_VARIANT_NO_BITOP3 (two-input XORs and v_bfi),
 *                         SLH_VARIANT_SPLIT_ADDS (two-input adds, 64-bit adds
 *                         as carry pairs).  A variant other than the default
 *                         exists for the default shape of its kernel
 *                         (tree_waves 4; fors_leaves_per_lane 2 and
 *                         fors_threads 256); the fused kernel has the
 *                         default only
 *   fused_wave0_chunks    fused mode: chains chunks (one chain of each of a
 *                         block's 64 leaves) that wave 0 of a workgroup runs
 *                         per TREE block while it also finishes the previous
 *                         block (T_len and the XMSS levels); the other waves
 *                         share the rest.  0 = the share that balances the
 *                         instruction counts (four waves: 8 / 11 / 14 for len 35 /
 *                         51 / 67, per block of an item); else 2 ..
 *                         fused_blocks_per_item x len - 6
 *   fused_waves           fused mode: waves per persistent workgroup, 4 or 2
 *                         (0 = 4; fast sets).  A TREE block's chains go to
 *                         the waves in whole chunks and each block ends at a
 *                         workgroup barrier; with two waves the chunk split
 *                         (fused_wave0_chunks default 17 / 24 / 31) leaves
 *                         less of a block's time unbalanced
 *   fused_blocks_per_item fused mode: TREE blocks per work item, 1 or 2
 *                         (0 = 1; fast sets).  With 2 the chunks of both
 *                         blocks are dealt out together (wave 0's default
 *                         share doubles), which balances the waves more
 *                         finely; staging per workgroup doubles
 *   fused_schedule        fused mode: SLH_FUSED_ITEMS (0 = this default):
 *                         workgroups take items of whole TREE blocks, whose
 *                         chains chunks are dealt to the waves by a fixed
 *                         share; SLH_FUSED_CHUNKS: workgroups take one TREE
 *                         block at a time and its waves take its chains
 *                         chunks one at a time, so slower waves and slower
 *                         workgroups (the SIMD serves older waves first)
 *                         take less; a rotating wave finishes each block
 *                         while the others start the next.  SLH_FUSED_CHUNKS
 *                         requires fused_waves 4 and fused_blocks_per_item
 *                         and fused_wave0_chunks 0 (fast sets) */
typedef struct {
    uint32_t fors_trees_per_group;
    uint32_t wgs_per_cu;
    uint32_t keep_chains;
    uint32_t split_max_blocks;
    uint32_t fors_leaves_per_lane;
    uint32_t fors_threads;
    uint32_t tree_waves;
    uint32_t layer_order;
    uint32_t variant_tree;
    uint32_t variant_fors;
    uint32_t variant_verify;
    uint32_t fused_wave0_chunks;
    uint32_t fused_waves;
    uint32_t fused_blocks_per_item;
    uint32_t fused_schedule;
} slh_tuning;
#define SLH_SPLIT_NEVER 0xFFFFFFFFu
#define SLH_FUSED_ITEMS 1u
#define SLH_FUSED_CHUNKS 2u
#define SLH_LAYERS_PARALLEL 0u
#define SLH_LAYERS_IN_ORDER 1u
#define SLH_VARIANT_DEFAULT 0u
#define SLH_VARIANT_NO_BITOP3 1u
#define SLH_VARIANT_SPLIT_ADDS 2u

/* Set or read the knobs of parameter set `param` on a context.  Setting
 * waits for the context's pending work.  Errors: SLH_EINVAL. */
int slh_ctx_set_tuning(slh_ctx *ctx, uint32_t param, const slh_tuning *t);
int slh_ctx_get_tuning(const slh_ctx *ctx, uint32_t param, slh_tuning *t);

/* Turn per-phase timing on or off for later slh_sign_batch calls.  When on,
 * the library records a HIP event before and after every kernel it
 * launches, on the caller's stream (the paper reports per-kernel throughput
 * in its Table 8; this is the same measurement).  Errors: SLH_EINVAL. */
int slh_ctx_profile(slh_ctx *ctx, int enable);

/* Trees of the hypertree that slh_sign_batch calls in SLH_MODE_DEDUP needed
 * (messages x d) and the distinct ones they computed, summed since the last
 * reset (FIPS 205 Algorithm 12 visits d trees per signature; the difference
 * is the TREE work the dedup saved).  Waits for the context's pending work;
 * reset != 0 clears the totals.  Errors: SLH_EINVAL, SLH_EDEVICE. */
int slh_ctx_dedup_stats(slh_ctx *ctx, uint64_t *trees, uint64_t *distinct, int reset);

/* Accumulated GPU time per phase since the last reset.  Host arrays of
 * SLH_NPHASES entries: ms[i] milliseconds, launches[i] kernel launches,
 * messages[i] messages processed.  Waits for the recorded events.  reset != 0
 * clears the totals.  Errors: SLH_EINVAL, SLH_EDEVICE. */
int slh_ctx_phase_times(slh_ctx *ctx, double *ms, uint64_t *launches, uint64_t *messages,
                        int reset);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of sign requests (this library's own; the   */
/* paper signs fixed batches).                                              */
/* ---------------------------------------------------------------------- */
typedef struct slh_server slh_server;

/* Server configuration (0 selects the default in brackets).
 *   lanes        batches in flight at once, each with its own signing
 *                context, stream and buffers, so that they overlap on the
 *                GPU [4, at most 8]
 *   max_batch    requests per launch [4096]
 *   min_batch    launch as soon as this many wait and a lane is free
 *                [0 = rule off]
 *   max_wait_us  launch when the oldest waiting request is this old [2000]
 *   msg_bytes    message buffer per lane; a batch takes requests in arrival
 *                order while their messages fit (admission by memory)
 *                [64 MiB]
 *   hbm_budget   working memory of each lane's signing context [4 GiB]
 *   mode         SLH_MODE_* of the launches [plain]
 *   queue_limit  waiting requests before slh_serve_submit says SLH_EBUSY
 *                [1 << 20]
 *   cache_layers upper hypertree layers cached per key on every lane by
 *                slh_serve_add_keys (slh_ctx_cache_keys; used in
 *                SLH_MODE_DEDUP), clamped to the set's limit [0 = none]
 * A batch is launched when it is full, when no lane is busy, when its
 * oldest request has waited max_wait_us times the number of busy lanes, or
 * by the min_batch rule.
 * Every lane keeps up to four streams busy (its own and its context's three
 * branch streams for mixed parameter sets).  The HIP runtime maps a
 * process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 unless the
 * environment says otherwise); lanes whose streams share a queue
 * serialise.  With 4 lanes, GPU_MAX_HW_QUEUES=16 cut the p50 latency at 90 %
 * of the saturated rate from 16.5 to 5.7 ms on MI355X; 32 was worse than 16. */
typedef struct {
    uint32_t lanes;
    uint32_t max_batch;
    uint32_t min_batch;
    uint32_t max_wait_us;
    uint64_t msg_bytes;
    uint64_t hbm_budget;
    uint32_t mode;
    uint32_t queue_limit;
    uint32_t cache_layers;
    uint32_t reserved;
} slh_serve_config;

/* One request of a replayed trace.  Offsets index the replay's host
 * buffers; arrival_s is the arrival time in seconds after the replay
 * starts (non-decreasing). */
typedef struct {
    uint32_t param;
    uint32_t key_slot;
    uint64_t msg_off;
    uint64_t msg_len;
    uint64_t sig_off;
    double arrival_s;
} slh_serve_request;

/* Outcome of a replay.  Latency = completion - arrival, over the requests
 * after the first `skip`. */
typedef struct {
    uint64_t completed;
    uint64_t launches;
    double wall_s;      /* replay start to last completion */
    double sig_per_s;   /* completed / wall_s */
    double p50_s, p99_s, mean_s, max_s;
    double mean_batch;  /* requests per launch */
} slh_serve_stats;

/* Create / destroy a server on GPU `device`.  cfg may be null (defaults).
 * Errors: SLH_EINVAL, SLH_ENOMEM, SLH_EDEVICE. */
int slh_serve_create(int device, const slh_serve_config *cfg, slh_server **out);
int slh_serve_destroy(slh_server *s);
const char *slh_serve_last_error(const slh_server *s);

/* Register secret keys (as slh_ctx_add_keys) on every lane; the slots are
 * the same on all lanes.  Not while the online scheduler runs. */
int slh_serve_add_keys(slh_server *s, uint32_t param, const uint8_t *sks, uint32_t count,
                       uint32_t *first_slot);
/* Tuning knobs (as slh_ctx_set_tuning) on every lane. */
int slh_serve_set_tuning(slh_server *s, uint32_t param, const slh_tuning *t);

/* Serve a trace on the calling thread: each request is released to the
 * scheduler at its arrival time, signatures are written to sigs (host,
 * sigs_bytes long) at sig_off, latencies (seconds) to latency_s[i] if not
 * null, and the summary to *stats if not null.  Returns when every request
 * has completed.  Errors: SLH_EINVAL (a request of an unknown set, with a
 * key slot that is missing or holds another set's key, or outside the
 * buffers; nothing is served),
 * SLH_EBUSY (online scheduler running), SLH_EDEVICE. */
int slh_serve_replay(slh_server *s, const slh_serve_request *reqs, uint64_t n, const uint8_t *msgs,
                     uint64_t msgs_bytes, uint8_t *sigs, uint64_t sigs_bytes, double *latency_s,
                     uint64_t skip, slh_serve_stats *stats);

/* Online use: start a scheduler thread, submit requests as they arrive
 * (the message is copied; `tag` identifies the result), poll completed
 * results, stop (waits until every submitted request has completed).
 * slh_serve_submit returns SLH_EBUSY when queue_limit requests wait, and
 * SLH_EINVAL (nothing queued) for an unknown set, a key slot that is missing
 * or holds another set's key, or a message longer than msg_bytes.
 * slh_serve_poll copies up to `max` results: tags[i], the signature at
 * sigs + i * sig_stride (sig_stride >= 49856), latency_s[i] if not null;
 * *n is the number copied.  Submit and poll may be called from any thread. */
int slh_serve_start(slh_server *s);
int slh_serve_submit(slh_server *s, uint32_t param, uint32_t key_slot, const uint8_t *msg,
                     uint64_t len, uint64_t tag);
int slh_serve_poll(slh_server *s, uint64_t *tags, uint8_t *sigs, uint64_t sig_stride,
                   double *latency_s, uint32_t max, uint32_t *n);
int slh_serve_stop(slh_server *s);

#ifdef __cplusplus
}
#endif
#endif
