/*
 * slh_oracle.h -- plain CPU reference of SPHINCS+ / SLH-DSA signing with the
 * SHA2 and SHAKE "simple" instantiations.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU baseline of the benchmark can compare the GPU library
 * against an obviously correct implementation.  The GPU product never links,
 * loads or calls it, and it shares no code, header or table with the GPU
 * sources.
 *
 * What is computed and where it is defined:
 *   - The paper (HERO-Sign, arXiv 2512.23969) accelerates SPHINCS+ signature
 *     generation: its Section II-A describes WOTS+, FORS, MSS (XMSS) and the
 *     hypertree, its Table 1 lists the -f parameter sets, and its Fig. 2
 *     listing gives the signing flow (hash_message, message_to_indices,
 *     fors_sign, then d layers of merkle_sign).  The paper reorders that
 *     work for the GPU but computes the same signature.
 *   - The exact arithmetic is the scheme's own: FIPS 205 (SLH-DSA) internal
 *     functions with the SHA2 instantiation of its Section 11.2 (SHA-256 and
 *     SHA-512 from FIPS 180-4, HMAC from FIPS 198-1, MGF1 from RFC 8017) or
 *     the SHAKE instantiation of its Section 11.1 (Keccak-f[1600] and
 *     SHAKE256 from FIPS 202), for the parameter sets of its Table 2.
 *
 * Readings taken where the paper is silent:
 *   - FIPS 205 internal functions (no context prefix, raw message M).
 *   - FORS indices via base_2b, most-significant bit first.
 *   - n = 24 and n = 32 use SHA-512 for H, T_l, H_msg and PRF_msg; F and PRF
 *     always use SHA-256.
 *   - deterministic signing: opt_rand = PK.seed unless addrnd is given.
 *
 * Precision: every value is an exact byte string; there is no floating point.
 *
 * Memory: every buffer belongs to the caller.  Only or_sign_ext and
 * or_verify_ext allocate (the encoded message M'); or_sign / or_verify /
 * or_keygen use bounded stack arrays sized by the compile-time limits below.  Functions return 0 on success and
 * a negative value on a bad argument (unknown parameters, sizes beyond the
 * limits); verify returns 1 (valid) or 0 (invalid).
 */
#ifndef SLH_ORACLE_H
#define SLH_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Upper limits on parameters accepted by this oracle (the three -f sets and
 * tiny sets for brute-force tests fit in them). */
#define OR_MAX_N 32
#define OR_MAX_LEN 70     /* WOTS+ chains per key (67 for n = 32) */
#define OR_MAX_K 64       /* FORS trees */
#define OR_MAX_A 14       /* FORS tree height (14 for 192s / 256s) */
#define OR_MAX_HP 9       /* XMSS tree height h' (9 for 128s / 192s) */
#define OR_MAX_D 32       /* hypertree layers */

/* A parameter set (FIPS 205 Table 2 naming; the paper's Table 1 gives
 * n, h, d, log t = a, k and w for the -f sets). lg_w is fixed to 4. */
typedef struct {
    int n;      /* security parameter in bytes */
    int h;      /* total hypertree height */
    int d;      /* hypertree layers */
    int hp;     /* h' = h / d, height of one XMSS tree */
    int a;      /* FORS tree height (log t) */
    int k;      /* number of FORS trees */
    int lg_w;   /* log2 of the Winternitz parameter (4) */
    int len1;   /* 8n / lg_w */
    int len2;   /* checksum digits */
    int len;    /* len1 + len2 */
    int m;      /* digest bytes taken from H_msg */
    int wide;   /* 1: H, T_l, H_msg, PRF_msg use SHA-512 (n >= 24) */
    int shake;  /* 1: every hash is SHAKE256 (FIPS 205 Section 11.1) */
} or_params;

/* id 1 = SHA2-128f, 2 = SHA2-192f, 3 = SHA2-256f, 4 = SHA2-128s,
 * 5 = SHA2-192s, 6 = SHA2-256s; 7..12 = the SHAKE sets in the same order. */
int or_params_get(int id, or_params *p);
/* Fill derived fields (len1, len2, len, m, wide) of a custom set from
 * n, h, d, a, k.  Returns 0 or -1 if outside the limits. */
int or_params_custom(int n, int h, int d, int a, int k, or_params *p);
size_t or_sig_bytes(const or_params *p);

/* FIPS 180-4 / FIPS 198-1 / RFC 8017 primitives. */
void or_sha256(const uint8_t *in, size_t len, uint8_t out[32]);
/* FIPS 202: SHAKE256 with `outlen` output bytes, and SHA3-256. */
void or_shake256(const uint8_t *in, size_t len, uint8_t *out, size_t outlen);
void or_sha3_256(const uint8_t *in, size_t len, uint8_t out[32]);
void or_sha512(const uint8_t *in, size_t len, uint8_t out[64]);
void or_hmac_sha256(const uint8_t *key, size_t klen, const uint8_t *msg,
                    size_t mlen, uint8_t out[32]);
void or_hmac_sha512(const uint8_t *key, size_t klen, const uint8_t *msg,
                    size_t mlen, uint8_t out[64]);
void or_mgf1_sha256(const uint8_t *seed, size_t slen, uint8_t *out, size_t outlen);
void or_mgf1_sha512(const uint8_t *seed, size_t slen, uint8_t *out, size_t outlen);
/* The round constants and initial values in use (for the prime-root pins). */
void or_sha256_constants(uint32_t k[64], uint32_t iv[8]);
void or_sha512_constants(uint64_t k[80], uint64_t iv[8]);

/* Tweakable hashes of FIPS 205 Section 11.2; adrs is the full 32-byte ADRS. */
void or_prf(const or_params *p, const uint8_t *pk_seed, const uint8_t *sk_seed,
            const uint8_t adrs[32], uint8_t *out);
void or_f(const or_params *p, const uint8_t *pk_seed, const uint8_t adrs[32],
          const uint8_t *m1, uint8_t *out);
void or_h(const or_params *p, const uint8_t *pk_seed, const uint8_t adrs[32],
          const uint8_t *m2, uint8_t *out);
void or_t(const or_params *p, const uint8_t *pk_seed, const uint8_t adrs[32],
          const uint8_t *ml, size_t l_blocks, uint8_t *out);
void or_prf_msg(const or_params *p, const uint8_t *sk_prf, const uint8_t *opt_rand,
                const uint8_t *msg, size_t mlen, uint8_t *out);
void or_h_msg(const or_params *p, const uint8_t *r, const uint8_t *pk_seed,
              const uint8_t *pk_root, const uint8_t *msg, size_t mlen, uint8_t *out);

/* base_2b (FIPS 205 Algorithm 4). */
void or_base_2b(const uint8_t *x, int b, int out_len, uint32_t *out);

/* Component functions exposed for the structural tests. */
void or_wots_pkgen(const or_params *p, const uint8_t *sk_seed, const uint8_t *pk_seed,
                   const uint8_t adrs[32], uint8_t *pk);
void or_xmss_node(const or_params *p, const uint8_t *sk_seed, uint32_t i, uint32_t z,
                  const uint8_t *pk_seed, const uint8_t adrs[32], uint8_t *node);
void or_fors_node(const or_params *p, const uint8_t *sk_seed, uint32_t i, uint32_t z,
                  const uint8_t *pk_seed, const uint8_t adrs[32], uint8_t *node);
/* FORS public key recomputed from a FORS signature (Algorithm 17). */
void or_fors_pk_from_sig(const or_params *p, const uint8_t *sig_fors, const uint8_t *md,
                         const uint8_t *pk_seed, const uint8_t adrs[32], uint8_t *pk);
/* XMSS root recomputed from an XMSS signature (Algorithm 11). */
void or_xmss_pk_from_sig(const or_params *p, uint32_t idx, const uint8_t *sig_xmss,
                         const uint8_t *msg_n, const uint8_t *pk_seed,
                         const uint8_t adrs[32], uint8_t *root);
/* Digest split of Algorithm 19: md bytes, idx_tree, idx_leaf. */
void or_split_digest(const or_params *p, const uint8_t *digest, uint8_t *md,
                     uint64_t *idx_tree, uint32_t *idx_leaf);

/* Key generation from explicit seeds (Algorithm 18).
 * sk = SK.seed | SK.prf | PK.seed | PK.root (4n), pk = PK.seed | PK.root (2n). */
int or_keygen(const or_params *p, const uint8_t *sk_seed, const uint8_t *sk_prf,
              const uint8_t *pk_seed, uint8_t *sk, uint8_t *pk);
/* Signing (Algorithm 19).  addrnd == NULL selects deterministic signing
 * (opt_rand = PK.seed). */
int or_sign(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *sk,
            const uint8_t *addrnd, uint8_t *sig);
/* Verification (Algorithm 20): 1 valid, 0 invalid, negative on bad params. */
int or_verify(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *sig,
              size_t siglen, const uint8_t *pk);

/* External interface of FIPS 205 (Section 10).  ph selects the message
 * encoding: OR_PURE (Algorithms 22 / 24: M' = 0 | len(ctx) | ctx | M) or
 * OR_PH_SHA256 / OR_PH_SHA512 (Algorithms 23 / 25: M' = 1 | len(ctx) | ctx |
 * OID(PH) | PH(M)).  ctxlen <= 255.  or_encode_ext writes M' to out (room for
 * 2 + ctxlen + max(mlen, 75) bytes) and returns its length, or -1 on bad
 * arguments.  or_sign_ext / or_verify_ext sign / verify M' with the internal
 * functions (addrnd NULL: deterministic); they allocate M' on the heap. */
#define OR_PURE 0
#define OR_PH_SHA256 1
#define OR_PH_SHA512 2
long or_encode_ext(const uint8_t *msg, size_t mlen, const uint8_t *ctx, size_t ctxlen, int ph,
                   uint8_t *out);
int or_sign_ext(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *ctx,
                size_t ctxlen, int ph, const uint8_t *sk, const uint8_t *addrnd, uint8_t *sig);
int or_verify_ext(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *ctx,
                  size_t ctxlen, int ph, const uint8_t *sig, size_t siglen, const uint8_t *pk);

/* Per-thread call counters (reset / read).  Index: 0 F, 1 PRF, 2 H, 3 T_l,
 * 4 SHA-256 compressions, 5 SHA-512 compressions, 6 PRF_msg, 7 H_msg,
 * 8 Keccak-f[1600] permutations. */
#define OR_NCOUNTERS 9
void or_counters_reset(void);
void or_counters_get(uint64_t out[OR_NCOUNTERS]);

#ifdef __cplusplus
}
#endif
#endif
