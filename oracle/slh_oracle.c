/*
 * slh_oracle.c -- plain CPU reference of SPHINCS+ signing (SHA2 "simple").
 *
 * TEST INFRASTRUCTURE ONLY (see slh_oracle.h).  Nothing in the GPU library
 * includes, links or calls this file.
 *
 * Written for clarity, not speed: every function follows one definition,
 * step by step, in the order the definition gives them.  No precomputed
 * midstates, no batching, no reordering.  Each function names the passage it
 * follows: FIPS 180-4 (SHA-2), FIPS 198-1 (HMAC), RFC 8017 Appendix B.2.1
 * (MGF1) and FIPS 205 (SLH-DSA: Sections 4-9 and 11.2), and where the paper
 * describes the same step, the paper's section (HERO-Sign, Section II-A
 * background and the Fig. 2 signing listing).
 */
#include "slh_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counters (per thread, so that a multi-threaded timing run is race free).  */
/* ------------------------------------------------------------------------ */
static __thread uint64_t g_cnt[OR_NCOUNTERS];
enum { C_F = 0, C_PRF, C_H, C_T, C_SHA256_BLK, C_SHA512_BLK, C_PRFMSG, C_HMSG, C_KECCAK };

void or_counters_reset(void) { memset(g_cnt, 0, sizeof g_cnt); }
void or_counters_get(uint64_t out[OR_NCOUNTERS]) { memcpy(out, g_cnt, sizeof g_cnt); }

/* ------------------------------------------------------------------------ */
/* SHA-256, FIPS 180-4 Sections 4.1.2, 4.2.2, 5.1.1, 5.3.3, 6.2.             */
/* ------------------------------------------------------------------------ */
static const uint32_t K256[64] = {
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
    0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u};
static const uint32_t IV256[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                                  0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};

static uint32_t rotr32(uint32_t x, int r) { return (x >> r) | (x << (32 - r)); }

/* One application of the SHA-256 compression function to a 64-byte block. */
static void sha256_block(uint32_t H[8], const uint8_t blk[64])
{
    uint32_t W[64];
    g_cnt[C_SHA256_BLK]++;
    for (int t = 0; t < 16; t++)
        W[t] = ((uint32_t)blk[4 * t] << 24) | ((uint32_t)blk[4 * t + 1] << 16) |
               ((uint32_t)blk[4 * t + 2] << 8) | (uint32_t)blk[4 * t + 3];
    for (int t = 16; t < 64; t++) {
        uint32_t s0 = rotr32(W[t - 15], 7) ^ rotr32(W[t - 15], 18) ^ (W[t - 15] >> 3);
        uint32_t s1 = rotr32(W[t - 2], 17) ^ rotr32(W[t - 2], 19) ^ (W[t - 2] >> 10);
        W[t] = s1 + W[t - 7] + s0 + W[t - 16];
    }
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
    for (int t = 0; t < 64; t++) {
        uint32_t S1 = rotr32(e, 6) ^ rotr32(e, 11) ^ rotr32(e, 25);
        uint32_t ch = (e & f) ^ (~e & g);
        uint32_t T1 = h + S1 + ch + K256[t] + W[t];
        uint32_t S0 = rotr32(a, 2) ^ rotr32(a, 13) ^ rotr32(a, 22);
        uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
        uint32_t T2 = S0 + maj;
        h = g; g = f; f = e; e = d + T1; d = c; c = b; b = a; a = T1 + T2;
    }
    H[0] += a; H[1] += b; H[2] += c; H[3] += d; H[4] += e; H[5] += f; H[6] += g; H[7] += h;
}

/* Incremental SHA-256 over a sequence of byte strings (padding per 5.1.1). */
typedef struct { uint32_t H[8]; uint8_t buf[64]; size_t fill; uint64_t total; } sha256_ctx;

static void sha256_init(sha256_ctx *c)
{
    memcpy(c->H, IV256, sizeof IV256);
    c->fill = 0;
    c->total = 0;
}
static void sha256_update(sha256_ctx *c, const uint8_t *in, size_t len)
{
    c->total += len;
    while (len > 0) {
        size_t take = 64 - c->fill;
        if (take > len) take = len;
        memcpy(c->buf + c->fill, in, take);
        c->fill += take; in += take; len -= take;
        if (c->fill == 64) { sha256_block(c->H, c->buf); c->fill = 0; }
    }
}
static void sha256_final(sha256_ctx *c, uint8_t out[32])
{
    uint64_t bits = c->total * 8;
    uint8_t pad = 0x80, zero = 0, lenbe[8];
    sha256_update(c, &pad, 1);
    while (c->fill != 56) sha256_update(c, &zero, 1);
    for (int i = 0; i < 8; i++) lenbe[i] = (uint8_t)(bits >> (56 - 8 * i));
    sha256_update(c, lenbe, 8);
    for (int i = 0; i < 8; i++) {
        out[4 * i] = (uint8_t)(c->H[i] >> 24); out[4 * i + 1] = (uint8_t)(c->H[i] >> 16);
        out[4 * i + 2] = (uint8_t)(c->H[i] >> 8); out[4 * i + 3] = (uint8_t)c->H[i];
    }
}

void or_sha256(const uint8_t *in, size_t len, uint8_t out[32])
{
    sha256_ctx c;
    sha256_init(&c);
    sha256_update(&c, in, len);
    sha256_final(&c, out);
}

/* ------------------------------------------------------------------------ */
/* SHA-512, FIPS 180-4 Sections 4.1.3, 4.2.3, 5.1.2, 5.3.5, 6.4.             */
/* ------------------------------------------------------------------------ */
static const uint64_t K512[80] = {
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
static const uint64_t IV512[8] = {0x6a09e667f3bcc908ull, 0xbb67ae8584caa73bull,
                                  0x3c6ef372fe94f82bull, 0xa54ff53a5f1d36f1ull,
                                  0x510e527fade682d1ull, 0x9b05688c2b3e6c1full,
                                  0x1f83d9abfb41bd6bull, 0x5be0cd19137e2179ull};

static uint64_t rotr64(uint64_t x, int r) { return (x >> r) | (x << (64 - r)); }

static void sha512_block(uint64_t H[8], const uint8_t blk[128])
{
    uint64_t W[80];
    g_cnt[C_SHA512_BLK]++;
    for (int t = 0; t < 16; t++) {
        uint64_t w = 0;
        for (int j = 0; j < 8; j++) w = (w << 8) | blk[8 * t + j];
        W[t] = w;
    }
    for (int t = 16; t < 80; t++) {
        uint64_t s0 = rotr64(W[t - 15], 1) ^ rotr64(W[t - 15], 8) ^ (W[t - 15] >> 7);
        uint64_t s1 = rotr64(W[t - 2], 19) ^ rotr64(W[t - 2], 61) ^ (W[t - 2] >> 6);
        W[t] = s1 + W[t - 7] + s0 + W[t - 16];
    }
    uint64_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
    for (int t = 0; t < 80; t++) {
        uint64_t S1 = rotr64(e, 14) ^ rotr64(e, 18) ^ rotr64(e, 41);
        uint64_t ch = (e & f) ^ (~e & g);
        uint64_t T1 = h + S1 + ch + K512[t] + W[t];
        uint64_t S0 = rotr64(a, 28) ^ rotr64(a, 34) ^ rotr64(a, 39);
        uint64_t maj = (a & b) ^ (a & c) ^ (b & c);
        uint64_t T2 = S0 + maj;
        h = g; g = f; f = e; e = d + T1; d = c; c = b; b = a; a = T1 + T2;
    }
    H[0] += a; H[1] += b; H[2] += c; H[3] += d; H[4] += e; H[5] += f; H[6] += g; H[7] += h;
}

typedef struct { uint64_t H[8]; uint8_t buf[128]; size_t fill; uint64_t total; } sha512_ctx;

static void sha512_init(sha512_ctx *c)
{
    memcpy(c->H, IV512, sizeof IV512);
    c->fill = 0;
    c->total = 0;
}
static void sha512_update(sha512_ctx *c, const uint8_t *in, size_t len)
{
    c->total += len;
    while (len > 0) {
        size_t take = 128 - c->fill;
        if (take > len) take = len;
        memcpy(c->buf + c->fill, in, take);
        c->fill += take; in += take; len -= take;
        if (c->fill == 128) { sha512_block(c->H, c->buf); c->fill = 0; }
    }
}
static void sha512_final(sha512_ctx *c, uint8_t out[64])
{
    /* 128-bit big-endian length; messages here are far below 2^64 bits. */
    uint64_t bits = c->total * 8;
    uint8_t pad = 0x80, zero = 0, lenbe[16];
    sha512_update(c, &pad, 1);
    while (c->fill != 112) sha512_update(c, &zero, 1);
    memset(lenbe, 0, 8);
    for (int i = 0; i < 8; i++) lenbe[8 + i] = (uint8_t)(bits >> (56 - 8 * i));
    sha512_update(c, lenbe, 16);
    for (int i = 0; i < 8; i++)
        for (int j = 0; j < 8; j++) out[8 * i + j] = (uint8_t)(c->H[i] >> (56 - 8 * j));
}

void or_sha512(const uint8_t *in, size_t len, uint8_t out[64])
{
    sha512_ctx c;
    sha512_init(&c);
    sha512_update(&c, in, len);
    sha512_final(&c, out);
}

void or_sha256_constants(uint32_t k[64], uint32_t iv[8])
{
    memcpy(k, K256, sizeof K256);
    memcpy(iv, IV256, sizeof IV256);
}
void or_sha512_constants(uint64_t k[80], uint64_t iv[8])
{
    memcpy(k, K512, sizeof K512);
    memcpy(iv, IV512, sizeof IV512);
}

/* ------------------------------------------------------------------------ */
/* HMAC (FIPS 198-1 Section 4) and MGF1 (RFC 8017 Appendix B.2.1).          */
/* Keys here are never longer than a block, so no key hashing is needed,    */
/* but it is implemented for completeness of the definition.                */
/* ------------------------------------------------------------------------ */
void or_hmac_sha256(const uint8_t *key, size_t klen, const uint8_t *msg, size_t mlen,
                    uint8_t out[32])
{
    uint8_t k0[64], ipad[64], opad[64], inner[32];
    memset(k0, 0, sizeof k0);
    if (klen > 64) or_sha256(key, klen, k0); else memcpy(k0, key, klen);
    for (int i = 0; i < 64; i++) { ipad[i] = k0[i] ^ 0x36; opad[i] = k0[i] ^ 0x5c; }
    sha256_ctx c;
    sha256_init(&c); sha256_update(&c, ipad, 64); sha256_update(&c, msg, mlen);
    sha256_final(&c, inner);
    sha256_init(&c); sha256_update(&c, opad, 64); sha256_update(&c, inner, 32);
    sha256_final(&c, out);
}

void or_hmac_sha512(const uint8_t *key, size_t klen, const uint8_t *msg, size_t mlen,
                    uint8_t out[64])
{
    uint8_t k0[128], ipad[128], opad[128], inner[64];
    memset(k0, 0, sizeof k0);
    if (klen > 128) or_sha512(key, klen, k0); else memcpy(k0, key, klen);
    for (int i = 0; i < 128; i++) { ipad[i] = k0[i] ^ 0x36; opad[i] = k0[i] ^ 0x5c; }
    sha512_ctx c;
    sha512_init(&c); sha512_update(&c, ipad, 128); sha512_update(&c, msg, mlen);
    sha512_final(&c, inner);
    sha512_init(&c); sha512_update(&c, opad, 128); sha512_update(&c, inner, 64);
    sha512_final(&c, out);
}

/* MGF1: concatenate Hash(seed || I2OSP(counter, 4)) for counter = 0, 1, ...
 * and keep the first outlen bytes. */
void or_mgf1_sha256(const uint8_t *seed, size_t slen, uint8_t *out, size_t outlen)
{
    size_t done = 0;
    for (uint32_t ctr = 0; done < outlen; ctr++) {
        uint8_t c4[4] = {(uint8_t)(ctr >> 24), (uint8_t)(ctr >> 16), (uint8_t)(ctr >> 8),
                         (uint8_t)ctr};
        uint8_t dig[32];
        sha256_ctx c;
        sha256_init(&c); sha256_update(&c, seed, slen); sha256_update(&c, c4, 4);
        sha256_final(&c, dig);
        size_t take = outlen - done < 32 ? outlen - done : 32;
        memcpy(out + done, dig, take);
        done += take;
    }
}

void or_mgf1_sha512(const uint8_t *seed, size_t slen, uint8_t *out, size_t outlen)
{
    size_t done = 0;
    for (uint32_t ctr = 0; done < outlen; ctr++) {
        uint8_t c4[4] = {(uint8_t)(ctr >> 24), (uint8_t)(ctr >> 16), (uint8_t)(ctr >> 8),
                         (uint8_t)ctr};
        uint8_t dig[64];
        sha512_ctx c;
        sha512_init(&c); sha512_update(&c, seed, slen); sha512_update(&c, c4, 4);
        sha512_final(&c, dig);
        size_t take = outlen - done < 64 ? outlen - done : 64;
        memcpy(out + done, dig, take);
        done += take;
    }
}

/* ------------------------------------------------------------------------ */
/* Parameter sets: the paper's Table 1 (n, h, d, log t, k, w) completed with */
/* the derived quantities of FIPS 205 Section 5 (len1, len2) and Alg. 19 (m) */
/* ------------------------------------------------------------------------ */
static int ceil_div(int x, int y) { return (x + y - 1) / y; }

int or_params_custom(int n, int h, int d, int a, int k, or_params *p)
{
    if (n != 16 && n != 24 && n != 32) return -1;
    if (d <= 0 || h % d != 0 || h / d > OR_MAX_HP || d > OR_MAX_D) return -1;
    if (a <= 0 || a > OR_MAX_A || k <= 0 || k > OR_MAX_K) return -1;
    if (h - h / d > 64) return -1;
    memset(p, 0, sizeof *p);
    p->n = n; p->h = h; p->d = d; p->hp = h / d; p->a = a; p->k = k; p->lg_w = 4;
    p->len1 = ceil_div(8 * n, p->lg_w);
    /* gen_len2 (FIPS 205 Algorithm 1): the number of base-w digits needed
     * to hold the largest checksum len1 * (w - 1). */
    {
        int w = 1 << p->lg_w;
        int max_csum = p->len1 * (w - 1);
        int capacity = w;
        p->len2 = 1;
        while (capacity <= max_csum) {
            p->len2++;
            capacity *= w;
        }
    }
    p->len = p->len1 + p->len2;
    if (p->len > OR_MAX_LEN) return -1;
    p->m = ceil_div(k * a, 8) + ceil_div(h - h / d, 8) + ceil_div(h / d, 8);
    p->wide = n >= 24;
    return 0;
}

int or_params_get(int id, or_params *p)
{
    switch (id) {
    case 1: return or_params_custom(16, 66, 22, 6, 33, p);  /* SHA2-128f */
    case 2: return or_params_custom(24, 66, 22, 8, 33, p);  /* SHA2-192f */
    case 3: return or_params_custom(32, 68, 17, 9, 35, p);  /* SHA2-256f */
    case 4: return or_params_custom(16, 63, 7, 12, 14, p);  /* SHA2-128s */
    case 5: return or_params_custom(24, 63, 7, 14, 17, p);  /* SHA2-192s */
    case 6: return or_params_custom(32, 64, 8, 14, 22, p);  /* SHA2-256s */
    default:
        /* the SHAKE sets share the shapes of their SHA2 counterparts */
        if (id >= 7 && id <= 12 && or_params_get(id - 6, p) == 0) {
            p->shake = 1;
            p->wide = 0;
            return 0;
        }
        return -1;
    }
}

size_t or_sig_bytes(const or_params *p)
{
    return (size_t)p->n * (1 + (size_t)p->k * (p->a + 1) + p->h + (size_t)p->d * p->len);
}

/* ------------------------------------------------------------------------ */
/* Keccak-f[1600] and the SHAKE256 / SHA3-256 sponges (FIPS 202).            */
/* The state is 25 lanes A[x + 5 y] of 64 bits; byte i of the sponge is byte */
/* i % 8 (little-endian) of lane i / 8.  The round constants and rotation    */
/* offsets are computed from their definitions (Algorithms 5 and 2).         */
/* ------------------------------------------------------------------------ */
static uint64_t g_keccak_rc[24];
static int g_keccak_rho[25];
static int g_keccak_ready;
static void keccak_init_tables(void);
/* filled once when the library is loaded, before any thread can use them */
__attribute__((constructor)) static void keccak_tables_at_load(void) { keccak_init_tables(); }

/* rc(t) of FIPS 202 Algorithm 5: an LFSR over GF(2)[x] / (x^8 + x^6 + x^5 + x^4 + 1) */
static int keccak_rc_bit(int t)
{
    if (t % 255 == 0) return 1;
    unsigned r = 1; /* R[0] is bit 0 */
    for (int i = 1; i <= t % 255; i++) {
        r <<= 1;                      /* R = 0 || R */
        if (r & 0x100) r ^= 0x171;    /* R[0], R[4], R[5], R[6] ^= R[8]; truncate to 8 bits */
    }
    return r & 1;
}

static void keccak_init_tables(void)
{
    if (g_keccak_ready) return;
    for (int ir = 0; ir < 24; ir++) {
        uint64_t rc = 0;
        for (int j = 0; j <= 6; j++)
            if (keccak_rc_bit(j + 7 * ir)) rc |= (uint64_t)1 << ((1 << j) - 1);
        g_keccak_rc[ir] = rc;
    }
    g_keccak_rho[0] = 0;
    int x = 1, y = 0;
    for (int t = 0; t < 24; t++) {  /* Algorithm 2 (rho) */
        g_keccak_rho[x + 5 * y] = ((t + 1) * (t + 2) / 2) % 64;
        int nx = y, ny = (2 * x + 3 * y) % 5;
        x = nx;
        y = ny;
    }
    g_keccak_ready = 1;
}

static uint64_t rotl64(uint64_t v, int r) { return r ? (v << r) | (v >> (64 - r)) : v; }

static void keccak_f1600(uint64_t A[25])
{
    g_cnt[C_KECCAK]++;
    keccak_init_tables();
    for (int ir = 0; ir < 24; ir++) {
        uint64_t C[5], D[5], B[25];
        for (int x = 0; x < 5; x++) C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];   /* theta */
        for (int x = 0; x < 5; x++) D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
        for (int i = 0; i < 25; i++) A[i] ^= D[i % 5];
        for (int x = 0; x < 5; x++)                                                           /* rho, pi */
            for (int y = 0; y < 5; y++) B[y + 5 * ((2 * x + 3 * y) % 5)] = rotl64(A[x + 5 * y], g_keccak_rho[x + 5 * y]);
        for (int y = 0; y < 5; y++)                                                           /* chi */
            for (int x = 0; x < 5; x++)
                A[x + 5 * y] = B[x + 5 * y] ^ (~B[(x + 1) % 5 + 5 * y] & B[(x + 2) % 5 + 5 * y]);
        A[0] ^= g_keccak_rc[ir];                                                              /* iota */
    }
}

typedef struct {
    uint64_t A[25];
    size_t rate, pos;
} sponge_ctx;

static void sponge_init(sponge_ctx *c, size_t rate)
{
    memset(c, 0, sizeof *c);
    c->rate = rate;
}
static void sponge_byte(sponge_ctx *c, size_t i, uint8_t b) { c->A[i / 8] ^= (uint64_t)b << (8 * (i % 8)); }
static void sponge_absorb(sponge_ctx *c, const uint8_t *in, size_t len)
{
    for (size_t i = 0; i < len; i++) {
        sponge_byte(c, c->pos++, in[i]);
        if (c->pos == c->rate) {
            keccak_f1600(c->A);
            c->pos = 0;
        }
    }
}
/* domain suffix and pad10*1: 0x1F for SHAKE, 0x06 for SHA-3 */
static void sponge_finish(sponge_ctx *c, uint8_t suffix)
{
    sponge_byte(c, c->pos, suffix);
    sponge_byte(c, c->rate - 1, 0x80);
    keccak_f1600(c->A);
    c->pos = 0;
}
static void sponge_squeeze(sponge_ctx *c, uint8_t *out, size_t len)
{
    for (size_t i = 0; i < len; i++) {
        if (c->pos == c->rate) {
            keccak_f1600(c->A);
            c->pos = 0;
        }
        out[i] = (uint8_t)(c->A[c->pos / 8] >> (8 * (c->pos % 8)));
        c->pos++;
    }
}

void or_shake256(const uint8_t *in, size_t len, uint8_t *out, size_t outlen)
{
    sponge_ctx c;
    sponge_init(&c, 136);
    sponge_absorb(&c, in, len);
    sponge_finish(&c, 0x1F);
    sponge_squeeze(&c, out, outlen);
}

void or_sha3_256(const uint8_t *in, size_t len, uint8_t out[32])
{
    sponge_ctx c;
    sponge_init(&c, 136);
    sponge_absorb(&c, in, len);
    sponge_finish(&c, 0x06);
    sponge_squeeze(&c, out, 32);
}

/* ------------------------------------------------------------------------ */
/* ADRS (FIPS 205 Section 4.2 and Table 1): 32 bytes, all big-endian:        */
/*   [0,4) layer  [4,16) tree  [16,20) type  [20,24) [24,28) [28,32) words.  */
/* ------------------------------------------------------------------------ */
enum { WOTS_HASH = 0, WOTS_PK = 1, TREE = 2, FORS_TREE = 3, FORS_ROOTS = 4, WOTS_PRF = 5,
       FORS_PRF = 6 };

static void put32(uint8_t *p, uint32_t v)
{
    p[0] = (uint8_t)(v >> 24); p[1] = (uint8_t)(v >> 16); p[2] = (uint8_t)(v >> 8); p[3] = (uint8_t)v;
}
static uint32_t get32(const uint8_t *p)
{
    return ((uint32_t)p[0] << 24) | ((uint32_t)p[1] << 16) | ((uint32_t)p[2] << 8) | p[3];
}
static void adrs_set_layer(uint8_t *A, uint32_t l) { put32(A + 0, l); }
/* tree address is 12 bytes; the values used here fit in the low 8 bytes */
static void adrs_set_tree(uint8_t *A, uint64_t t)
{
    put32(A + 4, 0);
    put32(A + 8, (uint32_t)(t >> 32));
    put32(A + 12, (uint32_t)t);
}
static void adrs_set_type_and_clear(uint8_t *A, uint32_t type)
{
    put32(A + 16, type);
    memset(A + 20, 0, 12);
}
static void adrs_set_keypair(uint8_t *A, uint32_t i) { put32(A + 20, i); }
static uint32_t adrs_get_keypair(const uint8_t *A) { return get32(A + 20); }
static void adrs_set_chain(uint8_t *A, uint32_t i) { put32(A + 24, i); }
static void adrs_set_tree_height(uint8_t *A, uint32_t z) { put32(A + 24, z); }
static void adrs_set_hash(uint8_t *A, uint32_t i) { put32(A + 28, i); }
static void adrs_set_tree_index(uint8_t *A, uint32_t i) { put32(A + 28, i); }
static uint32_t adrs_get_tree_index(const uint8_t *A) { return get32(A + 28); }

/* Compressed address ADRSc of Section 11.2: ADRS[3] | ADRS[8:16] | ADRS[19] | ADRS[20:32]. */
static void adrs_compress(const uint8_t *A, uint8_t c[22])
{
    c[0] = A[3];
    memcpy(c + 1, A + 8, 8);
    c[9] = A[19];
    memcpy(c + 10, A + 20, 12);
}

/* ------------------------------------------------------------------------ */
/* Tweakable hashes, FIPS 205 Section 11.2.1 (n = 16) and 11.2.2 (n >= 24).  */
/* ------------------------------------------------------------------------ */
/* Trunc_n(SHA-256(PK.seed || toByte(0, 64 - n) || ADRSc || M)) */
static void th256(const or_params *p, const uint8_t *pk_seed, const uint8_t *A,
                  const uint8_t *m, size_t mlen, uint8_t *out)
{
    uint8_t zeros[64] = {0}, ac[22], dig[32];
    sha256_ctx c;
    adrs_compress(A, ac);
    sha256_init(&c);
    sha256_update(&c, pk_seed, p->n);
    sha256_update(&c, zeros, 64 - p->n);
    sha256_update(&c, ac, 22);
    sha256_update(&c, m, mlen);
    sha256_final(&c, dig);
    memcpy(out, dig, p->n);
}
/* Trunc_n(SHA-512(PK.seed || toByte(0, 128 - n) || ADRSc || M)) */
static void th512(const or_params *p, const uint8_t *pk_seed, const uint8_t *A,
                  const uint8_t *m, size_t mlen, uint8_t *out)
{
    uint8_t zeros[128] = {0}, ac[22], dig[64];
    sha512_ctx c;
    adrs_compress(A, ac);
    sha512_init(&c);
    sha512_update(&c, pk_seed, p->n);
    sha512_update(&c, zeros, 128 - p->n);
    sha512_update(&c, ac, 22);
    sha512_update(&c, m, mlen);
    sha512_final(&c, dig);
    memcpy(out, dig, p->n);
}

/* SHAKE256(PK.seed || ADRS || M, 8n) with the full 32-byte ADRS (FIPS 205
 * Section 11.1: PRF, F, H and T_l of the SHAKE sets). */
static void thshake(const or_params *p, const uint8_t *pk_seed, const uint8_t *A,
                    const uint8_t *m, size_t mlen, uint8_t *out)
{
    sponge_ctx c;
    sponge_init(&c, 136);
    sponge_absorb(&c, pk_seed, p->n);
    sponge_absorb(&c, A, 32);
    sponge_absorb(&c, m, mlen);
    sponge_finish(&c, 0x1F);
    sponge_squeeze(&c, out, p->n);
}

void or_prf(const or_params *p, const uint8_t *pk_seed, const uint8_t *sk_seed,
            const uint8_t adrs[32], uint8_t *out)
{
    g_cnt[C_PRF]++;
    if (p->shake) thshake(p, pk_seed, adrs, sk_seed, p->n, out);
    else th256(p, pk_seed, adrs, sk_seed, p->n, out);  /* SHA-256 in every SHA2 category */
}

void or_f(const or_params *p, const uint8_t *pk_seed, const uint8_t adrs[32],
          const uint8_t *m1, uint8_t *out)
{
    g_cnt[C_F]++;
    if (p->shake) thshake(p, pk_seed, adrs, m1, p->n, out);
    else th256(p, pk_seed, adrs, m1, p->n, out);  /* SHA-256 in every SHA2 category */
}

void or_h(const or_params *p, const uint8_t *pk_seed, const uint8_t adrs[32],
          const uint8_t *m2, uint8_t *out)
{
    g_cnt[C_H]++;
    if (p->shake) thshake(p, pk_seed, adrs, m2, 2 * (size_t)p->n, out);
    else if (p->wide) th512(p, pk_seed, adrs, m2, 2 * (size_t)p->n, out);
    else th256(p, pk_seed, adrs, m2, 2 * (size_t)p->n, out);
}

void or_t(const or_params *p, const uint8_t *pk_seed, const uint8_t adrs[32],
          const uint8_t *ml, size_t l_blocks, uint8_t *out)
{
    g_cnt[C_T]++;
    if (p->shake) thshake(p, pk_seed, adrs, ml, l_blocks * p->n, out);
    else if (p->wide) th512(p, pk_seed, adrs, ml, l_blocks * p->n, out);
    else th256(p, pk_seed, adrs, ml, l_blocks * p->n, out);
}

/* PRF_msg(SK.prf, opt_rand, M) = Trunc_n(HMAC-SHA-X(SK.prf, opt_rand || M)) */
void or_prf_msg(const or_params *p, const uint8_t *sk_prf, const uint8_t *opt_rand,
                const uint8_t *msg, size_t mlen, uint8_t *out)
{
    /* HMAC over the concatenation opt_rand || M, written out without a
     * temporary copy of M by feeding the inner hash in two parts. */
    g_cnt[C_PRFMSG]++;
    if (p->shake) {  /* SHAKE256(SK.prf || opt_rand || M, 8n) */
        sponge_ctx c;
        sponge_init(&c, 136);
        sponge_absorb(&c, sk_prf, p->n);
        sponge_absorb(&c, opt_rand, p->n);
        sponge_absorb(&c, msg, mlen);
        sponge_finish(&c, 0x1F);
        sponge_squeeze(&c, out, p->n);
        return;
    }
    if (!p->wide) {
        uint8_t k0[64] = {0}, ipad[64], opad[64], inner[32], mac[32];
        memcpy(k0, sk_prf, p->n);
        for (int i = 0; i < 64; i++) { ipad[i] = k0[i] ^ 0x36; opad[i] = k0[i] ^ 0x5c; }
        sha256_ctx c;
        sha256_init(&c); sha256_update(&c, ipad, 64); sha256_update(&c, opt_rand, p->n);
        sha256_update(&c, msg, mlen); sha256_final(&c, inner);
        sha256_init(&c); sha256_update(&c, opad, 64); sha256_update(&c, inner, 32);
        sha256_final(&c, mac);
        memcpy(out, mac, p->n);
    } else {
        uint8_t k0[128] = {0}, ipad[128], opad[128], inner[64], mac[64];
        memcpy(k0, sk_prf, p->n);
        for (int i = 0; i < 128; i++) { ipad[i] = k0[i] ^ 0x36; opad[i] = k0[i] ^ 0x5c; }
        sha512_ctx c;
        sha512_init(&c); sha512_update(&c, ipad, 128); sha512_update(&c, opt_rand, p->n);
        sha512_update(&c, msg, mlen); sha512_final(&c, inner);
        sha512_init(&c); sha512_update(&c, opad, 128); sha512_update(&c, inner, 64);
        sha512_final(&c, mac);
        memcpy(out, mac, p->n);
    }
}

/* H_msg(R, PK.seed, PK.root, M) =
 *   MGF1-SHA-X(R || PK.seed || SHA-X(R || PK.seed || PK.root || M), m) */
void or_h_msg(const or_params *p, const uint8_t *r, const uint8_t *pk_seed,
              const uint8_t *pk_root, const uint8_t *msg, size_t mlen, uint8_t *out)
{
    uint8_t seed[2 * OR_MAX_N + 64];
    size_t n = p->n;
    g_cnt[C_HMSG]++;
    if (p->shake) {  /* SHAKE256(R || PK.seed || PK.root || M, 8m) */
        sponge_ctx c;
        sponge_init(&c, 136);
        sponge_absorb(&c, r, n);
        sponge_absorb(&c, pk_seed, n);
        sponge_absorb(&c, pk_root, n);
        sponge_absorb(&c, msg, mlen);
        sponge_finish(&c, 0x1F);
        sponge_squeeze(&c, out, p->m);
        return;
    }
    memcpy(seed, r, n);
    memcpy(seed + n, pk_seed, n);
    if (!p->wide) {
        sha256_ctx c;
        sha256_init(&c);
        sha256_update(&c, r, n); sha256_update(&c, pk_seed, n); sha256_update(&c, pk_root, n);
        sha256_update(&c, msg, mlen);
        sha256_final(&c, seed + 2 * n);
        or_mgf1_sha256(seed, 2 * n + 32, out, p->m);
    } else {
        sha512_ctx c;
        sha512_init(&c);
        sha512_update(&c, r, n); sha512_update(&c, pk_seed, n); sha512_update(&c, pk_root, n);
        sha512_update(&c, msg, mlen);
        sha512_final(&c, seed + 2 * n);
        or_mgf1_sha512(seed, 2 * n + 64, out, p->m);
    }
}

/* ------------------------------------------------------------------------ */
/* base_2b, FIPS 205 Algorithm 4: X as a big-endian bit string, MSB first.   */
/* ------------------------------------------------------------------------ */
void or_base_2b(const uint8_t *x, int b, int out_len, uint32_t *out)
{
    size_t in = 0;
    int bits = 0;
    uint64_t total = 0;
    for (int o = 0; o < out_len; o++) {
        while (bits < b) {
            total = (total << 8) + x[in];
            in++;
            bits += 8;
        }
        bits -= b;
        out[o] = (uint32_t)((total >> bits) & ((1u << b) - 1));
        /* The definition lets total grow without bound; the bits above the
         * unread ones never reach an output, so drop them to stay in 64 bits. */
        total &= (bits ? ((1ull << bits) - 1) : 0);
    }
}

/* ------------------------------------------------------------------------ */
/* WOTS+ (FIPS 205 Section 5; paper Section II-A "Winternitz One-Time        */
/* Signature Scheme": len = len1 + len2 independent chains).                 */
/* ------------------------------------------------------------------------ */
/* chain (Algorithm 5): s applications of F starting at hash address i. */
static void chain(const or_params *p, const uint8_t *x, uint32_t i, uint32_t s,
                  const uint8_t *pk_seed, uint8_t *A, uint8_t *out)
{
    uint8_t tmp[OR_MAX_N];
    memcpy(tmp, x, p->n);
    for (uint32_t j = i; j < i + s; j++) {
        adrs_set_hash(A, j);
        or_f(p, pk_seed, A, tmp, tmp);
    }
    memcpy(out, tmp, p->n);
}

/* wots_pkGen (Algorithm 6). */
void or_wots_pkgen(const or_params *p, const uint8_t *sk_seed, const uint8_t *pk_seed,
                   const uint8_t adrs[32], uint8_t *pk)
{
    uint8_t A[32], skA[32], pkA[32], sk[OR_MAX_N];
    uint8_t tmp[OR_MAX_LEN * OR_MAX_N];
    int w = 1 << p->lg_w;
    memcpy(A, adrs, 32);
    memcpy(skA, adrs, 32);
    adrs_set_type_and_clear(skA, WOTS_PRF);
    adrs_set_keypair(skA, adrs_get_keypair(A));
    for (int i = 0; i < p->len; i++) {
        adrs_set_chain(skA, (uint32_t)i);
        or_prf(p, pk_seed, sk_seed, skA, sk);
        adrs_set_chain(A, (uint32_t)i);
        chain(p, sk, 0, (uint32_t)(w - 1), pk_seed, A, tmp + (size_t)i * p->n);
    }
    memcpy(pkA, A, 32);
    adrs_set_type_and_clear(pkA, WOTS_PK);
    adrs_set_keypair(pkA, adrs_get_keypair(A));
    or_t(p, pk_seed, pkA, tmp, (size_t)p->len, pk);
}

/* Message digits plus checksum digits (Algorithms 7 and 8, first part). */
static void wots_digits(const or_params *p, const uint8_t *msg, uint32_t *digits)
{
    int w = 1 << p->lg_w;
    uint32_t csum = 0;
    or_base_2b(msg, p->lg_w, p->len1, digits);
    for (int i = 0; i < p->len1; i++) csum += (uint32_t)(w - 1) - digits[i];
    csum <<= ((8 - ((p->len2 * p->lg_w) % 8)) % 8);
    {
        int nb = (p->len2 * p->lg_w + 7) / 8;  /* toByte(csum, ceil(len2*lg_w/8)) */
        uint8_t cb[4];
        for (int i = 0; i < nb; i++) cb[i] = (uint8_t)(csum >> (8 * (nb - 1 - i)));
        or_base_2b(cb, p->lg_w, p->len2, digits + p->len1);
    }
}

/* wots_sign (Algorithm 7). */
static void wots_sign(const or_params *p, const uint8_t *msg, const uint8_t *sk_seed,
                      const uint8_t *pk_seed, uint8_t *A, uint8_t *sig)
{
    uint32_t digits[OR_MAX_LEN];
    uint8_t skA[32], sk[OR_MAX_N];
    wots_digits(p, msg, digits);
    memcpy(skA, A, 32);
    adrs_set_type_and_clear(skA, WOTS_PRF);
    adrs_set_keypair(skA, adrs_get_keypair(A));
    for (int i = 0; i < p->len; i++) {
        adrs_set_chain(skA, (uint32_t)i);
        or_prf(p, pk_seed, sk_seed, skA, sk);
        adrs_set_chain(A, (uint32_t)i);
        chain(p, sk, 0, digits[i], pk_seed, A, sig + (size_t)i * p->n);
    }
}

/* wots_pkFromSig (Algorithm 8). */
static void wots_pk_from_sig(const or_params *p, const uint8_t *sig, const uint8_t *msg,
                             const uint8_t *pk_seed, uint8_t *A, uint8_t *pk)
{
    uint32_t digits[OR_MAX_LEN];
    uint8_t tmp[OR_MAX_LEN * OR_MAX_N], pkA[32];
    int w = 1 << p->lg_w;
    wots_digits(p, msg, digits);
    for (int i = 0; i < p->len; i++) {
        adrs_set_chain(A, (uint32_t)i);
        chain(p, sig + (size_t)i * p->n, digits[i], (uint32_t)(w - 1) - digits[i], pk_seed, A,
              tmp + (size_t)i * p->n);
    }
    memcpy(pkA, A, 32);
    adrs_set_type_and_clear(pkA, WOTS_PK);
    adrs_set_keypair(pkA, adrs_get_keypair(A));
    or_t(p, pk_seed, pkA, tmp, (size_t)p->len, pk);
}

/* ------------------------------------------------------------------------ */
/* XMSS (FIPS 205 Section 6; paper Section II-A "Merkle Signature Scheme").  */
/* ------------------------------------------------------------------------ */
/* xmss_node (Algorithm 9), recursive as defined. */
void or_xmss_node(const or_params *p, const uint8_t *sk_seed, uint32_t i, uint32_t z,
                  const uint8_t *pk_seed, const uint8_t adrs[32], uint8_t *node)
{
    uint8_t A[32];
    memcpy(A, adrs, 32);
    if (z == 0) {
        adrs_set_type_and_clear(A, WOTS_HASH);
        adrs_set_keypair(A, i);
        or_wots_pkgen(p, sk_seed, pk_seed, A, node);
    } else {
        uint8_t lr[2 * OR_MAX_N];
        or_xmss_node(p, sk_seed, 2 * i, z - 1, pk_seed, adrs, lr);
        or_xmss_node(p, sk_seed, 2 * i + 1, z - 1, pk_seed, adrs, lr + p->n);
        adrs_set_type_and_clear(A, TREE);
        adrs_set_tree_height(A, z);
        adrs_set_tree_index(A, i);
        or_h(p, pk_seed, A, lr, node);
    }
}

/* xmss_sign (Algorithm 10): WOTS+ signature of keypair idx, then h' auth nodes. */
static void xmss_sign(const or_params *p, const uint8_t *msg, const uint8_t *sk_seed,
                      uint32_t idx, const uint8_t *pk_seed, const uint8_t *adrs, uint8_t *sig)
{
    uint8_t A[32];
    uint8_t *auth = sig + (size_t)p->len * p->n;
    for (int j = 0; j < p->hp; j++) {
        uint32_t k = (idx >> j) ^ 1u;
        or_xmss_node(p, sk_seed, k, (uint32_t)j, pk_seed, adrs, auth + (size_t)j * p->n);
    }
    memcpy(A, adrs, 32);
    adrs_set_type_and_clear(A, WOTS_HASH);
    adrs_set_keypair(A, idx);
    wots_sign(p, msg, sk_seed, pk_seed, A, sig);
}

/* xmss_pkFromSig (Algorithm 11). */
void or_xmss_pk_from_sig(const or_params *p, uint32_t idx, const uint8_t *sig_xmss,
                         const uint8_t *msg_n, const uint8_t *pk_seed,
                         const uint8_t adrs[32], uint8_t *root)
{
    uint8_t A[32], node0[OR_MAX_N], buf[2 * OR_MAX_N];
    const uint8_t *auth = sig_xmss + (size_t)p->len * p->n;
    memcpy(A, adrs, 32);
    adrs_set_type_and_clear(A, WOTS_HASH);
    adrs_set_keypair(A, idx);
    wots_pk_from_sig(p, sig_xmss, msg_n, pk_seed, A, node0);
    adrs_set_type_and_clear(A, TREE);
    adrs_set_tree_index(A, idx);
    for (int k = 0; k < p->hp; k++) {
        adrs_set_tree_height(A, (uint32_t)k + 1);
        if (((idx >> k) & 1u) == 0) {
            adrs_set_tree_index(A, adrs_get_tree_index(A) / 2);
            memcpy(buf, node0, p->n);
            memcpy(buf + p->n, auth + (size_t)k * p->n, p->n);
        } else {
            adrs_set_tree_index(A, (adrs_get_tree_index(A) - 1) / 2);
            memcpy(buf, auth + (size_t)k * p->n, p->n);
            memcpy(buf + p->n, node0, p->n);
        }
        or_h(p, pk_seed, A, buf, node0);
    }
    memcpy(root, node0, p->n);
}

/* ------------------------------------------------------------------------ */
/* Hypertree (FIPS 205 Section 7; paper Section II-A "Hypertree" and the    */
/* Fig. 2 listing: leaf_idx = tree mod 2^h', tree >>= h' per layer).         */
/* ------------------------------------------------------------------------ */
/* ht_sign (Algorithm 12). */
static void ht_sign(const or_params *p, const uint8_t *msg, const uint8_t *sk_seed,
                    const uint8_t *pk_seed, uint64_t idx_tree, uint32_t idx_leaf,
                    uint8_t *sig_ht)
{
    uint8_t A[32] = {0}, root[OR_MAX_N];
    size_t xmss_bytes = (size_t)(p->len + p->hp) * p->n;
    adrs_set_tree(A, idx_tree);
    xmss_sign(p, msg, sk_seed, idx_leaf, pk_seed, A, sig_ht);
    or_xmss_pk_from_sig(p, idx_leaf, sig_ht, msg, pk_seed, A, root);
    for (int j = 1; j < p->d; j++) {
        idx_leaf = (uint32_t)(idx_tree & ((1ull << p->hp) - 1));
        idx_tree = idx_tree >> p->hp;
        adrs_set_layer(A, (uint32_t)j);
        adrs_set_tree(A, idx_tree);
        uint8_t *s = sig_ht + (size_t)j * xmss_bytes;
        xmss_sign(p, root, sk_seed, idx_leaf, pk_seed, A, s);
        if (j < p->d - 1) or_xmss_pk_from_sig(p, idx_leaf, s, root, pk_seed, A, root);
    }
}

/* ht_verify (Algorithm 13). */
static int ht_verify(const or_params *p, const uint8_t *msg, const uint8_t *sig_ht,
                     const uint8_t *pk_seed, uint64_t idx_tree, uint32_t idx_leaf,
                     const uint8_t *pk_root)
{
    uint8_t A[32] = {0}, node[OR_MAX_N];
    size_t xmss_bytes = (size_t)(p->len + p->hp) * p->n;
    adrs_set_tree(A, idx_tree);
    or_xmss_pk_from_sig(p, idx_leaf, sig_ht, msg, pk_seed, A, node);
    for (int j = 1; j < p->d; j++) {
        idx_leaf = (uint32_t)(idx_tree & ((1ull << p->hp) - 1));
        idx_tree = idx_tree >> p->hp;
        adrs_set_layer(A, (uint32_t)j);
        adrs_set_tree(A, idx_tree);
        or_xmss_pk_from_sig(p, idx_leaf, sig_ht + (size_t)j * xmss_bytes, node, pk_seed, A,
                            node);
    }
    return memcmp(node, pk_root, p->n) == 0;
}

/* ------------------------------------------------------------------------ */
/* FORS (FIPS 205 Section 8; paper Section II-A "FORS Signature").           */
/* ------------------------------------------------------------------------ */
/* fors_skGen (Algorithm 14). */
static void fors_skgen(const or_params *p, const uint8_t *sk_seed, const uint8_t *pk_seed,
                       const uint8_t *adrs, uint32_t idx, uint8_t *sk)
{
    uint8_t skA[32];
    memcpy(skA, adrs, 32);
    adrs_set_type_and_clear(skA, FORS_PRF);
    adrs_set_keypair(skA, adrs_get_keypair(adrs));
    adrs_set_tree_index(skA, idx);
    or_prf(p, pk_seed, sk_seed, skA, sk);
}

/* fors_node (Algorithm 15), recursive as defined. */
void or_fors_node(const or_params *p, const uint8_t *sk_seed, uint32_t i, uint32_t z,
                  const uint8_t *pk_seed, const uint8_t adrs[32], uint8_t *node)
{
    uint8_t A[32];
    memcpy(A, adrs, 32);
    if (z == 0) {
        uint8_t sk[OR_MAX_N];
        fors_skgen(p, sk_seed, pk_seed, adrs, i, sk);
        adrs_set_tree_height(A, 0);
        adrs_set_tree_index(A, i);
        or_f(p, pk_seed, A, sk, node);
    } else {
        uint8_t lr[2 * OR_MAX_N];
        or_fors_node(p, sk_seed, 2 * i, z - 1, pk_seed, adrs, lr);
        or_fors_node(p, sk_seed, 2 * i + 1, z - 1, pk_seed, adrs, lr + p->n);
        adrs_set_tree_height(A, z);
        adrs_set_tree_index(A, i);
        or_h(p, pk_seed, A, lr, node);
    }
}

/* fors_sign (Algorithm 16): per tree, the selected secret value and a auth nodes. */
static void fors_sign(const or_params *p, const uint8_t *md, const uint8_t *sk_seed,
                      const uint8_t *pk_seed, const uint8_t *adrs, uint8_t *sig)
{
    uint32_t idx[OR_MAX_K];
    or_base_2b(md, p->a, p->k, idx);
    for (int i = 0; i < p->k; i++) {
        uint8_t *s = sig + (size_t)i * (p->a + 1) * p->n;
        fors_skgen(p, sk_seed, pk_seed, adrs, ((uint32_t)i << p->a) + idx[i], s);
        for (int j = 0; j < p->a; j++) {
            uint32_t sib = (idx[i] >> j) ^ 1u;
            or_fors_node(p, sk_seed, ((uint32_t)i << (p->a - j)) + sib, (uint32_t)j, pk_seed,
                         adrs, s + (size_t)(j + 1) * p->n);
        }
    }
}

/* fors_pkFromSig (Algorithm 17). */
void or_fors_pk_from_sig(const or_params *p, const uint8_t *sig_fors, const uint8_t *md,
                         const uint8_t *pk_seed, const uint8_t adrs[32], uint8_t *pk)
{
    uint32_t idx[OR_MAX_K];
    uint8_t A[32], pkA[32], node0[OR_MAX_N], buf[2 * OR_MAX_N];
    uint8_t roots[OR_MAX_K * OR_MAX_N];
    memcpy(A, adrs, 32);
    or_base_2b(md, p->a, p->k, idx);
    for (int i = 0; i < p->k; i++) {
        const uint8_t *s = sig_fors + (size_t)i * (p->a + 1) * p->n;
        const uint8_t *auth = s + p->n;
        adrs_set_tree_height(A, 0);
        adrs_set_tree_index(A, ((uint32_t)i << p->a) + idx[i]);
        or_f(p, pk_seed, A, s, node0);
        for (int j = 0; j < p->a; j++) {
            adrs_set_tree_height(A, (uint32_t)j + 1);
            if (((idx[i] >> j) & 1u) == 0) {
                adrs_set_tree_index(A, adrs_get_tree_index(A) / 2);
                memcpy(buf, node0, p->n);
                memcpy(buf + p->n, auth + (size_t)j * p->n, p->n);
            } else {
                adrs_set_tree_index(A, (adrs_get_tree_index(A) - 1) / 2);
                memcpy(buf, auth + (size_t)j * p->n, p->n);
                memcpy(buf + p->n, node0, p->n);
            }
            or_h(p, pk_seed, A, buf, node0);
        }
        memcpy(roots + (size_t)i * p->n, node0, p->n);
    }
    memcpy(pkA, adrs, 32);
    adrs_set_type_and_clear(pkA, FORS_ROOTS);
    adrs_set_keypair(pkA, adrs_get_keypair(adrs));
    or_t(p, pk_seed, pkA, roots, (size_t)p->k, pk);
}

/* ------------------------------------------------------------------------ */
/* SLH-DSA internal functions (FIPS 205 Section 9; paper Fig. 2 listing).    */
/* ------------------------------------------------------------------------ */
void or_split_digest(const or_params *p, const uint8_t *digest, uint8_t *md,
                     uint64_t *idx_tree, uint32_t *idx_leaf)
{
    int md_bytes = (p->k * p->a + 7) / 8;
    int tree_bits = p->h - p->hp;
    int tree_bytes = (tree_bits + 7) / 8;
    int leaf_bytes = (p->hp + 7) / 8;
    uint64_t t = 0;
    uint32_t l = 0;
    memcpy(md, digest, md_bytes);
    for (int i = 0; i < tree_bytes; i++) t = (t << 8) | digest[md_bytes + i];   /* toInt */
    for (int i = 0; i < leaf_bytes; i++) l = (l << 8) | digest[md_bytes + tree_bytes + i];
    if (tree_bits < 64) t &= (1ull << tree_bits) - 1;   /* mod 2^(h - h/d) */
    l &= (1u << p->hp) - 1;                             /* mod 2^(h/d) */
    *idx_tree = t;
    *idx_leaf = l;
}

/* slh_keygen_internal (Algorithm 18). */
int or_keygen(const or_params *p, const uint8_t *sk_seed, const uint8_t *sk_prf,
              const uint8_t *pk_seed, uint8_t *sk, uint8_t *pk)
{
    uint8_t A[32] = {0}, root[OR_MAX_N];
    if (!p || p->n > OR_MAX_N) return -1;
    adrs_set_layer(A, (uint32_t)(p->d - 1));
    or_xmss_node(p, sk_seed, 0, (uint32_t)p->hp, pk_seed, A, root);
    memcpy(sk, sk_seed, p->n);
    memcpy(sk + p->n, sk_prf, p->n);
    memcpy(sk + 2 * p->n, pk_seed, p->n);
    memcpy(sk + 3 * p->n, root, p->n);
    memcpy(pk, pk_seed, p->n);
    memcpy(pk + p->n, root, p->n);
    return 0;
}

/* slh_sign_internal (Algorithm 19). */
int or_sign(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *sk,
            const uint8_t *addrnd, uint8_t *sig)
{
    const uint8_t *sk_seed = sk, *sk_prf = sk + p->n, *pk_seed = sk + 2 * p->n,
                  *pk_root = sk + 3 * p->n;
    uint8_t digest[128], md[128], A[32] = {0}, pk_fors[OR_MAX_N];
    uint64_t idx_tree;
    uint32_t idx_leaf;
    if (!p || p->n > OR_MAX_N || p->m > 128) return -1;
    const uint8_t *opt_rand = addrnd ? addrnd : pk_seed;
    or_prf_msg(p, sk_prf, opt_rand, msg, mlen, sig);             /* R */
    or_h_msg(p, sig, pk_seed, pk_root, msg, mlen, digest);
    or_split_digest(p, digest, md, &idx_tree, &idx_leaf);
    adrs_set_tree(A, idx_tree);
    adrs_set_type_and_clear(A, FORS_TREE);
    adrs_set_keypair(A, idx_leaf);
    uint8_t *sig_fors = sig + p->n;
    fors_sign(p, md, sk_seed, pk_seed, A, sig_fors);
    or_fors_pk_from_sig(p, sig_fors, md, pk_seed, A, pk_fors);
    uint8_t *sig_ht = sig_fors + (size_t)p->k * (p->a + 1) * p->n;
    ht_sign(p, pk_fors, sk_seed, pk_seed, idx_tree, idx_leaf, sig_ht);
    return 0;
}

/* slh_verify_internal (Algorithm 20). */
int or_verify(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *sig,
              size_t siglen, const uint8_t *pk)
{
    const uint8_t *pk_seed = pk, *pk_root = pk + p->n;
    uint8_t digest[128], md[128], A[32] = {0}, pk_fors[OR_MAX_N];
    uint64_t idx_tree;
    uint32_t idx_leaf;
    if (!p || p->n > OR_MAX_N || p->m > 128) return -1;
    if (siglen != or_sig_bytes(p)) return 0;
    or_h_msg(p, sig, pk_seed, pk_root, msg, mlen, digest);
    or_split_digest(p, digest, md, &idx_tree, &idx_leaf);
    adrs_set_tree(A, idx_tree);
    adrs_set_type_and_clear(A, FORS_TREE);
    adrs_set_keypair(A, idx_leaf);
    const uint8_t *sig_fors = sig + p->n;
    or_fors_pk_from_sig(p, sig_fors, md, pk_seed, A, pk_fors);
    const uint8_t *sig_ht = sig_fors + (size_t)p->k * (p->a + 1) * p->n;
    return ht_verify(p, pk_fors, sig_ht, pk_seed, idx_tree, idx_leaf, pk_root);
}


/* ---------------------------------------------------------------------- */
/* External interface (FIPS 205 Section 10).                               */

/* DER encodings of the hash function identifiers (FIPS 205 Section 10.2.2):
 * id-sha256 = 2.16.840.1.101.3.4.2.1 and id-sha512 = 2.16.840.1.101.3.4.2.3,
 * each as tag 06, length 09 and the nine content octets. */
static const uint8_t OID_SHA256[11] = {0x06, 0x09, 0x60, 0x86, 0x48, 0x01, 0x65, 0x03, 0x04, 0x02, 0x01};
static const uint8_t OID_SHA512[11] = {0x06, 0x09, 0x60, 0x86, 0x48, 0x01, 0x65, 0x03, 0x04, 0x02, 0x03};

long or_encode_ext(const uint8_t *msg, size_t mlen, const uint8_t *ctx, size_t ctxlen, int ph,
                   uint8_t *out)
{
    if (ctxlen > 255 || (ph != OR_PURE && ph != OR_PH_SHA256 && ph != OR_PH_SHA512)) return -1;
    size_t o = 0;
    out[o++] = (uint8_t)(ph == OR_PURE ? 0 : 1);      /* toByte(0 or 1, 1) */
    out[o++] = (uint8_t)ctxlen;                       /* toByte(|ctx|, 1) */
    if (ctxlen) memcpy(out + o, ctx, ctxlen);
    o += ctxlen;
    if (ph == OR_PURE) {
        if (mlen) memcpy(out + o, msg, mlen);
        o += mlen;
    } else if (ph == OR_PH_SHA256) {
        memcpy(out + o, OID_SHA256, 11);
        o += 11;
        or_sha256(msg, mlen, out + o);
        o += 32;
    } else {
        memcpy(out + o, OID_SHA512, 11);
        o += 11;
        or_sha512(msg, mlen, out + o);
        o += 64;
    }
    return (long)o;
}

static uint8_t *encode_alloc(const uint8_t *msg, size_t mlen, const uint8_t *ctx, size_t ctxlen, int ph,
                             long *len)
{
    uint8_t *buf = (uint8_t *)malloc(2 + ctxlen + (mlen > 75 ? mlen : 75));
    if (!buf) return NULL;
    *len = or_encode_ext(msg, mlen, ctx, ctxlen, ph, buf);
    if (*len < 0) {
        free(buf);
        return NULL;
    }
    return buf;
}

/* slh_sign (Algorithm 22) and hash_slh_sign (Algorithm 23). */
int or_sign_ext(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *ctx,
                size_t ctxlen, int ph, const uint8_t *sk, const uint8_t *addrnd, uint8_t *sig)
{
    long len;
    uint8_t *mp = encode_alloc(msg, mlen, ctx, ctxlen, ph, &len);
    if (!mp) return -1;
    int rc = or_sign(p, mp, (size_t)len, sk, addrnd, sig);
    free(mp);
    return rc;
}

/* slh_verify (Algorithm 24) and hash_slh_verify (Algorithm 25). */
int or_verify_ext(const or_params *p, const uint8_t *msg, size_t mlen, const uint8_t *ctx,
                  size_t ctxlen, int ph, const uint8_t *sig, size_t siglen, const uint8_t *pk)
{
    long len;
    uint8_t *mp = encode_alloc(msg, mlen, ctx, ctxlen, ph, &len);
    if (!mp) return -1;
    int rc = or_verify(p, mp, (size_t)len, sig, siglen, pk);
    free(mp);
    return rc;
}
