/*
 * FlexProofs CPU oracle -- SHA-256 and hashing to F_r.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper models its two hash functions H, H' : {0,1}* -> F_p as random oracles
 * (Preliminaries) without fixing an instantiation.  Reading used here:
 *   SHA-256 (FIPS 180-4), and hash_to_field from RFC 9380 with
 *   expand_message_xmd(SHA-256), one element, L = 48 bytes, reduced mod r,
 * with a distinct domain-separation tag per use.
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static const uint32_t K256[64] = {
    0x428a2f98, 0x71374491, 0xb5c0fbcf, 0xe9b5dba5, 0x3956c25b, 0x59f111f1, 0x923f82a4, 0xab1c5ed5,
    0xd807aa98, 0x12835b01, 0x243185be, 0x550c7dc3, 0x72be5d74, 0x80deb1fe, 0x9bdc06a7, 0xc19bf174,
    0xe49b69c1, 0xefbe4786, 0x0fc19dc6, 0x240ca1cc, 0x2de92c6f, 0x4a7484aa, 0x5cb0a9dc, 0x76f988da,
    0x983e5152, 0xa831c66d, 0xb00327c8, 0xbf597fc7, 0xc6e00bf3, 0xd5a79147, 0x06ca6351, 0x14292967,
    0x27b70a85, 0x2e1b2138, 0x4d2c6dfc, 0x53380d13, 0x650a7354, 0x766a0abb, 0x81c2c92e, 0x92722c85,
    0xa2bfe8a1, 0xa81a664b, 0xc24b8b70, 0xc76c51a3, 0xd192e819, 0xd6990624, 0xf40e3585, 0x106aa070,
    0x19a4c116, 0x1e376c08, 0x2748774c, 0x34b0bcb5, 0x391c0cb3, 0x4ed8aa4a, 0x5b9cca4f, 0x682e6ff3,
    0x748f82ee, 0x78a5636f, 0x84c87814, 0x8cc70208, 0x90befffa, 0xa4506ceb, 0xbef9a3f7, 0xc67178f2};

static uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

static void compress(uint32_t h[8], const uint8_t blk[64]) {
    uint32_t w[64];
    for (int i = 0; i < 16; i++)
        w[i] = ((uint32_t)blk[4 * i] << 24) | ((uint32_t)blk[4 * i + 1] << 16) |
               ((uint32_t)blk[4 * i + 2] << 8) | blk[4 * i + 3];
    for (int i = 16; i < 64; i++) {
        uint32_t s0 = rotr(w[i - 15], 7) ^ rotr(w[i - 15], 18) ^ (w[i - 15] >> 3);
        uint32_t s1 = rotr(w[i - 2], 17) ^ rotr(w[i - 2], 19) ^ (w[i - 2] >> 10);
        w[i] = w[i - 16] + s0 + w[i - 7] + s1;
    }
    uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
    for (int i = 0; i < 64; i++) {
        uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
        uint32_t ch = (e & f) ^ (~e & g);
        uint32_t t1 = hh + S1 + ch + K256[i] + w[i];
        uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
        uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
        uint32_t t2 = S0 + mj;
        hh = g; g = f; f = e; e = d + t1; d = c; c = b; b = a; a = t1 + t2;
    }
    h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

void sha256(uint8_t out[32], const uint8_t *msg, size_t len) {
    uint32_t h[8] = {0x6a09e667, 0xbb67ae85, 0x3c6ef372, 0xa54ff53a,
                     0x510e527f, 0x9b05688c, 0x1f83d9ab, 0x5be0cd19};
    size_t full = len / 64;
    for (size_t i = 0; i < full; i++) compress(h, msg + 64 * i);
    uint8_t tail[128];
    size_t rem = len - 64 * full;
    memset(tail, 0, sizeof tail);
    memcpy(tail, msg + 64 * full, rem);
    tail[rem] = 0x80;
    size_t tl = (rem + 1 + 8 <= 64) ? 64 : 128;
    uint64_t bits = (uint64_t)len * 8;
    for (int i = 0; i < 8; i++) tail[tl - 1 - i] = (uint8_t)(bits >> (8 * i));
    compress(h, tail);
    if (tl == 128) compress(h, tail + 64);
    for (int i = 0; i < 8; i++) {
        out[4 * i] = (uint8_t)(h[i] >> 24);
        out[4 * i + 1] = (uint8_t)(h[i] >> 16);
        out[4 * i + 2] = (uint8_t)(h[i] >> 8);
        out[4 * i + 3] = (uint8_t)h[i];
    }
}

/* RFC 9380, section 5.3.1, with H = SHA-256 (b_in_bytes = 32, s_in_bytes = 64) */
void expand_message_xmd(uint8_t *out, size_t len_out, const uint8_t *msg, size_t mlen,
                        const uint8_t *dst, size_t dlen) {
    size_t ell = (len_out + 31) / 32;
    bytes m0 = {0};
    uint8_t zpad[64] = {0};
    bytes_put(&m0, zpad, 64);
    bytes_put(&m0, msg, mlen);
    uint8_t lib[3] = {(uint8_t)(len_out >> 8), (uint8_t)len_out, 0};
    bytes_put(&m0, lib, 3);
    bytes_put(&m0, dst, dlen);
    uint8_t dl = (uint8_t)dlen;
    bytes_put(&m0, &dl, 1);
    uint8_t b0[32], bi[32];
    sha256(b0, m0.p, m0.n);
    bytes_free(&m0);
    for (size_t i = 1; i <= ell; i++) {
        bytes mi = {0};
        uint8_t x[32];
        for (int k = 0; k < 32; k++) x[k] = (i == 1) ? b0[k] : (uint8_t)(b0[k] ^ bi[k]);
        bytes_put(&mi, x, 32);
        uint8_t ib = (uint8_t)i;
        bytes_put(&mi, &ib, 1);
        bytes_put(&mi, dst, dlen);
        bytes_put(&mi, &dl, 1);
        sha256(bi, mi.p, mi.n);
        bytes_free(&mi);
        size_t off = 32 * (i - 1), take = len_out - off < 32 ? len_out - off : 32;
        memcpy(out + off, bi, take);
    }
}

void hash_to_fr(fe *o, const char *dst, const uint8_t *msg, size_t mlen) {
    uint8_t u[48];
    expand_message_xmd(u, 48, msg, mlen, (const uint8_t *)dst, strlen(dst));
    mf_from_be_wide(&MR, o, u, 48);
}

void bytes_put(bytes *b, const void *src, size_t n) {
    if (b->n + n > b->cap) {
        size_t nc = b->cap ? b->cap : 256;
        while (nc < b->n + n) nc *= 2;
        b->p = (uint8_t *)realloc(b->p, nc);
        b->cap = nc;
    }
    if (n) memcpy(b->p + b->n, src, n);
    b->n += n;
}

void bytes_put_u64(bytes *b, uint64_t v) {
    uint8_t t[8];
    for (int i = 0; i < 8; i++) t[i] = (uint8_t)(v >> (56 - 8 * i));
    bytes_put(b, t, 8);
}

void bytes_free(bytes *b) { free(b->p); b->p = NULL; b->n = b->cap = 0; }
