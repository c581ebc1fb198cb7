/*
 * FlexProofs CPU oracle -- byte-level entry points for the primitive layers, used by
 * the tests that pin the oracle to mathematics (field, group law, pairing,
 * hashing).  All inputs and outputs are canonical big-endian encodings:
 * F_p / F_r 32 B, G1 64 B (x||y, identity = zeros), G2 128 B (x.c0||x.c1||y.c0||y.c1),
 * G_T 384 B (12 F_p coefficients, c0.c0.c0 first).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <string.h>
#include "oracle.h"

OR_API void or_init_api(void) { or_init(); }

static const modulus *mod_of(int which) { return which ? &MR : &MP; }

/* op: 0 add, 1 sub, 2 mul, 3 inv, 4 neg, 5 sqrt (F_p only; returns 1 if square) */
OR_API int or_field_op(int which, int op, const uint8_t a[32], const uint8_t b[32], uint8_t out[32]) {
    or_init();
    const modulus *M = mod_of(which);
    fe x, y, z;
    if (mf_from_be(M, &x, a)) return -1;
    if (op <= 2 && mf_from_be(M, &y, b)) return -1;
    int ret = 0;
    switch (op) {
    case 0: mf_add(M, &z, &x, &y); break;
    case 1: mf_sub(M, &z, &x, &y); break;
    case 2: mf_mul(M, &z, &x, &y); break;
    case 3: mf_inv(M, &z, &x); break;
    case 4: mf_neg(M, &z, &x); break;
    case 5: if (which) return -1; ret = fp_sqrt(&z, &x); if (!ret) memset(&z, 0, sizeof z); break;
    default: return -1;
    }
    mf_to_be(M, out, &z);
    return ret;
}

/* F_p2 ops on 64-byte (c0||c1): 0 mul, 1 inv, 2 sqrt (returns 1 if square) */
OR_API int or_fp2_op(int op, const uint8_t a[64], const uint8_t b[64], uint8_t out[64]) {
    or_init();
    fp2 x, y, z;
    if (mf_from_be(&MP, &x.c0, a) || mf_from_be(&MP, &x.c1, a + 32)) return -1;
    int ret = 0;
    switch (op) {
    case 0:
        if (mf_from_be(&MP, &y.c0, b) || mf_from_be(&MP, &y.c1, b + 32)) return -1;
        fp2_mul(&z, &x, &y);
        break;
    case 1: fp2_inv(&z, &x); break;
    case 2: ret = fp2_sqrt(&z, &x); if (!ret) fp2_zero(&z); break;
    default: return -1;
    }
    mf_to_be(&MP, out, &z.c0);
    mf_to_be(&MP, out + 32, &z.c1);
    return ret;
}

OR_API int or_fp12_op(int op, const uint8_t a[384], const uint8_t b[384], uint8_t out[384]) {
    or_init();
    fp12 x, y, z;
    if (fp12_from_bytes(&x, a)) return -1;
    switch (op) {
    case 0: if (fp12_from_bytes(&y, b)) return -1; fp12_mul(&z, &x, &y); break;
    case 1: fp12_inv(&z, &x); break;
    case 2: final_exp(&z, &x); break;
    case 3: { /* power by a canonical F_r scalar given in b[0..32) */
        fe k;
        if (mf_from_be(&MR, &k, b)) return -1;
        fp12_pow_fr(&z, &x, &k);
        break;
    }
    default: return -1;
    }
    fp12_to_bytes(out, &z);
    return 0;
}

OR_API int or_g1_op(int op, const uint8_t P[64], const uint8_t Q_or_k[64], uint8_t out[64]) {
    or_init();
    g1a a, b, c;
    if (g1_from_bytes(&a, P)) return -1;
    switch (op) {
    case 0: if (g1_from_bytes(&b, Q_or_k)) return -1; g1_add(&c, &a, &b); break;
    case 1: { fe k; if (mf_from_be(&MR, &k, Q_or_k)) return -1; g1_mul(&c, &a, &k); break; }
    case 2: g1_neg(&c, &a); break;
    case 3: { /* multiply by an arbitrary 256-bit integer (not reduced mod r) */
        uint64_t k[4];
        for (int i = 0; i < 4; i++) {
            uint64_t w = 0;
            for (int q = 0; q < 8; q++) w = (w << 8) | Q_or_k[(3 - i) * 8 + q];
            k[i] = w;
        }
        g1j t;
        g1j_mul_canon(&t, &a, k);
        g1j_to_a(&c, &t);
        break;
    }
    default: return -1;
    }
    g1_to_bytes(out, &c);
    return 0;
}

OR_API int or_g1_check(const uint8_t P[64]) { or_init(); g1a a; return g1_from_bytes(&a, P) == 0; }

extern void g2_frobenius(g2a *o, const g2a *Q);
OR_API int or_g2_op(int op, const uint8_t P[128], const uint8_t Q_or_k[128], uint8_t out[128]) {
    or_init();
    g2a a, b, c;
    if (g2_from_bytes(&a, P)) return -1;
    switch (op) {
    case 0: if (g2_from_bytes(&b, Q_or_k)) return -1; g2_add(&c, &a, &b); break;
    case 1: { fe k; if (mf_from_be(&MR, &k, Q_or_k)) return -1; g2_mul(&c, &a, &k); break; }
    case 2: g2_neg(&c, &a); break;
    case 3: g2_frobenius(&c, &a); break;
    case 4: { /* multiply by an arbitrary 256-bit integer */
        uint64_t k[4];
        for (int i = 0; i < 4; i++) {
            uint64_t w = 0;
            for (int q = 0; q < 8; q++) w = (w << 8) | Q_or_k[(3 - i) * 8 + q];
            k[i] = w;
        }
        g2j acc, base;
        g2j_set_inf(&acc);
        g2j_from_a(&base, &a);
        for (int i = 255; i >= 0; i--) {
            g2j_dbl(&acc, &acc);
            if ((k[i / 64] >> (i % 64)) & 1) g2j_add(&acc, &acc, &base);
        }
        g2j_to_a(&c, &acc);
        break;
    }
    default: return -1;
    }
    g2_to_bytes(out, &c);
    return 0;
}

OR_API int or_g2_check(const uint8_t P[128]) { or_init(); g2a a; return g2_from_bytes(&a, P) == 0; }

OR_API void or_generators(uint8_t g1[64], uint8_t g2[128]) {
    or_init();
    g1_to_bytes(g1, &G1_GEN);
    g2_to_bytes(g2, &G2_GEN);
}

OR_API int or_pairing(const uint8_t *P, const uint8_t *Q, uint64_t n, uint8_t out[384]) {
    or_init();
    g1a *a = (g1a *)__builtin_alloca(n * sizeof(g1a) + 1);
    g2a *b = (g2a *)__builtin_alloca(n * sizeof(g2a) + 1);
    for (uint64_t i = 0; i < n; i++)
        if (g1_from_bytes(&a[i], P + 64 * i) || g2_from_bytes(&b[i], Q + 128 * i)) return -1;
    fp12 f;
    multi_pairing(&f, a, b, n);
    fp12_to_bytes(out, &f);
    return 0;
}

/* compression: kind 1 = G1 (64 -> 32), 2 = G2 (128 -> 64); decompress with negative kind */
OR_API int or_compress(int kind, const uint8_t *in, uint8_t *out) {
    or_init();
    if (kind == 1) { g1a a; if (g1_from_bytes(&a, in)) return -1; g1_compress(out, &a); return 0; }
    if (kind == 2) { g2a a; if (g2_from_bytes(&a, in)) return -1; g2_compress(out, &a); return 0; }
    if (kind == -1) { g1a a; if (g1_decompress(&a, in)) return -1; g1_to_bytes(out, &a); return 0; }
    if (kind == -2) { g2a a; if (g2_decompress(&a, in)) return -1; g2_to_bytes(out, &a); return 0; }
    return -1;
}

OR_API void or_sha256(const uint8_t *msg, uint64_t len, uint8_t out[32]) { sha256(out, msg, len); }

OR_API void or_xmd(const uint8_t *msg, uint64_t mlen, const uint8_t *dst, uint64_t dlen, uint8_t *out, uint64_t olen) {
    expand_message_xmd(out, olen, msg, mlen, dst, dlen);
}

OR_API void or_h2f(const char *dst, const uint8_t *msg, uint64_t mlen, uint8_t out[32]) {
    or_init();
    fe x;
    hash_to_fr(&x, dst, msg, mlen);
    mf_to_be(&MR, out, &x);
}
