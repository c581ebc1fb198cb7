/*
 * FlexProofs CPU oracle -- internal declarations.
 *
 * TEST INFRASTRUCTURE ONLY.  This directory is the plain, slow reference that the
 * GPU library is checked against.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code with the GPU
 * library and includes nothing from it.
 *
 * Arithmetic model (paper, Preliminaries "Bilinear Group"; evaluation section
 * names the BN_SNARK1 curve): BN254 with u = 0x44E992B44A6909F1,
 *   p = 36u^4+36u^3+24u^2+6u+1,  r = 36u^4+36u^3+18u^2+6u+1,
 *   E  : y^2 = x^3 + 3 over F_p,     g1 = (1, 2)
 *   E' : y^2 = x^3 + 3/xi over F_p2  (D-type sextic twist), xi = 9 + i
 *   F_p2 = F_p[i]/(i^2+1), F_p6 = F_p2[v]/(v^3 - xi), F_p12 = F_p6[w]/(w^2 - v)
 *   e = optimal ate pairing, final exponent exactly (p^12 - 1)/r.
 * Field elements are held as 4 x 64-bit little-endian limbs in Montgomery form
 * (R = 2^256); every value leaving the oracle is canonical.
 */
#ifndef FP_ORACLE_H
#define FP_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#define OR_API __attribute__((visibility("default")))

typedef struct { uint64_t l[4]; } fe;          /* element of F_p or F_r (Montgomery) */

typedef struct {
    uint64_t m[4];      /* modulus */
    uint64_t r2[4];     /* 2^512 mod m */
    uint64_t one[4];    /* 2^256 mod m (Montgomery 1) */
    uint64_t ninv;      /* -m^{-1} mod 2^64 */
} modulus;

extern modulus MP;  /* base field p */
extern modulus MR;  /* scalar field r */

void or_init(void);

/* ---- generic prime field ---- */
void mf_add(const modulus *M, fe *o, const fe *a, const fe *b);
void mf_sub(const modulus *M, fe *o, const fe *a, const fe *b);
void mf_neg(const modulus *M, fe *o, const fe *a);
void mf_mul(const modulus *M, fe *o, const fe *a, const fe *b);
void mf_pow(const modulus *M, fe *o, const fe *a, const uint64_t *e, int nlimbs);
void mf_inv(const modulus *M, fe *o, const fe *a);       /* a^(m-2); 0 -> 0 */
void mf_from_u64(const modulus *M, fe *o, uint64_t v);
void mf_one(const modulus *M, fe *o);
int  mf_is_zero(const fe *a);
int  mf_eq(const fe *a, const fe *b);
/* canonical big-endian 32 bytes <-> Montgomery; from_be returns -1 if >= modulus */
int  mf_from_be(const modulus *M, fe *o, const uint8_t b[32]);
void mf_to_be(const modulus *M, uint8_t b[32], const fe *a);
int  mf_from_le(const modulus *M, fe *o, const uint8_t b[32]);
void mf_to_canon(const modulus *M, uint64_t out[4], const fe *a);
/* wide big-endian byte string (up to 64 bytes) reduced mod M */
void mf_from_be_wide(const modulus *M, fe *o, const uint8_t *b, size_t len);

#define fp_add(o,a,b) mf_add(&MP,o,a,b)
#define fp_sub(o,a,b) mf_sub(&MP,o,a,b)
#define fp_neg(o,a)   mf_neg(&MP,o,a)
#define fp_mul(o,a,b) mf_mul(&MP,o,a,b)
#define fp_inv(o,a)   mf_inv(&MP,o,a)
#define fr_add(o,a,b) mf_add(&MR,o,a,b)
#define fr_sub(o,a,b) mf_sub(&MR,o,a,b)
#define fr_neg(o,a)   mf_neg(&MR,o,a)
#define fr_mul(o,a,b) mf_mul(&MR,o,a,b)
#define fr_inv(o,a)   mf_inv(&MR,o,a)

int fp_sqrt(fe *o, const fe *a);    /* returns 1 if a is a square (p = 3 mod 4) */
int fp_is_larger(const fe *y);      /* canonical y > (p-1)/2 */

/* ---- tower ---- */
typedef struct { fe c0, c1; } fp2;
typedef struct { fp2 c0, c1, c2; } fp6;
typedef struct { fp6 c0, c1; } fp12;

void fp2_add(fp2 *o, const fp2 *a, const fp2 *b);
void fp2_sub(fp2 *o, const fp2 *a, const fp2 *b);
void fp2_neg(fp2 *o, const fp2 *a);
void fp2_mul(fp2 *o, const fp2 *a, const fp2 *b);
void fp2_mul_fp(fp2 *o, const fp2 *a, const fe *b);
void fp2_inv(fp2 *o, const fp2 *a);
void fp2_conj(fp2 *o, const fp2 *a);
void fp2_mul_xi(fp2 *o, const fp2 *a);
void fp2_zero(fp2 *o);
void fp2_one(fp2 *o);
int  fp2_is_zero(const fp2 *a);
int  fp2_eq(const fp2 *a, const fp2 *b);
void fp2_pow(fp2 *o, const fp2 *a, const uint64_t *e, int nlimbs);
int  fp2_sqrt(fp2 *o, const fp2 *a);
int  fp2_is_larger(const fp2 *y);

void fp6_add(fp6 *o, const fp6 *a, const fp6 *b);
void fp6_sub(fp6 *o, const fp6 *a, const fp6 *b);
void fp6_neg(fp6 *o, const fp6 *a);
void fp6_mul(fp6 *o, const fp6 *a, const fp6 *b);
void fp6_mul_v(fp6 *o, const fp6 *a);
void fp6_inv(fp6 *o, const fp6 *a);
void fp6_zero(fp6 *o);
void fp6_one(fp6 *o);

void fp12_mul(fp12 *o, const fp12 *a, const fp12 *b);
void fp12_inv(fp12 *o, const fp12 *a);
void fp12_conj(fp12 *o, const fp12 *a);
void fp12_one(fp12 *o);
int  fp12_eq(const fp12 *a, const fp12 *b);
int  fp12_is_one(const fp12 *a);
void fp12_pow(fp12 *o, const fp12 *a, const uint64_t *e, int nlimbs);
void fp12_pow_fr(fp12 *o, const fp12 *a, const fe *k);   /* k: Montgomery F_r */
void fp12_to_bytes(uint8_t out[384], const fp12 *a);
int  fp12_from_bytes(fp12 *o, const uint8_t in[384]);

/* ---- groups ---- */
typedef struct { fe x, y; int inf; } g1a;       /* affine */
typedef struct { fe X, Y, Z; } g1j;             /* Jacobian, Z = 0 is infinity */
typedef struct { fp2 x, y; int inf; } g2a;
typedef struct { fp2 X, Y, Z; } g2j;

extern g1a G1_GEN;
extern g2a G2_GEN;

void g1j_from_a(g1j *o, const g1a *a);
void g1j_to_a(g1a *o, const g1j *a);
void g1j_set_inf(g1j *o);
void g1j_dbl(g1j *o, const g1j *a);
void g1j_add(g1j *o, const g1j *a, const g1j *b);
void g1j_neg(g1j *o, const g1j *a);
void g1_mul(g1a *o, const g1a *P, const fe *k);           /* k Montgomery F_r */
void g1j_mul_canon(g1j *o, const g1a *P, const uint64_t k[4]); /* k canonical integer */
void g1_add(g1a *o, const g1a *a, const g1a *b);
void g1_neg(g1a *o, const g1a *a);
int  g1_eq(const g1a *a, const g1a *b);
int  g1_on_curve(const g1a *a);
void g1_to_bytes(uint8_t out[64], const g1a *a);         /* x||y BE; identity = zeros */
int  g1_from_bytes(g1a *o, const uint8_t in[64]);        /* checks on-curve */
void g1_compress(uint8_t out[32], const g1a *a);
int  g1_decompress(g1a *o, const uint8_t in[32]);

void g2j_from_a(g2j *o, const g2a *a);
void g2j_to_a(g2a *o, const g2j *a);
void g2j_set_inf(g2j *o);
void g2j_dbl(g2j *o, const g2j *a);
void g2j_add(g2j *o, const g2j *a, const g2j *b);
void g2_mul(g2a *o, const g2a *P, const fe *k);
void g2_add(g2a *o, const g2a *a, const g2a *b);
void g2_neg(g2a *o, const g2a *a);
int  g2_eq(const g2a *a, const g2a *b);
int  g2_on_curve(const g2a *a);
void g2_to_bytes(uint8_t out[128], const g2a *a);        /* x.c0||x.c1||y.c0||y.c1 */
int  g2_from_bytes(g2a *o, const uint8_t in[128]);
void g2_compress(uint8_t out[64], const g2a *a);
int  g2_decompress(g2a *o, const uint8_t in[64]);

/* ---- pairing ---- */
void miller_loop(fp12 *f, const g1a *P, const g2a *Q);
void final_exp(fp12 *o, const fp12 *f);
void pairing(fp12 *o, const g1a *P, const g2a *Q);
/* prod_i e(P_i, Q_i) */
void multi_pairing(fp12 *o, const g1a *P, const g2a *Q, size_t n);

/* ---- hashing ---- */
void sha256(uint8_t out[32], const uint8_t *msg, size_t len);
void expand_message_xmd(uint8_t *out, size_t len_out, const uint8_t *msg, size_t mlen,
                        const uint8_t *dst, size_t dlen);
void hash_to_fr(fe *o, const char *dst, const uint8_t *msg, size_t mlen);

/* growable byte buffer for transcripts */
typedef struct { uint8_t *p; size_t n, cap; } bytes;
void bytes_put(bytes *b, const void *src, size_t n);
void bytes_put_u64(bytes *b, uint64_t v);
void bytes_free(bytes *b);

#endif
