/*
 * FlexProofs CPU oracle -- prime fields F_p, F_r and the tower F_p2/F_p6/F_p12.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Montgomery multiplication (CIOS, 4 x 64-bit limbs, R = 2^256).  The constants
 * R^2 mod m and -m^{-1} mod 2^64 are derived at start-up from the modulus alone
 * (repeated doubling and a Newton iteration), so nothing here is a table copied
 * from elsewhere.  Tower formulas are the schoolbook products for the defining
 * polynomials i^2 = -1, v^3 = xi = 9 + i, w^2 = v.
 */
#include <string.h>
#include "oracle.h"

modulus MP, MR;

static const uint64_t P_LIMBS[4] = {0x3c208c16d87cfd47ULL, 0x97816a916871ca8dULL,
                                    0xb85045b68181585dULL, 0x30644e72e131a029ULL};
static const uint64_t R_LIMBS[4] = {0x43e1f593f0000001ULL, 0x2833e84879b97091ULL,
                                    0xb85045b68181585dULL, 0x30644e72e131a029ULL};

static int geq4(const uint64_t a[4], const uint64_t b[4]) {
    for (int i = 3; i >= 0; i--) {
        if (a[i] > b[i]) return 1;
        if (a[i] < b[i]) return 0;
    }
    return 1;
}

static uint64_t sub4(uint64_t o[4], const uint64_t a[4], const uint64_t b[4]) {
    unsigned __int128 borrow = 0;
    for (int i = 0; i < 4; i++) {
        unsigned __int128 d = (unsigned __int128)a[i] - b[i] - borrow;
        o[i] = (uint64_t)d;
        borrow = (d >> 64) ? 1 : 0;
    }
    return (uint64_t)borrow;
}

static uint64_t add4(uint64_t o[4], const uint64_t a[4], const uint64_t b[4]) {
    unsigned __int128 c = 0;
    for (int i = 0; i < 4; i++) {
        c += (unsigned __int128)a[i] + b[i];
        o[i] = (uint64_t)c;
        c >>= 64;
    }
    return (uint64_t)c;
}

/* (a + b) mod m for a, b < m */
static void addmod4(const uint64_t m[4], uint64_t o[4], const uint64_t a[4], const uint64_t b[4]) {
    uint64_t t[4];
    uint64_t carry = add4(t, a, b);
    if (carry || geq4(t, m)) sub4(t, t, m);
    memcpy(o, t, 32);
}

static void init_modulus(modulus *M, const uint64_t m[4]) {
    memcpy(M->m, m, 32);
    /* -m^{-1} mod 2^64 by Newton iteration: x <- x(2 - m0 x) doubles correct bits */
    uint64_t x = 1;
    for (int i = 0; i < 7; i++) x *= 2 - m[0] * x;
    M->ninv = (uint64_t)0 - x;
    /* R mod m and R^2 mod m by repeated doubling of 1 */
    uint64_t t[4] = {1, 0, 0, 0};
    for (int i = 0; i < 256; i++) addmod4(m, t, t, t);
    memcpy(M->one, t, 32);
    for (int i = 0; i < 256; i++) addmod4(m, t, t, t);
    memcpy(M->r2, t, 32);
}

void mf_add(const modulus *M, fe *o, const fe *a, const fe *b) { addmod4(M->m, o->l, a->l, b->l); }

void mf_sub(const modulus *M, fe *o, const fe *a, const fe *b) {
    uint64_t t[4];
    if (sub4(t, a->l, b->l)) add4(t, t, M->m);
    memcpy(o->l, t, 32);
}

void mf_neg(const modulus *M, fe *o, const fe *a) {
    fe z = {{0, 0, 0, 0}};
    mf_sub(M, o, &z, a);
}

void mf_mul(const modulus *M, fe *o, const fe *a, const fe *b) {
    uint64_t t[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 4; i++) {
        unsigned __int128 c = 0;
        for (int j = 0; j < 4; j++) {
            c += (unsigned __int128)a->l[j] * b->l[i] + t[j];
            t[j] = (uint64_t)c;
            c >>= 64;
        }
        c += t[4];
        t[4] = (uint64_t)c;
        t[5] = (uint64_t)(c >> 64);
        uint64_t mq = t[0] * M->ninv;
        c = (unsigned __int128)mq * M->m[0] + t[0];
        c >>= 64;
        for (int j = 1; j < 4; j++) {
            c += (unsigned __int128)mq * M->m[j] + t[j];
            t[j - 1] = (uint64_t)c;
            c >>= 64;
        }
        c += t[4];
        t[3] = (uint64_t)c;
        t[4] = t[5] + (uint64_t)(c >> 64);
    }
    uint64_t res[4] = {t[0], t[1], t[2], t[3]};
    if (t[4] || geq4(res, M->m)) sub4(res, res, M->m);
    memcpy(o->l, res, 32);
}

void mf_one(const modulus *M, fe *o) { memcpy(o->l, M->one, 32); }

void mf_from_u64(const modulus *M, fe *o, uint64_t v) {
    fe t = {{v, 0, 0, 0}}, r2;
    memcpy(r2.l, M->r2, 32);
    mf_mul(M, o, &t, &r2);
}

void mf_pow(const modulus *M, fe *o, const fe *a, const uint64_t *e, int nlimbs) {
    fe acc, base = *a;
    mf_one(M, &acc);
    for (int i = nlimbs * 64 - 1; i >= 0; i--) {
        mf_mul(M, &acc, &acc, &acc);
        if ((e[i / 64] >> (i % 64)) & 1) mf_mul(M, &acc, &acc, &base);
    }
    *o = acc;
}

void mf_inv(const modulus *M, fe *o, const fe *a) {
    uint64_t e[4];
    uint64_t two[4] = {2, 0, 0, 0};
    sub4(e, M->m, two);
    mf_pow(M, o, a, e, 4);
}

int mf_is_zero(const fe *a) { return (a->l[0] | a->l[1] | a->l[2] | a->l[3]) == 0; }
int mf_eq(const fe *a, const fe *b) { return memcmp(a->l, b->l, 32) == 0; }

void mf_to_canon(const modulus *M, uint64_t out[4], const fe *a) {
    fe one = {{1, 0, 0, 0}}, t;
    mf_mul(M, &t, a, &one);
    memcpy(out, t.l, 32);
}

static int from_limbs(const modulus *M, fe *o, const uint64_t v[4]) {
    if (geq4(v, M->m)) return -1;
    fe t, r2;
    memcpy(t.l, v, 32);
    memcpy(r2.l, M->r2, 32);
    mf_mul(M, o, &t, &r2);
    return 0;
}

int mf_from_be(const modulus *M, fe *o, const uint8_t b[32]) {
    uint64_t v[4];
    for (int i = 0; i < 4; i++) {
        uint64_t w = 0;
        for (int k = 0; k < 8; k++) w = (w << 8) | b[(3 - i) * 8 + k];
        v[i] = w;
    }
    return from_limbs(M, o, v);
}

int mf_from_le(const modulus *M, fe *o, const uint8_t b[32]) {
    uint64_t v[4];
    for (int i = 0; i < 4; i++) {
        uint64_t w = 0;
        for (int k = 7; k >= 0; k--) w = (w << 8) | b[i * 8 + k];
        v[i] = w;
    }
    return from_limbs(M, o, v);
}

void mf_to_be(const modulus *M, uint8_t b[32], const fe *a) {
    uint64_t v[4];
    mf_to_canon(M, v, a);
    for (int i = 0; i < 4; i++)
        for (int k = 0; k < 8; k++) b[(3 - i) * 8 + k] = (uint8_t)(v[i] >> (56 - 8 * k));
}

/* Horner over bytes: acc = acc*256 + byte, all mod M (plain, any length) */
void mf_from_be_wide(const modulus *M, fe *o, const uint8_t *b, size_t len) {
    fe acc = {{0, 0, 0, 0}}, k256, byte;
    mf_from_u64(M, &k256, 256);
    for (size_t i = 0; i < len; i++) {
        mf_mul(M, &acc, &acc, &k256);
        mf_from_u64(M, &byte, b[i]);
        mf_add(M, &acc, &acc, &byte);
    }
    *o = acc;
}

/* square root in F_p for p = 3 (mod 4): a^((p+1)/4), then checked by squaring */
int fp_sqrt(fe *o, const fe *a) {
    uint64_t e[4];
    uint64_t one[4] = {1, 0, 0, 0};
    add4(e, MP.m, one);               /* p + 1 fits: p < 2^254 */
    for (int i = 0; i < 4; i++) e[i] = (e[i] >> 2) | (i < 3 ? e[i + 1] << 62 : 0);
    fe s, chk;
    mf_pow(&MP, &s, a, e, 4);
    fp_mul(&chk, &s, &s);
    if (!mf_eq(&chk, a)) return 0;
    *o = s;
    return 1;
}

int fp_is_larger(const fe *y) {
    uint64_t c[4], h[4];
    mf_to_canon(&MP, c, y);
    /* (p-1)/2 */
    for (int i = 0; i < 4; i++) h[i] = (MP.m[i] >> 1) | (i < 3 ? MP.m[i + 1] << 63 : 0);
    return !geq4(h, c);   /* c > h */
}

/* ------------------------------ F_p2 ------------------------------ */
void fp2_add(fp2 *o, const fp2 *a, const fp2 *b) { fp_add(&o->c0, &a->c0, &b->c0); fp_add(&o->c1, &a->c1, &b->c1); }
void fp2_sub(fp2 *o, const fp2 *a, const fp2 *b) { fp_sub(&o->c0, &a->c0, &b->c0); fp_sub(&o->c1, &a->c1, &b->c1); }
void fp2_neg(fp2 *o, const fp2 *a) { fp_neg(&o->c0, &a->c0); fp_neg(&o->c1, &a->c1); }
void fp2_zero(fp2 *o) { memset(o, 0, sizeof *o); }
void fp2_one(fp2 *o) { memset(o, 0, sizeof *o); mf_one(&MP, &o->c0); }
int fp2_is_zero(const fp2 *a) { return mf_is_zero(&a->c0) && mf_is_zero(&a->c1); }
int fp2_eq(const fp2 *a, const fp2 *b) { return mf_eq(&a->c0, &b->c0) && mf_eq(&a->c1, &b->c1); }

void fp2_mul(fp2 *o, const fp2 *a, const fp2 *b) {
    fe t0, t1, t2, t3;
    fp_mul(&t0, &a->c0, &b->c0);
    fp_mul(&t1, &a->c1, &b->c1);
    fp_mul(&t2, &a->c0, &b->c1);
    fp_mul(&t3, &a->c1, &b->c0);
    fp_sub(&o->c0, &t0, &t1);
    fp_add(&o->c1, &t2, &t3);
}

void fp2_mul_fp(fp2 *o, const fp2 *a, const fe *b) { fp_mul(&o->c0, &a->c0, b); fp_mul(&o->c1, &a->c1, b); }

void fp2_conj(fp2 *o, const fp2 *a) { o->c0 = a->c0; fp_neg(&o->c1, &a->c1); }

void fp2_inv(fp2 *o, const fp2 *a) {
    fe n, t;
    fp_mul(&n, &a->c0, &a->c0);
    fp_mul(&t, &a->c1, &a->c1);
    fp_add(&n, &n, &t);
    fp_inv(&n, &n);
    fp2 c;
    fp2_conj(&c, a);
    fp2_mul_fp(o, &c, &n);
}

void fp2_mul_xi(fp2 *o, const fp2 *a) {
    fp2 xi;
    mf_from_u64(&MP, &xi.c0, 9);
    mf_from_u64(&MP, &xi.c1, 1);
    fp2_mul(o, a, &xi);
}

void fp2_pow(fp2 *o, const fp2 *a, const uint64_t *e, int nlimbs) {
    fp2 acc, base = *a;
    fp2_one(&acc);
    for (int i = nlimbs * 64 - 1; i >= 0; i--) {
        fp2_mul(&acc, &acc, &acc);
        if ((e[i / 64] >> (i % 64)) & 1) fp2_mul(&acc, &acc, &base);
    }
    *o = acc;
}

/*
 * Square root in F_p2 = F_p(i), i^2 = -1, by the norm method: for a = a0 + a1 i,
 * n = a0^2 + a1^2 must be a square s^2 in F_p; then x0^2 = (a0 + s)/2 (or (a0 - s)/2)
 * and x1 = a1 / (2 x0).  The candidate is verified by squaring.
 */
int fp2_sqrt(fp2 *o, const fp2 *a) {
    if (fp2_is_zero(a)) { fp2_zero(o); return 1; }
    if (mf_is_zero(&a->c1)) {
        fe s;
        if (fp_sqrt(&s, &a->c0)) { o->c0 = s; memset(&o->c1, 0, sizeof(fe)); return 1; }
        fe na;
        fp_neg(&na, &a->c0);
        if (fp_sqrt(&s, &na)) { memset(&o->c0, 0, sizeof(fe)); o->c1 = s; return 1; }
        return 0;
    }
    fe n, t, s, half, two, x0, x1;
    fp_mul(&n, &a->c0, &a->c0);
    fp_mul(&t, &a->c1, &a->c1);
    fp_add(&n, &n, &t);
    if (!fp_sqrt(&s, &n)) return 0;
    mf_from_u64(&MP, &two, 2);
    fp_inv(&half, &two);
    fp_add(&t, &a->c0, &s);
    fp_mul(&t, &t, &half);
    if (!fp_sqrt(&x0, &t)) {
        fp_sub(&t, &a->c0, &s);
        fp_mul(&t, &t, &half);
        if (!fp_sqrt(&x0, &t)) return 0;
    }
    fe d;
    fp_add(&d, &x0, &x0);
    fp_inv(&d, &d);
    fp_mul(&x1, &a->c1, &d);
    fp2 cand = {x0, x1}, chk;
    fp2_mul(&chk, &cand, &cand);
    if (!fp2_eq(&chk, a)) return 0;
    *o = cand;
    return 1;
}

/* ordering used for the compressed-point sign bit: compare c1 first, then c0 */
int fp2_is_larger(const fp2 *y) {
    if (!mf_is_zero(&y->c1)) return fp_is_larger(&y->c1);
    return fp_is_larger(&y->c0);
}

/* ------------------------------ F_p6 ------------------------------ */
void fp6_add(fp6 *o, const fp6 *a, const fp6 *b) { fp2_add(&o->c0, &a->c0, &b->c0); fp2_add(&o->c1, &a->c1, &b->c1); fp2_add(&o->c2, &a->c2, &b->c2); }
void fp6_sub(fp6 *o, const fp6 *a, const fp6 *b) { fp2_sub(&o->c0, &a->c0, &b->c0); fp2_sub(&o->c1, &a->c1, &b->c1); fp2_sub(&o->c2, &a->c2, &b->c2); }
void fp6_neg(fp6 *o, const fp6 *a) { fp2_neg(&o->c0, &a->c0); fp2_neg(&o->c1, &a->c1); fp2_neg(&o->c2, &a->c2); }
void fp6_zero(fp6 *o) { memset(o, 0, sizeof *o); }
void fp6_one(fp6 *o) { memset(o, 0, sizeof *o); fp2_one(&o->c0); }

/* schoolbook product modulo v^3 = xi */
void fp6_mul(fp6 *o, const fp6 *a, const fp6 *b) {
    fp2 p00, p01, p02, p10, p11, p12, p20, p21, p22, t;
    fp2_mul(&p00, &a->c0, &b->c0); fp2_mul(&p01, &a->c0, &b->c1); fp2_mul(&p02, &a->c0, &b->c2);
    fp2_mul(&p10, &a->c1, &b->c0); fp2_mul(&p11, &a->c1, &b->c1); fp2_mul(&p12, &a->c1, &b->c2);
    fp2_mul(&p20, &a->c2, &b->c0); fp2_mul(&p21, &a->c2, &b->c1); fp2_mul(&p22, &a->c2, &b->c2);
    fp6 r;
    /* degree 3 and 4 terms wrap around with a factor xi */
    fp2_add(&t, &p12, &p21); fp2_mul_xi(&t, &t); fp2_add(&r.c0, &p00, &t);
    fp2_mul_xi(&t, &p22); fp2_add(&r.c1, &p01, &p10); fp2_add(&r.c1, &r.c1, &t);
    fp2_add(&r.c2, &p02, &p11); fp2_add(&r.c2, &r.c2, &p20);
    *o = r;
}

void fp6_mul_v(fp6 *o, const fp6 *a) {
    fp6 r;
    fp2_mul_xi(&r.c0, &a->c2);
    r.c1 = a->c0;
    r.c2 = a->c1;
    *o = r;
}

void fp6_inv(fp6 *o, const fp6 *a) {
    fp2 A, B, C, t, F;
    fp2_mul(&A, &a->c0, &a->c0); fp2_mul(&t, &a->c1, &a->c2); fp2_mul_xi(&t, &t); fp2_sub(&A, &A, &t);
    fp2_mul(&B, &a->c2, &a->c2); fp2_mul_xi(&B, &B); fp2_mul(&t, &a->c0, &a->c1); fp2_sub(&B, &B, &t);
    fp2_mul(&C, &a->c1, &a->c1); fp2_mul(&t, &a->c0, &a->c2); fp2_sub(&C, &C, &t);
    fp2_mul(&F, &a->c0, &A);
    fp2_mul(&t, &a->c2, &B); fp2_mul_xi(&t, &t); fp2_add(&F, &F, &t);
    fp2_mul(&t, &a->c1, &C); fp2_mul_xi(&t, &t); fp2_add(&F, &F, &t);
    fp2_inv(&F, &F);
    fp2_mul(&o->c0, &A, &F);
    fp2_mul(&o->c1, &B, &F);
    fp2_mul(&o->c2, &C, &F);
}

/* ------------------------------ F_p12 ------------------------------ */
void fp12_one(fp12 *o) { fp6_one(&o->c0); fp6_zero(&o->c1); }

void fp12_mul(fp12 *o, const fp12 *a, const fp12 *b) {
    fp6 t0, t1, t2, t3;
    fp6_mul(&t0, &a->c0, &b->c0);
    fp6_mul(&t1, &a->c1, &b->c1);
    fp6_mul(&t2, &a->c0, &b->c1);
    fp6_mul(&t3, &a->c1, &b->c0);
    fp6_mul_v(&t1, &t1);
    fp6_add(&o->c0, &t0, &t1);
    fp6_add(&o->c1, &t2, &t3);
}

void fp12_conj(fp12 *o, const fp12 *a) { o->c0 = a->c0; fp6_neg(&o->c1, &a->c1); }

void fp12_inv(fp12 *o, const fp12 *a) {
    fp6 t0, t1;
    fp6_mul(&t0, &a->c0, &a->c0);
    fp6_mul(&t1, &a->c1, &a->c1);
    fp6_mul_v(&t1, &t1);
    fp6_sub(&t0, &t0, &t1);
    fp6_inv(&t0, &t0);
    fp6_mul(&o->c0, &a->c0, &t0);
    fp6_mul(&t1, &a->c1, &t0);
    fp6_neg(&o->c1, &t1);
}

int fp12_eq(const fp12 *a, const fp12 *b) { return memcmp(a, b, sizeof *a) == 0; }

int fp12_is_one(const fp12 *a) {
    fp12 one;
    fp12_one(&one);
    return fp12_eq(a, &one);
}

void fp12_pow(fp12 *o, const fp12 *a, const uint64_t *e, int nlimbs) {
    fp12 acc, base = *a;
    fp12_one(&acc);
    for (int i = nlimbs * 64 - 1; i >= 0; i--) {
        fp12_mul(&acc, &acc, &acc);
        if ((e[i / 64] >> (i % 64)) & 1) fp12_mul(&acc, &acc, &base);
    }
    *o = acc;
}

void fp12_pow_fr(fp12 *o, const fp12 *a, const fe *k) {
    uint64_t c[4];
    mf_to_canon(&MR, c, k);
    fp12_pow(o, a, c, 4);
}

static const fe *fp12_coeff(const fp12 *a, int idx) {
    const fp6 *h = idx < 6 ? &a->c0 : &a->c1;
    int j = idx % 6;
    const fp2 *q = j < 2 ? &h->c0 : (j < 4 ? &h->c1 : &h->c2);
    return (j & 1) ? &q->c1 : &q->c0;
}

void fp12_to_bytes(uint8_t out[384], const fp12 *a) {
    for (int i = 0; i < 12; i++) mf_to_be(&MP, out + 32 * i, fp12_coeff(a, i));
}

int fp12_from_bytes(fp12 *o, const uint8_t in[384]) {
    for (int i = 0; i < 12; i++)
        if (mf_from_be(&MP, (fe *)fp12_coeff(o, i), in + 32 * i)) return -1;
    return 0;
}

extern void curve_init(void);
void or_init(void) {
    static int done = 0;
    if (done) return;
    init_modulus(&MP, P_LIMBS);
    init_modulus(&MR, R_LIMBS);
    curve_init();
    done = 1;
}
