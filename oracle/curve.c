/*
 * FlexProofs CPU oracle -- G1, G2 and the optimal ate pairing on BN254.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Group law: textbook Jacobian doubling/addition (x = X/Z^2, y = Y/Z^3) with the
 * special cases P = Q and P = -Q handled explicitly; scalar multiplication is
 * plain double-and-add.  Pairing (paper, Preliminaries "Bilinear Group": the
 * type-3 pairing e and the multi-pairing A*B = prod e(A[i], B[i])): affine Miller
 * loop over 6u+2 using chord/tangent lines through the untwisted points
 * psi(x, y) = (x w^2, y w^3), followed by the two Frobenius lines, then the final
 * exponentiation f^((p^12-1)/r) by plain square-and-multiply.  The exponent and
 * the Frobenius constants xi^((p-1)/3), xi^((p-1)/2) are computed at start-up
 * with small multiprecision routines written here.
 */
#include <assert.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

g1a G1_GEN;
g2a G2_GEN;

/* ---------- tiny multiprecision (little-endian 64-bit limbs) ---------- */
#define BN_MAX 56
typedef struct { uint64_t l[BN_MAX]; int n; } bn;

static void bn_set(bn *a, const uint64_t *v, int n) { memset(a, 0, sizeof *a); memcpy(a->l, v, 8 * n); a->n = n; }
static void bn_norm(bn *a) { while (a->n > 0 && a->l[a->n - 1] == 0) a->n--; }
static void bn_mul(bn *o, const bn *a, const bn *b) {
    bn r;
    memset(&r, 0, sizeof r);
    for (int i = 0; i < a->n; i++) {
        unsigned __int128 c = 0;
        for (int j = 0; j < b->n; j++) {
            c += (unsigned __int128)a->l[i] * b->l[j] + r.l[i + j];
            r.l[i + j] = (uint64_t)c;
            c >>= 64;
        }
        r.l[i + b->n] = (uint64_t)c;
    }
    r.n = a->n + b->n;
    assert(r.n <= BN_MAX);
    bn_norm(&r);
    *o = r;
}
static void bn_sub_small(bn *a, uint64_t v) {
    for (int i = 0; i < a->n && v; i++) {
        uint64_t old = a->l[i];
        a->l[i] = old - v;
        v = old < v ? 1 : 0;
    }
    bn_norm(a);
}
static int bn_bit(const bn *a, int i) { return (int)((a->l[i / 64] >> (i % 64)) & 1); }
static int bn_bits(const bn *a) {
    if (a->n == 0) return 0;
    return 64 * (a->n - 1) + 64 - __builtin_clzll(a->l[a->n - 1]);
}
/* binary long division q = a / d, returns 1 if exact */
static int bn_div(bn *q, const bn *a, const bn *d) {
    bn rem, qq;
    memset(&rem, 0, sizeof rem);
    memset(&qq, 0, sizeof qq);
    int nd = d->n + 1;
    for (int i = bn_bits(a) - 1; i >= 0; i--) {
        /* rem = 2*rem + bit */
        uint64_t carry = (uint64_t)bn_bit(a, i);
        for (int k = 0; k < nd; k++) {
            uint64_t nc = rem.l[k] >> 63;
            rem.l[k] = (rem.l[k] << 1) | carry;
            carry = nc;
        }
        /* if rem >= d: rem -= d */
        int ge = 1;
        for (int k = nd - 1; k >= 0; k--) {
            uint64_t dk = k < d->n ? d->l[k] : 0;
            if (rem.l[k] != dk) { ge = rem.l[k] > dk; break; }
        }
        if (ge) {
            unsigned __int128 br = 0;
            for (int k = 0; k < nd; k++) {
                uint64_t dk = k < d->n ? d->l[k] : 0;
                unsigned __int128 t = (unsigned __int128)rem.l[k] - dk - br;
                rem.l[k] = (uint64_t)t;
                br = (t >> 64) ? 1 : 0;
            }
            qq.l[i / 64] |= 1ULL << (i % 64);
        }
    }
    qq.n = BN_MAX;
    bn_norm(&qq);
    *q = qq;
    for (int k = 0; k < nd; k++)
        if (rem.l[k]) return 0;
    return 1;
}

static bn FE_EXP;             /* (p^12 - 1) / r */
static fp2 FROB_X, FROB_Y;    /* xi^((p-1)/3), xi^((p-1)/2) */
static fp2 TWIST_B;           /* 3 / xi, the twist's constant */
static const uint64_t ATE_LOOP = 0x9d797039be763ba8ULL;  /* low 64 bits of 6u+2; bit 64 is set */
static const int ATE_TOP = 64;                           /* 6u+2 has 65 bits */

static void set_fp_small(fe *o, uint64_t v) { mf_from_u64(&MP, o, v); }

static int fp_from_dec(fe *o, const char *s) {
    fe acc = {{0, 0, 0, 0}}, ten, d;
    set_fp_small(&ten, 10);
    for (; *s; s++) {
        fp_mul(&acc, &acc, &ten);
        set_fp_small(&d, (uint64_t)(*s - '0'));
        fp_add(&acc, &acc, &d);
    }
    *o = acc;
    return 0;
}

void curve_init(void) {
    /* G1 generator (1, 2) */
    set_fp_small(&G1_GEN.x, 1);
    set_fp_small(&G1_GEN.y, 2);
    G1_GEN.inf = 0;
    /* G2 generator: the conventional BN254 (alt_bn128) generator of the order-r subgroup */
    fp_from_dec(&G2_GEN.x.c0, "10857046999023057135944570762232829481370756359578518086990519993285655852781");
    fp_from_dec(&G2_GEN.x.c1, "11559732032986387107991004021392285783925812861821192530917403151452391805634");
    fp_from_dec(&G2_GEN.y.c0, "8495653923123431417604973247489272438418190587263600148770280649306958101930");
    fp_from_dec(&G2_GEN.y.c1, "4082367875863433681332203403145435568316851327593401208105741076214120093531");
    G2_GEN.inf = 0;

    bn p, r, t, q;
    bn_set(&p, MP.m, 4);
    bn_set(&r, MR.m, 4);
    /* FE_EXP = (p^12 - 1) / r */
    bn_set(&t, (const uint64_t[]){1}, 1);
    for (int i = 0; i < 12; i++) bn_mul(&t, &t, &p);
    bn_sub_small(&t, 1);
    int exact = bn_div(&FE_EXP, &t, &r);
    assert(exact);
    /* Frobenius constants on the twist */
    bn pm1 = p, three, two;
    bn_sub_small(&pm1, 1);
    bn_set(&three, (const uint64_t[]){3}, 1);
    bn_set(&two, (const uint64_t[]){2}, 1);
    fp2 xi;
    set_fp_small(&xi.c0, 9);
    set_fp_small(&xi.c1, 1);
    exact = bn_div(&q, &pm1, &three);
    assert(exact);
    fp2_pow(&FROB_X, &xi, q.l, q.n);
    exact = bn_div(&q, &pm1, &two);
    assert(exact);
    fp2_pow(&FROB_Y, &xi, q.l, q.n);
    fp2 three2, xinv;
    fp2_zero(&three2);
    set_fp_small(&three2.c0, 3);
    fp2_inv(&xinv, &xi);
    fp2_mul(&TWIST_B, &three2, &xinv);
    (void)exact;
}

/* ------------------------------ G1 ------------------------------ */
void g1j_set_inf(g1j *o) { memset(o, 0, sizeof *o); mf_one(&MP, &o->X); mf_one(&MP, &o->Y); }
static int g1j_is_inf(const g1j *a) { return mf_is_zero(&a->Z); }

void g1j_from_a(g1j *o, const g1a *a) {
    if (a->inf) { g1j_set_inf(o); return; }
    o->X = a->x; o->Y = a->y; mf_one(&MP, &o->Z);
}

void g1j_to_a(g1a *o, const g1j *a) {
    if (g1j_is_inf(a)) { memset(o, 0, sizeof *o); o->inf = 1; return; }
    fe zi, zi2, zi3;
    fp_inv(&zi, &a->Z);
    fp_mul(&zi2, &zi, &zi);
    fp_mul(&zi3, &zi2, &zi);
    fp_mul(&o->x, &a->X, &zi2);
    fp_mul(&o->y, &a->Y, &zi3);
    o->inf = 0;
}

void g1j_dbl(g1j *o, const g1j *a) {
    if (g1j_is_inf(a) || mf_is_zero(&a->Y)) { g1j_set_inf(o); return; }
    fe A, B, C, S, M, t, X3, Y3, Z3;
    fp_mul(&A, &a->X, &a->X);
    fp_mul(&B, &a->Y, &a->Y);
    fp_mul(&C, &B, &B);
    fp_mul(&S, &a->X, &B); fp_add(&S, &S, &S); fp_add(&S, &S, &S);       /* 4XB */
    fp_add(&M, &A, &A); fp_add(&M, &M, &A);                              /* 3A */
    fp_mul(&X3, &M, &M); fp_sub(&X3, &X3, &S); fp_sub(&X3, &X3, &S);
    fp_sub(&t, &S, &X3); fp_mul(&Y3, &M, &t);
    fp_add(&C, &C, &C); fp_add(&C, &C, &C); fp_add(&C, &C, &C);          /* 8C */
    fp_sub(&Y3, &Y3, &C);
    fp_mul(&Z3, &a->Y, &a->Z); fp_add(&Z3, &Z3, &Z3);
    o->X = X3; o->Y = Y3; o->Z = Z3;
}

void g1j_add(g1j *o, const g1j *a, const g1j *b) {
    if (g1j_is_inf(a)) { *o = *b; return; }
    if (g1j_is_inf(b)) { *o = *a; return; }
    fe Z1Z1, Z2Z2, U1, U2, S1, S2, H, R, t;
    fp_mul(&Z1Z1, &a->Z, &a->Z);
    fp_mul(&Z2Z2, &b->Z, &b->Z);
    fp_mul(&U1, &a->X, &Z2Z2);
    fp_mul(&U2, &b->X, &Z1Z1);
    fp_mul(&S1, &a->Y, &b->Z); fp_mul(&S1, &S1, &Z2Z2);
    fp_mul(&S2, &b->Y, &a->Z); fp_mul(&S2, &S2, &Z1Z1);
    fp_sub(&H, &U2, &U1);
    fp_sub(&R, &S2, &S1);
    if (mf_is_zero(&H)) {
        if (mf_is_zero(&R)) { g1j_dbl(o, a); return; }
        g1j_set_inf(o);
        return;
    }
    fe H2, H3, U1H2, X3, Y3, Z3;
    fp_mul(&H2, &H, &H);
    fp_mul(&H3, &H2, &H);
    fp_mul(&U1H2, &U1, &H2);
    fp_mul(&X3, &R, &R); fp_sub(&X3, &X3, &H3); fp_sub(&X3, &X3, &U1H2); fp_sub(&X3, &X3, &U1H2);
    fp_sub(&t, &U1H2, &X3); fp_mul(&Y3, &R, &t);
    fp_mul(&t, &S1, &H3); fp_sub(&Y3, &Y3, &t);
    fp_mul(&Z3, &a->Z, &b->Z); fp_mul(&Z3, &Z3, &H);
    o->X = X3; o->Y = Y3; o->Z = Z3;
}

void g1j_neg(g1j *o, const g1j *a) { *o = *a; fp_neg(&o->Y, &a->Y); }

void g1j_mul_canon(g1j *o, const g1a *P, const uint64_t k[4]) {
    g1j acc, base;
    g1j_set_inf(&acc);
    g1j_from_a(&base, P);
    for (int i = 255; i >= 0; i--) {
        g1j_dbl(&acc, &acc);
        if ((k[i / 64] >> (i % 64)) & 1) g1j_add(&acc, &acc, &base);
    }
    *o = acc;
}

void g1_mul(g1a *o, const g1a *P, const fe *k) {
    uint64_t c[4];
    mf_to_canon(&MR, c, k);
    g1j t;
    g1j_mul_canon(&t, P, c);
    g1j_to_a(o, &t);
}

void g1_add(g1a *o, const g1a *a, const g1a *b) {
    g1j x, y;
    g1j_from_a(&x, a);
    g1j_from_a(&y, b);
    g1j_add(&x, &x, &y);
    g1j_to_a(o, &x);
}

void g1_neg(g1a *o, const g1a *a) { *o = *a; if (!a->inf) fp_neg(&o->y, &a->y); }

int g1_eq(const g1a *a, const g1a *b) {
    if (a->inf || b->inf) return a->inf == b->inf;
    return mf_eq(&a->x, &b->x) && mf_eq(&a->y, &b->y);
}

int g1_on_curve(const g1a *a) {
    if (a->inf) return 1;
    fe l, rr, three;
    fp_mul(&l, &a->y, &a->y);
    fp_mul(&rr, &a->x, &a->x);
    fp_mul(&rr, &rr, &a->x);
    set_fp_small(&three, 3);
    fp_add(&rr, &rr, &three);
    return mf_eq(&l, &rr);
}

void g1_to_bytes(uint8_t out[64], const g1a *a) {
    if (a->inf) { memset(out, 0, 64); return; }
    mf_to_be(&MP, out, &a->x);
    mf_to_be(&MP, out + 32, &a->y);
}

int g1_from_bytes(g1a *o, const uint8_t in[64]) {
    static const uint8_t zero[64];
    if (memcmp(in, zero, 64) == 0) { memset(o, 0, sizeof *o); o->inf = 1; return 0; }
    if (mf_from_be(&MP, &o->x, in) || mf_from_be(&MP, &o->y, in + 32)) return -1;
    o->inf = 0;
    return g1_on_curve(o) ? 0 : -1;
}

void g1_compress(uint8_t out[32], const g1a *a) {
    if (a->inf) { memset(out, 0, 32); out[0] = 0x80; return; }
    mf_to_be(&MP, out, &a->x);
    if (fp_is_larger(&a->y)) out[0] |= 0x40;
}

int g1_decompress(g1a *o, const uint8_t in[32]) {
    uint8_t buf[32];
    memcpy(buf, in, 32);
    int inf = buf[0] & 0x80, big = buf[0] & 0x40;
    buf[0] &= 0x3f;
    if (inf) {
        for (int i = 0; i < 32; i++) if (buf[i] || (i == 0 && big)) return -1;
        memset(o, 0, sizeof *o);
        o->inf = 1;
        return 0;
    }
    if (mf_from_be(&MP, &o->x, buf)) return -1;
    fe rhs, three, y;
    fp_mul(&rhs, &o->x, &o->x);
    fp_mul(&rhs, &rhs, &o->x);
    set_fp_small(&three, 3);
    fp_add(&rhs, &rhs, &three);
    if (!fp_sqrt(&y, &rhs)) return -1;
    if (fp_is_larger(&y) != (big != 0)) fp_neg(&y, &y);
    o->y = y;
    o->inf = 0;
    return 0;
}

/* ------------------------------ G2 ------------------------------ */

void g2j_set_inf(g2j *o) { memset(o, 0, sizeof *o); fp2_one(&o->X); fp2_one(&o->Y); }
static int g2j_is_inf(const g2j *a) { return fp2_is_zero(&a->Z); }

void g2j_from_a(g2j *o, const g2a *a) {
    if (a->inf) { g2j_set_inf(o); return; }
    o->X = a->x; o->Y = a->y; fp2_one(&o->Z);
}

void g2j_to_a(g2a *o, const g2j *a) {
    if (g2j_is_inf(a)) { memset(o, 0, sizeof *o); o->inf = 1; return; }
    fp2 zi, zi2, zi3;
    fp2_inv(&zi, &a->Z);
    fp2_mul(&zi2, &zi, &zi);
    fp2_mul(&zi3, &zi2, &zi);
    fp2_mul(&o->x, &a->X, &zi2);
    fp2_mul(&o->y, &a->Y, &zi3);
    o->inf = 0;
}

void g2j_dbl(g2j *o, const g2j *a) {
    if (g2j_is_inf(a) || fp2_is_zero(&a->Y)) { g2j_set_inf(o); return; }
    fp2 A, B, C, S, M, t, X3, Y3, Z3;
    fp2_mul(&A, &a->X, &a->X);
    fp2_mul(&B, &a->Y, &a->Y);
    fp2_mul(&C, &B, &B);
    fp2_mul(&S, &a->X, &B); fp2_add(&S, &S, &S); fp2_add(&S, &S, &S);
    fp2_add(&M, &A, &A); fp2_add(&M, &M, &A);
    fp2_mul(&X3, &M, &M); fp2_sub(&X3, &X3, &S); fp2_sub(&X3, &X3, &S);
    fp2_sub(&t, &S, &X3); fp2_mul(&Y3, &M, &t);
    fp2_add(&C, &C, &C); fp2_add(&C, &C, &C); fp2_add(&C, &C, &C);
    fp2_sub(&Y3, &Y3, &C);
    fp2_mul(&Z3, &a->Y, &a->Z); fp2_add(&Z3, &Z3, &Z3);
    o->X = X3; o->Y = Y3; o->Z = Z3;
}

void g2j_add(g2j *o, const g2j *a, const g2j *b) {
    if (g2j_is_inf(a)) { *o = *b; return; }
    if (g2j_is_inf(b)) { *o = *a; return; }
    fp2 Z1Z1, Z2Z2, U1, U2, S1, S2, H, R, t;
    fp2_mul(&Z1Z1, &a->Z, &a->Z);
    fp2_mul(&Z2Z2, &b->Z, &b->Z);
    fp2_mul(&U1, &a->X, &Z2Z2);
    fp2_mul(&U2, &b->X, &Z1Z1);
    fp2_mul(&S1, &a->Y, &b->Z); fp2_mul(&S1, &S1, &Z2Z2);
    fp2_mul(&S2, &b->Y, &a->Z); fp2_mul(&S2, &S2, &Z1Z1);
    fp2_sub(&H, &U2, &U1);
    fp2_sub(&R, &S2, &S1);
    if (fp2_is_zero(&H)) {
        if (fp2_is_zero(&R)) { g2j_dbl(o, a); return; }
        g2j_set_inf(o);
        return;
    }
    fp2 H2, H3, U1H2, X3, Y3, Z3;
    fp2_mul(&H2, &H, &H);
    fp2_mul(&H3, &H2, &H);
    fp2_mul(&U1H2, &U1, &H2);
    fp2_mul(&X3, &R, &R); fp2_sub(&X3, &X3, &H3); fp2_sub(&X3, &X3, &U1H2); fp2_sub(&X3, &X3, &U1H2);
    fp2_sub(&t, &U1H2, &X3); fp2_mul(&Y3, &R, &t);
    fp2_mul(&t, &S1, &H3); fp2_sub(&Y3, &Y3, &t);
    fp2_mul(&Z3, &a->Z, &b->Z); fp2_mul(&Z3, &Z3, &H);
    o->X = X3; o->Y = Y3; o->Z = Z3;
}

void g2_mul(g2a *o, const g2a *P, const fe *k) {
    uint64_t c[4];
    mf_to_canon(&MR, c, k);
    g2j acc, base;
    g2j_set_inf(&acc);
    g2j_from_a(&base, P);
    for (int i = 255; i >= 0; i--) {
        g2j_dbl(&acc, &acc);
        if ((c[i / 64] >> (i % 64)) & 1) g2j_add(&acc, &acc, &base);
    }
    g2j_to_a(o, &acc);
}

void g2_add(g2a *o, const g2a *a, const g2a *b) {
    g2j x, y;
    g2j_from_a(&x, a);
    g2j_from_a(&y, b);
    g2j_add(&x, &x, &y);
    g2j_to_a(o, &x);
}

void g2_neg(g2a *o, const g2a *a) { *o = *a; if (!a->inf) fp2_neg(&o->y, &a->y); }

int g2_eq(const g2a *a, const g2a *b) {
    if (a->inf || b->inf) return a->inf == b->inf;
    return fp2_eq(&a->x, &b->x) && fp2_eq(&a->y, &b->y);
}

int g2_on_curve(const g2a *a) {
    if (a->inf) return 1;
    fp2 l, rr;
    fp2_mul(&l, &a->y, &a->y);
    fp2_mul(&rr, &a->x, &a->x);
    fp2_mul(&rr, &rr, &a->x);
    fp2_add(&rr, &rr, &TWIST_B);
    return fp2_eq(&l, &rr);
}

void g2_to_bytes(uint8_t out[128], const g2a *a) {
    if (a->inf) { memset(out, 0, 128); return; }
    mf_to_be(&MP, out, &a->x.c0);
    mf_to_be(&MP, out + 32, &a->x.c1);
    mf_to_be(&MP, out + 64, &a->y.c0);
    mf_to_be(&MP, out + 96, &a->y.c1);
}

int g2_from_bytes(g2a *o, const uint8_t in[128]) {
    static const uint8_t zero[128];
    if (memcmp(in, zero, 128) == 0) { memset(o, 0, sizeof *o); o->inf = 1; return 0; }
    if (mf_from_be(&MP, &o->x.c0, in) || mf_from_be(&MP, &o->x.c1, in + 32) ||
        mf_from_be(&MP, &o->y.c0, in + 64) || mf_from_be(&MP, &o->y.c1, in + 96))
        return -1;
    o->inf = 0;
    return g2_on_curve(o) ? 0 : -1;
}

void g2_compress(uint8_t out[64], const g2a *a) {
    if (a->inf) { memset(out, 0, 64); out[0] = 0x80; return; }
    mf_to_be(&MP, out, &a->x.c0);
    mf_to_be(&MP, out + 32, &a->x.c1);
    if (fp2_is_larger(&a->y)) out[0] |= 0x40;
}

int g2_decompress(g2a *o, const uint8_t in[64]) {
    uint8_t buf[64];
    memcpy(buf, in, 64);
    int inf = buf[0] & 0x80, big = buf[0] & 0x40;
    buf[0] &= 0x3f;
    if (inf) {
        for (int i = 0; i < 64; i++) if (buf[i] || (i == 0 && big)) return -1;
        memset(o, 0, sizeof *o);
        o->inf = 1;
        return 0;
    }
    if (mf_from_be(&MP, &o->x.c0, buf) || mf_from_be(&MP, &o->x.c1, buf + 32)) return -1;
    fp2 rhs, y;
    fp2_mul(&rhs, &o->x, &o->x);
    fp2_mul(&rhs, &rhs, &o->x);
    fp2_add(&rhs, &rhs, &TWIST_B);
    if (!fp2_sqrt(&y, &rhs)) return -1;
    if (fp2_is_larger(&y) != (big != 0)) fp2_neg(&y, &y);
    o->y = y;
    o->inf = 0;
    return 0;
}

/* p-power Frobenius of a twist point: psi^-1(pi(psi(Q))) */
void g2_frobenius(g2a *o, const g2a *Q) {
    if (Q->inf) { *o = *Q; return; }
    fp2 x, y;
    fp2_conj(&x, &Q->x);
    fp2_conj(&y, &Q->y);
    fp2_mul(&o->x, &x, &FROB_X);
    fp2_mul(&o->y, &y, &FROB_Y);
    o->inf = 0;
}

/* ------------------------------ pairing ------------------------------ */
/* value at P of the line through psi(T) with slope lambda*w:
 *   l = yP + w * ( -lambda xP + (lambda xT - yT) v )                    */
static void line_value(fp12 *l, const fp2 *lambda, const g2a *T, const g1a *P) {
    memset(l, 0, sizeof *l);
    l->c0.c0.c0 = P->y;
    fp2 t;
    fp2_mul_fp(&t, lambda, &P->x);
    fp2_neg(&l->c1.c0, &t);
    fp2_mul(&t, lambda, &T->x);
    fp2_sub(&l->c1.c1, &t, &T->y);
}

/* f <- f * l_{T,T}(P), T <- 2T */
static void step_double(fp12 *f, g2a *T, const g1a *P) {
    fp2 num, den, lambda, t;
    fp2_mul(&num, &T->x, &T->x);
    fp2_add(&t, &num, &num);
    fp2_add(&num, &t, &num);            /* 3 x^2 */
    fp2_add(&den, &T->y, &T->y);        /* 2 y */
    fp2_inv(&den, &den);
    fp2_mul(&lambda, &num, &den);
    fp12 l;
    line_value(&l, &lambda, T, P);
    fp12_mul(f, f, &l);
    fp2 x3, y3;
    fp2_mul(&x3, &lambda, &lambda);
    fp2_sub(&x3, &x3, &T->x);
    fp2_sub(&x3, &x3, &T->x);
    fp2_sub(&t, &T->x, &x3);
    fp2_mul(&y3, &lambda, &t);
    fp2_sub(&y3, &y3, &T->y);
    T->x = x3;
    T->y = y3;
}

/* f <- f * l_{T,Q}(P), T <- T + Q  (T != +-Q on every call made below) */
static void step_add(fp12 *f, g2a *T, const g2a *Q, const g1a *P) {
    fp2 num, den, lambda, t;
    fp2_sub(&num, &Q->y, &T->y);
    fp2_sub(&den, &Q->x, &T->x);
    assert(!fp2_is_zero(&den));
    fp2_inv(&den, &den);
    fp2_mul(&lambda, &num, &den);
    fp12 l;
    line_value(&l, &lambda, T, P);
    fp12_mul(f, f, &l);
    fp2 x3, y3;
    fp2_mul(&x3, &lambda, &lambda);
    fp2_sub(&x3, &x3, &T->x);
    fp2_sub(&x3, &x3, &Q->x);
    fp2_sub(&t, &T->x, &x3);
    fp2_mul(&y3, &lambda, &t);
    fp2_sub(&y3, &y3, &T->y);
    T->x = x3;
    T->y = y3;
}

void miller_loop(fp12 *f, const g1a *P, const g2a *Q) {
    fp12_one(f);
    if (P->inf || Q->inf) return;
    g2a T = *Q;
    for (int i = ATE_TOP - 1; i >= 0; i--) {
        fp12_mul(f, f, f);
        step_double(f, &T, P);
        if ((ATE_LOOP >> i) & 1) step_add(f, &T, Q, P);
    }
    g2a Q1, Q2;
    g2_frobenius(&Q1, Q);
    g2_frobenius(&Q2, &Q1);
    g2_neg(&Q2, &Q2);
    step_add(f, &T, &Q1, P);
    step_add(f, &T, &Q2, P);
}

void final_exp(fp12 *o, const fp12 *f) { fp12_pow(o, f, FE_EXP.l, FE_EXP.n); }

void pairing(fp12 *o, const g1a *P, const g2a *Q) {
    fp12 f;
    miller_loop(&f, P, Q);
    final_exp(o, &f);
}

/* the final exponentiation is a group homomorphism, so one is applied to the
 * product of the Miller values */
void multi_pairing(fp12 *o, const g1a *P, const g2a *Q, size_t n) {
    fp12 acc, f;
    fp12_one(&acc);
    for (size_t i = 0; i < n; i++) {
        miller_loop(&f, &P[i], &Q[i]);
        fp12_mul(&acc, &acc, &f);
    }
    final_exp(o, &acc);
}
