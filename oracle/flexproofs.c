/*
 * FlexProofs CPU oracle -- PST, the FC scheme with batch openings, and the VC
 * scheme's Commit / OpenAll / Verify, plus the naive one-proof-at-a-time openers
 * used to pin OpenAll.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Notation: L = log2 N, lK = floor(L/2), K = 2^lK subvectors (the FC vector
 * length), lM = L - lK, M = 2^lM entries per subvector; i = jM + a.  For even L,
 * K = M = mu = sqrt(N) as in the paper (section 4.1).
 *
 * Readings of points the paper leaves open (transcript layout, hash domains,
 * the faster-verifier data, PST details, Merkle leaves) are stated next to the
 * code that uses them.  All group outputs are exact, so every byte is unique.
 */
#include <assert.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define DST_SETUP "FLEXPROOFS-V1-SETUP"
#define DST_FC_R "FLEXPROOFS-V1-FC-R"
#define DST_FC_X "FLEXPROOFS-V1-FC-X"
#define DST_FC_Z "FLEXPROOFS-V1-FC-Z"
#define DST_RHO "FLEXPROOFS-V1-RHO"
#define DST_EVAL "FLEXPROOFS-V1-EVAL"

typedef struct {
    uint32_t L, lK, lM;
    uint64_t N, K, M;
    fe *s;          /* PST trapdoor s_0..s_{lM-1} (test setup only) */
    fe beta;        /* FC trapdoor */
    g1a **ek;       /* ek[k][c] = eq_k(c; s) g1 for k = 0..lM, c < 2^k */
    g2a *vk;        /* vk[t] = s_t g2 */
    g2a *h;         /* h[k] = beta^k g2, k < 2K-1;  FC key v[i] = h[2i] */
    g1a g1beta;     /* beta g1 */
} params;

typedef struct {
    const params *pp;
    fe *m;          /* N entries (Montgomery F_r) */
    g1a *Cj;        /* K PST commitments (aux) */
    fp12 C;         /* VC commitment */
} commitment;

typedef struct {
    uint32_t t;
    uint64_t first;
    fp12 *Lgt, *Rgt;
    g1a *Lg1, *Rg1;
    fe *x;
    g1a A;
    g2a v, piv;
} fcproof;

typedef struct {
    const commitment *cm;
    uint32_t b;
    uint64_t nb;
    fcproof *bt;
    uint8_t *mt;    /* Merkle tree, heap order, node n at 32n, root = node 1, leaf i = node N+i */
    fe *rho;        /* K */
    fe *y;          /* fold tree rows, level h node w at (off(h)+w)*M */
    g1a *D;         /* fold tree commitments, level h node w at off(h)+w */
    g1a *W;         /* HyperEval quotient commitments, depth d prefix p at 2^d-1+p */
} opening;

/* set by tests: check the FC correctness invariant after every round */
static int g_check_invariant = 0;
static long g_invariant_checks = 0, g_invariant_failures = 0;

static uint64_t lvl_off(uint64_t K, uint32_t h) { return 2 * K - (2 * K >> h); }

static void enc_fr(uint8_t o[32], const fe *a) { mf_to_be(&MR, o, a); }
static void put_fr(bytes *b, const fe *a) { uint8_t t[32]; enc_fr(t, a); bytes_put(b, t, 32); }
static void put_g1(bytes *b, const g1a *a) { uint8_t t[64]; g1_to_bytes(t, a); bytes_put(b, t, 64); }
static void put_g2(bytes *b, const g2a *a) { uint8_t t[128]; g2_to_bytes(t, a); bytes_put(b, t, 128); }
static void put_gt(bytes *b, const fp12 *a) { uint8_t t[384]; fp12_to_bytes(t, a); bytes_put(b, t, 384); }

/* sum_i k_i P_i by definition (plain double-and-add per term) */
static void g1_msm(g1a *o, const g1a *P, const fe *k, size_t n) {
    g1j acc, t;
    g1j_set_inf(&acc);
    for (size_t i = 0; i < n; i++) {
        uint64_t c[4];
        mf_to_canon(&MR, c, &k[i]);
        g1j_mul_canon(&t, &P[i], c);
        g1j_add(&acc, &acc, &t);
    }
    g1j_to_a(o, &acc);
}

static void g2_msm(g2a *o, const g2a *P, const fe *k, size_t n) {
    g2j acc, t;
    g2j_set_inf(&acc);
    for (size_t i = 0; i < n; i++) {
        g2a q;
        g2_mul(&q, &P[i], &k[i]);
        g2j_from_a(&t, &q);
        g2j_add(&acc, &acc, &t);
    }
    g2j_to_a(o, &acc);
}

/* ================================ Setup ================================ */
/*
 * PC.Setup(1, log M) and FC.Setup(1^K) (VC.Setup, Eq. vcpp).  Test trapdoor:
 *   s_t = H2F(DST_SETUP, seed || "s" || t),  beta = H2F(DST_SETUP, seed || "beta").
 * PST keys in the Lagrange basis at every level k <= lM, with variable x_t paired
 * to bit t of the index (Eq. multi-extension):
 *   ek_k[c] = prod_{t<k} (c_t s_t + (1-c_t)(1-s_t)) g1.
 * FC keys (FC.Setup): v = (g2^{beta^{2i}})_{i<K}.  The faster verifier (section 3)
 * needs a commitment key for polynomials of degree 2K-2 in G2, so all powers
 * h_k = beta^k g2, k < 2K-1, are published (v[i] = h_{2i}) together with beta g1.
 */
OR_API void *or_setup(uint32_t log_n, const uint8_t seed[32]) {
    or_init();
    if (log_n < 2 || log_n > 30) return NULL;
    params *pp = (params *)calloc(1, sizeof *pp);
    pp->L = log_n;
    pp->lK = log_n / 2;
    pp->lM = log_n - pp->lK;
    pp->N = 1ULL << log_n;
    pp->K = 1ULL << pp->lK;
    pp->M = 1ULL << pp->lM;
    pp->s = (fe *)calloc(pp->lM, sizeof(fe));
    for (uint32_t t = 0; t < pp->lM; t++) {
        bytes b = {0};
        bytes_put(&b, seed, 32);
        bytes_put(&b, "s", 1);
        bytes_put_u64(&b, t);
        hash_to_fr(&pp->s[t], DST_SETUP, b.p, b.n);
        bytes_free(&b);
    }
    {
        bytes b = {0};
        bytes_put(&b, seed, 32);
        bytes_put(&b, "beta", 4);
        hash_to_fr(&pp->beta, DST_SETUP, b.p, b.n);
        bytes_free(&b);
    }
    fe one;
    mf_one(&MR, &one);
    pp->ek = (g1a **)calloc(pp->lM + 1, sizeof(g1a *));
    for (uint32_t k = 0; k <= pp->lM; k++) {
        uint64_t n = 1ULL << k;
        pp->ek[k] = (g1a *)calloc(n, sizeof(g1a));
        #pragma omp parallel for schedule(dynamic, 16)
        for (uint64_t c = 0; c < n; c++) {
            fe e = one, f;
            for (uint32_t t = 0; t < k; t++) {
                if ((c >> t) & 1) f = pp->s[t];
                else fr_sub(&f, &one, &pp->s[t]);
                fr_mul(&e, &e, &f);
            }
            g1_mul(&pp->ek[k][c], &G1_GEN, &e);
        }
    }
    pp->vk = (g2a *)calloc(pp->lM, sizeof(g2a));
    for (uint32_t t = 0; t < pp->lM; t++) g2_mul(&pp->vk[t], &G2_GEN, &pp->s[t]);
    uint64_t nh = 2 * pp->K - 1;
    pp->h = (g2a *)calloc(nh, sizeof(g2a));
    fe *pw = (fe *)calloc(nh, sizeof(fe));
    pw[0] = one;
    for (uint64_t k = 1; k < nh; k++) fr_mul(&pw[k], &pw[k - 1], &pp->beta);
    #pragma omp parallel for schedule(dynamic, 4)
    for (uint64_t k = 0; k < nh; k++) g2_mul(&pp->h[k], &G2_GEN, &pw[k]);
    free(pw);
    g1_mul(&pp->g1beta, &G1_GEN, &pp->beta);
    return pp;
}

OR_API void or_params_free(void *p) {
    params *pp = (params *)p;
    if (!pp) return;
    for (uint32_t k = 0; k <= pp->lM; k++) free(pp->ek[k]);
    free(pp->ek);
    free(pp->vk);
    free(pp->h);
    free(pp->s);
    free(pp);
}

/* what: 0 ek level idx (2^idx x 64 B), 1 vk (lM x 128 B), 2 h (2K-1 x 128 B),
 *       3 g1beta (64 B), 4 trapdoor s (lM x 32 B) then beta (32 B) */
OR_API int or_params_export(void *p, int what, uint32_t idx, uint8_t *out) {
    params *pp = (params *)p;
    switch (what) {
    case 0:
        if (idx > pp->lM) return -1;
        for (uint64_t c = 0; c < (1ULL << idx); c++) g1_to_bytes(out + 64 * c, &pp->ek[idx][c]);
        return 0;
    case 1:
        for (uint32_t t = 0; t < pp->lM; t++) g2_to_bytes(out + 128 * t, &pp->vk[t]);
        return 0;
    case 2:
        for (uint64_t k = 0; k < 2 * pp->K - 1; k++) g2_to_bytes(out + 128 * k, &pp->h[k]);
        return 0;
    case 3:
        g1_to_bytes(out, &pp->g1beta);
        return 0;
    case 4:
        for (uint32_t t = 0; t < pp->lM; t++) enc_fr(out + 32 * t, &pp->s[t]);
        enc_fr(out + 32 * pp->lM, &pp->beta);
        return 0;
    }
    return -1;
}

/* ================================ Commit ================================ */
/* PC.Commit: C_j = sum_a m[jM+a] ek_lM[a] = f_j(s) g1 (Eq. genCi);
 * FC.Commit: C = Cvec * v = prod_j e(C_j, v[j])   (Eq. genC, FC.Commit) */
OR_API void *or_commit(void *p, const uint8_t *m_le, uint64_t n) {
    params *pp = (params *)p;
    if (n != pp->N) return NULL;
    commitment *cm = (commitment *)calloc(1, sizeof *cm);
    cm->pp = pp;
    cm->m = (fe *)calloc(n, sizeof(fe));
    for (uint64_t i = 0; i < n; i++)
        if (mf_from_le(&MR, &cm->m[i], m_le + 32 * i)) { free(cm->m); free(cm); return NULL; }
    cm->Cj = (g1a *)calloc(pp->K, sizeof(g1a));
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t j = 0; j < pp->K; j++) g1_msm(&cm->Cj[j], pp->ek[pp->lM], &cm->m[j * pp->M], pp->M);
    g2a *v = (g2a *)calloc(pp->K, sizeof(g2a));
    for (uint64_t j = 0; j < pp->K; j++) v[j] = pp->h[2 * j];
    /* Miller values in parallel, then one final exponentiation of their product */
    fp12 *f = (fp12 *)calloc(pp->K, sizeof(fp12));
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t j = 0; j < pp->K; j++) miller_loop(&f[j], &cm->Cj[j], &v[j]);
    fp12 acc;
    fp12_one(&acc);
    for (uint64_t j = 0; j < pp->K; j++) fp12_mul(&acc, &acc, &f[j]);
    final_exp(&cm->C, &acc);
    free(f);
    free(v);
    return cm;
}

OR_API void or_commit_free(void *c) {
    commitment *cm = (commitment *)c;
    if (!cm) return;
    free(cm->m);
    free(cm->Cj);
    free(cm);
}

OR_API int or_commit_export(void *c, uint8_t *Cj, uint8_t C[384]) {
    commitment *cm = (commitment *)c;
    for (uint64_t j = 0; j < cm->pp->K; j++) g1_to_bytes(Cj + 64 * j, &cm->Cj[j]);
    fp12_to_bytes(C, &cm->C);
    return 0;
}

/* ============================ FC.BOpen ============================ */
/*
 * Reading of the batching coefficients r_i = H(b^(i), C, {b^(k)}, {y_k}) (FC.BOpen,
 * Eq. eqn:b): every b^(i) here is a unit vector u_{a_i}, encoded by its index, and
 * the whole statement is hashed once into a seed.  The statement list is hashed in
 * chunks of FC_CHUNK entries so that the chunk digests can be computed in parallel:
 *   H_q   = SHA-256((a_i || enc(y_i)) for i in [q FC_CHUNK, (q+1) FC_CHUNK) cap [0, t)),
 *   sigma = SHA-256(DST_FC_R || enc(C) || t || H_0 || H_1 || ...),
 *   r_i   = H2F(DST_FC_R, sigma || i).
 */
#define FC_CHUNK 32
static void fc_batch_coeffs(fe *r, const fp12 *C, const uint64_t *idx, const g1a *y, uint32_t t) {
    bytes b = {0};
    bytes_put(&b, DST_FC_R, strlen(DST_FC_R));
    put_gt(&b, C);
    bytes_put_u64(&b, t);
    for (uint32_t q = 0; q * FC_CHUNK < t; q++) {
        bytes c = {0};
        for (uint32_t i = q * FC_CHUNK; i < t && i < (q + 1) * FC_CHUNK; i++) {
            bytes_put_u64(&c, idx[i]);
            put_g1(&c, &y[i]);
        }
        uint8_t hq[32];
        sha256(hq, c.p, c.n);
        bytes_free(&c);
        bytes_put(&b, hq, 32);
    }
    uint8_t sigma[32];
    sha256(sigma, b.p, b.n);
    bytes_free(&b);
    for (uint32_t i = 0; i < t; i++) {
        bytes m = {0};
        bytes_put(&m, sigma, 32);
        bytes_put_u64(&m, i);
        hash_to_fr(&r[i], DST_FC_R, m.p, m.n);
        bytes_free(&m);
    }
}

/* x_j = H'(x_{j-1}, L_j, R_j) with x_0 the empty string (Eq. folding) */
static int fc_challenge(fe *x, const fe *xprev, int first, const fp12 *Lgt, const g1a *Lg1,
                        const fp12 *Rgt, const g1a *Rg1) {
    bytes b = {0};
    if (!first) put_fr(&b, xprev);
    put_gt(&b, Lgt);
    put_g1(&b, Lg1);
    put_gt(&b, Rgt);
    put_g1(&b, Rg1);
    hash_to_fr(x, DST_FC_X, b.p, b.n);
    bytes_free(&b);
    return mf_is_zero(x) ? -1 : 0;
}

static fe fc_z_challenge(const fe *xl, const g2a *vl) {
    bytes b = {0};
    put_fr(&b, xl);
    put_g2(&b, vl);
    fe z;
    hash_to_fr(&z, DST_FC_Z, b.p, b.n);
    bytes_free(&b);
    return z;
}

/* coefficients of f_v(X) = prod_{j=1}^{l} (1 + x_j^{-1} X^{2^{l-j+1}}), degree 2K-2:
 * v_l = f_v(beta) g2 is the folded FC key (v_j = (v_{j-1})_L o ((v_{j-1})_R)^{1/x_j}). */
static fe *fv_coeffs(const fe *xinv, uint32_t l, uint64_t K) {
    uint64_t deg = 2 * K - 2;
    fe *c = (fe *)calloc(deg + 1, sizeof(fe));
    mf_one(&MR, &c[0]);
    uint64_t cur = 0;
    for (uint32_t j = 1; j <= l; j++) {
        uint64_t e = 1ULL << (l - j + 1);
        for (int64_t k = (int64_t)cur; k >= 0; k--) {
            fe t;
            fr_mul(&t, &c[k], &xinv[j - 1]);
            fr_add(&c[k + e], &c[k + e], &t);
        }
        cur += e;
    }
    assert(cur == deg);
    return c;
}

static fe poly_eval(const fe *c, uint64_t deg, const fe *z) {
    fe acc = c[deg];
    for (int64_t k = (int64_t)deg - 1; k >= 0; k--) {
        fr_mul(&acc, &acc, z);
        fr_add(&acc, &acc, &c[k]);
    }
    return acc;
}

/*
 * FC.BOpen(C, A, {u_{a_i}}, {y_i = A[a_i]}) with the faster verifier (section 3):
 * l halving rounds of Eq. folding on (A, v, b) with dense b = sum_i r_i u_{a_i}
 * (Eq. eqn:b), then the folded key v_l and a KZG-style proof in G2 that
 * v_l = f_v(beta) g2, opened at z = H'(x_l, v_l): pi_v = q(beta) g2 with
 * q = (f_v - f_v(z)) / (X - z).
 */
static int fc_bopen_b(fcproof *pr, const params *pp, const fp12 *C, const g1a *Avec, const fe *bvec,
                      const g1a *claim);

static int fc_bopen(fcproof *pr, const params *pp, const fp12 *C, const g1a *Avec,
                    const uint64_t *idx, uint32_t t) {
    uint64_t K = pp->K;
    pr->t = t;
    pr->first = idx[0];
    fe *b = (fe *)calloc(K, sizeof(fe));
    fe *r = (fe *)calloc(t, sizeof(fe));
    g1a *yv = (g1a *)calloc(t, sizeof(g1a));
    for (uint32_t i = 0; i < t; i++) yv[i] = Avec[idx[i]];
    fc_batch_coeffs(r, C, idx, yv, t);
    for (uint32_t i = 0; i < t; i++) fr_add(&b[idx[i]], &b[idx[i]], &r[i]);
    /* the claim y = prod y_i^{r_i} (Eq. comy), for the invariant bookkeeping */
    g1a Cg1;
    memset(&Cg1, 0, sizeof Cg1);
    if (g_check_invariant) g1_msm(&Cg1, yv, r, t);
    int rc = fc_bopen_b(pr, pp, C, Avec, b, &Cg1);
    free(b); free(r); free(yv);
    return rc;
}

/* The rounds of FC.BOpen for a given dense b (Eq. folding) and the faster verifier's pi_v;
 * claim: <A, b>, used only by the invariant bookkeeping */
static int fc_bopen_b(fcproof *pr, const params *pp, const fp12 *C, const g1a *Avec, const fe *bvec,
                      const g1a *claim) {
    uint64_t K = pp->K;
    uint32_t l = pp->lK;
    pr->Lgt = (fp12 *)calloc(l, sizeof(fp12));
    pr->Rgt = (fp12 *)calloc(l, sizeof(fp12));
    pr->Lg1 = (g1a *)calloc(l, sizeof(g1a));
    pr->Rg1 = (g1a *)calloc(l, sizeof(g1a));
    pr->x = (fe *)calloc(l, sizeof(fe));
    g1a *A = (g1a *)malloc(K * sizeof(g1a));
    g2a *v = (g2a *)malloc(K * sizeof(g2a));
    fe *b = (fe *)calloc(K, sizeof(fe));
    memcpy(A, Avec, K * sizeof(g1a));
    memcpy(b, bvec, K * sizeof(fe));
    for (uint64_t i = 0; i < K; i++) v[i] = pp->h[2 * i];
    /* invariant bookkeeping: the verifier's running pair C_j = (C_gt, C_g1) */
    fp12 Cgt = *C;
    g1a Cg1 = *claim;
    fe *xinv = (fe *)calloc(l, sizeof(fe));
    int rc = 0;
    for (uint32_t j = 1; j <= l; j++) {
        uint64_t h = K >> j;
        multi_pairing(&pr->Lgt[j - 1], A + h, v, h);
        multi_pairing(&pr->Rgt[j - 1], A, v + h, h);
        g1_msm(&pr->Lg1[j - 1], A + h, b, h);
        g1_msm(&pr->Rg1[j - 1], A, b + h, h);
        if (fc_challenge(&pr->x[j - 1], j > 1 ? &pr->x[j - 2] : NULL, j == 1, &pr->Lgt[j - 1],
                         &pr->Lg1[j - 1], &pr->Rgt[j - 1], &pr->Rg1[j - 1])) {
            rc = -2;
            break;
        }
        fe x = pr->x[j - 1];
        fr_inv(&xinv[j - 1], &x);
        for (uint64_t i = 0; i < h; i++) {
            g1a t1;
            g1_mul(&t1, &A[h + i], &x);
            g1_add(&A[i], &A[i], &t1);
            g2a t2;
            g2_mul(&t2, &v[h + i], &xinv[j - 1]);
            g2_add(&v[i], &v[i], &t2);
            fe t3;
            fr_mul(&t3, &b[h + i], &xinv[j - 1]);
            fr_add(&b[i], &b[i], &t3);
        }
        if (g_check_invariant) {
            /* C_j = L_j^{x_j} o C_{j-1} o R_j^{1/x_j} must equal (A_j * v_j, <A_j, b_j>) */
            fp12 a1, a2;
            fp12_pow_fr(&a1, &pr->Lgt[j - 1], &x);
            fp12_pow_fr(&a2, &pr->Rgt[j - 1], &xinv[j - 1]);
            fp12_mul(&Cgt, &Cgt, &a1);
            fp12_mul(&Cgt, &Cgt, &a2);
            g1a s1, s2;
            g1_mul(&s1, &pr->Lg1[j - 1], &x);
            g1_mul(&s2, &pr->Rg1[j - 1], &xinv[j - 1]);
            g1_add(&Cg1, &Cg1, &s1);
            g1_add(&Cg1, &Cg1, &s2);
            fp12 want_gt;
            g1a want_g1;
            multi_pairing(&want_gt, A, v, h);
            g1_msm(&want_g1, A, b, h);
            #pragma omp atomic
            g_invariant_checks++;
            if (!fp12_eq(&want_gt, &Cgt) || !g1_eq(&want_g1, &Cg1)) {
                #pragma omp atomic
                g_invariant_failures++;
            }
        }
    }
    if (rc == 0) {
        pr->A = A[0];
        pr->v = v[0];
        fe *c = fv_coeffs(xinv, l, K);
        uint64_t deg = 2 * K - 2;
        fe z = fc_z_challenge(&pr->x[l - 1], &pr->v);
        /* synthetic division by (X - z): q_{k-1} = c_k + z q_k */
        fe *q = (fe *)calloc(deg, sizeof(fe));
        fe carry = {{0, 0, 0, 0}};
        for (int64_t k = (int64_t)deg; k >= 1; k--) {
            fe t1;
            fr_mul(&t1, &carry, &z);
            fr_add(&carry, &c[k], &t1);
            q[k - 1] = carry;
        }
        g2_msm(&pr->piv, pp->h, q, deg);
        free(q);
        free(c);
    }
    free(xinv);
    free(A);
    free(v);
    free(b);
    return rc;
}

static void fcproof_free(fcproof *pr) {
    free(pr->Lgt); free(pr->Rgt); free(pr->Lg1); free(pr->Rg1); free(pr->x);
}

/* ============================ OpenAll ============================ */
static void merkle_leaf(uint8_t out[32], const fe *m, const g1a *Cj) {
    uint8_t buf[1 + 32 + 64];
    buf[0] = 0x00;
    enc_fr(buf + 1, m);
    g1_to_bytes(buf + 33, Cj);
    sha256(out, buf, sizeof buf);
}

static void merkle_node(uint8_t out[32], const uint8_t *l, const uint8_t *r) {
    uint8_t buf[65];
    buf[0] = 0x01;
    memcpy(buf + 1, l, 32);
    memcpy(buf + 33, r, 32);
    sha256(out, buf, sizeof buf);
}

static void rho_challenge(fe *o, const fp12 *C, const uint8_t root[32], uint64_t j) {
    bytes b = {0};
    put_gt(&b, C);
    bytes_put(&b, root, 32);
    bytes_put_u64(&b, j);
    hash_to_fr(o, DST_RHO, b.p, b.n);
    bytes_free(&b);
}

/* PST quotient commitment for prefix table T of size 2^k (k >= 1):
 * Q = T_hi - T_lo, committed with ek_{k-1} */
static void pst_quotient(g1a *o, const params *pp, const fe *T, uint32_t k) {
    uint64_t half = 1ULL << (k - 1);
    fe *Q = (fe *)malloc(half * sizeof(fe));
    for (uint64_t c = 0; c < half; c++) fr_sub(&Q[c], &T[half + c], &T[c]);
    g1_msm(o, pp->ek[k - 1], Q, half);
    free(Q);
}

/* VC.OpenAll: Protocol 1 made non-interactive (section 4.2). */
OR_API void *or_open_all(void *c, uint32_t b) {
    commitment *cm = (commitment *)c;
    const params *pp = cm->pp;
    uint64_t K = pp->K, M = pp->M, N = pp->N;
    if (b < 1 || b > K) return NULL;
    opening *op = (opening *)calloc(1, sizeof *op);
    op->cm = cm;
    op->b = b;
    op->nb = (K + b - 1) / b;
    op->bt = (fcproof *)calloc(op->nb, sizeof(fcproof));
    /* Step 1: one FC batch proof per block S_k = [kb, min((k+1)b, K)) (Eq. genFCBatchProof) */
    int fail = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t k = 0; k < op->nb; k++) {
        uint64_t lo = k * b, hi = lo + b < K ? lo + b : K;
        uint32_t t = (uint32_t)(hi - lo);
        uint64_t *idx = (uint64_t *)malloc(t * sizeof(uint64_t));
        for (uint32_t i = 0; i < t; i++) idx[i] = lo + i;
        if (fc_bopen(&op->bt[k], pp, &cm->C, cm->Cj, idx, t)) fail = 1;
        free(idx);
    }
    if (fail) return NULL;
    /* Step 2, Fiat-Shamir variant: Merkle tree over per-entry leaves
     * SHA-256(0x00 || m_i || C_j); nodes SHA-256(0x01 || left || right);
     * rho_j = H2F(DST_RHO, C || root || j). */
    op->mt = (uint8_t *)calloc(2 * N, 32);
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; i++) merkle_leaf(op->mt + 32 * (N + i), &cm->m[i], &cm->Cj[i / M]);
    for (uint64_t n = N - 1; n >= 1; n--) merkle_node(op->mt + 32 * n, op->mt + 64 * n, op->mt + 64 * n + 32);
    op->rho = (fe *)calloc(K, sizeof(fe));
    for (uint64_t j = 0; j < K; j++) rho_challenge(&op->rho[j], &cm->C, op->mt + 32, j);
    /* Step 2.1: g_j = rho_j f_j, D_j = C_j^{rho_j} (Eq. ProverRand), then the
     * bottom-up folding tree (Sub-protocol): g_w = g_wl + g_wr, D_w = D_wl D_wr. */
    op->y = (fe *)calloc((2 * K - 1) * M, sizeof(fe));
    op->D = (g1a *)calloc(2 * K - 1, sizeof(g1a));
    for (uint64_t j = 0; j < K; j++)
        for (uint64_t a = 0; a < M; a++) fr_mul(&op->y[j * M + a], &op->rho[j], &cm->m[j * M + a]);
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t j = 0; j < K; j++) g1_mul(&op->D[j], &cm->Cj[j], &op->rho[j]);
    for (uint32_t h = 1; h <= pp->lK; h++) {
        uint64_t nw = K >> h, o = lvl_off(K, h), oc = lvl_off(K, h - 1);
        for (uint64_t w = 0; w < nw; w++) {
            for (uint64_t a = 0; a < M; a++)
                fr_add(&op->y[(o + w) * M + a], &op->y[(oc + 2 * w) * M + a], &op->y[(oc + 2 * w + 1) * M + a]);
            g1_add(&op->D[o + w], &op->D[oc + 2 * w], &op->D[oc + 2 * w + 1]);
        }
    }
    /* Step 2.2: PC.HyperEval on g* (root row): every depth d < lM and prefix p */
    const fe *g = &op->y[lvl_off(K, pp->lK) * M];
    op->W = (g1a *)calloc(M - 1, sizeof(g1a));
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t n = 0; n < M - 1; n++) {
        uint32_t d = 63 - __builtin_clzll(n + 1);
        uint64_t p = n + 1 - (1ULL << d);
        uint32_t k = pp->lM - d;
        pst_quotient(&op->W[n], pp, g + p * (1ULL << k), k);
    }
    return op;
}

OR_API void or_open_free(void *o) {
    opening *op = (opening *)o;
    if (!op) return;
    for (uint64_t k = 0; k < op->nb; k++) fcproof_free(&op->bt[k]);
    free(op->bt);
    free(op->mt);
    free(op->rho);
    free(op->y);
    free(op->D);
    free(op->W);
    free(op);
}

/* per round: L.gt(384) L.g1(64) R.gt(384) R.g1(64) */
static void export_fc_rounds(uint8_t *out, const fcproof *pr, uint32_t l) {
    for (uint32_t j = 0; j < l; j++) {
        uint8_t *q = out + j * 896;
        fp12_to_bytes(q, &pr->Lgt[j]);
        g1_to_bytes(q + 384, &pr->Lg1[j]);
        fp12_to_bytes(q + 448, &pr->Rgt[j]);
        g1_to_bytes(q + 832, &pr->Rg1[j]);
    }
}

/* A_l(64) v_l(128) pi_v(128) */
static void export_fc_tail(uint8_t *out, const fcproof *pr) {
    g1_to_bytes(out, &pr->A);
    g2_to_bytes(out + 64, &pr->v);
    g2_to_bytes(out + 192, &pr->piv);
}

/*
 * Step 1 of OpenAll(b) for the listed blocks only (section 4.2, Protocol 1 Step 1: one
 * FC.BOpen per block S_k, Eq. genFCBatchProof), for parity checks of sizes whose whole
 * OpenAll is too slow here.  Block q of the list is written as or_open_export's formats
 * 0, 1 and 2 at rounds + 896*lK*q, tail + 320*q and xs + 32*lK*q.  Returns 0, or -1 for a
 * bad b or block index, -2 for a zero challenge.
 */
OR_API int or_open_blocks(void *c, uint32_t b, const uint64_t *ks, uint64_t n, uint8_t *rounds,
                          uint8_t *tail, uint8_t *xs) {
    commitment *cm = (commitment *)c;
    const params *pp = cm->pp;
    uint64_t K = pp->K;
    uint32_t l = pp->lK;
    if (b < 1 || b > K) return -1;
    uint64_t nb = (K + b - 1) / b;
    for (uint64_t q = 0; q < n; q++)
        if (ks[q] >= nb) return -1;
    int fail = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t q = 0; q < n; q++) {
        uint64_t lo = ks[q] * b, hi = lo + b < K ? lo + b : K;
        uint32_t t = (uint32_t)(hi - lo);
        uint64_t *idx = (uint64_t *)malloc(t * sizeof(uint64_t));
        for (uint32_t i = 0; i < t; i++) idx[i] = lo + i;
        fcproof pr;
        memset(&pr, 0, sizeof pr);
        if (fc_bopen(&pr, pp, &cm->C, cm->Cj, idx, t)) {
            fail = 1;
        } else {
            export_fc_rounds(rounds + 896ULL * l * q, &pr, l);
            export_fc_tail(tail + 320 * q, &pr);
            for (uint32_t j = 0; j < l; j++) enc_fr(xs + 32ULL * (l * q + j), &pr.x[j]);
        }
        fcproof_free(&pr);
        free(idx);
    }
    return fail ? -2 : 0;
}

/*
 * Bulk canonical arrays, for parity checks:
 *  0: per batch k (idx), per round: L.gt(384) L.g1(64) R.gt(384) R.g1(64)
 *  1: per batch: A_l(64) v_l(128) pi_v(128)
 *  2: per batch: x_1..x_l (32 each)
 *  3: Merkle tree, 2N x 32 (node 0 unused)
 *  4: rho, K x 32
 *  5: fold rows y, (2K-1)M x 32
 *  6: fold commitments D, (2K-1) x 64
 *  7: HyperEval W, (M-1) x 64
 */
OR_API int or_open_export(void *o, int what, uint64_t idx, uint8_t *out) {
    opening *op = (opening *)o;
    const params *pp = op->cm->pp;
    uint64_t K = pp->K, M = pp->M, N = pp->N;
    uint32_t l = pp->lK;
    if ((what <= 2) && idx >= op->nb) return -1;
    switch (what) {
    case 0:
        export_fc_rounds(out, &op->bt[idx], l);
        return 0;
    case 1:
        export_fc_tail(out, &op->bt[idx]);
        return 0;
    case 2:
        for (uint32_t j = 0; j < l; j++) enc_fr(out + 32 * j, &op->bt[idx].x[j]);
        return 0;
    case 3:
        memcpy(out, op->mt, 2 * N * 32);
        return 0;
    case 4:
        for (uint64_t j = 0; j < K; j++) enc_fr(out + 32 * j, &op->rho[j]);
        return 0;
    case 5:
        for (uint64_t i = 0; i < (2 * K - 1) * M; i++) enc_fr(out + 32 * i, &op->y[i]);
        return 0;
    case 6:
        for (uint64_t i = 0; i < 2 * K - 1; i++) g1_to_bytes(out + 64 * i, &op->D[i]);
        return 0;
    case 7:
        for (uint64_t i = 0; i < M - 1; i++) g1_to_bytes(out + 64 * i, &op->W[i]);
        return 0;
    }
    return -1;
}

/* ============================ proof wire format ============================ */
/*
 * pi_i for i = jM + a, block k = floor(j/b), t = |S_k| (section 4.3, "Proof size"):
 *   (C_{a'})_{a' in S_k}                      t x G1   (compressed, 32 B)
 *   {L_j, R_j}_{j=1..lK} as (gt, g1) pairs    2lK x (G_T 384 B + G1 32 B)
 *   A_l (G1), v_l (G2, 64 B), pi_v (G2)
 *   (D_{h, sib}, y_{h, sib, a})_{h<lK}        lK x (G1 + F_r)
 *   (W_{d, a >> (lM-d)})_{d<lM}               lM x G1
 *   Merkle path of leaf i, leaf level first   L x 32 B
 */
OR_API uint64_t or_proof_len(uint32_t log_n, uint32_t t) {
    uint32_t lK = log_n / 2, lM = log_n - lK;
    return 32ULL * t + lK * (2ULL * 384 + 2 * 32) + 32 + 64 + 64 + lK * 64ULL + lM * 32ULL + 32ULL * log_n;
}

static size_t assemble(uint8_t *out, const params *pp, uint64_t i, uint32_t b,
                       const g1a *Cj, const fcproof *pr, const g1a *Dsib, const fe *ysib,
                       const g1a *Wpath, const uint8_t *mpath) {
    uint64_t M = pp->M, K = pp->K;
    uint64_t j = i / M, k = j / b;
    uint64_t lo = k * b, hi = lo + b < K ? lo + b : K;
    uint8_t *q = out;
    for (uint64_t a2 = lo; a2 < hi; a2++) { g1_compress(q, &Cj[a2]); q += 32; }
    for (uint32_t r = 0; r < pp->lK; r++) {
        fp12_to_bytes(q, &pr->Lgt[r]); q += 384;
        g1_compress(q, &pr->Lg1[r]); q += 32;
        fp12_to_bytes(q, &pr->Rgt[r]); q += 384;
        g1_compress(q, &pr->Rg1[r]); q += 32;
    }
    g1_compress(q, &pr->A); q += 32;
    g2_compress(q, &pr->v); q += 64;
    g2_compress(q, &pr->piv); q += 64;
    for (uint32_t h = 0; h < pp->lK; h++) {
        g1_compress(q, &Dsib[h]); q += 32;
        enc_fr(q, &ysib[h]); q += 32;
    }
    for (uint32_t d = 0; d < pp->lM; d++) { g1_compress(q, &Wpath[d]); q += 32; }
    memcpy(q, mpath, 32ULL * pp->L);
    q += 32ULL * pp->L;
    return (size_t)(q - out);
}

OR_API int or_proof(void *o, uint64_t i, uint8_t *out, size_t cap, size_t *len) {
    opening *op = (opening *)o;
    const params *pp = op->cm->pp;
    uint64_t M = pp->M, K = pp->K, N = pp->N;
    if (i >= N) return -1;
    uint64_t j = i / M, a = i % M, k = j / op->b;
    uint32_t t = op->bt[k].t;
    size_t need = or_proof_len(pp->L, t);
    if (cap < need) return -1;
    g1a *Dsib = (g1a *)calloc(pp->lK, sizeof(g1a));
    fe *ysib = (fe *)calloc(pp->lK, sizeof(fe));
    g1a *Wp = (g1a *)calloc(pp->lM, sizeof(g1a));
    uint8_t *mp = (uint8_t *)malloc(32ULL * pp->L);
    for (uint32_t h = 0; h < pp->lK; h++) {
        uint64_t w = (j >> h) ^ 1, node = lvl_off(K, h) + w;
        Dsib[h] = op->D[node];
        ysib[h] = op->y[node * M + a];
    }
    for (uint32_t d = 0; d < pp->lM; d++) Wp[d] = op->W[(1ULL << d) - 1 + (a >> (pp->lM - d))];
    for (uint32_t h = 0; h < pp->L; h++) memcpy(mp + 32 * h, op->mt + 32 * (((N + i) >> h) ^ 1), 32);
    *len = assemble(out, pp, i, op->b, op->cm->Cj, &op->bt[k], Dsib, ysib, Wp, mp);
    free(Dsib); free(ysib); free(Wp); free(mp);
    return *len == need ? 0 : -1;
}

/* ============================ VC.Verify ============================ */
/* FC.BVerify (section 3, Eq. comy, with the faster verifier and the O(|I| log mu)
 * closed form b_l = sum_i r_i prod_k (1/x_k)^{bit_{l-k}(a_i)}, Eq. b_l) */
static int fc_bverify_b(const params *pp, const fp12 *C, const g1a *claim, const fe *bv, const uint64_t *bidx,
                        uint64_t nterm, const fp12 *Lgt, const g1a *Lg1, const fp12 *Rgt, const g1a *Rg1,
                        const g1a *Al, const g2a *vl, const g2a *piv);

static int fc_bverify(const params *pp, const fp12 *C, const uint64_t *idx, const g1a *yv, uint32_t t,
                      const fp12 *Lgt, const g1a *Lg1, const fp12 *Rgt, const g1a *Rg1,
                      const g1a *Al, const g2a *vl, const g2a *piv) {
    fe *r = (fe *)calloc(t, sizeof(fe));
    fc_batch_coeffs(r, C, idx, yv, t);
    g1a Cg1;
    g1_msm(&Cg1, yv, r, t);
    int ok = fc_bverify_b(pp, C, &Cg1, r, idx, t, Lgt, Lg1, Rgt, Rg1, Al, vl, piv);
    free(r);
    return ok;
}

/* the checks of FC.BVerify for b = sum_i bv[i] u_{bidx[i]} and the claimed <A, b> */
static int fc_bverify_b(const params *pp, const fp12 *C, const g1a *claim, const fe *bv, const uint64_t *bidx,
                        uint64_t nterm, const fp12 *Lgt, const g1a *Lg1, const fp12 *Rgt, const g1a *Rg1,
                        const g1a *Al, const g2a *vl, const g2a *piv) {
    uint32_t l = pp->lK;
    g1a Cg1 = *claim;
    fp12 Cgt = *C;
    fe *x = (fe *)calloc(l, sizeof(fe)), *xinv = (fe *)calloc(l, sizeof(fe));
    int ok = 1;
    for (uint32_t j = 1; j <= l && ok; j++) {
        if (fc_challenge(&x[j - 1], j > 1 ? &x[j - 2] : NULL, j == 1, &Lgt[j - 1], &Lg1[j - 1], &Rgt[j - 1], &Rg1[j - 1])) {
            ok = 0;
            break;
        }
        fr_inv(&xinv[j - 1], &x[j - 1]);
        fp12 a1, a2;
        fp12_pow_fr(&a1, &Lgt[j - 1], &x[j - 1]);
        fp12_pow_fr(&a2, &Rgt[j - 1], &xinv[j - 1]);
        fp12_mul(&Cgt, &Cgt, &a1);
        fp12_mul(&Cgt, &Cgt, &a2);
        g1a s1, s2;
        g1_mul(&s1, &Lg1[j - 1], &x[j - 1]);
        g1_mul(&s2, &Rg1[j - 1], &xinv[j - 1]);
        g1_add(&Cg1, &Cg1, &s1);
        g1_add(&Cg1, &Cg1, &s2);
    }
    if (ok) {
        /* b_l by the closed form */
        fe bl = {{0, 0, 0, 0}};
        for (uint64_t i = 0; i < nterm; i++) {
            fe term = bv[i];
            for (uint32_t k = 1; k <= l; k++)
                if ((bidx[i] >> (l - k)) & 1) fr_mul(&term, &term, &xinv[k - 1]);
            fr_add(&bl, &bl, &term);
        }
        /* v_l is checked by e(beta g1 - z g1, pi_v) = e(g1, v_l - f_v(z) g2) */
        fe z = fc_z_challenge(&x[l - 1], vl);
        fe *c = fv_coeffs(xinv, l, pp->K);
        fe fz = poly_eval(c, 2 * pp->K - 2, &z);
        free(c);
        g1a zg, lhs1;
        g1_mul(&zg, &G1_GEN, &z);
        g1_neg(&zg, &zg);
        g1_add(&lhs1, &pp->g1beta, &zg);
        g2a fzg, rhs2;
        g2_mul(&fzg, &G2_GEN, &fz);
        g2_neg(&fzg, &fzg);
        g2_add(&rhs2, vl, &fzg);
        g1a P2[2];
        g2a Q2[2];
        P2[0] = lhs1; Q2[0] = *piv;
        g1_neg(&P2[1], &G1_GEN); Q2[1] = rhs2;
        fp12 chk;
        multi_pairing(&chk, P2, Q2, 2);
        if (!fp12_is_one(&chk)) ok = 0;
        /* final check C_l = (A_l * v_l, <A_l, b_l>) */
        fp12 e1;
        pairing(&e1, Al, vl);
        g1a bA;
        g1_mul(&bA, Al, &bl);
        if (!fp12_eq(&e1, &Cgt) || !g1_eq(&bA, &Cg1)) ok = 0;
    }
    free(x); free(xinv);
    return ok;
}

/* PC.Verify for PST at the boolean point Bin(a):
 * e(D - y g1, g2) = prod_{d<lM} e(W_d, (s_{lM-1-d} - a_{lM-1-d}) g2) */
static int pst_verify(const params *pp, const g1a *D, uint64_t a, const fe *y, const g1a *Wp) {
    uint32_t lM = pp->lM;
    g1a *P = (g1a *)calloc(lM + 1, sizeof(g1a));
    g2a *Q = (g2a *)calloc(lM + 1, sizeof(g2a));
    g1a yg;
    g1_mul(&yg, &G1_GEN, y);
    g1_neg(&yg, &yg);
    g1_add(&P[0], D, &yg);
    g2_neg(&Q[0], &G2_GEN);
    for (uint32_t d = 0; d < lM; d++) {
        uint32_t var = lM - 1 - d;
        P[d + 1] = Wp[d];
        if ((a >> var) & 1) {
            g2a ng;
            g2_neg(&ng, &G2_GEN);
            g2_add(&Q[d + 1], &pp->vk[var], &ng);
        } else {
            Q[d + 1] = pp->vk[var];
        }
    }
    fp12 chk;
    multi_pairing(&chk, P, Q, lM + 1);
    free(P); free(Q);
    return fp12_is_one(&chk);
}

/* VC.Verify(C, i, m_i, pi_i) with batch size b: returns 1 accept, 0 reject, <0 malformed */
OR_API int or_verify(void *p, const uint8_t Cbytes[384], uint64_t n, uint32_t b, uint64_t i,
                     const uint8_t mi_le[32], const uint8_t *proof, size_t len) {
    const params *pp = (const params *)p;
    uint64_t K = pp->K, M = pp->M;
    if (n != pp->N || i >= n || b < 1 || b > K) return -1;
    uint64_t j = i / M, a = i % M, k = j / b;
    uint64_t lo = k * b, hi = lo + b < K ? lo + b : K;
    uint32_t t = (uint32_t)(hi - lo), l = pp->lK;
    if (len != or_proof_len(pp->L, t)) return -1;
    fp12 C;
    fe mi;
    if (fp12_from_bytes(&C, Cbytes) || mf_from_le(&MR, &mi, mi_le)) return -1;
    const uint8_t *q = proof;
    g1a *blk = (g1a *)calloc(t, sizeof(g1a));
    fp12 *Lgt = (fp12 *)calloc(l, sizeof(fp12)), *Rgt = (fp12 *)calloc(l, sizeof(fp12));
    g1a *Lg1 = (g1a *)calloc(l, sizeof(g1a)), *Rg1 = (g1a *)calloc(l, sizeof(g1a));
    g1a *Dsib = (g1a *)calloc(l, sizeof(g1a)), *Wp = (g1a *)calloc(pp->lM, sizeof(g1a));
    fe *ysib = (fe *)calloc(l, sizeof(fe));
    uint64_t *idx = (uint64_t *)calloc(t, sizeof(uint64_t));
    g1a Al;
    g2a vl, piv;
    int ok = 1;
    for (uint32_t u = 0; u < t && ok; u++) { idx[u] = lo + u; if (g1_decompress(&blk[u], q)) ok = 0;
        q += 32; }
    for (uint32_t r = 0; r < l && ok; r++) {
        if (fp12_from_bytes(&Lgt[r], q)) ok = 0;
        q += 384;
        if (g1_decompress(&Lg1[r], q)) ok = 0;
        q += 32;
        if (fp12_from_bytes(&Rgt[r], q)) ok = 0;
        q += 384;
        if (g1_decompress(&Rg1[r], q)) ok = 0;
        q += 32;
    }
    if (ok && g1_decompress(&Al, q)) ok = 0;
    q += 32;
    if (ok && g2_decompress(&vl, q)) ok = 0;
    q += 64;
    if (ok && g2_decompress(&piv, q)) ok = 0;
    q += 64;
    for (uint32_t h = 0; h < l && ok; h++) {
        if (g1_decompress(&Dsib[h], q)) ok = 0;
        q += 32;
        if (mf_from_be(&MR, &ysib[h], q)) ok = 0;
        q += 32;
    }
    for (uint32_t d = 0; d < pp->lM && ok; d++) { if (g1_decompress(&Wp[d], q)) ok = 0;
        q += 32; }
    const uint8_t *mpath = q;
    int result = ok ? 1 : 0;
    /* Part 1: C_j is the (j)-th element of the vector committed in C (Step 1) */
    if (result && !fc_bverify(pp, &C, idx, blk, t, Lgt, Lg1, Rgt, Rg1, &Al, &vl, &piv)) result = 0;
    if (result) {
        const g1a *Cj = &blk[j - lo];
        /* Part 2: Merkle membership of (m_i, C_j) and the common challenge rho_j */
        uint8_t node[32];
        merkle_leaf(node, &mi, Cj);
        uint64_t pos = pp->N + i;
        for (uint32_t h = 0; h < pp->L; h++, pos >>= 1) {
            if (pos & 1) merkle_node(node, mpath + 32 * h, node);
            else merkle_node(node, node, mpath + 32 * h);
        }
        fe rho;
        rho_challenge(&rho, &C, node, j);
        /* Part 3: fold up the tree (Sub-protocol; Eq. VerifierRand) */
        g1a Dstar;
        fe ystar;
        g1_mul(&Dstar, Cj, &rho);
        fr_mul(&ystar, &rho, &mi);
        for (uint32_t h = 0; h < l; h++) {
            g1_add(&Dstar, &Dstar, &Dsib[h]);
            fr_add(&ystar, &ystar, &ysib[h]);
        }
        /* Part 4: PC.Verify(D*, Bin(a), y*_a, pi*_a) */
        if (!pst_verify(pp, &Dstar, a, &ystar, Wp)) result = 0;
    }
    free(blk); free(Lgt); free(Rgt); free(Lg1); free(Rg1); free(Dsib); free(Wp); free(ysib); free(idx);
    return result;
}

/* ================= evaluation proof at a point (section 4.3) ================= */
/*
 * f_m(r) with r = (r_{L-1}, ..., r_0): entry i = jM + a pairs its bit k with x_k, so the bits of
 * j go with r_L = (r_{L-1}, ..., r_{lM}) and those of a with r_R = (r_{lM-1}, ..., r_0).
 *   T_j = prod_{c<lK} (j_c r_{lM+c} + (1 - j_c)(1 - r_{lM+c})),  C_F = sum_j T_j C_j,
 *   F = sum_j T_j f_j, whose table is g[a] = sum_j T_j m[jM + a], evaluated at r_R by PST.
 * Reading: the paper gives the three steps but no transcript.  The FC statement is the one
 * query vector T with claimed value C_F, batched (Eq. b) with
 *   sigma_E = SHA-256(DST_EVAL || enc(C) || enc(r_{L-1}) || ... || enc(r_0) || enc(C_F)),
 *   r_0 = H2F(DST_EVAL, sigma_E || 0),  b = r_0 T,  claimed <C, b> = r_0 C_F;
 * rounds, x_j, z and pi_v as in FC.BOpen.  Proof bytes: C_F (32) || lK rounds (L_gt 384,
 * L_g1 32, R_gt 384, R_g1 32) || A_l 32 || v_l 64 || pi_v 64 || y = F(r_R) (32, big-endian)
 * || W_0 .. W_{lM-1} (32 each).
 */
static fe pst_eval_generic(g1a *Wout, const params *pp, const fe *table, const fe *z);

static void eq_top(fe *T, const params *pp, const fe *r) {
    fe one;
    mf_one(&MR, &one);
    for (uint64_t j = 0; j < pp->K; j++) {
        fe acc = one;
        for (uint32_t c = 0; c < pp->lK; c++) {
            fe f;
            if ((j >> c) & 1) f = r[pp->lM + c];
            else fr_sub(&f, &one, &r[pp->lM + c]);
            fr_mul(&acc, &acc, &f);
        }
        T[j] = acc;
    }
}

static void eval_r0(fe *r0, const fp12 *C, const fe *r, uint32_t L, const g1a *CF) {
    bytes b = {0};
    bytes_put(&b, DST_EVAL, strlen(DST_EVAL));
    put_gt(&b, C);
    for (int k = (int)L - 1; k >= 0; k--) put_fr(&b, &r[k]);
    put_g1(&b, CF);
    uint8_t sigma[32];
    sha256(sigma, b.p, b.n);
    bytes_free(&b);
    bytes m = {0};
    bytes_put(&m, sigma, 32);
    bytes_put_u64(&m, 0);
    hash_to_fr(r0, DST_EVAL, m.p, m.n);
    bytes_free(&m);
}

OR_API uint64_t or_eval_proof_len(uint32_t log_n) {
    uint32_t lK = log_n / 2, lM = log_n - lK;
    return 32 + 832ULL * lK + 160 + 32 + 32ULL * lM;
}

static int parse_point(fe *r, const uint8_t *r_le, uint32_t L) {
    for (uint32_t k = 0; k < L; k++)
        if (mf_from_le(&MR, &r[k], r_le + 32 * k)) return -1;
    return 0;
}

OR_API int or_eval_proof(void *c, const uint8_t *r_le, uint8_t *out, size_t cap, size_t *len) {
    commitment *cm = (commitment *)c;
    const params *pp = cm->pp;
    uint64_t K = pp->K, M = pp->M;
    uint32_t L = pp->L, lK = pp->lK, lM = pp->lM;
    if (cap < or_eval_proof_len(L)) return -1;
    fe *r = (fe *)calloc(L, sizeof(fe));
    if (parse_point(r, r_le, L)) { free(r); return -1; }
    fe *T = (fe *)calloc(K, sizeof(fe)), *b = (fe *)calloc(K, sizeof(fe)), *g = (fe *)calloc(M, sizeof(fe));
    eq_top(T, pp, r);
    g1a CF, claim;
    g1_msm(&CF, cm->Cj, T, K);
    fe r0;
    eval_r0(&r0, &cm->C, r, L, &CF);
    for (uint64_t j = 0; j < K; j++) fr_mul(&b[j], &r0, &T[j]);
    g1_mul(&claim, &CF, &r0);
    fcproof pr;
    memset(&pr, 0, sizeof pr);
    int rc = fc_bopen_b(&pr, pp, &cm->C, cm->Cj, b, &claim);
    if (rc == 0) {
        for (uint64_t a = 0; a < M; a++) {
            fe acc = {{0, 0, 0, 0}};
            for (uint64_t j = 0; j < K; j++) {
                fe t;
                fr_mul(&t, &T[j], &cm->m[j * M + a]);
                fr_add(&acc, &acc, &t);
            }
            g[a] = acc;
        }
        g1a *W = (g1a *)calloc(lM, sizeof(g1a));
        fe y = pst_eval_generic(W, pp, g, r);  /* z_k = r_k for the low lM variables */
        uint8_t *q = out;
        g1_compress(q, &CF); q += 32;
        for (uint32_t j = 0; j < lK; j++) {
            fp12_to_bytes(q, &pr.Lgt[j]); q += 384;
            g1_compress(q, &pr.Lg1[j]); q += 32;
            fp12_to_bytes(q, &pr.Rgt[j]); q += 384;
            g1_compress(q, &pr.Rg1[j]); q += 32;
        }
        g1_compress(q, &pr.A); q += 32;
        g2_compress(q, &pr.v); q += 64;
        g2_compress(q, &pr.piv); q += 64;
        enc_fr(q, &y); q += 32;
        for (uint32_t d = 0; d < lM; d++) { g1_compress(q, &W[d]); q += 32; }
        *len = (size_t)(q - out);
        free(W);
    }
    fcproof_free(&pr);
    free(r); free(T); free(b); free(g);
    return rc ? -1 : 0;
}

/* 1 accept, 0 reject, -1 malformed C or point */
OR_API int or_eval_verify(void *p, const uint8_t Cbytes[384], const uint8_t *r_le, const uint8_t *proof, size_t len) {
    const params *pp = (const params *)p;
    uint64_t K = pp->K;
    uint32_t L = pp->L, l = pp->lK, lM = pp->lM;
    if (len != or_eval_proof_len(L)) return -1;
    fp12 C;
    if (fp12_from_bytes(&C, Cbytes)) return -1;
    fe *r = (fe *)calloc(L, sizeof(fe));
    if (parse_point(r, r_le, L)) { free(r); return -1; }
    fp12 *Lgt = (fp12 *)calloc(l, sizeof(fp12)), *Rgt = (fp12 *)calloc(l, sizeof(fp12));
    g1a *Lg1 = (g1a *)calloc(l, sizeof(g1a)), *Rg1 = (g1a *)calloc(l, sizeof(g1a)), *W = (g1a *)calloc(lM, sizeof(g1a));
    g1a CF, Al;
    g2a vl, piv;
    fe y;
    const uint8_t *q = proof;
    int ok = g1_decompress(&CF, q) == 0;
    q += 32;
    for (uint32_t j = 0; j < l && ok; j++) {
        if (fp12_from_bytes(&Lgt[j], q)) ok = 0;
        q += 384;
        if (g1_decompress(&Lg1[j], q)) ok = 0;
        q += 32;
        if (fp12_from_bytes(&Rgt[j], q)) ok = 0;
        q += 384;
        if (g1_decompress(&Rg1[j], q)) ok = 0;
        q += 32;
    }
    if (ok && g1_decompress(&Al, q)) ok = 0;
    q += 32;
    if (ok && g2_decompress(&vl, q)) ok = 0;
    q += 64;
    if (ok && g2_decompress(&piv, q)) ok = 0;
    q += 64;
    if (ok && mf_from_be(&MR, &y, q)) ok = 0;
    q += 32;
    for (uint32_t d = 0; d < lM && ok; d++) { if (g1_decompress(&W[d], q)) ok = 0;
        q += 32; }
    if (ok) {
        /* Part 1: C_F = <C, T(r_L)> by FC.BVerify on the dense query r_0 T */
        fe *T = (fe *)calloc(K, sizeof(fe)), *b = (fe *)calloc(K, sizeof(fe));
        uint64_t *bidx = (uint64_t *)calloc(K, sizeof(uint64_t));
        eq_top(T, pp, r);
        fe r0;
        eval_r0(&r0, &C, r, L, &CF);
        for (uint64_t j = 0; j < K; j++) { fr_mul(&b[j], &r0, &T[j]); bidx[j] = j; }
        g1a claim;
        g1_mul(&claim, &CF, &r0);
        if (!fc_bverify_b(pp, &C, &claim, b, bidx, K, Lgt, Lg1, Rgt, Rg1, &Al, &vl, &piv)) ok = 0;
        free(T); free(b); free(bidx);
    }
    if (ok) {
        /* Part 2: PC.Verify at r_R: e(C_F - y g1, g2) = prod_d e(W_d, (s_var - r_var) g2) */
        g1a *P = (g1a *)calloc(lM + 1, sizeof(g1a));
        g2a *Q = (g2a *)calloc(lM + 1, sizeof(g2a));
        g1a yg;
        g1_mul(&yg, &G1_GEN, &y);
        g1_neg(&yg, &yg);
        g1_add(&P[0], &CF, &yg);
        g2_neg(&Q[0], &G2_GEN);
        for (uint32_t d = 0; d < lM; d++) {
            uint32_t var = lM - 1 - d;
            g2a rg;
            g2_mul(&rg, &G2_GEN, &r[var]);
            g2_neg(&rg, &rg);
            P[d + 1] = W[d];
            g2_add(&Q[d + 1], &pp->vk[var], &rg);
        }
        fp12 chk;
        multi_pairing(&chk, P, Q, lM + 1);
        if (!fp12_is_one(&chk)) ok = 0;
        free(P); free(Q);
    }
    free(r); free(Lgt); free(Rgt); free(Lg1); free(Rg1); free(W);
    return ok;
}

/* PST commitment of a table of M values (Montgomery limbs little-endian 32-byte canonical
 * input) with ek_{lM}: an independent route to C_F for the tests */
OR_API int or_pst_commit(void *p, const uint8_t *tab_le, uint8_t out[64]) {
    const params *pp = (const params *)p;
    uint64_t M = pp->M;
    fe *t = (fe *)calloc(M, sizeof(fe));
    for (uint64_t a = 0; a < M; a++)
        if (mf_from_le(&MR, &t[a], tab_le + 32 * a)) { free(t); return -1; }
    g1a o;
    g1_msm(&o, pp->ek[pp->lM], t, M);
    g1_to_bytes(out, &o);
    free(t);
    return 0;
}

/* ============================ naive openers ============================ */
/* PC.Eval at an arbitrary point z = (z_{lM-1}, ..., z_0), eliminating the most
 * significant variable first: with T the current table, q_d = T_hi - T_lo and the
 * next table is T_lo + z_{var} (T_hi - T_lo).  Returns the evaluation. */
static fe pst_eval_generic(g1a *Wout, const params *pp, const fe *table, const fe *z) {
    uint32_t lM = pp->lM;
    uint64_t n = pp->M;
    fe *T = (fe *)malloc(n * sizeof(fe));
    memcpy(T, table, n * sizeof(fe));
    for (uint32_t d = 0; d < lM; d++) {
        uint32_t k = lM - d;
        pst_quotient(&Wout[d], pp, T, k);
        uint64_t half = 1ULL << (k - 1);
        for (uint64_t c = 0; c < half; c++) {
            fe diff, t;
            fr_sub(&diff, &T[half + c], &T[c]);
            fr_mul(&t, &diff, &z[lM - 1 - d]);
            fr_add(&T[c], &T[c], &t);
        }
    }
    fe y = T[0];
    free(T);
    return y;
}

/* pi_i built from scratch with nothing shared with OpenAll: fresh commitments,
 * the FC batch proof of its own block, a freshly built Merkle tree, sibling
 * subtree sums taken directly over the leaves they cover, and a generic PST
 * evaluation proof of g* = sum_j rho_j f_j at Bin(a). */
OR_API int or_naive_proof(void *p, const uint8_t *m_le, uint64_t n, uint32_t b, uint64_t i,
                          uint8_t *out, size_t cap, size_t *len) {
    params *pp = (params *)p;
    uint64_t K = pp->K, M = pp->M, N = pp->N;
    if (n != N || i >= N || b < 1 || b > K) return -1;
    commitment *cm = (commitment *)or_commit(pp, m_le, n);
    if (!cm) return -1;
    uint64_t j = i / M, a = i % M, k = j / b;
    uint64_t lo = k * b, hi = lo + b < K ? lo + b : K;
    uint32_t t = (uint32_t)(hi - lo);
    if (cap < or_proof_len(pp->L, t)) { or_commit_free(cm); return -1; }
    uint64_t *idx = (uint64_t *)malloc(t * sizeof(uint64_t));
    for (uint32_t u = 0; u < t; u++) idx[u] = lo + u;
    fcproof pr;
    memset(&pr, 0, sizeof pr);
    int rc = fc_bopen(&pr, pp, &cm->C, cm->Cj, idx, t);
    free(idx);
    if (rc) { or_commit_free(cm); return -1; }
    /* Merkle tree from scratch, path read off level by level */
    uint8_t *level = (uint8_t *)malloc(32 * N);
    for (uint64_t q = 0; q < N; q++) merkle_leaf(level + 32 * q, &cm->m[q], &cm->Cj[q / M]);
    uint8_t *mpath = (uint8_t *)malloc(32ULL * pp->L);
    uint64_t pos = i, width = N;
    for (uint32_t h = 0; h < pp->L; h++) {
        memcpy(mpath + 32 * h, level + 32 * (pos ^ 1), 32);
        for (uint64_t q = 0; q < width / 2; q++) merkle_node(level + 32 * q, level + 64 * q, level + 64 * q + 32);
        width /= 2;
        pos >>= 1;
    }
    fe *rho = (fe *)calloc(K, sizeof(fe));
    for (uint64_t jj = 0; jj < K; jj++) rho_challenge(&rho[jj], &cm->C, level, jj);
    free(level);
    /* sibling subtree at height h covers leaves [w 2^h, (w+1) 2^h), w = (j >> h) ^ 1 */
    g1a *Dsib = (g1a *)calloc(pp->lK, sizeof(g1a));
    fe *ysib = (fe *)calloc(pp->lK, sizeof(fe));
    for (uint32_t h = 0; h < pp->lK; h++) {
        uint64_t w = (j >> h) ^ 1, s = w << h, e = (w + 1) << h;
        g1_msm(&Dsib[h], &cm->Cj[s], &rho[s], e - s);
        fe acc = {{0, 0, 0, 0}}, tt;
        for (uint64_t q = s; q < e; q++) { fr_mul(&tt, &rho[q], &cm->m[q * M + a]); fr_add(&acc, &acc, &tt); }
        ysib[h] = acc;
    }
    fe *g = (fe *)calloc(M, sizeof(fe));
    for (uint64_t jj = 0; jj < K; jj++)
        for (uint64_t c = 0; c < M; c++) {
            fe tt;
            fr_mul(&tt, &rho[jj], &cm->m[jj * M + c]);
            fr_add(&g[c], &g[c], &tt);
        }
    fe *z = (fe *)calloc(pp->lM, sizeof(fe));
    for (uint32_t v = 0; v < pp->lM; v++) if ((a >> v) & 1) mf_one(&MR, &z[v]);
    g1a *Wp = (g1a *)calloc(pp->lM, sizeof(g1a));
    (void)pst_eval_generic(Wp, pp, g, z);
    *len = assemble(out, pp, i, b, cm->Cj, &pr, Dsib, ysib, Wp, mpath);
    fcproof_free(&pr);
    free(mpath); free(rho); free(Dsib); free(ysib); free(g); free(z); free(Wp);
    or_commit_free(cm);
    return 0;
}

/* The two-step method (section 4.1): an FC proof that C_j = <C, u_j> (b = 1 batch)
 * plus a PST proof of f_j(Bin(a)) = m[i] against C_j.  Outputs the PST part only
 * (lM x 64 B uncompressed W and the 32 B value), for the linearity pin
 * W(OpenAll, a) = sum_j rho_j W(two-step, j, a). */
OR_API int or_two_step_pst(void *c, uint64_t i, uint8_t *Wout, uint8_t yout[32]) {
    commitment *cm = (commitment *)c;
    const params *pp = cm->pp;
    uint64_t M = pp->M, j = i / M, a = i % M;
    fe *z = (fe *)calloc(pp->lM, sizeof(fe));
    for (uint32_t v = 0; v < pp->lM; v++) if ((a >> v) & 1) mf_one(&MR, &z[v]);
    g1a *Wp = (g1a *)calloc(pp->lM, sizeof(g1a));
    fe y = pst_eval_generic(Wp, pp, &cm->m[j * M], z);
    for (uint32_t d = 0; d < pp->lM; d++) g1_to_bytes(Wout + 64 * d, &Wp[d]);
    enc_fr(yout, &y);
    int ok = pst_verify(pp, &cm->Cj[j], a, &y, Wp);
    free(z); free(Wp);
    return ok;
}

/* FC proof of a single index j (two-step method, first step) and its verification */
OR_API int or_two_step_fc(void *c, uint64_t j) {
    commitment *cm = (commitment *)c;
    const params *pp = cm->pp;
    if (j >= pp->K) return -1;
    fcproof pr;
    memset(&pr, 0, sizeof pr);
    uint64_t idx = j;
    if (fc_bopen(&pr, pp, &cm->C, cm->Cj, &idx, 1)) return -1;
    int ok = fc_bverify(pp, &cm->C, &idx, &cm->Cj[j], 1, pr.Lgt, pr.Lg1, pr.Rgt, pr.Rg1, &pr.A, &pr.v, &pr.piv);
    fcproof_free(&pr);
    return ok;
}

/* FC.BOpen then FC.BVerify on an explicit statement; the claimed values y_i may be
 * replaced by the caller (bad_slot >= 0 substitutes g1 there) to exercise the
 * batching lemma (Lemma 1): a wrong claim must be rejected. */
OR_API int or_fc_roundtrip(void *c, const uint64_t *idx, uint32_t t, int bad_slot) {
    commitment *cm = (commitment *)c;
    const params *pp = cm->pp;
    fcproof pr;
    memset(&pr, 0, sizeof pr);
    if (fc_bopen(&pr, pp, &cm->C, cm->Cj, idx, t)) return -1;
    g1a *yv = (g1a *)calloc(t, sizeof(g1a));
    for (uint32_t i = 0; i < t; i++) yv[i] = cm->Cj[idx[i]];
    if (bad_slot >= 0 && (uint32_t)bad_slot < t) yv[bad_slot] = G1_GEN;
    int ok = fc_bverify(pp, &cm->C, idx, yv, t, pr.Lgt, pr.Lg1, pr.Rgt, pr.Rg1, &pr.A, &pr.v, &pr.piv);
    free(yv);
    fcproof_free(&pr);
    return ok;
}

OR_API void or_set_invariant_check(int on) { g_check_invariant = on; g_invariant_checks = 0; g_invariant_failures = 0; }
OR_API long or_invariant_checks(void) { return g_invariant_checks; }
OR_API long or_invariant_failures(void) { return g_invariant_failures; }
