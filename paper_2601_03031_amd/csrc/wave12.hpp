// Wave-cooperative F_p12 arithmetic for latency-bound chains (device only).
//
// One workgroup of WAVE12_T = 64 lanes owns F_p12 values held in LDS as 12 base
// coefficients in memory order (c0.c0.c0, c0.c0.c1, ..., c1.c2.c1; F_p2 coefficient
// j = 3h + q multiplies w^{2q+h}).  Each operation spreads its independent base-field
// products across lanes and recombines them in short LDS phases:
//  * wmul: Karatsuba at all three levels gives 3 x 6 x 3 = 54 independent products;
//    lane t = 18P + 3Q + R forms its operands as sums of input coefficients
//    (P: a0 b0 | a1 b1 | (a0+a1)(b0+b1); Q: F_p6 pairs 00 11 22 (12) (01) (02);
//    R: F_p2 pairs re re | im im | (re+im)(re+im)), then three phases undo the
//    Karatsuba levels;
//  * wcsqr: Granger-Scott squaring in the cyclotomic subgroup, 9 F_p2 squares =
//    18 products;
//  * Frobenius maps, conjugation and the inverse used by the final exponentiation.
// Every routine must be called by all lanes of the workgroup and ends in a barrier.
#pragma once
#include "tower.hpp"

#define WAVE12_T 64

struct W12 {
  fe pr[56];
  fp2 m[18];
  fp2 s6[9];
};

__device__ __forceinline__ void wsync() { __syncthreads(); }

__device__ __forceinline__ fp2 ld2(const fe *X, int j) { return {X[2 * j], X[2 * j + 1]}; }
__device__ __forceinline__ void st2(fe *X, int j, const fp2 &v) { X[2 * j] = v.c0; X[2 * j + 1] = v.c1; }

// D = X * Y (D may alias X or Y)
__device__ __noinline__ void wmul(const fe *X, const fe *Y, fe *D, W12 &w) {
  int t = threadIdx.x;
  if (t < 54) {
    int P = t / 18, Q = (t / 3) % 6, R = t % 3;
    // F_p6-level coefficient sets: Q = 0,1,2 single; 3 = {1,2}; 4 = {0,1}; 5 = {0,2}
    int q0 = Q < 3 ? Q : (Q == 3 ? 1 : 0);
    int q1 = Q < 3 ? -1 : (Q == 3 ? 2 : (Q == 4 ? 1 : 2));
    fe a = fe_zero(), b = fe_zero();
    for (int hh = 0; hh < 2; hh++) {
      bool hin = (P == 2) || (P == hh);
      for (int qi = 0; qi < 2; qi++) {
        int qq = qi ? q1 : q0;
        bool qin = qq >= 0;
        int qs = qin ? qq : 0;
        for (int rr = 0; rr < 2; rr++) {
          bool in = hin && qin && ((R == 2) || (R == rr));
          int k = 6 * hh + 2 * qs + rr;
          fe xa = in ? X[k] : fe_zero(), xb = in ? Y[k] : fe_zero();
          a = fp_add(a, xa);
          b = fp_add(b, xb);
        }
      }
    }
    w.pr[t] = fp_mul(a, b);
  }
  wsync();
  if (t < 18) {
    const fe *p = &w.pr[3 * t];
    fe re = fp_sub(p[0], p[1]);
    fe im = fp_sub(fp_sub(p[2], p[0]), p[1]);
    w.m[t] = {re, im};
  }
  wsync();
  if (t < 9) {
    int P = t / 3, c = t % 3;
    const fp2 *M = &w.m[6 * P];
    fp2 r;
    if (c == 0) r = f2_add(M[0], f2_mul_xi(f2_sub(f2_sub(M[3], M[1]), M[2])));
    else if (c == 1) r = f2_add(f2_sub(f2_sub(M[4], M[0]), M[1]), f2_mul_xi(M[2]));
    else r = f2_add(f2_sub(f2_sub(M[5], M[0]), M[2]), M[1]);
    w.s6[t] = r;
  }
  wsync();
  if (t < 6) {
    int h = t / 3, q = t % 3;
    const fp2 *V = w.s6;  // V[3P + c]
    fp2 r;
    if (h == 1) r = f2_sub(f2_sub(V[6 + q], V[q]), V[3 + q]);
    else if (q == 0) r = f2_add(V[0], f2_mul_xi(V[5]));
    else r = f2_add(V[q], V[3 + q - 1]);
    st2(D, 3 * h + q, r);
  }
  wsync();
}

// D = X^2 for X in the cyclotomic subgroup (D may alias X)
__device__ __noinline__ void wcsqr(const fe *X, fe *D, W12 &w) {
  int t = threadIdx.x;
  if (t < 18) {
    int s = t >> 1, e = t & 1;
    // F_p2 coefficients squared: a0, b1, a0+b1 | b0, a2, b0+a2 | a1, b2, a1+b2  (j = 3h + q)
    const int J1[9] = {0, 4, 0, 3, 2, 3, 1, 5, 1};
    const int J2[9] = {-1, -1, 4, -1, -1, 2, -1, -1, 5};
    int j1 = J1[s], j2 = J2[s];
    fp2 x = ld2(X, j1);
    fp2 y = j2 >= 0 ? ld2(X, j2) : f2_zero();
    x = f2_add(x, y);
    w.pr[t] = e ? fp_mul(x.c0, x.c1) : fp_mul(fp_add(x.c0, x.c1), fp_sub(x.c0, x.c1));
  }
  wsync();
  if (t < 9) w.m[t] = {w.pr[2 * t], fp_dbl(w.pr[2 * t + 1])};
  wsync();
  if (t < 6) {
    const fp2 *Q = w.m;
    fp2 r, xj;
    switch (t) {
      case 0: r = f2_add(Q[0], f2_mul_xi(Q[1])); xj = f2_neg(ld2(X, 0)); st2(D, 0, f2_add(r, f2_dbl(f2_add(r, xj)))); break;
      case 1: r = f2_sub(f2_sub(Q[2], Q[0]), Q[1]); xj = ld2(X, 4); st2(D, 4, f2_add(r, f2_dbl(f2_add(r, xj)))); break;
      case 2: r = f2_mul_xi(f2_sub(f2_sub(Q[8], Q[6]), Q[7])); xj = ld2(X, 3); st2(D, 3, f2_add(r, f2_dbl(f2_add(r, xj)))); break;
      case 3: r = f2_add(Q[6], f2_mul_xi(Q[7])); xj = f2_neg(ld2(X, 2)); st2(D, 2, f2_add(r, f2_dbl(f2_add(r, xj)))); break;
      case 4: r = f2_add(Q[3], f2_mul_xi(Q[4])); xj = f2_neg(ld2(X, 1)); st2(D, 1, f2_add(r, f2_dbl(f2_add(r, xj)))); break;
      default: r = f2_sub(f2_sub(Q[5], Q[3]), Q[4]); xj = ld2(X, 5); st2(D, 5, f2_add(r, f2_dbl(f2_add(r, xj)))); break;
    }
  }
  wsync();
}

// D = conj(X) = X^{p^6}
__device__ __noinline__ void wconj(const fe *X, fe *D) {
  int t = threadIdx.x;
  if (t < 12) D[t] = t < 6 ? X[t] : fp_neg(X[t]);
  wsync();
}

__device__ __noinline__ void wcopy(const fe *X, fe *D) {
  int t = threadIdx.x;
  if (t < 12) D[t] = X[t];
  wsync();
}

// D = X^{p^e}, e = 1, 2, 3: coefficient j (power w^k, k = 2q + h) maps to conj^e(c) gamma_e,k
__device__ __noinline__ void wfrob(const fe *X, fe *D, int e) {
  int t = threadIdx.x;
  fe out = fe_zero();
  if (t < 12) {
    int j = t >> 1, comp = t & 1;
    int h = j / 3, q = j % 3, k = 2 * q + h;
    fp2 c = ld2(X, j);
    if (e & 1) c = f2_conj(c);
    if (k == 0) {
      out = comp ? c.c1 : c.c0;
    } else if (e == 2) {
      const uint32_t *g2[6] = {bn::P_ONE, bn::FROB2_1, bn::FROB2_2, bn::FROB2_3, bn::FROB2_4, bn::FROB2_5};
      out = fp_mul(comp ? c.c1 : c.c0, fe_const(g2[k]));
    } else {
      const uint32_t *g0[6] = {bn::P_ONE, bn::FROB1_1_0, bn::FROB1_2_0, bn::FROB1_3_0, bn::FROB1_4_0, bn::FROB1_5_0};
      const uint32_t *g1[6] = {bn::P_ONE, bn::FROB1_1_1, bn::FROB1_2_1, bn::FROB1_3_1, bn::FROB1_4_1, bn::FROB1_5_1};
      const uint32_t *h0[6] = {bn::P_ONE, bn::FROB3_1_0, bn::FROB3_2_0, bn::FROB3_3_0, bn::FROB3_4_0, bn::FROB3_5_0};
      const uint32_t *h1[6] = {bn::P_ONE, bn::FROB3_1_1, bn::FROB3_2_1, bn::FROB3_3_1, bn::FROB3_4_1, bn::FROB3_5_1};
      fe gr = fe_const(e == 1 ? g0[k] : h0[k]), gi = fe_const(e == 1 ? g1[k] : h1[k]);
      // (c0 + c1 i)(gr + gi i)
      out = comp ? fp_add(fp_mul(c.c0, gi), fp_mul(c.c1, gr)) : fp_sub(fp_mul(c.c0, gr), fp_mul(c.c1, gi));
    }
  }
  wsync();
  if (t < 12) D[t] = out;
  wsync();
}

// D = X^{-1}: with n = X conj(X) in F_p6 (c1 = 0), X^{-1} = conj(X) n^{-1}; the F_p6
// inverse is taken by one lane
__device__ __noinline__ void winv(const fe *X, fe *D, fe *T0, fe *T1, W12 &w) {
  wconj(X, T0);
  wmul(X, T0, T1, w);  // T1 = n (c1 = 0)
  if (threadIdx.x == 0) {
    fp6 n = {ld2(T1, 0), ld2(T1, 1), ld2(T1, 2)};
    fp6 ni = f6_inv(n);
    st2(T1, 0, ni.c0);
    st2(T1, 1, ni.c1);
    st2(T1, 2, ni.c2);
    for (int k = 6; k < 12; k++) T1[k] = fe_zero();
  }
  wsync();
  wmul(T0, T1, D, w);
}

// D = X^u (u the BN parameter), X cyclotomic; D must not alias X
__device__ __noinline__ void wpow_u(const fe *X, fe *D, W12 &w) {
  wcopy(X, D);
  for (int i = 61; i >= 0; i--) {
    wcsqr(D, D, w);
    if ((bn::BN_U >> i) & 1) wmul(D, X, D, w);
  }
}
