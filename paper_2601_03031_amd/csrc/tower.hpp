// Extension tower for the BN254 pairing:
//   F_p2 = F_p[i]/(i^2 + 1),  F_p6 = F_p2[v]/(v^3 - xi), xi = 9 + i,
//   F_p12 = F_p6[w]/(w^2 - v).
// Products use Karatsuba at every level (3 / 6 / 18 base products), squaring in
// F_p12 uses the complex method, and squaring in the cyclotomic subgroup uses the
// Granger-Scott formula written for this tower (coefficients regrouped over
// F_p4 = F_p2[t], t = w^3).  Frobenius maps use the constants gamma_k = xi^{k(p^j-1)/6}
// generated in constants.hpp.
#pragma once
#include "field.hpp"

struct fp2 {
  fe c0, c1;
};
struct fp6 {
  fp2 c0, c1, c2;
};
struct fp12 {
  fp6 c0, c1;
};

// ------------------------------------------------------------------ F_p2
DEV fp2 f2_zero() { return {fe_zero(), fe_zero()}; }
DEV fp2 f2_one() { return {f_one<FpP>(), fe_zero()}; }
DEV fp2 f2_const(const uint32_t *a, const uint32_t *b) { return {fe_const(a), fe_const(b)}; }
DEV bool f2_is_zero(const fp2 &a) { return fe_is_zero(a.c0) && fe_is_zero(a.c1); }
DEV bool f2_eq(const fp2 &a, const fp2 &b) { return fe_eq(a.c0, b.c0) && fe_eq(a.c1, b.c1); }
DEV fp2 f2_add(const fp2 &a, const fp2 &b) { return {fp_add(a.c0, b.c0), fp_add(a.c1, b.c1)}; }
DEV fp2 f2_sub(const fp2 &a, const fp2 &b) { return {fp_sub(a.c0, b.c0), fp_sub(a.c1, b.c1)}; }
DEV fp2 f2_neg(const fp2 &a) { return {fp_neg(a.c0), fp_neg(a.c1)}; }
DEV fp2 f2_dbl(const fp2 &a) { return {fp_dbl(a.c0), fp_dbl(a.c1)}; }
DEV fp2 f2_half(const fp2 &a) { return {fp_half(a.c0), fp_half(a.c1)}; }
DEV fp2 f2_conj(const fp2 &a) { return {a.c0, fp_neg(a.c1)}; }
DEV fp2 f2_mul_fp(const fp2 &a, const fe &b) { return {fp_mul(a.c0, b), fp_mul(a.c1, b)}; }

DEV fp2 f2_mul(const fp2 &a, const fp2 &b) {
  fe v0 = fp_mul(a.c0, b.c0);
  fe v1 = fp_mul(a.c1, b.c1);
  fe s = fp_mul(fp_add(a.c0, a.c1), fp_add(b.c0, b.c1));
  return {fp_sub(v0, v1), fp_sub(fp_sub(s, v0), v1)};
}

DEV fp2 f2_sqr(const fp2 &a) {
  // (a0 + a1 i)^2 = (a0 + a1)(a0 - a1) + 2 a0 a1 i
  fe t = fp_mul(a.c0, a.c1);
  return {fp_mul(fp_add(a.c0, a.c1), fp_sub(a.c0, a.c1)), fp_dbl(t)};
}

// multiply by xi = 9 + i: (9 a0 - a1) + (a0 + 9 a1) i
DEV fp2 f2_mul_xi(const fp2 &a) {
  fe a0_8 = fp_dbl(fp_dbl(fp_dbl(a.c0)));
  fe a1_8 = fp_dbl(fp_dbl(fp_dbl(a.c1)));
  return {fp_sub(fp_add(a0_8, a.c0), a.c1), fp_add(fp_add(a1_8, a.c1), a.c0)};
}

inline NOINL fp2 f2_inv(const fp2 &a) {
  fe n = fp_add(fp_sqr(a.c0), fp_sqr(a.c1));
  fe ni = fp_inv_fast(n);
  return {fp_mul(a.c0, ni), fp_neg(fp_mul(a.c1, ni))};
}

// ------------------------------------------------------------------ F_p6
DEV fp6 f6_zero() { return {f2_zero(), f2_zero(), f2_zero()}; }
DEV fp6 f6_one() { return {f2_one(), f2_zero(), f2_zero()}; }
DEV fp6 f6_add(const fp6 &a, const fp6 &b) { return {f2_add(a.c0, b.c0), f2_add(a.c1, b.c1), f2_add(a.c2, b.c2)}; }
DEV fp6 f6_sub(const fp6 &a, const fp6 &b) { return {f2_sub(a.c0, b.c0), f2_sub(a.c1, b.c1), f2_sub(a.c2, b.c2)}; }
DEV fp6 f6_neg(const fp6 &a) { return {f2_neg(a.c0), f2_neg(a.c1), f2_neg(a.c2)}; }
DEV fp6 f6_mul_v(const fp6 &a) { return {f2_mul_xi(a.c2), a.c0, a.c1}; }

inline NOINL fp6 f6_mul(const fp6 &a, const fp6 &b) {
  fp2 v0 = f2_mul(a.c0, b.c0), v1 = f2_mul(a.c1, b.c1), v2 = f2_mul(a.c2, b.c2);
  fp2 t12 = f2_mul(f2_add(a.c1, a.c2), f2_add(b.c1, b.c2));
  fp2 t01 = f2_mul(f2_add(a.c0, a.c1), f2_add(b.c0, b.c1));
  fp2 t02 = f2_mul(f2_add(a.c0, a.c2), f2_add(b.c0, b.c2));
  fp6 r;
  r.c0 = f2_add(v0, f2_mul_xi(f2_sub(f2_sub(t12, v1), v2)));
  r.c1 = f2_add(f2_sub(f2_sub(t01, v0), v1), f2_mul_xi(v2));
  r.c2 = f2_add(f2_sub(f2_sub(t02, v0), v2), v1);
  return r;
}

// a * (b0 + b1 v)
inline NOINL fp6 f6_mul_01(const fp6 &a, const fp2 &b0, const fp2 &b1) {
  fp2 v0 = f2_mul(a.c0, b0), v1 = f2_mul(a.c1, b1);
  fp2 t01 = f2_mul(f2_add(a.c0, a.c1), f2_add(b0, b1));
  fp6 r;
  r.c0 = f2_add(v0, f2_mul_xi(f2_mul(a.c2, b1)));
  r.c1 = f2_sub(f2_sub(t01, v0), v1);
  r.c2 = f2_add(v1, f2_mul(a.c2, b0));
  return r;
}

DEV fp6 f6_mul_0(const fp6 &a, const fp2 &b0) { return {f2_mul(a.c0, b0), f2_mul(a.c1, b0), f2_mul(a.c2, b0)}; }

inline NOINL fp6 f6_inv(const fp6 &a) {
  fp2 A = f2_sub(f2_sqr(a.c0), f2_mul_xi(f2_mul(a.c1, a.c2)));
  fp2 B = f2_sub(f2_mul_xi(f2_sqr(a.c2)), f2_mul(a.c0, a.c1));
  fp2 C = f2_sub(f2_sqr(a.c1), f2_mul(a.c0, a.c2));
  fp2 F = f2_add(f2_mul(a.c0, A), f2_mul_xi(f2_add(f2_mul(a.c2, B), f2_mul(a.c1, C))));
  fp2 Fi = f2_inv(F);
  return {f2_mul(A, Fi), f2_mul(B, Fi), f2_mul(C, Fi)};
}

// ------------------------------------------------------------------ F_p12
DEV fp12 f12_one() { return {f6_one(), f6_zero()}; }
DEV fp12 f12_conj(const fp12 &a) { return {a.c0, f6_neg(a.c1)}; }

inline NOINL bool f12_eq(const fp12 &a, const fp12 &b) {
  const fe *x = &a.c0.c0.c0, *y = &b.c0.c0.c0;
  bool eq = true;
  for (int i = 0; i < 12; i++) eq = eq && fe_eq(x[i], y[i]);
  return eq;
}

inline NOINL fp12 f12_mul(const fp12 &a, const fp12 &b) {
  fp6 v0 = f6_mul(a.c0, b.c0), v1 = f6_mul(a.c1, b.c1);
  fp6 t = f6_mul(f6_add(a.c0, a.c1), f6_add(b.c0, b.c1));
  return {f6_add(v0, f6_mul_v(v1)), f6_sub(f6_sub(t, v0), v1)};
}

inline NOINL fp12 f12_sqr(const fp12 &a) {
  // (a0 + a1 w)^2 = (a0^2 + v a1^2) + 2 a0 a1 w, with
  // a0^2 + v a1^2 = (a0 + a1)(a0 + v a1) - a0 a1 - v a0 a1
  fp6 ab = f6_mul(a.c0, a.c1);
  fp6 t = f6_mul(f6_add(a.c0, a.c1), f6_add(a.c0, f6_mul_v(a.c1)));
  return {f6_sub(f6_sub(t, ab), f6_mul_v(ab)), f6_add(ab, ab)};
}

// a * (l0 + (l1 + l2 v) w): a line value with coefficients at w^0, w^1, w^3
inline NOINL fp12 f12_mul_line(const fp12 &a, const fp2 &l0, const fp2 &l1, const fp2 &l2) {
  fp6 v0 = f6_mul_0(a.c0, l0);
  fp6 v1 = f6_mul_01(a.c1, l1, l2);
  fp6 t = f6_mul_01(f6_add(a.c0, a.c1), f2_add(l0, l1), l2);
  return {f6_add(v0, f6_mul_v(v1)), f6_sub(f6_sub(t, v0), v1)};
}

inline NOINL fp12 f12_inv(const fp12 &a) {
  fp6 t = f6_sub(f6_mul(a.c0, a.c0), f6_mul_v(f6_mul(a.c1, a.c1)));
  fp6 ti = f6_inv(t);
  return {f6_mul(a.c0, ti), f6_neg(f6_mul(a.c1, ti))};
}

// Frobenius: the coefficient of w^k (k = 0..5; w^0..w^5 = c0.c0, c1.c0, c0.c1, c1.c1,
// c0.c2, c1.c2) is mapped to conj(c) gamma1_k (p), c gamma2_k (p^2), conj(c) gamma3_k (p^3)
inline NOINL fp12 f12_frob1(const fp12 &a) {
  fp12 r;
  r.c0.c0 = f2_conj(a.c0.c0);
  r.c1.c0 = f2_mul(f2_conj(a.c1.c0), f2_const(bn::FROB1_1_0, bn::FROB1_1_1));
  r.c0.c1 = f2_mul(f2_conj(a.c0.c1), f2_const(bn::FROB1_2_0, bn::FROB1_2_1));
  r.c1.c1 = f2_mul(f2_conj(a.c1.c1), f2_const(bn::FROB1_3_0, bn::FROB1_3_1));
  r.c0.c2 = f2_mul(f2_conj(a.c0.c2), f2_const(bn::FROB1_4_0, bn::FROB1_4_1));
  r.c1.c2 = f2_mul(f2_conj(a.c1.c2), f2_const(bn::FROB1_5_0, bn::FROB1_5_1));
  return r;
}

inline NOINL fp12 f12_frob2(const fp12 &a) {
  fp12 r;
  r.c0.c0 = a.c0.c0;
  r.c1.c0 = f2_mul_fp(a.c1.c0, fe_const(bn::FROB2_1));
  r.c0.c1 = f2_mul_fp(a.c0.c1, fe_const(bn::FROB2_2));
  r.c1.c1 = f2_mul_fp(a.c1.c1, fe_const(bn::FROB2_3));
  r.c0.c2 = f2_mul_fp(a.c0.c2, fe_const(bn::FROB2_4));
  r.c1.c2 = f2_mul_fp(a.c1.c2, fe_const(bn::FROB2_5));
  return r;
}

inline NOINL fp12 f12_frob3(const fp12 &a) {
  fp12 r;
  r.c0.c0 = f2_conj(a.c0.c0);
  r.c1.c0 = f2_mul(f2_conj(a.c1.c0), f2_const(bn::FROB3_1_0, bn::FROB3_1_1));
  r.c0.c1 = f2_mul(f2_conj(a.c0.c1), f2_const(bn::FROB3_2_0, bn::FROB3_2_1));
  r.c1.c1 = f2_mul(f2_conj(a.c1.c1), f2_const(bn::FROB3_3_0, bn::FROB3_3_1));
  r.c0.c2 = f2_mul(f2_conj(a.c0.c2), f2_const(bn::FROB3_4_0, bn::FROB3_4_1));
  r.c1.c2 = f2_mul(f2_conj(a.c1.c2), f2_const(bn::FROB3_5_0, bn::FROB3_5_1));
  return r;
}

// Squaring in the cyclotomic subgroup (Granger-Scott).  With t = w^3 (t^2 = xi) the
// element regroups over F_p4 = F_p2[t] as A + B w + C w^2 with A = a0 + b1 t,
// B = b0 + a2 t, C = a1 + b2 t, and its square is
//   (3A^2 - 2 conj A) + (3 t C^2 + 2 conj B) w + (3 B^2 - 2 conj C) w^2.
inline NOINL fp12 f12_cyclo_sqr(const fp12 &f) {
  const fp2 &a0 = f.c0.c0, &a1 = f.c0.c1, &a2 = f.c0.c2;
  const fp2 &b0 = f.c1.c0, &b1 = f.c1.c1, &b2 = f.c1.c2;
  // (x + y t)^2 = (x^2 + xi y^2) + 2 x y t; 2xy = (x+y)^2 - x^2 - y^2
  fp2 x2 = f2_sqr(a0), y2 = f2_sqr(b1);
  fp2 A0 = f2_add(x2, f2_mul_xi(y2)), A1 = f2_sub(f2_sub(f2_sqr(f2_add(a0, b1)), x2), y2);
  x2 = f2_sqr(b0);
  y2 = f2_sqr(a2);
  fp2 B0 = f2_add(x2, f2_mul_xi(y2)), B1 = f2_sub(f2_sub(f2_sqr(f2_add(b0, a2)), x2), y2);
  x2 = f2_sqr(a1);
  y2 = f2_sqr(b2);
  fp2 C0 = f2_add(x2, f2_mul_xi(y2)), C1 = f2_sub(f2_sub(f2_sqr(f2_add(a1, b2)), x2), y2);
  fp12 r;
  // 3X - 2x = X + 2(X - x);  3X + 2x = X + 2(X + x)
  r.c0.c0 = f2_add(A0, f2_dbl(f2_sub(A0, a0)));
  r.c1.c1 = f2_add(A1, f2_dbl(f2_add(A1, b1)));
  fp2 tC1 = f2_mul_xi(C1);  // t C^2 = xi C1 + C0 t
  r.c1.c0 = f2_add(tC1, f2_dbl(f2_add(tC1, b0)));
  r.c0.c2 = f2_add(C0, f2_dbl(f2_sub(C0, a2)));
  r.c0.c1 = f2_add(B0, f2_dbl(f2_sub(B0, a1)));
  r.c1.c2 = f2_add(B1, f2_dbl(f2_add(B1, b2)));
  return r;
}

// f^u in the cyclotomic subgroup (u = BN parameter, 63 bits, positive)
inline NOINL fp12 f12_cyclo_pow_u(const fp12 &f) {
  fp12 acc = f;
  for (int i = 61; i >= 0; i--) {
    acc = f12_cyclo_sqr(acc);
    if ((bn::BN_U >> i) & 1) acc = f12_mul(acc, f);
  }
  return acc;
}

// f^((p^12-1)/r): easy part f^((p^6-1)(p^2+1)), then the hard part exponent
// (p^4-p^2+1)/r = l0 + l1 p + l2 p^2 + p^3 with l2 = 6u^2+1, l1 = -36u^3-18u^2-12u+1,
// l0 = -36u^3-30u^2-18u-2 (an exact decomposition, checked in gen_constants.py).
inline NOINL fp12 f12_final_exp(const fp12 &f0) {
  fp12 f = f12_mul(f12_conj(f0), f12_inv(f0));
  f = f12_mul(f12_frob2(f), f);
  // now in the cyclotomic subgroup: inverse = conjugate
  fp12 a = f12_cyclo_pow_u(f);   // f^u
  fp12 b = f12_cyclo_pow_u(a);   // f^{u^2}
  fp12 c = f12_cyclo_pow_u(b);   // f^{u^3}
  fp12 c2 = f12_cyclo_sqr(c), c4 = f12_cyclo_sqr(c2), c8 = f12_cyclo_sqr(c4);
  fp12 c9 = f12_mul(c8, c), c18 = f12_cyclo_sqr(c9), c36 = f12_cyclo_sqr(c18);
  fp12 b2 = f12_cyclo_sqr(b), b3 = f12_mul(b2, b), b6 = f12_cyclo_sqr(b3);
  fp12 b12 = f12_cyclo_sqr(b6), b18 = f12_mul(b12, b6), b30 = f12_mul(b18, b12);
  fp12 a2 = f12_cyclo_sqr(a), a3 = f12_mul(a2, a), a6 = f12_cyclo_sqr(a3);
  fp12 a12 = f12_cyclo_sqr(a6), a18 = f12_mul(a12, a6);
  fp12 f2 = f12_cyclo_sqr(f);
  fp12 t0 = f12_conj(f12_mul(f12_mul(c36, b30), f12_mul(a18, f2)));   // f^{l0}
  fp12 t1 = f12_mul(f12_conj(f12_mul(f12_mul(c36, b18), a12)), f);   // f^{l1}
  fp12 t2 = f12_mul(b6, f);                                          // f^{l2}
  return f12_mul(f12_mul(t0, f12_frob1(t1)), f12_mul(f12_frob2(t2), f12_frob3(f)));
}
