// G1 (y^2 = x^3 + 3 over F_p) and G2 (the D-type twist y^2 = x^3 + 3/xi over F_p2)
// group arithmetic.  One template body serves both groups through a small traits
// class over the coordinate field.  Points in memory are affine with the identity
// encoded as (0, 0) (not on either curve); in registers they are Jacobian
// (x = X/Z^2, y = Y/Z^3, Z = 0 is the identity).  Formulas: doubling dbl-2009-l,
// mixed addition madd-2007-bl and addition add-2007-bl (a = 0), with the
// exceptional cases (equal or opposite inputs, identity) handled explicitly.
#pragma once
#include "tower.hpp"

struct OpsG1 {
  using T = fe;
  static DEV T add(const T &a, const T &b) { return fp_add(a, b); }
  static DEV T sub(const T &a, const T &b) { return fp_sub(a, b); }
  static DEV T mul(const T &a, const T &b) { return fp_mul(a, b); }
  static DEV T sqr(const T &a) { return fp_sqr(a); }
  static DEV T dbl(const T &a) { return fp_dbl(a); }
  static DEV T neg(const T &a) { return fp_neg(a); }
  static DEV T zero() { return fe_zero(); }
  static DEV T one() { return f_one<FpP>(); }
  static DEV bool is_zero(const T &a) { return fe_is_zero(a); }
  static NOINL T inv(const T &a) { return fp_inv_fast(a); }
  static DEV T b() { return f_mul_small<FpP>(f_one<FpP>(), 3); }
};

struct OpsG2 {
  using T = fp2;
  static DEV T add(const T &a, const T &b) { return f2_add(a, b); }
  static DEV T sub(const T &a, const T &b) { return f2_sub(a, b); }
  static DEV T mul(const T &a, const T &b) { return f2_mul(a, b); }
  static DEV T sqr(const T &a) { return f2_sqr(a); }
  static DEV T dbl(const T &a) { return f2_dbl(a); }
  static DEV T neg(const T &a) { return f2_neg(a); }
  static DEV T zero() { return f2_zero(); }
  static DEV T one() { return f2_one(); }
  static DEV bool is_zero(const T &a) { return f2_is_zero(a); }
  static NOINL T inv(const T &a) { return f2_inv(a); }
  static DEV T b() { return f2_const(bn::TWIST_B0, bn::TWIST_B1); }
};

template <class O> struct aff {
  typename O::T x, y;  // identity = (0, 0)
};
template <class O> struct jac {
  typename O::T X, Y, Z;
};

using g1_aff = aff<OpsG1>;
using g2_aff = aff<OpsG2>;
using g1_jac = jac<OpsG1>;
using g2_jac = jac<OpsG2>;

template <class O> DEV bool aff_is_inf(const aff<O> &p) { return O::is_zero(p.x) && O::is_zero(p.y); }
template <class O> DEV aff<O> aff_inf() { return {O::zero(), O::zero()}; }
template <class O> DEV aff<O> aff_neg(const aff<O> &p) {
  return aff_is_inf(p) ? p : aff<O>{p.x, O::neg(p.y)};
}

template <class O> DEV jac<O> jac_inf() { return {O::one(), O::one(), O::zero()}; }
template <class O> DEV bool jac_is_inf(const jac<O> &p) { return O::is_zero(p.Z); }
template <class O> DEV jac<O> jac_from_aff(const aff<O> &p) {
  return aff_is_inf(p) ? jac_inf<O>() : jac<O>{p.x, p.y, O::one()};
}
template <class O> DEV jac<O> jac_neg(const jac<O> &p) { return {p.X, O::neg(p.Y), p.Z}; }

template <class O> NOINL jac<O> jac_dbl(const jac<O> &p) {
  using T = typename O::T;
  if (jac_is_inf(p)) return p;
  T A = O::sqr(p.X), B = O::sqr(p.Y), C = O::sqr(B);
  T D = O::dbl(O::sub(O::sub(O::sqr(O::add(p.X, B)), A), C));
  T E = O::add(O::dbl(A), A), F = O::sqr(E);
  jac<O> r;
  r.X = O::sub(F, O::dbl(D));
  T C8 = O::dbl(O::dbl(O::dbl(C)));
  r.Y = O::sub(O::mul(E, O::sub(D, r.X)), C8);
  r.Z = O::dbl(O::mul(p.Y, p.Z));
  return r;
}

// p + q with q affine
template <class O> NOINL jac<O> jac_madd(const jac<O> &p, const aff<O> &q) {
  using T = typename O::T;
  if (aff_is_inf(q)) return p;
  if (jac_is_inf(p)) return jac_from_aff(q);
  T Z1Z1 = O::sqr(p.Z);
  T U2 = O::mul(q.x, Z1Z1);
  T S2 = O::mul(q.y, O::mul(p.Z, Z1Z1));
  T H = O::sub(U2, p.X);
  T rr = O::dbl(O::sub(S2, p.Y));
  if (O::is_zero(H)) {
    if (O::is_zero(rr)) return jac_dbl(p);
    return jac_inf<O>();
  }
  T HH = O::sqr(H);
  T I = O::dbl(O::dbl(HH));
  T J = O::mul(H, I);
  T V = O::mul(p.X, I);
  jac<O> r;
  r.X = O::sub(O::sub(O::sqr(rr), J), O::dbl(V));
  r.Y = O::sub(O::mul(rr, O::sub(V, r.X)), O::dbl(O::mul(p.Y, J)));
  r.Z = O::sub(O::sub(O::sqr(O::add(p.Z, H)), Z1Z1), HH);
  return r;
}

template <class O> NOINL jac<O> jac_add(const jac<O> &p, const jac<O> &q) {
  using T = typename O::T;
  if (jac_is_inf(p)) return q;
  if (jac_is_inf(q)) return p;
  T Z1Z1 = O::sqr(p.Z), Z2Z2 = O::sqr(q.Z);
  T U1 = O::mul(p.X, Z2Z2), U2 = O::mul(q.X, Z1Z1);
  T S1 = O::mul(p.Y, O::mul(q.Z, Z2Z2)), S2 = O::mul(q.Y, O::mul(p.Z, Z1Z1));
  T H = O::sub(U2, U1);
  T rr = O::dbl(O::sub(S2, S1));
  if (O::is_zero(H)) {
    if (O::is_zero(rr)) return jac_dbl(p);
    return jac_inf<O>();
  }
  T I = O::sqr(O::dbl(H));
  T J = O::mul(H, I);
  T V = O::mul(U1, I);
  jac<O> r;
  r.X = O::sub(O::sub(O::sqr(rr), J), O::dbl(V));
  r.Y = O::sub(O::mul(rr, O::sub(V, r.X)), O::dbl(O::mul(S1, J)));
  r.Z = O::mul(O::sub(O::sub(O::sqr(O::add(p.Z, q.Z)), Z1Z1), Z2Z2), H);
  return r;
}

template <class O> NOINL aff<O> jac_to_aff(const jac<O> &p) {
  if (jac_is_inf(p)) return aff_inf<O>();
  typename O::T zi = O::inv(p.Z), zi2 = O::sqr(zi);
  return {O::mul(p.X, zi2), O::mul(p.Y, O::mul(zi2, zi))};
}

// with a precomputed inverse of Z (batch inversion)
template <class O> DEV aff<O> jac_to_aff_zi(const jac<O> &p, const typename O::T &zi) {
  if (jac_is_inf(p)) return aff_inf<O>();
  typename O::T zi2 = O::sqr(zi);
  return {O::mul(p.X, zi2), O::mul(p.Y, O::mul(zi2, zi))};
}

// k P for a canonical 256-bit scalar (little-endian 32-bit words), left to right,
// 4-bit fixed windows over a table of 1P..15P kept in Jacobian form
template <class O> NOINL jac<O> scalar_mul(const aff<O> &P, const uint32_t k[8]) {
  jac<O> tab[16];
  tab[0] = jac_inf<O>();
  tab[1] = jac_from_aff(P);
  tab[2] = jac_dbl(tab[1]);
  for (int i = 3; i < 16; i++) tab[i] = jac_madd(tab[i - 1], P);
  jac<O> acc = jac_inf<O>();
  for (int w = 63; w >= 0; w--) {
    acc = jac_dbl(jac_dbl(jac_dbl(jac_dbl(acc))));
    uint32_t d = (k[w >> 3] >> ((w & 7) * 4)) & 15;
    if (d) acc = jac_add(acc, tab[d]);
  }
  return acc;
}

#include "glv.hpp"

// k P on G1 with the GLV split k = k_0 + k_1 lam: bases B0 = sign(k_0) P and
// B1 = sign(k_1) phi(P), phi(x, y) = (beta x, y); joint 2-bit windows d0 + 4 d1 over the
// table d0 B0 + d1 B1 (Jacobian), two doublings and at most one addition per window
inline NOINL g1_jac g1_mul_glv(const g1_aff &P, const glv::Dec &d) {
  if (aff_is_inf(P) || d.nbits == 0) return jac_inf<OpsG1>();
  g1_aff B0 = P, B1 = {fp_mul(P.x, fe_const(bn::GLV_BETA)), P.y};
  if (d.neg & 1) B0 = aff_neg(B0);
  if (d.neg & 2) B1 = aff_neg(B1);
  g1_jac T[16];
  T[0] = jac_inf<OpsG1>();
  T[1] = jac_from_aff(B0);
  T[2] = jac_dbl(T[1]);
  T[3] = jac_madd(T[2], B0);
  T[4] = jac_from_aff(B1);
  T[8] = jac_dbl(T[4]);
  T[12] = jac_madd(T[8], B1);
  for (int d1 = 1; d1 < 4; d1++)
    for (int d0 = 1; d0 < 4; d0++) T[d0 + 4 * d1] = jac_add(T[4 * d1], T[d0]);
  int nw = (int)(d.nbits + 1) / 2;
  g1_jac acc = T[glv::digit2(d, (uint32_t)(nw - 1))];
  for (int w = nw - 2; w >= 0; w--) {
    acc = jac_dbl(jac_dbl(acc));
    uint32_t dg = glv::digit2(d, (uint32_t)w);
    if (dg) acc = jac_add(acc, T[dg]);
  }
  return acc;
}

template <class O> DEV bool aff_on_curve(const aff<O> &p) {
  if (aff_is_inf(p)) return true;
  typename O::T l = O::sqr(p.y), r = O::add(O::mul(O::sqr(p.x), p.x), O::b());
  return O::is_zero(O::sub(l, r));
}

// p-power Frobenius of a twist point: (conj(x) xi^{(p-1)/3}, conj(y) xi^{(p-1)/2})
DEV g2_aff g2_frobenius(const g2_aff &q) {
  if (aff_is_inf(q)) return q;
  return {f2_mul(f2_conj(q.x), f2_const(bn::FROB1_2_0, bn::FROB1_2_1)),
          f2_mul(f2_conj(q.y), f2_const(bn::FROB1_3_0, bn::FROB1_3_1))};
}
