// Optimal ate pairing on BN254: Miller loop over 6u+2 with homogeneous projective
// coordinates for the twist point T (x = X/Z, y = Y/Z), followed by the two
// Frobenius lines, and the final exponentiation of tower.hpp.
//
// Line values are taken at P = (xP, yP) in G1 through the untwisted points
// psi(x, y) = (x w^2, y w^3); a line with slope lambda*w through psi(T) evaluates to
// yP - lambda xP w + (lambda xT - yT) v w, stored as (l0, l1, l2) at w^0, w^1, w^3.
// Each line below is that value times a factor in F_p2, which the final
// exponentiation removes.
//   doubling (times 2YZ):          l0 = 2YZ yP, l1 = -3X^2 xP, l2 = Y^2 - 3b'Z^2
//   addition with affine Q=(x2,y2) (times iota = X - x2 Z, theta = Y - y2 Z):
//                                  l0 = iota yP, l1 = -theta xP, l2 = theta x2 - iota y2
#pragma once
#include "curve.hpp"

struct proj2 {
  fp2 X, Y, Z;
};

// T <- 2T, returns the tangent line
inline NOINL void miller_dbl(proj2 &T, const fe &xP, const fe &yP, fp2 &l0, fp2 &l1, fp2 &l2) {
  fp2 B = f2_sqr(T.Y), C = f2_sqr(T.Z);
  fp2 E = f2_mul(f2_add(f2_dbl(C), C), OpsG2::b());   // 3 b' Z^2
  fp2 F = f2_add(f2_dbl(E), E);                        // 9 b' Z^2
  fp2 H = f2_sub(f2_sqr(f2_add(T.Y, T.Z)), f2_add(B, C));  // 2YZ
  fp2 X2 = f2_sqr(T.X);
  l0 = f2_mul_fp(H, yP);
  l1 = f2_neg(f2_mul_fp(f2_add(f2_dbl(X2), X2), xP));
  l2 = f2_sub(B, E);
  fp2 A = f2_half(f2_mul(T.X, T.Y));
  fp2 G = f2_half(f2_add(B, F));
  fp2 E2 = f2_sqr(E);
  proj2 R;
  R.X = f2_mul(A, f2_sub(B, F));
  R.Y = f2_sub(f2_sqr(G), f2_add(f2_dbl(E2), E2));
  R.Z = f2_mul(B, H);
  T = R;
}

// T <- T + Q (Q affine, T != +-Q), returns the chord line
inline NOINL void miller_add(proj2 &T, const g2_aff &Q, const fe &xP, const fe &yP, fp2 &l0, fp2 &l1, fp2 &l2) {
  fp2 theta = f2_sub(T.Y, f2_mul(Q.y, T.Z));
  fp2 iota = f2_sub(T.X, f2_mul(Q.x, T.Z));
  l0 = f2_mul_fp(iota, yP);
  l1 = f2_neg(f2_mul_fp(theta, xP));
  l2 = f2_sub(f2_mul(theta, Q.x), f2_mul(iota, Q.y));
  fp2 C = f2_sqr(theta), D = f2_sqr(iota);
  fp2 E = f2_mul(iota, D);
  fp2 F = f2_mul(T.Z, C);
  fp2 G = f2_mul(T.X, D);
  fp2 H = f2_sub(f2_add(E, F), f2_dbl(G));
  proj2 R;
  R.X = f2_mul(iota, H);
  R.Y = f2_sub(f2_mul(theta, f2_sub(G, H)), f2_mul(T.Y, E));
  R.Z = f2_mul(T.Z, E);
  T = R;
}

// Miller value f_{6u+2,Q}(P) times the two Frobenius lines (unreduced)
inline NOINL fp12 miller_loop(const g1_aff &P, const g2_aff &Q) {
  fp12 f = f12_one();
  if (aff_is_inf(P) || aff_is_inf(Q)) return f;
  proj2 T = {Q.x, Q.y, f2_one()};
  const g2_aff Qn = aff_neg(Q);
  fp2 l0, l1, l2;
  // over the non-adjacent form of 6u + 2 (d_65 = 1 starts T = Q; d_64 = 0): 21 additions of
  // +-Q against 36 for the binary digits
  for (int i = 64; i >= 0; i--) {
    if (i != 64) f = f12_sqr(f);
    miller_dbl(T, P.x, P.y, l0, l1, l2);
    f = f12_mul_line(f, l0, l1, l2);
    const bool pos = i < 64 && ((bn::ATE_NAF_POS >> i) & 1), neg = i < 64 && ((bn::ATE_NAF_NEG >> i) & 1);
    if (pos || neg) {
      miller_add(T, pos ? Q : Qn, P.x, P.y, l0, l1, l2);
      f = f12_mul_line(f, l0, l1, l2);
    }
  }
  g2_aff Q1 = g2_frobenius(Q);
  g2_aff Q2 = aff_neg(g2_frobenius(Q1));
  miller_add(T, Q1, P.x, P.y, l0, l1, l2);
  f = f12_mul_line(f, l0, l1, l2);
  miller_add(T, Q2, P.x, P.y, l0, l1, l2);
  f = f12_mul_line(f, l0, l1, l2);
  return f;
}
