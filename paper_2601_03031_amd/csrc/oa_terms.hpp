// Terms of the next round of FC.BOpen, taken before that round's challenge is known.
//
// In a round on arrays A (G1), V (G2), b (F_r) of length n = 2h (per batch, at offset k K),
// L = (prod_{i<h} e(A[h+i], V[i]), sum_i b[i] A[h+i]) and
// R = (prod_{i<h} e(A[i], V[h+i]), sum_i b[h+i] A[i]); every term is a pair (a, v)
// contributing e(A[a], V[v]) and b[v] A[a].  The fold with challenge x gives
// A'[i] = A[i] + x A[h+i], V'[i] = V[i] + x^{-1} V[h+i], b'[i] = b[i] + x^{-1} b[h+i]
// (Eq. folding).  With q = h/2, bilinearity splits the next round's L', R' into groups
// over the current arrays:
//   L' = U_L X_L^x Y_L^{1/x}, U_L: (q+i, i), (h+q+i, h+i); X_L: (h+q+i, i); Y_L: (q+i, h+i)
//   R' = U_R X_R^x Y_R^{1/x}, U_R: (i, q+i), (h+i, h+q+i); X_R: (h+i, q+i); Y_R: (i, h+q+i)
// (i < q; the same exponents apply to the G1 sums), so every Miller loop and scalar
// multiplication of the next round runs while the current challenge is being derived.
//
// Output layout per call (nb batches): the U area holds group (2k + side) at
// [(2k + side) 2q, +2q); the XY area, after the U area, holds group (4k + g) at
// nb 4q + [(4k + g) q, +q) with g = 0: X_L, 1: Y_L, 2: X_R, 3: Y_R.
#pragma once
#include <cstdint>

namespace oat {

struct Term {
  uint64_t a, v, out;  // A and V (and b) indices including the batch offset; output index
};

// term id in [0, nb 8q)
__host__ __device__ inline Term term(uint64_t id, uint64_t K, uint64_t nb, uint64_t q) {
  uint64_t k = id / (8 * q), r = id % (8 * q), h = 2 * q, base = k * K;
  Term t;
  if (r < 4 * q) {
    uint64_t side = r / (2 * q), u = r % (2 * q), part = u / q, i = u % q;
    if (side == 0) {
      t.a = part ? h + q + i : q + i;
      t.v = part ? h + i : i;
    } else {
      t.a = part ? h + i : i;
      t.v = part ? h + q + i : q + i;
    }
    t.out = (2 * k + side) * (2 * q) + u;
  } else {
    uint64_t g = (r - 4 * q) / q, i = (r - 4 * q) % q;
    switch (g) {
      case 0: t.a = h + q + i; t.v = i; break;          // X_L
      case 1: t.a = q + i; t.v = h + i; break;          // Y_L
      case 2: t.a = h + i; t.v = q + i; break;          // X_R
      default: t.a = i; t.v = h + q + i; break;         // Y_R
    }
    t.out = nb * 4 * q + (4 * k + g) * q + i;
  }
  t.a += base;
  t.v += base;
  return t;
}

}  // namespace oat
