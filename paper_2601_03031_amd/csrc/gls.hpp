// Scalar decomposition for G2 scalar multiplication with the endomorphism psi
// (Galbraith-Lin-Scott): psi acts on G2 as multiplication by lam = p mod r, and a scalar
// k < r is written k = sum_j k_j lam^j (mod r) with |k_j| < 2^65 by Babai rounding
// against a reduced basis of the lattice {x : x0 + x1 lam + x2 lam^2 + x3 lam^3 = 0 mod r}
// (basis and rounding constants are generated in gen_slp.py).  Single lane, host and
// device.
#pragma once
#include <cstdint>
#include "slp_progs.hpp"

namespace gls {

struct Dec {
  uint32_t mag[4][3];  // |k_j|, little-endian 32-bit limbs
  uint32_t neg;        // bit j: k_j < 0
  uint32_t nbits;      // bit length of max_j |k_j| (0 when k = 0)
};

// k: canonical scalar, 8 little-endian 32-bit limbs
__host__ __device__ inline Dec decompose(const uint32_t *k) {
  Dec d;
  uint32_t acc[4][4];
  for (int j = 0; j < 4; j++)
    for (int w = 0; w < 4; w++) acc[j][w] = j == 0 ? k[w] : 0u;
  for (int i = 0; i < 4; i++) {
    // c_i = floor(k G_i / 2^256); only c_i mod 2^128 is needed (words 8..11 of the product)
    uint32_t prod[14] = {0};
    for (int a = 0; a < 8; a++) {
      uint64_t carry = 0;
      for (int b = 0; b < 6; b++) {
        uint64_t t = (uint64_t)k[a] * slp::GLS_G[i][b] + prod[a + b] + carry;
        prod[a + b] = (uint32_t)t;
        carry = t >> 32;
      }
      prod[a + 6] = (uint32_t)carry;
    }
    const uint32_t *c = prod + 8;
    for (int j = 0; j < 4; j++) {
      // term = c * |B_ij| mod 2^128; k_j -= sign(B_ij) term
      uint32_t b[2] = {(uint32_t)slp::GLS_B_ABS[i][j], (uint32_t)(slp::GLS_B_ABS[i][j] >> 32)};
      uint32_t term[4] = {0, 0, 0, 0};
      for (int a = 0; a < 4; a++) {
        uint64_t carry = 0;
        for (int bb = 0; bb < 2 && a + bb < 4; bb++) {
          uint64_t t = (uint64_t)c[a] * b[bb] + term[a + bb] + carry;
          term[a + bb] = (uint32_t)t;
          carry = t >> 32;
        }
        if (a + 2 < 4) term[a + 2] += (uint32_t)carry;
      }
      bool sub = slp::GLS_B_NEG[i][j] == 0;
      uint64_t cy = sub ? 1 : 0;  // a - t = a + ~t + 1
      for (int w = 0; w < 4; w++) {
        uint64_t t = (uint64_t)acc[j][w] + (sub ? (uint32_t)~term[w] : term[w]) + cy;
        acc[j][w] = (uint32_t)t;
        cy = t >> 32;
      }
    }
  }
  d.neg = 0;
  uint32_t top = 0;
  for (int j = 0; j < 4; j++) {
    uint32_t m[4];
    if (acc[j][3] >> 31) {
      d.neg |= 1u << j;
      uint64_t cy = 1;
      for (int w = 0; w < 4; w++) {
        uint64_t t = (uint64_t)(uint32_t)~acc[j][w] + cy;
        m[w] = (uint32_t)t;
        cy = t >> 32;
      }
    } else {
      for (int w = 0; w < 4; w++) m[w] = acc[j][w];
    }
    for (int w = 0; w < 3; w++) d.mag[j][w] = m[w];
    top |= (m[3] != 0) ? 0xffffffffu : 0u;  // cannot happen: |k_j| < 2^65
  }
  uint32_t nb = 0;
  for (int j = 0; j < 4; j++)
    for (int w = 2; w >= 0; w--)
      if (d.mag[j][w]) {
        uint32_t v = d.mag[j][w];
        uint32_t bl = 32 * w + 32 - __builtin_clz(v);
        nb = bl > nb ? bl : nb;
        break;
      }
  d.nbits = top ? 0xffffffffu : nb;
  return d;
}

// The part of the split with bits [lo, lo + width) of each |k_j| (signs kept), width <= 32:
// with g_lo = g^{2^lo} (or 2^lo Q), the parts over consecutive ranges multiply (add) to the whole.
__host__ __device__ inline Dec chunk(const Dec &d, int lo, int width) {
  Dec c;
  uint32_t top = 0;
  for (int j = 0; j < 4; j++) {
    int w = lo >> 5, s = lo & 31;
    uint64_t v = d.mag[j][w] >> s;
    if (s && w + 1 < 3) v |= (uint64_t)d.mag[j][w + 1] << (32 - s);
    v &= width == 32 ? 0xffffffffull : ((1ull << width) - 1);
    c.mag[j][0] = (uint32_t)v;
    c.mag[j][1] = c.mag[j][2] = 0;
    top |= c.mag[j][0];
  }
  c.neg = d.neg;
  c.nbits = (d.nbits == 0 || top == 0) ? 0 : 32 - __builtin_clz(top);
  return c;
}

// digit of bit position t: bit j is bit t of |k_j|
__host__ __device__ inline uint32_t digit(const Dec &d, uint32_t t) {
  uint32_t r = 0;
  for (int j = 0; j < 4; j++) r |= ((d.mag[j][t >> 5] >> (t & 31)) & 1u) << j;
  return r;
}

}  // namespace gls
