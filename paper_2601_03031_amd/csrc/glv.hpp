#pragma once
#include <cstdint>
#include "constants.hpp"

// Scalar decomposition for G1 scalar multiplication with phi(x, y) = (beta x, y), which
// acts as multiplication by a cube root of unity lam mod r (Gallant-Lambert-Vanstone):
// k = k_0 + k_1 lam (mod r), |k_i| < 2^128, from a reduced basis of
// {(a, b) : a + b lam = 0 mod r} and truncated Babai rounding (bn::GLV_* constants).
namespace glv {

struct Dec {
  uint32_t mag[2][4];  // |k_j|
  uint32_t neg;        // bit j: k_j < 0
  uint32_t nbits;      // bit length of max |k_j|
};

__host__ __device__ inline Dec decompose(const uint32_t *k) {
  // k_j = [j = 0] k + sum_i c'_i B_ij (mod 2^192), c'_i = floor(k |G_i| / 2^256)
  uint32_t acc[2][6];
  for (int j = 0; j < 2; j++)
    for (int w = 0; w < 6; w++) acc[j][w] = j == 0 ? k[w] : 0u;
  for (int i = 0; i < 2; i++) {
    uint32_t prod[13] = {0};
    for (int a = 0; a < 8; a++) {
      uint64_t carry = 0;
      for (int b = 0; b < 5; b++) {
        uint64_t t = (uint64_t)k[a] * bn::GLV_G_ABS[i][b] + prod[a + b] + carry;
        prod[a + b] = (uint32_t)t;
        carry = t >> 32;
      }
      prod[a + 5] = (uint32_t)carry;
    }
    const uint32_t *c = prod + 8;  // c'_i < 2^130: words 8..12
    for (int j = 0; j < 2; j++) {
      uint32_t term[6] = {0, 0, 0, 0, 0, 0};
      for (int a = 0; a < 5; a++) {
        uint64_t carry = 0;
        for (int b = 0; b < 4 && a + b < 6; b++) {
          uint64_t t = (uint64_t)c[a] * bn::GLV_B_ABS[i][j][b] + term[a + b] + carry;
          term[a + b] = (uint32_t)t;
          carry = t >> 32;
        }
        if (a + 4 < 6) term[a + 4] += (uint32_t)carry;
      }
      bool sub = bn::GLV_B_NEG[i][j] != 0;  // + c' B_ij: subtract when B_ij < 0
      uint64_t cy = sub ? 1 : 0;
      for (int w = 0; w < 6; w++) {
        uint64_t t = (uint64_t)acc[j][w] + (sub ? (uint32_t)~term[w] : term[w]) + cy;
        acc[j][w] = (uint32_t)t;
        cy = t >> 32;
      }
    }
  }
  Dec d;
  d.neg = 0;
  uint32_t nb = 0;
  for (int j = 0; j < 2; j++) {
    uint32_t m[6];
    if (acc[j][5] >> 31) {
      d.neg |= 1u << j;
      uint64_t cy = 1;
      for (int w = 0; w < 6; w++) {
        uint64_t t = (uint64_t)(uint32_t)~acc[j][w] + cy;
        m[w] = (uint32_t)t;
        cy = t >> 32;
      }
    } else {
      for (int w = 0; w < 6; w++) m[w] = acc[j][w];
    }
    for (int w = 0; w < 4; w++) d.mag[j][w] = m[w];
    for (int w = 3; w >= 0; w--)
      if (m[w]) {
        uint32_t bl = 32 * w + 32 - __builtin_clz(m[w]);
        nb = bl > nb ? bl : nb;
        break;
      }
  }
  d.nbits = nb;
  return d;
}

// joint 2-bit digit of window w: d0 + 4 d1 with d_j the bits 2w, 2w+1 of |k_j|
// bit length of a little-endian magnitude of n words
__host__ __device__ inline uint32_t mag_bits(const uint32_t *m, int n) {
  for (int w = n - 1; w >= 0; w--)
    if (m[w]) return 32 * w + 32 - __builtin_clz(m[w]);
  return 0;
}

// The part of the split with bits [32 t, 32 t + 32) of each |k_j| (signs kept): with
// P_t = 2^{32 t} P, k P = sum_{t < 4} chunk_t(k) P_t.
__host__ __device__ inline Dec chunk(const Dec &d, int t) {
  Dec c;
  for (int j = 0; j < 2; j++) {
    c.mag[j][0] = d.mag[j][t];
    c.mag[j][1] = c.mag[j][2] = c.mag[j][3] = 0;
  }
  c.neg = d.neg;
  uint32_t a = mag_bits(c.mag[0], 1), b = mag_bits(c.mag[1], 1);
  c.nbits = d.nbits == 0 ? 0 : (a > b ? a : b);
  return c;
}

__host__ __device__ inline uint32_t digit2(const Dec &d, uint32_t w) {
  uint32_t b = 2 * w;
  uint32_t d0 = (d.mag[0][b >> 5] >> (b & 31)) & 3u, d1 = (d.mag[1][b >> 5] >> (b & 31)) & 3u;
  return d0 | (d1 << 2);
}

}  // namespace glv
