// Prime-field arithmetic for BN254 on the CDNA4 integer pipes.
//
// Elements are 8 x 32-bit little-endian limbs in Montgomery form (R = 2^256),
// always fully reduced to [0, m).  Multiplication is word-serial Montgomery
// (coarsely integrated operand scanning) built on 32x32+64 -> 64 multiply-adds,
// which the compiler lowers to v_mad_u64_u32.  The same code serves F_p (curve
// coordinates) and F_r (scalars), selected by a traits class.  Everything is
// __host__ __device__ so the arithmetic can also be exercised on the CPU.
#pragma once
#include <cstdint>
#include "constants.hpp"

#ifndef __HIPCC__
#define __host__
#define __device__
#define __forceinline__ inline
#endif

#define HD __host__ __device__
#define DEV __host__ __device__ __forceinline__
// large routines are kept out of line so every kernel does not carry its own copy
#define NOINL __host__ __device__ __attribute__((noinline))

struct FpP {
  static constexpr const uint32_t *M = bn::P_MOD;
  static constexpr uint32_t INV = bn::P_INV;
  static constexpr const uint32_t *ONE = bn::P_ONE;
  static constexpr const uint32_t *R2 = bn::P_R2;
  static constexpr const uint32_t *MINUS2 = bn::P_MINUS_2;
};
struct FpR {
  static constexpr const uint32_t *M = bn::R_MOD;
  static constexpr uint32_t INV = bn::R_INV;
  static constexpr const uint32_t *ONE = bn::R_ONE;
  static constexpr const uint32_t *R2 = bn::R_R2;
  static constexpr const uint32_t *MINUS2 = bn::R_MINUS_2;
};

#ifdef VC_WIDE
#include "field_wide.hpp"
#else
struct fe {
  uint32_t l[8];
};

// Host builds may count field multiplications (to state per-operation work exactly).
#if !defined(__HIP_DEVICE_COMPILE__) && defined(VC_COUNT_MULS)
inline uint64_t &fmul_counter() {
  static thread_local uint64_t c = 0;
  return c;
}
#define COUNT_FMUL() (fmul_counter()++)
#else
#define COUNT_FMUL()
#endif

DEV fe fe_zero() {
  fe o;
#pragma unroll
  for (int i = 0; i < 8; i++) o.l[i] = 0;
  return o;
}

DEV fe fe_const(const uint32_t *c) {
  fe o;
#pragma unroll
  for (int i = 0; i < 8; i++) o.l[i] = c[i];
  return o;
}

template <class F> DEV fe f_one() { return fe_const(F::ONE); }

DEV bool fe_is_zero(const fe &a) {
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) t |= a.l[i];
  return t == 0;
}

DEV bool fe_eq(const fe &a, const fe &b) {
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) t |= a.l[i] ^ b.l[i];
  return t == 0;
}

// a - m if a >= m (a < 2m, a < 2^256)
template <class F> DEV void f_reduce_once(fe &a) {
  uint32_t d[8];
  uint64_t bw = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    uint64_t t = (uint64_t)a.l[i] - F::M[i] - bw;
    d[i] = (uint32_t)t;
    bw = t >> 63;
  }
#pragma unroll
  for (int i = 0; i < 8; i++) a.l[i] = bw ? a.l[i] : d[i];
}

template <class F> DEV fe f_add(const fe &a, const fe &b) {
  fe s;
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    c += (uint64_t)a.l[i] + b.l[i];
    s.l[i] = (uint32_t)c;
    c >>= 32;
  }
  f_reduce_once<F>(s);  // m < 2^254, so the sum never carries out of 256 bits
  return s;
}

template <class F> DEV fe f_sub(const fe &a, const fe &b) {
  fe d;
  uint64_t bw = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    uint64_t t = (uint64_t)a.l[i] - b.l[i] - bw;
    d.l[i] = (uint32_t)t;
    bw = t >> 63;
  }
  // add m back when the difference went negative
  uint64_t c = 0;
  uint32_t mask = bw ? 0xffffffffu : 0u;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    c += (uint64_t)d.l[i] + (F::M[i] & mask);
    d.l[i] = (uint32_t)c;
    c >>= 32;
  }
  return d;
}

template <class F> DEV fe f_neg(const fe &a) { return f_sub<F>(fe_zero(), a); }
template <class F> DEV fe f_dbl(const fe &a) { return f_add<F>(a, a); }

// a / 2 mod m
template <class F> DEV fe f_half(const fe &a) {
  uint32_t mask = (a.l[0] & 1) ? 0xffffffffu : 0u;
  uint32_t t[9];
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    c += (uint64_t)a.l[i] + (F::M[i] & mask);
    t[i] = (uint32_t)c;
    c >>= 32;
  }
  t[8] = (uint32_t)c;
  fe o;
#pragma unroll
  for (int i = 0; i < 8; i++) o.l[i] = (t[i] >> 1) | (t[i + 1] << 31);
  return o;
}

// Montgomery product a b R^{-1} mod m (CIOS, one reduction word per operand word)
template <class F> DEV fe f_mul(const fe &a, const fe &b) {
  COUNT_FMUL();
  uint32_t t[10];
#pragma unroll
  for (int j = 0; j < 10; j++) t[j] = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      c = (uint64_t)a.l[j] * b.l[i] + t[j] + (c >> 32);
      t[j] = (uint32_t)c;
    }
    uint64_t s = (uint64_t)t[8] + (c >> 32);
    t[8] = (uint32_t)s;
    t[9] = (uint32_t)(s >> 32);
    uint32_t mq = t[0] * F::INV;
    c = (uint64_t)mq * F::M[0] + t[0];
#pragma unroll
    for (int j = 1; j < 8; j++) {
      c = (uint64_t)mq * F::M[j] + t[j] + (c >> 32);
      t[j - 1] = (uint32_t)c;
    }
    s = (uint64_t)t[8] + (c >> 32);
    t[7] = (uint32_t)s;
    t[8] = t[9] + (uint32_t)(s >> 32);
  }
  fe o;
#pragma unroll
  for (int j = 0; j < 8; j++) o.l[j] = t[j];
  f_reduce_once<F>(o);
  return o;
}

template <class F> DEV fe f_sqr(const fe &a) { return f_mul<F>(a, a); }

// small constant multiple by repeated doubling/adding
template <class F> DEV fe f_mul_small(const fe &a, int k) {
  fe acc = fe_zero(), base = a;
  while (k) {
    if (k & 1) acc = f_add<F>(acc, base);
    base = f_dbl<F>(base);
    k >>= 1;
  }
  return acc;
}

template <class F> DEV fe f_to_mont(const fe &a) { return f_mul<F>(a, fe_const(F::R2)); }
template <class F> DEV fe f_from_mont(const fe &a) {
  fe one = fe_zero();
  one.l[0] = 1;
  return f_mul<F>(a, one);
}

// a^e for a fixed 256-bit exponent (little-endian limbs)
template <class F> NOINL fe f_pow(const fe &a, const uint32_t *e) {
  fe acc = f_one<F>();
  for (int i = 255; i >= 0; i--) {
    acc = f_sqr<F>(acc);
    if ((e[i >> 5] >> (i & 31)) & 1) acc = f_mul<F>(acc, a);
  }
  return acc;
}

template <class F> NOINL fe f_inv(const fe &a) { return f_pow<F>(a, F::MINUS2); }

// canonical integer compare: a > b
DEV bool fe_gt_canon(const fe &a, const uint32_t *b) {
  bool gt = false, decided = false;
#pragma unroll
  for (int i = 7; i >= 0; i--) {
    if (!decided && a.l[i] != b[i]) {
      gt = a.l[i] > b[i];
      decided = true;
    }
  }
  return gt;
}

DEV bool fe_lt_mod(const fe &a, const uint32_t *m) {
  uint64_t bw = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    uint64_t t = (uint64_t)a.l[i] - m[i] - bw;
    bw = t >> 63;
  }
  return bw != 0;
}

DEV uint32_t fe_word(const fe &a, int i) { return a.l[i]; }
DEV fe fe_from_words(const uint32_t *w) { return fe_const(w); }

// Inverse by the binary extended Euclidean algorithm (variable time; the inputs
// here are public).  Input and output in Montgomery form: the integer inverse of
// A = aR is a^{-1} R^{-1}, and one Montgomery product with R^3 gives a^{-1} R.
template <class F> NOINL fe f_inv_binary(const fe &A, const uint32_t *R3) {
  if (fe_is_zero(A)) return fe_zero();
  fe u = A, v = fe_const(F::M), x1 = fe_zero(), x2 = fe_zero();
  x1.l[0] = 1;
  auto is_one = [](const fe &a) {
    uint32_t t = a.l[0] ^ 1u;
    for (int i = 1; i < 8; i++) t |= a.l[i];
    return t == 0;
  };
  auto shr1 = [](fe &a) {
    for (int i = 0; i < 7; i++) a.l[i] = (a.l[i] >> 1) | (a.l[i + 1] << 31);
    a.l[7] >>= 1;
  };
  auto geq = [](const fe &a, const fe &b) {
    for (int i = 7; i >= 0; i--)
      if (a.l[i] != b.l[i]) return a.l[i] > b.l[i];
    return true;
  };
  auto subi = [](fe &a, const fe &b) {
    uint64_t bw = 0;
    for (int i = 0; i < 8; i++) {
      uint64_t t = (uint64_t)a.l[i] - b.l[i] - bw;
      a.l[i] = (uint32_t)t;
      bw = t >> 63;
    }
  };
  while (!is_one(u) && !is_one(v)) {
    while ((u.l[0] & 1) == 0) { shr1(u); x1 = f_half<F>(x1); }
    while ((v.l[0] & 1) == 0) { shr1(v); x2 = f_half<F>(x2); }
    if (geq(u, v)) { subi(u, v); x1 = f_sub<F>(x1, x2); }
    else { subi(v, u); x2 = f_sub<F>(x2, x1); }
  }
  fe r = is_one(u) ? x1 : x2;
  return f_mul<F>(r, fe_const(R3));
}
#endif  // VC_WIDE

#define fp_add f_add<FpP>
#define fp_sub f_sub<FpP>
#define fp_neg f_neg<FpP>
#define fp_dbl f_dbl<FpP>
#define fp_mul f_mul<FpP>
#define fp_sqr f_sqr<FpP>
#define fp_half f_half<FpP>
#define fp_inv f_inv<FpP>
#define fr_add f_add<FpR>
#define fr_sub f_sub<FpR>
#define fr_mul f_mul<FpR>
#define fr_inv f_inv<FpR>

#define fp_inv_fast(a) f_inv_binary<FpP>(a, bn::P_R3)
#define fr_inv_fast(a) f_inv_binary<FpR>(a, bn::R_R3)
