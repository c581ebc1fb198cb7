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
#if defined(VC_WIDE) || defined(VC_INLINE_HELPERS)
// (the 8-lane kernels hold a few registers per element: their helpers are inlined, so that
// operands passed by reference stay in registers instead of going through scratch memory;
// a one-lane file may ask for the same)
#define NOINL __host__ __device__ __forceinline__
#else
#define NOINL __host__ __device__ __attribute__((noinline))
#endif

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
// Modular inverse by the binary extended GCD with batched steps (after T. Pornin,
// "Optimized Binary GCD for Modular Inversion", 2020).  Invariants: x u = a and x v = b
// (mod m), starting from a = x, b = m, u = 1, v = 0.  Each outer round takes 30 binary-GCD
// steps (if a is odd: order a >= b by a swap, a -= b; then a /= 2) on 64-bit
// approximations of a and b (their low 30 bits, exact, and the top 34 bits of the longer
// one), recording the steps as a 2 x 2 integer matrix, and then applies the matrix to the
// full a, b (an exact division by 2^30) and to u, v (a Montgomery division by 2^30 mod m).
// It ends when a = 0, so b = gcd = 1 and v = x^{-1}.  All values depend only on the input,
// so a wave-uniform input keeps the whole computation on the scalar unit.
namespace bingcd {

DEV int bitlen(const fe &a) {
  for (int i = 7; i >= 0; i--)
    if (a.l[i]) return 32 * i + 32 - __builtin_clz(a.l[i]);
  return 0;
}

// 64-bit approximation: low 30 bits of a, then the 34 bits of a below bit n
DEV uint64_t approx(const fe &a, int n) {
  uint64_t lo = a.l[0] & 0x3fffffffu;
  if (n <= 64) return (uint64_t)a.l[0] | ((uint64_t)a.l[1] << 32);
  int s = n - 34, w = s >> 5, sh = s & 31;
  // words w, w + 1, w + 2 (zero past the top) picked by selects: an index into the limbs
  // would put the element in scratch memory
  uint32_t a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    a0 = i == w ? a.l[i] : a0;
    a1 = i == w + 1 ? a.l[i] : a1;
    a2 = i == w + 2 ? a.l[i] : a2;
  }
  uint64_t v = (uint64_t)a0 >> sh;
  v |= (uint64_t)a1 << (32 - sh);
  if (sh > 30) v |= (uint64_t)a2 << (64 - sh);
  return lo | ((v & 0x3ffffffffull) << 30);
}

// (f a + g b) / 2^30 (exact) as a signed value: magnitude in r, returns true if negative
DEV bool lin_shift(const fe &a, const fe &b, int32_t f, int32_t g, fe &r) {
  uint32_t t[9];
  int64_t acc = 0;
  for (int i = 0; i < 8; i++) {
    acc += (int64_t)a.l[i] * f;
    t[i] = (uint32_t)acc;
    acc >>= 32;
  }
  t[8] = (uint32_t)acc;
  int64_t top = acc;
  acc = 0;
  for (int i = 0; i < 8; i++) {
    acc += (int64_t)t[i] + (int64_t)b.l[i] * g;
    t[i] = (uint32_t)acc;
    acc >>= 32;
  }
  top += acc;
  // top: the signed value of bits 256.. ; shift the 9-limb value right by 30
  uint32_t w8 = (uint32_t)top;
  for (int i = 0; i < 8; i++) r.l[i] = (t[i] >> 30) | ((i < 7 ? t[i + 1] : w8) << 2);
  bool neg = top < 0;
  if (neg) {
    uint64_t c = 1;
    for (int i = 0; i < 8; i++) {
      c += (uint32_t)~r.l[i];
      r.l[i] = (uint32_t)c;
      c >>= 32;
    }
  }
  return neg;
}

// (f u + g v) / 2^30 mod m for u, v in [0, m), |f|, |g| <= 2^30; result in [0, m)
template <class F> DEV fe mont_shift(const fe &u, const fe &v, int32_t f, int32_t g) {
  uint32_t t[8];
  int64_t acc = 0;
  uint32_t w[8];
  for (int i = 0; i < 8; i++) {
    acc += (int64_t)u.l[i] * f;
    w[i] = (uint32_t)acc;
    acc >>= 32;
  }
  int64_t top = acc;
  acc = 0;
  for (int i = 0; i < 8; i++) {
    acc += (int64_t)w[i] + (int64_t)v.l[i] * g;
    w[i] = (uint32_t)acc;
    acc >>= 32;
  }
  top += acc;
  // add q m with q = -t m^{-1} mod 2^30, making the low 30 bits zero
  uint32_t q = (w[0] * F::INV) & 0x3fffffffu;
  acc = 0;
  for (int i = 0; i < 8; i++) {
    acc += (int64_t)w[i] + (int64_t)q * F::M[i];
    t[i] = (uint32_t)acc;
    acc >>= 32;
  }
  top += acc;
  fe r;
  uint32_t w8 = (uint32_t)top;
  for (int i = 0; i < 8; i++) r.l[i] = (t[i] >> 30) | ((i < 7 ? t[i + 1] : w8) << 2);
  int64_t hi = top >> 30;   // the shifted value is r + hi 2^256, in (-2m, 3m)
  // normalise into [0, m): add m while negative, subtract m while >= m
  for (int k = 0; k < 2; k++) {
    if (hi < 0) {
      uint64_t c = 0;
      for (int i = 0; i < 8; i++) {
        c += (uint64_t)r.l[i] + F::M[i];
        r.l[i] = (uint32_t)c;
        c >>= 32;
      }
      hi += (int64_t)c;
    }
  }
  for (int k = 0; k < 2; k++) {
    uint32_t d[8];
    int64_t bw = 0;
    for (int i = 0; i < 8; i++) {
      int64_t x = (int64_t)r.l[i] - F::M[i] + bw;
      d[i] = (uint32_t)x;
      bw = x >> 32;
    }
    if (hi + bw >= 0) {
      for (int i = 0; i < 8; i++) r.l[i] = d[i];
      hi += bw;
    }
  }
  return r;
}

// With U, the values are known to be the same in every lane and are kept in scalar
// registers (readfirstlane is a no-op on them).
template <bool U> DEV uint32_t uni(uint32_t x) {
#ifdef __HIP_DEVICE_COMPILE__
  return U ? __builtin_amdgcn_readfirstlane(x) : x;
#else
  return x;
#endif
}
template <bool U> DEV void uni(fe &a) {
  for (int i = 0; i < 8; i++) a.l[i] = uni<U>(a.l[i]);
}

// x^{-1} mod m for 0 < x < m (x canonical, not in Montgomery form); false if the step
// budget ran out (never expected: 2 len(m) - 1 steps suffice for the exact algorithm)
template <class F, bool U = false> DEV bool inverse(const fe &x, fe &out, int *rounds = nullptr) {
  fe a = x, b = fe_const(F::M), u = fe_zero(), v = fe_zero();
  u.l[0] = 1;
  int it = 0;
  for (; it < 40; it++) {
    uni<U>(a); uni<U>(b); uni<U>(u); uni<U>(v);
    if (fe_is_zero(a)) break;
    int na = bitlen(a), nb = bitlen(b);
    int n = na > nb ? na : nb;
    uint64_t xa = approx(a, n), xb = approx(b, n);
    // |f|, |g| <= 2^j after j steps; the step is written without branches on 32-bit
    // halves so that a uniform input stays on the scalar unit
    uint32_t alo = uni<U>((uint32_t)xa), ahi = uni<U>((uint32_t)(xa >> 32));
    uint32_t blo = uni<U>((uint32_t)xb), bhi = uni<U>((uint32_t)(xb >> 32));
    int32_t f0 = 1, g0 = 0, f1 = 0, g1 = 1;
    for (int j = 0; j < 30; j++) {
      uint32_t odd = alo & 1u;
      uint32_t lt = (uint32_t)(ahi < bhi) | ((uint32_t)(ahi == bhi) & (uint32_t)(alo < blo));
      uint32_t sw = 0u - (odd & lt), od = 0u - odd;
      uint32_t t;
      t = (alo ^ blo) & sw; alo ^= t; blo ^= t;
      t = (ahi ^ bhi) & sw; ahi ^= t; bhi ^= t;
      int32_t ts;
      ts = (f0 ^ f1) & (int32_t)sw; f0 ^= ts; f1 ^= ts;
      ts = (g0 ^ g1) & (int32_t)sw; g0 ^= ts; g1 ^= ts;
      uint32_t sl = blo & od, sh = bhi & od;
      uint32_t nlo = alo - sl;
      ahi = ahi - sh - (uint32_t)(alo < sl);
      alo = nlo;
      f0 -= f1 & (int32_t)od;
      g0 -= g1 & (int32_t)od;
      alo = (alo >> 1) | (ahi << 31);
      ahi >>= 1;
      f1 *= 2;
      g1 *= 2;
    }
    fe a2, b2;
    if (lin_shift(a, b, f0, g0, a2)) { f0 = -f0; g0 = -g0; }
    if (lin_shift(a, b, f1, g1, b2)) { f1 = -f1; g1 = -g1; }
    fe u2 = mont_shift<F>(u, v, f0, g0), v2 = mont_shift<F>(u, v, f1, g1);
    a = a2; b = b2; u = u2; v = v2;
  }
  fe one = fe_zero();
  one.l[0] = 1;
  out = v;
  if (rounds) *rounds = it;
  return fe_is_zero(a) && fe_eq(b, one);
}

}  // namespace bingcd

// Montgomery-form inverse: (aR)^{-1} R^3 R^{-1} = a^{-1} R (R3 = R^3 mod m); 0 maps to 0
template <class F> NOINL fe f_inv_binary(const fe &A, const uint32_t *R3) {
  if (fe_is_zero(A)) return fe_zero();
  fe r;
  if (!bingcd::inverse<F>(A, r)) return f_inv<F>(A);
  return f_mul<F>(r, fe_const(R3));
}

#ifdef __HIPCC__
// the same for an input that is equal in every lane of the wavefront: the value is made
// explicitly uniform so that the computation runs on the scalar unit
template <class F> __device__ __forceinline__ fe f_inv_uniform(const fe &A, const uint32_t *R3) {
  fe a;
#pragma unroll
  for (int i = 0; i < 8; i++) a.l[i] = __builtin_amdgcn_readfirstlane(A.l[i]);
  if (fe_is_zero(a)) return fe_zero();
  fe r;
  if (!bingcd::inverse<F, true>(a, r)) return f_inv<F>(a);
  return f_mul<F>(r, fe_const(R3));
}
#endif
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
