// Wide prime-field arithmetic: one field element spread over an aligned group of 8
// lanes, lane g = (lane & 7) holding 32-bit limb g (little-endian), Montgomery form
// with R = 2^256, fully reduced.  Selected by defining VC_WIDE before field.hpp; the
// tower, curve and pairing headers then run unchanged with every base-field
// operation shared by 8 lanes, which cuts the latency of a dependent chain of field
// operations about 5x compared with one lane per element.
//
// Cross-lane steps: limb broadcasts with ds_swizzle (and-mask 0x18 keeps the group),
// one-limb shifts with DPP row shifts, and carry/borrow propagation with wave
// ballots: with G = generate and P = propagate masks (bit 7 of every group cleared so
// chains never cross groups), the carry into each limb is ((G|P) + G) ^ (G|P) ^ G.
// All 8 lanes of a group must be active together (ballots see only active lanes).
#pragma once

struct fe {
  uint32_t v;
};

#define COUNT_FMUL()

__device__ __forceinline__ int wlane() { return (int)__lane_id(); }
__device__ __forceinline__ int wg() { return wlane() & 7; }

// limb c[g] of a constant
__device__ __forceinline__ uint32_t lane_pick(const uint32_t *c) {
  int g = wg();
  uint32_t v = c[0];
#pragma unroll
  for (int k = 1; k < 8; k++) v = (g == k) ? c[k] : v;
  return v;
}

template <int K> __device__ __forceinline__ uint32_t wbcast(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x18 | (K << 5));
}
__device__ __forceinline__ uint32_t wbcast_dyn(uint32_t x, int k) { return (uint32_t)__shfl((int)x, (wlane() & ~7) | k); }

// lane g receives lane g+1 (0 for g = 7), lane g receives lane g-1 (0 for g = 0)
__device__ __forceinline__ uint32_t wshdn(uint32_t x) {
  uint32_t v = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x101, 0xF, 0xF, true);
  return wg() == 7 ? 0u : v;
}
__device__ __forceinline__ uint32_t wshup(uint32_t x) {
  uint32_t v = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);
  return wg() == 0 ? 0u : v;
}

__device__ __forceinline__ uint32_t group_bits(uint64_t mask) { return (uint32_t)(mask >> (wlane() & ~7)) & 0xFFu; }

// carry-lookahead over the group's limbs: returns the carry into this limb, and
// whether the top limb carries out
__device__ __forceinline__ uint32_t wchain(bool gen, bool prop, bool &out) {
  uint64_t G = __ballot(gen), P = __ballot(prop);
  const uint64_t M7 = 0x7f7f7f7f7f7f7f7full;
  uint64_t g = G & M7, p = P & M7;
  uint64_t a = g | p;
  uint64_t C = (a + g) ^ a ^ g;
  int ln = wlane(), top = (ln & ~7) + 7;
  uint32_t c7 = (uint32_t)(C >> top) & 1u, g7 = (uint32_t)(G >> top) & 1u, p7 = (uint32_t)(P >> top) & 1u;
  out = (g7 | (p7 & c7)) != 0;
  return (uint32_t)(C >> ln) & 1u;
}

__device__ __forceinline__ fe fe_zero() { return {0u}; }
__device__ __forceinline__ fe fe_const(const uint32_t *c) { return {lane_pick(c)}; }
template <class F> __device__ __forceinline__ fe f_one() { return fe_const(F::ONE); }
__device__ __forceinline__ bool fe_is_zero(const fe &a) { return group_bits(__ballot(a.v != 0u)) == 0u; }
__device__ __forceinline__ bool fe_eq(const fe &a, const fe &b) { return group_bits(__ballot(a.v != b.v)) == 0u; }

// canonical limb i of a (broadcast to the group), and an element from 8 limbs
__device__ __forceinline__ uint32_t fe_word(const fe &a, int i) { return wbcast_dyn(a.v, i); }
__device__ __forceinline__ fe fe_from_words(const uint32_t *w) { return {lane_pick(w)}; }

// s - m if s >= m
template <class F> __device__ __forceinline__ uint32_t w_reduce(uint32_t s) {
  uint32_t mg = lane_pick(F::M);
  bool bout;
  uint32_t bin = wchain(s < mg, s == mg, bout);
  uint32_t d = s - mg - bin;
  return bout ? s : d;
}

template <class F> __device__ __forceinline__ fe f_add(const fe &a, const fe &b) {
  uint64_t s = (uint64_t)a.v + b.v;
  uint32_t lo = (uint32_t)s;
  bool out;
  uint32_t cin = wchain((s >> 32) != 0, lo == 0xFFFFFFFFu, out);
  return {w_reduce<F>(lo + cin)};
}

template <class F> __device__ __forceinline__ fe f_sub(const fe &a, const fe &b) {
  bool bout;
  uint32_t bin = wchain(a.v < b.v, a.v == b.v, bout);
  uint32_t d = a.v - b.v - bin;
  uint32_t mg = bout ? lane_pick(F::M) : 0u;
  uint64_t s = (uint64_t)d + mg;
  uint32_t lo = (uint32_t)s;
  bool out;
  uint32_t cin = wchain((s >> 32) != 0, lo == 0xFFFFFFFFu, out);
  return {lo + cin};
}

template <class F> __device__ __forceinline__ fe f_neg(const fe &a) { return f_sub<F>(fe_zero(), a); }
template <class F> __device__ __forceinline__ fe f_dbl(const fe &a) { return f_add<F>(a, a); }

template <class F> __device__ __forceinline__ fe f_half(const fe &a) {
  uint32_t odd = wbcast<0>(a.v) & 1u;
  uint32_t mg = odd ? lane_pick(F::M) : 0u;
  uint64_t s = (uint64_t)a.v + mg;
  uint32_t lo = (uint32_t)s;
  bool out;
  uint32_t cin = wchain((s >> 32) != 0, lo == 0xFFFFFFFFu, out);
  lo += cin;
  return {(lo >> 1) | (wshdn(lo) << 31)};
}

// Montgomery product: word-serial over b's limbs; lane g keeps limb g of the running
// value and a pending carry c (weight of limb g+1).  Each step adds a b_j and m p,
// m = (limb 0) * (-p^{-1}) mod 2^32, and shifts down one limb.
template <class F> __device__ __forceinline__ fe f_mul(const fe &a, const fe &b) {
  uint32_t mg = lane_pick(F::M);
  uint32_t bj[8];
  bj[0] = wbcast<0>(b.v); bj[1] = wbcast<1>(b.v); bj[2] = wbcast<2>(b.v); bj[3] = wbcast<3>(b.v);
  bj[4] = wbcast<4>(b.v); bj[5] = wbcast<5>(b.v); bj[6] = wbcast<6>(b.v); bj[7] = wbcast<7>(b.v);
  uint32_t t = 0, c = 0;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    uint64_t X = (uint64_t)a.v * bj[j] + t;
    uint32_t m = wbcast<0>((uint32_t)X) * F::INV;
    uint64_t Y = (uint64_t)m * mg + (uint32_t)X;
    uint64_t s = (uint64_t)wshdn((uint32_t)Y) + (X >> 32) + (Y >> 32) + c;
    t = (uint32_t)s;
    c = (uint32_t)(s >> 32);
  }
  uint64_t f = (uint64_t)t + wshup(c);
  uint32_t lo = (uint32_t)f;
  bool out;
  uint32_t cin = wchain((f >> 32) != 0, lo == 0xFFFFFFFFu, out);
  return {w_reduce<F>(lo + cin)};
}

template <class F> __device__ __forceinline__ fe f_sqr(const fe &a) { return f_mul<F>(a, a); }

template <class F> __device__ __forceinline__ fe f_mul_small(const fe &a, int k) {
  fe acc = fe_zero(), base = a;
  while (k) {
    if (k & 1) acc = f_add<F>(acc, base);
    base = f_dbl<F>(base);
    k >>= 1;
  }
  return acc;
}

template <class F> __device__ __forceinline__ fe f_to_mont(const fe &a) { return f_mul<F>(a, fe_const(F::R2)); }
template <class F> __device__ __forceinline__ fe f_from_mont(const fe &a) {
  fe one = {wg() == 0 ? 1u : 0u};
  return f_mul<F>(a, one);
}

template <class F> __device__ __attribute__((noinline)) fe f_pow(const fe &a, const uint32_t *e) {
  fe acc = f_one<F>();
  for (int i = 255; i >= 0; i--) {
    acc = f_sqr<F>(acc);
    if ((e[i >> 5] >> (i & 31)) & 1) acc = f_mul<F>(acc, a);
  }
  return acc;
}

template <class F> __device__ __attribute__((noinline)) fe f_inv(const fe &a) { return f_pow<F>(a, F::MINUS2); }
// the binary-GCD inverse of the one-lane layout is replaced by Fermat's inverse here
template <class F> __device__ __forceinline__ fe f_inv_binary(const fe &A, const uint32_t *) { return f_inv<F>(A); }
