// G2 scalar multiplication on the wave-cooperative engine: k Q (+ A) with the GLS split
// k = sum_j k_j lam^j, the signed bases B_j = sign(k_j) psi^j(Q), a table of the 15
// subset sums, and one doubling plus at most one table addition per bit of max |k_j|
// (65 bits).  Additions that meet equal x-coordinates (H = 0) are resolved exactly:
// equal points are doubled, opposite points give the identity.  The control code is
// shared by the device (DevCtx, all lanes of the workgroup) and the host model (HostCtx).
#pragma once
#include "slp.hpp"
#include "gls.hpp"

namespace g2m {
using slp::f29;

__host__ __device__ inline bool zero29(const f29 &x) {
  f29 c = slp::canon29(x);
  uint32_t t = 0;
  for (int j = 0; j < 9; j++) t |= c.l[j];
  return t == 0;
}

// p - x for an almost-reduced x (result in (0, p])
__host__ __device__ inline f29 neg29(const f29 &x) {
  f29 c = slp::canon29(x), o;
  int64_t bw = 0;
  for (int j = 0; j < 9; j++) {
    int64_t v = (int64_t)slp::P29[j] - c.l[j] + bw;
    o.l[j] = (uint32_t)v & SLP_M29;
    bw = v >> 29;
  }
  o.l[9] = o.l[10] = o.l[11] = 0;
  return o;
}

template <class Ctx> __host__ __device__ inline void copy_slots(Ctx &c, int dst, int src, int n) {
  for (int i = c.lane(); i < n; i += c.lanes()) c.S[dst + i] = c.S[src + i];
  c.sync();
}

// T = (A, 1) from the affine slots at abase
template <class Ctx> __host__ __device__ inline void load_affine(Ctx &c, int abase, const f29 &one, const f29 &zero) {
  for (int i = c.lane(); i < 6; i += c.lanes()) c.S[slp::G2_T_0 + i] = i < 4 ? c.S[abase + i] : (i == 4 ? one : zero);
  c.sync();
}

template <class Ctx> __host__ __device__ inline bool add_degenerate(Ctx &c, bool &doubling) {
  const f29 *S = c.S;
  bool h = zero29(S[slp::G2_H_0]) && zero29(S[slp::G2_H_1]);
  doubling = h && zero29(S[slp::G2_RR_0]) && zero29(S[slp::G2_RR_1]);
  return h;
}

// T += A (affine, at abase); inf says whether T is the identity, and is updated
template <class Ctx>
__host__ __device__ inline void add_affine(Ctx &c, bool &inf, int abase, const f29 &one, const f29 &zero) {
  if (inf) {
    load_affine(c, abase, one, zero);
    inf = false;
    return;
  }
  c.run(slp::PROG_G2_MADD, 0, abase, 0);
  bool dbl;
  if (add_degenerate(c, dbl)) {
    c.sync();
    if (dbl) {
      load_affine(c, abase, one, zero);
      c.run(slp::PROG_G2_DBL, 0, 0, 0);
    } else {
      inf = true;
    }
  }
}

// T += A (Jacobian, at abase; ainf when it is the identity); inf as in add_affine
template <class Ctx> __host__ __device__ inline void add_jac(Ctx &c, bool &inf, int abase, bool ainf) {
  if (ainf) return;
  if (inf) {
    copy_slots(c, slp::G2_T_0, abase, 6);
    inf = false;
    return;
  }
  c.run(slp::PROG_G2_ADD, 0, abase, 0);
  bool dbl;
  if (add_degenerate(c, dbl)) {
    c.sync();
    if (dbl) {
      copy_slots(c, slp::G2_T_0, abase, 6);
      c.run(slp::PROG_G2_DBL, 0, 0, 0);
    } else {
      inf = true;
    }
  }
}

// Q (affine) must be in slots xQ, yQ and the constants loaded; A (affine) at abase when
// has_a.  Leaves k Q + A in T (Jacobian) and returns true when the result is the identity.
template <class Ctx>
__host__ __device__ inline bool mul_add(Ctx &c, const gls::Dec &dec, bool qinf, bool has_a, int abase, const f29 &one,
                                        const f29 &zero) {
  f29 *S = c.S;
  bool inf = qinf || dec.nbits == 0;
  if (!inf) {
    c.run(slp::PROG_G2_PSI, 0, 0, 0);
    const int yslot[4] = {slp::G2_yQ_0, slp::G2_B1_y_0, slp::G2_B2_y_0, slp::G2_B3_y_0};
    for (int i = c.lane(); i < 8; i += c.lanes()) {
      int j = i >> 1;
      if (dec.neg >> j & 1) S[yslot[j] + (i & 1)] = neg29(S[yslot[j] + (i & 1)]);
    }
    c.sync();
    c.run(slp::PROG_G2_TABLE, 0, 0, 0);
    int t = (int)dec.nbits - 1;
    copy_slots(c, slp::G2_T_0, slp::G2_TB1_0 + 6 * ((int)gls::digit(dec, (uint32_t)t) - 1), 6);
    for (t = t - 1; t >= 0; t--) {
      if (!inf) c.run(slp::PROG_G2_DBL, 0, 0, 0);
      uint32_t d = gls::digit(dec, (uint32_t)t);
      if (!d) continue;
      int tb = slp::G2_TB1_0 + 6 * ((int)d - 1);
      if (inf) {
        copy_slots(c, slp::G2_T_0, tb, 6);
        inf = false;
        continue;
      }
      c.run(slp::PROG_G2_ADD, 0, tb, 0);
      bool dbl;
      if (add_degenerate(c, dbl)) {
        c.sync();
        if (dbl) {
          copy_slots(c, slp::G2_T_0, tb, 6);
          c.run(slp::PROG_G2_DBL, 0, 0, 0);
        } else {
          inf = true;
        }
      }
    }
  }
  if (has_a) add_affine(c, inf, abase, one, zero);
  return inf;
}

}  // namespace g2m
