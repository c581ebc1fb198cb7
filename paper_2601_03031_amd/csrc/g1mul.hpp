// G1 scalar multiplication on the wave-cooperative engine: k P (+ A) with the GLV split
// k = k_0 + k_1 lam (glv.hpp), the signed bases B0 = sign(k_0) P and
// B1 = sign(k_1) phi(P), phi(x, y) = (beta x, y), the 15-entry table of d0 B0 + d1 B1
// (0 <= d0, d1 < 4) and one program of two doublings plus an addition per 2-bit window
// (two doublings alone for a zero window).  Additions that meet equal x-coordinates
// (H = 0) are resolved exactly: equal points are doubled, opposite points give the
// identity.  The control code is shared by the device (DevCtx) and the host model (HostCtx).
#pragma once
#include "slp.hpp"
#include "glv.hpp"
#include "g2mul.hpp"

namespace g1m {
using slp::f29;

template <class Ctx> __host__ __device__ inline void copy3(Ctx &c, int dst, int src) {
  for (int i = c.lane(); i < 3; i += c.lanes()) c.S[dst + i] = c.S[src + i];
  c.sync();
}

// T = (A, 1) from the affine slots at abase
template <class Ctx> __host__ __device__ inline void load_affine(Ctx &c, int abase, const f29 &one) {
  for (int i = c.lane(); i < 3; i += c.lanes()) c.S[slp::G1_T_0 + i] = i < 2 ? c.S[abase + i] : one;
  c.sync();
}

// H = 0 after an addition: returns true, with dbl set when the points were equal
template <class Ctx> __host__ __device__ inline bool add_degenerate(Ctx &c, bool &dbl) {
  bool h = g2m::zero29(c.S[slp::G1_H]);
  dbl = h && g2m::zero29(c.S[slp::G1_RR]);
  return h;
}

// T += A (affine, at abase); inf says whether T is the identity, and is updated
template <class Ctx> __host__ __device__ inline void add_affine(Ctx &c, bool &inf, int abase, const f29 &one) {
  if (inf) {
    load_affine(c, abase, one);
    inf = false;
    return;
  }
  c.run(slp::PROG_G1_MADD, 0, abase, 0);
  bool dbl;
  if (add_degenerate(c, dbl)) {
    c.sync();
    if (dbl) {
      load_affine(c, abase, one);
      c.run(slp::PROG_G1_DBL, 0, 0, 0);
    } else {
      inf = true;
    }
  }
}

// T += A (Jacobian, at abase; ainf when it is the identity); inf as in add_affine
template <class Ctx> __host__ __device__ inline void add_jac(Ctx &c, bool &inf, int abase, bool ainf) {
  if (ainf) return;
  if (inf) {
    copy3(c, slp::G1_T_0, abase);
    inf = false;
    return;
  }
  c.run(slp::PROG_G1_ADD, 0, abase, 0);
  bool dbl;
  if (add_degenerate(c, dbl)) {
    c.sync();
    if (dbl) {
      copy3(c, slp::G1_T_0, abase);
      c.run(slp::PROG_G1_DBL, 0, 0, 0);
    } else {
      inf = true;
    }
  }
}

// P (affine) must be in slots xP, yP and the constants loaded; A (affine) at abase when
// has_a.  Leaves k P + A in T (Jacobian) and returns true when the result is the identity.
template <class Ctx>
__host__ __device__ inline bool mul_add(Ctx &c, const glv::Dec &dec, bool pinf, bool has_a, int abase, const f29 &one) {
  f29 *S = c.S;
  bool inf = pinf || dec.nbits == 0;
  if (!inf) {
    c.run(slp::PROG_G1_PHI, 0, 0, 0);
    if (c.lane() == 0) {
      f29 y = S[slp::G1_yP];
      S[slp::G1_B1_y] = (dec.neg & 2) ? g2m::neg29(y) : y;
      S[slp::G1_yP] = (dec.neg & 1) ? g2m::neg29(y) : y;
    }
    c.sync();
    c.run(slp::PROG_G1_TABLE, 0, 0, 0);
    int w = (int)(dec.nbits + 1) / 2 - 1;
    copy3(c, slp::G1_T_0, slp::G1_TB1_0 + 3 * ((int)glv::digit2(dec, (uint32_t)w) - 1));
    for (w = w - 1; w >= 0; w--) {
      uint32_t d = glv::digit2(dec, (uint32_t)w);
      if (!d) {
        if (!inf) c.run(slp::PROG_G1_DBL2, 0, 0, 0);
        continue;
      }
      int tb = slp::G1_TB1_0 + 3 * ((int)d - 1);
      if (inf) {
        copy3(c, slp::G1_T_0, tb);
        inf = false;
        continue;
      }
      c.run(slp::PROG_G1_DBL2_ADD, 0, tb, 0);
      bool dbl;
      if (add_degenerate(c, dbl)) {
        c.sync();
        if (dbl) {
          copy3(c, slp::G1_T_0, tb);
          c.run(slp::PROG_G1_DBL, 0, 0, 0);
        } else {
          inf = true;
        }
      }
    }
  }
  if (has_a) add_affine(c, inf, abase, one);
  return inf;
}

}  // namespace g1m
