// Exponentiation in the cyclotomic subgroup of F_p12 (G_T) on the wave-cooperative
// engine, with the 4-dimensional split of the exponent: G_T has order r and the p-power
// Frobenius acts on it as exponentiation by lam = p mod r, so with k = sum_j k_j lam^j
// (mod r), |k_j| < 2^65 (the decomposition used for G2), g^k = prod_j frob^j(g)^{k_j}.
// A negative k_j takes the conjugate (the inverse in the cyclotomic subgroup).  The 15
// products of subsets of the four bases form a table; then one cyclotomic squaring and
// at most one table product per bit of max |k_j|.  Control code shared by the device
// (DevCtx) and the host model (HostCtx).
#pragma once
#include "slp.hpp"
#include "gls.hpp"

namespace gtp {

// buffers of 12 slots at fb + 12 b: 0 the input, 1..15 the table, 16 and 17 the
// accumulator
static constexpr int NBUF = 18;

template <class Ctx> __host__ __device__ inline void copy12(Ctx &c, int dst, int src) {
  for (int i = c.lane(); i < 12; i += c.lanes()) c.S[dst + i] = c.S[src + i];
  c.sync();
}

// g^k for g (cyclotomic) in buffer 0 and k given by its decomposition; returns the buffer
// holding the result, or -1 when k = 0 (the result is 1)
template <class Ctx> __host__ __device__ inline int pow_cyc(Ctx &c, const gls::Dec &dec, int fb) {
  auto B = [fb](int b) { return fb + 12 * b; };
  if (dec.nbits == 0) return -1;
  const int frob[4] = {-1, slp::PROG_F12_FROB1, slp::PROG_F12_FROB2, slp::PROG_F12_FROB3};
  for (int j = 0; j < 4; j++) {
    int src = 0;
    if (j) {
      c.run(frob[j], B(0), B(0), B(16));
      src = 16;
    }
    if (dec.neg >> j & 1) c.run(slp::PROG_F12_CONJ, B(src), B(src), B(1 << j));
    else copy12(c, B(1 << j), B(src));
  }
  for (int d = 3; d < 16; d++) {
    int lo = d & -d;
    if (d != lo) c.run(slp::PROG_F12_MUL, B(d - lo), B(lo), B(d));
  }
  int t = (int)dec.nbits - 1;
  int acc = 16;
  copy12(c, B(acc), B((int)gls::digit(dec, (uint32_t)t)));
  for (t = t - 1; t >= 0; t--) {
    c.run(slp::PROG_F12_CSQR, B(acc), B(acc), B(33 - acc));
    acc = 33 - acc;
    uint32_t d = gls::digit(dec, (uint32_t)t);
    if (d) {
      c.run(slp::PROG_F12_MUL, B(acc), B((int)d), B(33 - acc));
      acc = 33 - acc;
    }
  }
  return acc;
}

}  // namespace gtp
