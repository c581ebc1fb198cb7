// Device context of VC.Verify for one proof (k_verify.hip) and its launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "field.hpp"
#include "tower.hpp"
#include "curve.hpp"

#define VFLAG_BAD_INPUT 1  // commitment or m_i malformed: the call returns VC_EINVAL
#define VFLAG_BAD_PROOF 2  // a proof element does not decode: reject
#define VFLAG_ACCEPT 4

struct VCtx {
  uint32_t t, lK, lM, L;
  uint64_t N, i, j, a, lo;
  const uint8_t *proof, *Cb, *mib, *mpath;
  // decoded proof and inputs
  g1_aff *blk, *Lg1, *Rg1, *Al, *Dsib, *Wp;
  fp12 *Lgt, *Rgt, *C;
  g2_aff *vl, *piv;
  fe *ysib, *mi;
  // transcript values and jobs
  fe *r, *x, *xinv, *ms, *fz, *gts;
  g1_aff *mb, *mo;     // G1 multiplication bases and results
  g2_aff *fzg2;        // f_v(z) g2
  fp12 *gtb, *gto;     // G_T exponentiation bases and results (+ C last)
  // assembled
  g1_aff *Cg1, *bA, *pp;
  g2_aff *pq;
  fp12 *F, *E;         // Miller values, final exponentiations
  const g1_aff *g1beta;
  const g2_aff *vk;
  int *flags;
};

namespace kv {
void decode(const VCtx &c, hipStream_t st);
void transcript(const VCtx &c, hipStream_t st);
void assemble(const VCtx &c, hipStream_t st);
void compare(const VCtx &c, hipStream_t st);
}  // namespace kv
