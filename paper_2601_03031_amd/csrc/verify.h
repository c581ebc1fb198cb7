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
  uint32_t t, lK, lM, L, nmul;  // nmul: stride of the multiplication jobs (>= t + 2 lK + 4)
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
  fp12 *gtb, *gtp, *gto;  // G_T exponentiation bases, powers, and the product's inputs (powers + C last)
  // assembled
  g1_aff *Cg1, *bA, *pp;
  g2_aff *pq;
  fp12 *F, *E;         // Miller values, final exponentiations
  const g1_aff *g1beta;
  const g2_aff *vk;
  int *flags;
  // sub-array proofs (block and FC proof only): the Step 2 items are left out (points at
  // infinity, zero scalars, so their pairing checks hold trivially) and the block's entry j
  // must equal cj_expect, the commitment recomputed from the sub-array
  int fc_only;
  const g1_aff *cj_expect;
};

// Layout of the N serialized proofs in index order: proofs of batch k (entries i with
// i / (b M) = k) hold t_k = min(b, K - k b) block commitments and are len(t_k) bytes long; the
// last batch alone can be shorter.
struct PLayout {
  uint32_t L, lK, lM, b, t_last;
  uint64_t N, K, M, nb, len_full, len_last;
};

// Serialization of every proof of an open-all bundle (kps_serialize)
struct PSCtx {
  PLayout y;
  const g1_aff *Cj, *Lg1, *Rg1, *Al, *D, *W;
  const fp12 *Lgt, *Rgt;
  const g2_aff *vl, *piv;
  const fe *Y;
  const uint32_t *tree;
  uint8_t *out;
};

// Verification of all N proofs at once (kva_*): shared items are decoded once, from the proof
// that represents them, and the PST checks of all proofs combine with random weights
struct VACtx {
  PLayout y;
  const uint8_t *proofs, *m, *Cb, *seed;
  g1_aff *Cj, *Dn, *Wn;  // K block commitments, 2K - 2 D-tree siblings (heap order), M - 1 W (heap order)
  fp12 *C;
  uint32_t *root;        // N x 8 words: root of each proof's Merkle path
  fe *rho, *delta, *dy;  // K; N weights; N weighted y*
  uint8_t *odd;          // N: proof differs from the representatives it shares items with
  uint64_t *oddlist;
  uint32_t *oddcnt;
  fe *rowsum, *colsum, *sy;
  g1_aff *bases, *prod, *pp;
  fe *scal;
  g2_aff *pq;
  fp12 *E;
  const g2_aff *vk;
  int *flags;
};

// Verification of an evaluation proof at a point (kve_*): proof C_F || rounds || A_l v_l pi_v
// || y || W; point r_0 .. r_{L-1} (32 bytes little-endian each)
struct VECtx {
  uint32_t L, lK, lM;
  uint64_t K, M;
  const uint8_t *proof, *Cb, *rle;
  g1_aff *CF, *Lg1, *Rg1, *Al, *W;
  fp12 *Lgt, *Rgt, *C;
  g2_aff *vl, *piv;
  fe *r, *y, *T, *x, *xinv;
  fe *ms;            // G1 jobs: x_j Lg1_j, x_j^{-1} Rg1_j (2 lK), b_l A_l, r_0 C_F, y g1, z g1
  g1_aff *mb, *mo;
  fe *g2s;           // G2 jobs: f_v(z) g2, then r_{lM-1-d} g2 (d < lM)
  g2_aff *g2o;
  fe *gts;
  fp12 *gtb, *gtp, *gto;
  g1_aff *pp, *Cg1, *bA;
  g2_aff *pq;
  const g1_aff *g1beta;
  const g2_aff *vk;
  int *flags;
};

namespace kve {
void decode(const VECtx &c, hipStream_t st);
void transcript(const VECtx &c, hipStream_t st);
void assemble(const VECtx &c, hipStream_t st);
}  // namespace kve

namespace ksa {
void check(const uint8_t *proofs, uint64_t K, uint32_t b, uint64_t nb, uint64_t len_full, uint64_t len_last,
           const g1_aff *Cre, uint64_t *oddlist, uint32_t *oddcnt, int *flags, hipStream_t st);
}  // namespace ksa

namespace kva {
uint64_t nterms(const VACtx &c);
void serialize(const PSCtx &c, hipStream_t st);
void decode(const VACtx &c, hipStream_t st);
void roots(const VACtx &c, hipStream_t st);
void rho(const VACtx &c, hipStream_t st);
void same(const VACtx &c, hipStream_t st);
void proof(const VACtx &c, hipStream_t st);
void sums(const VACtx &c, hipStream_t st);
void terms(const VACtx &c, hipStream_t st);
void segsum(const VACtx &c, hipStream_t st);
void check(const VACtx &c, hipStream_t st);
}  // namespace kva

// kernels over n proofs at once, cs: device array of n contexts (tmax: largest t)
namespace kv {
void decode(const VCtx *cs, uint32_t n, uint32_t tmax, uint32_t lK, uint32_t lM, hipStream_t st);
void transcript(const VCtx *cs, uint32_t n, hipStream_t st);
void assemble(const VCtx *cs, uint32_t n, hipStream_t st);
void compare(const VCtx *cs, uint32_t n, hipStream_t st);
void fe_gather(const fp12 *F, uint64_t npair, uint32_t n, fp12 *G, hipStream_t st);
}  // namespace kv
