// Host-side declarations of the kernel launchers (k_g1.hip, k_hash.hip, k_verify.hip: one
// lane per element; k_wide.hip: eight lanes per element; k_slp.hip: the engine).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "field.hpp"
#include "tower.hpp"
#include "curve.hpp"

// Counters per segment for the one-launch reduction trees (at least the nodes of all levels
// above the first).
__host__ __device__ inline uint64_t tree_counters(uint64_t len) { return len + 64; }

#define VC_ERRBIT_RANGE 1
#define VC_ERRBIT_CHALLENGE 2

// Step 2 (Protocol 1 Step 2) of one job of a group: its entries, aux row and commitment, and
// the arrays of its proof bundle that Step 2 writes.  The Step 2 kernels take a table of G of
// these and a thread range per job (job x's threads follow job x - 1's), so one launch does the
// same step for every job of the group.  (In the wide-layout kernels fe is one limb per lane,
// so they reach these arrays through element offsets of wld/wst, never pointer arithmetic.)
struct S2Job {
  const fe *m;       // N entries (as kept by the commitment)
  const g1_aff *Cj;  // K subvector commitments
  const fp12 *C;     // the commitment
  uint32_t *tree;    // Merkle heap, 2N digests
  fe *rho, *Y;       // K challenges; the y-tree, (2K - 1) M canonical F_r
  g1_aff *D, *W;     // the D-tree, 2K - 1 points; HyperEval commitments, M - 1 points
};

// One job of a batched commit (VC.Commit of many vectors at once): its entries, keys, MSM
// schedule and outputs.  Jobs follow one another in the MSM's block range (blk0: job x has
// blocks blk0 .. + K nslice) and in the packed per-subvector arrays (k0: entries k0 .. + K).
struct CJob {
  const fe *m;          // N canonical entries
  const g1_aff *table;  // fixed-base table 2^{8 w} ek_{lM}[a] of the job's params
  const g2_aff *h;      // h of the job's params (v_j = h_{2j})
  g1_jac *part;         // K nslice partial sums of the MSM blocks
  g1_aff *Cj;           // the commitment's C_j
  fp12 *C;              // the commitment's C
  uint64_t M, K, nslice, blk0, k0;
  uint32_t nwin, S;     // 8-bit windows per entry, entries per MSM block
};

namespace kl {
void trapdoor(const uint8_t *seed, uint32_t lM, fe *s, fe *beta, hipStream_t st);
void ek_weights(uint32_t lM, const fe *s, fe *w, uint64_t n, hipStream_t st);
void pow_table(const fe *beta, fe *out, uint64_t n, hipStream_t st);
void msm_tables(const g1_aff *base, uint64_t M, uint32_t nwin, g1_aff *table, hipStream_t st);
void lift_u32(const uint32_t *in, uint64_t n, fe *out, hipStream_t st);
void check_fr(const fe *m, uint64_t n, int *err, hipStream_t st);
void zero_u32(uint32_t *p, uint64_t n, hipStream_t st);
// batched commit: every job's MSM blocks in one persistent launch of `grid` workgroups
// (msm_batch_grid: as many as stay resident), v_j of every job packed, Miller values padded
// with ones to Kmax per job, each C stored into its commitment
void msm_batch(const CJob *J, uint32_t n, uint64_t total, unsigned grid, hipStream_t st);
int msm_batch_grid(int device);
void commit_v(const CJob *J, uint32_t n, uint64_t total, g2_aff *v, hipStream_t st);
void commit_pad(const CJob *J, uint32_t n, uint64_t Kmax, const fp12 *Fc, fp12 *F, hipStream_t st);
void commit_store(const CJob *J, uint32_t n, const fp12 *Cs, hipStream_t st);
// canonical big-endian F_p encodings (32 B each) -> Montgomery form; >= p sets VC_ERRBIT_RANGE
void decode_fp(const uint8_t *in, uint64_t n, fe *out, int *err, hipStream_t st);
// points not on their curve set VC_ERRBIT_RANGE
void check_curve_g1(const g1_aff *p, uint64_t n, int *err, hipStream_t st);
void check_curve_g2(const g2_aff *p, uint64_t n, int *err, hipStream_t st);
// multiply-add throughput probe: blocks x 256 lanes, 8 iters multiply-adds each
void diag_mad(uint32_t seed, uint32_t iters, unsigned blocks, uint64_t *out, hipStream_t st);
void msm_slices(const fe *scal, uint64_t K, uint64_t M, uint32_t nwin, uint32_t S, const g1_aff *table, g1_jac *partial,
                hipStream_t st);
// the same over G2 (S nwin <= 1024), for the KZG proof over the fixed SRS points h_m
void msm_slices_g2(const fe *scal, uint64_t K, uint64_t M, uint32_t nwin, uint32_t S, const g2_aff *table, g2_jac *partial,
                   hipStream_t st);
void msm_tables_g2(const g2_aff *base, uint64_t M, uint32_t nwin, g2_aff *table, hipStream_t st);
// out[i] = canonical value of the Montgomery-form F_r element in[i]
void fr_canon(const fe *in, uint64_t n, fe *out, hipStream_t st);
// input s at in[s*stride]; output to (s odd ? out1 : out0)[(s >> 1) * ostride]
// one launch; cnt: nseg tree_counters(len) zeroed counters, zero again on return
void g1_reduce(g1_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st);
void g1_to_aff(const g1_jac *in, uint64_t stride, uint64_t n, g1_aff *out, uint64_t ostride, hipStream_t st);
void g2_to_aff(const g2_jac *in, uint64_t stride, uint64_t n, g2_aff *out, uint64_t ostride, hipStream_t st);
// Step 1's batches are job-major: batch x nbj + k is batch k of job x (nbj = ceil(K / b)
// batches per job; one job: nbj = nb).  Job x's aux row is Cj + x K, its commitment C[x].
void oa_init(const g1_aff *Cj, const g2_aff *h, uint64_t K, uint64_t nb, uint64_t nbj, g1_aff *A, g2_aff *V, fe *B,
             hipStream_t st);
// L[k lK] = L[0], R[k lK] = R[0] for batches k = 1 .. nb - 1 (round 1's G_T parts)
// L[k lK] = LT[k / nbj], R[k lK] = RT[k / nbj] for every batch k (round 1's G_T parts of each job)
void bcast_round1(const fp12 *LT, const fp12 *RT, uint64_t nb, uint64_t nbj, uint32_t lK, fp12 *L, fp12 *R,
                  hipStream_t st);
void fc_chunks(const g1_aff *Cj, uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, uint32_t *Hq, hipStream_t st);
void fc_sigma(const fp12 *C, uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, const uint32_t *Hq, uint32_t *sigma,
              hipStream_t st);
void fc_r(uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, const uint32_t *sigma, fe *B, hipStream_t st);
void oa_lr_aff(const g1_jac *S, uint64_t K, uint64_t nb, uint32_t j, uint32_t lK, g1_aff *Lg1, g1_aff *Rg1, hipStream_t st);
// x_j = H'(x_{j-1} || L_j || R_j) per batch (zero_round == j: batch 0's challenge is forced to
// zero, a test hook for the zero-challenge error; 0 leaves every challenge as hashed)
void oa_transcript(const fp12 *Lgt, const fp12 *Rgt, uint64_t nb, uint32_t j, uint32_t lK, const g1_aff *Lg1,
                   const g1_aff *Rg1, fe *X, fe *Xinv, int *err, uint32_t zero_round, hipStream_t st);
// L[k lK], R[k lK] = U[2k + side] + sum_{g, p} P[4 (4k + g) + p] over the 8 split parts of
// each side (affine)
// gws: 4 (2K - 1) elements per batch of global working space, used when K > 1024
void kzg_quotient(const fe *Xinv, const fe *X, const g2_aff *V, uint64_t K, uint64_t nb, uint32_t lK, fe *Q, fe *z,
                  fe *gws, hipStream_t st);
void merkle_leaves(const S2Job *J, uint32_t G, uint64_t M, uint64_t N, hipStream_t st);
void merkle_level(const S2Job *J, uint32_t G, uint64_t start, hipStream_t st);
void rho(const S2Job *J, uint32_t G, uint64_t K, hipStream_t st);
void glv_dec(const fe *X, uint64_t nb, uint32_t j, uint32_t lK, glv::Dec *out, hipStream_t st);
// the whole y-tree (level 0 from the entries, levels 1 .. lK) in passes of up to four levels
void ytree(const S2Job *J, uint32_t G, uint64_t M, uint64_t K, uint32_t lK, hipStream_t st);
void encode(const fe *in, uint64_t n, int mode, uint8_t *out, hipStream_t st);
void gather_encode(const fe *base, const uint64_t *idx, const int *mode, uint64_t n, uint8_t *out, hipStream_t st);
// evaluation proof at a point (k_hash.hip)
void ev_point(const uint8_t *rle, uint32_t L, fe *r, int *err, hipStream_t st);
void ev_eq(const fe *r, uint32_t lM, uint32_t lK, uint64_t K, fe *T, hipStream_t st);
void ev_sum(const g1_aff *P, uint64_t n, g1_aff *out, hipStream_t st);
void ev_r0(const fp12 *C, const fe *r, uint32_t L, const g1_aff *CF, const fe *T, uint64_t K, fe *B, hipStream_t st);
void ev_table(const fe *m, const fe *T, uint64_t K, uint64_t M, fe *g, hipStream_t st);
void ev_pst_step(fe *g, uint64_t half, const fe *rvar, fe *q, hipStream_t st);
void ev_finish(const g1_aff *prod, uint32_t lM, const fe *g, g1_aff *W, fe *y, hipStream_t st);
}  // namespace kl

// Wide-layout kernels (k_wide.hip, 8 lanes per field element); same memory layouts
// as above, passed untyped because the register types differ in that unit.
namespace klw {
void g1_mul(const void *P, int bc, const void *k, uint64_t n, void *out, hipStream_t st);
void g2_mul(const void *P, int bc, const void *k, uint64_t n, void *out, hipStream_t st);
void oa_g1terms(const void *A, const void *B, uint64_t K, uint64_t nb, uint64_t h, void *S, hipStream_t st);
void oa_fold_g1(const void *Ain, const void *Bin, void *Aout, void *Bout, const void *Xinv, const void *dec, uint64_t K,
                uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st);
// the direct rounds' Miller values, several pairs per product: returns the products per batch
// and side (stride K/2), the length of the F_p12 tree that follows
uint64_t oa_miller(const void *A, const void *V, uint64_t K, uint64_t nb, uint64_t h, void *F, hipStream_t st);
void oa_fold_g2(const void *Vin, void *Vout, const void *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j,
                uint32_t lK, hipStream_t st);
// HyperEval terms of every job's g* (the root row of its y-tree): level d of job x at
// S + (d G + x) M / 2, so the M / 2 terms of a level of all jobs are contiguous
void hyper_terms(const S2Job *J, uint32_t G, uint64_t K, const void *ek, uint64_t M, uint32_t lM, void *S, hipStream_t st);
// W of every job at level d from the reduced segment sums (segment x 2^d + p at in + (x 2^d + p) stride)
void w_aff(const S2Job *J, uint32_t G, const void *in, uint64_t stride, uint32_t d, hipStream_t st);
// D_j = rho_j C_j, the D-tree's leaves of every job
void d_leaves(const S2Job *J, uint32_t G, uint64_t K, hipStream_t st);
void g1_reduce(void *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st);
void g1_to_aff(const void *in, uint64_t stride, uint64_t n, void *out, uint64_t ostride, hipStream_t st);
void sum_g1(const void *data, uint64_t nseg, uint64_t len, void *out, hipStream_t st);
// batched commit: C_j of every job (into its commitment and packed at Cp + k0 + j)
void commit_sums(const CJob *J, uint32_t n, uint64_t total, void *Cp, hipStream_t st);
void dlevel(const S2Job *J, uint32_t G, uint64_t K, uint32_t h, hipStream_t st);
void diag_field(int which, int op, const void *a, const void *b, uint64_t n, void *out, hipStream_t st);
}  // namespace klw

// wave-cooperative engine (k_slp.hip): a 64-lane workgroup per pairing / product / element
namespace ks {
void miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n, fp12 *out, hipStream_t st);
void oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h, fp12 *F, hipStream_t st);
// one launch; cnt: nseg tree_counters(len) zeroed counters, zero again on return
void f12_reduce(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st);
// input s at in[s stride]; output to (s odd ? out1 : out0)[(s >> 1) ostride], or to
// out0[s ostride] when out1 is NULL
void final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out0, fp12 *out1, uint64_t ostride, hipStream_t st);
void oa_fold_g2(const g2_aff *Vin, g2_aff *Vout, const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK,
                hipStream_t st);
// sums of Jacobian segments on the engine, one launch (tree_counters(len) counters per segment)
void g1_tree(g1_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st);
void g2_tree(g2_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st);
// round-1 G1 terms on the engine (same layout as klw::oa_g1terms)
void oa_g1terms(const g1_aff *A, const fe *B, uint64_t K, uint64_t nb, uint64_t h, g1_jac *S, hipStream_t st);
void gt_pow(const fp12 *in, const fe *k, uint64_t n, fp12 *out, hipStream_t st);
// fused round kernels: G1 + G2 fold; Miller loops + G1 terms of the next round (oa_terms.hpp);
// final exponentiations of two strided lists
void oa_fold(const g1_aff *Ain, const fe *Bin, g1_aff *Aout, fe *Bout, const g2_aff *Vin, g2_aff *Vout, const fe *X,
             const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st);
// KZG terms split in four parts on the setup multiples hm[3 m + p - 1] = 2^{16 p} h_m: S2[4 id + p]
void kzg_terms_split(const g2_aff *h, const g2_aff *hm, const fe *Qc, uint64_t K, uint64_t nb, g2_jac *S2, hipStream_t st);
// M[3 s + m - 1] = 2^{16 m} Q_s (affine), Q_s = Q[(s / seg) segstride + s % seg]
void g2_dbl_mults(const g2_aff *Q, uint64_t seg, uint64_t segstride, uint64_t n, g2_aff *M, hipStream_t st);
void oa_pterms(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t q, fp12 *F, hipStream_t st);
// the G1 terms of the next round: whole multiplications, or split in four parts on the
// multiples M (whole arrays of length 4q, as made by fold_mults) with partials J and nb 8q
// arrival counters
void oa_g1terms_next(const g1_aff *A, const fe *B, uint64_t K, uint64_t nb, uint64_t q, g1_jac *S1, hipStream_t st);
void oa_g1terms_split(const g1_aff *A, const fe *B, const g1_aff *M, uint64_t K, uint64_t nb, uint64_t q, g1_jac *J,
                      uint32_t *cnt, g1_jac *S1, hipStream_t st);
void final_exp2(const fp12 *in0, uint64_t st0, uint64_t n0, fp12 *out0, const fp12 *in1, uint64_t st1, uint64_t n1, fp12 *out1,
                hipStream_t st);
// time-split multiplications: M[3 s + m - 1] = G[s]^{2^{16 m}}, = 2^{32 m} P[s] (m = 1..3);
// the split combine (4 parts per power and per G1 multiple, PE/PM[4 s + p]) and the
// product of U with the 8 G_T parts of each side
void gt_sqr_mults(const fp12 *G, uint64_t n, fp12 *M, hipStream_t st);
// (the points of the multiples are P[(s / seg) segstride + s % seg], s < n)
// the reduced G1 groups of the terms taken ahead made ready for the combine: affine (PU1,
// PX1) and PX1m[3 s + m - 1] = 2^{32 m} PX1[s]
void g1_finish(const g1_jac *PS, uint64_t nb, uint64_t q, g1_aff *PU1, g1_aff *PX1, g1_aff *PX1m, hipStream_t st);
// both in one launch: n1 G1 points in segments of seg1, n2 G2 points in segments of seg2
void fold_mults(const g1_aff *P, uint64_t seg1, uint64_t n1, const g2_aff *Q, uint64_t seg2, uint64_t n2, uint64_t segstride,
                g1_aff *M1, g2_aff *M2, hipStream_t st);
// the fold with four-part split multiplications on the multiples M1 = 2^{32 m} A[h + i],
// M2 = 2^{16 m} V[h + i]; partial results in J1, J2; 2 nb h arrival counters
void oa_fold_split(const g1_aff *Ain, const fe *Bin, g1_aff *Aout, fe *Bout, const g2_aff *Vin, g2_aff *Vout, const fe *X,
                   const fe *Xinv, const g1_aff *M1, const g2_aff *M2, g1_jac *J1, g2_jac *J2, uint32_t *cnt, uint64_t K,
                   uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st);
void oa_combine_split(const fp12 *PX, const fp12 *PXm, const g1_aff *PX1, const g1_aff *PX1m, const fe *k_even,
                      const fe *k_odd, uint64_t kstride, uint64_t nb, fp12 *PE, g1_jac *PM, hipStream_t st);
// L_j, R_j (G_T and G1 parts) from the U groups and the 8 parts per side of the combine
void oa_combine8(const fp12 *U, const fp12 *P, const g1_aff *U1, const g1_jac *P1, uint64_t nb, fp12 *L, fp12 *R, g1_aff *L1,
                 g1_aff *R1, uint64_t lK, hipStream_t st);
}  // namespace ks
