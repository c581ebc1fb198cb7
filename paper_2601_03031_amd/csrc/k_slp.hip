// Kernels on the wave-cooperative engine (slp.hpp): Miller loops, F_p12 product trees
// and the final exponentiation, one 64-lane workgroup per pairing / product / element.
#include "kcommon.hpp"
#include "slp.hpp"
#include "g2mul.hpp"

#define SLP_T 64

namespace {

__device__ __forceinline__ bool g1_inf(const g1_aff &P) { return fe_is_zero(P.x) && fe_is_zero(P.y); }
__device__ __forceinline__ bool g2_inf(const g2_aff &Q) {
  return fe_is_zero(Q.x.c0) && fe_is_zero(Q.x.c1) && fe_is_zero(Q.y.c0) && fe_is_zero(Q.y.c1);
}

using slp::f29;

template <int NCONST>
__device__ __forceinline__ void load_consts(f29 *S, int base, const uint32_t (*C)[9]) {
  for (int c = threadIdx.x; c < NCONST; c += SLP_T) {
    f29 v;
#pragma unroll
    for (int j = 0; j < 9; j++) v.l[j] = C[c][j];
    v.l[9] = v.l[10] = v.l[11] = 0;
    S[base + c] = v;
  }
}

// Miller loop of e(P, Q) into dst (12 coefficients); identity inputs give 1.
__device__ void miller_one(f29 *S, const g1_aff *P, const g2_aff *Q, fp12 *dst) {
  const int t = threadIdx.x;
  fe *out = reinterpret_cast<fe *>(dst);
  if (g1_inf(*P) || g2_inf(*Q)) {
    if (t < 12) out[t] = t == 0 ? f_one<FpP>() : fe_zero();
    return;
  }
  if (t < 2) S[slp::ML_xP + t] = slp::to29(t ? P->y : P->x);
  else if (t < 6) {
    const fe *q = reinterpret_cast<const fe *>(Q);
    S[slp::ML_xP + t] = slp::to29(q[t - 2]);  // xQ.0, xQ.1, yQ.0, yQ.1
  }
  load_consts<slp::ML_NCONST>(S, slp::ML_CBASE, slp::ML_CONSTS);
  __syncthreads();
  slp::run_seq<1>(S, slp::ML_SEQ, slp::ML_SEQ_LEN, 0, 0, 0);
  if (t < 12) out[t] = slp::from29(slp::canon29(S[slp::ML_f_0 + t]));
}

}  // namespace

// out[i] = Miller(P[i sp], Q[i sq])
__global__ void __launch_bounds__(SLP_T) ks_miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n,
                                                  fp12 *out) {
  __shared__ f29 S[slp::ML_NSLOT];
  uint64_t i = blockIdx.x;
  if (i >= n) return;
  miller_one(S, P + i * sp, Q + i * sq, out + i);
}

// side 0 (L) pairs A[h+i] with V[i], side 1 (R) A[i] with V[h+i]; F[(2k+side) K/2 + i]
__global__ void __launch_bounds__(SLP_T) ks_oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h,
                                                     fp12 *F) {
  __shared__ f29 S[slp::ML_NSLOT];
  uint64_t id = blockIdx.x;
  if (id >= nb * 2 * h) return;
  uint64_t k = id / (2 * h), r = id % (2 * h), side = r / h, i = r % h;
  const g1_aff *P = A + (side ? k * K + i : k * K + h + i);
  const g2_aff *Q = V + (side ? k * K + h + i : k * K + i);
  miller_one(S, P, Q, F + (k * 2 + side) * (K / 2) + i);
}

#define FE_SLOTS (slp::FE_NSLOT + 12 * slp::FE_NBUF)
#define FE_BUF(b) (slp::FE_NSLOT + 12 * (b))

// one tree step, a workgroup per product: data[g stride + 2 s q] *= data[g stride + 2 s q + s]
__global__ void __launch_bounds__(SLP_T) ks_f12_step(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, uint64_t s) {
  __shared__ f29 S[slp::FE_NSLOT + 36];
  uint64_t per = (len + 2 * s - 1) / (2 * s);
  uint64_t id = blockIdx.x;
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  uint64_t a = 2 * s * q, b = a + s;
  if (b >= len) return;
  fe *da = reinterpret_cast<fe *>(data + g * stride + a);
  const fe *db = reinterpret_cast<const fe *>(data + g * stride + b);
  int t = threadIdx.x;
  if (t < 12) { S[slp::FE_NSLOT + t] = slp::to29(da[t]); S[slp::FE_NSLOT + 12 + t] = slp::to29(db[t]); }
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  __syncthreads();
  slp::run_seq<4>(S, slp::F12_MUL_CALL, 1, slp::FE_NSLOT, 0, 0);
  if (t < 12) da[t] = slp::from29(slp::canon29(S[slp::FE_NSLOT + 24 + t]));
}

// f^((p^12 - 1)/r), a workgroup per input; input s at in[s in_stride], output to
// (s odd ? out1 : out0)[(s >> 1) ostride]
__global__ void __launch_bounds__(SLP_T) ks_final_exp(const fp12 *in, uint64_t in_stride, uint64_t n, fp12 *out0, fp12 *out1,
                                                     uint64_t ostride) {
  __shared__ f29 S[FE_SLOTS];
  uint64_t s = blockIdx.x;
  if (s >= n) return;
  int t = threadIdx.x;
  const fe *src = reinterpret_cast<const fe *>(in + s * in_stride);
  if (t < 12) S[FE_BUF(0) + t] = slp::to29(src[t]);
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  __syncthreads();
  slp::run_seq<4>(S, slp::FE_SEQ, slp::FE_SEQ_LEN, slp::FE_NSLOT, slp::FE_t, slp::FE_tinv);
  fp12 *o = (s & 1) ? out1 : out0;
  fe *dst = reinterpret_cast<fe *>(o + (s >> 1) * ostride);
  if (t < 12) dst[t] = slp::from29(slp::canon29(S[FE_BUF(slp::FE_RESULT) + t]));
}


// ---------------------------------------------------------------- G2 scalar multiplications
#define G2_SLOTS (slp::G2_NSLOT + 4)
#define G2_ABASE slp::G2_NSLOT

// out = k Q + A on the engine (A optional); results written as affine (oaff) or Jacobian (ojac)
__device__ void g2_job(f29 *S, gls::Dec *dec, const g2_aff *Q, const fe *k_mont, const g2_aff *A, g2_aff *oaff,
                       g2_jac *ojac) {
  const int t = threadIdx.x;
  if (t == 0) {
    fe kc = f_from_mont<FpR>(*k_mont);
    *dec = gls::decompose(kc.l);
  }
  const fe *q = reinterpret_cast<const fe *>(Q);
  if (t < 4) S[slp::G2_xQ_0 + t] = slp::to29(q[t]);
  if (A && t >= 4 && t < 8) S[G2_ABASE + t - 4] = slp::to29(reinterpret_cast<const fe *>(A)[t - 4]);
  load_consts<slp::G2_NCONST>(S, slp::G2_CBASE, slp::G2_CONSTS);
  __syncthreads();
  bool qinf = g2_inf(*Q), has_a = A && !g2_inf(*A);
  slp::DevCtx c{S};
  const f29 one = S[slp::G2_CBASE + 1], zero = S[slp::G2_CBASE];
  bool inf = g2m::mul_add(c, *dec, qinf, has_a, G2_ABASE, one, zero);
  if (ojac) {
    fe *o = reinterpret_cast<fe *>(ojac);
    if (t < 6) o[t] = inf ? ((t == 0 || t == 2) ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[slp::G2_T_0 + t]));
    return;
  }
  fe *o = reinterpret_cast<fe *>(oaff);
  if (inf) {
    if (t < 4) o[t] = fe_zero();
    return;
  }
  c.run(slp::PROG_G2_NORM, 0, 0, 0);
  {
    fe ti = f_inv_uniform<FpP>(slp::from29(slp::canon29(S[slp::G2_t])), bn::P_R3);
    if (t == 0) S[slp::G2_tinv] = slp::to29(ti);
  }
  __syncthreads();
  c.run(slp::PROG_G2_AFF, 0, 0, 0);
  if (t < 4) o[t] = slp::from29(slp::canon29(S[slp::G2_ax_0 + t]));
}

// v[i] = v[i] + x^{-1} v[h + i] for every batch k (Eq. folding)
__global__ void __launch_bounds__(SLP_T) ks_oa_fold_g2(g2_aff *V, const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j,
                                                      uint32_t lK) {
  __shared__ f29 S[G2_SLOTS];
  __shared__ gls::Dec dec;
  uint64_t id = blockIdx.x;
  if (id >= nb * h) return;
  uint64_t k = id / h, i = id % h;
  g2_job(S, &dec, V + k * K + h + i, Xinv + k * lK + (j - 1), V + k * K + i, V + k * K + i, nullptr);
}

// terms q_m h_m of the KZG proof of v_l (Jacobian)
__global__ void __launch_bounds__(SLP_T) ks_kzg_terms(const g2_aff *h, const fe *Qc, uint64_t K, uint64_t nb, g2_jac *S2) {
  __shared__ f29 S[G2_SLOTS];
  __shared__ gls::Dec dec;
  uint64_t n = 2 * K - 2;
  uint64_t id = blockIdx.x;
  if (id >= nb * n) return;
  g2_job(S, &dec, h + id % n, Qc + id, nullptr, nullptr, S2 + id);
}

// ---------------------------------------------------------------- G_T exponentiation
// out[s] = in[s]^k_s (k in Montgomery F_r form), square-and-multiply with the engine's
// F_p12 product (inputs need not lie in the cyclotomic subgroup)
__global__ void __launch_bounds__(SLP_T) ks_gt_pow(const fp12 *in, const fe *k_mont, uint64_t n, fp12 *out) {
  __shared__ f29 S[slp::FE_NSLOT + 36];
  __shared__ uint32_t kc[8];
  uint64_t s = blockIdx.x;
  if (s >= n) return;
  const int t = threadIdx.x;
  const fe *src = reinterpret_cast<const fe *>(in + s);
  if (t < 12) S[FE_BUF(0) + t] = slp::to29(src[t]);
  if (t == 0) {
    fe kcan = f_from_mont<FpR>(k_mont[s]);
    for (int w = 0; w < 8; w++) kc[w] = kcan.l[w];
  }
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  __syncthreads();
  int top = -1;
  for (int b = 255; b >= 0; b--)
    if ((kc[b >> 5] >> (b & 31)) & 1) { top = b; break; }
  fe *dst = reinterpret_cast<fe *>(out + s);
  if (top < 0) {
    if (t < 12) dst[t] = t == 0 ? f_one<FpP>() : fe_zero();
    return;
  }
  // accumulator alternates between buffers 1 and 2; buffer 0 holds the base
  if (t < 12) S[FE_BUF(1) + t] = S[FE_BUF(0) + t];
  __syncthreads();
  int acc = 1;
  for (int b = top - 1; b >= 0; b--) {
    slp::run1(S, slp::PROG_F12_MUL, FE_BUF(acc), FE_BUF(acc), FE_BUF(3 - acc));
    acc = 3 - acc;
    if ((kc[b >> 5] >> (b & 31)) & 1) {
      slp::run1(S, slp::PROG_F12_MUL, FE_BUF(acc), FE_BUF(0), FE_BUF(3 - acc));
      acc = 3 - acc;
    }
  }
  if (t < 12) dst[t] = slp::from29(slp::canon29(S[FE_BUF(acc) + t]));
}

namespace ks {
void miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n, fp12 *out, hipStream_t st) {
  if (n) LAUNCH(ks_miller, dim3((unsigned)n), dim3(SLP_T), 0, P, sp, Q, sq, n, out);
}
void oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h, fp12 *F, hipStream_t st) {
  LAUNCH(ks_oa_miller, dim3((unsigned)(nb * 2 * h)), dim3(SLP_T), 0, A, V, K, nb, h, F);
}
void f12_reduce(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st) {
  for (uint64_t s = 1; s < len; s <<= 1) {
    uint64_t per = (len + 2 * s - 1) / (2 * s);
    LAUNCH(ks_f12_step, dim3((unsigned)(nseg * per)), dim3(SLP_T), 0, data, nseg, stride, len, s);
  }
}
void final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out0, fp12 *out1, uint64_t ostride, hipStream_t st) {
  if (n) LAUNCH(ks_final_exp, dim3((unsigned)n), dim3(SLP_T), 0, in, stride, n, out0, out1, ostride);
}
void oa_fold_g2(g2_aff *V, const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st) {
  LAUNCH(ks_oa_fold_g2, dim3((unsigned)(nb * h)), dim3(SLP_T), 0, V, Xinv, K, nb, h, j, lK);
}
void kzg_terms(const g2_aff *h, const fe *Qc, uint64_t K, uint64_t nb, g2_jac *S2, hipStream_t st) {
  LAUNCH(ks_kzg_terms, dim3((unsigned)(nb * (2 * K - 2))), dim3(SLP_T), 0, h, Qc, K, nb, S2);
}
void gt_pow(const fp12 *in, const fe *k, uint64_t n, fp12 *out, hipStream_t st) {
  if (n) LAUNCH(ks_gt_pow, dim3((unsigned)n), dim3(SLP_T), 0, in, k, n, out);
}
}  // namespace ks
