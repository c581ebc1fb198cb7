// Kernels on the wave-cooperative engine (slp.hpp): Miller loops, F_p12 product trees
// and the final exponentiation, one 64-lane workgroup per pairing / product / element.
#include "kcommon.hpp"
#include "slp.hpp"
#include "g2mul.hpp"
#include "gtpow.hpp"
#include "g1mul.hpp"
#include "oa_terms.hpp"

#define SLP_T 64
// slp::run_seq stages a call sequence of at most 256 calls in LDS
static_assert(slp::ML_SEQ_LEN <= 256 && slp::FE_SEQ_LEN <= 256, "call sequence longer than its LDS copy");

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
  CHAIN_PRIORITY();
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

// Product of each segment data[g stride + 0 .. len) into data[g stride] in one launch: a
// workgroup per pair of the first level; of two sibling nodes, the workgroup that finishes
// second climbs to the parent (arrival counters as in k_jac_tree).
__global__ void __launch_bounds__(SLP_T) ks_f12_tree(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt) {
  CHAIN_PRIORITY();
  __shared__ f29 S[slp::FE_NSLOT + 36];
  __shared__ uint32_t arrived;
  uint64_t per = (len + 1) / 2;
  uint64_t id = blockIdx.x;
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  fp12 *seg = data + g * stride;
  uint32_t *c = cnt + g * tree_counters(len);
  const int t = threadIdx.x;
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  uint64_t s = 1, n = per, cb = 0;
  for (;;) {
    uint64_t a = 2 * s * q, b = a + s;
    if (b < len) {
      fe *da = reinterpret_cast<fe *>(seg + a);
      const fe *db = reinterpret_cast<const fe *>(seg + b);
      if (t < 12) {
        S[slp::FE_NSLOT + t] = slp::to29(da[t]);
        S[slp::FE_NSLOT + 12 + t] = slp::to29(db[t]);
      }
      __syncthreads();
      slp::run_seq<4>(S, slp::F12_MUL_CALL, 1, slp::FE_NSLOT, 0, 0);
      if (t < 12) da[t] = slp::from29(slp::canon29(S[slp::FE_NSLOT + 24 + t]));
    }
    if (n == 1) return;
    uint64_t nn = (n + 1) / 2, qp = q >> 1;
    if ((q ^ 1) < n) {
      __threadfence();
      __syncthreads();
      if (t == 0) {
        uint32_t old = atomicAdd(&c[cb + qp], 1u);
        if (old) c[cb + qp] = 0;
        arrived = old;
      }
      __syncthreads();
      if (!arrived) return;
      __threadfence();
    }
    cb += nn;
    q = qp;
    n = nn;
    s *= 2;
  }
}

// f^((p^12 - 1)/r), a workgroup per input; input s at in[s in_stride], output to
// (s odd ? out1 : out0)[(s >> 1) ostride]
__global__ void __launch_bounds__(SLP_T) ks_final_exp(const fp12 *in, uint64_t in_stride, uint64_t n, fp12 *out0, fp12 *out1,
                                                     uint64_t ostride) {
  CHAIN_PRIORITY();
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

// T (Jacobian, the identity when inf) to oaff
__device__ void g2_store_aff(f29 *S, bool inf, g2_aff *oaff) {
  const int t = threadIdx.x;
  fe *o = reinterpret_cast<fe *>(oaff);
  if (inf) {
    if (t < 4) o[t] = fe_zero();
    return;
  }
  slp::run1(S, slp::PROG_G2_NORM, 0, 0, 0);
  {
    fe ti = f_inv_uniform<FpP>(slp::from29(slp::canon29(S[slp::G2_t])), bn::P_R3);
    if (t == 0) S[slp::G2_tinv] = slp::to29(ti);
  }
  __syncthreads();
  slp::run1(S, slp::PROG_G2_AFF, 0, 0, 0);
  if (t < 4) o[t] = slp::from29(slp::canon29(S[slp::G2_ax_0 + t]));
}

// out = k Q + A on the engine (A optional); results written as affine (oaff) or Jacobian (ojac).
// With lo >= 0 only bits [lo, lo + width) of the GLS split of k are applied (gls::chunk).
__device__ void g2_job(f29 *S, gls::Dec *dec, const g2_aff *Q, const fe *k_mont, const g2_aff *A, g2_aff *oaff,
                       g2_jac *ojac, int lo = -1, int width = 0) {
  const int t = threadIdx.x;
  if (t == 0) {
    fe kc = f_from_mont<FpR>(*k_mont);
    gls::Dec d = gls::decompose(kc.l);
    *dec = lo < 0 ? d : gls::chunk(d, lo, width);
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
  g2_store_aff(S, inf, oaff);
}

// Vout[i] = Vin[i] + x^{-1} Vin[h + i] for every batch k (Eq. folding); Vout may be Vin
__global__ void __launch_bounds__(SLP_T) ks_oa_fold_g2(const g2_aff *Vin, g2_aff *Vout, const fe *Xinv, uint64_t K, uint64_t nb,
                                                      uint64_t h, uint32_t j, uint32_t lK) {
  __shared__ f29 S[G2_SLOTS];
  __shared__ gls::Dec dec;
  uint64_t id = blockIdx.x;
  if (id >= nb * h) return;
  uint64_t k = id / h, i = id % h;
  g2_job(S, &dec, Vin + k * K + h + i, Xinv + k * lK + (j - 1), Vin + k * K + i, Vout + k * K + i, nullptr);
}

// terms q_m h_m of the KZG proof of v_l with every multiplication split in four parts (bits
// [16 p, 16 p + 16) of the GLS split, 17 for p = 3) on the multiples hm[3 m + p - 1] =
// 2^{16 p} h_m made at setup: S2[4 id + p] (Jacobian) for term id = k (2K - 2) + m
__global__ void __launch_bounds__(SLP_T) ks_kzg_terms_split(const g2_aff *h, const g2_aff *hm, const fe *Qc, uint64_t K,
                                                           uint64_t nb, g2_jac *S2) {
  CHAIN_PRIORITY();
  __shared__ f29 S[G2_SLOTS];
  __shared__ gls::Dec dec;
  uint64_t n = 2 * K - 2;
  uint64_t id = blockIdx.x;
  if (id >= 4 * nb * n) return;
  uint64_t term = id >> 2, m = term % n;
  int part = (int)(id & 3);
  g2_job(S, &dec, part ? hm + 3 * m + part - 1 : h + m, Qc + term, nullptr, nullptr, S2 + id, 16 * part,
         part < 3 ? 16 : 17);
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

// ---------------------------------------------------------------- G1 scalar multiplications
#define G1_SLOTS (slp::G1_NSLOT + 2)
#define G1_ABASE slp::G1_NSLOT

// T (Jacobian, the identity when inf) to oaff
__device__ void g1_store_aff(f29 *S, bool inf, g1_aff *oaff) {
  const int t = threadIdx.x;
  fe *o = reinterpret_cast<fe *>(oaff);
  if (inf) {
    if (t < 2) o[t] = fe_zero();
    return;
  }
  {
    fe zi = f_inv_uniform<FpP>(slp::from29(slp::canon29(S[slp::G1_T_2])), bn::P_R3);
    if (t == 0) S[slp::G1_tinv] = slp::to29(zi);
  }
  __syncthreads();
  slp::run1(S, slp::PROG_G1_AFF, 0, 0, 0);
  if (t < 2) o[t] = slp::from29(slp::canon29(S[t ? slp::G1_ay : slp::G1_ax]));
}

// out = k P + A on the engine (A optional); results written as affine (oaff) or Jacobian (ojac).
// With chunk >= 0 only that 32-bit part of the GLV split of k is applied (glv::chunk).
__device__ void g1_job(f29 *S, glv::Dec *dec, const g1_aff *P, const fe *k_mont, const g1_aff *A, g1_aff *oaff,
                       g1_jac *ojac, int chunk = -1) {
  const int t = threadIdx.x;
  if (t == 0) {
    fe kc = f_from_mont<FpR>(*k_mont);
    glv::Dec d = glv::decompose(kc.l);
    *dec = chunk < 0 ? d : glv::chunk(d, chunk);
  }
  if (t < 2) S[slp::G1_xP + t] = slp::to29(t ? P->y : P->x);
  if (A && t >= 2 && t < 4) S[G1_ABASE + t - 2] = slp::to29(t == 3 ? A->y : A->x);
  load_consts<slp::G1_NCONST>(S, slp::G1_CBASE, slp::G1_CONSTS);
  __syncthreads();
  bool pinf = g1_inf(*P), has_a = A && !g1_inf(*A);
  slp::DevCtx c{S};
  bool inf = g1m::mul_add(c, *dec, pinf, has_a, G1_ABASE, S[slp::G1_CBASE + 1]);
  if (ojac) {
    fe *o = reinterpret_cast<fe *>(ojac);
    if (t < 3) o[t] = inf ? (t < 2 ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[slp::G1_T_0 + t]));
    return;
  }
  g1_store_aff(S, inf, oaff);
}

// ---------------------------------------------------------------- group sums on the engine
// Sum of each segment data[g stride + 0 .. len) of Jacobian points into data[g stride] in
// one launch: a workgroup per pair of the first level; of two sibling nodes, the workgroup
// that finishes second climbs to the parent (arrival counters as in ks_f12_tree).  The
// identity is any point with Z = 0; additions meeting equal x are resolved exactly.
template <bool G2>
__global__ void __launch_bounds__(SLP_T) ks_jac_tree(void *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt) {
  if (G2) CHAIN_PRIORITY();
  else AHEAD_PRIORITY();
  constexpr int NC = G2 ? 6 : 3;  // coordinates (F_p elements) per point
  __shared__ f29 S[G2 ? G2_SLOTS : G1_SLOTS];
  __shared__ uint32_t arrived;
  uint64_t per = (len + 1) / 2;
  uint64_t id = blockIdx.x;
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  fe *seg = reinterpret_cast<fe *>(data) + g * stride * NC;
  uint32_t *c = cnt + g * tree_counters(len);
  const int t = threadIdx.x;
  const int T0 = G2 ? slp::G2_T_0 : slp::G1_T_0, A0 = G2 ? slp::G2_TB1_0 : slp::G1_TB1_0;
  if (G2) load_consts<slp::G2_NCONST>(S, slp::G2_CBASE, slp::G2_CONSTS);
  else load_consts<slp::G1_NCONST>(S, slp::G1_CBASE, slp::G1_CONSTS);
  slp::DevCtx cx{S};
  uint64_t s = 1, n = per, cb = 0;
  for (;;) {
    uint64_t a = 2 * s * q, b = a + s;
    if (b < len) {
      fe *da = seg + a * NC;
      const fe *db = seg + b * NC;
      bool binf = G2 ? fe_is_zero(db[4]) && fe_is_zero(db[5]) : fe_is_zero(db[2]);
      if (!binf) {
        bool inf = G2 ? fe_is_zero(da[4]) && fe_is_zero(da[5]) : fe_is_zero(da[2]);
        if (t < NC) {
          S[T0 + t] = slp::to29(da[t]);
          S[A0 + t] = slp::to29(db[t]);
        }
        __syncthreads();
        if (G2) g2m::add_jac(cx, inf, A0, false);
        else g1m::add_jac(cx, inf, A0, false);
        fe one_or_zero = (G2 ? (t == 0 || t == 2) : t < 2) ? f_one<FpP>() : fe_zero();
        if (t < NC) da[t] = inf ? one_or_zero : slp::from29(slp::canon29(S[T0 + t]));
      }
    }
    if (n == 1) return;
    uint64_t nn = (n + 1) / 2, qp = q >> 1;
    if ((q ^ 1) < n) {
      __threadfence();
      __syncthreads();
      if (t == 0) {
        uint32_t old = atomicAdd(&c[cb + qp], 1u);
        if (old) c[cb + qp] = 0;
        arrived = old;
      }
      __syncthreads();
      if (!arrived) return;
      __threadfence();
    }
    cb += nn;
    q = qp;
    n = nn;
    s *= 2;
  }
}

// ---------------------------------------------------------------- Step 1 rounds, fused
// Round-1 (direct) G1 terms on the engine: b_L[i] A_R[i] (side 0) and b_R[i] A_L[i] (side 1)
// into S[(2k + side) (K / 2) + i] (Jacobian)
__global__ void __launch_bounds__(SLP_T) ks_oa_g1terms(const g1_aff *A, const fe *B, uint64_t K, uint64_t nb, uint64_t h,
                                                      g1_jac *Sout) {
  AHEAD_PRIORITY();
  __shared__ f29 S[G1_SLOTS];
  __shared__ glv::Dec d1;
  uint64_t id = blockIdx.x;
  if (id >= nb * 2 * h) return;
  uint64_t k = id / (2 * h), r = id % (2 * h), side = r / h, i = r % h;
  g1_job(S, &d1, A + (side ? k * K + i : k * K + h + i), B + (side ? k * K + h + i : k * K + i), nullptr, nullptr,
         Sout + (k * 2 + side) * (K / 2) + i);
}

template <int A_, int B_> struct imax { static constexpr int v = A_ > B_ ? A_ : B_; };

// The fold of round j (Eq. folding) for every batch: blocks [0, nb h) fold G1 and b,
// blocks [nb h, 2 nb h) fold G2.  Aout[i] = Ain[i] + x Ain[h + i], Bout[i] = Bin[i] +
// x^{-1} Bin[h + i], Vout[i] = Vin[i] + x^{-1} Vin[h + i].
__global__ void __launch_bounds__(SLP_T) ks_oa_fold(const g1_aff *Ain, const fe *Bin, g1_aff *Aout, fe *Bout, const g2_aff *Vin,
                                                   g2_aff *Vout, const fe *X, const fe *Xinv, uint64_t K, uint64_t nb,
                                                   uint64_t h, uint32_t j, uint32_t lK) {
  CHAIN_PRIORITY();
  __shared__ f29 S[imax<G1_SLOTS, G2_SLOTS>::v];
  __shared__ glv::Dec d1;
  __shared__ gls::Dec d2;
  uint64_t id = blockIdx.x;
  if (id >= 2 * nb * h) return;
  bool g2 = id >= nb * h;
  if (g2) id -= nb * h;
  uint64_t k = id / h, i = id % h, slot = k * lK + (j - 1);
  if (g2) {
    g2_job(S, &d2, Vin + k * K + h + i, Xinv + slot, Vin + k * K + i, Vout + k * K + i, nullptr);
    return;
  }
  if (threadIdx.x == 32) Bout[k * K + i] = fr_add(Bin[k * K + i], fr_mul(Bin[k * K + h + i], Xinv[slot]));
  g1_job(S, &d1, Ain + k * K + h + i, X + slot, Ain + k * K + i, Aout + k * K + i, nullptr);
}

// The next round's terms (oa_terms.hpp): the Miller loops into F[out], a workgroup per term
__global__ void __launch_bounds__(SLP_T) ks_oa_pterms(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t q,
                                                     fp12 *F) {
  CHAIN_PRIORITY();
  __shared__ f29 S[slp::ML_NSLOT];
  uint64_t id = blockIdx.x;
  if (id >= nb * 8 * q) return;
  oat::Term tm = oat::term(id, K, nb, q);
  miller_one(S, A + tm.a, V + tm.v, F + tm.out);
}

// The G1 terms b[v] A[a] of the next round into S1[out] (Jacobian), a workgroup per term
__global__ void __launch_bounds__(SLP_T) ks_oa_g1terms_next(const g1_aff *A, const fe *B, uint64_t K, uint64_t nb, uint64_t q,
                                                           g1_jac *S1) {
  AHEAD_PRIORITY();
  __shared__ f29 S[G1_SLOTS];
  __shared__ glv::Dec d1;
  uint64_t id = blockIdx.x;
  if (id >= nb * 8 * q) return;
  oat::Term tm = oat::term(id, K, nb, q);
  g1_job(S, &d1, A + tm.a, B + tm.v, nullptr, nullptr, S1 + tm.out);
}

// ---------------------------------------------------------------- cyclotomic G_T powers
#define GTP_SLOTS (slp::FE_NSLOT + 12 * gtp::NBUF)

// ---------------------------------------------------------------- split multiplications
// Multiples for the time-split multiplications: M[3 s + m - 1] = G[s]^{2^{16 m}} (cyclotomic
// squarings), a workgroup per (s, m), m = 1, 2, 3
__global__ void __launch_bounds__(SLP_T) ks_gt_sqr_mults(const fp12 *G, uint64_t n, fp12 *M) {
  CHAIN_PRIORITY();
  __shared__ f29 S[slp::FE_NSLOT + 24];
  uint64_t id = blockIdx.x;
  if (id >= 3 * n) return;
  uint64_t s = id / 3, m = id % 3 + 1;
  const int t = threadIdx.x;
  const fe *src = reinterpret_cast<const fe *>(G + s);
  if (t < 12) S[FE_BUF(0) + t] = slp::to29(src[t]);
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  __syncthreads();
  int b = 0;
  for (int i = 0; i < 16 * (int)m; i++) {
    slp::run1(S, slp::PROG_F12_CSQR, FE_BUF(b), FE_BUF(b), FE_BUF(1 - b));
    b = 1 - b;
  }
  fe *dst = reinterpret_cast<fe *>(M + 3 * s + m - 1);
  if (t < 12) dst[t] = slp::from29(slp::canon29(S[FE_BUF(b) + t]));
}

// point s of a segmented list: P[(s / seg) segstride + s % seg]
__device__ __forceinline__ uint64_t seg_index(uint64_t s, uint64_t seg, uint64_t segstride) {
  return (s / seg) * segstride + s % seg;
}

// 2^{32 m} P (affine) by 16 m double doublings on the engine
__device__ void g1_dbl_mult(f29 *S, const g1_aff *P, int m, g1_aff *o) {
  const int t = threadIdx.x;
  bool inf = g1_inf(*P);
  if (!inf) {
    load_consts<slp::G1_NCONST>(S, slp::G1_CBASE, slp::G1_CONSTS);
    if (t < 3) S[slp::G1_T_0 + t] = slp::to29(t == 2 ? f_one<FpP>() : t ? P->y : P->x);
    __syncthreads();
    for (int i = 0; i < 16 * m; i++) slp::run1(S, slp::PROG_G1_DBL2, 0, 0, 0);
  }
  g1_store_aff(S, inf, o);
}

// 2^{16 m} Q (affine) by 16 m doublings on the engine
__device__ void g2_dbl_mult(f29 *S, const g2_aff *Q, int m, g2_aff *o) {
  const int t = threadIdx.x;
  bool inf = g2_inf(*Q);
  if (!inf) {
    load_consts<slp::G2_NCONST>(S, slp::G2_CBASE, slp::G2_CONSTS);
    const fe *q = reinterpret_cast<const fe *>(Q);
    if (t < 6) S[slp::G2_T_0 + t] = t < 4 ? slp::to29(q[t]) : slp::to29(t == 4 ? f_one<FpP>() : fe_zero());
    __syncthreads();
    for (int i = 0; i < 16 * m; i++) slp::run1(S, slp::PROG_G2_DBL, 0, 0, 0);
  }
  g2_store_aff(S, inf, o);
}

// 2^{32 m} P (affine) for a Jacobian P (m = 0: P itself), on the engine
__device__ void g1_jac_mult_aff(f29 *S, const g1_jac *P, int m, g1_aff *o) {
  const int t = threadIdx.x;
  const fe *pj = reinterpret_cast<const fe *>(P);
  bool inf = fe_is_zero(pj[2]);
  if (!inf) {
    load_consts<slp::G1_NCONST>(S, slp::G1_CBASE, slp::G1_CONSTS);
    if (t < 3) S[slp::G1_T_0 + t] = slp::to29(pj[t]);
    __syncthreads();
    for (int i = 0; i < 16 * m; i++) slp::run1(S, slp::PROG_G1_DBL2, 0, 0, 0);
  }
  g1_store_aff(S, inf, o);
}

// M[3 s + m - 1] = 2^{16 m} Q_s (affine), Q_s as in seg_index, a workgroup per (s, m), m = 1, 2, 3
__global__ void __launch_bounds__(SLP_T) ks_g2_dbl_mults(const g2_aff *Q, uint64_t seg, uint64_t segstride, uint64_t n,
                                                        g2_aff *M) {
  __shared__ f29 S[G2_SLOTS];
  uint64_t id = blockIdx.x;
  if (id >= 3 * n) return;
  uint64_t s = id / 3, m = id % 3 + 1;
  g2_dbl_mult(S, Q + seg_index(s, seg, segstride), (int)m, M + 3 * s + m - 1);
}

// the multiples of a round's arrays in one launch: blocks [0, 3 n1) M1[3 s + m - 1] =
// 2^{32 m} P_s (G1, P_s at seg_index(s, seg1, segstride)), blocks [3 n1, 3 (n1 + n2))
// M2[3 s + m - 1] = 2^{16 m} Q_s (G2, seg2)
__global__ void __launch_bounds__(SLP_T) ks_fold_mults(const g1_aff *P, uint64_t seg1, uint64_t n1, const g2_aff *Q,
                                                      uint64_t seg2, uint64_t n2, uint64_t segstride, g1_aff *M1,
                                                      g2_aff *M2) {
  CHAIN_PRIORITY();
  __shared__ f29 S[imax<G1_SLOTS, G2_SLOTS>::v];
  uint64_t id = blockIdx.x;
  if (id >= 3 * (n1 + n2)) return;
  bool g2 = id >= 3 * n1;
  if (g2) id -= 3 * n1;
  uint64_t s = id / 3, m = id % 3 + 1;
  if (g2) g2_dbl_mult(S, Q + seg_index(s, seg2, segstride), (int)m, M2 + 3 * s + m - 1);
  else g1_dbl_mult(S, P + seg_index(s, seg1, segstride), (int)m, M1 + 3 * s + m - 1);
}

// of the four parts of one multiplication, the workgroup that finishes last returns true
// (and resets the counter); partial results written before are visible to it
__device__ bool last_of_four(uint32_t *cnt, uint32_t *flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t old = atomicAdd(cnt, 1u);
    if (old == 3) *cnt = 0;
    *flag = old == 3;
  }
  __syncthreads();
  bool last = *flag;
  if (last) __threadfence();
  return last;
}

// The fold of round j with every multiplication split in four parts run in parallel (M1
// covers the whole arrays, M1[3 (k 2h + i') + p - 1] for index i' of batch k; M2 the halves,
// M2[3 (k h + i) + p - 1] for V[h + i]):
// blocks [0, 4 nb h): part p of x A[h + i] on the base 2^{32 p} A[h + i] (M1, p > 0) with
// the p-th 32-bit chunk of the GLV split of x into J1[4 s + p]; blocks [4 nb h, 8 nb h):
// part p of x^{-1} V[h + i] on 2^{16 p} V[h + i] (M2) with bits [16 p, 16 p + 16) (17 for
// p = 3) of the GLS split into J2[4 s + p] (s = k h + i).  The last part to finish adds the
// four partial results and A[i] (V[i]) and writes the affine result; part 0 of G1 also
// folds b.  Same results as ks_oa_fold.
__global__ void __launch_bounds__(SLP_T) ks_oa_fold_split(const g1_aff *Ain, const fe *Bin, g1_aff *Aout, fe *Bout,
                                                         const g2_aff *Vin, g2_aff *Vout, const fe *X, const fe *Xinv,
                                                         const g1_aff *M1, const g2_aff *M2, g1_jac *J1, g2_jac *J2,
                                                         uint32_t *cnt, uint64_t K, uint64_t nb, uint64_t h, uint32_t j,
                                                         uint32_t lK) {
  CHAIN_PRIORITY();
  __shared__ f29 S[imax<G1_SLOTS, G2_SLOTS>::v];
  __shared__ glv::Dec d1;
  __shared__ gls::Dec d2;
  __shared__ uint32_t flag;
  uint64_t id = blockIdx.x, n = nb * h;
  if (id >= 8 * n) return;
  const int t = threadIdx.x;
  bool g2 = id >= 4 * n;
  if (g2) id -= 4 * n;
  uint64_t s = id >> 2, k = s / h, i = s % h, slot = k * lK + (j - 1);
  int part = (int)(id & 3);
  slp::DevCtx c{S};
  if (!g2) {
    if (part == 0 && t == 32) Bout[k * K + i] = fr_add(Bin[k * K + i], fr_mul(Bin[k * K + h + i], Xinv[slot]));
    g1_job(S, &d1, part ? M1 + 3 * (k * 2 * h + h + i) + part - 1 : Ain + k * K + h + i, X + slot, nullptr, nullptr,
           J1 + 4 * s + part, part);
    if (!last_of_four(cnt + s, &flag)) return;
    // sum of the parts (in the table slots) and A[i]
    const fe *pj = reinterpret_cast<const fe *>(J1 + 4 * s);
    if (t < 12) S[slp::G1_TB1_0 + t] = slp::to29(pj[t]);
    const g1_aff *A = Ain + k * K + i;
    if (t >= 12 && t < 14) S[G1_ABASE + t - 12] = slp::to29(t == 13 ? A->y : A->x);
    __syncthreads();
    bool inf = true;
    for (int p = 0; p < 4; p++) g1m::add_jac(c, inf, slp::G1_TB1_0 + 3 * p, fe_is_zero(J1[4 * s + p].Z));
    if (!g1_inf(*A)) g1m::add_affine(c, inf, G1_ABASE, S[slp::G1_CBASE + 1]);
    g1_store_aff(S, inf, Aout + k * K + i);
    return;
  }
  g2_job(S, &d2, part ? M2 + 3 * s + part - 1 : Vin + k * K + h + i, Xinv + slot, nullptr, nullptr, J2 + 4 * s + part,
         16 * part, part < 3 ? 16 : 17);
  if (!last_of_four(cnt + n + s, &flag)) return;
  const fe *pj = reinterpret_cast<const fe *>(J2 + 4 * s);
  if (t < 24) S[slp::G2_TB1_0 + t] = slp::to29(pj[t]);
  const fe *a = reinterpret_cast<const fe *>(Vin + k * K + i);
  if (t >= 24 && t < 28) S[G2_ABASE + t - 24] = slp::to29(a[t - 24]);
  __syncthreads();
  bool inf = true;
  for (int p = 0; p < 4; p++) {
    const g2_jac &Jp = J2[4 * s + p];
    g2m::add_jac(c, inf, slp::G2_TB1_0 + 6 * p, fe_is_zero(Jp.Z.c0) && fe_is_zero(Jp.Z.c1));
  }
  if (!g2_inf(Vin[k * K + i])) g2m::add_affine(c, inf, G2_ABASE, S[slp::G2_CBASE + 1], S[slp::G2_CBASE]);
  g2_store_aff(S, inf, Vout + k * K + i);
}

// The G1 terms b[v] A[a] of the next round (oa_terms.hpp, arrays of length 4q) with each
// multiplication split in four parts: part p on the multiple M[3 (k 4q + a') + p - 1] =
// 2^{32 p} A[k K + a'] (p > 0) with the p-th 32-bit chunk of the GLV split of b[v], into
// J[4 term + p]; the last part to finish writes the sum to S1[out] (Jacobian)
__global__ void __launch_bounds__(SLP_T) ks_oa_g1terms_split(const g1_aff *A, const fe *B, const g1_aff *M, uint64_t K,
                                                            uint64_t nb, uint64_t q, g1_jac *J, uint32_t *cnt, g1_jac *S1) {
  AHEAD_PRIORITY();
  __shared__ f29 S[G1_SLOTS];
  __shared__ glv::Dec d1;
  __shared__ uint32_t flag;
  uint64_t id = blockIdx.x;
  if (id >= 4 * nb * 8 * q) return;
  const int t = threadIdx.x;
  uint64_t term = id >> 2, k = term / (8 * q);
  int part = (int)(id & 3);
  oat::Term tm = oat::term(term, K, nb, q);
  g1_job(S, &d1, part ? M + 3 * (k * 4 * q + (tm.a - k * K)) + part - 1 : A + tm.a, B + tm.v, nullptr, nullptr,
         J + 4 * term + part, part);
  if (!last_of_four(cnt + term, &flag)) return;
  const fe *pj = reinterpret_cast<const fe *>(J + 4 * term);
  if (t < 12) S[slp::G1_TB1_0 + t] = slp::to29(pj[t]);
  __syncthreads();
  slp::DevCtx c{S};
  bool inf = true;
  for (int p = 0; p < 4; p++) g1m::add_jac(c, inf, slp::G1_TB1_0 + 3 * p, fe_is_zero(J[4 * term + p].Z));
  fe *o = reinterpret_cast<fe *>(S1 + tm.out);
  if (t < 3) o[t] = inf ? (t < 2 ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[slp::G1_T_0 + t]));
}


// The x-dependent part of a round taken ahead, each multiplication split in four parts run
// in parallel: for s < 4 nb and part p < 4, k_s = (s odd ? k_odd : k_even)[(s >> 2) kstride];
// blocks [0, 16 nb): PE[4 s + p] = (PX[s]^{2^{16 p}})^{chunk_p}, the Frobenius split of k_s
// restricted to bits [16 p, 16 p + 16) (17 bits for p = 3); blocks [16 nb, 32 nb):
// PM[4 s + p] = chunk_p(k_s) (2^{32 p} PX1[s]) (Jacobian).  Multiples come from
// ks_gt_sqr_mults and ks_g1_dbl_mults (PXm, PX1m).
__global__ void __launch_bounds__(SLP_T) ks_oa_combine_split(const fp12 *PX, const fp12 *PXm, const g1_aff *PX1,
                                                            const g1_aff *PX1m, const fe *k_even, const fe *k_odd,
                                                            uint64_t kstride, uint64_t nb, fp12 *PE, g1_jac *PM) {
  CHAIN_PRIORITY();
  __shared__ f29 S[imax<GTP_SLOTS, G1_SLOTS>::v];
  __shared__ gls::Dec dec;
  __shared__ glv::Dec d1;
  uint64_t id = blockIdx.x;
  if (id >= 32 * nb) return;
  const int t = threadIdx.x;
  bool g1 = id >= 16 * nb;
  if (g1) id -= 16 * nb;
  uint64_t s = id >> 2;
  int part = (int)(id & 3);
  const fe *k = (s & 1 ? k_odd : k_even) + (s >> 2) * kstride;
  if (g1) {
    g1_job(S, &d1, part ? PX1m + 3 * s + part - 1 : PX1 + s, k, nullptr, nullptr, PM + 4 * s + part, part);
    return;
  }
  if (t == 0) {
    fe kc = f_from_mont<FpR>(*k);
    dec = gls::chunk(gls::decompose(kc.l), 16 * part, part < 3 ? 16 : 17);
  }
  const fe *src = reinterpret_cast<const fe *>(part ? PXm + 3 * s + part - 1 : PX + s);
  if (t < 12) S[FE_BUF(0) + t] = slp::to29(src[t]);
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  __syncthreads();
  slp::DevCtx c{S};
  int r = gtp::pow_cyc(c, dec, slp::FE_NSLOT);
  fe *dst = reinterpret_cast<fe *>(PE + 4 * s + part);
  if (t < 12) dst[t] = r < 0 ? (t == 0 ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[FE_BUF(r) + t]));
}

// Both parts of L_j, R_j from the combine, in one launch.  Blocks [0, 2 nb):
// (side ? R : L)[k lK] = U[2k + side] prod_{g in {2 side, 2 side + 1}, p < 4} P[4 (4k + g) + p]
// (G_T, engine); blocks [2 nb, 4 nb): the G1 parts U1[2k + side] + sum of the 8 Jacobian
// parts P1[4 (4k + 2 side) + i] (a tree over 8 lanes), affine, into L1 / R1.
__global__ void __launch_bounds__(SLP_T) ks_oa_combine8(const fp12 *U, const fp12 *P, const g1_aff *U1, const g1_jac *P1,
                                                       uint64_t nb, fp12 *L, fp12 *R, g1_aff *L1, g1_aff *R1, uint64_t lK) {
  CHAIN_PRIORITY();
  __shared__ f29 S[slp::FE_NSLOT + 36];
  uint64_t id = blockIdx.x;
  if (id >= 4 * nb) return;
  if (id >= 2 * nb) {
    id -= 2 * nb;
    g1_jac *part = reinterpret_cast<g1_jac *>(S);  // 8 Jacobian points in the slot memory
    uint64_t k = id / 2, side = id % 2;
    const int t = threadIdx.x;
    if (t < 8) part[t] = P1[4 * (4 * k + 2 * side) + t];
    __syncthreads();
    for (int w = 4; w >= 1; w >>= 1) {
      if (t < w) part[t] = jac_add(part[t], part[t + w]);
      __syncthreads();
    }
    if (t == 0) (side ? R1 : L1)[k * lK] = jac_to_aff(jac_madd(part[0], U1[id]));
    return;
  }
  uint64_t k = id / 2, side = id % 2;
  const int t = threadIdx.x;
  const fe *u = reinterpret_cast<const fe *>(U + id);
  if (t < 12) S[FE_BUF(0) + t] = slp::to29(u[t]);
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  int acc = 0;
  for (int i = 0; i < 8; i++) {
    const fe *pi = reinterpret_cast<const fe *>(P + 4 * (4 * k + 2 * side) + i);
    if (t < 12) S[FE_BUF(1) + t] = slp::to29(pi[t]);
    __syncthreads();
    slp::run1(S, slp::PROG_F12_MUL, FE_BUF(acc), FE_BUF(1), FE_BUF(2 - acc));
    acc = 2 - acc;
  }
  fe *dst = reinterpret_cast<fe *>((side ? R : L) + k * lK);
  if (t < 12) dst[t] = slp::from29(slp::canon29(S[FE_BUF(acc) + t]));
}

// final exponentiations of two strided lists: job s < n0 takes in0[s st0] to out0[s], the
// others in1[(s - n0) st1] to out1[s - n0]
// final exponentiation of one F_p12 element on the engine
__device__ void fe_job(f29 *S, const fp12 *in, fp12 *out) {
  int t = threadIdx.x;
  const fe *src = reinterpret_cast<const fe *>(in);
  if (t < 12) S[FE_BUF(0) + t] = slp::to29(src[t]);
  load_consts<slp::FE_NCONST>(S, slp::FE_CBASE, slp::FE_CONSTS);
  __syncthreads();
  slp::run_seq<4>(S, slp::FE_SEQ, slp::FE_SEQ_LEN, slp::FE_NSLOT, slp::FE_t, slp::FE_tinv);
  fe *dst = reinterpret_cast<fe *>(out);
  if (t < 12) dst[t] = slp::from29(slp::canon29(S[FE_BUF(slp::FE_RESULT) + t]));
}

__global__ void __launch_bounds__(SLP_T) ks_final_exp2(const fp12 *in0, uint64_t st0, uint64_t n0, fp12 *out0, const fp12 *in1,
                                                      uint64_t st1, uint64_t n1, fp12 *out1) {
  CHAIN_PRIORITY();
  __shared__ f29 S[FE_SLOTS];
  uint64_t s = blockIdx.x;
  if (s >= n0 + n1) return;
  fe_job(S, s < n0 ? in0 + s * st0 : in1 + (s - n0) * st1, s < n0 ? out0 + s : out1 + (s - n0));
}

// The reduced G1 groups of the terms taken ahead (oa_terms.hpp, segment sums in PS) made
// ready for the combine: blocks [0, 2 nb): U group (2k + side) to PU1 (affine); blocks
// [2 nb, 18 nb): XY group s = 4k + g as PX1[s] (affine, m = 0) and PX1m[3 s + m - 1] =
// 2^{32 m} PX1[s] (m = 1..3)
__global__ void __launch_bounds__(SLP_T) ks_g1_finish(const g1_jac *PS, uint64_t nb, uint64_t q, g1_aff *PU1, g1_aff *PX1,
                                                     g1_aff *PX1m) {
  AHEAD_PRIORITY();
  __shared__ f29 S[G1_SLOTS];
  uint64_t id = blockIdx.x;
  if (id >= 18 * nb) return;
  if (id < 2 * nb) {
    g1_jac_mult_aff(S, PS + id * 2 * q, 0, PU1 + id);
    return;
  }
  id -= 2 * nb;
  uint64_t s = id >> 2;
  int m = (int)(id & 3);
  g1_jac_mult_aff(S, PS + nb * 4 * q + s * q, m, m ? PX1m + 3 * s + m - 1 : PX1 + s);
}

namespace ks {
void miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n, fp12 *out, hipStream_t st) {
  if (n) LAUNCH(ks_miller, dim3((unsigned)n), dim3(SLP_T), 0, P, sp, Q, sq, n, out);
}
void oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h, fp12 *F, hipStream_t st) {
  LAUNCH(ks_oa_miller, dim3((unsigned)(nb * 2 * h)), dim3(SLP_T), 0, A, V, K, nb, h, F);
}
void f12_reduce(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st) {
  if (len > 1) LAUNCH(ks_f12_tree, dim3((unsigned)(nseg * ((len + 1) / 2))), dim3(SLP_T), 0, data, nseg, stride, len, cnt);
}
void final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out0, fp12 *out1, uint64_t ostride, hipStream_t st) {
  if (!out1) {  // every output to out0[s ostride]
    out1 = out0 + ostride;
    ostride *= 2;
  }
  if (n) LAUNCH(ks_final_exp, dim3((unsigned)n), dim3(SLP_T), 0, in, stride, n, out0, out1, ostride);
}
void oa_fold_g2(const g2_aff *Vin, g2_aff *Vout, const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK,
                hipStream_t st) {
  LAUNCH(ks_oa_fold_g2, dim3((unsigned)(nb * h)), dim3(SLP_T), 0, Vin, Vout, Xinv, K, nb, h, j, lK);
}
void oa_fold(const g1_aff *Ain, const fe *Bin, g1_aff *Aout, fe *Bout, const g2_aff *Vin, g2_aff *Vout, const fe *X,
             const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st) {
  LAUNCH(ks_oa_fold, dim3((unsigned)(2 * nb * h)), dim3(SLP_T), 0, Ain, Bin, Aout, Bout, Vin, Vout, X, Xinv, K, nb, h, j, lK);
}
void oa_pterms(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t q, fp12 *F, hipStream_t st) {
  LAUNCH(ks_oa_pterms, dim3((unsigned)(nb * 8 * q)), dim3(SLP_T), 0, A, V, K, nb, q, F);
}
void gt_sqr_mults(const fp12 *G, uint64_t n, fp12 *M, hipStream_t st) {
  if (n) LAUNCH(ks_gt_sqr_mults, dim3((unsigned)(3 * n)), dim3(SLP_T), 0, G, n, M);
}
void g1_finish(const g1_jac *PS, uint64_t nb, uint64_t q, g1_aff *PU1, g1_aff *PX1, g1_aff *PX1m, hipStream_t st) {
  LAUNCH(ks_g1_finish, dim3((unsigned)(18 * nb)), dim3(SLP_T), 0, PS, nb, q, PU1, PX1, PX1m);
}
void oa_g1terms_next(const g1_aff *A, const fe *B, uint64_t K, uint64_t nb, uint64_t q, g1_jac *S1, hipStream_t st) {
  LAUNCH(ks_oa_g1terms_next, dim3((unsigned)(nb * 8 * q)), dim3(SLP_T), 0, A, B, K, nb, q, S1);
}
void oa_g1terms_split(const g1_aff *A, const fe *B, const g1_aff *M, uint64_t K, uint64_t nb, uint64_t q, g1_jac *J,
                      uint32_t *cnt, g1_jac *S1, hipStream_t st) {
  LAUNCH(ks_oa_g1terms_split, dim3((unsigned)(4 * nb * 8 * q)), dim3(SLP_T), 0, A, B, M, K, nb, q, J, cnt, S1);
}
void fold_mults(const g1_aff *P, uint64_t seg1, uint64_t n1, const g2_aff *Q, uint64_t seg2, uint64_t n2, uint64_t segstride,
                g1_aff *M1, g2_aff *M2, hipStream_t st) {
  if (n1 + n2)
    LAUNCH(ks_fold_mults, dim3((unsigned)(3 * (n1 + n2))), dim3(SLP_T), 0, P, seg1, n1, Q, seg2, n2, segstride, M1, M2);
}
void oa_fold_split(const g1_aff *Ain, const fe *Bin, g1_aff *Aout, fe *Bout, const g2_aff *Vin, g2_aff *Vout, const fe *X,
                   const fe *Xinv, const g1_aff *M1, const g2_aff *M2, g1_jac *J1, g2_jac *J2, uint32_t *cnt, uint64_t K,
                   uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st) {
  LAUNCH(ks_oa_fold_split, dim3((unsigned)(8 * nb * h)), dim3(SLP_T), 0, Ain, Bin, Aout, Bout, Vin, Vout, X, Xinv, M1, M2, J1,
         J2, cnt, K, nb, h, j, lK);
}
void oa_combine_split(const fp12 *PX, const fp12 *PXm, const g1_aff *PX1, const g1_aff *PX1m, const fe *k_even,
                      const fe *k_odd, uint64_t kstride, uint64_t nb, fp12 *PE, g1_jac *PM, hipStream_t st) {
  LAUNCH(ks_oa_combine_split, dim3((unsigned)(32 * nb)), dim3(SLP_T), 0, PX, PXm, PX1, PX1m, k_even, k_odd, kstride, nb, PE,
         PM);
}
void oa_combine8(const fp12 *U, const fp12 *P, const g1_aff *U1, const g1_jac *P1, uint64_t nb, fp12 *L, fp12 *R, g1_aff *L1,
                 g1_aff *R1, uint64_t lK, hipStream_t st) {
  LAUNCH(ks_oa_combine8, dim3((unsigned)(4 * nb)), dim3(SLP_T), 0, U, P, U1, P1, nb, L, R, L1, R1, lK);
}
void final_exp2(const fp12 *in0, uint64_t st0, uint64_t n0, fp12 *out0, const fp12 *in1, uint64_t st1, uint64_t n1, fp12 *out1,
                hipStream_t st) {
  if (n0 + n1) LAUNCH(ks_final_exp2, dim3((unsigned)(n0 + n1)), dim3(SLP_T), 0, in0, st0, n0, out0, in1, st1, n1, out1);
}
void g1_tree(g1_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st) {
  if (len > 1) LAUNCH(ks_jac_tree<false>, dim3((unsigned)(nseg * ((len + 1) / 2))), dim3(SLP_T), 0, data, nseg, stride, len, cnt);
}
void g2_tree(g2_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st) {
  if (len > 1) LAUNCH(ks_jac_tree<true>, dim3((unsigned)(nseg * ((len + 1) / 2))), dim3(SLP_T), 0, data, nseg, stride, len, cnt);
}
void oa_g1terms(const g1_aff *A, const fe *B, uint64_t K, uint64_t nb, uint64_t h, g1_jac *S, hipStream_t st) {
  LAUNCH(ks_oa_g1terms, dim3((unsigned)(nb * 2 * h)), dim3(SLP_T), 0, A, B, K, nb, h, S);
}
void kzg_terms_split(const g2_aff *h, const g2_aff *hm, const fe *Qc, uint64_t K, uint64_t nb, g2_jac *S2, hipStream_t st) {
  LAUNCH(ks_kzg_terms_split, dim3((unsigned)(4 * nb * (2 * K - 2))), dim3(SLP_T), 0, h, hm, Qc, K, nb, S2);
}
void g2_dbl_mults(const g2_aff *Q, uint64_t seg, uint64_t segstride, uint64_t n, g2_aff *M, hipStream_t st) {
  if (n) LAUNCH(ks_g2_dbl_mults, dim3((unsigned)(3 * n)), dim3(SLP_T), 0, Q, seg, segstride, n, M);
}
void gt_pow(const fp12 *in, const fe *k, uint64_t n, fp12 *out, hipStream_t st) {
  if (n) LAUNCH(ks_gt_pow, dim3((unsigned)n), dim3(SLP_T), 0, in, k, n, out);
}
}  // namespace ks
