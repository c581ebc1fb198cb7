// Kernels of VC.Verify for one opening proof (appendix C; section 3 FC.BVerify with the
// faster verifier; section 4.2 for the Merkle and folding parts):
//   kv_decode      point decompression and range checks, one thread per proof element
//   kv_transcript  Fiat-Shamir replay (r_i, x_j, z, rho_j), f_v(z), b_l, Merkle path, y*
//   kv_assemble    point sums and the pairs of the three pairing checks
//   kv_compare     the final equalities
// Scalar multiplications, G_T exponentiations, Miller loops and final exponentiations
// run in the shared kernels (wide layout and engine).
#include "kcommon.hpp"
#include "verify.h"

namespace {

__device__ fe rd_be(const uint8_t *b) {
  fe a;
  for (int i = 0; i < 8; i++)
    a.l[7 - i] = ((uint32_t)b[4 * i] << 24) | ((uint32_t)b[4 * i + 1] << 16) | ((uint32_t)b[4 * i + 2] << 8) | b[4 * i + 3];
  return a;
}

__device__ bool lt_words(const fe &a, const uint32_t *m) {
  for (int i = 7; i >= 0; i--)
    if (a.l[i] != m[i]) return a.l[i] < m[i];
  return false;
}

// canonical y > (p - 1)/2
__device__ bool larger(const fe &ymont) { return !lt_words(f_from_mont<FpP>(ymont), bn::P_HALF) && !fe_eq(f_from_mont<FpP>(ymont), fe_const(bn::P_HALF)); }

// square root in F_p (p = 3 mod 4): a^((p+1)/4), verified by squaring
__device__ bool fp_sqrt(const fe &a, fe &r) {
  r = f_pow<FpP>(a, bn::P_SQRT_EXP);
  return fe_eq(fp_sqr(r), a);
}

// square root in F_p2 through the norm: with n = a0^2 + a1^2 and s = sqrt(n),
// x0 = sqrt((a0 +- s)/2), x1 = a1 / (2 x0); verified by squaring
__device__ bool fp2_sqrt(const fp2 &a, fp2 &r) {
  if (fe_is_zero(a.c1)) {
    fe s;
    if (fp_sqrt(a.c0, s)) { r = {s, fe_zero()}; return true; }
    if (fp_sqrt(fp_neg(a.c0), s)) { r = {fe_zero(), s}; return true; }
    return false;
  }
  fe n = fp_add(fp_sqr(a.c0), fp_sqr(a.c1)), s;
  if (!fp_sqrt(n, s)) return false;
  fe t = fp_half(fp_add(a.c0, s)), x0;
  if (!fp_sqrt(t, x0)) {
    t = fp_half(fp_sub(a.c0, s));
    if (!fp_sqrt(t, x0)) return false;
  }
  fe x1 = fp_mul(a.c1, fp_inv_fast(fp_dbl(x0)));
  r = {x0, x1};
  fp2 chk = f2_sqr(r);
  return fe_eq(chk.c0, a.c0) && fe_eq(chk.c1, a.c1);
}

// compressed G1 (32 bytes): x, flag 0x80 identity, 0x40 y > (p - 1)/2
__device__ bool g1_decompress(const uint8_t *b, g1_aff &o) {
  uint8_t buf[32];
  for (int i = 0; i < 32; i++) buf[i] = b[i];
  bool inf = buf[0] & 0x80, big = buf[0] & 0x40;
  buf[0] &= 0x3f;
  o = {fe_zero(), fe_zero()};
  if (inf) {
    bool z = !big;
    for (int i = 0; i < 32; i++) z = z && buf[i] == 0;
    return z;
  }
  fe x = rd_be(buf);
  if (!lt_words(x, bn::P_MOD)) return false;
  x = f_to_mont<FpP>(x);
  fe rhs = fp_add(fp_mul(fp_sqr(x), x), f_mul_small<FpP>(f_one<FpP>(), 3));
  fe y;
  if (!fp_sqrt(rhs, y)) return false;
  if (larger(y) != big) y = fp_neg(y);
  o = {x, y};
  return true;
}

// compressed G2 (64 bytes): x.c0 || x.c1, sign from y.c1, or y.c0 when y.c1 = 0
__device__ bool g2_decompress(const uint8_t *b, g2_aff &o) {
  uint8_t buf[64];
  for (int i = 0; i < 64; i++) buf[i] = b[i];
  bool inf = buf[0] & 0x80, big = buf[0] & 0x40;
  buf[0] &= 0x3f;
  o = {f2_zero(), f2_zero()};
  if (inf) {
    bool z = !big;
    for (int i = 0; i < 64; i++) z = z && buf[i] == 0;
    return z;
  }
  fe x0 = rd_be(buf), x1 = rd_be(buf + 32);
  if (!lt_words(x0, bn::P_MOD) || !lt_words(x1, bn::P_MOD)) return false;
  fp2 x = {f_to_mont<FpP>(x0), f_to_mont<FpP>(x1)};
  fp2 rhs = f2_add(f2_mul(f2_sqr(x), x), f2_const(bn::TWIST_B0, bn::TWIST_B1));
  fp2 y;
  if (!fp2_sqrt(rhs, y)) return false;
  bool l = fe_is_zero(y.c1) ? larger(y.c0) : larger(y.c1);
  if (l != big) y = f2_neg(y);
  o = {x, y};
  return true;
}

__device__ bool gt_decode(const uint8_t *b, fp12 &f) {
  fe *w = reinterpret_cast<fe *>(&f);
  bool ok = true;
  for (int k = 0; k < 12; k++) {
    fe c = rd_be(b + 32 * k);
    ok = ok && lt_words(c, bn::P_MOD);
    w[k] = f_to_mont<FpP>(c);
  }
  return ok;
}

}  // namespace

// one thread per item of proof blockIdx.y (layout of the serialized proof, vc_proof_get)
__global__ void __launch_bounds__(TPB) kv_decode(const VCtx *cs) {
  const VCtx &c = cs[blockIdx.y];
  uint32_t id = (uint32_t)gtid();
  const uint32_t t = c.t, l = c.lK, lM = c.lM;
  const uint32_t n_items = t + 4 * l + 3 + 2 * l + lM + 2;
  if (id >= n_items) return;
  const uint8_t *pf = c.proof;
  bool ok = true;
  if (id < t) {
    ok = g1_decompress(pf + 32 * id, c.blk[id]);
  } else if ((id -= t) < 4 * l) {
    uint32_t r = id / 4, w = id % 4;
    const uint8_t *q = pf + 32 * t + (uint64_t)r * (2 * 384 + 2 * 32);
    if (w == 0) ok = gt_decode(q, c.Lgt[r]);
    else if (w == 1) ok = g1_decompress(q + 384, c.Lg1[r]);
    else if (w == 2) ok = gt_decode(q + 416, c.Rgt[r]);
    else ok = g1_decompress(q + 800, c.Rg1[r]);
  } else if ((id -= 4 * l) < 3) {
    const uint8_t *q = pf + 32 * t + (uint64_t)l * (2 * 384 + 2 * 32);
    if (id == 0) ok = g1_decompress(q, *c.Al);
    else if (id == 1) ok = g2_decompress(q + 32, *c.vl);
    else ok = g2_decompress(q + 96, *c.piv);
  } else if (c.fc_only && (id -= 3) < 2 * l + lM + 2 && id != 2 * l + lM) {
    // sub-array proof: no Step 2 items and no entry
    if (id < 2 * l) {
      if (id % 2 == 0) c.Dsib[id / 2] = g1_aff{fe_zero(), fe_zero()};
      else c.ysib[id / 2] = fe_zero();
    } else if (id < 2 * l + lM) {
      c.Wp[id - 2 * l] = g1_aff{fe_zero(), fe_zero()};
    } else {
      *c.mi = fe_zero();
    }
  } else if (c.fc_only) {
    if (!gt_decode(c.Cb, *c.C)) atomicOr(c.flags, VFLAG_BAD_INPUT);
  } else if ((id -= 3) < 2 * l) {
    const uint8_t *q = pf + 32 * t + (uint64_t)l * (2 * 384 + 2 * 32) + 160 + 64 * (id / 2);
    if (id % 2 == 0) {
      ok = g1_decompress(q, c.Dsib[id / 2]);
    } else {
      fe y = rd_be(q + 32);
      ok = lt_words(y, bn::R_MOD);
      c.ysib[id / 2] = f_to_mont<FpR>(y);
    }
  } else if ((id -= 2 * l) < lM) {
    const uint8_t *q = pf + 32 * t + (uint64_t)l * (2 * 384 + 2 * 32) + 160 + 64 * l + 32 * id;
    ok = g1_decompress(q, c.Wp[id]);
  } else if ((id -= lM) == 0) {
    if (!gt_decode(c.Cb, *c.C)) atomicOr(c.flags, VFLAG_BAD_INPUT);
  } else {
    fe m;
    for (int i = 0; i < 32; i++) reinterpret_cast<uint8_t *>(m.l)[i] = c.mib[i];  // little-endian limbs
    if (!lt_words(m, bn::R_MOD)) atomicOr(c.flags, VFLAG_BAD_INPUT);
    *c.mi = f_to_mont<FpR>(m);
  }
  if (!ok) atomicOr(c.flags, VFLAG_BAD_PROOF);
}

// Fiat-Shamir replay and scalar set-up, a workgroup per proof: chunk digests and the batching
// coefficients r_u one thread each, the challenge chain (x_j, z, f_v(z)) on thread 0 beside the
// Merkle path (rho_j, y*) on thread 64, then b_l as a tree of per-thread partial sums and the
// multiplication jobs in parallel
__global__ void __launch_bounds__(256) kv_transcript(const VCtx *cs) {
  const VCtx &c = cs[blockIdx.x];
  const int tid = threadIdx.x;
  const uint32_t t = c.t, l = c.lK;
  __shared__ uint32_t dig[1024][8];  // chunk digests: t <= 32768 (K of log N <= 30)
  __shared__ uint32_t sigma[8];
  __shared__ fe part[256];
  __shared__ fe s_z, s_rho, s_ystar;
  const uint32_t nch = (t + 31) / 32;
  // r_u = H2F(FC-R, sigma || u), sigma over the digests of 32-entry chunks
  for (uint32_t q = tid; q < nch; q += 256) {
    sha::Hasher hc;
    hc.init();
    for (uint32_t u = q * 32; u < t && u < q * 32 + 32; u++) {
      hc.u64(c.lo + u);
      hc.g1(c.blk[u]);
    }
    hc.final(dig[q]);
  }
  __syncthreads();
  if (tid == 0) {
    sha::Hasher hs;
    hs.init();
    hs.str(DSTR_FC_R);
    hs.gt(*c.C);
    hs.u64(t);
    for (uint32_t q = 0; q < nch; q++)
      for (int w = 0; w < 8; w++) hs.word(dig[q][w]);
    hs.final(sigma);
  }
  __syncthreads();
  for (uint32_t u = tid; u < t; u += 256) {
    sha::Hasher hs;
    sha::xmd_begin(hs);
    for (int w = 0; w < 8; w++) hs.word(sigma[w]);
    hs.u64(u);
    c.r[u] = sha::xmd_finish_fr(hs, DSTR_FC_R);
  }
  // round challenges x_j = H2F(FC-X, x_{j-1} || L_gt || L_g1 || R_gt || R_g1), the workgroup
  // hashing together: lanes write the message words into shared memory, all compress
  __shared__ uint32_t xmsg[16 + 8 + 2 * (96 + 16) + 32], xt2[16];
  for (uint32_t j = 0; j < l; j++) {
    const int pre = j > 0 ? 8 : 0;
    if (tid < 16) xmsg[tid] = 0;  // Z_pad
    const int e = j > 0 ? tid - 1 : tid;
    if (j > 0 && tid == 0) sha::put_words<FpR>(xmsg + 16, c.x[j - 1]);
    if (e >= 0 && e < 28) {
      int side = e / 14, q = e % 14;
      const fe *src = q < 12 ? reinterpret_cast<const fe *>(side ? c.Rgt + j : c.Lgt + j) + q
                             : reinterpret_cast<const fe *>(side ? c.Rg1 + j : c.Lg1 + j) + (q - 12);
      sha::put_words<FpP>(xmsg + 16 + pre + 112 * side + 8 * q, *src);
    }
    __syncthreads();
    fe x = sha::xmd_fr_coop(sha::Coop{tid, 256}, xmsg, 4 * (pre + 224), DSTR_FC_X, xt2);
    fe xi = f_inv_uniform<FpR>(x, bn::R_R3);
    if (tid == 0) {
      if (fe_is_zero(x)) atomicOr(c.flags, VFLAG_BAD_PROOF);
      c.x[j] = x;
      c.xinv[j] = xi;
    }
    __syncthreads();
  }
  if (tid == 0) {
    // z = H2F(FC-Z, x_l || v_l); f_v(z) = prod_j (1 + x_j^{-1} z^{2^{l-j+1}})
    sha::Hasher hz;
    sha::xmd_begin(hz);
    hz.field<FpR>(c.x[l - 1]);
    hz.g2(*c.vl);
    fe z = sha::xmd_finish_fr(hz, DSTR_FC_Z);
    fe fz = f_one<FpR>(), zp = fr_mul(z, z);  // z^{2^1}
    for (int j = (int)l; j >= 1; j--) {      // exponent 2^{l-j+1}: j = l first
      fz = fr_mul(fz, fr_add(f_one<FpR>(), fr_mul(c.xinv[j - 1], zp)));
      zp = fr_mul(zp, zp);
    }
    s_z = z;
    *c.fz = fz;
  } else if (tid == 64 && c.fc_only) {
    s_rho = fe_zero();
    s_ystar = fe_zero();
  } else if (tid == 64) {
    // Merkle path of leaf i = SHA-256(0x00 || m_i || C_j) up to the root
    const g1_aff &Cj = c.blk[c.j - c.lo];
    uint32_t mw[8], cw[16], node[8];
    fe mc = f_from_mont<FpR>(*c.mi);
    fe cx = f_from_mont<FpP>(Cj.x), cy = f_from_mont<FpP>(Cj.y);
    for (int q = 0; q < 8; q++) { mw[q] = mc.l[7 - q]; cw[q] = cx.l[7 - q]; cw[8 + q] = cy.l[7 - q]; }
    sha::merkle_leaf(node, mw, cw);
    uint64_t pos = c.N + c.i;
    for (uint32_t h = 0; h < c.L; h++, pos >>= 1) {
      uint32_t sib[8];
      const uint8_t *sb = c.mpath + 32 * h;
      for (int q = 0; q < 8; q++)
        sib[q] = ((uint32_t)sb[4 * q] << 24) | ((uint32_t)sb[4 * q + 1] << 16) | ((uint32_t)sb[4 * q + 2] << 8) | sb[4 * q + 3];
      uint32_t o[8];
      if (pos & 1) sha::merkle_node(o, sib, node);
      else sha::merkle_node(o, node, sib);
      for (int q = 0; q < 8; q++) node[q] = o[q];
    }
    sha::Hasher hr;
    sha::xmd_begin(hr);
    hr.gt(*c.C);
    for (int q = 0; q < 8; q++) hr.word(node[q]);
    hr.u64(c.j);
    fe rho = sha::xmd_finish_fr(hr, DSTR_RHO);
    fe ystar = fr_mul(rho, *c.mi);
    for (uint32_t h = 0; h < l; h++) ystar = fr_add(ystar, c.ysib[h]);
    s_rho = rho;
    s_ystar = ystar;
  }
  __syncthreads();
  // b_l = sum_u r_u prod_k (x_k^{-1})^{bit_{l-k}(a_u)}
  fe acc = fe_zero();
  for (uint32_t u = tid; u < t; u += 256) {
    fe term = c.r[u];
    for (uint32_t k = 1; k <= l; k++)
      if (((c.lo + u) >> (l - k)) & 1) term = fr_mul(term, c.xinv[k - 1]);
    acc = fr_add(acc, term);
  }
  part[tid] = acc;
  __syncthreads();
  for (int sft = 128; sft > 0; sft >>= 1) {
    if (tid < sft) part[tid] = fr_add(part[tid], part[tid + sft]);
    __syncthreads();
  }
  // G1 multiplication jobs: r_u blk_u; x_j Lg1_j; x_j^{-1} Rg1_j; b_l A_l; rho C_j; y* g1; z g1;
  // then (g1, 0) up to the stride of the job arrays
  const g1_aff g1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  for (uint32_t q = tid; q < c.nmul; q += 256) {
    g1_aff base = g1;
    fe k = fe_zero();
    if (q < t) {
      base = c.blk[q]; k = c.r[q];
    } else if (q < t + 2 * l) {
      uint32_t j = (q - t) / 2;
      if ((q - t) % 2 == 0) { base = c.Lg1[j]; k = c.x[j]; }
      else { base = c.Rg1[j]; k = c.xinv[j]; }
    } else if (q == t + 2 * l) {
      base = *c.Al; k = part[0];
    } else if (q == t + 2 * l + 1) {
      base = c.blk[c.j - c.lo]; k = s_rho;
    } else if (q == t + 2 * l + 2) {
      k = s_ystar;
    } else if (q == t + 2 * l + 3) {
      k = s_z;
    }
    c.mb[q] = base;
    c.ms[q] = k;
  }
  // G_T jobs: L_j^{x_j}, R_j^{1/x_j}
  for (uint32_t q = tid; q < 2 * l; q += 256) {
    c.gts[q] = (q % 2 == 0) ? c.x[q / 2] : c.xinv[q / 2];
    c.gtb[q] = (q % 2 == 0) ? c.Lgt[q / 2] : c.Rgt[q / 2];
  }
}

// point sums and pairing inputs, a workgroup per proof (the sum of the t + 2l products as a
// tree of per-thread partial sums)
__global__ void __launch_bounds__(256) kv_assemble(const VCtx *cs) {
  const VCtx &c = cs[blockIdx.x];
  __shared__ g1_jac sh[256];
  const int tid = threadIdx.x;
  const uint32_t t = c.t, l = c.lK, lM = c.lM;
  g1_jac acc = jac_inf<OpsG1>();
  for (uint32_t u = tid; u < t + 2 * l; u += 256) acc = jac_madd(acc, c.mo[u]);
  sh[tid] = acc;
  __syncthreads();
  for (int sft = 128; sft > 0; sft >>= 1) {
    if (tid < sft) sh[tid] = jac_add(sh[tid], sh[tid + sft]);
    __syncthreads();
  }
  // G_T product C prod L^x R^{1/x} gathers in gto[0..2l] with C last
  for (uint32_t q = tid; q < 2 * l; q += 256) c.gto[q] = c.gtp[q];
  if (tid != 0) return;
  *c.Cg1 = jac_to_aff(sh[0]);
  *c.bA = c.mo[t + 2 * l];
  g1_jac D = jac_from_aff(c.mo[t + 2 * l + 1]);
  for (uint32_t h = 0; h < l; h++) D = jac_madd(D, c.Dsib[h]);
  g1_aff P0 = jac_to_aff(jac_madd(D, aff_neg(c.mo[t + 2 * l + 2])));
  g1_aff g1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  g2_aff g2 = {f2_const(bn::G2X0, bn::G2X1), f2_const(bn::G2Y0, bn::G2Y1)};
  g1_aff Pk = jac_to_aff(jac_madd(jac_from_aff(*c.g1beta), aff_neg(c.mo[t + 2 * l + 3])));
  g2_aff Qk = jac_to_aff(jac_madd(jac_from_aff(*c.vl), aff_neg(*c.fzg2)));
  // pairs: (A_l, v_l) | (beta g1 - z g1, pi_v), (-g1, v_l - f_v(z) g2) | (D* - y* g1, -g2), (W_d, s'_d g2)
  c.pp[0] = *c.Al; c.pq[0] = *c.vl;
  c.pp[1] = Pk; c.pq[1] = *c.piv;
  c.pp[2] = aff_neg(g1); c.pq[2] = Qk;
  c.pp[3] = P0; c.pq[3] = aff_neg(g2);
  uint64_t a = c.a;
  for (uint32_t d = 0; d < lM; d++) {
    uint32_t var = lM - 1 - d;
    c.pp[4 + d] = c.Wp[d];
    g2_aff q = c.vk[var];
    if ((a >> var) & 1) q = jac_to_aff(jac_madd(jac_from_aff(q), aff_neg(g2)));
    c.pq[4 + d] = q;
  }
  c.gto[2 * l] = *c.C;
}

// the final equalities, a thread per proof
__global__ void __launch_bounds__(64) kv_compare(const VCtx *cs, uint32_t n) {
  uint64_t p = gtid();
  if (p >= n) return;
  const VCtx &c = cs[p];
  fp12 one;
  fe *o = reinterpret_cast<fe *>(&one);
  for (int k = 0; k < 12; k++) o[k] = k == 0 ? f_one<FpP>() : fe_zero();
  auto eq12 = [](const fp12 &a, const fp12 &b) {
    const fe *x = reinterpret_cast<const fe *>(&a), *y = reinterpret_cast<const fe *>(&b);
    bool e = true;
    for (int k = 0; k < 12; k++) e = e && fe_eq(x[k], y[k]);
    return e;
  };
  bool ok = eq12(c.E[0], c.gto[0]) && eq12(c.E[1], one) && eq12(c.E[2], one) && fe_eq(c.bA->x, c.Cg1->x) &&
            fe_eq(c.bA->y, c.Cg1->y);
  if (c.cj_expect) {
    const g1_aff &cj = c.blk[c.j - c.lo];
    ok = ok && fe_eq(cj.x, c.cj_expect->x) && fe_eq(cj.y, c.cj_expect->y);
  }
  if (ok) atomicOr(c.flags, VFLAG_ACCEPT);
}

// the three final exponentiations' inputs of every proof side by side (products of the pairs
// 0, 1..2 and 3..), so that one launch takes them all: G[3 p + r] = F[p npair + {0, 1, 3}[r]]
__global__ void __launch_bounds__(TPB) kv_fe_gather(const fp12 *F, uint64_t npair, uint32_t n, fp12 *G) {
  uint64_t id = gtid();
  if (id >= 3ull * n) return;
  uint64_t p = id / 3, r = id % 3;
  G[id] = F[p * npair + (r == 2 ? 3 : r)];
}

namespace kv {
void fe_gather(const fp12 *F, uint64_t npair, uint32_t n, fp12 *G, hipStream_t st) { L1(kv_fe_gather, 3ull * n, F, npair, n, G); }
void decode(const VCtx *cs, uint32_t n, uint32_t tmax, uint32_t lK, uint32_t lM, hipStream_t st) {
  uint32_t items = tmax + 4 * lK + 3 + 2 * lK + lM + 2;
  LAUNCH(kv_decode, dim3(nblk(items), n), dim3(TPB), 0, cs);
}
void transcript(const VCtx *cs, uint32_t n, hipStream_t st) { LAUNCH(kv_transcript, dim3(n), dim3(256), 0, cs); }
void assemble(const VCtx *cs, uint32_t n, hipStream_t st) { LAUNCH(kv_assemble, dim3(n), dim3(256), 0, cs); }
void compare(const VCtx *cs, uint32_t n, hipStream_t st) {
  LAUNCH(kv_compare, dim3((n + 63) / 64), dim3(64), 0, cs, n);
}
}  // namespace kv

// ------------------------------------------------------------------ every proof at once
// Serialization of all N proofs (the wire format of vc_proof_get) and their verification in
// one pass: items that honest proofs share (the block and FC proof of a batch, the D-tree
// siblings, the W commitments) are compared byte for byte with the proof that represents
// them and decoded once; the PST checks (section 4.2 Step 2, appendix C) of all proofs are
// combined with random 128-bit weights delta_i into one product of l_M + 1 pairings:
//   e(sum_i delta_i (D*_i - y*_i g1 + sum_d a_{i,var d} W_{i,d}), -g2) prod_d e(sum_i delta_i W_{i,d}, vk_{var d}) = 1
// with var d = l_M - 1 - d.  The FC part (FC.BVerify with the faster verifier) is the same
// for every proof of a batch and is checked once per batch by the one-proof verifier.
namespace {

__device__ uint64_t pl_bm(const PLayout &y) { return (uint64_t)y.b * y.M; }
__device__ uint64_t pl_batch(const PLayout &y, uint64_t i) { return i / pl_bm(y); }
__device__ uint32_t pl_t(const PLayout &y, uint64_t k) { return k == y.nb - 1 ? y.t_last : y.b; }
// byte offset of proof i
__device__ uint64_t pl_off(const PLayout &y, uint64_t i) {
  uint64_t k = pl_batch(y, i), bm = pl_bm(y);
  return k * bm * y.len_full + (i - k * bm) * (k == y.nb - 1 ? y.len_last : y.len_full);
}
// start of the Step 2 part (after block, rounds and tail) in a proof of batch k
__device__ uint64_t pl_step2(const PLayout &y, uint64_t k) { return 32ull * pl_t(y, k) + 832ull * y.lK + 160; }

__device__ void put_be(uint8_t *o, const fe &c) {
  for (int q = 0; q < 8; q++) {
    uint32_t w = c.l[7 - q];
    o[4 * q] = (uint8_t)(w >> 24);
    o[4 * q + 1] = (uint8_t)(w >> 16);
    o[4 * q + 2] = (uint8_t)(w >> 8);
    o[4 * q + 3] = (uint8_t)w;
  }
}
__device__ void put_g1c(uint8_t *o, const g1_aff &p) {
  if (aff_is_inf(p)) {
    for (int q = 0; q < 32; q++) o[q] = q == 0 ? 0x80 : 0;
    return;
  }
  put_be(o, f_from_mont<FpP>(p.x));
  if (larger(p.y)) o[0] |= 0x40;
}
__device__ void put_g2c(uint8_t *o, const g2_aff &p) {
  if (aff_is_inf(p)) {
    for (int q = 0; q < 64; q++) o[q] = q == 0 ? 0x80 : 0;
    return;
  }
  put_be(o, f_from_mont<FpP>(p.x.c0));
  put_be(o + 32, f_from_mont<FpP>(p.x.c1));
  if (fe_is_zero(p.y.c1) ? larger(p.y.c0) : larger(p.y.c1)) o[0] |= 0x40;
}

__device__ int ilog2(uint64_t v) {
  int r = 0;
  while (v >>= 1) r++;
  return r;
}
// heap index n of a D-tree sibling (levels h < lK of K >> h nodes) to (h, s)
__device__ void d_node(uint64_t n, uint64_t K, uint32_t &h, uint64_t &s) {
  h = 0;
  while (n >= (K >> h)) { n -= K >> h; h++; }
  s = n;
}
// heap index w of a W commitment to depth d and prefix p
__device__ void w_node(uint64_t w, uint32_t &d, uint64_t &p) {
  d = (uint32_t)ilog2(w + 1);
  p = w + 1 - (1ull << d);
}

}  // namespace

// one thread per (proof, item)
__global__ void __launch_bounds__(TPB) kps_serialize(PSCtx c) {
  const PLayout &y = c.y;
  const uint64_t per = y.b + 6ull * y.lK + 3 + y.lM + y.L;
  uint64_t id = gtid();
  if (id >= y.N * per) return;
  uint64_t i = id / per, q = id % per;
  uint64_t k = pl_batch(y, i), j = i / y.M, a = i % y.M, lo = k * y.b;
  uint32_t t = pl_t(y, k), l = y.lK;
  uint8_t *o = c.out + pl_off(y, i);
  if (q < t) { put_g1c(o + 32 * q, c.Cj[lo + q]); return; }
  q -= t;
  if (q < 4ull * l) {
    uint64_t r = q / 4, s = k * l + r;
    uint8_t *b = o + 32ull * t + 832 * r;
    switch (q % 4) {
      case 0: { const fe *g = reinterpret_cast<const fe *>(c.Lgt + s); for (int e = 0; e < 12; e++) put_be(b + 32 * e, f_from_mont<FpP>(g[e])); break; }
      case 1: put_g1c(b + 384, c.Lg1[s]); break;
      case 2: { const fe *g = reinterpret_cast<const fe *>(c.Rgt + s); for (int e = 0; e < 12; e++) put_be(b + 416 + 32 * e, f_from_mont<FpP>(g[e])); break; }
      default: put_g1c(b + 800, c.Rg1[s]);
    }
    return;
  }
  q -= 4ull * l;
  uint8_t *b1 = o + 32ull * t + 832ull * l;
  if (q < 3) {
    if (q == 0) put_g1c(b1, c.Al[k]);
    else if (q == 1) put_g2c(b1 + 32, c.vl[k]);
    else put_g2c(b1 + 96, c.piv[k]);
    return;
  }
  q -= 3;
  uint8_t *b2 = b1 + 160;
  if (q < 2ull * l) {
    uint32_t h = (uint32_t)(q / 2);
    uint64_t node = 2 * y.K - ((2 * y.K) >> h) + ((j >> h) ^ 1);
    if (q % 2 == 0) put_g1c(b2 + 64 * h, c.D[node]);
    else put_be(b2 + 64 * h + 32, c.Y[node * y.M + a]);  // stored canonical
    return;
  }
  q -= 2ull * l;
  if (q < y.lM) {
    put_g1c(b2 + 64ull * l + 32 * q, c.W[(1ull << q) - 1 + (a >> (y.lM - q))]);
    return;
  }
  q -= y.lM;
  if (q < y.L) {
    const uint32_t *nd = c.tree + 8 * (((y.N + i) >> q) ^ 1);
    uint8_t *m = b2 + 64ull * l + 32ull * y.lM + 32 * q;
    for (int w = 0; w < 8; w++) {
      m[4 * w] = (uint8_t)(nd[w] >> 24);
      m[4 * w + 1] = (uint8_t)(nd[w] >> 16);
      m[4 * w + 2] = (uint8_t)(nd[w] >> 8);
      m[4 * w + 3] = (uint8_t)nd[w];
    }
  }
}

// shared items, one thread each: K block commitments, 2K - 2 D-tree siblings, M - 1 W, C
__global__ void __launch_bounds__(TPB) kva_decode(VACtx c) {
  const PLayout &y = c.y;
  uint64_t id = gtid(), K = y.K;
  const uint64_t nD = 2 * K - 2, nW = y.M - 1;
  if (id >= K + nD + nW + 1) return;
  bool ok = true;
  if (id < K) {
    uint64_t j = id, k = j / y.b;
    ok = g1_decompress(c.proofs + pl_off(y, k * pl_bm(y)) + 32 * (j - k * y.b), c.Cj[j]);
  } else if ((id -= K) < nD) {
    uint32_t h;
    uint64_t s;
    d_node(id, K, h, s);
    uint64_t j = (s ^ 1) << h, i = j * y.M;
    ok = g1_decompress(c.proofs + pl_off(y, i) + pl_step2(y, pl_batch(y, i)) + 64 * h, c.Dn[id]);
  } else if ((id -= nD) < nW) {
    uint32_t d;
    uint64_t p;
    w_node(id, d, p);
    uint64_t i = p << (y.lM - d);
    ok = g1_decompress(c.proofs + pl_off(y, i) + pl_step2(y, 0) + 64ull * y.lK + 32 * d, c.Wn[id]);
  } else {
    if (!gt_decode(c.Cb, *c.C)) atomicOr(c.flags, VFLAG_BAD_INPUT);
  }
  if (!ok) atomicOr(c.flags, VFLAG_BAD_PROOF);
}

// the root of every proof's Merkle path from its leaf (m_i, C_j), one thread per proof
__global__ void __launch_bounds__(TPB) kva_roots(VACtx c) {
  const PLayout &y = c.y;
  uint64_t i = gtid();
  if (i >= y.N) return;
  uint64_t j = i / y.M;
  fe m;
  for (int q = 0; q < 8; q++) {
    const uint8_t *b = c.m + 32 * i + 4 * q;
    m.l[q] = (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
  }
  if (!lt_words(m, bn::R_MOD)) atomicOr(c.flags, VFLAG_BAD_INPUT);
  fe cx = f_from_mont<FpP>(c.Cj[j].x), cy = f_from_mont<FpP>(c.Cj[j].y);
  uint32_t mw[8], cw[16], node[8];
  for (int q = 0; q < 8; q++) { mw[q] = m.l[7 - q]; cw[q] = cx.l[7 - q]; cw[8 + q] = cy.l[7 - q]; }
  sha::merkle_leaf(node, mw, cw);
  const uint8_t *path = c.proofs + pl_off(y, i) + pl_step2(y, pl_batch(y, i)) + 64ull * y.lK + 32ull * y.lM;
  uint64_t pos = y.N + i;
  for (uint32_t h = 0; h < y.L; h++, pos >>= 1) {
    uint32_t sib[8], o[8];
    for (int q = 0; q < 8; q++) {
      const uint8_t *sb = path + 32 * h + 4 * q;
      sib[q] = ((uint32_t)sb[0] << 24) | ((uint32_t)sb[1] << 16) | ((uint32_t)sb[2] << 8) | sb[3];
    }
    if (pos & 1) sha::merkle_node(o, sib, node);
    else sha::merkle_node(o, node, sib);
    for (int q = 0; q < 8; q++) node[q] = o[q];
  }
  for (int q = 0; q < 8; q++) c.root[8 * i + q] = node[q];
}

// rho_j from C and the root of proof 0, one thread per j
__global__ void __launch_bounds__(64) kva_rho(VACtx c) {
  uint64_t j = gtid();
  if (j >= c.y.K) return;
  sha::Hasher hr;
  sha::xmd_begin(hr);
  hr.gt(*c.C);
  for (int q = 0; q < 8; q++) hr.word(c.root[q]);
  hr.u64(j);
  c.rho[j] = sha::xmd_finish_fr(hr, DSTR_RHO);
}

// a workgroup per proof: its block, FC proof, D-tree siblings and W against the proofs that
// represent them (16-byte words; every proof starts on a 32-byte boundary)
__global__ void __launch_bounds__(256) kva_same(VACtx c) {
  const PLayout &y = c.y;
  __shared__ int diff;
  uint64_t i = blockIdx.x;
  if (i >= y.N) return;
  const int t = threadIdx.x;
  if (t == 0) diff = 0;
  __syncthreads();
  uint64_t k = pl_batch(y, i), j = i / y.M, a = i % y.M, i0 = k * pl_bm(y);
  const uint4 *P = reinterpret_cast<const uint4 *>(c.proofs + pl_off(y, i));
  bool d = false;
  if (i != i0) {
    const uint4 *R = reinterpret_cast<const uint4 *>(c.proofs + pl_off(y, i0));
    uint64_t n16 = pl_step2(y, k) / 16;
    for (uint64_t q = t; q < n16; q += 256) {
      uint4 u = P[q], v = R[q];
      d |= u.x != v.x || u.y != v.y || u.z != v.z || u.w != v.w;
    }
  }
  // item x < lK: D-tree sibling of level x; lK <= x < lK + lM: W of depth x - lK (two words each)
  uint32_t nit = y.lK + y.lM;
  if ((uint32_t)t < 2 * nit) {
    uint32_t x = t / 2, half = t % 2;
    uint64_t ir, ofs_i, ofs_r;
    if (x < y.lK) {
      ir = ((j >> x) << x) * y.M;
      ofs_i = pl_step2(y, k) + 64ull * x;
      ofs_r = pl_step2(y, pl_batch(y, ir)) + 64ull * x;
    } else {
      uint32_t dd = x - y.lK;
      ir = (a >> (y.lM - dd)) << (y.lM - dd);
      ofs_i = pl_step2(y, k) + 64ull * y.lK + 32ull * dd;
      ofs_r = pl_step2(y, 0) + 64ull * y.lK + 32ull * dd;
    }
    if (ir != i) {
      uint4 u = reinterpret_cast<const uint4 *>(c.proofs + pl_off(y, i) + ofs_i)[half];
      uint4 v = reinterpret_cast<const uint4 *>(c.proofs + pl_off(y, ir) + ofs_r)[half];
      d |= u.x != v.x || u.y != v.y || u.z != v.z || u.w != v.w;
    }
  }
  if (d) atomicOr(&diff, 1);
  __syncthreads();
  if (t == 0) c.odd[i] = diff ? 1 : 0;
}

// one thread per proof: y*_i = rho_j m_i + sum of the y siblings, the weight delta_i =
// H(seed, i) (128 bits), and delta_i, delta_i y*_i (zero for a proof left to the one-proof
// verifier, which joins the list)
__global__ void __launch_bounds__(TPB) kva_proof(VACtx c) {
  const PLayout &y = c.y;
  uint64_t i = gtid();
  if (i >= y.N) return;
  bool odd = c.odd[i] != 0;
  for (int q = 0; q < 8; q++) odd = odd || c.root[8 * i + q] != c.root[q];
  uint64_t j = i / y.M;
  fe m;
  for (int q = 0; q < 8; q++) {
    const uint8_t *b = c.m + 32 * i + 4 * q;
    m.l[q] = (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
  }
  fe ys = fr_mul(c.rho[j], f_to_mont<FpR>(m));
  const uint8_t *s2 = c.proofs + pl_off(y, i) + pl_step2(y, pl_batch(y, i));
  for (uint32_t h = 0; h < y.lK; h++) {
    fe v = rd_be(s2 + 64 * h + 32);
    if (!lt_words(v, bn::R_MOD)) atomicOr(c.flags, VFLAG_BAD_PROOF);
    ys = fr_add(ys, f_to_mont<FpR>(v));
  }
  sha::Hasher hs;
  hs.init();
  hs.str(DSTR_VALL);
  hs.bytes(c.seed, 32);
  hs.u64(i);
  uint32_t dg[8];
  hs.final(dg);
  fe w = fe_zero();
  for (int q = 0; q < 4; q++) w.l[3 - q] = dg[q];
  w = f_to_mont<FpR>(w);
  if (odd) {
    uint32_t at = atomicAdd(c.oddcnt, 1u);
    c.oddlist[at] = i;  // at < N: one entry per proof at most
    w = fe_zero();
  }
  c.delta[i] = w;
  c.dy[i] = fr_mul(w, ys);
}

// sums of the weights: per row j (over a), per column a (over j), and of delta_i y*_i;
// workgroups [0, K) rows, [K, K + M) columns, K + M the total
__global__ void __launch_bounds__(256) kva_sums(VACtx c) {
  const PLayout &y = c.y;
  __shared__ fe sh[256];
  uint64_t g = blockIdx.x;
  const int t = threadIdx.x;
  fe acc = fe_zero();
  if (g < y.K) {
    for (uint64_t a = t; a < y.M; a += 256) acc = fr_add(acc, c.delta[g * y.M + a]);
  } else if (g < y.K + y.M) {
    uint64_t a = g - y.K;
    for (uint64_t j = t; j < y.K; j += 256) acc = fr_add(acc, c.delta[j * y.M + a]);
  } else {
    for (uint64_t i = t; i < y.N; i += 256) acc = fr_add(acc, c.dy[i]);
  }
  sh[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = fr_add(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) {
    if (g < y.K) c.rowsum[g] = sh[0];
    else if (g < y.K + y.M) c.colsum[g - y.K] = sh[0];
    else *c.sy = sh[0];
  }
}

// the multiplication terms, one thread each.  Segment 0 (3K + M - 2 terms), paired with -g2:
// rho_j Delta_j C_j; (sum of Delta over the subvectors whose sibling is D node (h, s)) D;
// (sum of the column weights over the upper half of W's range) W; -(sum delta y*) g1.
// Segment 1 + d (2^d terms), paired with vk_{l_M - 1 - d}: (sum over W's range) W.
__global__ void __launch_bounds__(TPB) kva_terms(VACtx c) {
  const PLayout &y = c.y;
  const uint64_t K = y.K, M = y.M, T0 = 3 * K + M - 2;
  uint64_t id = gtid();
  if (id >= T0 + M - 1) return;
  g1_aff base;
  fe k = fe_zero();
  if (id < K) {
    base = c.Cj[id];
    k = fr_mul(c.rho[id], c.rowsum[id]);
  } else if (id < 3 * K - 2) {
    uint64_t n = id - K, s;
    uint32_t h;
    d_node(n, K, h, s);
    base = c.Dn[n];
    uint64_t j0 = (s ^ 1) << h;
    for (uint64_t j = j0; j < j0 + (1ull << h); j++) k = fr_add(k, c.rowsum[j]);
  } else if (id < T0 - 1 || id >= T0) {
    bool upper = id < T0;
    uint64_t w = upper ? id - (3 * K - 2) : id - T0, p;
    uint32_t d;
    w_node(w, d, p);
    base = c.Wn[w];
    uint64_t len = 1ull << (y.lM - d), lo = p * len + (upper ? len / 2 : 0), hi = (p + 1) * len;
    for (uint64_t a = lo; a < hi; a++) k = fr_add(k, c.colsum[a]);
  } else {
    base = {fe_const(bn::G1X), fe_const(bn::G1Y)};
    k = fr_sub(fe_zero(), *c.sy);
  }
  c.bases[id] = base;
  c.scal[id] = k;
}

// a workgroup per segment: the sum of its products, and the pairing inputs
__global__ void __launch_bounds__(256) kva_segsum(VACtx c) {
  const PLayout &y = c.y;
  __shared__ g1_jac sh[256];
  const uint64_t T0 = 3 * y.K + y.M - 2;
  uint32_t g = blockIdx.x;
  if (g > y.lM) return;
  const int t = threadIdx.x;
  uint64_t lo = g == 0 ? 0 : T0 + (1ull << (g - 1)) - 1, len = g == 0 ? T0 : 1ull << (g - 1);
  g1_jac acc = jac_inf<OpsG1>();
  for (uint64_t q = t; q < len; q += 256) acc = jac_madd(acc, c.prod[lo + q]);
  sh[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = jac_add(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) {
    c.pp[g] = jac_to_aff(sh[0]);
    g2_aff g2 = {f2_const(bn::G2X0, bn::G2X1), f2_const(bn::G2Y0, bn::G2Y1)};
    c.pq[g] = g == 0 ? aff_neg(g2) : c.vk[y.lM - g];  // segment 1 + d: vk_{l_M - 1 - d}
  }
}

__global__ void __launch_bounds__(64) kva_check(VACtx c) {
  if (gtid() != 0) return;
  const fe *e = reinterpret_cast<const fe *>(c.E);
  bool one = fe_eq(e[0], f_one<FpP>());
  for (int q = 1; q < 12; q++) one = one && fe_is_zero(e[q]);
  if (one) atomicOr(c.flags, VFLAG_ACCEPT);
}

namespace kva {
uint64_t nterms(const VACtx &c) { return 3 * c.y.K + 2 * c.y.M - 3; }
void serialize(const PSCtx &c, hipStream_t st) {
  L1(kps_serialize, c.y.N * (c.y.b + 6ull * c.y.lK + 3 + c.y.lM + c.y.L), c);
}
void decode(const VACtx &c, hipStream_t st) { L1(kva_decode, 3 * c.y.K + c.y.M - 2, c); }
void roots(const VACtx &c, hipStream_t st) { L1(kva_roots, c.y.N, c); }
void rho(const VACtx &c, hipStream_t st) { LAUNCH(kva_rho, dim3((unsigned)((c.y.K + 63) / 64)), dim3(64), 0, c); }
void same(const VACtx &c, hipStream_t st) { LAUNCH(kva_same, dim3((unsigned)c.y.N), dim3(256), 0, c); }
void proof(const VACtx &c, hipStream_t st) { L1(kva_proof, c.y.N, c); }
void sums(const VACtx &c, hipStream_t st) { LAUNCH(kva_sums, dim3((unsigned)(c.y.K + c.y.M + 1)), dim3(256), 0, c); }
void terms(const VACtx &c, hipStream_t st) { L1(kva_terms, nterms(c), c); }
void segsum(const VACtx &c, hipStream_t st) { LAUNCH(kva_segsum, dim3(c.y.lM + 1), dim3(256), 0, c); }
void check(const VACtx &c, hipStream_t st) { LAUNCH(kva_check, dim3(1), dim3(64), 0, c); }
}  // namespace kva

// ------------------------------------------------------------------ evaluation proof at a point
// Verifier of the evaluation proof (section 4.3): FC.BVerify of C_F = <C, T(r_L)> on the dense
// query b = r_0 T (faster verifier), then PC.Verify of F at r_R:
//   e(C_F - y g1, g2) = prod_d e(W_d, (s_var - r_var) g2),  var = l_M - 1 - d.
// The pairs and the final equalities are laid out as for one opening proof (kv_compare).

// one thread per item: C_F, the rounds, A_l v_l pi_v, y, W, C and the point
__global__ void __launch_bounds__(TPB) kve_decode(VECtx c) {
  uint32_t id = (uint32_t)gtid();
  const uint32_t l = c.lK, lM = c.lM;
  if (id >= 1 + 4 * l + 3 + 1 + lM + 1 + c.L) return;
  const uint8_t *pf = c.proof;
  bool ok = true;
  if (id == 0) {
    ok = g1_decompress(pf, *c.CF);
  } else if ((id -= 1) < 4 * l) {
    uint32_t r = id / 4, w = id % 4;
    const uint8_t *q = pf + 32 + (uint64_t)r * (2 * 384 + 2 * 32);
    if (w == 0) ok = gt_decode(q, c.Lgt[r]);
    else if (w == 1) ok = g1_decompress(q + 384, c.Lg1[r]);
    else if (w == 2) ok = gt_decode(q + 416, c.Rgt[r]);
    else ok = g1_decompress(q + 800, c.Rg1[r]);
  } else if ((id -= 4 * l) < 3) {
    const uint8_t *q = pf + 32 + (uint64_t)l * (2 * 384 + 2 * 32);
    if (id == 0) ok = g1_decompress(q, *c.Al);
    else if (id == 1) ok = g2_decompress(q + 32, *c.vl);
    else ok = g2_decompress(q + 96, *c.piv);
  } else if ((id -= 3) == 0) {
    fe v = rd_be(pf + 32 + (uint64_t)l * (2 * 384 + 2 * 32) + 160);
    ok = lt_words(v, bn::R_MOD);
    *c.y = f_to_mont<FpR>(v);
  } else if ((id -= 1) < lM) {
    ok = g1_decompress(pf + 32 + (uint64_t)l * (2 * 384 + 2 * 32) + 192 + 32 * id, c.W[id]);
  } else if ((id -= lM) == 0) {
    if (!gt_decode(c.Cb, *c.C)) atomicOr(c.flags, VFLAG_BAD_INPUT);
  } else {
    uint32_t k = id - 1;
    fe v;
    for (int q = 0; q < 32; q++) reinterpret_cast<uint8_t *>(v.l)[q] = c.rle[32 * k + q];  // little-endian limbs
    if (!lt_words(v, bn::R_MOD)) atomicOr(c.flags, VFLAG_BAD_INPUT);
    c.r[k] = f_to_mont<FpR>(v);
  }
  if (!ok) atomicOr(c.flags, VFLAG_BAD_PROOF);
}

// r_0, the challenges x_j, z, f_v(z) (thread 0), b_l = r_0 sum_j T_j prod_k (x_k^{-1})^{bit_{l-k}(j)}
// as a tree, and the jobs (one workgroup)
__global__ void __launch_bounds__(256) kve_transcript(VECtx c) {
  const int tid = threadIdx.x;
  const uint32_t l = c.lK, lM = c.lM;
  __shared__ fe part[256];
  __shared__ fe s_r0, s_z;
  if (tid == 0) {
    sha::Hasher hs;
    hs.init();
    hs.str(DSTR_EVAL);
    hs.gt(*c.C);
    for (int k = (int)c.L - 1; k >= 0; k--) hs.field<FpR>(c.r[k]);
    hs.g1(*c.CF);
    uint32_t sigma[8];
    hs.final(sigma);
    sha::Hasher hx;
    sha::xmd_begin(hx);
    for (int w = 0; w < 8; w++) hx.word(sigma[w]);
    hx.u64(0);
    s_r0 = sha::xmd_finish_fr(hx, DSTR_EVAL);
  }
  // round challenges, the workgroup hashing together (as in kv_transcript)
  __shared__ uint32_t xmsg[16 + 8 + 2 * (96 + 16) + 32], xt2[16];
  for (uint32_t j = 0; j < l; j++) {
    const int pre = j > 0 ? 8 : 0;
    if (tid < 16) xmsg[tid] = 0;  // Z_pad
    const int e = j > 0 ? tid - 1 : tid;
    if (j > 0 && tid == 0) sha::put_words<FpR>(xmsg + 16, c.x[j - 1]);
    if (e >= 0 && e < 28) {
      int side = e / 14, q = e % 14;
      const fe *src = q < 12 ? reinterpret_cast<const fe *>(side ? c.Rgt + j : c.Lgt + j) + q
                             : reinterpret_cast<const fe *>(side ? c.Rg1 + j : c.Lg1 + j) + (q - 12);
      sha::put_words<FpP>(xmsg + 16 + pre + 112 * side + 8 * q, *src);
    }
    __syncthreads();
    fe x = sha::xmd_fr_coop(sha::Coop{tid, 256}, xmsg, 4 * (pre + 224), DSTR_FC_X, xt2);
    fe xi = f_inv_uniform<FpR>(x, bn::R_R3);
    if (tid == 0) {
      if (fe_is_zero(x)) atomicOr(c.flags, VFLAG_BAD_PROOF);
      c.x[j] = x;
      c.xinv[j] = xi;
    }
    __syncthreads();
  }
  if (tid == 0) {
    sha::Hasher hz;
    sha::xmd_begin(hz);
    hz.field<FpR>(c.x[l - 1]);
    hz.g2(*c.vl);
    fe z = sha::xmd_finish_fr(hz, DSTR_FC_Z);
    fe fz = f_one<FpR>(), zp = fr_mul(z, z);
    for (int j = (int)l; j >= 1; j--) {
      fz = fr_mul(fz, fr_add(f_one<FpR>(), fr_mul(c.xinv[j - 1], zp)));
      zp = fr_mul(zp, zp);
    }
    s_z = z;
    c.g2s[0] = fz;
  }
  __syncthreads();
  fe acc = fe_zero();
  for (uint64_t j = tid; j < c.K; j += 256) {
    fe term = c.T[j];
    for (uint32_t k = 1; k <= l; k++)
      if ((j >> (l - k)) & 1) term = fr_mul(term, c.xinv[k - 1]);
    acc = fr_add(acc, term);
  }
  part[tid] = acc;
  __syncthreads();
  for (int sft = 128; sft > 0; sft >>= 1) {
    if (tid < sft) part[tid] = fr_add(part[tid], part[tid + sft]);
    __syncthreads();
  }
  const g1_aff g1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  for (uint32_t q = tid; q < 2 * l + 4; q += 256) {
    g1_aff base = g1;
    fe k;
    if (q < 2 * l) {
      uint32_t j = q / 2;
      if (q % 2 == 0) { base = c.Lg1[j]; k = c.x[j]; }
      else { base = c.Rg1[j]; k = c.xinv[j]; }
    } else if (q == 2 * l) {
      base = *c.Al; k = fr_mul(s_r0, part[0]);
    } else if (q == 2 * l + 1) {
      base = *c.CF; k = s_r0;
    } else if (q == 2 * l + 2) {
      k = *c.y;
    } else {
      k = s_z;
    }
    c.mb[q] = base;
    c.ms[q] = k;
  }
  for (uint32_t d = tid; d < lM; d += 256) c.g2s[1 + d] = c.r[lM - 1 - d];
  for (uint32_t q = tid; q < 2 * l; q += 256) {
    c.gts[q] = (q % 2 == 0) ? c.x[q / 2] : c.xinv[q / 2];
    c.gtb[q] = (q % 2 == 0) ? c.Lgt[q / 2] : c.Rgt[q / 2];
  }
}

// point sums and the pairs (one thread)
__global__ void __launch_bounds__(64) kve_assemble(VECtx c) {
  if (gtid() != 0) return;
  const uint32_t l = c.lK, lM = c.lM;
  g1_jac acc = jac_from_aff(c.mo[2 * l + 1]);  // r_0 C_F
  for (uint32_t u = 0; u < 2 * l; u++) acc = jac_madd(acc, c.mo[u]);
  *c.Cg1 = jac_to_aff(acc);
  *c.bA = c.mo[2 * l];
  g1_aff g1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  g2_aff g2 = {f2_const(bn::G2X0, bn::G2X1), f2_const(bn::G2Y0, bn::G2Y1)};
  g1_aff Pk = jac_to_aff(jac_madd(jac_from_aff(*c.g1beta), aff_neg(c.mo[2 * l + 3])));
  g2_aff Qk = jac_to_aff(jac_madd(jac_from_aff(*c.vl), aff_neg(c.g2o[0])));
  g1_aff P0 = jac_to_aff(jac_madd(jac_from_aff(*c.CF), aff_neg(c.mo[2 * l + 2])));
  // pairs: (A_l, v_l) | (beta g1 - z g1, pi_v), (-g1, v_l - f_v(z) g2) | (C_F - y g1, -g2), (W_d, (s - r)_var g2)
  c.pp[0] = *c.Al; c.pq[0] = *c.vl;
  c.pp[1] = Pk; c.pq[1] = *c.piv;
  c.pp[2] = aff_neg(g1); c.pq[2] = Qk;
  c.pp[3] = P0; c.pq[3] = aff_neg(g2);
  for (uint32_t d = 0; d < lM; d++) {
    c.pp[4 + d] = c.W[d];
    c.pq[4 + d] = jac_to_aff(jac_madd(jac_from_aff(c.vk[lM - 1 - d]), aff_neg(c.g2o[1 + d])));
  }
  for (uint32_t q = 0; q < 2 * l; q++) c.gto[q] = c.gtp[q];
  c.gto[2 * l] = *c.C;
}

namespace kve {
void decode(const VECtx &c, hipStream_t st) { L1(kve_decode, 1 + 4 * c.lK + 3 + 1 + c.lM + 1 + c.L, c); }
void transcript(const VECtx &c, hipStream_t st) { LAUNCH(kve_transcript, dim3(1), dim3(256), 0, c); }
void assemble(const VECtx &c, hipStream_t st) { LAUNCH(kve_assemble, dim3(1), dim3(64), 0, c); }
}  // namespace kve

// ------------------------------------------------------------------ all sub-array proofs at once
// A workgroup per subvector j: its proof against the first proof of its batch (16-byte words;
// honest proofs of a batch are equal), and entry j of its block against the commitment
// recomputed from m_j.  Proofs that differ join the list checked alone.
__global__ void __launch_bounds__(256) ksa_check(const uint8_t *proofs, uint64_t K, uint32_t b, uint64_t nb,
                                                 uint64_t len_full, uint64_t len_last, const g1_aff *Cre,
                                                 uint64_t *oddlist, uint32_t *oddcnt, int *flags) {
  __shared__ int diff;
  uint64_t j = blockIdx.x;
  if (j >= K) return;
  const int t = threadIdx.x;
  uint64_t k = j / b, j0 = k * b, len = k == nb - 1 ? len_last : len_full;
  const uint8_t *P = proofs + k * (uint64_t)b * len_full + (j - j0) * len;
  const uint8_t *R = proofs + k * (uint64_t)b * len_full;
  if (t == 0) diff = 0;
  __syncthreads();
  bool d = false;
  if (j != j0) {
    const uint4 *p4 = reinterpret_cast<const uint4 *>(P), *r4 = reinterpret_cast<const uint4 *>(R);
    for (uint64_t q = t; q < len / 16; q += 256) {
      uint4 u = p4[q], v = r4[q];
      d |= u.x != v.x || u.y != v.y || u.z != v.z || u.w != v.w;
    }
  }
  if (d) atomicOr(&diff, 1);
  __syncthreads();
  if (t != 0) return;
  g1_aff e;
  bool ok = g1_decompress(P + 32 * (j - j0), e);
  if (!ok || !fe_eq(e.x, Cre[j].x) || !fe_eq(e.y, Cre[j].y)) atomicOr(flags, VFLAG_BAD_PROOF);
  if (diff) oddlist[atomicAdd(oddcnt, 1u)] = j;
}

namespace ksa {
void check(const uint8_t *proofs, uint64_t K, uint32_t b, uint64_t nb, uint64_t len_full, uint64_t len_last,
           const g1_aff *Cre, uint64_t *oddlist, uint32_t *oddcnt, int *flags, hipStream_t st) {
  LAUNCH(ksa_check, dim3((unsigned)K), dim3(256), 0, proofs, K, b, nb, len_full, len_last, Cre, oddlist, oddcnt, flags);
}
}  // namespace ksa
