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

// one thread per item; layout of the proof in VCtx::off_*
__global__ void __launch_bounds__(TPB) kv_decode(VCtx c) {
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

// Fiat-Shamir replay and scalar set-up (one thread)
__global__ void __launch_bounds__(64) kv_transcript(VCtx c) {
  if (gtid() != 0) return;
  const uint32_t t = c.t, l = c.lK;
  // batching coefficients r_u = H2F(FC-R, sigma || u), sigma over 32-entry chunk digests
  uint32_t sigma[8];
  {
    sha::Hasher hs;
    hs.init();
    hs.str(DSTR_FC_R);
    hs.gt(*c.C);
    hs.u64(t);
    for (uint32_t q = 0; q * 32 < t; q++) {
      sha::Hasher hc;
      hc.init();
      for (uint32_t u = q * 32; u < t && u < q * 32 + 32; u++) {
        hc.u64(c.lo + u);
        hc.g1(c.blk[u]);
      }
      uint32_t d[8];
      hc.final(d);
      for (int w = 0; w < 8; w++) hs.word(d[w]);
    }
    hs.final(sigma);
  }
  for (uint32_t u = 0; u < t; u++) {
    sha::Hasher hs;
    sha::xmd_begin(hs);
    for (int w = 0; w < 8; w++) hs.word(sigma[w]);
    hs.u64(u);
    c.r[u] = sha::xmd_finish_fr(hs, DSTR_FC_R);
  }
  // round challenges
  for (uint32_t j = 0; j < l; j++) {
    sha::Hasher hs;
    sha::xmd_begin(hs);
    if (j > 0) hs.field<FpR>(c.x[j - 1]);
    hs.gt(c.Lgt[j]);
    hs.g1(c.Lg1[j]);
    hs.gt(c.Rgt[j]);
    hs.g1(c.Rg1[j]);
    fe x = sha::xmd_finish_fr(hs, DSTR_FC_X);
    if (fe_is_zero(x)) atomicOr(c.flags, VFLAG_BAD_PROOF);
    c.x[j] = x;
    c.xinv[j] = fr_inv_fast(x);
  }
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
  // b_l = sum_u r_u prod_k (x_k^{-1})^{bit_{l-k}(a_u)}
  fe bl = fe_zero();
  for (uint32_t u = 0; u < t; u++) {
    fe term = c.r[u];
    for (uint32_t k = 1; k <= l; k++)
      if (((c.lo + u) >> (l - k)) & 1) term = fr_mul(term, c.xinv[k - 1]);
    bl = fr_add(bl, term);
  }
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
  // G1 multiplication jobs: r_u blk_u; x_j Lg1_j; x_j^{-1} Rg1_j; b_l A_l; rho C_j; y* g1; z g1
  uint32_t n = 0;
  for (uint32_t u = 0; u < t; u++) { c.mb[n] = c.blk[u]; c.ms[n++] = c.r[u]; }
  for (uint32_t j = 0; j < l; j++) {
    c.mb[n] = c.Lg1[j]; c.ms[n++] = c.x[j];
    c.mb[n] = c.Rg1[j]; c.ms[n++] = c.xinv[j];
  }
  g1_aff g1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  c.mb[n] = *c.Al; c.ms[n++] = bl;
  c.mb[n] = Cj; c.ms[n++] = rho;
  c.mb[n] = g1; c.ms[n++] = ystar;
  c.mb[n] = g1; c.ms[n++] = z;
  // G2 job: f_v(z) g2; G_T jobs: L_j^{x_j}, R_j^{1/x_j}
  *c.fz = fz;
  for (uint32_t j = 0; j < l; j++) {
    c.gts[2 * j] = c.x[j];
    c.gts[2 * j + 1] = c.xinv[j];
    c.gtb[2 * j] = c.Lgt[j];
    c.gtb[2 * j + 1] = c.Rgt[j];
  }
}

// point sums and pairing inputs (one thread)
__global__ void __launch_bounds__(64) kv_assemble(VCtx c) {
  if (gtid() != 0) return;
  const uint32_t t = c.t, l = c.lK, lM = c.lM;
  g1_jac acc = jac_inf<OpsG1>();
  for (uint32_t u = 0; u < t + 2 * l; u++) acc = jac_madd(acc, c.mo[u]);
  *c.Cg1 = jac_to_aff(acc);
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
  // G_T product C prod L^x R^{1/x} gathers in gto[0..2l] with C last
  c.gto[2 * l] = *c.C;
}

__global__ void __launch_bounds__(64) kv_compare(VCtx c) {
  if (gtid() != 0) return;
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
  if (ok) atomicOr(c.flags, VFLAG_ACCEPT);
}

namespace kv {
void decode(const VCtx &c, hipStream_t st) {
  uint32_t n = c.t + 4 * c.lK + 3 + 2 * c.lK + c.lM + 2;
  L1(kv_decode, n, c);
}
void transcript(const VCtx &c, hipStream_t st) { LAUNCH(kv_transcript, dim3(1), dim3(64), 0, c); }
void assemble(const VCtx &c, hipStream_t st) { LAUNCH(kv_assemble, dim3(1), dim3(64), 0, c); }
void compare(const VCtx &c, hipStream_t st) { LAUNCH(kv_compare, dim3(1), dim3(64), 0, c); }
}  // namespace kv
