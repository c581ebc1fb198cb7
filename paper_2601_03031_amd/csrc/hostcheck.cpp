// Host build of the device arithmetic headers (field, tower, curve, pairing, hash),
// exported with canonical big-endian byte encodings so CPU tests can compare the
// GPU path's arithmetic with the oracle before any kernel runs.  This is a test
// harness for the HIP code path; the library itself never runs it.
#include <cstring>
#include "field.hpp"
#include "tower.hpp"
#include "curve.hpp"
#include "pairing.hpp"
#include "hash.hpp"
#include "slp.hpp"
#include "gls.hpp"
#include "g2mul.hpp"
#include "gtpow.hpp"
#include "g1mul.hpp"
#include "oa_terms.hpp"

#define API extern "C" __attribute__((visibility("default")))

template <class F> static fe rd(const uint8_t *b) {
  fe a;
  for (int i = 0; i < 8; i++)
    a.l[7 - i] = ((uint32_t)b[4 * i] << 24) | ((uint32_t)b[4 * i + 1] << 16) | ((uint32_t)b[4 * i + 2] << 8) | b[4 * i + 3];
  return f_to_mont<F>(a);
}
template <class F> static void wr(uint8_t *b, const fe &m) {
  fe a = f_from_mont<F>(m);
  for (int i = 0; i < 8; i++) {
    uint32_t w = a.l[7 - i];
    b[4 * i] = w >> 24; b[4 * i + 1] = w >> 16; b[4 * i + 2] = w >> 8; b[4 * i + 3] = w;
  }
}
static fp2 rd2(const uint8_t *b) { return {rd<FpP>(b), rd<FpP>(b + 32)}; }
static void wr2(uint8_t *b, const fp2 &a) { wr<FpP>(b, a.c0); wr<FpP>(b + 32, a.c1); }
static fp12 rd12(const uint8_t *b) {
  fp12 f;
  fp6 *h[2] = {&f.c0, &f.c1};
  for (int a = 0; a < 2; a++) {
    fp2 *q[3] = {&h[a]->c0, &h[a]->c1, &h[a]->c2};
    for (int c = 0; c < 3; c++) *q[c] = rd2(b + 384 / 2 * a + 64 * c);
  }
  return f;
}
static void wr12(uint8_t *b, const fp12 &f) {
  const fp6 *h[2] = {&f.c0, &f.c1};
  for (int a = 0; a < 2; a++) {
    const fp2 *q[3] = {&h[a]->c0, &h[a]->c1, &h[a]->c2};
    for (int c = 0; c < 3; c++) wr2(b + 192 * a + 64 * c, *q[c]);
  }
}
static g1_aff rdg1(const uint8_t *b) { return {rd<FpP>(b), rd<FpP>(b + 32)}; }
static void wrg1(uint8_t *b, const g1_aff &p) { wr<FpP>(b, p.x); wr<FpP>(b + 32, p.y); }
static g2_aff rdg2(const uint8_t *b) { return {rd2(b), rd2(b + 64)}; }
static void wrg2(uint8_t *b, const g2_aff &p) { wr2(b, p.x); wr2(b + 64, p.y); }
static void canon_scalar(uint32_t k[8], const uint8_t *b) {
  for (int i = 0; i < 8; i++)
    k[7 - i] = ((uint32_t)b[4 * i] << 24) | ((uint32_t)b[4 * i + 1] << 16) | ((uint32_t)b[4 * i + 2] << 8) | b[4 * i + 3];
}

// batched binary GCD on a canonical integer 0 < x < m (which 0: p, 1: r): x^{-1} mod m
// (big-endian 32 bytes) and the number of outer rounds; returns 1 if it converged
API int hc_bingcd(int which, const uint8_t *x, uint8_t *out, int *rounds) {
  fe a, r;
  for (int i = 0; i < 8; i++) {
    const uint8_t *q = x + 28 - 4 * i;
    a.l[i] = (uint32_t)q[0] << 24 | (uint32_t)q[1] << 16 | (uint32_t)q[2] << 8 | q[3];
  }
  bool ok = which == 0 ? bingcd::inverse<FpP>(a, r, rounds) : bingcd::inverse<FpR>(a, r, rounds);
  for (int i = 0; i < 8; i++) {
    uint8_t *q = out + 28 - 4 * i;
    q[0] = (uint8_t)(r.l[i] >> 24); q[1] = (uint8_t)(r.l[i] >> 16); q[2] = (uint8_t)(r.l[i] >> 8); q[3] = (uint8_t)r.l[i];
  }
  return ok ? 1 : 0;
}

// op: 0 add 1 sub 2 mul 3 inv(Fermat) 4 inv(binary) 5 half
API int hc_field(int which, int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  if (which == 0) {
    fe x = rd<FpP>(a), y = rd<FpP>(b), z;
    switch (op) {
      case 0: z = fp_add(x, y); break;
      case 1: z = fp_sub(x, y); break;
      case 2: z = fp_mul(x, y); break;
      case 3: z = fp_inv(x); break;
      case 4: z = fp_inv_fast(x); break;
      case 5: z = fp_half(x); break;
      default: return -1;
    }
    wr<FpP>(out, z);
  } else {
    fe x = rd<FpR>(a), y = rd<FpR>(b), z;
    switch (op) {
      case 0: z = fr_add(x, y); break;
      case 1: z = fr_sub(x, y); break;
      case 2: z = fr_mul(x, y); break;
      case 3: z = fr_inv(x); break;
      case 4: z = fr_inv_fast(x); break;
      case 5: z = f_half<FpR>(x); break;
      default: return -1;
    }
    wr<FpR>(out, z);
  }
  return 0;
}

// op: 0 mul 1 sqr 2 inv 3 final_exp 4 frob1 5 frob2 6 frob3 7 cyclo_sqr 8 cyclo_pow_u
API int hc_fp12(int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  fp12 x = rd12(a), y = rd12(b), z;
  switch (op) {
    case 0: z = f12_mul(x, y); break;
    case 1: z = f12_sqr(x); break;
    case 2: z = f12_inv(x); break;
    case 3: z = f12_final_exp(x); break;
    case 4: z = f12_frob1(x); break;
    case 5: z = f12_frob2(x); break;
    case 6: z = f12_frob3(x); break;
    case 7: z = f12_cyclo_sqr(x); break;
    case 8: z = f12_cyclo_pow_u(x); break;
    default: return -1;
  }
  wr12(out, z);
  return 0;
}

API int hc_fp2(int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  fp2 x = rd2(a), y = rd2(b), z;
  switch (op) {
    case 0: z = f2_mul(x, y); break;
    case 1: z = f2_sqr(x); break;
    case 2: z = f2_inv(x); break;
    case 3: z = f2_mul_xi(x); break;
    default: return -1;
  }
  wr2(out, z);
  return 0;
}

// op: 0 add 1 dbl 2 scalar mul (k canonical BE in b) 3 madd
API int hc_g1(int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  g1_aff P = rdg1(a);
  if (op == 2) {
    uint32_t k[8];
    canon_scalar(k, b);
    wrg1(out, jac_to_aff(scalar_mul(P, k)));
    return 0;
  }
  g1_aff Q = rdg1(b);
  if (op == 0) wrg1(out, jac_to_aff(jac_add(jac_from_aff(P), jac_from_aff(Q))));
  else if (op == 1) wrg1(out, jac_to_aff(jac_dbl(jac_from_aff(P))));
  else if (op == 3) wrg1(out, jac_to_aff(jac_madd(jac_from_aff(P), Q)));
  else return -1;
  return 0;
}

API int hc_g2(int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  g2_aff P = rdg2(a);
  if (op == 2) {
    uint32_t k[8];
    canon_scalar(k, b);
    wrg2(out, jac_to_aff(scalar_mul(P, k)));
    return 0;
  }
  if (op == 4) { wrg2(out, g2_frobenius(P)); return 0; }
  g2_aff Q = rdg2(b);
  if (op == 0) wrg2(out, jac_to_aff(jac_add(jac_from_aff(P), jac_from_aff(Q))));
  else if (op == 1) wrg2(out, jac_to_aff(jac_dbl(jac_from_aff(P))));
  else if (op == 3) wrg2(out, jac_to_aff(jac_madd(jac_from_aff(P), Q)));
  else return -1;
  return 0;
}

API int hc_pairing(const uint8_t *P, const uint8_t *Q, uint8_t *out) {
  wr12(out, f12_final_exp(miller_loop(rdg1(P), rdg2(Q))));
  return 0;
}

API void hc_h2f(const char *dst, const uint8_t *msg, uint64_t len, uint8_t *out) {
  sha::Hasher h;
  sha::xmd_begin(h);
  h.bytes(msg, (int)len);
  wr<FpR>(out, sha::xmd_finish_fr(h, dst));
}

// the cooperative form used by the challenge kernels (one lane here): msg (len bytes, at
// most 1024) after Z_pad
API void hc_h2f_coop(const char *dst, const uint8_t *msg, uint64_t len, uint8_t *out) {
  static uint32_t w[16 + 256 + 32], t2[16];
  for (int i = 0; i < 16; i++) w[i] = 0;
  for (uint64_t i = 0; i < len; i++) sha::put_byte(w, 64 + (uint32_t)i, msg[i]);
  wr<FpR>(out, sha::xmd_fr_coop(sha::Coop{0, 1}, w, (uint32_t)len, dst, t2));
}

// SHA-256 through the cooperative form (len at most 1024)
API void hc_sha256_coop(const uint8_t *msg, uint64_t len, uint8_t *out) {
  static uint32_t w[256 + 32];
  for (uint64_t i = 0; i < len; i++) sha::put_byte(w, (uint32_t)i, msg[i]);
  uint32_t o[8];
  sha::sha_coop(sha::Coop{0, 1}, w, (uint32_t)len, o);
  for (int i = 0; i < 8; i++) {
    out[4 * i] = o[i] >> 24; out[4 * i + 1] = o[i] >> 16; out[4 * i + 2] = o[i] >> 8; out[4 * i + 3] = o[i];
  }
}

API void hc_sha256(const uint8_t *msg, uint64_t len, uint8_t *out) {
  sha::Hasher h;
  h.init();
  h.bytes(msg, (int)len);
  uint32_t o[8];
  h.final(o);
  for (int i = 0; i < 8; i++) { out[4 * i] = o[i] >> 24; out[4 * i + 1] = o[i] >> 16; out[4 * i + 2] = o[i] >> 8; out[4 * i + 3] = o[i]; }
}

API void hc_merkle_leaf(const uint8_t m[32], const uint8_t c[64], uint8_t out[32]) {
  uint32_t mw[8], cw[16], o[8];
  for (int i = 0; i < 8; i++) mw[i] = ((uint32_t)m[4 * i] << 24) | ((uint32_t)m[4 * i + 1] << 16) | ((uint32_t)m[4 * i + 2] << 8) | m[4 * i + 3];
  for (int i = 0; i < 16; i++) cw[i] = ((uint32_t)c[4 * i] << 24) | ((uint32_t)c[4 * i + 1] << 16) | ((uint32_t)c[4 * i + 2] << 8) | c[4 * i + 3];
  sha::merkle_leaf(o, mw, cw);
  for (int i = 0; i < 8; i++) { out[4 * i] = o[i] >> 24; out[4 * i + 1] = o[i] >> 16; out[4 * i + 2] = o[i] >> 8; out[4 * i + 3] = o[i]; }
}

API void hc_merkle_node(const uint8_t l[32], const uint8_t r[32], uint8_t out[32]) {
  uint32_t lw[8], rw[8], o[8];
  for (int i = 0; i < 8; i++) {
    lw[i] = ((uint32_t)l[4 * i] << 24) | ((uint32_t)l[4 * i + 1] << 16) | ((uint32_t)l[4 * i + 2] << 8) | l[4 * i + 3];
    rw[i] = ((uint32_t)r[4 * i] << 24) | ((uint32_t)r[4 * i + 1] << 16) | ((uint32_t)r[4 * i + 2] << 8) | r[4 * i + 3];
  }
  sha::merkle_node(o, lw, rw);
  for (int i = 0; i < 8; i++) { out[4 * i] = o[i] >> 24; out[4 * i + 1] = o[i] >> 16; out[4 * i + 2] = o[i] >> 8; out[4 * i + 3] = o[i]; }
}


// ---- the wave-cooperative engine's programs through the host model of the interpreter
static void ld_consts(slp::f29 *S, int base, const uint32_t (*C)[9], int n) {
  for (int c = 0; c < n; c++) {
    for (int j = 0; j < 9; j++) S[base + c].l[j] = C[c][j];
    S[base + c].l[9] = S[base + c].l[10] = S[base + c].l[11] = 0;
  }
}

// Miller loop of the engine (before the final exponentiation)
API int hc_slp_miller(const uint8_t *P, const uint8_t *Q, uint8_t *out) {
  static slp::f29 S[slp::ML_NSLOT];
  g1_aff p = rdg1(P);
  g2_aff q = rdg2(Q);
  const fe in[6] = {p.x, p.y, q.x.c0, q.x.c1, q.y.c0, q.y.c1};
  for (int k = 0; k < 6; k++) S[slp::ML_xP + k] = slp::to29(in[k]);
  ld_consts(S, slp::ML_CBASE, slp::ML_CONSTS, slp::ML_NCONST);
  for (int s = 0; s < slp::ML_SEQ_LEN; s++) slp::run_host(S, slp::ML_SEQ[s][0], 0, 0, 0);
  fp12 f;
  fe *fw = reinterpret_cast<fe *>(&f);
  for (int k = 0; k < 12; k++) fw[k] = slp::from29(slp::canon29(S[slp::ML_f_0 + k]));
  wr12(out, f);
  return 0;
}

// final exponentiation (op 0) or F_p12 product of a and b (op 1) on the engine
API int hc_slp_f12(int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  static slp::f29 S[slp::FE_NSLOT + 12 * slp::FE_NBUF];
  auto buf = [](int k) { return slp::FE_NSLOT + 12 * k; };
  fp12 x = rd12(a), y = rd12(b);
  const fe *xw = reinterpret_cast<const fe *>(&x), *yw = reinterpret_cast<const fe *>(&y);
  for (int k = 0; k < 12; k++) { S[buf(0) + k] = slp::to29(xw[k]); S[buf(1) + k] = slp::to29(yw[k]); }
  ld_consts(S, slp::FE_CBASE, slp::FE_CONSTS, slp::FE_NCONST);
  int res;
  if (op == 1) {
    slp::run_host(S, slp::PROG_F12_MUL, buf(0), buf(1), buf(2));
    res = 2;
  } else {
    for (int e = 0; e < slp::FE_SEQ_LEN; e++) {
      int prog = slp::FE_SEQ[e][0];
      if (prog == slp::PROG_INV) { S[slp::FE_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::FE_t])))); continue; }
      slp::run_host(S, prog, buf(slp::FE_SEQ[e][1]), buf(slp::FE_SEQ[e][2]), buf(slp::FE_SEQ[e][3]));
    }
    res = slp::FE_RESULT;
  }
  fp12 f;
  fe *fw = reinterpret_cast<fe *>(&f);
  for (int k = 0; k < 12; k++) fw[k] = slp::from29(slp::canon29(S[buf(res) + k]));
  wr12(out, f);
  return 0;
}


// radix-2^29 lane arithmetic on raw integers (big-endian 32 bytes, below 2p):
// op 0: sum_i k_i x_i mod p (reduced to [0, 2p), then canonical); op 1: Montgomery
// product a b 2^{-261} (canonical); op 2: the raw almost-reduced linear combination
static fe rd_raw(const uint8_t *b) {
  fe a;
  for (int i = 0; i < 8; i++)
    a.l[7 - i] = ((uint32_t)b[4 * i] << 24) | ((uint32_t)b[4 * i + 1] << 16) | ((uint32_t)b[4 * i + 2] << 8) | b[4 * i + 3];
  return a;
}
static void wr_raw(uint8_t *b, const fe &a) {
  for (int i = 0; i < 8; i++) {
    uint32_t w = a.l[7 - i];
    b[4 * i] = w >> 24; b[4 * i + 1] = w >> 16; b[4 * i + 2] = w >> 8; b[4 * i + 3] = w;
  }
}
API int hc_slp_lane(int op, int n, const int *k, const uint8_t *xs, uint8_t *out) {
  if (op == 1) {
    slp::f29 r = slp::canon29(slp::mont29(slp::to29(rd_raw(xs)), slp::to29(rd_raw(xs + 32))));
    wr_raw(out, slp::from29(r));
    return 0;
  }
  // op 0/2: one offset (a product factor); op 3/4: twice the offset (a 16-term sum whose two
  // halves each start at it, as the interpreter's linear combinations)
  int64_t acc[9];
  for (int j = 0; j < 9; j++) acc[j] = (op >= 3 ? 2 : 1) * slp::OFF29[j];
  for (int i = 0; i < n; i++) {
    slp::f29 x = slp::to29(rd_raw(xs + 32 * i));
    for (int j = 0; j < 9; j++) acc[j] += (int64_t)k[i] * (int32_t)x.l[j];
  }
  slp::f29 r = slp::red29(acc);
  wr_raw(out, slp::from29(op == 2 || op == 4 ? r : slp::canon29(r)));
  return 0;
}


// ---- host model of the 8-lane field layout (field_wide.hpp), lane for lane: element limbs
// g = 0..7 as an array, the cross-lane steps written out (ds_swizzle broadcasts of limb k,
// DPP shifts by one limb, the ballot carry-lookahead).  Raw Montgomery limbs in and out, no
// conversions, so that the range of every output can be checked at the inputs' extremes and
// compared bit for bit with the device (vc_diag_field's raw modes).
namespace w8 {
struct V { uint32_t v[8]; };
static void shdn(const uint32_t *x, uint32_t *o) { for (int g = 0; g < 8; g++) o[g] = g < 7 ? x[g + 1] : 0u; }
static void shup(const uint32_t *x, uint32_t *o) { for (int g = 0; g < 8; g++) o[g] = g ? x[g - 1] : 0u; }
// carry into each lane from per-lane generate/propagate flags, and the carry out of lane 7,
// exactly as wchain(): C = ((g|p) + g) ^ (g|p) ^ g over the lanes 0..6, lane 7's own flags
// decide the carry out
static uint32_t g_active = 0xFF;  // lanes taking part in the ballots (all 8 in the library)
static void chain(const bool *gen, const bool *prop, uint32_t *cin, bool &out) {
  uint32_t G = 0, P = 0;
  for (int g = 0; g < 8; g++) { G |= (uint32_t)gen[g] << g; P |= (uint32_t)prop[g] << g; }
  G &= g_active;  // a ballot sees only active lanes
  P &= g_active;
  uint32_t gg = G & 0x7f, pp = P & 0x7f, a = gg | pp;
  uint32_t C = (a + gg) ^ a ^ gg;
  for (int g = 0; g < 8; g++) cin[g] = (C >> g) & 1u;
  out = (((G >> 7) & 1u) | (((P >> 7) & 1u) & ((C >> 7) & 1u))) != 0;
}
static void reduce(const uint32_t *M, const uint32_t *s, uint32_t *o) {  // s - m if s >= m
  bool gen[8], prop[8], bout;
  uint32_t bin[8];
  for (int g = 0; g < 8; g++) { gen[g] = s[g] < M[g]; prop[g] = s[g] == M[g]; }
  chain(gen, prop, bin, bout);
  for (int g = 0; g < 8; g++) o[g] = bout ? s[g] : s[g] - M[g] - bin[g];
}
static void add(const uint32_t *M, const uint32_t *a, const uint32_t *b, uint32_t *o) {
  uint32_t lo[8], cin[8], t[8];
  bool gen[8], prop[8], out;
  for (int g = 0; g < 8; g++) {
    uint64_t s = (uint64_t)a[g] + b[g];
    lo[g] = (uint32_t)s;
    gen[g] = (s >> 32) != 0;
    prop[g] = lo[g] == 0xFFFFFFFFu;
  }
  chain(gen, prop, cin, out);
  for (int g = 0; g < 8; g++) t[g] = lo[g] + cin[g];
  reduce(M, t, o);
}
static void sub(const uint32_t *M, const uint32_t *a, const uint32_t *b, uint32_t *o) {
  bool gen[8], prop[8], bout, out;
  uint32_t bin[8], d[8], lo[8], cin[8];
  for (int g = 0; g < 8; g++) { gen[g] = a[g] < b[g]; prop[g] = a[g] == b[g]; }
  chain(gen, prop, bin, bout);
  for (int g = 0; g < 8; g++) {
    d[g] = a[g] - b[g] - bin[g];
    uint64_t s = (uint64_t)d[g] + (bout ? M[g] : 0u);
    lo[g] = (uint32_t)s;
    gen[g] = (s >> 32) != 0;
    prop[g] = lo[g] == 0xFFFFFFFFu;
  }
  chain(gen, prop, cin, out);
  for (int g = 0; g < 8; g++) o[g] = lo[g] + cin[g];
}
static void mul(const uint32_t *M, uint32_t INV, const uint32_t *a, const uint32_t *b, uint32_t *o) {
  uint32_t t[8] = {0}, c[8] = {0};
  for (int j = 0; j < 8; j++) {
    uint64_t X[8], Y[8];
    uint32_t ylo[8], yd[8];
    for (int g = 0; g < 8; g++) X[g] = (uint64_t)a[g] * b[j] + t[g];
    uint32_t m = (uint32_t)X[0] * INV;
    for (int g = 0; g < 8; g++) { Y[g] = (uint64_t)m * M[g] + (uint32_t)X[g]; ylo[g] = (uint32_t)Y[g]; }
    shdn(ylo, yd);
    for (int g = 0; g < 8; g++) {
      uint64_t s = (uint64_t)yd[g] + (X[g] >> 32) + (Y[g] >> 32) + c[g];
      t[g] = (uint32_t)s;
      c[g] = (uint32_t)(s >> 32);
    }
  }
  uint32_t cu[8], lo[8], cin[8], r[8];
  bool gen[8], prop[8], out;
  shup(c, cu);
  for (int g = 0; g < 8; g++) {
    uint64_t f = (uint64_t)t[g] + cu[g];
    lo[g] = (uint32_t)f;
    gen[g] = (f >> 32) != 0;
    prop[g] = lo[g] == 0xFFFFFFFFu;
  }
  chain(gen, prop, cin, out);
  for (int g = 0; g < 8; g++) r[g] = lo[g] + cin[g];
  reduce(M, r, o);
}
}  // namespace w8

// the lanes of a group that take part in the ballots (0xFF: all; the library's kernels keep
// every group whole)
API void hc_wide_active(uint32_t mask) { w8::g_active = mask & 0xFF; }

// op 0 mul, 1 add, 2 sub on raw little-endian limbs (32 bytes each); which 0: p, 1: r
API int hc_wide_raw(int which, int op, const uint8_t *a, const uint8_t *b, uint8_t *out) {
  const uint32_t *M = which ? bn::R_MOD : bn::P_MOD;
  const uint32_t INV = which ? bn::R_INV : bn::P_INV;
  uint32_t x[8], y[8], z[8];
  memcpy(x, a, 32);
  memcpy(y, b, 32);
  switch (op) {
    case 0: w8::mul(M, INV, x, y, z); break;
    case 1: w8::add(M, x, y, z); break;
    case 2: w8::sub(M, x, y, z); break;
    default: return -1;
  }
  memcpy(out, z, 32);
  return 0;
}

// GLS decomposition of a canonical scalar (big-endian 32 bytes): out = 4 signed 128-bit
// two's-complement values (little-endian 16 bytes each) and the bit length
API int hc_gls(const uint8_t *kb, uint8_t *out, uint32_t *nbits) {
  fe k = rd_raw(kb);
  gls::Dec d = gls::decompose(k.l);
  for (int j = 0; j < 4; j++) {
    uint32_t m[4] = {d.mag[j][0], d.mag[j][1], d.mag[j][2], 0};
    if (d.neg >> j & 1) {
      uint64_t cy = 1;
      for (int w = 0; w < 4; w++) { uint64_t t = (uint64_t)(uint32_t)~m[w] + cy; m[w] = (uint32_t)t; cy = t >> 32; }
    }
    for (int w = 0; w < 4; w++)
      for (int b = 0; b < 4; b++) out[16 * j + 4 * w + b] = (uint8_t)(m[w] >> (8 * b));
  }
  *nbits = d.nbits;
  return 0;
}


// k Q + A on the engine's host model (A may be null); out affine (128 bytes, zeros = identity)
API int hc_g2_mul(const uint8_t *Qb, const uint8_t *kb, const uint8_t *Ab, uint8_t *out) {
  static slp::f29 S[slp::G2_NSLOT + 4];
  g2_aff Q = rdg2(Qb);
  const fe *q = reinterpret_cast<const fe *>(&Q);
  for (int i = 0; i < 4; i++) S[slp::G2_xQ_0 + i] = slp::to29(q[i]);
  bool has_a = false;
  if (Ab) {
    g2_aff A = rdg2(Ab);
    const fe *a = reinterpret_cast<const fe *>(&A);
    for (int i = 0; i < 4; i++) S[slp::G2_NSLOT + i] = slp::to29(a[i]);
    has_a = !aff_is_inf(A);
  }
  ld_consts(S, slp::G2_CBASE, slp::G2_CONSTS, slp::G2_NCONST);
  fe k = rd_raw(kb);
  gls::Dec dec = gls::decompose(k.l);
  slp::HostCtx c{S};
  bool inf = g2m::mul_add(c, dec, aff_is_inf(Q), has_a, slp::G2_NSLOT, S[slp::G2_CBASE + 1], S[slp::G2_CBASE]);
  if (inf) { memset(out, 0, 128); return 0; }
  c.run(slp::PROG_G2_NORM, 0, 0, 0);
  S[slp::G2_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::G2_t]))));
  c.run(slp::PROG_G2_AFF, 0, 0, 0);
  g2_aff r;
  fe *rw = reinterpret_cast<fe *>(&r);
  for (int i = 0; i < 4; i++) rw[i] = slp::from29(slp::canon29(S[slp::G2_ax_0 + i]));
  wrg2(out, r);
  return 0;
}


// k P (+ A) on the engine (host model), affine result; k canonical 32 bytes big-endian
API int hc_g1_mul_engine(const uint8_t *Pb, const uint8_t *kb, const uint8_t *Ab, uint8_t *out) {
  static slp::f29 S[slp::G1_NSLOT + 2];
  g1_aff P = rdg1(Pb);
  S[slp::G1_xP] = slp::to29(P.x);
  S[slp::G1_yP] = slp::to29(P.y);
  bool has_a = false;
  if (Ab) {
    g1_aff A = rdg1(Ab);
    S[slp::G1_NSLOT] = slp::to29(A.x);
    S[slp::G1_NSLOT + 1] = slp::to29(A.y);
    has_a = !aff_is_inf(A);
  }
  ld_consts(S, slp::G1_CBASE, slp::G1_CONSTS, slp::G1_NCONST);
  fe k = rd_raw(kb);
  glv::Dec dec = glv::decompose(k.l);
  slp::HostCtx c{S};
  bool inf = g1m::mul_add(c, dec, aff_is_inf(P), has_a, slp::G1_NSLOT, S[slp::G1_CBASE + 1]);
  if (inf) { memset(out, 0, 64); return 0; }
  S[slp::G1_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::G1_T_2]))));
  c.run(slp::PROG_G1_AFF, 0, 0, 0);
  g1_aff r{slp::from29(slp::canon29(S[slp::G1_ax])), slp::from29(slp::canon29(S[slp::G1_ay]))};
  wrg1(out, r);
  return 0;
}

// k P as the sum over t < 4 of chunk_t(k) (2^{32 t} P) on the engine (host model): the split
// used to run the four parts in parallel
API int hc_g1_mul_split(const uint8_t *Pb, const uint8_t *kb, uint8_t *out) {
  static slp::f29 S[slp::G1_NSLOT + 2];
  g1_aff P = rdg1(Pb);
  fe k = rd_raw(kb);
  glv::Dec dec = glv::decompose(k.l);
  g1_jac acc = jac_inf<OpsG1>();
  g1_jac Pt = jac_from_aff(P);
  for (int t = 0; t < 4; t++) {
    if (t)
      for (int i = 0; i < 32; i++) Pt = jac_dbl(Pt);
    g1_aff Pa = jac_to_aff(Pt);
    S[slp::G1_xP] = slp::to29(Pa.x);
    S[slp::G1_yP] = slp::to29(Pa.y);
    ld_consts(S, slp::G1_CBASE, slp::G1_CONSTS, slp::G1_NCONST);
    slp::HostCtx c{S};
    bool inf = g1m::mul_add(c, glv::chunk(dec, t), aff_is_inf(Pa), false, slp::G1_NSLOT, S[slp::G1_CBASE + 1]);
    if (!inf) {
      g1_jac part{slp::from29(slp::canon29(S[slp::G1_T_0])), slp::from29(slp::canon29(S[slp::G1_T_1])),
                  slp::from29(slp::canon29(S[slp::G1_T_2]))};
      acc = jac_add(acc, part);
    }
  }
  wrg1(out, jac_to_aff(acc));
  return 0;
}

// The split fold on the engine (host model), as the GPU runs it: multiples 2^{32 t} P by
// repeated double doublings, the four chunked multiplications into Jacobian partials, then
// their sum in the table slots plus A (affine; may be null or the identity).  Out affine.
API int hc_fold_split_g1(const uint8_t *Pb, const uint8_t *kb, const uint8_t *Ab, uint8_t *out) {
  static slp::f29 S[slp::G1_NSLOT + 2];
  g1_aff P = rdg1(Pb);
  fe k = rd_raw(kb);
  glv::Dec dec = glv::decompose(k.l);
  slp::HostCtx c{S};
  fe part[4][3];
  bool pinf[4];
  for (int t = 0; t < 4; t++) {
    ld_consts(S, slp::G1_CBASE, slp::G1_CONSTS, slp::G1_NCONST);
    g1_aff base = P;
    if (t && !aff_is_inf(P)) {
      S[slp::G1_T_0] = slp::to29(P.x);
      S[slp::G1_T_1] = slp::to29(P.y);
      S[slp::G1_T_2] = slp::to29(f_one<FpP>());
      for (int i = 0; i < 16 * t; i++) c.run(slp::PROG_G1_DBL2, 0, 0, 0);
      S[slp::G1_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::G1_T_2]))));
      c.run(slp::PROG_G1_AFF, 0, 0, 0);
      base = {slp::from29(slp::canon29(S[slp::G1_ax])), slp::from29(slp::canon29(S[slp::G1_ay]))};
    }
    S[slp::G1_xP] = slp::to29(base.x);
    S[slp::G1_yP] = slp::to29(base.y);
    pinf[t] = g1m::mul_add(c, glv::chunk(dec, t), aff_is_inf(base), false, slp::G1_NSLOT, S[slp::G1_CBASE + 1]);
    for (int q = 0; q < 3; q++)
      part[t][q] = pinf[t] ? (q < 2 ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[slp::G1_T_0 + q]));
  }
  for (int t = 0; t < 4; t++)
    for (int q = 0; q < 3; q++) S[slp::G1_TB1_0 + 3 * t + q] = slp::to29(part[t][q]);
  bool inf = true;
  for (int t = 0; t < 4; t++) g1m::add_jac(c, inf, slp::G1_TB1_0 + 3 * t, fe_is_zero(part[t][2]));
  if (Ab) {
    g1_aff A = rdg1(Ab);
    S[slp::G1_NSLOT] = slp::to29(A.x);
    S[slp::G1_NSLOT + 1] = slp::to29(A.y);
    if (!aff_is_inf(A)) g1m::add_affine(c, inf, slp::G1_NSLOT, S[slp::G1_CBASE + 1]);
  }
  if (inf) { memset(out, 0, 64); return 0; }
  S[slp::G1_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::G1_T_2]))));
  c.run(slp::PROG_G1_AFF, 0, 0, 0);
  g1_aff r{slp::from29(slp::canon29(S[slp::G1_ax])), slp::from29(slp::canon29(S[slp::G1_ay]))};
  wrg1(out, r);
  return 0;
}

// the same for G2: multiples 2^{16 t} Q, bits [16 t, 16 t + w_t) of the GLS split
API int hc_fold_split_g2(const uint8_t *Qb, const uint8_t *kb, const uint8_t *Ab, uint8_t *out) {
  static slp::f29 S[slp::G2_NSLOT + 4];
  g2_aff Q = rdg2(Qb);
  fe k = rd_raw(kb);
  gls::Dec dec = gls::decompose(k.l);
  slp::HostCtx c{S};
  fe part[4][6];
  for (int t = 0; t < 4; t++) {
    ld_consts(S, slp::G2_CBASE, slp::G2_CONSTS, slp::G2_NCONST);
    g2_aff base = Q;
    const fe *q = reinterpret_cast<const fe *>(&Q);
    if (t && !aff_is_inf(Q)) {
      for (int i = 0; i < 6; i++) S[slp::G2_T_0 + i] = slp::to29(i < 4 ? q[i] : i == 4 ? f_one<FpP>() : fe_zero());
      for (int i = 0; i < 16 * t; i++) c.run(slp::PROG_G2_DBL, 0, 0, 0);
      c.run(slp::PROG_G2_NORM, 0, 0, 0);
      S[slp::G2_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::G2_t]))));
      c.run(slp::PROG_G2_AFF, 0, 0, 0);
      fe *bw = reinterpret_cast<fe *>(&base);
      for (int i = 0; i < 4; i++) bw[i] = slp::from29(slp::canon29(S[slp::G2_ax_0 + i]));
    }
    const fe *bq = reinterpret_cast<const fe *>(&base);
    for (int i = 0; i < 4; i++) S[slp::G2_xQ_0 + i] = slp::to29(bq[i]);
    bool pinf = g2m::mul_add(c, gls::chunk(dec, 16 * t, t < 3 ? 16 : 17), aff_is_inf(base), false, slp::G2_NSLOT,
                             S[slp::G2_CBASE + 1], S[slp::G2_CBASE]);
    for (int i = 0; i < 6; i++)
      part[t][i] = pinf ? ((i == 0 || i == 2) ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[slp::G2_T_0 + i]));
  }
  for (int t = 0; t < 4; t++)
    for (int i = 0; i < 6; i++) S[slp::G2_TB1_0 + 6 * t + i] = slp::to29(part[t][i]);
  bool inf = true;
  for (int t = 0; t < 4; t++) g2m::add_jac(c, inf, slp::G2_TB1_0 + 6 * t, fe_is_zero(part[t][4]) && fe_is_zero(part[t][5]));
  if (Ab) {
    g2_aff A = rdg2(Ab);
    const fe *a = reinterpret_cast<const fe *>(&A);
    for (int i = 0; i < 4; i++) S[slp::G2_NSLOT + i] = slp::to29(a[i]);
    if (!aff_is_inf(A)) g2m::add_affine(c, inf, slp::G2_NSLOT, S[slp::G2_CBASE + 1], S[slp::G2_CBASE]);
  }
  if (inf) { memset(out, 0, 128); return 0; }
  c.run(slp::PROG_G2_NORM, 0, 0, 0);
  S[slp::G2_tinv] = slp::to29(fp_inv_fast(slp::from29(slp::canon29(S[slp::G2_t]))));
  c.run(slp::PROG_G2_AFF, 0, 0, 0);
  g2_aff r;
  fe *rw = reinterpret_cast<fe *>(&r);
  for (int i = 0; i < 4; i++) rw[i] = slp::from29(slp::canon29(S[slp::G2_ax_0 + i]));
  wrg2(out, r);
  return 0;
}

// g^k as the product over t < 4 of pow(g^{2^{16 t}}, chunk of bits [16 t, 16 t + w_t)) with
// w_t = 16 (t < 3) or 17, on the engine (host model)
API int hc_gt_pow_split(const uint8_t *gb, const uint8_t *kb, uint8_t *out) {
  static slp::f29 S[slp::FE_NSLOT + 12 * gtp::NBUF];
  fp12 g = rd12(gb), acc = f12_one();
  fe k = rd_raw(kb);
  gls::Dec dec = gls::decompose(k.l);
  const fe *gw = reinterpret_cast<const fe *>(&g);
  ld_consts(S, slp::FE_CBASE, slp::FE_CONSTS, slp::FE_NCONST);
  for (int i = 0; i < 12; i++) S[slp::FE_NSLOT + i] = slp::to29(gw[i]);
  slp::HostCtx c{S};
  const int b0 = slp::FE_NSLOT, b17 = slp::FE_NSLOT + 12 * 17;
  for (int t = 0; t < 4; t++) {
    if (t) {
      for (int i = 0; i < 16; i++) {
        slp::run_host(S, slp::PROG_F12_CSQR, b0, b0, b17);
        for (int q = 0; q < 12; q++) S[b0 + q] = S[b17 + q];
      }
    }
    slp::f29 base[12];
    for (int q = 0; q < 12; q++) base[q] = S[b0 + q];
    int r = gtp::pow_cyc(c, gls::chunk(dec, 16 * t, t < 3 ? 16 : 17), slp::FE_NSLOT);
    if (r >= 0) {
      fp12 part;
      fe *pw = reinterpret_cast<fe *>(&part);
      for (int q = 0; q < 12; q++) pw[q] = slp::from29(slp::canon29(S[slp::FE_NSLOT + 12 * r + q]));
      acc = f12_mul(acc, part);
    }
    for (int q = 0; q < 12; q++) S[b0 + q] = base[q];
  }
  wr12(out, acc);
  return 0;
}

// g^k on the engine (host model) for g in the cyclotomic subgroup, k canonical (32 bytes
// big-endian) through the 4-dimensional Frobenius split
API int hc_gt_pow_cyc(const uint8_t *gb, const uint8_t *kb, uint8_t *out) {
  static slp::f29 S[slp::FE_NSLOT + 12 * gtp::NBUF];
  fp12 g = rd12(gb);
  const fe *gw = reinterpret_cast<const fe *>(&g);
  for (int i = 0; i < 12; i++) S[slp::FE_NSLOT + i] = slp::to29(gw[i]);
  ld_consts(S, slp::FE_CBASE, slp::FE_CONSTS, slp::FE_NCONST);
  fe k = rd_raw(kb);
  gls::Dec dec = gls::decompose(k.l);
  slp::HostCtx c{S};
  int r = gtp::pow_cyc(c, dec, slp::FE_NSLOT);
  fp12 f;
  fe *fw = reinterpret_cast<fe *>(&f);
  for (int i = 0; i < 12; i++)
    fw[i] = r < 0 ? (i == 0 ? f_one<FpP>() : fe_zero()) : slp::from29(slp::canon29(S[slp::FE_NSLOT + 12 * r + i]));
  wr12(out, f);
  return 0;
}

// Montgomery products (MUL operations) in the engine's programs, for the work model
// (9.. : G1 phi + table, two doublings + addition, two doublings, mixed addition, to affine;
// cyclotomic squaring; the three Frobenius maps):
// 0 Miller loop (whole sequence), 1 final exponentiation (whole sequence, without the
// one-lane inversion), 2 G2 psi images, 3 G2 table, 4 G2 doubling, 5 G2 addition,
// 6 G2 mixed addition, 7 G2 to affine (norm + affine), 8 F_p12 product
static uint64_t prog_muls(int prog) {
  const slp::ProgDesc d = slp::PROGS[prog];
  uint64_t n = 0;
  for (uint32_t i = 0; i < (uint32_t)d.nlev * d.width; i++) n += (slp::OPS[d.off + i][0] & 3) == 1;
  return n;
}
API uint64_t hc_engine_muls(int which) {
  uint64_t n = 0;
  switch (which) {
    case 0: for (int s = 0; s < slp::ML_SEQ_LEN; s++) n += prog_muls(slp::ML_SEQ[s][0]); return n;
    case 1:
      for (int e = 0; e < slp::FE_SEQ_LEN; e++)
        if (slp::FE_SEQ[e][0] != slp::PROG_INV) n += prog_muls(slp::FE_SEQ[e][0]);
      return n;
    case 2: return prog_muls(slp::PROG_G2_PSI);
    case 3: return prog_muls(slp::PROG_G2_TABLE);
    case 4: return prog_muls(slp::PROG_G2_DBL);
    case 5: return prog_muls(slp::PROG_G2_ADD);
    case 6: return prog_muls(slp::PROG_G2_MADD);
    case 7: return prog_muls(slp::PROG_G2_NORM) + prog_muls(slp::PROG_G2_AFF);
    case 8: return prog_muls(slp::PROG_F12_MUL);
    case 9: return prog_muls(slp::PROG_G1_PHI) + prog_muls(slp::PROG_G1_TABLE);
    case 10: return prog_muls(slp::PROG_G1_DBL2_ADD);
    case 11: return prog_muls(slp::PROG_G1_DBL2);
    case 12: return prog_muls(slp::PROG_G1_MADD);
    case 13: return prog_muls(slp::PROG_G1_AFF);
    case 14: return prog_muls(slp::PROG_F12_CSQR);
    case 15: return prog_muls(slp::PROG_F12_FROB1) + prog_muls(slp::PROG_F12_FROB2) + prog_muls(slp::PROG_F12_FROB3);
    case 16: return prog_muls(slp::PROG_G1_ADD);
  }
  return 0;
}


// k P on G1 through the GLV split (host build of the device formulas); P, out affine BE
API int hc_g1_mul_glv(const uint8_t *Pb, const uint8_t *kb, uint8_t *out, uint8_t *dec_out) {
  fe k = rd_raw(kb);
  glv::Dec d = glv::decompose(k.l);
  if (dec_out) memcpy(dec_out, &d, sizeof d);
  wrg1(out, jac_to_aff(g1_mul_glv(rdg1(Pb), d)));
  return 0;
}

#ifdef VC_COUNT_MULS
// Field multiplications (F_p or F_r, Montgomery) performed by one operation of the
// GPU path's formulas: 0 Miller loop, 1 final exponentiation, 2 G1 scalar mul
// (254-bit scalar), 3 G2 scalar mul, 4 G1 add, 5 G1 mixed add, 6 G2 add, 7 G2 mixed
// add, 8 G1 doubling, 9 G2 doubling, 10 F_p12 mul, 11 Jacobian->affine G1 (excluding
// the binary-GCD inversion), 12 Jacobian->affine G2, 13 F_p12 squaring (general).
API uint64_t hc_count(int op) {
  uint8_t gb1[64], gb2[128];
  g1_aff G1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  g2_aff G2 = {{fe_const(bn::G2X0), fe_const(bn::G2X1)}, {fe_const(bn::G2Y0), fe_const(bn::G2Y1)}};
  (void)gb1; (void)gb2;
  uint32_t k[8] = {0x9e3779b9u, 0x7f4a7c15u, 0xf39cc060u, 0x5cedc834u, 0x1082276bu, 0xf3a27251u, 0xbe8e7a8bu, 0x2a9d0c3fu};
  g1_jac P1 = jac_dbl(jac_from_aff(G1));
  g2_jac P2 = jac_dbl(jac_from_aff(G2));
  g1_aff A1 = jac_to_aff(P1);
  g2_aff A2 = jac_to_aff(P2);
  fp12 f = miller_loop(G1, G2);
  uint64_t &c = fmul_counter();
  c = 0;
  switch (op) {
    case 0: (void)miller_loop(A1, A2); break;
    case 1: (void)f12_final_exp(f); break;
    case 2: (void)scalar_mul(G1, k); break;
    case 3: (void)scalar_mul(G2, k); break;
    case 4: (void)jac_add(P1, jac_dbl(P1)); break;
    case 5: (void)jac_madd(jac_dbl(P1), G1); break;
    case 6: (void)jac_add(P2, jac_dbl(P2)); break;
    case 7: (void)jac_madd(jac_dbl(P2), G2); break;
    case 8: (void)jac_dbl(P1); break;
    case 9: (void)jac_dbl(P2); break;
    case 10: (void)f12_mul(f, f); break;
    case 11: (void)jac_to_aff(P1); break;
    case 12: (void)jac_to_aff(P2); break;
    case 13: (void)f12_sqr(f); break;
    default: return 0;
  }
  uint64_t n = c;
  // subtract the set-up work done inside the measured expression
  c = 0;
  switch (op) {
    case 4: (void)jac_dbl(P1); break;
    case 5: (void)jac_dbl(P1); break;
    case 6: (void)jac_dbl(P2); break;
    case 7: (void)jac_dbl(P2); break;
    default: break;
  }
  return n - c;
}
#endif

// the index map of the terms taken one round ahead (oa_terms.hpp): term id as (a, v, out)
API void hc_oa_term(uint64_t id, uint64_t K, uint64_t nb, uint64_t q, uint64_t *out) {
  oat::Term t = oat::term(id, K, nb, q);
  out[0] = t.a;
  out[1] = t.v;
  out[2] = t.out;
}
