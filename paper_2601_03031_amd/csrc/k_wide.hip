// Kernels in the wide layout (field_wide.hpp): 8 lanes per field element, so one
// 64-lane block serves 8 independent Miller loops, scalar multiplications or point
// sums.  These are the dependent-chain kernels of the proof rounds, whose count of
// independent items per launch is far below the lane count of the chip.
//
// Memory layouts are the same as everywhere else (32-byte little-endian field
// elements, points as consecutive elements): lane g of a group loads limb g.
#define VC_WIDE 1
#include <hip/hip_runtime.h>
#include "field.hpp"
#include "tower.hpp"
#include "curve.hpp"
#include "pairing.hpp"
#include "kernels.h"
#include "oa_terms.hpp"
#include "gls.hpp"

#define TPBW 64
#define GPB (TPBW / 8)  // groups (elements) per block

namespace prof {
void begin(const char *name, hipStream_t st);
void end(hipStream_t st);
void name_last(const char *name);
}  // namespace prof
namespace dbg {
bool on();
void check(const char *name, hipStream_t st);
}  // namespace dbg

static inline unsigned nblkw(uint64_t n) { return (unsigned)((n + GPB - 1) / GPB); }
__device__ __forceinline__ uint64_t wgid() { return (uint64_t)blockIdx.x * GPB + (threadIdx.x >> 3); }

// element idx of a type made of n field elements, lane g taking limb g of each
template <class T> __device__ __forceinline__ T wld(const void *base, uint64_t idx) {
  constexpr int n = sizeof(T) / 4;
  T r;
  uint32_t *rv = reinterpret_cast<uint32_t *>(&r);
  const uint32_t *src = static_cast<const uint32_t *>(base) + idx * (uint64_t)n * 8 + wg();
#pragma unroll
  for (int k = 0; k < n; k++) rv[k] = src[k * 8];
  return r;
}
template <class T> __device__ __forceinline__ void wst(void *base, uint64_t idx, const T &v) {
  constexpr int n = sizeof(T) / 4;
  const uint32_t *rv = reinterpret_cast<const uint32_t *>(&v);
  uint32_t *dst = static_cast<uint32_t *>(base) + idx * (uint64_t)n * 8 + wg();
#pragma unroll
  for (int k = 0; k < n; k++) dst[k * 8] = rv[k];
}

// canonical limbs of a scalar (every lane of the group gets all 8)
__device__ __forceinline__ void wunpack(uint32_t k[8], const fe &c) {
  k[0] = wbcast<0>(c.v); k[1] = wbcast<1>(c.v); k[2] = wbcast<2>(c.v); k[3] = wbcast<3>(c.v);
  k[4] = wbcast<4>(c.v); k[5] = wbcast<5>(c.v); k[6] = wbcast<6>(c.v); k[7] = wbcast<7>(c.v);
}
__device__ __forceinline__ void wscalar(uint32_t k[8], const fe &mont) { wunpack(k, f_from_mont<FpR>(mont)); }
__device__ __forceinline__ bool scalar_is_zero(const uint32_t k[8]) {
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) t |= k[i];
  return t == 0;
}

// k P on G2 with the 4-dimensional split k = sum_j k_j lam^j (psi = the twisted Frobenius
// acts as lam = p mod r): bases B_j = sign(k_j) psi^j(P), a table of the 15 nonzero subset
// sums (Jacobian), then one doubling and at most one addition per bit of max |k_j| (65 bits)
__device__ __forceinline__ g2_jac g2_mul_gls(const g2_aff &P, const gls::Dec &d) {
  if (aff_is_inf(P) || d.nbits == 0) return jac_inf<OpsG2>();
  g2_aff B[4];
  B[0] = P;
  for (int j = 1; j < 4; j++) B[j] = g2_frobenius(B[j - 1]);
  for (int j = 0; j < 4; j++)
    if (d.neg >> j & 1) B[j] = aff_neg(B[j]);
  g2_jac T[16];
  T[0] = jac_inf<OpsG2>();
  for (int e = 1; e < 16; e++) {
    const int j = __builtin_ctz(e);  // the lowest set bit: T[e] = T[e without it] + B_j
    T[e] = (e & (e - 1)) ? jac_madd(T[e & (e - 1)], B[j]) : jac_from_aff(B[j]);
  }
  int t = (int)d.nbits - 1;
  g2_jac acc = T[gls::digit(d, (uint32_t)t)];
  for (t = t - 1; t >= 0; t--) {
    acc = jac_dbl(acc);
    uint32_t dg = gls::digit(d, (uint32_t)t);
    if (dg) acc = jac_add(acc, T[dg]);
  }
  return acc;
}

// scalar multiplication by a canonical scalar: GLV split on G1, GLS split on G2
__device__ __forceinline__ g1_jac mul_any(const g1_aff &P, const uint32_t kk[8]) { return g1_mul_glv(P, glv::decompose(kk)); }
__device__ __forceinline__ g2_jac mul_any(const g2_aff &P, const uint32_t kk[8]) { return g2_mul_gls(P, gls::decompose(kk)); }

// ---------------------------------------------------------------- scalar multiplications
template <class O>
__global__ void __launch_bounds__(TPBW) kw_mul(const void *P, int broadcast, const void *k, uint64_t n, void *out) {
  uint64_t i = wgid();
  if (i >= n) return;
  uint32_t kk[8];
  wscalar(kk, wld<fe>(k, i));
  wst(out, i, jac_to_aff(mul_any(wld<aff<O>>(P, broadcast ? 0 : i), kk)));
}

// terms of <A_R, b_L> (side 0) and <A_L, b_R> (side 1), Jacobian
__global__ void __launch_bounds__(TPBW) kw_oa_g1terms(const void *A, const void *B, uint64_t K, uint64_t nb, uint64_t h,
                                                     void *S) {
  uint64_t id = wgid();
  if (id >= nb * 2 * h) return;
  uint64_t k = id / (2 * h), r = id % (2 * h), side = r / h, i = r % h;
  fe c = wld<fe>(B, side ? k * K + h + i : k * K + i);
  g1_jac out = jac_inf<OpsG1>();
  if (!fe_is_zero(c)) {
    uint32_t kk[8];
    wscalar(kk, c);
    out = mul_any(wld<g1_aff>(A, side ? k * K + i : k * K + h + i), kk);
  }
  wst(S, (k * 2 + side) * (K / 2) + i, out);
}

// A_j = A_L o A_R^{x_j}, b_j = b_L + b_R / x_j; x_j enters through its GLV split (per batch);
// the folded arrays go to Aout, Bout (which may be Ain, Bin)
__global__ void __launch_bounds__(TPBW) kw_oa_fold_g1(const void *Ain, const void *Bin, void *Aout, void *Bout, const void *Xinv,
                                                     const glv::Dec *dec, uint64_t K, uint64_t nb, uint64_t h, uint32_t j,
                                                     uint32_t lK) {
  uint64_t id = wgid();
  if (id >= nb * h) return;
  uint64_t k = id / h, i = id % h, slot = k * lK + (j - 1);
  glv::Dec d = dec[k];
  g1_jac t = g1_mul_glv(wld<g1_aff>(Ain, k * K + h + i), d);
  g1_aff a = jac_to_aff(jac_madd(t, wld<g1_aff>(Ain, k * K + i)));
  fe bl = wld<fe>(Bin, k * K + i), br = wld<fe>(Bin, k * K + h + i);
  fe b = fr_add(bl, fr_mul(br, wld<fe>(Xinv, slot)));
  wst(Aout, k * K + i, a);
  wst(Bout, k * K + i, b);
}

// Miller values of the direct rounds on the wide layout, for rounds whose batches fill the
// device: the pairs of L_j (side 0: A[h + i] with V[i]) and R_j (side 1: A[i] with V[h + i]),
// C consecutive pairs per 8-lane group sharing one accumulator (one F_p12 squaring per step for
// the C pairs, each pair's lines multiplied in turn).  Product ch of batch k, side s goes to
// F[(2k + s) K/2 + ch], ch < h / C; it is the product of the C pairs' Miller values, which
// differ from the engine's only by factors the final exponentiation removes.
template <int C>
__global__ void __launch_bounds__(TPBW) kw_oa_miller(const void *A, const void *V, uint64_t K, uint64_t nb, uint64_t h,
                                                    void *F) {
  const uint64_t nch = h / C;
  uint64_t id = wgid();
  if (id >= nb * 2 * nch) return;
  uint64_t k = id / (2 * nch), r = id % (2 * nch), side = r / nch, ch = r % nch;
  g1_aff P[C];
  g2_aff Q[C];
  proj2 T[C];
  bool live[C];
#pragma unroll
  for (int c = 0; c < C; c++) {
    const uint64_t i = ch * C + c;
    P[c] = wld<g1_aff>(A, side ? k * K + i : k * K + h + i);
    Q[c] = wld<g2_aff>(V, side ? k * K + h + i : k * K + i);
    live[c] = !aff_is_inf(P[c]) && !aff_is_inf(Q[c]);  // a pair with the identity contributes 1
    T[c] = {Q[c].x, Q[c].y, f2_one()};
  }
  fp12 f = f12_one();
  fp2 l0, l1, l2;
  // over the non-adjacent form of 6u + 2 (d_65 = 1 starts T = Q; d_64 = 0): 21 additions of
  // +-Q against 36 for the binary digits
  for (int i = 64; i >= 0; i--) {
    if (i != 64) f = f12_sqr(f);
#pragma unroll
    for (int c = 0; c < C; c++)
      if (live[c]) {
        miller_dbl(T[c], P[c].x, P[c].y, l0, l1, l2);
        f = f12_mul_line(f, l0, l1, l2);
      }
    const bool pos = i < 64 && ((bn::ATE_NAF_POS >> i) & 1), neg = i < 64 && ((bn::ATE_NAF_NEG >> i) & 1);
    if (pos || neg) {
#pragma unroll
      for (int c = 0; c < C; c++)
        if (live[c]) {
          miller_add(T[c], pos ? Q[c] : aff_neg(Q[c]), P[c].x, P[c].y, l0, l1, l2);
          f = f12_mul_line(f, l0, l1, l2);
        }
    }
  }
#pragma unroll
  for (int c = 0; c < C; c++)
    if (live[c]) {
      g2_aff Q1 = g2_frobenius(Q[c]);
      g2_aff Q2 = aff_neg(g2_frobenius(Q1));
      miller_add(T[c], Q1, P[c].x, P[c].y, l0, l1, l2);
      f = f12_mul_line(f, l0, l1, l2);
      miller_add(T[c], Q2, P[c].x, P[c].y, l0, l1, l2);
      f = f12_mul_line(f, l0, l1, l2);
    }
  wst(F, (k * 2 + side) * (K / 2) + ch, f);
}

// v_j = v_L o v_R^{1/x_j} (Eq. folding) on the wide layout: the direct rounds, where the batches
// fill the device and throughput decides; Vout may be Vin
__global__ void __launch_bounds__(TPBW) kw_oa_fold_g2(const void *Vin, void *Vout, const void *Xinv, uint64_t K,
                                                     uint64_t nb, uint64_t h, uint32_t j, uint32_t lK) {
  uint64_t id = wgid();
  if (id >= nb * h) return;
  uint64_t k = id / h, i = id % h, slot = k * lK + (j - 1);
  uint32_t kk[8];
  wscalar(kk, wld<fe>(Xinv, slot));
  g2_jac t = mul_any(wld<g2_aff>(Vin, k * K + h + i), kk);
  wst(Vout, k * K + i, jac_to_aff(jac_madd(t, wld<g2_aff>(Vin, k * K + i))));
}

// HyperEval terms (canonical differences of the folded table g* times PST keys) of every job:
// term r of level d of job x goes to S[(d G + x) M / 2 + r]
__global__ void __launch_bounds__(TPBW) kw_hyper_terms(const S2Job *J, uint32_t G, uint64_t K, const void *ek, uint64_t M,
                                                      uint32_t lM, void *S) {
  uint64_t id = wgid();
  uint64_t per = M / 2;
  if (id >= G * lM * per) return;
  const uint64_t x = id / (lM * per);
  // g*, the root row of the y-tree, as an element offset (fe here is one limb per lane)
  const void *g = J[x].Y;
  const uint64_t g0 = (2 * K - 2) * M;
  id %= lM * per;
  uint32_t d = (uint32_t)(id / per);
  uint64_t r = id % per;
  uint32_t k = lM - d;
  uint64_t half = 1ull << (k - 1);
  uint64_t p = r / half, c = r % half;
  fe q = fr_sub(wld<fe>(g, g0 + p * (2 * half) + half + c), wld<fe>(g, g0 + p * (2 * half) + c));
  g1_jac out = jac_inf<OpsG1>();
  if (!fe_is_zero(q)) {
    uint32_t kk[8];
    wunpack(kk, q);
    out = mul_any(wld<g1_aff>(ek, (1ull << (k - 1)) - 1 + c), kk);
  }
  wst(S, (d * G + x) * per + r, out);
}

// W of every job at level d: segment s = x 2^d + p (reduced at in + s stride) is W_x[2^d - 1 + p]
__global__ void __launch_bounds__(TPBW) kw_w_aff(const S2Job *J, uint32_t G, const void *in, uint64_t stride, uint32_t d) {
  uint64_t s = wgid();
  if (s >= ((uint64_t)G << d)) return;
  const uint64_t x = s >> d, p = s & ((1ull << d) - 1);
  g1_aff a = jac_to_aff(wld<g1_jac>(in, s * stride));
  wst(J[x].W, (1ull << d) - 1 + p, a);
}

// the D-tree's leaves D_j = rho_j C_j of every job
__global__ void __launch_bounds__(TPBW) kw_d_leaves(const S2Job *J, uint32_t G, uint64_t K) {
  uint64_t id = wgid();
  if (id >= G * K) return;
  const S2Job &jb = J[id / K];
  const uint64_t j = id % K;
  uint32_t kk[8];
  wscalar(kk, wld<fe>(jb.rho, j));
  wst(jb.D, j, jac_to_aff(mul_any(wld<g1_aff>(jb.Cj, j), kk)));
}

// ---------------------------------------------------------------- sums
template <class O>
__global__ void __launch_bounds__(TPBW) kw_jac_step(void *data, uint64_t nseg, uint64_t stride, uint64_t len, uint64_t s) {
  uint64_t per = (len + 2 * s - 1) / (2 * s);
  uint64_t id = wgid();
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  uint64_t a = 2 * s * q, b = a + s;
  if (b >= len) return;
  jac<O> x = wld<jac<O>>(data, g * stride + a), y = wld<jac<O>>(data, g * stride + b);
  wst(data, g * stride + a, jac_add(x, y));
}

template <class O>
__global__ void __launch_bounds__(TPBW) kw_jac_to_aff(const void *in, uint64_t stride, uint64_t n, void *out,
                                                     uint64_t ostride) {
  uint64_t i = wgid();
  if (i >= n) return;
  wst(out, i * ostride, jac_to_aff(wld<jac<O>>(in, i * stride)));
}

// out[s] = affine(sum_{q < len} data[s len + q])
__global__ void __launch_bounds__(TPBW) kw_sum_g1(const void *data, uint64_t nseg, uint64_t len, void *out) {
  uint64_t s = wgid();
  if (s >= nseg) return;
  g1_jac acc = wld<g1_jac>(data, s * len);
  for (uint64_t q = 1; q < len; q++) acc = jac_add(acc, wld<g1_jac>(data, s * len + q));
  wst(out, s, jac_to_aff(acc));
}

// C_j of every job of a batched commit: the sum of its nslice MSM block results, affine, into
// the job's commitment and into the packed array Cp (entry k0 + j)
__global__ void __launch_bounds__(TPBW) kw_commit_sums(const CJob *J, uint32_t n, uint64_t total, void *Cp) {
  uint64_t i = wgid();
  if (i >= total) return;
  uint32_t lo = 0, hi = n;  // the job holding packed entry i
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (J[mid].k0 <= i) lo = mid;
    else hi = mid;
  }
  const CJob &c = J[lo];
  const uint64_t j = i - c.k0;
  g1_jac acc = wld<g1_jac>(c.part, j * c.nslice);
  for (uint64_t q = 1; q < c.nslice; q++) acc = jac_add(acc, wld<g1_jac>(c.part, j * c.nslice + q));
  g1_aff a = jac_to_aff(acc);
  wst(c.Cj, j, a);
  wst(Cp, i, a);
}

__global__ void __launch_bounds__(TPBW) kw_dlevel(const S2Job *J, uint32_t G, uint64_t K, uint32_t h) {
  uint64_t w = wgid();
  if (w >= G * (K >> h)) return;
  g1_aff *D = J[w / (K >> h)].D;
  w %= K >> h;
  uint64_t off = 2 * K - ((2 * K) >> h), offc = 2 * K - ((2 * K) >> (h - 1));
  g1_aff l = wld<g1_aff>(D, offc + 2 * w), r = wld<g1_aff>(D, offc + 2 * w + 1);
  wst(D, off + w, jac_to_aff(jac_madd(jac_from_aff(l), r)));
}


// ---------------------------------------------------------------- diagnostics
// field operation on canonical inputs (limbs), for the layout self-test:
// op 0 mul, 1 add, 2 sub, 3 half, 4 inverse, 5 square; F_p if which == 0, F_r if 1;
// which 2 (F_p) / 3 (F_r): ops 0-2 on raw Montgomery limbs, no conversion either way
__global__ void __launch_bounds__(TPBW) kw_diag_field(int which, int op, const void *a, const void *b, uint64_t n,
                                                     void *out) {
  uint64_t i = wgid();
  if (i >= n) return;
  fe x = wld<fe>(a, i), y = wld<fe>(b, i), r;
  if (which >= 2) {
    // raw Montgomery limbs in and out (ops 0 mul, 1 add, 2 sub), to check the range of results
    if (which == 2) r = op == 0 ? f_mul<FpP>(x, y) : op == 1 ? f_add<FpP>(x, y) : f_sub<FpP>(x, y);
    else r = op == 0 ? f_mul<FpR>(x, y) : op == 1 ? f_add<FpR>(x, y) : f_sub<FpR>(x, y);
  } else if (which == 0) {
    x = f_to_mont<FpP>(x);
    y = f_to_mont<FpP>(y);
    switch (op) {
      case 0: r = fp_mul(x, y); break;
      case 1: r = fp_add(x, y); break;
      case 2: r = fp_sub(x, y); break;
      case 3: r = fp_half(x); break;
      case 4: r = fp_inv(x); break;
      default: r = fp_sqr(x); break;
    }
    r = f_from_mont<FpP>(r);
  } else {
    x = f_to_mont<FpR>(x);
    y = f_to_mont<FpR>(y);
    switch (op) {
      case 0: r = fr_mul(x, y); break;
      case 1: r = fr_add(x, y); break;
      case 2: r = fr_sub(x, y); break;
      case 3: r = f_half<FpR>(x); break;
      case 4: r = fr_inv(x); break;
      default: r = f_sqr<FpR>(x); break;
    }
    r = f_from_mont<FpR>(r);
  }
  wst(out, i, r);
}

// ---------------------------------------------------------------- launchers
namespace klw {
#define LW(kern, n, ...)                                                                     \
  do {                                                                                       \
    prof::begin(#kern, st);                                                                  \
    hipLaunchKernelGGL(kern, dim3(nblkw(n)), dim3(TPBW), 0, st, __VA_ARGS__);                \
    prof::end(st);                                                                           \
    prof::name_last(#kern);                                                                  \
    if (dbg::on()) dbg::check(#kern, st);                                                    \
  } while (0)

void g1_mul(const void *P, int bc, const void *k, uint64_t n, void *out, hipStream_t st) {
  if (n) LW(kw_mul<OpsG1>, n, P, bc, k, n, out);
}
void g2_mul(const void *P, int bc, const void *k, uint64_t n, void *out, hipStream_t st) {
  if (n) LW(kw_mul<OpsG2>, n, P, bc, k, n, out);
}
void oa_g1terms(const void *A, const void *B, uint64_t K, uint64_t nb, uint64_t h, void *S, hipStream_t st) {
  LW(kw_oa_g1terms, nb * 2 * h, A, B, K, nb, h, S);
}
void oa_fold_g1(const void *Ain, const void *Bin, void *Aout, void *Bout, const void *Xinv, const void *dec, uint64_t K,
                uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st) {
  LW(kw_oa_fold_g1, nb * h, Ain, Bin, Aout, Bout, Xinv, static_cast<const glv::Dec *>(dec), K, nb, h, j, lK);
}
uint64_t oa_miller(const void *A, const void *V, uint64_t K, uint64_t nb, uint64_t h, void *F, hipStream_t st) {
  // two pairs per product when the round has pairs enough to keep the device full with half
  // as many groups (2^20, b = 1: 886 -> 810 ms), four from 2^19 pairs; fewer pairs keep one
  // pair per group, whose parallelism they need (2^16, b = 1: 93 ms with one, 104 with two)
  if (nb * 2 * h >= (1ull << 19) && h >= 4) {
    LW(kw_oa_miller<4>, nb * 2 * (h / 4), A, V, K, nb, h, F);
    return h / 4;
  }
  if (nb * 2 * h >= (1ull << 18) && h >= 2) {
    LW(kw_oa_miller<2>, nb * 2 * (h / 2), A, V, K, nb, h, F);
    return h / 2;
  }
  LW(kw_oa_miller<1>, nb * 2 * h, A, V, K, nb, h, F);
  return h;
}
void oa_fold_g2(const void *Vin, void *Vout, const void *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j,
                uint32_t lK, hipStream_t st) {
  LW(kw_oa_fold_g2, nb * h, Vin, Vout, Xinv, K, nb, h, j, lK);
}
void hyper_terms(const S2Job *J, uint32_t G, uint64_t K, const void *ek, uint64_t M, uint32_t lM, void *S, hipStream_t st) {
  LW(kw_hyper_terms, G * lM * (M / 2), J, G, K, ek, M, lM, S);
}
void w_aff(const S2Job *J, uint32_t G, const void *in, uint64_t stride, uint32_t d, hipStream_t st) {
  LW(kw_w_aff, (uint64_t)G << d, J, G, in, stride, d);
}
void d_leaves(const S2Job *J, uint32_t G, uint64_t K, hipStream_t st) {
  LW(kw_d_leaves, G * K, J, G, K);
}
void g1_reduce(void *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st) {
  for (uint64_t s = 1; s < len; s <<= 1) {
    uint64_t per = (len + 2 * s - 1) / (2 * s);
    LW(kw_jac_step<OpsG1>, nseg * per, data, nseg, stride, len, s);
  }
}
void g1_to_aff(const void *in, uint64_t stride, uint64_t n, void *out, uint64_t ostride, hipStream_t st) {
  LW(kw_jac_to_aff<OpsG1>, n, in, stride, n, out, ostride);
}
void sum_g1(const void *data, uint64_t nseg, uint64_t len, void *out, hipStream_t st) { LW(kw_sum_g1, nseg, data, nseg, len, out); }
void commit_sums(const CJob *J, uint32_t n, uint64_t total, void *Cp, hipStream_t st) {
  if (total) LW(kw_commit_sums, total, J, n, total, Cp);
}
void dlevel(const S2Job *J, uint32_t G, uint64_t K, uint32_t h, hipStream_t st) {
  LW(kw_dlevel, G * (K >> h), J, G, K, h);
}
void diag_field(int which, int op, const void *a, const void *b, uint64_t n, void *out, hipStream_t st) {
  LW(kw_diag_field, n, which, op, a, b, n, out);
}
}  // namespace klw
