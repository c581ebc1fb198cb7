// Kernels: pairings: Miller loops, F_p12 product trees, final exponentiation.
#include "kcommon.hpp"
#include "wave12.hpp"


// ================================================================ pairing helpers
// out[i] = Miller(P[i*sp], Q[i*sq])
__global__ void __launch_bounds__(TPB) k_miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n, fp12 *out) {
  uint64_t i = gtid();
  if (i >= n) return;
  out[i] = miller_loop(P[i * sp], Q[i * sq]);
}

// one tree step over nseg segments: data[g*stride + 2 s q] *= data[g*stride + 2 s q + s]
__global__ void __launch_bounds__(TPB) k_f12_step(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, uint64_t s) {
  uint64_t per = (len + 2 * s - 1) / (2 * s);
  uint64_t id = gtid();
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  uint64_t a = 2 * s * q, b = a + s;
  if (b >= len) return;
  fp12 *d = data + g * stride;
  d[a] = f12_mul(d[a], d[b]);
}

__global__ void __launch_bounds__(TPB) k_final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out, uint64_t ostride) {
  uint64_t i = gtid();
  if (i >= n) return;
  out[i * ostride] = f12_final_exp(in[i * stride]);
}

// Miller values of both halves: side 0 (L) pairs A[h+i] with V[i], side 1 (R) A[i] with V[h+i]
__global__ void __launch_bounds__(TPB) k_oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h, fp12 *F) {
  uint64_t id = gtid();
  if (id >= nb * 2 * h) return;
  uint64_t k = id / (2 * h), r = id % (2 * h), side = r / h, i = r % h;
  const g1_aff &P = side ? A[k * K + i] : A[k * K + h + i];
  const g2_aff &Q = side ? V[k * K + h + i] : V[k * K + i];
  F[(k * 2 + side) * (K / 2) + i] = miller_loop(P, Q);
}

// Final exponentiation f^((p^12-1)/r), one wavefront per input (see wave12.hpp):
// easy part conj(f) f^{-1} then (.)^{p^2} (.), hard part through f^u, f^{u^2}, f^{u^3}
// and the p-power split of (p^4 - p^2 + 1)/r used by f12_final_exp.
// Input s is in[s * in_stride]; output goes to (s odd ? out1 : out0)[(s >> 1) * ostride].
#define FE_SLOTS 22
__global__ void __launch_bounds__(WAVE12_T) k_final_exp_wave(const fp12 *in, uint64_t in_stride, uint64_t n, fp12 *out0,
                                                             fp12 *out1, uint64_t ostride) {
  __shared__ fe S[FE_SLOTS * 12];
  __shared__ W12 w;
  uint64_t s = blockIdx.x;
  if (s >= n) return;
  int t = threadIdx.x;
#define SL(i) (S + 12 * (i))
  const fe *src = reinterpret_cast<const fe *>(in + s * in_stride);
  if (t < 12) SL(0)[t] = src[t];
  wsync();
  winv(SL(0), SL(1), SL(2), SL(3), w);       // f0^-1
  wconj(SL(0), SL(2));
  wmul(SL(2), SL(1), SL(4), w);              // f1 = conj(f0) f0^-1
  wfrob(SL(4), SL(5), 2);
  wmul(SL(5), SL(4), SL(5), w);              // f = f1^{p^2} f1, cyclotomic from here on
  wpow_u(SL(5), SL(6), w);                   // a = f^u
  wpow_u(SL(6), SL(7), w);                   // b = f^{u^2}
  wpow_u(SL(7), SL(8), w);                   // c = f^{u^3}
  wcsqr(SL(8), SL(9), w);
  wcsqr(SL(9), SL(9), w);
  wcsqr(SL(9), SL(9), w);                    // c^8
  wmul(SL(9), SL(8), SL(9), w);              // c^9
  wcsqr(SL(9), SL(9), w);
  wcsqr(SL(9), SL(9), w);                    // c^36
  wcsqr(SL(7), SL(10), w);
  wmul(SL(10), SL(7), SL(10), w);
  wcsqr(SL(10), SL(10), w);                  // b^6
  wcsqr(SL(10), SL(11), w);                  // b^12
  wmul(SL(11), SL(10), SL(12), w);           // b^18
  wmul(SL(12), SL(11), SL(13), w);           // b^30
  wcsqr(SL(6), SL(14), w);
  wmul(SL(14), SL(6), SL(14), w);
  wcsqr(SL(14), SL(14), w);                  // a^6
  wcsqr(SL(14), SL(15), w);                  // a^12
  wmul(SL(15), SL(14), SL(16), w);           // a^18
  wcsqr(SL(5), SL(17), w);                   // f^2
  wmul(SL(9), SL(13), SL(18), w);
  wmul(SL(16), SL(17), SL(19), w);
  wmul(SL(18), SL(19), SL(18), w);
  wconj(SL(18), SL(18));                     // t0 = f^{l0}
  wmul(SL(9), SL(12), SL(19), w);
  wmul(SL(19), SL(15), SL(19), w);
  wconj(SL(19), SL(19));
  wmul(SL(19), SL(5), SL(19), w);            // t1 = f^{l1}
  wmul(SL(10), SL(5), SL(20), w);            // t2 = f^{l2}
  wfrob(SL(19), SL(19), 1);
  wfrob(SL(20), SL(20), 2);
  wfrob(SL(5), SL(21), 3);
  wmul(SL(18), SL(19), SL(18), w);
  wmul(SL(20), SL(21), SL(20), w);
  wmul(SL(18), SL(20), SL(18), w);
  fp12 *o = (s & 1) ? out1 : out0;
  fe *dst = reinterpret_cast<fe *>(o + (s >> 1) * ostride);
  if (t < 12) dst[t] = SL(18)[t];
#undef SL
}

// one tree step with a wavefront per product: data[g*stride + 2sq] *= data[g*stride + 2sq + s]
__global__ void __launch_bounds__(WAVE12_T) k_f12_step_wave(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len,
                                                            uint64_t s) {
  __shared__ fe S[24];
  __shared__ W12 w;
  uint64_t per = (len + 2 * s - 1) / (2 * s);
  uint64_t id = blockIdx.x;
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  uint64_t a = 2 * s * q, b = a + s;
  if (b >= len) return;
  fe *da = reinterpret_cast<fe *>(data + g * stride + a);
  const fe *db = reinterpret_cast<const fe *>(data + g * stride + b);
  int t = threadIdx.x;
  if (t < 12) { S[t] = da[t]; S[12 + t] = db[t]; }
  wsync();
  wmul(S, S + 12, S, w);
  if (t < 12) da[t] = S[t];
}

namespace kl {
void miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n, fp12 *out, hipStream_t st) {
  if (n) L1(k_miller, n, P, sp, Q, sq, n, out);
}
void f12_reduce(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st) {
  for (uint64_t s = 1; s < len; s <<= 1) {
    uint64_t per = (len + 2 * s - 1) / (2 * s);
    LAUNCH(k_f12_step_wave, dim3((unsigned)(nseg * per)), dim3(WAVE12_T), 0, data, nseg, stride, len, s);
  }
}
void final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out0, fp12 *out1, uint64_t ostride, hipStream_t st) {
  if (n) LAUNCH(k_final_exp_wave, dim3((unsigned)n), dim3(WAVE12_T), 0, in, stride, n, out0, out1, ostride);
}
void oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h, fp12 *F, hipStream_t st) {
  L1(k_oa_miller, nb * 2 * h, A, V, K, nb, h, F);
}
}  // namespace kl
