// Kernels: pairings: Miller loops, F_p12 product trees, final exponentiation.
#include "kcommon.hpp"


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

namespace kl {
void miller(const g1_aff *P, uint64_t sp, const g2_aff *Q, uint64_t sq, uint64_t n, fp12 *out, hipStream_t st) {
  if (n) L1(k_miller, n, P, sp, Q, sq, n, out);
}
void f12_reduce(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st) {
  for (uint64_t s = 1; s < len; s <<= 1) {
    uint64_t per = (len + 2 * s - 1) / (2 * s);
    L1(k_f12_step, nseg * per, data, nseg, stride, len, s);
  }
}
void final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out, uint64_t ostride, hipStream_t st) {
  L1(k_final_exp, n, in, stride, n, out, ostride);
}
void oa_miller(const g1_aff *A, const g2_aff *V, uint64_t K, uint64_t nb, uint64_t h, fp12 *F, hipStream_t st) {
  L1(k_oa_miller, nb * 2 * h, A, V, K, nb, h, F);
}
}  // namespace kl
