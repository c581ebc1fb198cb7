// Kernels: G2: setup keys, fold of v, KZG proof terms.
#include "kcommon.hpp"


__global__ void __launch_bounds__(TPB) k_g2_mul(const g2_aff *P, int broadcast, const fe *k, uint64_t n, g2_aff *out) {
  uint64_t i = gtid();
  if (i >= n) return;
  uint32_t kk[8];
  canon_scalar(kk, k[i]);
  out[i] = jac_to_aff(scalar_mul(P[broadcast ? 0 : i], kk));
}

// v_j = v_L o v_R^{1/x_j}
__global__ void __launch_bounds__(TPB) k_oa_fold_g2(g2_aff *V, const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK) {
  uint64_t id = gtid();
  if (id >= nb * h) return;
  uint64_t k = id / h, i = id % h;
  uint32_t kk[8];
  canon_scalar(kk, Xinv[k * lK + (j - 1)]);
  g2_jac t = scalar_mul(V[k * K + h + i], kk);
  V[k * K + i] = jac_to_aff(jac_madd(t, V[k * K + i]));
}

// terms q_m h_m of pi_v
__global__ void __launch_bounds__(TPB) k_kzg_terms(const g2_aff *h, const fe *Q, uint64_t K, uint64_t nb, g2_jac *S) {
  uint64_t n = 2 * K - 2;
  uint64_t id = gtid();
  if (id >= nb * n) return;
  uint64_t m = id % n;
  uint32_t kk[8];
  canon_scalar(kk, Q[id]);
  S[id] = scalar_mul(h[m], kk);
}

namespace kl {
void g2_mul(const g2_aff *P, int bc, const fe *k, uint64_t n, g2_aff *out, hipStream_t st) { if (n) L1(k_g2_mul, n, P, bc, k, n, out); }
void g2_reduce(g2_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st) {
  for (uint64_t s = 1; s < len; s <<= 1) {
    uint64_t per = (len + 2 * s - 1) / (2 * s);
    L1(k_jac_step<OpsG2>, nseg * per, data, nseg, stride, len, s);
  }
}
void g2_to_aff(const g2_jac *in, uint64_t stride, uint64_t n, g2_aff *out, uint64_t ostride, hipStream_t st) {
  L1(k_jac_to_aff<OpsG2>, n, in, stride, n, out, ostride);
}
void oa_fold_g2(g2_aff *V, const fe *Xinv, uint64_t K, uint64_t nb, uint64_t h, uint32_t j, uint32_t lK, hipStream_t st) {
  L1(k_oa_fold_g2, nb * h, V, Xinv, K, nb, h, j, lK);
}
void kzg_terms(const g2_aff *h, const fe *Q, uint64_t K, uint64_t nb, g2_jac *S, hipStream_t st) {
  L1(k_kzg_terms, nb * (2 * K - 2), h, Q, K, nb, S);
}
}  // namespace kl
