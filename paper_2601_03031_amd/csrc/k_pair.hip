// Kernels: F_p12 product trees and the final exponentiation, one wavefront per F_p12 operation.
#include "kcommon.hpp"
#include "wave12.hpp"


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
void f12_reduce(fp12 *data, uint64_t nseg, uint64_t stride, uint64_t len, hipStream_t st) {
  for (uint64_t s = 1; s < len; s <<= 1) {
    uint64_t per = (len + 2 * s - 1) / (2 * s);
    LAUNCH(k_f12_step_wave, dim3((unsigned)(nseg * per)), dim3(WAVE12_T), 0, data, nseg, stride, len, s);
  }
}
void final_exp(const fp12 *in, uint64_t stride, uint64_t n, fp12 *out0, fp12 *out1, uint64_t ostride, hipStream_t st) {
  if (n) LAUNCH(k_final_exp_wave, dim3((unsigned)n), dim3(WAVE12_T), 0, in, stride, n, out0, out1, ostride);
}
}  // namespace kl
