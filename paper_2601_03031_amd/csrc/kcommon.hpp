#pragma once
// Shared prelude of the kernel translation units: layouts, launch helpers,
// domain tags and the generic segmented-reduction kernels.
//
// Layouts (all device arrays, little-endian 32-bit limbs):
//   fe        32 B  (Montgomery F_p or F_r, or a canonical F_r scalar where noted)
//   g1_aff    64 B  x, y            (identity = zeros)
//   g2_aff   128 B  x.c0 x.c1 y.c0 y.c1
//   fp12     384 B  c0.c0.c0 c0.c0.c1 c0.c1.c0 ... c1.c2.c1
//   g1_jac    96 B, g2_jac 192 B (scratch only)
// Per-batch state of the FC openings is stored batch-major with stride K.
#include <hip/hip_runtime.h>
#include "field.hpp"
#include "tower.hpp"
#include "curve.hpp"
#include "pairing.hpp"
#include "hash.hpp"
#include "kernels.h"

#define TPB 128

static inline unsigned nblk(uint64_t n, unsigned tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }
__device__ __forceinline__ uint64_t gtid() { return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Kernels on the dependent chain of rounds raise their waves' issue priority, so that
// waves of work taken ahead that share a SIMD with them yield to them: 3 for the pairing
// side, folds, combine and transcript, 2 for the multiples and the G1 side of the terms;
// Step 2 keeps the default.
#define CHAIN_PRIORITY() __builtin_amdgcn_s_setprio(3)
#define AHEAD_PRIORITY() __builtin_amdgcn_s_setprio(2)

#define DSTR_SETUP "FLEXPROOFS-V1-SETUP"
#define DSTR_FC_R "FLEXPROOFS-V1-FC-R"
#define DSTR_FC_X "FLEXPROOFS-V1-FC-X"
#define DSTR_FC_Z "FLEXPROOFS-V1-FC-Z"
#define DSTR_RHO "FLEXPROOFS-V1-RHO"
#define DSTR_VALL "FLEXPROOFS-V1-VERIFY-ALL"
#define DSTR_EVAL "FLEXPROOFS-V1-EVAL"

__device__ __forceinline__ void canon_scalar(uint32_t k[8], const fe &mont) {
  fe c = f_from_mont<FpR>(mont);
#pragma unroll
  for (int i = 0; i < 8; i++) k[i] = c.l[i];
}

// Sum of each segment data[g stride + 0 .. len) into data[g stride] in one launch: a thread per
// pair of the first level; of two sibling nodes, the one that finishes second climbs to the
// parent (arrival counters cnt[g tree_counters(len) + ...], zero before the launch and reset
// by their second arrival).
template <class O>
__global__ void __launch_bounds__(TPB) k_jac_tree(jac<O> *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt) {
  uint64_t per = (len + 1) / 2;
  uint64_t id = gtid();
  if (id >= nseg * per) return;
  uint64_t g = id / per, q = id % per;
  jac<O> *d = data + g * stride;
  uint32_t *c = cnt + g * tree_counters(len);
  uint64_t s = 1, n = per, cb = 0;
  for (;;) {
    uint64_t a = 2 * s * q, b = a + s;
    if (b < len) d[a] = jac_add(d[a], d[b]);
    if (n == 1) return;
    uint64_t nn = (n + 1) / 2, qp = q >> 1;
    if ((q ^ 1) < n) {
      __threadfence();
      uint32_t old = atomicAdd(&c[cb + qp], 1u);
      if (!old) return;
      c[cb + qp] = 0;
      __threadfence();
    }
    cb += nn;
    q = qp;
    n = nn;
    s *= 2;
  }
}
template <class O>
__global__ void __launch_bounds__(TPB) k_jac_to_aff(const jac<O> *in, uint64_t stride, uint64_t n, aff<O> *out, uint64_t ostride) {
  uint64_t i = gtid();
  if (i >= n) return;
  out[i * ostride] = jac_to_aff(in[i * stride]);
}
// optional per-kernel timing (HIP events on the launch stream), enabled through vc_profile_enable
namespace prof {
void begin(const char *name, hipStream_t st);
void end(hipStream_t st);
void name_last(const char *name);
}
namespace dbg {
// VC_DEBUG_SYNC=1 in the environment: synchronize after every launch and report the
// first failing kernel on stderr (diagnostics only)
bool on();
void check(const char *name, hipStream_t st);
}  // namespace dbg
#define LAUNCH(kern, grid, block, shm, ...)                                 \
  do {                                                                     \
    prof::begin(#kern, st);                                                \
    hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);           \
    prof::end(st);                                                         \
    prof::name_last(#kern);                                                \
    if (dbg::on()) dbg::check(#kern, st);                                  \
  } while (0)
#define L1(kern, n, ...) LAUNCH(kern, dim3(nblk(n)), dim3(TPB), 0, __VA_ARGS__)
