// Kernels: G1: setup keys, commitment MSM, fold of A, fold tree, HyperEval, encoding.
// (the curve helpers are inlined here: passed by reference to out-of-line calls, the MSM's
// points went through scratch memory)
#define VC_INLINE_HELPERS 1
#include "kcommon.hpp"

#define MSM_MAXE 8192
#define MSM_G2_MAXE 8192  // S nwin for the G2 MSM (with its 256 Jacobian G2 points, 48 KB, 82 KB of LDS)

// weights of the Lagrange keys at every level: node n = 2^k - 1 + c holds eq_k(c; s)
__global__ void __launch_bounds__(TPB) k_ek_weights(uint32_t lM, const fe *s, fe *w, uint64_t n_total) {
  uint64_t n = gtid();
  if (n >= n_total) return;
  uint32_t k = 63 - __clzll(n + 1);
  uint64_t c = n + 1 - (1ull << k);
  fe acc = f_one<FpR>();
  for (uint32_t t = 0; t < k; t++) {
    fe f = ((c >> t) & 1) ? s[t] : fr_sub(f_one<FpR>(), s[t]);
    acc = fr_mul(acc, f);
  }
  w[n] = acc;
}

// out[k] = beta^k
__global__ void __launch_bounds__(TPB) k_pow_table(const fe *beta, fe *out, uint64_t n) {
  uint64_t k = gtid();
  if (k >= n) return;
  fe acc = f_one<FpR>(), b = *beta;
  for (int i = 63 - __clzll(k | 1); i >= 0; i--) {
    acc = fr_mul(acc, acc);
    if ((k >> i) & 1) acc = fr_mul(acc, b);
  }
  out[k] = acc;
}

// table[w M + a] = 2^{8w} base[a] for w < nwin
template <class O>
__global__ void __launch_bounds__(TPB) k_msm_tables(const aff<O> *base, uint64_t M, uint32_t nwin, aff<O> *table) {
  uint64_t a = gtid();
  if (a >= M) return;
  jac<O> acc = jac_from_aff(base[a]);
  table[a] = base[a];
  for (uint32_t w = 1; w < nwin; w++) {
    for (int d = 0; d < 8; d++) acc = jac_dbl(acc);
    table[(uint64_t)w * M + a] = jac_to_aff(acc);
  }
}

// out[i] = in[i] out of Montgomery form (F_r)
__global__ void __launch_bounds__(TPB) k_fr_canon(const fe *in, uint64_t n, fe *out) {
  uint64_t i = gtid();
  if (i >= n) return;
  out[i] = f_from_mont<FpR>(in[i]);
}

// ================================================================ commit
__global__ void __launch_bounds__(TPB) k_lift_u32(const uint32_t *in, uint64_t n, fe *out) {
  uint64_t i = gtid();
  if (i >= n) return;
  fe v = fe_zero();
  v.l[0] = in[i];
  out[i] = v;
}

// Throughput probe of the 32 x 32 -> 64-bit multiply-add that the Montgomery products are
// built from (v_mad_u64_u32): every lane runs 8 independent chains of `iters` steps
// x <- lo(x) * b + x (one instruction, no moves); the results are stored so that no chain
// is dropped.
__global__ void __launch_bounds__(256) k_diag_mad(uint32_t seed, uint32_t iters, uint64_t *out) {
  uint32_t a = seed ^ (uint32_t)gtid();
  uint32_t b = a * 2654435761u + 12345u;
  uint64_t x[8];
#pragma unroll
  for (int k = 0; k < 8; k++) x[k] = a + 977u * k;
  for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
    for (int k = 0; k < 8; k++) x[k] = (uint64_t)(uint32_t)x[k] * b + x[k];
  }
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) r ^= x[k];
  out[gtid()] = r;
}

// plain zero fill: flags and arrival counters that must start at zero (a kernel, so that a
// caller capturing the launches in a graph records no memset node)
__global__ void __launch_bounds__(TPB) k_zero_u32(uint32_t *p, uint64_t n) {
  uint64_t i = gtid();
  if (i < n) p[i] = 0;
}

__global__ void __launch_bounds__(TPB) k_check_fr(const fe *m, uint64_t n, int *err) {
  uint64_t i = gtid();
  if (i >= n) return;
  if (!fe_lt_mod(m[i], bn::R_MOD)) atomicOr(err, VC_ERRBIT_RANGE);
}

// canonical 32-byte big-endian F_p encodings -> Montgomery form; a value >= p sets the range
// bit (and is stored as zero)
__global__ void __launch_bounds__(TPB) k_decode_fp(const uint8_t *in, uint64_t n, fe *out, int *err) {
  uint64_t i = gtid();
  if (i >= n) return;
  fe c;
  const uint8_t *b = in + 32 * i;
  for (int q = 0; q < 8; q++)
    c.l[7 - q] = ((uint32_t)b[4 * q] << 24) | ((uint32_t)b[4 * q + 1] << 16) | ((uint32_t)b[4 * q + 2] << 8) | b[4 * q + 3];
  if (!fe_lt_mod(c, bn::P_MOD)) {
    atomicOr(err, VC_ERRBIT_RANGE);
    c = fe_zero();
  }
  out[i] = f_to_mont<FpP>(c);
}

// points off the curve (G1: y^2 = x^3 + 3; G2: the twist) set the range bit
template <class O>
__global__ void __launch_bounds__(TPB) k_check_curve(const aff<O> *p, uint64_t n, int *err) {
  uint64_t i = gtid();
  if (i >= n) return;
  if (!aff_on_curve(p[i])) atomicOr(err, VC_ERRBIT_RANGE);
}

// Batched MSM with shared bases: C_j = sum_a m[jM+a] ek[a] (canonical scalars).  Block
// (j, slice) handles bases [slice*S, (slice+1)*S); every (base, window) pair with a nonzero
// 8-bit digit is counting-sorted by digit in LDS, thread d sums bucket d over the
// precomputed table points 2^{8w} ek[a], and the block reduces sum_d d B_d with a suffix
// scan.  S nwin <= MSM_MAXE (G1), MSM_G2_MAXE (G2).  (A tree over bucket ranges that merges
// (S, W) pairs with doublings does a quarter of the scan's additions but measured slower:
// with one block per CU at N = 2^16 the block's latency sets the time, and its doubling
// chains are longer than the scan's eight steps.)  One (j, slice) block: blk = j nslice + slice.
template <class O>
__device__ __forceinline__ void msm_slice(const fe *scal, uint64_t M, uint32_t nwin, uint32_t S, const aff<O> *table,
                                          jac<O> *partial, uint64_t blk) {
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t off[256];
  constexpr uint32_t MAXE = sizeof(typename O::T) > sizeof(fe) ? MSM_G2_MAXE : MSM_MAXE;
  // the sorted digits and, once the buckets are summed, the bucket sums share one array
  constexpr size_t ENT_B = MAXE * sizeof(uint32_t), RED_B = 256 * sizeof(jac<O>);
  __shared__ __align__(16) uint8_t pool[ENT_B > RED_B ? ENT_B : RED_B];
  uint32_t *ent = reinterpret_cast<uint32_t *>(pool);
  jac<O> *red = reinterpret_cast<jac<O> *>(pool);
  uint32_t nslice = (uint32_t)((M + S - 1) / S);
  uint64_t j = blk / nslice;
  uint32_t sl = blk % nslice;
  uint64_t a0 = (uint64_t)sl * S;
  uint32_t na = (uint32_t)((a0 + S <= M) ? S : (M - a0));
  uint32_t t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const fe *sc = scal + j * M + a0;
  uint32_t ne = na * nwin;
  for (uint32_t e = t; e < ne; e += 256) {
    uint32_t a = e / nwin, w = e % nwin;
    uint32_t d = (sc[a].l[w >> 2] >> ((w & 3) * 8)) & 0xff;
    if (d) atomicAdd(&cnt[d], 1u);
  }
  __syncthreads();
  if (t == 0) {
    uint32_t s = 0;
    for (int d = 0; d < 256; d++) { off[d] = s; s += cnt[d]; }
  }
  __syncthreads();
  uint32_t start = off[t], len = cnt[t];
  __syncthreads();
  for (uint32_t e = t; e < ne; e += 256) {
    uint32_t a = e / nwin, w = e % nwin;
    uint32_t d = (sc[a].l[w >> 2] >> ((w & 3) * 8)) & 0xff;
    if (d) {
      uint32_t pos = atomicAdd(&off[d], 1u);
      ent[pos] = w * (uint32_t)M + (uint32_t)(a0 + a);
    }
  }
  __syncthreads();
  jac<O> acc = jac_inf<O>();
  for (uint32_t q = 0; q < len; q++) acc = jac_madd(acc, table[ent[start + q]]);
  if (t == 0) acc = jac_inf<O>();
  __syncthreads();  // every bucket is summed before the sums overwrite the digits
  red[t] = acc;
  __syncthreads();
  // suffix sums T_d = sum_{d' >= d} B_{d'}
  for (uint32_t s = 1; s < 256; s <<= 1) {
    jac<O> v = red[t];
    if (t + s < 256) v = jac_add(v, red[t + s]);
    __syncthreads();
    red[t] = v;
    __syncthreads();
  }
  if (t == 0) red[0] = jac_inf<O>();
  __syncthreads();
  // sum_{d >= 1} T_d
  for (uint32_t s = 128; s >= 1; s >>= 1) {
    if (t < s) red[t] = jac_add(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) partial[blk] = red[0];
}

template <class O>
__global__ void __launch_bounds__(256) k_msm_slices(const fe *scal, uint64_t M, uint32_t nwin, uint32_t S,
                                                    const aff<O> *table, jac<O> *partial) {
  msm_slice<O>(scal, M, nwin, S, table, partial, blockIdx.x);
}

// ================================================================ batched commit
// job x of a batched commit owns blocks [J[x].blk0, J[x + 1].blk0) and packed entries
// [J[x].k0, J[x + 1].k0): binary search over the table (job 0 starts at 0)
__device__ __forceinline__ uint32_t job_of_blk(const CJob *J, uint32_t n, uint64_t b) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (J[mid].blk0 <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint32_t job_of_k(const CJob *J, uint32_t n, uint64_t i) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (J[mid].k0 <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The PC.Commit MSMs of every job in one persistent launch: each workgroup takes blocks
// blockIdx.x, blockIdx.x + gridDim.x, ... of all jobs' (j, slice) blocks (jobs of uneven N, entry
// width and slice length side by side; every block sorts at most MSM_MAXE digits).
__global__ void __launch_bounds__(256) k_msm_batch(const CJob *J, uint32_t n, uint64_t total) {
  for (uint64_t b = blockIdx.x; b < total; b += gridDim.x) {
    const CJob &c = J[job_of_blk(J, n, b)];
    msm_slice<OpsG1>(c.m, c.M, c.nwin, c.S, c.table, c.part, b - c.blk0);
    __syncthreads();  // the next block reuses the shared arrays
  }
}

// v[k0 + j] = h[2 j] of each job (FC.Commit pairs C_j with v_j = h_{2j})
__global__ void __launch_bounds__(TPB) k_commit_v(const CJob *J, uint32_t n, uint64_t total, g2_aff *v) {
  uint64_t i = gtid();
  if (i >= total) return;
  const CJob &c = J[job_of_k(J, n, i)];
  v[i] = c.h[2 * (i - c.k0)];
}

// Miller values of job x at F[x Kmax + j], padded with ones up to Kmax
__global__ void __launch_bounds__(TPB) k_commit_pad(const CJob *J, uint32_t n, uint64_t Kmax, const fp12 *Fc, fp12 *F) {
  uint64_t id = gtid();
  if (id >= n * Kmax) return;
  const CJob &c = J[id / Kmax];
  const uint64_t j = id % Kmax;
  F[id] = j < c.K ? Fc[c.k0 + j] : f12_one();
}

// C of job x into its commitment
__global__ void __launch_bounds__(TPB) k_commit_store(const CJob *J, uint32_t n, const fp12 *Cs) {
  uint64_t x = gtid();
  if (x >= n) return;
  *J[x].C = Cs[x];
}

// ================================================================ open-all, step 1
// Round 1's G_T parts are the same for every batch of a job (A = aux and V = v in all of
// them): copy job x's L_1, R_1 (LT[x], RT[x]) to slot 0 of the row of every batch of job x
// (batches job-major, nbj per job)
__global__ void __launch_bounds__(TPB) k_bcast_round1(const fp12 *LT, const fp12 *RT, uint64_t nb, uint64_t nbj,
                                                      uint32_t lK, fp12 *L, fp12 *R) {
  const uint64_t words = sizeof(fp12) / 4;
  uint64_t id = gtid();
  if (id >= 2 * nb * words) return;
  uint64_t w = id % words, r = id / words, side = r & 1, k = r >> 1;
  const uint32_t *src = reinterpret_cast<const uint32_t *>(side ? RT : LT) + (k / nbj) * words;
  uint32_t *dst = reinterpret_cast<uint32_t *>(side ? R : L) + k * lK * words;
  dst[w] = src[w];
}

// Batches are job-major: batch x nbj + k is batch k of job x, whose aux row is Cj + x K
__global__ void __launch_bounds__(TPB) k_oa_init(const g1_aff *Cj, const g2_aff *h, uint64_t K, uint64_t nb, uint64_t nbj,
                                                 g1_aff *A, g2_aff *V, fe *B) {
  uint64_t id = gtid();
  if (id >= nb * K) return;
  uint64_t i = id % K;
  A[id] = Cj[(id / (nbj * K)) * K + i];
  V[id] = h[2 * i];
  B[id] = fe_zero();
}

// Several levels of the y-tree (fold rows, canonical F_r) in one pass: thread (g, a) takes
// the 2^S nodes g 2^S .. (g + 1) 2^S - 1 of level h0 in column a (at level 0 their values
// y[0][j][a] = rho_j m[jM + a], written out first: the Montgomery product of a
// Montgomery-form rho with a canonical m is the canonical product) and writes their sums at
// levels h0 + 1 .. h0 + S.  The nodes are taken left to right with one pending left sibling
// per level (a binary counter: S + 1 live elements); the steps are expanded at compile time
// (ystep), so every index is fixed and nothing goes to scratch memory.  Consecutive threads
// take consecutive columns, so every row access is coalesced; the entries are read once and
// every node is written once.
struct YCtx {
  const fe *m, *rho;
  fe *Y;
  uint64_t M, K, g, a, in;
  uint32_t h0;
};

// node Q has reached level h0 + L: keep it as a left child, or add it to its left sibling and
// write the parent at level h0 + L + 1, then carry on upward
template <int S, int Q, int L>
__device__ __forceinline__ void ycarry(const YCtx &c, fe (&pend)[S], fe cur) {
  if constexpr (L < S) {
    if constexpr (((Q >> L) & 1) == 0) {
      pend[L] = cur;
    } else {
      cur = fr_add(pend[L], cur);
      const uint64_t out = 2 * c.K - ((2 * c.K) >> (c.h0 + L + 1));
      c.Y[(out + (c.g << (S - L - 1)) + (Q >> (L + 1))) * c.M + c.a] = cur;
      ycarry<S, Q, L + 1>(c, pend, cur);
    }
  }
}

template <int S, int Q>
__device__ __forceinline__ void ystep(const YCtx &c, fe (&pend)[S]) {
  if constexpr (Q < (1 << S)) {
    const uint64_t node = (c.g << S) + Q;
    fe cur;
    if (c.h0 == 0) {
      cur = fr_mul(c.rho[node], c.m[node * c.M + c.a]);
      c.Y[node * c.M + c.a] = cur;
    } else {
      cur = c.Y[(c.in + node) * c.M + c.a];
    }
    ycarry<S, Q, 0>(c, pend, cur);
    ystep<S, Q + 1>(c, pend);
  }
}

template <int S>
__global__ void __launch_bounds__(TPB) k_ytree(const S2Job *J, uint32_t G, uint64_t M, uint64_t K, uint32_t h0) {
  const uint64_t groups = (K >> h0) >> S;
  uint64_t id = gtid();
  if (id >= G * groups * M) return;
  const S2Job &jb = J[id / (groups * M)];  // each job's threads in turn
  id %= groups * M;
  YCtx c{jb.m, jb.rho, jb.Y, M, K, id / M, id % M, 2 * K - ((2 * K) >> h0), h0};
  fe pend[S > 0 ? S : 1];
  if constexpr (S == 0) {
    // level 0 alone (K = 1): the rows of the nodes
    c.Y[c.g * M + c.a] = fr_mul(c.rho[c.g], c.m[c.g * M + c.a]);
  } else {
    ystep<S, 0>(c, pend);
  }
}

// ================================================================ export
// canonical big-endian encoding of n field elements; mode 0: Montgomery F_p, 1: Montgomery F_r, 2: canonical
__global__ void __launch_bounds__(TPB) k_encode(const fe *in, uint64_t n, int mode, uint8_t *out) {
  uint64_t i = gtid();
  if (i >= n) return;
  fe c = in[i];
  if (mode == 0) c = f_from_mont<FpP>(c);
  else if (mode == 1) c = f_from_mont<FpR>(c);
  for (int q = 0; q < 8; q++) {
    uint32_t w = c.l[7 - q];
    out[i * 32 + 4 * q] = (uint8_t)(w >> 24);
    out[i * 32 + 4 * q + 1] = (uint8_t)(w >> 16);
    out[i * 32 + 4 * q + 2] = (uint8_t)(w >> 8);
    out[i * 32 + 4 * q + 3] = (uint8_t)w;
  }
}

// gather n 32-byte items from arbitrary element offsets (in units of fe) and encode them
__global__ void __launch_bounds__(TPB) k_gather_encode(const fe *base, const uint64_t *idx, const int *mode, uint64_t n, uint8_t *out) {
  uint64_t i = gtid();
  if (i >= n) return;
  fe c = base[idx[i]];
  if (mode[i] == 0) c = f_from_mont<FpP>(c);
  else if (mode[i] == 1) c = f_from_mont<FpR>(c);
  for (int q = 0; q < 8; q++) {
    uint32_t w = (mode[i] == 3) ? c.l[q] : c.l[7 - q];  // mode 3: a digest stored as big-endian words
    out[i * 32 + 4 * q] = (uint8_t)(w >> 24);
    out[i * 32 + 4 * q + 1] = (uint8_t)(w >> 16);
    out[i * 32 + 4 * q + 2] = (uint8_t)(w >> 8);
    out[i * 32 + 4 * q + 3] = (uint8_t)w;
  }
}


// GLV split of the round challenge x_j of every batch (one thread per batch)
__global__ void __launch_bounds__(TPB) k_glv_dec(const fe *X, uint64_t nb, uint32_t j, uint32_t lK, glv::Dec *out) {
  uint64_t k = gtid();
  if (k >= nb) return;
  fe c = f_from_mont<FpR>(X[k * lK + (j - 1)]);
  out[k] = glv::decompose(c.l);
}

namespace kl {
void ek_weights(uint32_t lM, const fe *s, fe *w, uint64_t n, hipStream_t st) { L1(k_ek_weights, n, lM, s, w, n); }
void pow_table(const fe *beta, fe *out, uint64_t n, hipStream_t st) { L1(k_pow_table, n, beta, out, n); }
void msm_tables(const g1_aff *base, uint64_t M, uint32_t nwin, g1_aff *table, hipStream_t st) {
  L1(k_msm_tables<OpsG1>, M, base, M, nwin, table);
}
void msm_tables_g2(const g2_aff *base, uint64_t M, uint32_t nwin, g2_aff *table, hipStream_t st) {
  L1(k_msm_tables<OpsG2>, M, base, M, nwin, table);
}
void lift_u32(const uint32_t *in, uint64_t n, fe *out, hipStream_t st) { L1(k_lift_u32, n, in, n, out); }
void check_fr(const fe *m, uint64_t n, int *err, hipStream_t st) { L1(k_check_fr, n, m, n, err); }
void zero_u32(uint32_t *p, uint64_t n, hipStream_t st) { if (n) L1(k_zero_u32, n, p, n); }
void decode_fp(const uint8_t *in, uint64_t n, fe *out, int *err, hipStream_t st) { if (n) L1(k_decode_fp, n, in, n, out, err); }
void check_curve_g1(const g1_aff *p, uint64_t n, int *err, hipStream_t st) { if (n) L1(k_check_curve<OpsG1>, n, p, n, err); }
void check_curve_g2(const g2_aff *p, uint64_t n, int *err, hipStream_t st) { if (n) L1(k_check_curve<OpsG2>, n, p, n, err); }
void diag_mad(uint32_t seed, uint32_t iters, unsigned blocks, uint64_t *out, hipStream_t st) {
  LAUNCH(k_diag_mad, dim3(blocks), dim3(256), 0, seed, iters, out);
}
void msm_slices(const fe *scal, uint64_t K, uint64_t M, uint32_t nwin, uint32_t S, const g1_aff *table, g1_jac *partial,
                hipStream_t st) {
  uint64_t nslice = (M + S - 1) / S;
  LAUNCH(k_msm_slices<OpsG1>, dim3((unsigned)(K * nslice)), dim3(256), 0, scal, M, nwin, S, table, partial);
}
void msm_batch(const CJob *J, uint32_t n, uint64_t total, unsigned grid, hipStream_t st) {
  if (total) LAUNCH(k_msm_batch, dim3(grid), dim3(256), 0, J, n, total);
}
int msm_batch_grid(int device) {
  // workgroups resident per compute unit (shared memory and registers allow), times the units
  int per = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_msm_batch, 256, 0) != hipSuccess || per < 1) per = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 256;
  return per * cus;
}
void commit_v(const CJob *J, uint32_t n, uint64_t total, g2_aff *v, hipStream_t st) { L1(k_commit_v, total, J, n, total, v); }
void commit_pad(const CJob *J, uint32_t n, uint64_t Kmax, const fp12 *Fc, fp12 *F, hipStream_t st) {
  L1(k_commit_pad, n * Kmax, J, n, Kmax, Fc, F);
}
void commit_store(const CJob *J, uint32_t n, const fp12 *Cs, hipStream_t st) { L1(k_commit_store, n, J, n, Cs); }
void msm_slices_g2(const fe *scal, uint64_t K, uint64_t M, uint32_t nwin, uint32_t S, const g2_aff *table, g2_jac *partial,
                   hipStream_t st) {
  uint64_t nslice = (M + S - 1) / S;
  LAUNCH(k_msm_slices<OpsG2>, dim3((unsigned)(K * nslice)), dim3(256), 0, scal, M, nwin, S, table, partial);
}
void fr_canon(const fe *in, uint64_t n, fe *out, hipStream_t st) { L1(k_fr_canon, n, in, n, out); }
void g1_reduce(g1_jac *data, uint64_t nseg, uint64_t stride, uint64_t len, uint32_t *cnt, hipStream_t st) {
  if (len > 1) L1(k_jac_tree<OpsG1>, nseg * ((len + 1) / 2), data, nseg, stride, len, cnt);
}
void g2_to_aff(const g2_jac *in, uint64_t stride, uint64_t n, g2_aff *out, uint64_t ostride, hipStream_t st) {
  L1(k_jac_to_aff<OpsG2>, n, in, stride, n, out, ostride);
}
void g1_to_aff(const g1_jac *in, uint64_t stride, uint64_t n, g1_aff *out, uint64_t ostride, hipStream_t st) {
  L1(k_jac_to_aff<OpsG1>, n, in, stride, n, out, ostride);
}
void bcast_round1(const fp12 *LT, const fp12 *RT, uint64_t nb, uint64_t nbj, uint32_t lK, fp12 *L, fp12 *R,
                  hipStream_t st) {
  L1(k_bcast_round1, 2 * nb * (sizeof(fp12) / 4), LT, RT, nb, nbj, lK, L, R);
}
void oa_init(const g1_aff *Cj, const g2_aff *h, uint64_t K, uint64_t nb, uint64_t nbj, g1_aff *A, g2_aff *V, fe *B,
             hipStream_t st) {
  L1(k_oa_init, nb * K, Cj, h, K, nb, nbj, A, V, B);
}
void glv_dec(const fe *X, uint64_t nb, uint32_t j, uint32_t lK, glv::Dec *out, hipStream_t st) {
  L1(k_glv_dec, nb, X, nb, j, lK, out);
}
void ytree(const S2Job *J, uint32_t G, uint64_t M, uint64_t K, uint32_t lK, hipStream_t st) {
  // passes of four levels (the last pass takes what remains); level 0 is made in the first,
  // which takes two levels below G N = 2^24 so that its G N / 4 threads still fill the device
  uint32_t h0 = 0;
  if (lK == 0) {
    L1(k_ytree<0>, G * M, J, G, M, K, 0u);
    return;
  }
  while (h0 < lK) {
    const uint32_t want = (h0 == 0 && G * K * M < (1ull << 24)) ? 2 : 4;
    const uint32_t s = lK - h0 >= want ? want : lK - h0;
    const uint64_t n = G * ((K >> h0) >> s) * M;
    switch (s) {
      case 4: L1(k_ytree<4>, n, J, G, M, K, h0); break;
      case 3: L1(k_ytree<3>, n, J, G, M, K, h0); break;
      case 2: L1(k_ytree<2>, n, J, G, M, K, h0); break;
      default: L1(k_ytree<1>, n, J, G, M, K, h0); break;
    }
    h0 += s;
  }
}
void encode(const fe *in, uint64_t n, int mode, uint8_t *out, hipStream_t st) { if (n) L1(k_encode, n, in, n, mode, out); }
void gather_encode(const fe *base, const uint64_t *idx, const int *mode, uint64_t n, uint8_t *out, hipStream_t st) {
  if (n) L1(k_gather_encode, n, base, idx, mode, n, out);
}
}  // namespace kl
