// Kernels: transcript and Merkle hashing, batching coefficients, KZG quotient.
// (helpers inlined: out of line, the SHA-256 state and message blocks passed by reference went
// through scratch memory)
#define VC_INLINE_HELPERS 1
#include "kcommon.hpp"

#define FC_CHUNK 32
#define KZG_T 1024
#define KZG_PER 2  // coefficients per thread: D = 2K - 1 <= 2 KZG_T, so K <= 1024

// ================================================================ setup
// s_t = H2F(DST_SETUP, seed || "s" || t) for t < lM, beta = H2F(DST_SETUP, seed || "beta")
__global__ void __launch_bounds__(TPB) k_trapdoor(const uint8_t *seed, uint32_t lM, fe *s, fe *beta) {
  uint32_t t = (uint32_t)gtid();
  if (t > lM) return;
  sha::Hasher h;
  sha::xmd_begin(h);
  for (int i = 0; i < 32; i++) h.byte(seed[i]);
  if (t < lM) {
    h.byte('s');
    h.u64(t);
    s[t] = sha::xmd_finish_fr(h, DSTR_SETUP);
  } else {
    h.byte('b'); h.byte('e'); h.byte('t'); h.byte('a');
    *beta = sha::xmd_finish_fr(h, DSTR_SETUP);
  }
}

// chunk digests of the batch statement: H_q over (a_i || enc(C_{a_i})) for 32 entries; a
// workgroup of 64 per chunk, one lane per entry writes the message words (sha::Coop)
__global__ void __launch_bounds__(64) k_fc_chunks(const g1_aff *Cj, uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj,
                                                 uint32_t *Hq) {
  CHAIN_PRIORITY();
  __shared__ uint32_t msg[FC_CHUNK * 18 + 18];
  uint64_t id = blockIdx.x;
  uint64_t qmax = (b + FC_CHUNK - 1) / FC_CHUNK;
  if (id >= nb * qmax) return;
  // batch k of job x (batches job-major, nbj per job), whose aux row is Cj + x K
  uint64_t kk = id / qmax, q = id % qmax, k = kk % nbj;
  Cj += (kk / nbj) * K;
  uint64_t lo = k * b, hi = (lo + b < K) ? lo + b : K;
  uint64_t s = lo + q * FC_CHUNK;
  if (s >= hi) return;
  int n = (int)(((s + FC_CHUNK < hi) ? s + FC_CHUNK : hi) - s);
  const int t = threadIdx.x;
  if (t < n) {
    uint64_t a = s + t;
    msg[18 * t] = (uint32_t)(a >> 32);
    msg[18 * t + 1] = (uint32_t)a;
    sha::put_words<FpP>(msg + 18 * t + 2, Cj[a].x);
    sha::put_words<FpP>(msg + 18 * t + 10, Cj[a].y);
  }
  __syncthreads();
  uint32_t out[8];
  sha::sha_coop(sha::Coop{t, 64}, msg, 72u * n, out);
  if (t == 0)
    for (int w = 0; w < 8; w++) Hq[id * 8 + w] = out[w];
}

// sigma_k = SHA-256(DST_FC_R || enc(C) || t || H_0 || H_1 ...), a workgroup of 64 per batch
// (message in dynamic shared memory, fc_sigma_shm bytes)
__host__ __device__ inline size_t fc_sigma_shm(uint32_t b) {
  return ((410 + 32 * (size_t)((b + FC_CHUNK - 1) / FC_CHUNK) + 72 + 3) / 4) * 4;
}
__global__ void __launch_bounds__(64) k_fc_sigma(const fp12 *C, uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj,
                                                const uint32_t *Hq, uint32_t *sigma) {
  CHAIN_PRIORITY();
  extern __shared__ uint32_t mw[];
  const uint64_t kk = blockIdx.x;
  if (kk >= nb) return;
  const uint64_t k = kk % nbj;  // batch k of job kk / nbj, whose commitment is C[kk / nbj]
  C += kk / nbj;
  const int t = threadIdx.x;
  uint64_t qmax = (b + FC_CHUNK - 1) / FC_CHUNK;
  uint64_t lo = k * b, hi = (lo + b < K) ? lo + b : K;
  uint64_t cnt = hi - lo, nq = (cnt + FC_CHUNK - 1) / FC_CHUNK;
  const char *dst = DSTR_FC_R;
  const uint32_t dl = (uint32_t)sha::cstrlen(dst);
  if ((uint32_t)t < dl) sha::put_byte(mw, t, (uint8_t)dst[t]);
  if (t < 12) sha::put_field_bytes<FpP>(mw, dl + 32 * t, reinterpret_cast<const fe *>(C)[t]);
  if (t >= 12 && t < 20) sha::put_byte(mw, dl + 384 + (t - 12), (uint32_t)(cnt >> (8 * (19 - t))) & 0xff);
  const uint32_t off = dl + 392;
  for (uint64_t w = t; w < 8 * nq; w += 64) {
    uint32_t v = Hq[kk * qmax * 8 + w];
    for (int i = 0; i < 4; i++) sha::put_byte(mw, off + 4 * (uint32_t)w + i, v >> (24 - 8 * i));
  }
  __syncthreads();
  uint32_t out[8];
  sha::sha_coop(sha::Coop{t, 64}, mw, off + 32 * (uint32_t)nq, out);
  if (t == 0)
    for (int w = 0; w < 8; w++) sigma[kk * 8 + w] = out[w];
}

// r_i = H2F(DST_FC_R, sigma_k || i), a workgroup of 64 per entry: the sparse exponent
// vector b = sum r_i u_{a_i}
__global__ void __launch_bounds__(64) k_fc_r(uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, const uint32_t *sigma,
                                            fe *B) {
  CHAIN_PRIORITY();
  __shared__ uint32_t w[16 + 10 + 32], t2[16];
  uint64_t id = blockIdx.x;
  if (id >= nb * (uint64_t)b) return;
  uint64_t kk = id / b, i = id % b;
  uint64_t a = (kk % nbj) * b + i;  // entry i of batch kk % nbj of its job
  if (a >= K) return;
  const int t = threadIdx.x;
  if (t < 16) w[t] = 0;
  else if (t < 24) w[t] = sigma[kk * 8 + t - 16];
  else if (t < 26) w[t] = t == 24 ? (uint32_t)(i >> 32) : (uint32_t)i;
  __syncthreads();
  fe r = sha::xmd_fr_coop(sha::Coop{t, 64}, w, 40, DSTR_FC_R, t2);
  if (t == 0) B[kk * K + a] = r;
}

// affine G1 parts of L_j, R_j from the reduced term sums, one thread per (batch, side)
__global__ void __launch_bounds__(TPB) k_oa_lr_aff(const g1_jac *S, uint64_t K, uint64_t nb, uint32_t j, uint32_t lK,
                                                   g1_aff *Lg1, g1_aff *Rg1) {
  uint64_t id = gtid();
  if (id >= 2 * nb) return;
  uint64_t k = id / 2, side = id % 2;
  g1_aff a = jac_to_aff(S[(k * 2 + side) * (K / 2)]);
  (side ? Rg1 : Lg1)[k * lK + (j - 1)] = a;
}

// per batch: hash L_j, R_j into x_j, keep x_j and 1/x_j.  A workgroup of 64 per batch:
// lanes encode x_{j-1} and the 28 coordinates of L_j, R_j in parallel (sha::Coop), and the
// inverse runs on the scalar unit.
__global__ void __launch_bounds__(64) k_oa_transcript(const fp12 *Lgt, const fp12 *Rgt, uint64_t nb, uint32_t j,
                                                     uint32_t lK, const g1_aff *Lg1, const g1_aff *Rg1, fe *X, fe *Xinv,
                                                     int *err, uint32_t zero_round) {
  CHAIN_PRIORITY();
  __shared__ uint32_t msg[16 + 8 + 2 * (96 + 16) + 32], t2[16];
  uint64_t k = blockIdx.x;
  if (k >= nb) return;
  uint64_t slot = k * lK + (j - 1);
  const int t = threadIdx.x;
  const int pre = j > 1 ? 8 : 0;
  if (t < 16) msg[t] = 0;  // Z_pad
  // element e: x_{j-1} (F_r) if j > 1, then L_gt (12), L_g1 (2), R_gt (12), R_g1 (2)
  const int e = j > 1 ? t - 1 : t;
  if (j > 1 && t == 0) sha::put_words<FpR>(msg + 16, X[slot - 1]);
  if (e >= 0 && e < 28) {
    int side = e / 14, q = e % 14;
    const fe *src = q < 12 ? reinterpret_cast<const fe *>((side ? Rgt : Lgt) + slot) + q
                           : reinterpret_cast<const fe *>((side ? Rg1 : Lg1) + slot) + (q - 12);
    sha::put_words<FpP>(msg + 16 + pre + 112 * side + 8 * q, *src);
  }
  __syncthreads();
  fe x = sha::xmd_fr_coop(sha::Coop{t, 64}, msg, 4 * (pre + 224), DSTR_FC_X, t2);
  if (zero_round == j && k == 0) x = fe_zero();  // test hook: the host forces a zero challenge
  fe xi = f_inv_uniform<FpR>(x, bn::R_R3);
  if (t == 0) {
    if (fe_is_zero(x)) atomicOr(err, VC_ERRBIT_CHALLENGE);
    X[slot] = x;
    Xinv[slot] = xi;
  }
}

// ---------------------------------------------------------------- KZG proof of v_l
// f_v(X) = prod_{j=1}^{l} (1 + x_j^{-1} X^{2^{l-j+1}}): only even powers X^{2s} (s < K) occur,
// with coefficient prod over the set bits t of s of x_{l-t}^{-1}.  z = H2F(DST_FC_Z, x_l || v_l);
// q = (f_v - f_v(z)) / (X - z) has q_m = sum_{i > m} c_i z^{i-m-1} (m < D - 1), that is
// q_m = c_{m+1} + z q_{m+1} with q_{D-1} = 0: a suffix scan whose step with offset s adds
// z^s q[m + s] to q[m] (the multiplier z^s is the same for every element, so a step costs one
// product and no inverse is needed).  One block of KZG_T threads per batch, D = 2K - 1.

// c_{m+1}, the scan's input at m
__device__ __forceinline__ fe kzg_coef(const fe *Xinv, uint64_t k, uint32_t lK, uint64_t m) {
  const uint64_t i = m + 1;
  if (i & 1) return fe_zero();
  const uint64_t s2 = i >> 1;
  fe c = f_one<FpR>();
  for (uint32_t bt = 0; bt < lK; bt++)
    if ((s2 >> bt) & 1) c = fr_mul(c, Xinv[k * lK + (lK - bt) - 1]);
  return c;
}

__global__ void __launch_bounds__(KZG_T) k_kzg_quotient(const fe *Xinv, const fe *X, const g2_aff *V, uint64_t K,
                                                      uint32_t lK, fe *Q, fe *zout) {
  CHAIN_PRIORITY();
  extern __shared__ fe sh[];  // D - 1 elements
  uint64_t k = blockIdx.x;
  const uint64_t n = 2 * K - 2;
  fe *acc = sh;
  __shared__ uint32_t zmsg[16 + 8 + 32 + 24], t2[16];
  uint32_t t = threadIdx.x;
  // z = H2F(DST_FC_Z, x_l || v_l): lanes encode, every wave hashes (sha::Coop)
  if (t < 16) zmsg[t] = 0;
  if (t == 16) sha::put_words<FpR>(zmsg + 16, X[k * lK + lK - 1]);
  if (t > 16 && t <= 20) sha::put_words<FpP>(zmsg + 24 + 8 * (t - 17), reinterpret_cast<const fe *>(V + k * K)[t - 17]);
  __syncthreads();
  const fe zz = sha::xmd_fr_coop(sha::Coop{(int)t, KZG_T}, zmsg, 160, DSTR_FC_Z, t2);
  if (t == 0) zout[k] = zz;
  for (uint64_t m = t; m < n; m += KZG_T) acc[m] = kzg_coef(Xinv, k, lK, m);
  __syncthreads();
  fe zs = zz;  // z^s
  for (uint64_t s = 1; s < n; s <<= 1) {
    fe vals[KZG_PER];
    int nv = 0;
    for (uint64_t m = t; m < n; m += KZG_T, nv++) vals[nv] = (m + s < n) ? fr_add(acc[m], fr_mul(zs, acc[m + s])) : acc[m];
    __syncthreads();
    nv = 0;
    for (uint64_t m = t; m < n; m += KZG_T, nv++) acc[m] = vals[nv];
    __syncthreads();
    zs = fr_mul(zs, zs);
  }
  for (uint64_t m = t; m < n; m += KZG_T) Q[k * n + m] = acc[m];
}

// The same quotient for K > 1024, whose 2K - 2 working values do not fit in shared memory: the
// scan runs over two global arrays, read and written alternately, with the same operations in
// the same order.  gws: 4 (2K - 1) elements per batch.
__global__ void __launch_bounds__(KZG_T) k_kzg_quotient_g(const fe *Xinv, const fe *X, const g2_aff *V, uint64_t K,
                                                        uint32_t lK, fe *Q, fe *zout, fe *gws) {
  CHAIN_PRIORITY();
  uint64_t k = blockIdx.x;
  const uint64_t n = 2 * K - 2;
  fe *aa = gws + k * 4 * (2 * K - 1), *ab = aa + n;
  __shared__ uint32_t zmsg[16 + 8 + 32 + 24], t2[16];
  uint32_t t = threadIdx.x;
  if (t < 16) zmsg[t] = 0;
  if (t == 16) sha::put_words<FpR>(zmsg + 16, X[k * lK + lK - 1]);
  if (t > 16 && t <= 20) sha::put_words<FpP>(zmsg + 24 + 8 * (t - 17), reinterpret_cast<const fe *>(V + k * K)[t - 17]);
  __syncthreads();
  const fe zz = sha::xmd_fr_coop(sha::Coop{(int)t, KZG_T}, zmsg, 160, DSTR_FC_Z, t2);
  if (t == 0) zout[k] = zz;
  for (uint64_t m = t; m < n; m += KZG_T) aa[m] = kzg_coef(Xinv, k, lK, m);
  __syncthreads();
  fe zs = zz;
  for (uint64_t s = 1; s < n; s <<= 1) {
    for (uint64_t m = t; m < n; m += KZG_T) ab[m] = (m + s < n) ? fr_add(aa[m], fr_mul(zs, aa[m + s])) : aa[m];
    __syncthreads();
    fe *tmp = aa; aa = ab; ab = tmp;
    zs = fr_mul(zs, zs);
  }
  for (uint64_t m = t; m < n; m += KZG_T) Q[k * n + m] = aa[m];
}

// ================================================================ open-all, step 2
// Merkle leaves SHA-256(0x00 || m_i || C_j), stored as 8 big-endian words per node;
// node n of the heap (root = 1, leaf i = N + i) at tree[8n]
__global__ void __launch_bounds__(TPB) k_merkle_leaves(const S2Job *J, uint32_t G, uint64_t M, uint64_t N) {
  uint64_t id = gtid();
  if (id >= G * N) return;
  const S2Job &jb = J[id / N];
  const uint64_t i = id % N;
  const fe *m = jb.m;
  const g1_aff *Cj = jb.Cj;
  uint32_t *tree = jb.tree;
  uint32_t mw[8], cw[16];
  const fe &mi = m[i];
#pragma unroll
  for (int q = 0; q < 8; q++) mw[q] = mi.l[7 - q];
  const g1_aff &c = Cj[i / M];
  fe x = f_from_mont<FpP>(c.x), y = f_from_mont<FpP>(c.y);
#pragma unroll
  for (int q = 0; q < 8; q++) { cw[q] = x.l[7 - q]; cw[8 + q] = y.l[7 - q]; }
  uint32_t o[8];
  sha::merkle_leaf(o, mw, cw);
#pragma unroll
  for (int q = 0; q < 8; q++) tree[(N + i) * 8 + q] = o[q];
}

// nodes [start, 2 start): node n = SHA-256(0x01 || node 2n || node 2n+1)
__global__ void __launch_bounds__(TPB) k_merkle_level(const S2Job *J, uint32_t G, uint64_t start) {
  uint64_t id = gtid();
  if (id >= G * start) return;
  uint32_t *tree = J[id / start].tree;
  uint64_t n = start + id % start;
  uint32_t l[8], r[8], o[8];
#pragma unroll
  for (int q = 0; q < 8; q++) { l[q] = tree[16 * n + q]; r[q] = tree[16 * n + 8 + q]; }
  sha::merkle_node(o, l, r);
#pragma unroll
  for (int q = 0; q < 8; q++) tree[8 * n + q] = o[q];
}

// rho_j = H2F(DST_RHO, C || root || j)
__global__ void __launch_bounds__(TPB) k_rho(const S2Job *J, uint32_t G, uint64_t K) {
  uint64_t id = gtid();
  if (id >= G * K) return;
  const S2Job &jb = J[id / K];
  const uint64_t j = id % K;
  sha::Hasher hs;
  sha::xmd_begin(hs);
  hs.gt(*jb.C);
  for (int q = 0; q < 8; q++) hs.word(jb.tree[8 + q]);
  hs.u64(j);
  jb.rho[j] = sha::xmd_finish_fr(hs, DSTR_RHO);
}

namespace kl {
void trapdoor(const uint8_t *seed, uint32_t lM, fe *s, fe *beta, hipStream_t st) { L1(k_trapdoor, lM + 1, seed, lM, s, beta); }
void fc_chunks(const g1_aff *Cj, uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, uint32_t *Hq, hipStream_t st) {
  LAUNCH(k_fc_chunks, dim3((unsigned)(nb * ((b + FC_CHUNK - 1) / FC_CHUNK))), dim3(64), 0, Cj, K, b, nb, nbj, Hq);
}
void fc_sigma(const fp12 *C, uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, const uint32_t *Hq, uint32_t *sigma,
              hipStream_t st) {
  LAUNCH(k_fc_sigma, dim3((unsigned)nb), dim3(64), fc_sigma_shm(b), C, K, b, nb, nbj, Hq, sigma);
}
void fc_r(uint64_t K, uint32_t b, uint64_t nb, uint64_t nbj, const uint32_t *sigma, fe *B, hipStream_t st) {
  LAUNCH(k_fc_r, dim3((unsigned)(nb * b)), dim3(64), 0, K, b, nb, nbj, sigma, B);
}
void oa_lr_aff(const g1_jac *S, uint64_t K, uint64_t nb, uint32_t j, uint32_t lK, g1_aff *Lg1, g1_aff *Rg1, hipStream_t st) {
  L1(k_oa_lr_aff, 2 * nb, S, K, nb, j, lK, Lg1, Rg1);
}
void oa_transcript(const fp12 *Lgt, const fp12 *Rgt, uint64_t nb, uint32_t j, uint32_t lK, const g1_aff *Lg1,
                   const g1_aff *Rg1, fe *X, fe *Xinv, int *err, uint32_t zero_round, hipStream_t st) {
  LAUNCH(k_oa_transcript, dim3((unsigned)nb), dim3(64), 0, Lgt, Rgt, nb, j, lK, Lg1, Rg1, X, Xinv, err, zero_round);
}
void kzg_quotient(const fe *Xinv, const fe *X, const g2_aff *V, uint64_t K, uint64_t nb, uint32_t lK, fe *Q, fe *z,
                  fe *gws, hipStream_t st) {
  if (K > KZG_T) {
    LAUNCH(k_kzg_quotient_g, dim3((unsigned)nb), dim3(KZG_T), 0, Xinv, X, V, K, lK, Q, z, gws);
    return;
  }
  size_t shm = (2 * K - 2) * sizeof(fe);
  static const bool attr_set = [] {  // once per process (thread-safe initialisation)
    (void)hipFuncSetAttribute((const void *)k_kzg_quotient, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (2 * KZG_T) * (int)sizeof(fe));
    return true;
  }();
  (void)attr_set;
  LAUNCH(k_kzg_quotient, dim3((unsigned)nb), dim3(KZG_T), shm, Xinv, X, V, K, lK, Q, z);
}
void merkle_leaves(const S2Job *J, uint32_t G, uint64_t M, uint64_t N, hipStream_t st) {
  L1(k_merkle_leaves, G * N, J, G, M, N);
}
void merkle_level(const S2Job *J, uint32_t G, uint64_t start, hipStream_t st) { L1(k_merkle_level, G * start, J, G, start); }
void rho(const S2Job *J, uint32_t G, uint64_t K, hipStream_t st) { L1(k_rho, G * K, J, G, K); }
}  // namespace kl

// ------------------------------------------------------------------ evaluation proof at a point
// f_m at r = (r_{L-1}, ..., r_0) (section 4.3): entry i = jM + a pairs its bit k with x_k.
// T_j = prod_{c<lK} (j_c r_{lM+c} + (1 - j_c)(1 - r_{lM+c})); C_F = sum_j T_j C_j; the FC
// statement is the query T with claimed value C_F, batched with r_0 = H2F(EVAL, sigma_E || 0),
// sigma_E = SHA-256(EVAL || C || r_{L-1} || ... || r_0 || C_F); F's table g[a] = sum_j T_j
// m[jM + a] is opened at r_R by PST, eliminating x_{lM-1} first.

// r_k from 32 little-endian bytes (range-checked), Montgomery form; a thread per k
__global__ void __launch_bounds__(64) k_ev_point(const uint8_t *rle, uint32_t L, fe *r, int *err) {
  uint32_t k = (uint32_t)gtid();
  if (k >= L) return;
  fe v;
  for (int q = 0; q < 8; q++) {
    const uint8_t *b = rle + 32 * k + 4 * q;
    v.l[q] = (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
  }
  if (!fe_lt_mod(v, bn::R_MOD)) atomicOr(err, VC_ERRBIT_RANGE);
  r[k] = f_to_mont<FpR>(v);
}

// T_j, a thread per j < K
__global__ void __launch_bounds__(TPB) k_ev_eq(const fe *r, uint32_t lM, uint32_t lK, uint64_t K, fe *T) {
  uint64_t j = gtid();
  if (j >= K) return;
  fe acc = f_one<FpR>();
  for (uint32_t c = 0; c < lK; c++) {
    fe rc = r[lM + c];
    acc = fr_mul(acc, ((j >> c) & 1) ? rc : fr_sub(f_one<FpR>(), rc));
  }
  T[j] = acc;
}

// the sum of n affine points (one workgroup of 256)
__global__ void __launch_bounds__(256) k_ev_sum(const g1_aff *P, uint64_t n, g1_aff *out) {
  __shared__ g1_jac sh[256];
  const int t = threadIdx.x;
  g1_jac acc = jac_inf<OpsG1>();
  for (uint64_t q = t; q < n; q += 256) acc = jac_madd(acc, P[q]);
  sh[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = jac_add(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) *out = jac_to_aff(sh[0]);
}

// r_0 on thread 0, then b = r_0 T (one workgroup)
__global__ void __launch_bounds__(256) k_ev_r0(const fp12 *C, const fe *r, uint32_t L, const g1_aff *CF, const fe *T,
                                               uint64_t K, fe *B) {
  CHAIN_PRIORITY();
  __shared__ fe r0;
  if (threadIdx.x == 0) {
    sha::Hasher hs;
    hs.init();
    hs.str(DSTR_EVAL);
    hs.gt(*C);
    for (int k = (int)L - 1; k >= 0; k--) hs.field<FpR>(r[k]);
    hs.g1(*CF);
    uint32_t sigma[8];
    hs.final(sigma);
    sha::Hasher hx;
    sha::xmd_begin(hx);
    for (int w = 0; w < 8; w++) hx.word(sigma[w]);
    hx.u64(0);
    r0 = sha::xmd_finish_fr(hx, DSTR_EVAL);
  }
  __syncthreads();
  for (uint64_t j = threadIdx.x; j < K; j += 256) B[j] = fr_mul(r0, T[j]);
}

// g[a] = sum_j T_j m[jM + a] (m canonical, T and g Montgomery), a thread per a
__global__ void __launch_bounds__(TPB) k_ev_table(const fe *m, const fe *T, uint64_t K, uint64_t M, fe *g) {
  uint64_t a = gtid();
  if (a >= M) return;
  fe acc = fe_zero();
  for (uint64_t j = 0; j < K; j++) acc = fr_add(acc, fr_mul(T[j], m[j * M + a]));  // T R * m / R: canonical
  g[a] = f_to_mont<FpR>(acc);
}

// one PST step on a table of 2 half entries: q = hi - lo, lo += r q; a thread per c < half
__global__ void __launch_bounds__(TPB) k_ev_pst_step(fe *g, uint64_t half, const fe *rvar, fe *q) {
  uint64_t c = gtid();
  if (c >= half) return;
  fe d = fr_sub(g[half + c], g[c]);
  q[c] = d;
  g[c] = fr_add(g[c], fr_mul(*rvar, d));
}

// W_d = sum of segment d of the products (entries [2^{lM-1-d} - 1, 2^{lM-d} - 1)); y = g[0]
__global__ void __launch_bounds__(256) k_ev_finish(const g1_aff *prod, uint32_t lM, const fe *g, g1_aff *W, fe *y) {
  __shared__ g1_jac sh[256];
  uint32_t d = blockIdx.x;
  if (d >= lM) return;
  const int t = threadIdx.x;
  uint64_t len = 1ull << (lM - 1 - d), lo = len - 1;
  g1_jac acc = jac_inf<OpsG1>();
  for (uint64_t q = t; q < len; q += 256) acc = jac_madd(acc, prod[lo + q]);
  sh[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = jac_add(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) {
    W[d] = jac_to_aff(sh[0]);
    if (d == 0) *y = g[0];
  }
}

namespace kl {
void ev_point(const uint8_t *rle, uint32_t L, fe *r, int *err, hipStream_t st) {
  LAUNCH(k_ev_point, dim3(1), dim3(64), 0, rle, L, r, err);
}
void ev_eq(const fe *r, uint32_t lM, uint32_t lK, uint64_t K, fe *T, hipStream_t st) { L1(k_ev_eq, K, r, lM, lK, K, T); }
void ev_sum(const g1_aff *P, uint64_t n, g1_aff *out, hipStream_t st) {
  LAUNCH(k_ev_sum, dim3(1), dim3(256), 0, P, n, out);
}
void ev_r0(const fp12 *C, const fe *r, uint32_t L, const g1_aff *CF, const fe *T, uint64_t K, fe *B, hipStream_t st) {
  LAUNCH(k_ev_r0, dim3(1), dim3(256), 0, C, r, L, CF, T, K, B);
}
void ev_table(const fe *m, const fe *T, uint64_t K, uint64_t M, fe *g, hipStream_t st) { L1(k_ev_table, M, m, T, K, M, g); }
void ev_pst_step(fe *g, uint64_t half, const fe *rvar, fe *q, hipStream_t st) { L1(k_ev_pst_step, half, g, half, rvar, q); }
void ev_finish(const g1_aff *prod, uint32_t lM, const fe *g, g1_aff *W, fe *y, hipStream_t st) {
  LAUNCH(k_ev_finish, dim3(lM), dim3(256), 0, prod, lM, g, W, y);
}
}  // namespace kl
