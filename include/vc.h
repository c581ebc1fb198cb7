/*
 * FlexProofs vector commitment on one MI355X (gfx950): C ABI.
 *
 * The scheme (paper, section 4, "A VC Scheme with Linear-Time OpenAll") commits to a
 * vector m in F_r^N, N = 2^L, in two layers: the N entries are split into K = 2^floor(L/2)
 * subvectors of M = N/K entries, each committed with the multilinear PST scheme
 * (Eq. genCi), and the K commitments are committed with the pairing-based functional
 * commitment of section 3 (Eq. genC).  OpenAll (Protocol 1 and its Sub-protocol,
 * made non-interactive with a Merkle tree as in section 4.2) produces all N opening
 * proofs: ceil(K/b) FC batch proofs (Step 1) plus a randomized folding tree and
 * PC.HyperEval on the folded polynomial (Step 2).  Curve: BN254 (the paper's
 * BN_SNARK1), optimal ate pairing.
 *
 * Conventions for every entry point:
 *  - Return value: VC_OK (0) or a negative VC_E* code; the verifiers (vc_verify,
 *    vc_verify_all, vc_verify_subarray, vc_verify_eval) return 1 (accept), 0 (reject) or a
 *    negative code.  vc_strerror() names a code (with the HIP error text of the calling
 *    thread's last failure for VC_EDEVICE).
 *  - Device pointers are borrowed for the duration of the call and must be device
 *    memory on the params' device.  `stream` is a hipStream_t (NULL = default
 *    stream); work is ordered on it and every call is synchronous on return.
 *    vc_open_all also runs work on five side streams of the params' default executor
 *    (joined to `stream` before it returns); they overlap only if the process has at
 *    least six hardware queues (environment GPU_MAX_HW_QUEUES, read by HIP at its first
 *    device use; the Python package raises it to 16), otherwise they share queues and run
 *    partly in sequence, with the same results.
 *  - Handles (vc_params, vc_commitment, vc_proofs, vc_exec, vc_server) own their device
 *    memory and are released with the matching *_free, in any order (each keeps its own
 *    device id; a release reports nothing and leaves no HIP error behind).  A commitment
 *    or proof bundle is used only while its params live; a vc_proofs handle does not
 *    reference the commitment it was made from.
 *  - Field entries and scalars are canonical (< r) 32-byte little-endian integers
 *    unless stated otherwise; serialized group elements are canonical big-endian:
 *    G1 64 B (x || y), G2 128 B (x.c0 || x.c1 || y.c0 || y.c1), G_T 384 B (12 F_p
 *    coefficients, c0.c0.c0 first), identity = all zero bytes.
 */
#ifndef FLEXPROOFS_VC_H
#define FLEXPROOFS_VC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VC_OK 0
#define VC_EINVAL (-1)     /* bad size, b out of [1, K], entry >= r, malformed proof */
#define VC_ENOMEM (-2)     /* device allocation failed */
#define VC_EDEVICE (-3)    /* HIP runtime error */
#define VC_ENOTIMPL (-4)
#define VC_ECHALLENGE (-5) /* a Fiat-Shamir challenge was zero (probability ~2^-254) */

/* Largest log2 N: at N = 2^30 an open-all with b = log^2 N, its entries and commitment hold
 * about 212 GB of device memory (measured; the entries, their copy in the commitment, the
 * Merkle tree and the y-tree dominate, about 192 N bytes), which fits the 288 GB of one
 * MI355X; 2^31 does not.  Per-element thread indices stay below 2^32 up to this size. */
#define VC_MAX_LOG_N 30

typedef struct vc_params vc_params;
typedef struct vc_commitment vc_commitment;
typedef struct vc_proofs vc_proofs;
typedef struct vc_exec vc_exec;

/* VC.Setup(1^lambda, 1^N) (Eq. vcpp): PST keys for log M variables and FC keys for
 * K entries, derived from a seeded TEST trapdoor (insecure: the paper requires a
 * trusted setup).  2 <= log_n <= VC_MAX_LOG_N.  The keys stay resident on `device`. */
int vc_setup(uint32_t log_n, const uint8_t seed[32], int device, vc_params **out);

/* Parameters from an externally made SRS (PC.Setup, section 4.1; FC.Setup, section 3; the
 * faster verifier's extra G2 powers, section 3): srs (host, borrowed for the call) is the
 * concatenation, in this order, of ek_k for k = 0..log M (2^k G1 points each, the
 * Lagrange-basis keys of k variables), vk (log M G2 points s_k g2), h (2K - 1 G2 points
 * beta^k g2) and beta g1 (one G1 point) -- exactly what vc_params_export returns for what 0
 * (idx 0..log M), 1, 2 and 3.  Each coordinate is 32 B canonical big-endian; G2
 * coordinates are (c0, c1).  len fixes N: it must equal 64 (2M - 1) + 128 log M +
 * 128 (2K - 1) + 64 for some 2 <= log N <= VC_MAX_LOG_N (K = 2^floor(log N / 2),
 * M = N / K), else VC_EINVAL.  A coordinate >= p or a point off its curve (G1, or the
 * twist for G2) gives VC_EINVAL; points are not checked for membership in the order-r
 * subgroup of the twist, nor the keys for coming from one trapdoor (the caller trusts the
 * setup that made them).  The keys and the tables derived from them stay resident on
 * `device`; free with vc_params_free. */
int vc_params_load(const uint8_t *srs, size_t len, int device, vc_params **out);

/* VC.Commit(m) (Eq. genCi, genC).  m_dev: n entries on the device, either n x 32 B
 * canonical little-endian (entry_bits = 256) or n x uint32 (entry_bits = 32, the
 * entries are the integers themselves).  n must equal 2^log_n of the params.
 * Writes the commitment C (G_T, 384 B) to C_out (host) and returns the handle that
 * keeps aux = (C_0..C_{K-1}) and a copy of m on the device.  VC_EINVAL if an entry
 * is >= r. */
int vc_commit(const vc_params *pp, const void *m_dev, uint64_t n, uint32_t entry_bits, void *stream,
              vc_commitment **out, uint8_t C_out[384]);

/* VC.Commit without device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same commitment
 * as vc_commit, from the same kernels, but no handle: m_dev and n as for vc_commit, with
 * n <= 2^20.  Writes C_0..C_{K-1} to Cj_out (device, K x 64 B canonical big-endian affine
 * x || y, the identity as zeros: the bytes of vc_commitment_export(cm, 0)) and C to C_out
 * (host, 384 B; may be NULL).  All scratch (about 33 MiB at n = 2^20) lives in one static
 * device array of 34 MiB that each GPU the library runs on holds until the process ends;
 * the call clears what must start at zero.  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (any streams, any params) race and must be serialized by the
 * caller.  Synchronous on return.  VC_EINVAL: n != N of the params, n > 2^20, bad
 * entry_bits, or an entry >= r.  The params (vc_setup) were allocated beforehand. */
int vc_commit_noalloc(const vc_params *pp, const void *m_dev, uint64_t n, uint32_t entry_bits, void *stream,
                      void *Cj_out, uint8_t C_out[384]);

/* VC.Commit (Eq. genCi, genC) of n independent vectors at once: job i commits m_devs[i] (as
 * m_dev of vc_commit, N of pps[i] entries of entry_bits[i] = 32 or 256 bits) on params
 * pps[i] (jobs may share params; all on one device).  All jobs' PC.Commit MSMs run in one
 * persistent launch (workgroups take the (subvector, slice) blocks of every job in turn, jobs
 * of uneven N and entry width side by side), their C_j in one launch, and FC.Commit of all
 * jobs in one Miller-loop launch, one product tree and one final-exponentiation launch.
 * outs[i] receives job i's commitment (the same as vc_commit's), C_out (host, n x 384 B, may
 * be NULL) the C's.  Work runs on `stream` with the workspace and counters of executor ex
 * (NULL: the default executor of pps[0], so the call must not overlap other calls on those
 * params).  Synchronous on return.  VC_EINVAL on a bad argument or an entry >= r (then every
 * outs[i] is NULL). */
int vc_commit_batch(uint32_t n, const vc_params *const *pps, const void *const *m_devs, const uint32_t *entry_bits,
                    vc_exec *ex, void *stream, vc_commitment **outs, uint8_t *C_out);

/* Autotuner of the commit MSM's schedule: for each log2 N in [log_lo, log_hi] and entry width
 * 32 and 256, times the commit MSM kernel (on seeded entries, on `device`) for every slice
 * length from 1024 to 8192 digits per workgroup (capped at a whole subvector) and keeps the
 * fastest.  The choices go into a process-wide table that vc_commit and vc_commit_batch use
 * (results never depend on it: the MSM is exact); with path non-NULL they are also written
 * there as text lines "log_n entry_bits entries_per_block".  Builds test parameters for each
 * size (about as long as vc_setup).  VC_EINVAL for a bad range or an unwritable path. */
int vc_tune_msm(int device, uint32_t log_lo, uint32_t log_hi, const char *path);

/* Replaces the process-wide MSM schedule table with the one in file `path` (as written by
 * vc_tune_msm); NULL restores the default schedule (the most entries a workgroup's shared
 * memory sorts).  VC_EINVAL for an unreadable or malformed file (the table is then unchanged).
 * vc_commit_noalloc always uses the default schedule (its scratch is sized for it). */
int vc_tune_load(const char *path);

/* VC.OpenAll(aux, m) with batch size b, 1 <= b <= K (Protocol 1): all N proofs,
 * kept on the device in shared form (one FC batch proof per block of b
 * subvectors, the folding tree, the HyperEval commitments and the Merkle tree). */
int vc_open_all(const vc_params *pp, const vc_commitment *cm, uint32_t b, void *stream, vc_proofs **out);

/* Executor: the streams, events, workspace and reduction counters that vc_commit,
 * vc_open_all and vc_verify use.  Every vc_params holds a default one (six streams), so calls
 * on the same params must not overlap; calls that run at the same time need executors of
 * their own.  nstreams in [1, 6]: the executor's own stream plus the five side streams of an
 * open-all mapped onto nstreams streams in turn.  Six give one job the most overlap; with
 * many jobs at once fewer streams per job (1 or 2) keep the jobs from sharing hardware
 * queues (GPU_MAX_HW_QUEUES, read once when HIP starts).  Results do not depend on it.
 * Created on `device`, owned by the caller, released with vc_exec_free (after the calls
 * that use it have returned).  VC_EINVAL for nstreams outside [1, 6]. */
int vc_exec_create(int device, uint32_t nstreams, vc_exec **out);
void vc_exec_free(vc_exec *ex);

/* HIP graphs for batched commits on executor ex (on != 0; off by default): vc_commit_batch on
 * this executor captures its fused launch chain (MSM, C_j sums, Miller loops, product tree,
 * final exponentiations, encoding) into a graph on the executor's own stream, and replays the
 * graph on later calls with the same batch shape (number of jobs and the sizes of every
 * packed array) while the executor's workspace stays where it was; the jobs' entries and
 * outputs are reached through the job table the call writes before the replay.  Results are
 * the same as without graphs.  Turning graphs off releases the graph.  Not while profiling
 * (then the chain runs eagerly).  vc_exec_graph_stats: stats[0] captures, stats[1] replays. */
int vc_exec_set_graphs(vc_exec *ex, int on);

/* Step 1 scheduling of open-alls on executor ex (§3 Eq. (folding), Protocol 1 Step 1): their
 * rounds take the next round's terms one round ahead (shorter dependent chain, about four times
 * the Miller loops) while batches x K <= max_pairs, and run direct (the paper's order) above
 * it; the default is 4096.  0 makes every round direct.  Results are the same either way; the
 * footprint reported by vc_open_all_footprint assumes the default. */
int vc_exec_set_ahead(vc_exec *ex, uint64_t max_pairs);
int vc_exec_graph_stats(const vc_exec *ex, uint64_t stats[2]);

/* vc_open_all (Protocol 1, §4.2) on executor ex (of the params' device) instead of the
 * params' default one; `stream` as for vc_open_all. */
int vc_open_all_ex(const vc_params *pp, const vc_commitment *cm, uint32_t b, vc_exec *ex, void *stream,
                   vc_proofs **out);

/* Batched jobs: OpenAll (Protocol 1, §4.2) for n independent vectors, job i on params
 * pps[i] (jobs may share params) with commitment cms[i] and batch size bs[i]; its proofs in
 * outs[i] (n entries), each as from vc_open_all.  At most nexec jobs run at a time, one per
 * executor exs[0..nexec) (each with its own host thread and stream); the jobs are
 * independent latency-bound chains, so several of them share the device; the largest
 * vectors are started first.  All params and
 * executors must be on one device and the executors distinct (VC_EINVAL otherwise).  Returns
 * VC_OK, or the first error; on error every outs[i] is NULL.  While profiling is enabled the jobs run one at a time. */
int vc_open_all_batch(uint32_t n, const vc_params *const *pps, const vc_commitment *const *cms, const uint32_t *bs,
                      uint32_t nexec, vc_exec *const *exs, vc_proofs **outs);

/* Batched jobs with fused launches: as vc_open_all_batch, but jobs on the same params with
 * the same b are opened together, in groups of at most max_group jobs (in input order).  A
 * group is one open-all whose Step 1 (Protocol 1, Eq. genFCBatchProof) runs the batches of
 * all its jobs in lockstep, job after job in one array, so each kernel launch takes the same
 * step of every job's batches (round 1's G_T parts are computed once per job); Step 2 runs
 * job after job on a side stream.  Each outs[i] holds the same bytes as vc_open_all of job
 * i alone.  At most nexec groups run at a time (largest first), one per executor; a group
 * takes workspace for all its batches.  When more than one group runs at a time, groups of
 * several jobs run every Step 1 round direct (measured faster on a shared device), unless
 * the executor's schedule was set with vc_exec_set_ahead.  A failure in any job (including a
 * zero challenge, VC_ECHALLENGE) fails the call: every outs[i] is NULL.  max_group = 1 is
 * vc_open_all_batch. */
int vc_open_all_grouped(uint32_t n, const vc_params *const *pps, const vc_commitment *const *cms,
                        const uint32_t *bs, uint32_t max_group, uint32_t nexec, vc_exec *const *exs,
                        vc_proofs **outs);

/* Device bytes one vc_open_all of (pp, b) holds while it runs: proof bundle, workspace and
 * reduction counters (the bundle stays with the returned proofs).  Host-only: nothing is
 * allocated or launched.  VC_EINVAL for b outside [1, K]. */
int vc_open_all_footprint(const vc_params *pp, uint32_t b, uint64_t *bytes);

/* Serving loop (OpenAll requests of Protocol 1, §4.2, arriving over time): nexec executors of
 * nstreams streams each, one host thread each.  Requests start in arrival order (the oldest
 * waiting request is never overtaken), each when an executor is free and the device bytes the
 * server holds stay within hbm_budget.  Those bytes are: the proof bundles of running requests
 * and of finished ones not yet collected, and the workspace and counters every executor keeps
 * between requests (exact sizes from the open-all's own layout).  A request adds its bundle and
 * what its executor's workspace must grow by; when the oldest does not fit, idle executors
 * release what they keep.  Proofs returned by vc_server_wait belong to the caller and leave
 * the budget.  Collect tickets in submission order: a finished request's bundle counts until
 * it is collected, so waiting first for a later ticket that cannot start would block.
 * VC_EINVAL for nexec outside [1, 64], nstreams outside [1, 6] or a zero budget. */
typedef struct vc_server vc_server;
int vc_server_create(int device, uint32_t nexec, uint32_t nstreams, uint64_t hbm_budget, vc_server **out);
/* Queue a request (params and commitment must stay alive until it is waited for); returns its
 * ticket.  VC_ENOMEM if its footprint alone exceeds the budget, VC_EINVAL for bad arguments. */
int vc_server_submit(vc_server *sv, const vc_params *pp, const vc_commitment *cm, uint32_t b, uint64_t *ticket);
/* Block until request `ticket` has finished; then its proofs (as from vc_open_all) in *out and
 * its return code.  times_ms (optional): [0] time waiting before it started, [1] time from
 * submission to completion (the request's latency).  Each ticket is waited for once, by one
 * thread; VC_EINVAL for an unknown ticket. */
int vc_server_wait(vc_server *sv, uint64_t ticket, vc_proofs **out, double times_ms[2]);
/* Accounting of the budget: stats[0] bytes held now, stats[1] the most held at any time (at
 * most the budget), stats[2] the budget. */
int vc_server_stats(vc_server *sv, uint64_t stats[3]);
/* Finish the running requests, drop the waiting ones and release everything (proofs not
 * collected included).  Not concurrent with other calls on sv. */
void vc_server_free(vc_server *sv);

/* All N proofs of a bundle serialized on the device, in index order, each exactly as
 * vc_proof_get writes it: proofs of batch k (entries i with i / (b M) = k) are
 * vc_proof_len(log N, t_k) bytes long, t_k = min(b, K - k b), and proof i starts where proof
 * i - 1 ends.  dst: device memory of cap bytes, or NULL to get the total length only; *len:
 * the total.  VC_EINVAL if cap is too small. */
int vc_proofs_serialize(const vc_proofs *pr, void *dst, uint64_t cap, uint64_t *len);

/* Verification of all N proofs at once (VC.Verify, appendix C, for every i; section 3
 * FC.BVerify and section 4.2 Step 2).  proofs: the N serialized proofs on the device as
 * vc_proofs_serialize lays them out (16-byte aligned, len bytes in all); m: the N entries on
 * the device, 32 little-endian bytes each; C: the 384-byte commitment (host); seed: 32 bytes
 * (host) from which the random weights of the combined check derive, to be chosen at random
 * after the proofs are fixed.  Items that honest proofs share are compared byte for byte
 * with the proof that represents them; the PST checks of all proofs are combined with random
 * 128-bit weights into one product of log M + 1 pairings (a false accept has probability
 * about 2^-128); the FC part is checked once per batch, and every proof that differs from a
 * representative is checked alone with vc_verify.  Returns 1 if every proof is accepted, 0 if
 * one is rejected, VC_EINVAL for malformed inputs (lengths, alignment, C, entries >= r).
 * n_single (optional): the number of proofs checked alone. */
int vc_verify_all(const vc_params *pp, const uint8_t C[384], uint32_t b, const void *m, const void *proofs,
                  uint64_t len, const uint8_t seed[32], uint64_t *n_single);

/* OpenAll for consecutive sub-arrays (section 4.3): Step 1 alone, the FC batch proofs that
 * open every subvector commitment C_j (j < K), each proving that sub-array m_j (entries
 * [j M, (j + 1) M)) is the j-th segment of the committed vector.  The bundle holds no Merkle
 * tree, y-tree, D-tree or W: vc_proof_get, vc_proofs_serialize and the Step 2 exports
 * (merkle, rho, y, D, W) return VC_EINVAL on it; vc_subarray_proof_get and the FC exports
 * work.  Otherwise as vc_open_all. */
int vc_open_subarrays(const vc_params *pp, const vc_commitment *cm, uint32_t b, void *stream, vc_proofs **out);
/* Length of a sub-array proof whose block holds t subvector commitments: the block, the FC
 * proof (L_j, R_j, A_l, v_l, pi_v) in the wire format of vc_proof_get, which it prefixes. */
uint64_t vc_subarray_proof_len(uint32_t log_n, uint32_t t);
/* The sub-array proof of subvector j (< K) into buf (cap bytes), *len its length; from a
 * vc_open_subarrays or a vc_open_all bundle (then it is the first part of proof j M). */
int vc_subarray_proof_get(const vc_proofs *pr, uint64_t j, uint8_t *buf, size_t cap, size_t *len);
/* Sub-array verification: recomputes PC.Commit of m_j (M entries of 32 little-endian bytes,
 * host), requires it to be entry j of the proof's block, and checks the block with FC.BVerify
 * and the faster verifier (section 3).  1 accept, 0 reject, VC_EINVAL for malformed inputs
 * (lengths, C, an entry >= r). */
int vc_verify_subarray(const vc_params *pp, const uint8_t C[384], uint32_t b, uint64_t j, const uint8_t *m_j,
                       const uint8_t *proof, size_t len);
/* All K sub-array proofs at once: m (device) holds the N entries (32 little-endian bytes
 * each), proofs (device, 16-byte aligned) the K sub-array proofs in order (proof j after
 * proof j - 1, each vc_subarray_proof_len(log N, t_k) bytes), len bytes in all.  Every C_j
 * is recomputed (PC.Commit) and must be entry j of its proof's block; proofs are compared
 * with the first of their batch (honest ones are equal) and the FC part is checked once per
 * batch and for every proof that differs.  1 if all are accepted, 0 if one is rejected,
 * VC_EINVAL for malformed inputs; n_single (optional): the proofs checked by the verifier. */
int vc_verify_subarrays_all(const vc_params *pp, const uint8_t C[384], uint32_t b, const void *m, const void *proofs,
                            uint64_t len, uint64_t *n_single);

/* Evaluation proof of the committed vector's multilinear extension at a point (section 4.3,
 * compatibility with multilinear zkSNARKs): r holds log N little-endian 32-byte field
 * elements r_0 .. r_{log N - 1} (host), x_k paired with bit k of the index (Eq. f_m).  The
 * proof: C_F = sum_j T_j(r_L) C_j (32 bytes), an FC proof that C_F = <C, T(r_L)> (the
 * rounds, A_l, v_l, pi_v, as in vc_proof_get; the query batched with r_0 = H2F(EVAL,
 * SHA-256(EVAL || C || r_{log N - 1} || ... || r_0 || C_F) || 0)), y = f_m(r) (32 bytes,
 * big-endian) and the PST proof of F = sum_j T_j(r_L) f_j at r_R (log M commitments, the
 * quotient of x_{log M - 1} first), vc_eval_proof_len(log N) bytes into out (cap bytes,
 * host); *len its length.  VC_EINVAL for r_k >= r or a short buffer. */
uint64_t vc_eval_proof_len(uint32_t log_n);
int vc_eval_proof(const vc_params *pp, const vc_commitment *cm, const uint8_t *r, void *stream, uint8_t *out,
                  size_t cap, size_t *len);
/* Verification of an evaluation proof (host buffers): FC.BVerify of C_F = <C, T(r_L)> with
 * the faster verifier (section 3) and PC.Verify of F at r_R, e(C_F - y g1, g2) =
 * prod_d e(W_d, (s_var - r_var) g2).  1 accept, 0 reject, VC_EINVAL for malformed inputs
 * (length, C, r_k >= r). */
int vc_verify_eval(const vc_params *pp, const uint8_t C[384], const uint8_t *r, const uint8_t *proof, size_t len);

/* Serialized length of a proof whose block holds t subvector commitments. */
uint64_t vc_proof_len(uint32_t log_n, uint32_t t);

/* Serialize pi_i into buf (host, cap bytes): the block's commitments, the FC batch
 * proof (L_j, R_j, A_l, v_l and the proof of v_l), the fold-tree siblings, the PST
 * proof and the Merkle path, with compressed G1 (32 B) / G2 (64 B) points. */
int vc_proof_get(const vc_proofs *pr, uint64_t i, uint8_t *buf, size_t cap, size_t *len);

/* VC.Verify(C, i, m_i, pi_i) for a proof made with batch size b; m_i is 32 B
 * little-endian.  Returns 1 accept, 0 reject, VC_EINVAL for malformed input. */
int vc_verify(const vc_params *pp, const uint8_t C[384], uint64_t n, uint32_t b, uint64_t i,
              const uint8_t m_i[32], const uint8_t *proof, size_t len);

/* Bulk canonical arrays for parity checks (host destination, cap bytes).
 * params:     what 0 ek level idx (2^idx x G1), 1 vk (log M x G2), 2 h (2K-1 x G2), 3 beta g1
 * commitment: what 0 C_j (K x G1), 1 C (G_T)
 * proofs:     what 0 rounds of batch idx (log K x [L.gt L.g1 R.gt R.g1]), 1 [A_l v_l pi_v] of
 *             batch idx, 2 challenges x_j of batch idx (32 B BE each), 3 Merkle tree (2N x 32 B,
 *             node 1 = root), 4 rho (K x 32 B BE), 5 fold rows ((2K-1) M x 32 B BE),
 *             6 fold commitments ((2K-1) x G1), 7 HyperEval commitments ((M-1) x G1) */
int vc_params_export(const vc_params *pp, int what, uint32_t idx, void *dst, size_t cap, size_t *len);
int vc_commitment_export(const vc_commitment *cm, int what, void *dst, size_t cap, size_t *len);
int vc_proofs_export(const vc_proofs *pr, int what, uint64_t idx, void *dst, size_t cap, size_t *len);

/* Per-kernel timing for measurement: while enabled, every kernel launch of the
 * library (or, after vc_profile_only(name), only launches of the kernel with that
 * name; NULL selects all again) is bracketed by HIP events recorded on its own stream.
 * vc_profile_read writes one line per kernel, "<name> <launches> <total_ms>\n", into
 * buf (NUL-terminated, truncated to cap) and returns the size needed.
 * vc_profile_enable also clears previous records (waiting for the device first if
 * there are any).  The events come from a pool kept until the process ends.  Not
 * thread-safe. */
void vc_profile_enable(int on);
void vc_profile_only(const char *kernel);
int vc_profile_read(char *buf, size_t cap);

/* Test hook for the zero-challenge error (section 3, FC.BOpen: the fold needs x_j^{-1}, so
 * a challenge of zero ends the proof; a hashed challenge is zero with probability about
 * 2^-254, so nothing else reaches that path).  round >= 1: every later open-all
 * (vc_open_all, vc_open_all_ex, vc_open_all_batch, the serving loop, sub-arrays,
 * evaluation proofs) replaces batch 0's challenge x_round by zero and returns
 * VC_ECHALLENGE, releasing the bundle it made; 0 (the default) turns the hook off.
 * Process-wide; for tests only. */
void vc_test_zero_challenge(uint32_t round);

/* Self-test of the device field layer used by the proof rounds (8 lanes per
 * element): one operation on n pairs of canonical 32-byte little-endian host inputs,
 * results to out (n x 32 B).  op: 0 mul, 1 add, 2 sub, 3 halve, 4 inverse, 5 square;
 * which: 0 = F_p, 1 = F_r.  Inputs must be < the modulus.  which 2 (F_p) or 3 (F_r): raw
 * Montgomery limbs in and out with no conversion (ops 0 mul, 1 add, 2 sub), any 256-bit
 * inputs, for checking the layout's output range. */
int vc_diag_field(int which, int op, uint64_t n, const void *a, const void *b, void *out);

/* Diagnostic: the y-tree passes of Step 2 (the randomized folding tree, Protocol 1 Step 2
 * Eq. ProverRand; all weights rho_j = 1) over commitment cm's entries, alone on the device:
 * writes the best of five timed runs (after a warm-up), in milliseconds, to ms.  Their
 * algorithmic traffic is 32 (N + (2K - 1) M) bytes (the entries read once, every node written
 * once), for an HBM throughput figure free of the concurrent Step 1 kernels. */
int vc_diag_fold(const vc_commitment *cm, double *ms);

/* Diagnostic: measured throughput of the 32 x 32 -> 64-bit multiply-add on `device`, in
 * 10^12 multiply-adds per second (best of five timed launches of a probe kernel that keeps
 * every SIMD busy with independent chains).  The roofline's ALU peak. */
int vc_diag_mad_rate(int device, double *tera_per_s);

void vc_params_free(vc_params *pp);
void vc_commitment_free(vc_commitment *cm);
void vc_proofs_free(vc_proofs *pr);
const char *vc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
