// FlexProofs C ABI (include/vc.h): host orchestration of the HIP kernels.
//
// Every arithmetic step runs in kernels (kernels.hip); this file only sizes and
// carves device buffers, orders launches on the caller's stream, and formats the
// proof bytes (point compression is a byte-level encoding of values the device
// already produced in canonical form).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <string>
#include <vector>
#include <thread>
#include <atomic>
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include "kernels.h"
#include "verify.h"
#include "vc.h"

#define VC_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local char g_last_error[256] = "";

int hip_fail(hipError_t e, const char *where) {
  snprintf(g_last_error, sizeof g_last_error, "%s: %s", where, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? VC_ENOMEM : VC_EDEVICE;
}

#define CK(x)                                         \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #x);    \
  } while (0)
#define CKL(where)                                    \
  do {                                                \
    hipError_t e_ = hipGetLastError();                \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// A bump allocator over one device allocation.
struct Carve {
  size_t off = 0;
  template <class T> size_t take(uint64_t n) {
    size_t o = off;
    off = align_up(off + n * sizeof(T));
    return o;
  }
};

template <class T> T *at(void *base, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }

}  // namespace

// ------------------------------------------------------------------ profiling hooks
namespace {
struct ProfRec {
  const char *name;
  hipEvent_t e0, e1;
};
bool g_prof = false;
std::string g_prof_only;          // empty: every kernel
std::atomic<uint32_t> g_zero_round{0};  // test hook: round whose batch-0 challenge is forced to zero
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;  // timing events, reused across profiling runs
size_t g_prof_next = 0;
thread_local hipEvent_t g_prof_open = nullptr;

hipEvent_t prof_event() {
  if (g_prof_next == g_prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof_pool.push_back(e);
  }
  return g_prof_pool[g_prof_next++];
}
}  // namespace

namespace dbg {
bool on() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("VC_DEBUG_SYNC");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}
void check(const char *name, hipStream_t st) {
  hipError_t e0 = hipGetLastError();
  hipError_t e1 = hipStreamSynchronize(st);
  hipError_t e2 = hipGetLastError();
  if (e0 != hipSuccess || e1 != hipSuccess || e2 != hipSuccess)
    fprintf(stderr, "[vc debug] after %s: %s / %s / %s\n", name, hipGetErrorString(e0), hipGetErrorString(e1),
            hipGetErrorString(e2));
}
}  // namespace dbg

namespace prof {
void begin(const char *name, hipStream_t st) {
  g_prof_open = nullptr;
  if (!g_prof || (!g_prof_only.empty() && g_prof_only != name)) return;
  g_prof_open = prof_event();
  if (g_prof_open) (void)hipEventRecord(g_prof_open, st);
}
void end(hipStream_t st) {
  if (!g_prof || !g_prof_open) return;
  hipEvent_t e1 = prof_event();
  if (!e1) { g_prof_open = nullptr; return; }
  (void)hipEventRecord(e1, st);
  g_prof_recs.push_back({nullptr, g_prof_open, e1});
  g_prof_open = nullptr;
}
void name_last(const char *name) {
  if (g_prof && !g_prof_recs.empty() && !g_prof_recs.back().name) g_prof_recs.back().name = name;
}
}  // namespace prof

// Per-call resources of open-all (and commit / verify): side streams (default priority),
// fork/join events, the grow-only workspace and the arrival counters of the one-launch
// reduction trees (zeroed once; each tree leaves its counters zero again).  Calls that run at
// the same time need executors of their own; each params holds a default one.  An executor
// owns 1..6 streams: main (the job's stream in batch calls) and the five side streams map
// onto them in turn, so with fewer than six the side work shares streams (same results,
// less overlap inside one job, fewer hardware queues per job when many jobs run at once).
struct vc_exec {
  int device;
  void *ws = nullptr;
  size_t ws_size = 0;
  hipStream_t own[6] = {};
  uint32_t nown = 0;
  hipStream_t main = nullptr;
  hipStream_t side[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev[23] = {};
  uint32_t *cnt = nullptr;
  uint64_t cnt_n = 0;
  bool cnt_dirty = false;  // counters to be zeroed before the next use (new, or left by a failed call)
  // batched commits: capture their fused launch chain into a HIP graph and replay it while the
  // batch shape and the workspace stay the same (vc_exec_set_graphs)
  bool graphs = false;
  hipGraphExec_t cgraph = nullptr;
  std::vector<uint64_t> ckey;  // the shape and buffers the graph was captured for
  uint64_t captures = 0, replays = 0;
  uint64_t ahead_max = 0;  // open-alls take terms one round ahead when batches x K <= this (vc_exec_set_ahead)
  bool ahead_set = false;  // set by the caller (else batched calls may choose for it)
};

static void drop_graph(vc_exec *ex) {
  if (ex->cgraph) (void)hipGraphExecDestroy(ex->cgraph);
  ex->cgraph = nullptr;
  ex->ckey.clear();
}

struct vc_params {
  int device;
  uint32_t L, lK, lM;
  uint64_t N, K, M;
  void *mem = nullptr;      // all keys in one allocation
  g1_aff *ek, *g1gen, *g1beta, *table;
  g2_aff *vk, *h, *g2gen;
  g2_aff *htab;  // 2^{8 w} h_m (w < 32, m < 2K - 2): fixed-base table of the KZG proof's MSM
  g2_aff *hm;    // 2^{16 p} h_m (p = 1..3, m < 2K - 2) for the split KZG terms
  vc_exec *ex = nullptr;  // default executor of calls on these params
};

// Step 1 takes the next round's terms ahead (oa_terms.hpp) when the batches leave the
// device mostly idle: at most this many (batch, index) pairs per round.  Beyond it the
// doubled Miller-loop count of that scheme costs more than the shorter chain saves.
static constexpr uint64_t AHEAD_MAX_PAIRS = 4096;
// in the ahead mode, rounds of more than this many pairs (batches x h) still run direct: the
// device is full there and the terms taken ahead (twice the Miller loops) cost more than the
// shorter chain saves; the first round at or below it is the first taken ahead
static constexpr uint64_t DIRECT_MIN = 512;
// folds of at most this many pairs (batches x h) run as four-part split multiplications
static constexpr uint64_t FOLD_SPLIT_MAX = 256;
// direct-round Miller loops and G2 folds of at least this many (batch, index) pairs run on the
// wide layout (8 lanes per element, throughput), smaller ones on the engine (latency)
static constexpr uint64_t WIDE_FOLD_MIN = 4096;
// bases per block of the KZG proof's G2 MSM (times 32 windows: at most 8192 digits): long
// slices when the MSMs of all batches give at least KZG_LONG_MIN_BLOCKS blocks (the bucket
// reduction, about 2300 G2 additions per block, is then spread over eight times the digits),
// short ones otherwise (more blocks, shorter chains, for few batches)
static constexpr uint32_t KZG_S = 32, KZG_S_LONG = 256;
static constexpr uint64_t KZG_LONG_MIN_BLOCKS = 512;
// KZG proofs of at most this many split jobs (4 per term) run as split multiplications
// instead of the MSM: when the device is nearly idle the shorter chain wins
static constexpr uint64_t KZG_SPLIT_MAX = 8192;

// fork: `to` waits for the work issued so far on `from`
static int stream_wait(vc_exec *ex, int slot, hipStream_t from, hipStream_t to) {
  CK(hipEventRecord(ex->ev[slot], from));
  CK(hipStreamWaitEvent(to, ex->ev[slot], 0));
  return VC_OK;
}
// the same split in two: mark the work issued so far on a stream, wait for the mark later
static int ev_mark(vc_exec *ex, int slot, hipStream_t from) {
  CK(hipEventRecord(ex->ev[slot], from));
  return VC_OK;
}
static int ev_wait(vc_exec *ex, int slot, hipStream_t to) {
  CK(hipStreamWaitEvent(to, ex->ev[slot], 0));
  return VC_OK;
}

struct vc_commitment {
  const vc_params *pp;
  int device = 0;  // its own copy: a handle may be released after its params
  void *mem = nullptr;
  fe *m;          // N canonical entries
  g1_aff *Cj;     // K
  fp12 *C;        // 1
};

struct vc_proofs {
  const vc_params *pp;
  int device = 0;  // its own copy: a handle may be released after its params
  uint32_t b;
  uint64_t nb;
  void *mem = nullptr;  // the proof bundle
  size_t o_Cj, o_C, o_Lgt, o_Rgt, o_Lg1, o_Rg1, o_X, o_Al, o_vl, o_piv, o_tree, o_rho, o_Y, o_D, o_W;
  bool step2 = true;    // false: sub-array proofs only (Step 1), no Merkle tree, y-tree, D-tree or W
  size_t o_CF = 0, o_yv = 0, o_We = 0;  // evaluation proof: C_F, F(r_R), the PST quotients W_d
};

// At least n zeroed arrival counters.  New ones are cleared on the call's stream `st`, ahead of
// every launch of the call (its side streams fork from st later): a plain hipMemset runs on the
// null stream, which the non-blocking streams of the executor do not wait for.
static int ensure_cnt(vc_exec *ex, uint64_t n, hipStream_t st) {
  if (ex->cnt_n < n) {
    if (ex->cnt) CK(hipFree(ex->cnt));
    ex->cnt = nullptr;
    ex->cnt_n = 0;
    CK(hipMalloc(&ex->cnt, n * sizeof(uint32_t)));
    ex->cnt_n = n;
    ex->cnt_dirty = true;
  }
  if (ex->cnt_dirty) {
    CK(hipMemsetAsync(ex->cnt, 0, ex->cnt_n * sizeof(uint32_t), st));
    ex->cnt_dirty = false;
  }
  return VC_OK;
}

static int ensure_ws(vc_exec *ex, size_t need) {
  if (ex->ws_size >= need) return VC_OK;
  if (ex->ws) CK(hipFree(ex->ws));
  ex->ws = nullptr;
  ex->ws_size = 0;
  CK(hipMalloc(&ex->ws, need));
  ex->ws_size = need;
  return VC_OK;
}

// release the workspace and counters an executor keeps between calls (its next call
// allocates them again)
static void exec_release(vc_exec *ex) {
  (void)hipSetDevice(ex->device);
  drop_graph(ex);  // it refers to the buffers released below
  if (ex->ws) (void)hipFree(ex->ws);
  if (ex->cnt) (void)hipFree(ex->cnt);
  ex->ws = nullptr;
  ex->ws_size = 0;
  ex->cnt = nullptr;
  ex->cnt_n = 0;
  ex->cnt_dirty = false;
}

VC_API void vc_exec_free(vc_exec *ex) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!ex) return;
  (void)hipSetDevice(ex->device);
  drop_graph(ex);
  if (ex->ws) (void)hipFree(ex->ws);
  if (ex->cnt) (void)hipFree(ex->cnt);
  for (auto sd : ex->own)
    if (sd) (void)hipStreamDestroy(sd);
  for (auto ev : ex->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete ex;
  (void)hipGetLastError();  // a release reports nothing and leaves no error behind
}

VC_API int vc_exec_set_graphs(vc_exec *ex, int on) {
  if (!ex) return VC_EINVAL;
  ex->graphs = on != 0;
  if (!ex->graphs) {
    (void)hipSetDevice(ex->device);
    drop_graph(ex);
  }
  return VC_OK;
}

VC_API int vc_exec_set_ahead(vc_exec *ex, uint64_t max_pairs) {
  if (!ex) return VC_EINVAL;
  ex->ahead_max = max_pairs;
  ex->ahead_set = true;
  return VC_OK;
}

VC_API int vc_exec_graph_stats(const vc_exec *ex, uint64_t stats[2]) {
  if (!ex || !stats) return VC_EINVAL;
  stats[0] = ex->captures;
  stats[1] = ex->replays;
  return VC_OK;
}

VC_API int vc_exec_create(int device, uint32_t nstreams, vc_exec **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!out) return VC_EINVAL;
  *out = nullptr;
  if (nstreams < 1 || nstreams > 6) return VC_EINVAL;
  CK(hipSetDevice(device));
  vc_exec *ex = new vc_exec();
  ex->device = device;
  ex->ahead_max = AHEAD_MAX_PAIRS;
  hipError_t e = hipSuccess;
  for (uint32_t i = 0; i < nstreams && e == hipSuccess; i++) {
    e = hipStreamCreateWithFlags(&ex->own[i], hipStreamNonBlocking);
    if (e == hipSuccess) ex->nown = i + 1;
  }
  if (e == hipSuccess) {
    ex->main = ex->own[0];
    for (uint32_t i = 0; i < 5; i++) ex->side[i] = ex->own[(i + 1) % nstreams];
  }
  for (auto &ev : ex->ev)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    vc_exec_free(ex);
    return hip_fail(e, "vc_exec_create");
  }
  *out = ex;
  return VC_OK;
}

static const uint32_t NWIN = 32;  // 8-bit windows of a 256-bit scalar

VC_API uint64_t vc_proof_len(uint32_t log_n, uint32_t t) {
  uint32_t lK = log_n / 2, lM = log_n - lK;
  return 32ull * t + lK * (2ull * 384 + 2 * 32) + 32 + 64 + 64 + lK * 64ull + lM * 32ull + 32ull * log_n;
}

VC_API const char *vc_strerror(int code) {
  switch (code) {
    case VC_OK: return "ok";
    case VC_EINVAL: return "invalid argument";
    case VC_ENOMEM: return "device out of memory";
    case VC_EDEVICE: return g_last_error[0] ? g_last_error : "device error";
    case VC_ENOTIMPL: return "not implemented";
    case VC_ECHALLENGE: return "zero Fiat-Shamir challenge";
  }
  return "unknown error";
}

// ------------------------------------------------------------------ setup
// the parameters' executor and key memory for N = 2^log_n (keys not yet written)
static int params_alloc(uint32_t log_n, int device, vc_params **out) {
  vc_params *pp = new vc_params();
  pp->device = device;
  if (int rc = vc_exec_create(device, 6, &pp->ex)) {
    vc_params_free(pp);
    return rc;
  }
  pp->L = log_n;
  pp->lK = log_n / 2;
  pp->lM = log_n - pp->lK;
  pp->N = 1ull << log_n;
  pp->K = 1ull << pp->lK;
  pp->M = 1ull << pp->lM;
  uint64_t K = pp->K, M = pp->M, lM = pp->lM;
  Carve c;
  size_t o_ek = c.take<g1_aff>(2 * M - 1), o_g1 = c.take<g1_aff>(1), o_g1b = c.take<g1_aff>(1);
  size_t o_tab = c.take<g1_aff>(NWIN * M), o_vk = c.take<g2_aff>(lM), o_h = c.take<g2_aff>(2 * K - 1);
  size_t o_g2 = c.take<g2_aff>(1), o_htab = c.take<g2_aff>(NWIN * (2 * K - 2)), o_hm = c.take<g2_aff>(3 * (2 * K - 2));
  hipError_t e = hipMalloc(&pp->mem, c.off);
  if (e != hipSuccess) {
    vc_params_free(pp);
    return hip_fail(e, "vc_setup alloc");
  }
  pp->ek = at<g1_aff>(pp->mem, o_ek);
  pp->g1gen = at<g1_aff>(pp->mem, o_g1);
  pp->g1beta = at<g1_aff>(pp->mem, o_g1b);
  pp->table = at<g1_aff>(pp->mem, o_tab);
  pp->vk = at<g2_aff>(pp->mem, o_vk);
  pp->h = at<g2_aff>(pp->mem, o_h);
  pp->g2gen = at<g2_aff>(pp->mem, o_g2);
  pp->htab = at<g2_aff>(pp->mem, o_htab);
  pp->hm = at<g2_aff>(pp->mem, o_hm);
  g1_aff g1 = {fe_const(bn::G1X), fe_const(bn::G1Y)};
  g2_aff g2 = {{fe_const(bn::G2X0), fe_const(bn::G2X1)}, {fe_const(bn::G2Y0), fe_const(bn::G2Y1)}};
  e = hipMemcpy(pp->g1gen, &g1, sizeof g1, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pp->g2gen, &g2, sizeof g2, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    vc_params_free(pp);
    return hip_fail(e, "vc_setup");
  }
  *out = pp;
  return VC_OK;
}

// fixed-base tables of the keys: the commit MSM's 2^{8 w} ek_{l_M}[a], the KZG MSM's
// 2^{8 w} h_m and the split KZG terms' 2^{16 p} h_m
static void params_tables(vc_params *pp, hipStream_t st) {
  const uint64_t K = pp->K, M = pp->M;
  kl::msm_tables_g2(pp->h, 2 * K - 2, NWIN, pp->htab, st);
  ks::g2_dbl_mults(pp->h, 2 * K - 2, 0, 2 * K - 2, pp->hm, st);
  kl::msm_tables(pp->ek + (M - 1), M, NWIN, pp->table, st);
}

VC_API int vc_setup(uint32_t log_n, const uint8_t seed[32], int device, vc_params **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!out || !seed || log_n < 2 || log_n > VC_MAX_LOG_N) return VC_EINVAL;
  *out = nullptr;
  CK(hipSetDevice(device));
  vc_params *pp = nullptr;
  if (int rc = params_alloc(log_n, device, &pp)) return rc;
  vc_exec *ex = pp->ex;
  const uint64_t K = pp->K, M = pp->M, lM = pp->lM;
  // temporaries: seed, trapdoor, weights
  Carve t;
  size_t o_seed = t.take<uint8_t>(32), o_s = t.take<fe>(lM + 1), o_beta = t.take<fe>(1);
  size_t o_w = t.take<fe>(2 * M - 1), o_pw = t.take<fe>(2 * K - 1);
  int rc = ensure_ws(ex, t.off);
  if (rc) { vc_params_free(pp); return rc; }
  hipStream_t st = nullptr;
  void *ws = ex->ws;
  hipError_t e = hipMemcpy(at<uint8_t>(ws, o_seed), seed, 32, hipMemcpyHostToDevice);
  if (e != hipSuccess) { vc_params_free(pp); return hip_fail(e, "vc_setup"); }
  fe *s = at<fe>(ws, o_s), *beta = at<fe>(ws, o_beta), *w = at<fe>(ws, o_w), *pw = at<fe>(ws, o_pw);
  kl::trapdoor(at<uint8_t>(ws, o_seed), pp->lM, s, beta, st);
  kl::ek_weights(pp->lM, s, w, 2 * M - 1, st);
  klw::g1_mul(pp->g1gen, 1, w, 2 * M - 1, pp->ek, st);
  klw::g2_mul(pp->g2gen, 1, s, lM, pp->vk, st);
  kl::pow_table(beta, pw, 2 * K - 1, st);
  klw::g2_mul(pp->g2gen, 1, pw, 2 * K - 1, pp->h, st);
  klw::g1_mul(pp->g1gen, 1, beta, 1, pp->g1beta, st);
  params_tables(pp, st);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) { vc_params_free(pp); return hip_fail(e, "vc_setup"); }
  *out = pp;
  return VC_OK;
}

// bytes of an SRS for N = 2^log_n in vc_params_load's layout
static uint64_t srs_bytes(uint32_t log_n) {
  const uint64_t lK = log_n / 2, lM = log_n - lK, K = 1ull << lK, M = 1ull << lM;
  return 64 * (2 * M - 1) + 128 * lM + 128 * (2 * K - 1) + 64;
}

VC_API int vc_params_load(const uint8_t *srs, size_t len, int device, vc_params **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!out || !srs) return VC_EINVAL;
  *out = nullptr;
  uint32_t log_n = 0;
  for (uint32_t L = 2; L <= VC_MAX_LOG_N && !log_n; L++)
    if (srs_bytes(L) == len) log_n = L;
  if (!log_n) return VC_EINVAL;
  CK(hipSetDevice(device));
  vc_params *pp = nullptr;
  if (int rc = params_alloc(log_n, device, &pp)) return rc;
  const uint64_t K = pp->K, M = pp->M, lM = pp->lM;
  const uint64_t n_ek = 2 * (2 * M - 1), n_vk = 4 * lM, n_h = 4 * (2 * K - 1), n_fe = len / 32;
  Carve t;
  size_t o_err = t.take<int>(1), o_in = t.take<uint8_t>(len), o_fe = t.take<fe>(n_fe);
  int rc = ensure_ws(pp->ex, t.off);
  if (rc) { vc_params_free(pp); return rc; }
  hipStream_t st = nullptr;
  void *ws = pp->ex->ws;
  int *err = at<int>(ws, o_err);
  fe *v = at<fe>(ws, o_fe);
  int herr = 0;
  hipError_t e = hipMemcpy(at<uint8_t>(ws, o_in), srs, len, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    kl::zero_u32(reinterpret_cast<uint32_t *>(err), 1, st);
    kl::decode_fp(at<uint8_t>(ws, o_in), n_fe, v, err, st);
    e = hipGetLastError();
  }
  // the decoded elements are the key arrays' memory images, in the order ek, vk, h, beta g1
  if (e == hipSuccess) e = hipMemcpyAsync(pp->ek, v, n_ek * sizeof(fe), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(pp->vk, v + n_ek, n_vk * sizeof(fe), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(pp->h, v + n_ek + n_vk, n_h * sizeof(fe), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(pp->g1beta, v + n_ek + n_vk + n_h, 2 * sizeof(fe), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) {
    kl::check_curve_g1(pp->ek, 2 * M - 1, err, st);
    kl::check_curve_g1(pp->g1beta, 1, err, st);
    kl::check_curve_g2(pp->vk, lM, err, st);
    kl::check_curve_g2(pp->h, 2 * K - 1, err, st);
    params_tables(pp, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) { vc_params_free(pp); return hip_fail(e, "vc_params_load"); }
  if (herr) { vc_params_free(pp); return VC_EINVAL; }
  *out = pp;
  return VC_OK;
}

VC_API void vc_params_free(vc_params *pp) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp) return;
  (void)hipSetDevice(pp->device);
  if (pp->mem) (void)hipFree(pp->mem);
  vc_exec_free(pp->ex);
  delete pp;
  (void)hipGetLastError();  // a release reports nothing and leaves no error behind
}

// ------------------------------------------------------------------ commit
// ------------------------------------------------------------------ MSM schedule
// Entries per block of the commit MSM (its slice length S), per (log N, entry bits): the
// autotuner's choice (vc_tune_msm, vc_tune_load), else as many as a block's shared-memory sort
// holds (MSM_MAXE = 8192 digits).  Process-wide; results do not depend on it.
namespace {
std::mutex g_tune_mu;
std::map<std::pair<uint32_t, uint32_t>, uint32_t> g_tune;
constexpr uint32_t MSM_DIGITS = 8192;  // digits one MSM block sorts in shared memory

uint32_t msm_slice_len(uint32_t L, uint64_t M, uint32_t bits) {
  const uint32_t nwin = bits == 32 ? 4 : NWIN;
  uint32_t S = MSM_DIGITS / nwin;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({L, bits});
    if (it != g_tune.end()) S = it->second;
  }
  if (S > M) S = (uint32_t)M;
  return S;
}
}  // namespace

VC_API int vc_commit(const vc_params *cpp, const void *m_dev, uint64_t n, uint32_t entry_bits, void *stream,
                     vc_commitment **out, uint8_t C_out[384]) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!cpp || !m_dev || !out || n != cpp->N || (entry_bits != 32 && entry_bits != 256)) return VC_EINVAL;
  const vc_params *pp = cpp;
  vc_exec *ex = pp->ex;
  *out = nullptr;
  CK(hipSetDevice(pp->device));
  hipStream_t st = (hipStream_t)stream;
  uint64_t N = pp->N, K = pp->K, M = pp->M;
  vc_commitment *cm = new vc_commitment();
  cm->pp = pp;
  cm->device = pp->device;
  Carve c;
  size_t o_m = c.take<fe>(N), o_Cj = c.take<g1_aff>(K), o_C = c.take<fp12>(1);
  hipError_t e = hipMalloc(&cm->mem, c.off);
  if (e != hipSuccess) { delete cm; return hip_fail(e, "vc_commit alloc"); }
  cm->m = at<fe>(cm->mem, o_m);
  cm->Cj = at<g1_aff>(cm->mem, o_Cj);
  cm->C = at<fp12>(cm->mem, o_C);
  uint32_t nwin = entry_bits == 32 ? 4 : NWIN;
  uint32_t S = msm_slice_len(pp->L, M, entry_bits);
  uint64_t nslice = (M + S - 1) / S;
  Carve t;
  size_t o_err = t.take<int>(1), o_part = t.take<g1_jac>(K * nslice), o_F = t.take<fp12>(K), o_enc = t.take<uint8_t>(384);
  int rc = ensure_ws(ex, t.off);
  if (rc) { vc_commitment_free(cm); return rc; }
  void *ws = ex->ws;
  int *err = at<int>(ws, o_err);
  CK(hipMemsetAsync(err, 0, sizeof(int), st));
  if (entry_bits == 32) {
    kl::lift_u32((const uint32_t *)m_dev, N, cm->m, st);
  } else {
    CK(hipMemcpyAsync(cm->m, m_dev, N * sizeof(fe), hipMemcpyDeviceToDevice, st));
    kl::check_fr(cm->m, N, err, st);
  }
  // PC.Commit for every subvector: K MSMs of M terms over the shared Lagrange keys
  g1_jac *part = at<g1_jac>(ws, o_part);
  kl::msm_slices(cm->m, K, M, nwin, S, pp->table, part, st);
  klw::sum_g1(part, K, nslice, cm->Cj, st);
  // FC.Commit: C = prod_j e(C_j, v[j]), v[j] = h[2j]
  fp12 *F = at<fp12>(ws, o_F);
  ks::miller(cm->Cj, 1, pp->h, 2, K, F, st);
  if (int rc = ensure_cnt(ex, tree_counters(K), st)) { vc_commitment_free(cm); return rc; }
  ks::f12_reduce(F, 1, K, K, ex->cnt, st);
  ks::final_exp(F, 1, 1, cm->C, nullptr, 1, st);
  uint8_t *enc = at<uint8_t>(ws, o_enc);
  kl::encode(reinterpret_cast<const fe *>(cm->C), 12, 0, enc, st);
  int herr = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && C_out) e = hipMemcpyAsync(C_out, enc, 384, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    ex->cnt_dirty = true;  // the product tree may have stopped half way
    vc_commitment_free(cm);
    return hip_fail(e, "vc_commit");
  }
  if (herr & VC_ERRBIT_RANGE) { vc_commitment_free(cm); return VC_EINVAL; }
  *out = cm;
  return VC_OK;
}

VC_API void vc_commitment_free(vc_commitment *cm) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!cm) return;
  (void)hipSetDevice(cm->device);
  if (cm->mem) (void)hipFree(cm->mem);
  delete cm;
  (void)hipGetLastError();  // a release reports nothing and leaves no error behind
}

// ------------------------------------------------------------------ batched commit
// VC.Commit of n vectors at once: every job's PC.Commit MSM blocks in one persistent launch
// (k_msm_batch), their C_j in one launch, all FC.Commit Miller loops in one launch over the
// packed (C_j, v_j) pairs, one product tree over per-job segments padded with ones, and one
// final exponentiation launch for all C.
VC_API int vc_commit_batch(uint32_t n, const vc_params *const *pps, const void *const *m_devs, const uint32_t *entry_bits,
                           vc_exec *exa, void *stream, vc_commitment **outs, uint8_t *C_out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pps || !m_devs || !entry_bits || !outs) return VC_EINVAL;
  for (uint32_t i = 0; i < n; i++) outs[i] = nullptr;
  if (n == 0) return VC_OK;
  for (uint32_t i = 0; i < n; i++)
    if (!pps[i] || !m_devs[i] || (entry_bits[i] != 32 && entry_bits[i] != 256) || pps[i]->device != pps[0]->device)
      return VC_EINVAL;
  vc_exec *ex = exa ? exa : pps[0]->ex;
  if (ex->device != pps[0]->device) return VC_EINVAL;
  CK(hipSetDevice(pps[0]->device));
  hipStream_t st = (hipStream_t)stream;
  struct Release {
    std::vector<vc_commitment *> c;
    bool keep = false;
    ~Release() {
      if (!keep)
        for (vc_commitment *q : c) vc_commitment_free(q);
    }
  } rel;
  std::vector<CJob> J(n);
  uint64_t blocks = 0, totalK = 0, parts = 0, Kmax = 0;
  for (uint32_t x = 0; x < n; x++) {
    const vc_params *pp = pps[x];
    vc_commitment *cm = new vc_commitment();
    rel.c.push_back(cm);
    cm->pp = pp;
    cm->device = pp->device;
    Carve c;
    size_t o_m = c.take<fe>(pp->N), o_Cj = c.take<g1_aff>(pp->K), o_C = c.take<fp12>(1);
    hipError_t e = hipMalloc(&cm->mem, c.off);
    if (e != hipSuccess) return hip_fail(e, "vc_commit_batch alloc");
    cm->m = at<fe>(cm->mem, o_m);
    cm->Cj = at<g1_aff>(cm->mem, o_Cj);
    cm->C = at<fp12>(cm->mem, o_C);
    const uint32_t S = msm_slice_len(pp->L, pp->M, entry_bits[x]);
    const uint64_t nslice = (pp->M + S - 1) / S;
    J[x] = {cm->m, pp->table, pp->h, nullptr, cm->Cj, cm->C, pp->M, pp->K, nslice, blocks, totalK,
            entry_bits[x] == 32 ? 4u : NWIN, S};
    blocks += pp->K * nslice;
    parts += pp->K * nslice;
    totalK += pp->K;
    Kmax = std::max<uint64_t>(Kmax, pp->K);
  }
  Carve t;
  size_t o_err = t.take<int>(1), o_J = t.take<CJob>(n), o_part = t.take<g1_jac>(parts), o_Cp = t.take<g1_aff>(totalK),
         o_v = t.take<g2_aff>(totalK), o_Fc = t.take<fp12>(totalK), o_F = t.take<fp12>(n * Kmax),
         o_Cs = t.take<fp12>(n), o_enc = t.take<uint8_t>(384ull * n);
  if (int rc = ensure_ws(ex, t.off)) return rc;
  if (int rc = ensure_cnt(ex, n * tree_counters(Kmax), st)) return rc;
  void *ws = ex->ws;
  for (uint64_t x = 0, o = 0; x < n; o += J[x].K * J[x].nslice, x++) J[x].part = at<g1_jac>(ws, o_part) + o;
  int *err = at<int>(ws, o_err);
  CJob *Jd = at<CJob>(ws, o_J);
  kl::zero_u32(reinterpret_cast<uint32_t *>(err), 1, st);
  CK(hipMemcpyAsync(Jd, J.data(), n * sizeof(CJob), hipMemcpyHostToDevice, st));
  for (uint32_t x = 0; x < n; x++) {
    vc_commitment *cm = rel.c[x];
    if (entry_bits[x] == 32) {
      kl::lift_u32(static_cast<const uint32_t *>(m_devs[x]), pps[x]->N, cm->m, st);
    } else {
      CK(hipMemcpyAsync(cm->m, m_devs[x], pps[x]->N * sizeof(fe), hipMemcpyDeviceToDevice, st));
      kl::check_fr(cm->m, pps[x]->N, err, st);
    }
  }
  const unsigned grid = (unsigned)std::min<uint64_t>(blocks, kl::msm_batch_grid(pps[0]->device));
  g1_aff *Cp = at<g1_aff>(ws, o_Cp);
  g2_aff *v = at<g2_aff>(ws, o_v);
  fp12 *Fc = at<fp12>(ws, o_Fc), *F = at<fp12>(ws, o_F), *Cs = at<fp12>(ws, o_Cs);
  uint8_t *enc = at<uint8_t>(ws, o_enc);
  // the fused chain: its arguments are the workspace's buffers and the batch's shape; each
  // job's entries and outputs are reached through the job table written above
  auto chain = [&](hipStream_t s) {
    kl::msm_batch(Jd, n, blocks, grid, s);
    klw::commit_sums(Jd, n, totalK, Cp, s);
    kl::commit_v(Jd, n, totalK, v, s);
    ks::miller(Cp, 1, v, 1, totalK, Fc, s);
    kl::commit_pad(Jd, n, Kmax, Fc, F, s);
    ks::f12_reduce(F, n, Kmax, Kmax, ex->cnt, s);
    // (input s goes to (s odd ? out1 : out0)[(s >> 1) ostride]: Cs[s] for every job)
    ks::final_exp(F, Kmax, n, Cs, Cs + 1, 2, s);
    kl::commit_store(Jd, n, Cs, s);
    kl::encode(reinterpret_cast<const fe *>(Cs), 12ull * n, 0, enc, s);
  };
  if (!ex->graphs || g_prof || dbg::on()) {
    chain(st);
  } else {
    // captured on the executor's own stream (the caller's may be the null stream, which cannot
    // be captured) and replayed there between the caller's work before and after it
    std::vector<uint64_t> key = {n, blocks, totalK, Kmax, grid, (uint64_t)(uintptr_t)ws, (uint64_t)(uintptr_t)ex->cnt,
                                 o_J, o_part, o_Cp, o_v, o_Fc, o_F, o_Cs, o_enc};
    hipStream_t gs = ex->main;
    if (!ex->cgraph || key != ex->ckey) {
      drop_graph(ex);
      hipGraph_t g = nullptr;
      CK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      chain(gs);
      hipError_t ec = hipStreamEndCapture(gs, &g);
      if (ec == hipSuccess) ec = hipGraphInstantiate(&ex->cgraph, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (ec != hipSuccess) {
        ex->cgraph = nullptr;
        return hip_fail(ec, "vc_commit_batch capture");
      }
      ex->ckey = key;
      ex->captures++;
    }
    if (int rc = stream_wait(ex, 0, st, gs)) return rc;
    CK(hipGraphLaunch(ex->cgraph, gs));
    ex->replays++;
    if (int rc = stream_wait(ex, 1, gs, st)) return rc;
  }
  int herr = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && C_out) e = hipMemcpyAsync(C_out, enc, 384ull * n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    ex->cnt_dirty = true;  // the product tree may have stopped half way
    return hip_fail(e, "vc_commit_batch");
  }
  if (herr & VC_ERRBIT_RANGE) return VC_EINVAL;
  rel.keep = true;
  for (uint32_t x = 0; x < n; x++) outs[x] = rel.c[x];
  return VC_OK;
}

// ------------------------------------------------------------------ MSM schedule autotuner
namespace {
// seeded entries below 2^253 (host, splitmix64), for timing only
void tune_entries(std::vector<fe> &m, uint64_t seed) {
  uint64_t z = seed;
  auto next = [&]() {
    z += 0x9e3779b97f4a7c15ull;
    uint64_t r = z;
    r = (r ^ (r >> 30)) * 0xbf58476d1ce4e5b9ull;
    r = (r ^ (r >> 27)) * 0x94d049bb133111ebull;
    return r ^ (r >> 31);
  };
  for (fe &v : m) {
    for (int q = 0; q < 8; q += 2) {
      uint64_t r = next();
      v.l[q] = (uint32_t)r;
      v.l[q + 1] = (uint32_t)(r >> 32);
    }
    v.l[7] &= (1u << 29) - 1;
  }
}
}  // namespace

VC_API int vc_tune_msm(int device, uint32_t log_lo, uint32_t log_hi, const char *path) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (log_lo < 2 || log_hi > VC_MAX_LOG_N || log_lo > log_hi) return VC_EINVAL;
  CK(hipSetDevice(device));
  const int grid = kl::msm_batch_grid(device);
  std::map<std::pair<uint32_t, uint32_t>, uint32_t> best;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CK(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  static const uint8_t seed[32] = {'t', 'u', 'n', 'e'};
  for (uint32_t L = log_lo; L <= log_hi && e == hipSuccess; L++) {
    vc_params *pp = nullptr;
    if (int rc = vc_setup(L, seed, device, &pp)) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    std::vector<fe> hm(pp->N);
    tune_entries(hm, 0x5eed0000ull + L);
    const uint64_t maxparts = pp->K * pp->M;  // partial sums at the shortest slice (S = 1)
    Carve t;
    size_t o_m = t.take<fe>(pp->N), o_part = t.take<g1_jac>(std::min<uint64_t>(maxparts, pp->K * (pp->M + 31) / 32 + pp->K)),
           o_J = t.take<CJob>(1);
    void *d = nullptr;
    e = hipMalloc(&d, t.off);
    if (e == hipSuccess) e = hipMemcpy(at<fe>(d, o_m), hm.data(), pp->N * sizeof(fe), hipMemcpyHostToDevice);
    for (uint32_t bits : {32u, 256u}) {
      const uint32_t nwin = bits == 32 ? 4 : NWIN;
      float best_ms = 0;
      uint32_t best_S = 0;
      // candidates: blocks of 1024 .. 8192 digits (a 32-bit entry has 4, a full one 32), at
      // most a whole subvector (S >= 32 or S = M: within the partial-sum buffer)
      std::vector<uint32_t> cand;
      for (uint32_t digits = 1024; digits <= MSM_DIGITS; digits *= 2) {
        const uint32_t S = (uint32_t)std::min<uint64_t>(digits / nwin, pp->M);
        if (cand.empty() || cand.back() != S) cand.push_back(S);
      }
      for (uint32_t S : cand) {
        if (e != hipSuccess) break;
        const uint64_t nslice = (pp->M + S - 1) / S;
        CJob j = {at<fe>(d, o_m), pp->table, pp->h, at<g1_jac>(d, o_part), nullptr, nullptr, pp->M, pp->K, nslice, 0, 0,
                  nwin, S};
        e = hipMemcpy(at<CJob>(d, o_J), &j, sizeof j, hipMemcpyHostToDevice);
        const uint64_t blocks = pp->K * nslice;
        const unsigned g = (unsigned)std::min<uint64_t>(blocks, grid);
        float ms_best = 0;
        for (int rep = 0; rep < 4 && e == hipSuccess; rep++) {
          e = hipEventRecord(e0, nullptr);
          if (e == hipSuccess) {
            kl::msm_batch(at<CJob>(d, o_J), 1, blocks, g, nullptr);
            e = hipGetLastError();
          }
          if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0 && (ms_best == 0 || ms < ms_best)) ms_best = ms;  // rep 0 warms up
        }
        if (e == hipSuccess && (best_S == 0 || ms_best < best_ms)) {
          best_ms = ms_best;
          best_S = S;
        }
      }
      if (best_S) best[{L, bits}] = best_S;
    }
    if (d) (void)hipFree(d);
    vc_params_free(pp);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "vc_tune_msm");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &kv : best) g_tune[kv.first] = kv.second;
  }
  if (path) {
    FILE *f = fopen(path, "w");
    if (!f) return VC_EINVAL;
    fprintf(f, "# commit MSM slice lengths: log_n entry_bits entries_per_block\n");
    for (auto &kv : best) fprintf(f, "%u %u %u\n", kv.first.first, kv.first.second, kv.second);
    if (fclose(f) != 0) return VC_EINVAL;
  }
  return VC_OK;
}

VC_API int vc_tune_load(const char *path) {
  std::map<std::pair<uint32_t, uint32_t>, uint32_t> tab;
  if (path) {
    FILE *f = fopen(path, "r");
    if (!f) return VC_EINVAL;
    char line[256];
    int bad = 0;
    while (fgets(line, sizeof line, f)) {
      if (line[0] == '#' || line[0] == '\n') continue;
      unsigned L = 0, bits = 0, S = 0;
      if (sscanf(line, "%u %u %u", &L, &bits, &S) != 3 || L < 2 || L > VC_MAX_LOG_N || (bits != 32 && bits != 256) ||
          S < 1 || S * (bits == 32 ? 4u : NWIN) > MSM_DIGITS) {
        bad = 1;
        break;
      }
      tab[{L, bits}] = S;
    }
    fclose(f);
    if (bad) return VC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = tab;  // NULL: back to the default schedule
  return VC_OK;
}

// ------------------------------------------------------------------ commit without allocation
// vc_commit_noalloc keeps all of its scratch (entries, MSM partial sums, Miller values, tree
// counters, C_j before encoding, C) in one file-scope device array: every GPU the library runs
// on holds its own copy until the process ends.  On the host the array's name only stands for
// the symbol; kernels and copies get the device address that hipGetSymbolAddress returned for
// the current device, looked up once per device.
static constexpr uint64_t NOALLOC_MAX_N = 1ull << 20;
static constexpr size_t NOALLOC_SCRATCH_BYTES = 34ull << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, void *> g_scratch_addr;  // device -> address of its copy of `scratch`

// `device` must be current
int scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return VC_OK;
  }
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "scratch address");
  if (!ptr) return hip_fail(hipErrorInvalidSymbol, "scratch address");
  g_scratch_addr[device] = ptr;
  *out = ptr;
  return VC_OK;
}
}  // namespace

VC_API int vc_commit_noalloc(const vc_params *pp, const void *m_dev, uint64_t n, uint32_t entry_bits, void *stream,
                             void *Cj_out, uint8_t C_out[384]) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp || !m_dev || !Cj_out || n != pp->N || (entry_bits != 32 && entry_bits != 256)) return VC_EINVAL;
  if (n > NOALLOC_MAX_N) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  void *base = nullptr;
  if (int rc = scratch_address(pp->device, &base)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t N = pp->N, K = pp->K, M = pp->M;
  // the same MSM shape as vc_commit
  const uint32_t nwin = entry_bits == 32 ? 4 : NWIN;
  uint32_t S = (uint32_t)(8192 / nwin);
  if (S > M) S = (uint32_t)M;
  const uint64_t nslice = (M + S - 1) / S;
  Carve t;
  size_t o_err = t.take<int>(1), o_m = t.take<fe>(N), o_part = t.take<g1_jac>(K * nslice), o_F = t.take<fp12>(K);
  size_t o_cnt = t.take<uint32_t>(tree_counters(K)), o_Cj = t.take<g1_aff>(K), o_C = t.take<fp12>(1);
  size_t o_enc = t.take<uint8_t>(384);
  if (t.off > NOALLOC_SCRATCH_BYTES) return VC_EINVAL;
  int *err = at<int>(base, o_err);
  fe *m = at<fe>(base, o_m);
  g1_jac *part = at<g1_jac>(base, o_part);
  fp12 *F = at<fp12>(base, o_F), *C = at<fp12>(base, o_C);
  uint32_t *cnt = at<uint32_t>(base, o_cnt);
  g1_aff *Cj = at<g1_aff>(base, o_Cj);
  uint8_t *enc = at<uint8_t>(base, o_enc);
  // the array keeps the last call's contents: clear the flag and the counters (a call that
  // failed part way may have left counters set)
  kl::zero_u32(reinterpret_cast<uint32_t *>(err), 1, st);
  kl::zero_u32(cnt, tree_counters(K), st);
  if (entry_bits == 32) {
    kl::lift_u32((const uint32_t *)m_dev, N, m, st);
  } else {
    CK(hipMemcpyAsync(m, m_dev, N * sizeof(fe), hipMemcpyDeviceToDevice, st));
    kl::check_fr(m, N, err, st);
  }
  kl::msm_slices(m, K, M, nwin, S, pp->table, part, st);
  klw::sum_g1(part, K, nslice, Cj, st);
  ks::miller(Cj, 1, pp->h, 2, K, F, st);
  ks::f12_reduce(F, 1, K, K, cnt, st);
  ks::final_exp(F, 1, 1, C, nullptr, 1, st);
  kl::encode(reinterpret_cast<const fe *>(Cj), 2 * K, 0, static_cast<uint8_t *>(Cj_out), st);
  kl::encode(reinterpret_cast<const fe *>(C), 12, 0, enc, st);
  int herr = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && C_out) e = hipMemcpyAsync(C_out, enc, 384, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "vc_commit_noalloc");
  if (herr & VC_ERRBIT_RANGE) return VC_EINVAL;
  return VC_OK;
}

// ------------------------------------------------------------------ open-all
// With `footprint` set: only the device bytes the call would hold (proof bundle, workspace,
// counters) are stored there; nothing is allocated or launched, and cm, ex, out may be NULL.
// With step2 false only Step 1 runs: the FC batch proofs that open every C_j (the sub-array
// form of OpenAll, section 4.3).
// With eval_r (host, log N little-endian 32-byte values r_0 .. r_{L-1}) the one batch b = K
// proves C_F = <C, T(r_L)> and the PST part opens F at r_R in place of Step 2 (section 4.3,
// evaluation proof at a point).
// Open-all of G jobs on the same params with the same b (G = 1: one job).  Their batches run
// as one Step 1 of G nbj batches, job-major (batch x nbj + k is batch k of job x), so every
// launch takes the same step of all the jobs' batches; Step 2 runs job after job on its side
// stream.  With G > 1 the Step 1 outputs are made in the workspace and copied to each job's
// bundle at the end; a zero challenge in any job fails the call for all of them.
static int open_all_group(const vc_params *cpp, const vc_commitment *const *cms, uint32_t G, uint32_t b, vc_exec *ex,
                          hipStream_t st, vc_proofs **outs, uint64_t *footprint = nullptr, bool step2 = true,
                          const uint8_t *eval_r = nullptr, uint64_t *parts = nullptr) {
  if (!cpp || b < 1 || b > cpp->K || G < 1) return VC_EINVAL;
  if (!footprint) {
    if (!cms || !outs || !ex || ex->device != cpp->device) return VC_EINVAL;
    for (uint32_t x = 0; x < G; x++)
      if (!cms[x] || cms[x]->pp != cpp) return VC_EINVAL;
  }
  if ((eval_r || !step2) && G != 1) return VC_EINVAL;  // sub-arrays and evaluation proofs: one job
  if (eval_r && (b != cpp->K || step2)) return VC_EINVAL;  // an evaluation proof is one batch, no Step 2
  const vc_params *pp = cpp;
  if (outs)
    for (uint32_t x = 0; x < G; x++) outs[x] = nullptr;
  if (!footprint) CK(hipSetDevice(pp->device));
  const uint64_t N = pp->N, K = pp->K, M = pp->M;
  const uint32_t lK = pp->lK, lM = pp->lM;
  const uint64_t nbj = (K + b - 1) / b;  // batches per job
  const uint64_t nb = G * nbj;           // batches of the whole Step 1
  const bool grp = G > 1;
  const uint64_t qmax = (b + 31) / 32;
  const uint64_t nq = 2 * K - 2;  // KZG quotient length
  // ---- the proof bundle
  vc_proofs *pr = new vc_proofs();
  pr->pp = pp;
  pr->device = pp->device;
  pr->b = b;
  pr->nb = nbj;
  pr->step2 = step2;
  const uint64_t with2 = step2 ? 1 : 0;  // Step 2 arrays are left out of a sub-array bundle
  const uint64_t ev = eval_r ? 1 : 0;
  Carve c;
  pr->o_Cj = c.take<g1_aff>(K);
  pr->o_C = c.take<fp12>(1);
  pr->o_Lgt = c.take<fp12>(nbj * lK);
  pr->o_Rgt = c.take<fp12>(nbj * lK);
  pr->o_Lg1 = c.take<g1_aff>(nbj * lK);
  pr->o_Rg1 = c.take<g1_aff>(nbj * lK);
  pr->o_X = c.take<fe>(nbj * lK);
  pr->o_Al = c.take<g1_aff>(nbj);
  pr->o_vl = c.take<g2_aff>(nbj);
  pr->o_piv = c.take<g2_aff>(nbj);
  pr->o_tree = c.take<fe>(with2 * 2 * N);
  pr->o_rho = c.take<fe>(with2 * K);
  pr->o_Y = c.take<fe>(with2 * (2 * K - 1) * M);
  pr->o_D = c.take<g1_aff>(with2 * (2 * K - 1));
  pr->o_W = c.take<g1_aff>(with2 * (M - 1));
  pr->o_CF = c.take<g1_aff>(ev);
  pr->o_yv = c.take<fe>(ev);
  pr->o_We = c.take<g1_aff>(ev * lM);
  // ---- scratch
  Carve t;
  size_t o_err = t.take<int>(1), o_A = t.take<g1_aff>(nb * K), o_V = t.take<g2_aff>(nb * K), o_B = t.take<fe>(nb * K);
  size_t o_F = t.take<fp12>(nb * K), o_S = t.take<g1_jac>(nb * K), o_Hq = t.take<uint32_t>(nb * qmax * 8);
  size_t o_sig = t.take<uint32_t>(nb * 8), o_Xi = t.take<fe>(nb * lK), o_Q = t.take<fe>(nb * nq), o_z = t.take<fe>(nb);
  // KZG proof: split terms (4 partial results per term) or, with many terms, canonical
  // quotient coefficients and the per-block partial sums of its MSM
  const bool kzg_split = 4 * nb * nq <= KZG_SPLIT_MAX;
  const uint32_t kzg_s = nb * ((nq + KZG_S_LONG - 1) / KZG_S_LONG) >= KZG_LONG_MIN_BLOCKS ? KZG_S_LONG : KZG_S;
  const uint64_t kzg_nslice = (nq + kzg_s - 1) / kzg_s, kzg_len = kzg_split ? 4 * nq : kzg_nslice;
  size_t o_Qc = t.take<fe>(nb * nq), o_S2 = t.take<g2_jac>(nb * kzg_len), o_HS = t.take<g1_jac>(with2 * G * lM * (M / 2));
  size_t o_J = t.take<S2Job>(with2 * G);  // Step 2's job table
  size_t o_dec = t.take<glv::Dec>(nb);
  size_t o_KQ = t.take<fe>(K > 1024 ? nb * 4 * (2 * K - 1) : 0);  // the KZG quotient's scans beyond shared memory
  // round 1's G_T parts of each job; with several jobs, their aux rows and commitments side
  // by side and the Step 1 outputs of all batches (copied to the bundles at the end)
  size_t o_LT = t.take<fp12>(G), o_RT = t.take<fp12>(G);
  size_t o_CjG = t.take<g1_aff>(grp ? G * K : 0), o_CG = t.take<fp12>(grp ? G : 0);
  size_t o_gLgt = t.take<fp12>(grp ? nb * lK : 0), o_gRgt = t.take<fp12>(grp ? nb * lK : 0);
  size_t o_gLg1 = t.take<g1_aff>(grp ? nb * lK : 0), o_gRg1 = t.take<g1_aff>(grp ? nb * lK : 0);
  size_t o_gX = t.take<fe>(grp ? nb * lK : 0), o_gpiv = t.take<g2_aff>(grp ? nb : 0);
  // evaluation proof: point, T, the terms of C_F, F's table, the PST quotients and their products
  size_t o_rle = t.take<uint8_t>(ev * 32 * pp->L), o_er = t.take<fe>(ev * pp->L), o_T = t.take<fe>(ev * K),
         o_pK = t.take<g1_aff>(ev * K), o_eg = t.take<fe>(ev * M), o_eq = t.take<fe>(ev * M), o_pW = t.take<g1_aff>(ev * M);
  // Step 1 arrays of alternate rounds, and the terms taken one round ahead (oa_terms.hpp)
  const bool ahead = lK >= 2 && nb * K <= (ex ? ex->ahead_max : AHEAD_MAX_PAIRS);
  const uint64_t nterm = ahead ? 2 * nb * K : 0;
  size_t o_A2 = t.take<g1_aff>(nb * K), o_V2 = t.take<g2_aff>(nb * K), o_B2 = t.take<fe>(nb * K);
  size_t o_F2 = t.take<fp12>(2 * nterm), o_PS = t.take<g1_jac>(2 * nterm);
  size_t o_PU = t.take<fp12>(ahead ? 4 * nb : 0), o_PX = t.take<fp12>(ahead ? 8 * nb : 0);
  size_t o_PXm = t.take<fp12>(ahead ? 24 * nb : 0), o_PE = t.take<fp12>(ahead ? 16 * nb : 0);
  size_t o_PU1 = t.take<g1_aff>(ahead ? 4 * nb : 0), o_PX1 = t.take<g1_aff>(ahead ? 8 * nb : 0);
  size_t o_PX1m = t.take<g1_aff>(ahead ? 24 * nb : 0), o_PM = t.take<g1_jac>(ahead ? 16 * nb : 0);
  // split folds: multiples of the halves A[h + i], V[h + i] and the four partial results
  auto split_round = [&](uint32_t j) { return ahead && j <= lK && nb * (K >> j) <= FOLD_SPLIT_MAX; };
  // first round whose L, R come from terms taken ahead (rounds before it run direct)
  uint32_t j0 = 2;
  while (j0 < lK && nb * (K >> j0) > DIRECT_MIN) j0++;
  const uint64_t nsplit = ahead ? std::min<uint64_t>(nb * K / 2, FOLD_SPLIT_MAX) : 0;
  // (multiples of whole arrays, one set per round parity; the G1 terms split likewise use them)
  size_t o_FM1 = t.take<g1_aff>(2 * 6 * nsplit), o_FM2 = t.take<g2_aff>(2 * 6 * nsplit);
  size_t o_FJ1 = t.take<g1_jac>(4 * nsplit), o_FJ2 = t.take<g2_jac>(4 * nsplit), o_GJ = t.take<g1_jac>(16 * nsplit);
  const uint64_t c_dir = 2 * nb * tree_counters(K / 2), c_u = 2 * nb * tree_counters(K / 2),
                 c_xy = 4 * nb * tree_counters(K / 4);
  const uint64_t c_kzg = nb * tree_counters(kzg_len);
  const uint64_t n_cnt = 2 * c_dir + 4 * (c_u + c_xy) + 6 * nsplit + c_kzg;
  if (footprint) {
    *footprint = G * c.off + t.off + n_cnt * sizeof(uint32_t);
    if (parts) {
      parts[0] = G * c.off;  // the proof bundles
      parts[1] = t.off;  // the executor's workspace
      parts[2] = n_cnt;  // arrival counters
    }
    delete pr;
    return VC_OK;
  }
  // one bundle per job (same layout); on every error return below they are released
  // (hipFree waits for the work in flight) and the executor's counters are cleared before
  // their next use (trees may have stopped half way)
  struct Release {
    std::vector<vc_proofs *> p;
    vc_exec *ex;
    bool keep = false;
    ~Release() {
      if (keep) return;
      for (vc_proofs *q : p) vc_proofs_free(q);
      if (!p.empty()) ex->cnt_dirty = true;
    }
  } release{{}, ex};
  for (uint32_t x = 0; x < G; x++) {
    vc_proofs *q = x == 0 ? pr : new vc_proofs(*pr);
    q->mem = nullptr;
    release.p.push_back(q);
    hipError_t e = hipMalloc(&q->mem, c.off);
    if (e != hipSuccess) return hip_fail(e, "vc_open_all alloc");
  }
  auto bundle = [&](uint32_t x) { return release.p[x]->mem; };
  void *bm = bundle(0);
  g1_aff *Cj = at<g1_aff>(bm, pr->o_Cj);
  fp12 *C = at<fp12>(bm, pr->o_C);
  int rc = ensure_ws(ex, t.off);
  if (rc) return rc;
  void *ws = ex->ws;
  // Step 1 outputs: the bundle's arrays for one job, else the workspace's
  fp12 *Lgt = grp ? at<fp12>(ws, o_gLgt) : at<fp12>(bm, pr->o_Lgt);
  fp12 *Rgt = grp ? at<fp12>(ws, o_gRgt) : at<fp12>(bm, pr->o_Rgt);
  g1_aff *Lg1 = grp ? at<g1_aff>(ws, o_gLg1) : at<g1_aff>(bm, pr->o_Lg1);
  g1_aff *Rg1 = grp ? at<g1_aff>(ws, o_gRg1) : at<g1_aff>(bm, pr->o_Rg1);
  fe *X = grp ? at<fe>(ws, o_gX) : at<fe>(bm, pr->o_X);
  g2_aff *piv = grp ? at<g2_aff>(ws, o_gpiv) : at<g2_aff>(bm, pr->o_piv);
  g1_aff *CjG = grp ? at<g1_aff>(ws, o_CjG) : Cj;  // every job's aux row
  fp12 *CG = grp ? at<fp12>(ws, o_CG) : C;         // every job's commitment
  fp12 *LT = at<fp12>(ws, o_LT), *RT = at<fp12>(ws, o_RT);
  int *err = at<int>(ws, o_err);
  g1_aff *A = at<g1_aff>(ws, o_A);
  g2_aff *V = at<g2_aff>(ws, o_V);
  fe *B = at<fe>(ws, o_B);
  fp12 *F = at<fp12>(ws, o_F);
  g1_jac *S = at<g1_jac>(ws, o_S);
  uint32_t *Hq = at<uint32_t>(ws, o_Hq), *sigma = at<uint32_t>(ws, o_sig);
  fe *Xinv = at<fe>(ws, o_Xi), *Q = at<fe>(ws, o_Q), *z = at<fe>(ws, o_z);
  g2_jac *S2 = at<g2_jac>(ws, o_S2);
  fe *Qc = at<fe>(ws, o_Qc);
  g1_jac *HS = at<g1_jac>(ws, o_HS);
  glv::Dec *gdec = at<glv::Dec>(ws, o_dec);
  g1_aff *Ab[2] = {A, at<g1_aff>(ws, o_A2)};
  g2_aff *Vb[2] = {V, at<g2_aff>(ws, o_V2)};
  fe *Bb[2] = {B, at<fe>(ws, o_B2)};
  fp12 *F2[2] = {at<fp12>(ws, o_F2), at<fp12>(ws, o_F2) + nterm};
  g1_jac *PS[2] = {at<g1_jac>(ws, o_PS), at<g1_jac>(ws, o_PS) + nterm};
  fp12 *PU[2] = {at<fp12>(ws, o_PU), at<fp12>(ws, o_PU) + 2 * nb};
  fp12 *PX[2] = {at<fp12>(ws, o_PX), at<fp12>(ws, o_PX) + 4 * nb};
  fp12 *PXm[2] = {at<fp12>(ws, o_PXm), at<fp12>(ws, o_PXm) + 12 * nb};
  g1_aff *PX1m[2] = {at<g1_aff>(ws, o_PX1m), at<g1_aff>(ws, o_PX1m) + 12 * nb};
  fp12 *PE = at<fp12>(ws, o_PE);
  g1_aff *PU1[2] = {at<g1_aff>(ws, o_PU1), at<g1_aff>(ws, o_PU1) + 2 * nb};
  g1_aff *PX1[2] = {at<g1_aff>(ws, o_PX1), at<g1_aff>(ws, o_PX1) + 4 * nb};
  g1_jac *PM = at<g1_jac>(ws, o_PM);
  g1_aff *FM1[2] = {at<g1_aff>(ws, o_FM1), at<g1_aff>(ws, o_FM1) + 6 * nsplit};
  g2_aff *FM2[2] = {at<g2_aff>(ws, o_FM2), at<g2_aff>(ws, o_FM2) + 6 * nsplit};
  g1_jac *FJ1 = at<g1_jac>(ws, o_FJ1), *GJ = at<g1_jac>(ws, o_GJ);
  g2_jac *FJ2 = at<g2_jac>(ws, o_FJ2);
  // reduction-tree counters: round-1 (or every direct round) products, and per stream the
  // U and XY groups of the terms taken ahead (F_p12 on side stream 3, G1 on the caller's)
  if (int rc2 = ensure_cnt(ex, n_cnt, st)) return rc2;
  // (the counters of the terms' trees per round parity, whose streams run concurrently)
  uint32_t *cnt_dir = ex->cnt, *cnt_t = cnt_dir + c_dir;
  uint32_t *cnt_fu[2] = {cnt_t, cnt_t + 2 * (c_u + c_xy)}, *cnt_fxy[2] = {cnt_fu[0] + c_u, cnt_fu[1] + c_u};
  uint32_t *cnt_gu[2] = {cnt_fxy[0] + c_xy, cnt_fxy[1] + c_xy}, *cnt_gxy[2] = {cnt_gu[0] + c_u, cnt_gu[1] + c_u};
  uint32_t *cnt_fold = cnt_t + 4 * (c_u + c_xy), *cnt_kzg = cnt_fold + 2 * nsplit, *cnt_g1dir = cnt_kzg + c_kzg,
           *cnt_g1s = cnt_g1dir + c_dir;

  kl::zero_u32(reinterpret_cast<uint32_t *>(err), 1, st);
  for (uint32_t x = 0; x < G; x++) {
    void *bx = bundle(x);
    CK(hipMemcpyAsync(at<g1_aff>(bx, pr->o_Cj), cms[x]->Cj, K * sizeof(g1_aff), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(at<fp12>(bx, pr->o_C), cms[x]->C, sizeof(fp12), hipMemcpyDeviceToDevice, st));
    if (grp) {
      CK(hipMemcpyAsync(CjG + x * K, cms[x]->Cj, K * sizeof(g1_aff), hipMemcpyDeviceToDevice, st));
      CK(hipMemcpyAsync(CG + x, cms[x]->C, sizeof(fp12), hipMemcpyDeviceToDevice, st));
    }
    if (step2) kl::zero_u32(at<uint32_t>(bx, pr->o_tree), 8, st);  // heap node 0 is unused
  }
  // Step 2's job table: each launch takes all G jobs, their inputs and bundle arrays through it
  std::vector<S2Job> jobs(step2 ? G : 0);
  for (uint32_t x = 0; x < jobs.size(); x++) {
    void *bx = bundle(x);
    jobs[x] = {cms[x]->m, at<g1_aff>(bx, pr->o_Cj), at<fp12>(bx, pr->o_C), at<uint32_t>(bx, pr->o_tree),
               at<fe>(bx, pr->o_rho), at<fe>(bx, pr->o_Y), at<g1_aff>(bx, pr->o_D), at<g1_aff>(bx, pr->o_W)};
  }
  S2Job *J = at<S2Job>(ws, o_J);
  if (step2) CK(hipMemcpyAsync(J, jobs.data(), G * sizeof(S2Job), hipMemcpyHostToDevice, st));

  // ---- Step 2 runs on side stream 1, concurrently with Step 1: Merkle tree (Fiat-Shamir),
  // randomized folding tree, HyperEval on g* (Protocol 1 Step 2 and its Sub-protocol).  Its
  // launches are issued after those of the first Step 1 round, which is on the critical path.
  hipStream_t s1 = ex->side[0], s2 = ex->side[1];
  if (int rc2 = ev_mark(ex, 0, st)) return rc2;
  auto launch_step2 = [&]() -> int {
    if (int rc2 = ev_wait(ex, 0, s1)) return rc2;
    hipStream_t st = s1;  // launches below go to side stream 1
    kl::merkle_leaves(J, G, M, N, st);
    for (uint64_t s = N / 2; s >= 1; s /= 2) kl::merkle_level(J, G, s, st);
    kl::rho(J, G, K, st);
    kl::ytree(J, G, M, K, lK, st);
    klw::d_leaves(J, G, K, st);
    for (uint32_t h = 1; h <= lK; h++) klw::dlevel(J, G, K, h, st);
    klw::hyper_terms(J, G, K, pp->ek, M, lM, HS, st);
    for (uint32_t d = 0; d < lM; d++) {
      // level d of every job: G 2^d segments of M / 2^{d+1} terms, contiguous
      uint64_t half = M >> (d + 1);
      g1_jac *base = HS + (uint64_t)d * G * (M / 2);
      klw::g1_reduce(base, (uint64_t)G << d, half, half, st);
      klw::w_aff(J, G, base, half, d, st);
    }
    return VC_OK;
  };

  // ---- Step 1: FC.BOpen for every block, all blocks in lockstep (Protocol 1, Eq. genFCBatchProof).
  // Round j works on the arrays A, V, b of buffer (j - 1) & 1; its fold writes buffer j & 1.
  // Round 1 (and every round when the batches alone fill the device) computes L_j, R_j
  // directly: Miller loops, product tree and final exponentiation on the caller's stream,
  // the G1 parts on side stream 2, the folds on side streams 2 (G1) and 3 (G2).
  // Otherwise (ahead) the terms of round j + 1 are computed from the arrays of round j - 1
  // while x_{j-1} and x_j are derived (oa_terms.hpp), and round j + 1 only raises them to
  // x_j, x_j^{-1} and multiplies: the Miller loops and final exponentiations leave the
  // chain of dependent rounds.  Then side stream 2 runs the fused folds and side stream 3
  // the terms; each launch pairs the G1 and the pairing-side work of its step.
  // Streams of the ahead mode: side 2 the folds and the multiples, sides 3 and 4 the
  // pairing side of the terms of even and odd rounds (Miller loops, products, final
  // exponentiations), side 5 their G1 side; the caller's stream combines and hashes.
  hipStream_t sg = s2, sf = ex->side[2], sfp[2] = {ex->side[2], ex->side[3]}, sq = ex->side[4];
  kl::oa_init(CjG, pp->h, K, nb, nbj, A, V, B, st);
  // Round 1's Miller loops pair A = aux with v, which do not depend on the batching vectors b:
  // they start on side stream 1 as soon as the arrays are set, beside the hashing of r (event 22
  // marks them done)
  uint64_t nprod1 = K / 2;
  {
    if (int rc2 = stream_wait(ex, 21, st, s1)) return rc2;
    const uint64_t h1 = K / 2;
    if (G * h1 >= WIDE_FOLD_MIN) nprod1 = klw::oa_miller(CjG, Vb[0], K, G, h1, F, s1);
    else ks::oa_miller(CjG, Vb[0], K, G, h1, F, s1);
    if (int rc2 = ev_mark(ex, 22, s1)) return rc2;
  }
  // the pairing side of the terms (side streams 3 and 4) reads only the arrays: it is ordered
  // after their set-up, not after the hashing of r
  if (int rc2 = stream_wait(ex, 2, st, sf)) return rc2;
  if (ahead)
    if (int rc2 = stream_wait(ex, 17, st, sfp[1])) return rc2;
  // multiples 2^{32 m} A[i] (m = 1..3) of the whole arrays A of round j (for its split fold
  // and the split G1 terms of round j + 1) and 2^{16 m} V[h + i] of the halves V[h..) (for
  // its split fold), into set j & 1 (round 1 on side stream 1, later rounds on the fold
  // stream)
  auto launch_fold_mults = [&](uint32_t j, hipStream_t s) {
    const uint64_t n = K >> (j - 1), hh = n / 2;
    const int cur = (j - 1) & 1;
    ks::fold_mults(Ab[cur], n, nb * n, Vb[cur] + hh, hh, nb * hh, K, FM1[j & 1], FM2[j & 1], s);
  };
  // the multiples of the round-1 arrays (for the split fold of round 1 and the split G1 terms of
  // round 2, whose chain they start) on side stream 5 beside the round-1 Miller loops, as soon as
  // the arrays are set (event 15 marks them done)
  if (split_round(1)) {
    if (int rc2 = ev_wait(ex, 21, sq)) return rc2;
    launch_fold_mults(1, sq);
    if (int rc2 = ev_mark(ex, 15, sq)) return rc2;
  }
  fe *er = at<fe>(ws, o_er), *eT = at<fe>(ws, o_T), *eg = at<fe>(ws, o_eg), *eq = at<fe>(ws, o_eq);
  if (eval_r) {
    // the point, T(r_L), C_F = sum_j T_j C_j, then b = r_0 T for the one batch
    CK(hipMemcpyAsync(at<void>(ws, o_rle), eval_r, 32ull * pp->L, hipMemcpyHostToDevice, st));
    kl::ev_point(at<uint8_t>(ws, o_rle), pp->L, er, err, st);
    kl::ev_eq(er, lM, lK, K, eT, st);
    klw::g1_mul(Cj, 0, eT, K, at<g1_aff>(ws, o_pK), st);
    kl::ev_sum(at<g1_aff>(ws, o_pK), K, at<g1_aff>(bm, pr->o_CF), st);
    kl::ev_r0(C, er, pp->L, at<g1_aff>(bm, pr->o_CF), eT, K, B, st);
  } else {
    kl::fc_chunks(CjG, K, b, nb, nbj, Hq, st);
    kl::fc_sigma(CG, K, b, nb, nbj, Hq, sigma, st);
    kl::fc_r(K, b, nb, nbj, sigma, B, st);
  }
  // the PST part of an evaluation proof on side stream 1, beside the FC rounds: F's table,
  // then l_M steps eliminating x_{lM-1} first, the quotients' products with ek_0 .. ek_{lM-1}
  // (contiguous at the start of ek, in the same order) and their sums
  auto launch_pst = [&]() -> int {
    if (int rc2 = stream_wait(ex, 20, st, s1)) return rc2;
    kl::ev_table(cms[0]->m, eT, K, M, eg, s1);
    for (uint32_t d = 0; d < lM; d++) {
      uint32_t k = lM - d;
      uint64_t half = 1ull << (k - 1);
      kl::ev_pst_step(eg, half, er + (k - 1), eq + (half - 1), s1);
    }
    klw::g1_mul(pp->ek, 0, eq, M - 1, at<g1_aff>(ws, o_pW), s1);
    kl::ev_finish(at<g1_aff>(ws, o_pW), lM, eg, at<g1_aff>(bm, pr->o_We), at<fe>(bm, pr->o_yv), s1);
    return VC_OK;
  };
  if (int rc2 = stream_wait(ex, 1, st, sg)) return rc2;
  if (ahead)
    if (int rc2 = stream_wait(ex, 18, st, sq)) return rc2;
  // terms of round jn >= 2 from the arrays of round jn - 1 (one buffer set per round parity):
  // the pairing side (Miller loops, group products, final exponentiations, squaring
  // multiples) on side stream 3 + (jn & 1), ready at event 6 + (jn & 1) ...
  auto launch_terms = [&](uint32_t jn) -> int {
    uint64_t q = K >> jn;
    int par = jn & 1, src = (jn - 2) & 1;
    hipStream_t s = sfp[par];
    ks::oa_pterms(Ab[src], Vb[src], K, nb, q, F2[par], s);
    ks::f12_reduce(F2[par], 2 * nb, 2 * q, 2 * q, cnt_fu[par], s);
    ks::f12_reduce(F2[par] + nb * 4 * q, 4 * nb, q, q, cnt_fxy[par], s);
    ks::final_exp2(F2[par], 2 * q, 2 * nb, PU[par], F2[par] + nb * 4 * q, q, 4 * nb, PX[par], s);
    ks::gt_sqr_mults(PX[par], 4 * nb, PXm[par], s);
    return ev_mark(ex, 6 + par, s);
  };
  // ... and the G1 side (terms, split in four parts when the arrays of round jn - 1 have
  // multiples, group sums, affine forms and multiples) on side stream 5, ready at event
  // 8 + (jn & 1)
  auto launch_g1terms = [&](uint32_t jn) -> int {
    uint64_t q = K >> jn;
    int par = jn & 1, src = (jn - 2) & 1;
    if (split_round(jn - 1))
      ks::oa_g1terms_split(Ab[src], Bb[src], FM1[(jn - 1) & 1], K, nb, q, GJ, cnt_g1s, PS[par], sq);
    else
      ks::oa_g1terms_next(Ab[src], Bb[src], K, nb, q, PS[par], sq);
    ks::g1_tree(PS[par], 2 * nb, 2 * q, 2 * q, cnt_gu[par], sq);
    ks::g1_tree(PS[par] + nb * 4 * q, 4 * nb, q, q, cnt_gxy[par], sq);
    ks::g1_finish(PS[par], nb, q, PU1[par], PX1[par], PX1m[par], sq);
    return ev_mark(ex, 8 + par, sq);
  };
  for (uint32_t j = 1; j <= lK; j++) {
    const uint64_t h = K >> j;
    const int cur = (j - 1) & 1, nxt = j & 1;
    if (!ahead || j < j0) {
      if (ahead) {
        ks::oa_g1terms(Ab[cur], Bb[cur], K, nb, h, S, sg);
        ks::g1_tree(S, 2 * nb, K / 2, h, cnt_g1dir, sg);
      } else {
        klw::oa_g1terms(Ab[cur], Bb[cur], K, nb, h, S, sg);
        klw::g1_reduce(S, 2 * nb, K / 2, h, sg);
      }
      kl::oa_lr_aff(S, K, nb, j, lK, Lg1, Rg1, sg);
      if (int rc2 = ev_mark(ex, 3, sg)) return rc2;
      // round 1 pairs the same A = aux with the same v in every batch of a job: its G_T
      // parts are computed once per job (from the aux rows; the first G rows of V all hold v)
      // and copied to the job's batches
      const uint64_t nbm = j == 1 ? G : nb;
      const g1_aff *Am = j == 1 ? CjG : Ab[cur];
      uint64_t nprod = h;  // Miller products per batch and side, reduced by the tree below
      if (j == 1) nprod = nprod1;  // round 1's Miller loops run on side stream 1 (above)
      else if (nbm * h >= WIDE_FOLD_MIN) nprod = klw::oa_miller(Am, Vb[cur], K, nbm, h, F, st);
      else ks::oa_miller(Am, Vb[cur], K, nbm, h, F, st);
      // the terms of round j0 from the arrays of the last direct round, after its Miller
      // loops (the G1 side after the multiples of the arrays); from the arrays of round 1 as
      // soon as they are set (their stream waits for nothing else), beside the round-1 Miller
      // loops
      if (ahead && j + 1 == j0) {
        if (j > 1)
          if (int rc2 = stream_wait(ex, 19, st, sfp[j0 & 1])) return rc2;
        if (int rc2 = launch_terms(j0)) return rc2;
        if (j == 1) {
          if (split_round(1))
            if (int rc2 = ev_wait(ex, 15, sq)) return rc2;
        } else if (int rc2 = stream_wait(ex, 16, sg, sq)) {  // the fold into these arrays, their multiples
          return rc2;
        }
        if (int rc2 = launch_g1terms(j0)) return rc2;
      }
      if (j == 1)
        if (int rc2 = ev_wait(ex, 22, st)) return rc2;
      ks::f12_reduce(F, 2 * nbm, K / 2, nprod, cnt_dir, st);
      if (j == 1) {
        ks::final_exp(F, K / 2, 2 * nbm, LT, RT, 1, st);
        kl::bcast_round1(LT, RT, nb, nbj, lK, Lgt, Rgt, st);
      } else {
        ks::final_exp(F, K / 2, 2 * nbm, Lgt + (j - 1), Rgt + (j - 1), lK, st);
      }
      if (int rc2 = ev_wait(ex, 3, st)) return rc2;
    } else {
      // L_j, R_j from the terms taken from the arrays of round j - 1 and x_{j-1}
      const int par = j & 1;
      if (int rc2 = ev_wait(ex, 6 + par, st)) return rc2;
      if (int rc2 = ev_wait(ex, 8 + par, st)) return rc2;
      ks::oa_combine_split(PX[par], PXm[par], PX1[par], PX1m[par], X + (j - 2), Xinv + (j - 2), lK, nb, PE, PM, st);
      ks::oa_combine8(PU[par], PE, PU1[par], PM, nb, Lgt + (j - 1), Rgt + (j - 1), Lg1 + (j - 1), Rg1 + (j - 1), lK, st);
    }
    kl::oa_transcript(Lgt, Rgt, nb, j, lK, Lg1, Rg1, X, Xinv, err, g_zero_round.load(), st);
    // fold with x_j into the other buffer
    if (ahead) {
      if (int rc2 = stream_wait(ex, 4, st, sg)) return rc2;
      if (j == 1 && split_round(1))
        if (int rc2 = ev_wait(ex, 15, sg)) return rc2;
      if (split_round(j))
        ks::oa_fold_split(Ab[cur], Bb[cur], Ab[nxt], Bb[nxt], Vb[cur], Vb[nxt], X, Xinv, FM1[j & 1], FM2[j & 1], FJ1, FJ2,
                          cnt_fold, K, nb, h, j, lK, sg);
      else
        ks::oa_fold(Ab[cur], Bb[cur], Ab[nxt], Bb[nxt], Vb[cur], Vb[nxt], X, Xinv, K, nb, h, j, lK, sg);
      // a direct next round reads the folded arrays on the caller's stream
      if (j + 1 < j0)
        if (int rc2 = stream_wait(ex, 11, sg, st)) return rc2;
      // terms of round j + 2 from the arrays of round j + 1 (just folded)
      if (j + 2 <= lK && j + 2 > j0) {
        if (int rc2 = stream_wait(ex, 10, sg, sfp[j & 1])) return rc2;
        if (int rc2 = launch_terms(j + 2)) return rc2;
      }
      if (split_round(j + 1)) launch_fold_mults(j + 1, sg);
      if (j + 2 <= lK && j + 2 > j0) {
        if (int rc2 = stream_wait(ex, 16, sg, sq)) return rc2;
        if (int rc2 = launch_g1terms(j + 2)) return rc2;
      }
    } else {
      if (int rc2 = stream_wait(ex, 4, st, sg)) return rc2;
      kl::glv_dec(X, nb, j, lK, gdec, sg);
      klw::oa_fold_g1(Ab[cur], Bb[cur], Ab[nxt], Bb[nxt], Xinv, gdec, K, nb, h, j, lK, sg);
      if (int rc2 = stream_wait(ex, 5, st, sf)) return rc2;
      if (nb * h >= WIDE_FOLD_MIN) klw::oa_fold_g2(Vb[cur], Vb[nxt], Xinv, K, nb, h, j, lK, sf);
      else ks::oa_fold_g2(Vb[cur], Vb[nxt], Xinv, K, nb, h, j, lK, sf);
      if (int rc2 = stream_wait(ex, 11, sg, st)) return rc2;
      if (int rc2 = stream_wait(ex, 12, sf, st)) return rc2;
    }
    if (j == std::min<uint32_t>(2, lK))
      if (int rc2 = step2 ? launch_step2() : eval_r ? launch_pst() : VC_OK) return rc2;
  }
  if (ahead)
    if (int rc2 = stream_wait(ex, 11, sg, st)) return rc2;
  A = Ab[lK & 1];
  V = Vb[lK & 1];
  for (uint32_t x = 0; x < G; x++) {
    void *bx = bundle(x);
    CK(hipMemcpy2DAsync(at<g1_aff>(bx, pr->o_Al), sizeof(g1_aff), A + x * nbj * K, K * sizeof(g1_aff), sizeof(g1_aff),
                        nbj, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpy2DAsync(at<g2_aff>(bx, pr->o_vl), sizeof(g2_aff), V + x * nbj * K, K * sizeof(g2_aff), sizeof(g2_aff),
                        nbj, hipMemcpyDeviceToDevice, st));
  }
  // faster verifier: KZG-style proof in G2 that v_l = f_v(beta) g2
  kl::kzg_quotient(Xinv, X, V, K, nb, lK, Q, z, at<fe>(ws, o_KQ), st);
  if (kzg_split) {
    ks::kzg_terms_split(pp->h, pp->hm, Q, K, nb, S2, st);
  } else {
    kl::fr_canon(Q, nb * nq, Qc, st);
    kl::msm_slices_g2(Qc, nb, nq, NWIN, kzg_s, pp->htab, S2, st);
  }
  ks::g2_tree(S2, nb, kzg_len, kzg_len, cnt_kzg, st);
  kl::g2_to_aff(S2, kzg_len, nb, piv, 1, st);
  // each job's rows of the Step 1 outputs into its bundle
  for (uint32_t x = 0; grp && x < G; x++) {
    void *bx = bundle(x);
    const uint64_t r0 = x * nbj * lK, nr = nbj * lK;
    CK(hipMemcpyAsync(at<fp12>(bx, pr->o_Lgt), Lgt + r0, nr * sizeof(fp12), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(at<fp12>(bx, pr->o_Rgt), Rgt + r0, nr * sizeof(fp12), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(at<g1_aff>(bx, pr->o_Lg1), Lg1 + r0, nr * sizeof(g1_aff), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(at<g1_aff>(bx, pr->o_Rg1), Rg1 + r0, nr * sizeof(g1_aff), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(at<fe>(bx, pr->o_X), X + r0, nr * sizeof(fe), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(at<g2_aff>(bx, pr->o_piv), piv + x * nbj, nbj * sizeof(g2_aff), hipMemcpyDeviceToDevice, st));
  }
  // join Step 2
  if (int rc2 = stream_wait(ex, 13, s1, st)) return rc2;
  CKL("vc_open_all launch");
  int herr = 0;
  CK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (herr & VC_ERRBIT_CHALLENGE) return VC_ECHALLENGE;
  if (eval_r && (herr & VC_ERRBIT_RANGE)) return VC_EINVAL;
  release.keep = true;
  for (uint32_t x = 0; x < G; x++) outs[x] = release.p[x];
  return VC_OK;
}

static int open_all_impl(const vc_params *cpp, const vc_commitment *cm, uint32_t b, vc_exec *ex, hipStream_t st,
                         vc_proofs **out, uint64_t *footprint = nullptr, bool step2 = true,
                         const uint8_t *eval_r = nullptr, uint64_t *parts = nullptr) {
  if (!footprint && !cm) return VC_EINVAL;
  return open_all_group(cpp, cm ? &cm : nullptr, 1, b, ex, st, out, footprint, step2, eval_r, parts);
}

VC_API int vc_open_all(const vc_params *pp, const vc_commitment *cm, uint32_t b, void *stream, vc_proofs **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp) return VC_EINVAL;
  return open_all_impl(pp, cm, b, pp->ex, (hipStream_t)stream, out);
}

VC_API int vc_open_subarrays(const vc_params *pp, const vc_commitment *cm, uint32_t b, void *stream, vc_proofs **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp) return VC_EINVAL;
  return open_all_impl(pp, cm, b, pp->ex, (hipStream_t)stream, out, nullptr, false);
}

VC_API int vc_open_all_ex(const vc_params *pp, const vc_commitment *cm, uint32_t b, vc_exec *ex, void *stream,
                          vc_proofs **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  return open_all_impl(pp, cm, b, ex, (hipStream_t)stream, out);
}

// Several open-all jobs.  Jobs on the same params with the same b form groups of at most
// max_group jobs, each group one fused open-all (open_all_group); host thread t takes the next
// group (largest first) and runs it on executor t (its own streams and workspace) and that
// executor's stream, at most nexec groups at a time.
VC_API int vc_open_all_grouped(uint32_t n, const vc_params *const *pps, const vc_commitment *const *cms,
                               const uint32_t *bs, uint32_t max_group, uint32_t nexec, vc_exec *const *exs,
                               vc_proofs **outs) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pps || !cms || !bs || !exs || !outs || nexec < 1 || max_group < 1) return VC_EINVAL;
  for (uint32_t i = 0; i < n; i++) outs[i] = nullptr;
  // every executor on one device and none twice (each one is driven by its own host thread)
  for (uint32_t t = 0; t < nexec; t++) {
    if (!exs[t] || exs[t]->device != exs[0]->device) return VC_EINVAL;
    for (uint32_t u = 0; u < t; u++)
      if (exs[u] == exs[t]) return VC_EINVAL;
  }
  for (uint32_t i = 0; i < n; i++)
    if (!pps[i] || !cms[i] || cms[i]->pp != pps[i] || pps[i]->device != exs[0]->device || bs[i] < 1 ||
        bs[i] > pps[i]->K)
      return VC_EINVAL;
  if (n == 0) return VC_OK;
  if (g_prof) nexec = 1;  // the profiling hooks keep one record list
  // groups: jobs in input order per (params, b), cut into pieces of at most max_group
  std::vector<std::vector<uint32_t>> groups;
  {
    std::vector<std::pair<std::pair<const vc_params *, uint32_t>, uint32_t>> key(n);
    for (uint32_t i = 0; i < n; i++) key[i] = {{pps[i], bs[i]}, i};
    std::stable_sort(key.begin(), key.end(), [](const auto &a, const auto &b) {
      return a.first.first != b.first.first ? a.first.first < b.first.first : a.first.second < b.first.second;
    });
    for (uint32_t i = 0; i < n; i++) {
      if (i == 0 || key[i].first != key[i - 1].first || groups.back().size() >= max_group) groups.emplace_back();
      groups.back().push_back(key[i].second);
    }
  }
  // largest groups (entries) first, so that the last ones to start are short
  std::stable_sort(groups.begin(), groups.end(), [&](const auto &a, const auto &b) {
    return pps[a[0]]->N * a.size() > pps[b[0]]->N * b.size();
  });
  const uint32_t ng = (uint32_t)groups.size();
  if (nexec > ng) nexec = ng;
  // Fused groups of several jobs that share the device with other groups run every Step 1
  // round direct: there the lookahead's extra Miller loops and final exponentiations cost more
  // than its shorter chain saves (64-job mix: 101 against 138 ms), while one-job groups keep
  // it (253 against 272 ms).  An executor whose threshold the caller set keeps it.
  const bool shared = nexec > 1;
  std::atomic<uint32_t> next{0};
  std::vector<int> rcs(ng, VC_OK);
  std::vector<std::string> msgs(ng);  // error text of each group (kept per thread by hip_fail)
  auto worker = [&](vc_exec *ex) {
    hipError_t e = hipSetDevice(ex->device);
    std::vector<const vc_commitment *> gc;
    std::vector<vc_proofs *> go;
    for (;;) {
      uint32_t o = next.fetch_add(1);
      if (o >= ng) break;
      const auto &g = groups[o];
      if (e != hipSuccess) {
        rcs[o] = hip_fail(e, "vc_open_all_batch worker");
      } else {
        g_last_error[0] = 0;
        gc.clear();
        for (uint32_t i : g) gc.push_back(cms[i]);
        go.assign(g.size(), nullptr);
        const uint64_t amax = ex->ahead_max;
        if (shared && g.size() > 1 && !ex->ahead_set) ex->ahead_max = 0;
        rcs[o] = open_all_group(pps[g[0]], gc.data(), (uint32_t)g.size(), bs[g[0]], ex, ex->main, go.data());
        ex->ahead_max = amax;
        for (size_t x = 0; x < g.size(); x++) outs[g[x]] = go[x];
      }
      if (rcs[o] != VC_OK) msgs[o] = g_last_error;
    }
  };
  std::vector<std::thread> th;
  for (uint32_t t = 1; t < nexec; t++) th.emplace_back(worker, exs[t]);
  worker(exs[0]);
  for (auto &x : th) x.join();
  int rc = VC_OK;
  for (uint32_t o = 0; o < ng && rc == VC_OK; o++)
    if (rcs[o] != VC_OK) {
      rc = rcs[o];
      snprintf(g_last_error, sizeof g_last_error, "%s", msgs[o].c_str());
    }
  if (rc != VC_OK)
    for (uint32_t i = 0; i < n; i++) {
      vc_proofs_free(outs[i]);
      outs[i] = nullptr;
    }
  return rc;
}

VC_API int vc_open_all_batch(uint32_t n, const vc_params *const *pps, const vc_commitment *const *cms, const uint32_t *bs,
                             uint32_t nexec, vc_exec *const *exs, vc_proofs **outs) {
  return vc_open_all_grouped(n, pps, cms, bs, 1, nexec, exs, outs);
}

VC_API int vc_open_all_footprint(const vc_params *pp, uint32_t b, uint64_t *bytes) {
  if (!bytes) return VC_EINVAL;
  *bytes = 0;
  return open_all_impl(pp, nullptr, b, nullptr, nullptr, nullptr, bytes);
}

// ------------------------------------------------------------------ serving loop
// Requests wait in arrival order; a worker thread per executor takes the oldest one once it is
// free and its bytes fit the budget (the oldest waits, and the ones behind it with it, until
// they do: no request is overtaken).  The budget counts every byte the server holds: the proof
// bundles of running requests and of finished ones not yet collected by vc_server_wait, and
// the workspace and counters each executor keeps between requests.  A request needs its bundle
// plus whatever its executor's workspace and counters must grow by; when it does not fit, idle
// executors release what they keep.
struct vc_server {
  using clock = std::chrono::steady_clock;
  struct Req {
    const vc_params *pp;
    const vc_commitment *cm;
    uint32_t b;
    uint64_t bundle, ws, cnt;  // bytes of its proof bundle; workspace bytes and counters it needs
    uint64_t held = 0;         // bytes charged for it (its bundle while the server holds it)
    int state = 0;             // 0 waiting, 1 running, 2 done
    int rc = VC_OK;
    vc_proofs *out = nullptr;
    std::string err;
    clock::time_point t_sub, t_start, t_done;
  };
  int device = 0;
  uint64_t budget = 0;
  std::vector<vc_exec *> exs;
  std::vector<std::thread> th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, Req> reqs;  // element addresses stay valid while others come and go
  std::deque<uint64_t> queue;
  uint64_t next_ticket = 1, in_use = 0, peak = 0;
  bool stop = false;

  static uint64_t kept(const vc_exec *ex) { return ex->ws_size + ex->cnt_n * sizeof(uint32_t); }
  // bytes request r adds when it runs on ex
  static uint64_t need(const Req &r, const vc_exec *ex) {
    uint64_t grow_ws = r.ws > ex->ws_size ? r.ws - ex->ws_size : 0;
    uint64_t grow_cnt = r.cnt > ex->cnt_n ? (r.cnt - ex->cnt_n) * sizeof(uint32_t) : 0;
    return r.bundle + grow_ws + grow_cnt;
  }

  void worker(vc_exec *ex) {
    (void)hipSetDevice(ex->device);
    for (;;) {
      std::unique_lock<std::mutex> lk(mu);
      Req *r = nullptr;
      uint64_t add = 0;
      for (;;) {
        if (stop) return;
        if (!queue.empty()) {
          Req &f = reqs[queue.front()];
          add = need(f, ex);
          if (in_use + add <= budget) {
            r = &f;
            break;
          }
          if (kept(ex)) {
            // idle and keeping memory while the oldest request does not fit: release it (the
            // executor's own thread frees it, outside the lock)
            uint64_t k = kept(ex);
            lk.unlock();
            exec_release(ex);
            lk.lock();
            in_use -= k;
            continue;
          }
        }
        cv_work.wait(lk);
      }
      uint64_t id = queue.front();
      queue.pop_front();
      r->state = 1;
      r->t_start = clock::now();
      r->held = r->bundle;
      in_use += add;
      peak = std::max(peak, in_use);
      lk.unlock();
      cv_work.notify_all();  // the next one may fit as well
      vc_proofs *out = nullptr;
      g_last_error[0] = 0;
      uint64_t before = kept(ex);
      int rc = open_all_impl(r->pp, r->cm, r->b, ex, ex->main, &out);
      std::string err = rc != VC_OK ? std::string(g_last_error) : std::string();
      lk.lock();
      // what the executor keeps now is charged in full (a failed call may have grown less)
      in_use += kept(ex);
      in_use -= before + (add - r->bundle);
      if (rc != VC_OK) {
        in_use -= r->held;
        r->held = 0;
      }
      r->rc = rc;
      r->out = out;
      r->err = err;
      r->t_done = clock::now();
      r->state = 2;
      (void)id;
      lk.unlock();
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

VC_API void vc_server_free(vc_server *sv) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  for (auto &t : sv->th) t.join();
  for (auto &kv : sv->reqs) vc_proofs_free(kv.second.out);  // finished, never collected
  for (auto ex : sv->exs) vc_exec_free(ex);
  delete sv;
}

VC_API int vc_server_create(int device, uint32_t nexec, uint32_t nstreams, uint64_t hbm_budget, vc_server **out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!out) return VC_EINVAL;
  *out = nullptr;
  if (nexec < 1 || nexec > 64 || nstreams < 1 || nstreams > 6 || hbm_budget == 0) return VC_EINVAL;
  vc_server *sv = new vc_server();
  sv->device = device;
  sv->budget = hbm_budget;
  for (uint32_t i = 0; i < nexec; i++) {
    vc_exec *ex = nullptr;
    if (int rc = vc_exec_create(device, nstreams, &ex)) {
      vc_server_free(sv);
      return rc;
    }
    sv->exs.push_back(ex);
  }
  for (auto ex : sv->exs) sv->th.emplace_back(&vc_server::worker, sv, ex);
  *out = sv;
  return VC_OK;
}

VC_API int vc_server_submit(vc_server *sv, const vc_params *pp, const vc_commitment *cm, uint32_t b, uint64_t *ticket) {
  if (!sv || !pp || !cm || !ticket || cm->pp != pp || pp->device != sv->device) return VC_EINVAL;
  *ticket = 0;
  uint64_t foot = 0, parts[3] = {0, 0, 0};
  if (int rc = open_all_impl(pp, nullptr, b, nullptr, nullptr, nullptr, &foot, true, nullptr, parts)) return rc;
  if (foot > sv->budget) {
    snprintf(g_last_error, sizeof g_last_error, "request needs %llu bytes, budget %llu", (unsigned long long)foot,
             (unsigned long long)sv->budget);
    return VC_ENOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    uint64_t id = sv->next_ticket++;
    vc_server::Req &r = sv->reqs[id];
    r.pp = pp;
    r.cm = cm;
    r.b = b;
    r.bundle = parts[0];
    r.ws = parts[1];
    r.cnt = parts[2];
    r.t_sub = vc_server::clock::now();
    sv->queue.push_back(id);
    *ticket = id;
  }
  sv->cv_work.notify_all();
  return VC_OK;
}

VC_API int vc_server_wait(vc_server *sv, uint64_t ticket, vc_proofs **out, double times_ms[2]) {
  if (!sv || !out) return VC_EINVAL;
  *out = nullptr;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return VC_EINVAL;
  vc_server::Req *r = &it->second;
  sv->cv_done.wait(lk, [&] { return r->state == 2; });
  if (times_ms) {
    times_ms[0] = std::chrono::duration<double, std::milli>(r->t_start - r->t_sub).count();
    times_ms[1] = std::chrono::duration<double, std::milli>(r->t_done - r->t_sub).count();
  }
  int rc = r->rc;
  *out = r->out;
  if (rc != VC_OK) snprintf(g_last_error, sizeof g_last_error, "%s", r->err.c_str());
  sv->in_use -= r->held;  // the bundle now belongs to the caller
  sv->reqs.erase(ticket);
  lk.unlock();
  sv->cv_work.notify_all();
  return rc;
}

VC_API int vc_server_stats(vc_server *sv, uint64_t stats[3]) {
  if (!sv || !stats) return VC_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  stats[0] = sv->in_use;
  stats[1] = sv->peak;
  stats[2] = sv->budget;
  return VC_OK;
}

VC_API void vc_proofs_free(vc_proofs *pr) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pr) return;
  (void)hipSetDevice(pr->device);
  if (pr->mem) (void)hipFree(pr->mem);
  delete pr;
  (void)hipGetLastError();  // a release reports nothing and leaves no error behind
}

// ------------------------------------------------------------------ gathering / export
namespace {

// gather items (offsets in 32-byte units from base, encoding mode) as canonical BE bytes
int gather(const void *base, const std::vector<uint64_t> &idx, const std::vector<int> &mode, std::vector<uint8_t> &outb) {
  uint64_t n = idx.size();
  outb.assign(n * 32, 0);
  if (!n) return VC_OK;
  void *d = nullptr;
  Carve c;
  size_t oi = c.take<uint64_t>(n), om = c.take<int>(n), oo = c.take<uint8_t>(n * 32);
  CK(hipMalloc(&d, c.off));
  hipError_t e = hipMemcpy(at<void>(d, oi), idx.data(), n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(at<void>(d, om), mode.data(), n * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    kl::gather_encode(static_cast<const fe *>(base), at<uint64_t>(d, oi), at<int>(d, om), n, at<uint8_t>(d, oo), nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(outb.data(), at<void>(d, oo), n * 32, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "gather");
  return VC_OK;
}

// contiguous run of n 32-byte items starting at byte offset off
void push_run(std::vector<uint64_t> &idx, std::vector<int> &mode, size_t off, uint64_t n, int md) {
  for (uint64_t q = 0; q < n; q++) {
    idx.push_back(off / 32 + q);
    mode.push_back(md);
  }
}

const uint8_t P_HALF_BE[32] = {0x18, 0x32, 0x27, 0x39, 0x70, 0x98, 0xd0, 0x14, 0xdc, 0x28, 0x22, 0xdb, 0x40, 0xc0, 0xac, 0x2e,
                               0xcb, 0xc0, 0xb5, 0x48, 0xb4, 0x38, 0xe5, 0x46, 0x9e, 0x10, 0x46, 0x0b, 0x6c, 0x3e, 0x7e, 0xa3};

bool all_zero(const uint8_t *p, size_t n) {
  for (size_t i = 0; i < n; i++)
    if (p[i]) return false;
  return true;
}
bool larger(const uint8_t *y) { return memcmp(y, P_HALF_BE, 32) > 0; }

// compressed G1 from canonical x||y: x with flag bits (0x80 identity, 0x40 y > (p-1)/2)
void compress_g1(uint8_t *o, const uint8_t *xy) {
  if (all_zero(xy, 64)) { memset(o, 0, 32); o[0] = 0x80; return; }
  memcpy(o, xy, 32);
  if (larger(xy + 32)) o[0] |= 0x40;
}
// compressed G2 from x.c0||x.c1||y.c0||y.c1; the sign compares y.c1 first, then y.c0
void compress_g2(uint8_t *o, const uint8_t *xy) {
  if (all_zero(xy, 128)) { memset(o, 0, 64); o[0] = 0x80; return; }
  memcpy(o, xy, 64);
  bool big = all_zero(xy + 96, 32) ? larger(xy + 64) : larger(xy + 96);
  if (big) o[0] |= 0x40;
}

}  // namespace

VC_API uint64_t vc_eval_proof_len(uint32_t log_n) {
  uint32_t lK = log_n / 2, lM = log_n - lK;
  return 32 + lK * (2ull * 384 + 2 * 32) + 160 + 32 + 32ull * lM;
}

// Evaluation proof of f_m at r (section 4.3): one open-all batch over T(r_L) with the PST part
// in place of Step 2; bytes C_F || rounds || A_l v_l pi_v || F(r_R) || W_0 .. W_{lM-1}.
VC_API int vc_eval_proof(const vc_params *pp, const vc_commitment *cm, const uint8_t *r, void *stream, uint8_t *out,
                         size_t cap, size_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp || !cm || !r || !out || !len) return VC_EINVAL;
  const uint32_t lK = pp->lK, lM = pp->lM;
  const uint64_t need = vc_eval_proof_len(pp->L);
  if (cap < need) return VC_EINVAL;
  vc_proofs *pr = nullptr;
  if (int rc = open_all_impl(pp, cm, (uint32_t)pp->K, pp->ex, (hipStream_t)stream, &pr, nullptr, false, r)) return rc;
  struct Release {
    vc_proofs *p;
    ~Release() { vc_proofs_free(p); }
  } release{pr};
  std::vector<uint64_t> idx;
  std::vector<int> mode;
  push_run(idx, mode, pr->o_CF, 2, 0);
  for (uint32_t q = 0; q < lK; q++) {
    push_run(idx, mode, pr->o_Lgt + q * 384, 12, 0);
    push_run(idx, mode, pr->o_Lg1 + q * 64, 2, 0);
    push_run(idx, mode, pr->o_Rgt + q * 384, 12, 0);
    push_run(idx, mode, pr->o_Rg1 + q * 64, 2, 0);
  }
  push_run(idx, mode, pr->o_Al, 2, 0);
  push_run(idx, mode, pr->o_vl, 4, 0);
  push_run(idx, mode, pr->o_piv, 4, 0);
  push_run(idx, mode, pr->o_yv, 1, 1);
  for (uint32_t d = 0; d < lM; d++) push_run(idx, mode, pr->o_We + d * 64, 2, 0);
  std::vector<uint8_t> g;
  if (int rc = gather(pr->mem, idx, mode, g)) return rc;
  const uint8_t *s = g.data();
  uint8_t *q = out;
  compress_g1(q, s); q += 32; s += 64;
  for (uint32_t k = 0; k < lK; k++) {
    memcpy(q, s, 384); q += 384; s += 384;
    compress_g1(q, s); q += 32; s += 64;
    memcpy(q, s, 384); q += 384; s += 384;
    compress_g1(q, s); q += 32; s += 64;
  }
  compress_g1(q, s); q += 32; s += 64;
  compress_g2(q, s); q += 64; s += 128;
  compress_g2(q, s); q += 64; s += 128;
  memcpy(q, s, 32); q += 32; s += 32;
  for (uint32_t d = 0; d < lM; d++, q += 32, s += 64) compress_g1(q, s);
  *len = (size_t)(q - out);
  return *len == need ? VC_OK : VC_EDEVICE;
}

VC_API uint64_t vc_subarray_proof_len(uint32_t log_n, uint32_t t) {
  uint32_t lK = log_n / 2;
  return 32ull * t + lK * (2ull * 384 + 2 * 32) + 32 + 64 + 64;
}

VC_API int vc_subarray_proof_get(const vc_proofs *pr, uint64_t j, uint8_t *buf, size_t cap, size_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pr || !buf || !len) return VC_EINVAL;
  const vc_params *pp = pr->pp;
  const uint64_t K = pp->K;
  const uint32_t lK = pp->lK;
  if (j >= K) return VC_EINVAL;
  uint64_t k = j / pr->b, lo = k * pr->b, hi = lo + pr->b < K ? lo + pr->b : K;
  uint64_t need = vc_subarray_proof_len(pp->L, (uint32_t)(hi - lo));
  if (cap < need) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  std::vector<uint64_t> idx;
  std::vector<int> mode;
  for (uint64_t q = lo; q < hi; q++) push_run(idx, mode, pr->o_Cj + q * 64, 2, 0);
  for (uint32_t r = 0; r < lK; r++) {
    uint64_t s = k * lK + r;
    push_run(idx, mode, pr->o_Lgt + s * 384, 12, 0);
    push_run(idx, mode, pr->o_Lg1 + s * 64, 2, 0);
    push_run(idx, mode, pr->o_Rgt + s * 384, 12, 0);
    push_run(idx, mode, pr->o_Rg1 + s * 64, 2, 0);
  }
  push_run(idx, mode, pr->o_Al + k * 64, 2, 0);
  push_run(idx, mode, pr->o_vl + k * 128, 4, 0);
  push_run(idx, mode, pr->o_piv + k * 128, 4, 0);
  std::vector<uint8_t> g;
  int rc = gather(pr->mem, idx, mode, g);
  if (rc) return rc;
  const uint8_t *s = g.data();
  uint8_t *q = buf;
  for (uint64_t t = lo; t < hi; t++, s += 64, q += 32) compress_g1(q, s);
  for (uint32_t r = 0; r < lK; r++) {
    memcpy(q, s, 384); q += 384; s += 384;
    compress_g1(q, s); q += 32; s += 64;
    memcpy(q, s, 384); q += 384; s += 384;
    compress_g1(q, s); q += 32; s += 64;
  }
  compress_g1(q, s); q += 32; s += 64;
  compress_g2(q, s); q += 64; s += 128;
  compress_g2(q, s); q += 64;
  *len = (size_t)(q - buf);
  return *len == need ? VC_OK : VC_EDEVICE;
}

VC_API int vc_proof_get(const vc_proofs *pr, uint64_t i, uint8_t *buf, size_t cap, size_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pr || !buf || !len) return VC_EINVAL;
  const vc_params *pp = pr->pp;
  const uint64_t N = pp->N, K = pp->K, M = pp->M;
  const uint32_t lK = pp->lK, lM = pp->lM, L = pp->L;
  if (i >= N || !pr->step2) return VC_EINVAL;
  uint64_t j = i / M, a = i % M, k = j / pr->b;
  uint64_t lo = k * pr->b, hi = lo + pr->b < K ? lo + pr->b : K;
  uint64_t need = vc_proof_len(L, (uint32_t)(hi - lo));
  if (cap < need) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  std::vector<uint64_t> idx;
  std::vector<int> mode;
  for (uint64_t q = lo; q < hi; q++) push_run(idx, mode, pr->o_Cj + q * 64, 2, 0);
  for (uint32_t r = 0; r < lK; r++) {
    uint64_t s = k * lK + r;
    push_run(idx, mode, pr->o_Lgt + s * 384, 12, 0);
    push_run(idx, mode, pr->o_Lg1 + s * 64, 2, 0);
    push_run(idx, mode, pr->o_Rgt + s * 384, 12, 0);
    push_run(idx, mode, pr->o_Rg1 + s * 64, 2, 0);
  }
  push_run(idx, mode, pr->o_Al + k * 64, 2, 0);
  push_run(idx, mode, pr->o_vl + k * 128, 4, 0);
  push_run(idx, mode, pr->o_piv + k * 128, 4, 0);
  for (uint32_t h = 0; h < lK; h++) {
    uint64_t node = 2 * K - ((2 * K) >> h) + ((j >> h) ^ 1);
    push_run(idx, mode, pr->o_D + node * 64, 2, 0);
    push_run(idx, mode, pr->o_Y + (node * M + a) * 32, 1, 2);
  }
  for (uint32_t d = 0; d < lM; d++) push_run(idx, mode, pr->o_W + ((1ull << d) - 1 + (a >> (lM - d))) * 64, 2, 0);
  for (uint32_t h = 0; h < L; h++) push_run(idx, mode, pr->o_tree + (((N + i) >> h) ^ 1) * 32, 1, 3);
  std::vector<uint8_t> g;
  int rc = gather(pr->mem, idx, mode, g);
  if (rc) return rc;
  const uint8_t *s = g.data();
  uint8_t *q = buf;
  for (uint64_t t = lo; t < hi; t++, s += 64, q += 32) compress_g1(q, s);
  for (uint32_t r = 0; r < lK; r++) {
    memcpy(q, s, 384); q += 384; s += 384;
    compress_g1(q, s); q += 32; s += 64;
    memcpy(q, s, 384); q += 384; s += 384;
    compress_g1(q, s); q += 32; s += 64;
  }
  compress_g1(q, s); q += 32; s += 64;
  compress_g2(q, s); q += 64; s += 128;
  compress_g2(q, s); q += 64; s += 128;
  for (uint32_t h = 0; h < lK; h++) {
    compress_g1(q, s); q += 32; s += 64;
    memcpy(q, s, 32); q += 32; s += 32;
  }
  for (uint32_t d = 0; d < lM; d++) { compress_g1(q, s); q += 32; s += 64; }
  memcpy(q, s, 32ull * L);
  q += 32ull * L;
  *len = (size_t)(q - buf);
  return *len == need ? VC_OK : VC_EDEVICE;
}

static int export_items(const void *base, const std::vector<uint64_t> &idx, const std::vector<int> &mode, void *dst,
                        size_t cap, size_t *len) {
  size_t need = idx.size() * 32;
  if (len) *len = need;
  if (!dst || cap < need) return VC_EINVAL;
  std::vector<uint8_t> g;
  int rc = gather(base, idx, mode, g);
  if (rc) return rc;
  memcpy(dst, g.data(), need);
  return VC_OK;
}

VC_API int vc_params_export(const vc_params *pp, int what, uint32_t idx_, void *dst, size_t cap, size_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  std::vector<uint64_t> idx;
  std::vector<int> mode;
  size_t base = 0;
  auto off = [&](const void *p) { return (size_t)(static_cast<const char *>(p) - static_cast<const char *>(pp->mem)); };
  switch (what) {
    case 0:
      if (idx_ > pp->lM) return VC_EINVAL;
      base = off(pp->ek + ((1ull << idx_) - 1));
      push_run(idx, mode, base, 2ull << idx_, 0);
      break;
    case 1: push_run(idx, mode, off(pp->vk), 4ull * pp->lM, 0); break;
    case 2: push_run(idx, mode, off(pp->h), 4 * (2 * pp->K - 1), 0); break;
    case 3: push_run(idx, mode, off(pp->g1beta), 2, 0); break;
    default: return VC_EINVAL;
  }
  return export_items(pp->mem, idx, mode, dst, cap, len);
}

VC_API int vc_commitment_export(const vc_commitment *cm, int what, void *dst, size_t cap, size_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!cm) return VC_EINVAL;
  CK(hipSetDevice(cm->pp->device));
  std::vector<uint64_t> idx;
  std::vector<int> mode;
  auto off = [&](const void *p) { return (size_t)(static_cast<const char *>(p) - static_cast<const char *>(cm->mem)); };
  if (what == 0) push_run(idx, mode, off(cm->Cj), 2 * cm->pp->K, 0);
  else if (what == 1) push_run(idx, mode, off(cm->C), 12, 0);
  else return VC_EINVAL;
  return export_items(cm->mem, idx, mode, dst, cap, len);
}

VC_API int vc_proofs_export(const vc_proofs *pr, int what, uint64_t k, void *dst, size_t cap, size_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pr) return VC_EINVAL;
  const vc_params *pp = pr->pp;
  const uint64_t N = pp->N, K = pp->K, M = pp->M;
  const uint32_t lK = pp->lK;
  CK(hipSetDevice(pp->device));
  if (what <= 2 && k >= pr->nb) return VC_EINVAL;
  if (what >= 3 && !pr->step2) return VC_EINVAL;  // a sub-array bundle has no Step 2 arrays
  std::vector<uint64_t> idx;
  std::vector<int> mode;
  switch (what) {
    case 0:
      for (uint32_t r = 0; r < lK; r++) {
        uint64_t s = k * lK + r;
        push_run(idx, mode, pr->o_Lgt + s * 384, 12, 0);
        push_run(idx, mode, pr->o_Lg1 + s * 64, 2, 0);
        push_run(idx, mode, pr->o_Rgt + s * 384, 12, 0);
        push_run(idx, mode, pr->o_Rg1 + s * 64, 2, 0);
      }
      break;
    case 1:
      push_run(idx, mode, pr->o_Al + k * 64, 2, 0);
      push_run(idx, mode, pr->o_vl + k * 128, 4, 0);
      push_run(idx, mode, pr->o_piv + k * 128, 4, 0);
      break;
    case 2: push_run(idx, mode, pr->o_X + k * lK * 32, lK, 1); break;
    case 3: push_run(idx, mode, pr->o_tree, 2 * N, 3); break;
    case 4: push_run(idx, mode, pr->o_rho, K, 1); break;
    case 5: push_run(idx, mode, pr->o_Y, (2 * K - 1) * M, 2); break;
    case 6: push_run(idx, mode, pr->o_D, 2 * (2 * K - 1), 0); break;
    case 7: push_run(idx, mode, pr->o_W, 2 * (M - 1), 0); break;
    default: return VC_EINVAL;
  }
  return export_items(pr->mem, idx, mode, dst, cap, len);
}

// VC.Verify (appendix C) of n proofs at once, each as its own check: FC.BVerify on the proof's
// block with the faster verifier, the Merkle path to rho_j, the fold-up of D* and y*, and the
// PST check at Bin(a).  Proof q is entry idx[q]; its bytes (vc_proof_len(L, t) of them) are at
// the device address pf[q] and its entry (32 bytes, little-endian) at mi[q]; Cb: the commitment
// bytes on the device.  verdict[q]: 1 accept, 0 reject, VC_EINVAL malformed C or entry.
// fc_only: sub-array proofs (block and FC proof), the block's entry j checked against
// cj_expect[j] (an array over the K subvectors).
static int verify_many(const vc_params *pp, const uint8_t *Cb, uint32_t b, uint32_t n, const uint64_t *idx,
                       const uint8_t *const *pf, const uint8_t *const *mi, hipStream_t st, int *verdict,
                       bool fc_only = false, const g1_aff *cj_expect = nullptr) {
  if (n == 0) return VC_OK;
  const uint64_t K = pp->K, M = pp->M;
  const uint32_t lK = pp->lK, lM = pp->lM, L = pp->L;
  const uint32_t tmax = b, nmul = tmax + 2 * lK + 4, npair = 4 + lM;
  vc_exec *ex = pp->ex;
  Carve c;
  size_t o_ctx = c.take<VCtx>(n), o_blk = c.take<g1_aff>((uint64_t)n * tmax), o_Lg1 = c.take<g1_aff>(n * lK),
         o_Rg1 = c.take<g1_aff>(n * lK), o_Al = c.take<g1_aff>(n), o_D = c.take<g1_aff>(n * lK), o_W = c.take<g1_aff>(n * lM),
         o_Lgt = c.take<fp12>(n * lK), o_Rgt = c.take<fp12>(n * lK), o_Cgt = c.take<fp12>(n), o_vl = c.take<g2_aff>(n),
         o_piv = c.take<g2_aff>(n), o_ys = c.take<fe>(n * lK), o_mi = c.take<fe>(n), o_r = c.take<fe>((uint64_t)n * tmax),
         o_x = c.take<fe>(n * lK), o_xi = c.take<fe>(n * lK), o_ms = c.take<fe>((uint64_t)n * nmul), o_fz = c.take<fe>(n),
         o_gts = c.take<fe>(2 * n * lK), o_mb = c.take<g1_aff>((uint64_t)n * nmul), o_mo = c.take<g1_aff>((uint64_t)n * nmul),
         o_fzg2 = c.take<g2_aff>(n), o_gtb = c.take<fp12>(2 * n * lK), o_gtp = c.take<fp12>(2 * n * lK),
         o_gto = c.take<fp12>(n * (2 * lK + 1)), o_Cg1 = c.take<g1_aff>(n), o_bA = c.take<g1_aff>(n),
         o_pp = c.take<g1_aff>(n * npair), o_pq = c.take<g2_aff>(n * npair), o_F = c.take<fp12>(n * npair),
         o_E = c.take<fp12>(3 * n), o_G = c.take<fp12>(3 * n), o_fl = c.take<int>(n);
  // the three product trees below run one after another and share one counter area
  const uint64_t tc = tree_counters(npair > 2 * lK + 1 ? npair : 2 * lK + 1);
  if (int rc = ensure_cnt(ex, n * tc, st)) return rc;
  void *d = nullptr;
  CK(hipMalloc(&d, c.off));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } free_d{d};
  std::vector<VCtx> xs(n);
  for (uint32_t q = 0; q < n; q++) {
    VCtx &x = xs[q];
    const uint64_t i = idx[q], j = i / M, a = i % M, k = j / b, lo = k * b, hi = lo + b < K ? lo + b : K;
    const uint32_t t = (uint32_t)(hi - lo);
    x.t = t; x.lK = lK; x.lM = lM; x.L = L; x.nmul = nmul;
    x.N = pp->N; x.i = i; x.j = j; x.a = a; x.lo = lo;
    x.proof = pf[q]; x.Cb = Cb; x.mib = mi[q];
    x.mpath = x.proof + (vc_proof_len(L, t) - 32ull * L);
    x.blk = at<g1_aff>(d, o_blk) + (uint64_t)q * tmax; x.Lg1 = at<g1_aff>(d, o_Lg1) + q * lK;
    x.Rg1 = at<g1_aff>(d, o_Rg1) + q * lK; x.Al = at<g1_aff>(d, o_Al) + q; x.Dsib = at<g1_aff>(d, o_D) + q * lK;
    x.Wp = at<g1_aff>(d, o_W) + q * lM; x.Lgt = at<fp12>(d, o_Lgt) + q * lK; x.Rgt = at<fp12>(d, o_Rgt) + q * lK;
    x.C = at<fp12>(d, o_Cgt) + q; x.vl = at<g2_aff>(d, o_vl) + q; x.piv = at<g2_aff>(d, o_piv) + q;
    x.ysib = at<fe>(d, o_ys) + q * lK; x.mi = at<fe>(d, o_mi) + q; x.r = at<fe>(d, o_r) + (uint64_t)q * tmax;
    x.x = at<fe>(d, o_x) + q * lK; x.xinv = at<fe>(d, o_xi) + q * lK; x.ms = at<fe>(d, o_ms) + (uint64_t)q * nmul;
    x.fz = at<fe>(d, o_fz) + q; x.gts = at<fe>(d, o_gts) + 2 * q * lK; x.mb = at<g1_aff>(d, o_mb) + (uint64_t)q * nmul;
    x.mo = at<g1_aff>(d, o_mo) + (uint64_t)q * nmul; x.fzg2 = at<g2_aff>(d, o_fzg2) + q;
    x.gtb = at<fp12>(d, o_gtb) + 2 * q * lK; x.gtp = at<fp12>(d, o_gtp) + 2 * q * lK;
    x.gto = at<fp12>(d, o_gto) + q * (2 * lK + 1); x.Cg1 = at<g1_aff>(d, o_Cg1) + q; x.bA = at<g1_aff>(d, o_bA) + q;
    x.pp = at<g1_aff>(d, o_pp) + q * npair; x.pq = at<g2_aff>(d, o_pq) + q * npair; x.F = at<fp12>(d, o_F) + q * npair;
    x.E = at<fp12>(d, o_E) + 3 * q; x.g1beta = pp->g1beta; x.vk = pp->vk; x.flags = at<int>(d, o_fl) + q;
    x.fc_only = fc_only ? 1 : 0;
    x.cj_expect = cj_expect ? cj_expect + j : nullptr;
    if (fc_only) x.mpath = nullptr;
  }
  const VCtx *cs = at<VCtx>(d, o_ctx);
  fp12 *F = at<fp12>(d, o_F), *E = at<fp12>(d, o_E);
  std::vector<int> flags(n, 0);
  hipError_t e = hipMemcpyAsync(at<void>(d, o_ctx), xs.data(), n * sizeof(VCtx), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(at<int>(d, o_fl), 0, n * sizeof(int), st);
  if (e == hipSuccess) {
    kv::decode(cs, n, tmax, lK, lM, st);
    kv::transcript(cs, n, st);
    klw::g1_mul(at<g1_aff>(d, o_mb), 0, at<fe>(d, o_ms), (uint64_t)n * nmul, at<g1_aff>(d, o_mo), st);
    klw::g2_mul(pp->g2gen, 1, at<fe>(d, o_fz), n, at<g2_aff>(d, o_fzg2), st);
    ks::gt_pow(at<fp12>(d, o_gtb), at<fe>(d, o_gts), 2 * n * lK, at<fp12>(d, o_gtp), st);
    kv::assemble(cs, n, st);
    ks::f12_reduce(at<fp12>(d, o_gto), n, 2 * lK + 1, 2 * lK + 1, ex->cnt, st);
    ks::miller(at<g1_aff>(d, o_pp), 1, at<g2_aff>(d, o_pq), 1, (uint64_t)n * npair, F, st);
    ks::f12_reduce(F + 1, n, npair, 2, ex->cnt, st);
    ks::f12_reduce(F + 3, n, npair, npair - 3, ex->cnt, st);
    // all 3n final exponentiations in one launch: E[s] (input s even to out0[(s / 2) 2], odd to
    // out1 = out0 + 1)
    kv::fe_gather(F, npair, n, at<fp12>(d, o_G), st);
    ks::final_exp(at<fp12>(d, o_G), 1, 3ull * n, E, E + 1, 2, st);
    kv::compare(cs, n, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), at<int>(d, o_fl), n * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    ex->cnt_dirty = true;  // the product trees may have stopped half way
    return hip_fail(e, "vc_verify");
  }
  for (uint32_t q = 0; q < n; q++)
    verdict[q] = (flags[q] & VFLAG_BAD_INPUT) ? VC_EINVAL : (flags[q] & VFLAG_BAD_PROOF) ? 0 : (flags[q] & VFLAG_ACCEPT) ? 1 : 0;
  return VC_OK;
}

// VC.Verify (appendix C) of one proof: verify_many on a device copy of the inputs.
VC_API int vc_verify(const vc_params *pp, const uint8_t C[384], uint64_t n, uint32_t b, uint64_t i, const uint8_t m_i[32],
                     const uint8_t *proof, size_t len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp || !C || !m_i || !proof || n != pp->N || i >= n || b < 1 || b > pp->K) return VC_EINVAL;
  const uint64_t K = pp->K, M = pp->M;
  const uint64_t j = i / M, k = j / b, lo = k * b, hi = lo + b < K ? lo + b : K;
  if (len != vc_proof_len(pp->L, (uint32_t)(hi - lo))) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  hipStream_t st = pp->ex->side[0];
  void *d = nullptr;
  CK(hipMalloc(&d, len + 384 + 32));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } free_d{d};
  uint8_t *dp = static_cast<uint8_t *>(d), *dC = dp + len, *dm = dC + 384;
  CK(hipMemcpyAsync(dp, proof, len, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dC, C, 384, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dm, m_i, 32, hipMemcpyHostToDevice, st));
  const uint8_t *pf[1] = {dp}, *mi[1] = {dm};
  int v = 0;
  if (int rc = verify_many(pp, dC, b, 1, &i, pf, mi, st, &v)) return rc;
  return v;
}

// ------------------------------------------------------------------ profiling C ABI
VC_API void vc_profile_enable(int on) {
  if (!g_prof_recs.empty()) (void)hipDeviceSynchronize();  // recorded events may still be pending
  g_prof_recs.clear();
  g_prof_next = 0;
  g_prof = on != 0;
}

VC_API void vc_profile_only(const char *kernel) { g_prof_only = kernel ? kernel : ""; }

VC_API void vc_test_zero_challenge(uint32_t round) { g_zero_round.store(round); }

// one line per kernel: "<name> <launches> <total_ms>\n"; returns bytes needed
VC_API int vc_profile_read(char *buf, size_t cap) {
  struct Agg { std::string name; uint64_t n; double ms; };
  std::vector<Agg> agg;
  for (auto &r : g_prof_recs) {
    float ms = 0;
    if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
    std::string nm = r.name ? r.name : "?";
    bool found = false;
    for (auto &a : agg)
      if (a.name == nm) { a.n++; a.ms += ms; found = true; break; }
    if (!found) agg.push_back({nm, 1, ms});
  }
  std::string out;
  char line[256];
  for (auto &a : agg) {
    snprintf(line, sizeof line, "%s %llu %.6f\n", a.name.c_str(), (unsigned long long)a.n, a.ms);
    out += line;
  }
  if (buf && cap > 0) {
    size_t n = out.size() < cap - 1 ? out.size() : cap - 1;
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return (int)out.size() + 1;
}

// ------------------------------------------------------------------ diagnostics
// Runs one base-field operation on n pairs of canonical 32-byte little-endian inputs
// Verification of an evaluation proof at a point (section 4.3): FC.BVerify of C_F = <C, T(r_L)>
// with the faster verifier, and PC.Verify of F at r_R; the final equalities as for one opening
// proof.
VC_API int vc_verify_eval(const vc_params *pp, const uint8_t C[384], const uint8_t *r, const uint8_t *proof,
                          size_t len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp || !C || !r || !proof || len != vc_eval_proof_len(pp->L)) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  vc_exec *ex = pp->ex;
  hipStream_t st = ex->side[0];
  const uint32_t L = pp->L, l = pp->lK, lM = pp->lM, npair = 4 + lM, nmul = 2 * l + 4;
  const uint64_t K = pp->K;
  Carve w;
  size_t o_pf = w.take<uint8_t>(len), o_Cb = w.take<uint8_t>(384), o_rle = w.take<uint8_t>(32 * L),
         o_CF = w.take<g1_aff>(1), o_Lg1 = w.take<g1_aff>(l), o_Rg1 = w.take<g1_aff>(l), o_Al = w.take<g1_aff>(1),
         o_W = w.take<g1_aff>(lM), o_Lgt = w.take<fp12>(l), o_Rgt = w.take<fp12>(l), o_C = w.take<fp12>(1),
         o_vl = w.take<g2_aff>(1), o_piv = w.take<g2_aff>(1), o_r = w.take<fe>(L), o_y = w.take<fe>(1),
         o_T = w.take<fe>(K), o_x = w.take<fe>(l), o_xi = w.take<fe>(l), o_ms = w.take<fe>(nmul),
         o_mb = w.take<g1_aff>(nmul), o_mo = w.take<g1_aff>(nmul), o_g2s = w.take<fe>(1 + lM),
         o_g2o = w.take<g2_aff>(1 + lM), o_gts = w.take<fe>(2 * l), o_gtb = w.take<fp12>(2 * l),
         o_gtp = w.take<fp12>(2 * l), o_gto = w.take<fp12>(2 * l + 1), o_pp = w.take<g1_aff>(npair),
         o_pq = w.take<g2_aff>(npair), o_F = w.take<fp12>(npair), o_E = w.take<fp12>(3), o_Cg1 = w.take<g1_aff>(1),
         o_bA = w.take<g1_aff>(1), o_fl = w.take<int>(1), o_ctx = w.take<VCtx>(1), o_G = w.take<fp12>(3);
  if (int rc = ensure_cnt(ex, tree_counters(npair > 2 * l + 1 ? npair : 2 * l + 1), st)) return rc;
  void *d = nullptr;
  CK(hipMalloc(&d, w.off));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } free_d{d};
  VECtx c;
  c.L = L; c.lK = l; c.lM = lM; c.K = K; c.M = pp->M;
  c.proof = at<uint8_t>(d, o_pf); c.Cb = at<uint8_t>(d, o_Cb); c.rle = at<uint8_t>(d, o_rle);
  c.CF = at<g1_aff>(d, o_CF); c.Lg1 = at<g1_aff>(d, o_Lg1); c.Rg1 = at<g1_aff>(d, o_Rg1); c.Al = at<g1_aff>(d, o_Al);
  c.W = at<g1_aff>(d, o_W); c.Lgt = at<fp12>(d, o_Lgt); c.Rgt = at<fp12>(d, o_Rgt); c.C = at<fp12>(d, o_C);
  c.vl = at<g2_aff>(d, o_vl); c.piv = at<g2_aff>(d, o_piv); c.r = at<fe>(d, o_r); c.y = at<fe>(d, o_y);
  c.T = at<fe>(d, o_T); c.x = at<fe>(d, o_x); c.xinv = at<fe>(d, o_xi); c.ms = at<fe>(d, o_ms);
  c.mb = at<g1_aff>(d, o_mb); c.mo = at<g1_aff>(d, o_mo); c.g2s = at<fe>(d, o_g2s); c.g2o = at<g2_aff>(d, o_g2o);
  c.gts = at<fe>(d, o_gts); c.gtb = at<fp12>(d, o_gtb); c.gtp = at<fp12>(d, o_gtp); c.gto = at<fp12>(d, o_gto);
  c.pp = at<g1_aff>(d, o_pp); c.pq = at<g2_aff>(d, o_pq); c.Cg1 = at<g1_aff>(d, o_Cg1); c.bA = at<g1_aff>(d, o_bA);
  c.g1beta = pp->g1beta; c.vk = pp->vk; c.flags = at<int>(d, o_fl);
  // the final equalities reuse the one-proof comparison
  VCtx x = {};
  x.E = at<fp12>(d, o_E); x.gto = c.gto; x.bA = c.bA; x.Cg1 = c.Cg1; x.flags = c.flags;
  fp12 *F = at<fp12>(d, o_F), *E = x.E;
  int flags = 0;
  hipError_t e = hipMemcpyAsync(at<void>(d, o_pf), proof, len, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(at<void>(d, o_Cb), C, 384, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(at<void>(d, o_rle), r, 32ull * L, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(at<void>(d, o_ctx), &x, sizeof x, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(c.flags, 0, sizeof(int), st);
  if (e == hipSuccess) {
    kve::decode(c, st);
    kl::ev_eq(c.r, lM, l, K, c.T, st);
    kve::transcript(c, st);
    klw::g1_mul(c.mb, 0, c.ms, nmul, c.mo, st);
    klw::g2_mul(pp->g2gen, 1, c.g2s, 1 + lM, c.g2o, st);
    ks::gt_pow(c.gtb, c.gts, 2 * l, c.gtp, st);
    kve::assemble(c, st);
    ks::f12_reduce(c.gto, 1, 2 * l + 1, 2 * l + 1, ex->cnt, st);
    ks::miller(c.pp, 1, c.pq, 1, npair, F, st);
    ks::f12_reduce(F + 1, 1, npair, 2, ex->cnt, st);
    ks::f12_reduce(F + 3, 1, npair, npair - 3, ex->cnt, st);
    kv::fe_gather(F, npair, 1, at<fp12>(d, o_G), st);
    ks::final_exp(at<fp12>(d, o_G), 1, 3, E, E + 1, 2, st);
    kv::compare(at<VCtx>(d, o_ctx), 1, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, c.flags, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    ex->cnt_dirty = true;  // the product trees may have stopped half way
    return hip_fail(e, "vc_verify_eval");
  }
  if (flags & VFLAG_BAD_INPUT) return VC_EINVAL;
  if (flags & VFLAG_BAD_PROOF) return 0;
  return (flags & VFLAG_ACCEPT) ? 1 : 0;
}

// Sub-array verification (section 4.3): the commitment of m_j is recomputed (PC.Commit, the
// MSM of the commit) and must be entry j of the proof's block, whose FC proof must hold.
VC_API int vc_verify_subarray(const vc_params *pp, const uint8_t C[384], uint32_t b, uint64_t j, const uint8_t *m_j,
                              const uint8_t *proof, size_t len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pp || !C || !m_j || !proof || j >= pp->K || b < 1 || b > pp->K) return VC_EINVAL;
  const uint64_t K = pp->K, M = pp->M;
  const uint64_t k = j / b, lo = k * b, hi = lo + b < K ? lo + b : K;
  if (len != vc_subarray_proof_len(pp->L, (uint32_t)(hi - lo))) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  hipStream_t st = pp->ex->side[0];
  uint32_t S = (uint32_t)(8192 / NWIN);
  if (S > M) S = (uint32_t)M;
  const uint64_t nslice = (M + S - 1) / S;
  Carve w;
  size_t o_pf = w.take<uint8_t>(len), o_C = w.take<uint8_t>(384), o_m = w.take<fe>(M), o_err = w.take<int>(1),
         o_part = w.take<g1_jac>(nslice), o_cj = w.take<g1_aff>(K);
  void *d = nullptr;
  CK(hipMalloc(&d, w.off));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } free_d{d};
  int *err = at<int>(d, o_err);
  CK(hipMemcpyAsync(at<void>(d, o_pf), proof, len, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(at<void>(d, o_C), C, 384, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(at<void>(d, o_m), m_j, M * 32, hipMemcpyHostToDevice, st));
  CK(hipMemsetAsync(err, 0, sizeof(int), st));
  kl::check_fr(at<fe>(d, o_m), M, err, st);
  kl::msm_slices(at<fe>(d, o_m), 1, M, NWIN, S, pp->table, at<g1_jac>(d, o_part), st);
  klw::sum_g1(at<g1_jac>(d, o_part), 1, nslice, at<g1_aff>(d, o_cj) + j, st);  // entry j of the K
  int herr = 0;
  CK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (herr & VC_ERRBIT_RANGE) return VC_EINVAL;
  const uint64_t i = j * M;
  const uint8_t *pf[1] = {at<uint8_t>(d, o_pf)}, *mi[1] = {at<uint8_t>(d, o_C)};  // (no entry is read)
  int v = 0;
  if (int rc = verify_many(pp, at<uint8_t>(d, o_C), b, 1, &i, pf, mi, st, &v, true, at<g1_aff>(d, o_cj))) return rc;
  return v;
}

// All K sub-array proofs at once (section 4.3): every C_j recomputed with the commit's MSM
// and found at its place in its proof's block; proofs compared with the first of their batch;
// one FC check per batch and per differing proof, in one pass of the verifier.
VC_API int vc_verify_subarrays_all(const vc_params *pp, const uint8_t C[384], uint32_t b, const void *m,
                                   const void *proofs, uint64_t len, uint64_t *n_single) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (n_single) *n_single = 0;
  if (!pp || !C || !m || !proofs || b < 1 || b > pp->K) return VC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(proofs) & 15) != 0) return VC_EINVAL;
  const uint64_t K = pp->K, M = pp->M, N = pp->N, nb = (K + b - 1) / b;
  const uint32_t t_last = (uint32_t)(K - (nb - 1) * b);
  const uint64_t len_full = vc_subarray_proof_len(pp->L, b), len_last = vc_subarray_proof_len(pp->L, t_last);
  if (len != (nb - 1) * b * len_full + t_last * len_last) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  vc_exec *ex = pp->ex;
  hipStream_t st = ex->main;
  uint32_t S = (uint32_t)(8192 / NWIN);
  if (S > M) S = (uint32_t)M;
  const uint64_t nslice = (M + S - 1) / S;
  Carve w;
  size_t o_Cb = w.take<uint8_t>(384), o_err = w.take<int>(1), o_fl = w.take<int>(1), o_oc = w.take<uint32_t>(1),
         o_part = w.take<g1_jac>(K * nslice), o_Cre = w.take<g1_aff>(K), o_ol = w.take<uint64_t>(K);
  void *d = nullptr;
  CK(hipMalloc(&d, w.off));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } free_d{d};
  const uint8_t *P = static_cast<const uint8_t *>(proofs);
  g1_aff *Cre = at<g1_aff>(d, o_Cre);
  CK(hipMemcpyAsync(at<void>(d, o_Cb), C, 384, hipMemcpyHostToDevice, st));
  CK(hipMemsetAsync(at<void>(d, o_err), 0, sizeof(int), st));
  CK(hipMemsetAsync(at<void>(d, o_fl), 0, sizeof(int), st));
  CK(hipMemsetAsync(at<void>(d, o_oc), 0, sizeof(uint32_t), st));
  kl::check_fr(static_cast<const fe *>(m), N, at<int>(d, o_err), st);
  kl::msm_slices(static_cast<const fe *>(m), K, M, NWIN, S, pp->table, at<g1_jac>(d, o_part), st);
  klw::sum_g1(at<g1_jac>(d, o_part), K, nslice, Cre, st);
  ksa::check(P, K, b, nb, len_full, len_last, Cre, at<uint64_t>(d, o_ol), at<uint32_t>(d, o_oc), at<int>(d, o_fl), st);
  int herr = 0, flags = 0;
  uint32_t nodd = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, at<int>(d, o_err), sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, at<int>(d, o_fl), sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nodd, at<uint32_t>(d, o_oc), sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "vc_verify_subarrays_all");
  if (herr & VC_ERRBIT_RANGE) return VC_EINVAL;
  if (flags & VFLAG_BAD_PROOF) return 0;
  std::vector<uint64_t> single;
  for (uint64_t k = 0; k < nb; k++) single.push_back(k * b);
  if (nodd) {
    std::vector<uint64_t> ol(nodd);
    CK(hipMemcpy(ol.data(), at<uint64_t>(d, o_ol), nodd * sizeof(uint64_t), hipMemcpyDeviceToHost));
    single.insert(single.end(), ol.begin(), ol.end());
  }
  std::sort(single.begin(), single.end());
  single.erase(std::unique(single.begin(), single.end()), single.end());
  std::vector<uint64_t> idx(single.size());
  std::vector<const uint8_t *> pfs(single.size()), mis(single.size(), at<uint8_t>(d, o_Cb));  // (no entry is read)
  for (size_t q = 0; q < single.size(); q++) {
    uint64_t j = single[q], k = j / b;
    idx[q] = j * M;
    pfs[q] = P + k * b * len_full + (j - k * b) * (k == nb - 1 ? len_last : len_full);
  }
  std::vector<int> v(single.size(), 0);
  const uint32_t chunk = 4096;
  for (size_t q0 = 0; q0 < single.size(); q0 += chunk) {
    uint32_t nq = (uint32_t)std::min<size_t>(chunk, single.size() - q0);
    if (int rc = verify_many(pp, at<uint8_t>(d, o_Cb), b, nq, idx.data() + q0, pfs.data() + q0, mis.data() + q0, st,
                             v.data() + q0, true, Cre))
      return rc;
    if (n_single) *n_single += nq;
    for (uint32_t q = 0; q < nq; q++) {
      if (v[q0 + q] < 0) return v[q0 + q];
      if (v[q0 + q] != 1) return 0;
    }
  }
  return 1;
}

// ------------------------------------------------------------------ every proof at once
static PLayout proof_layout(const vc_params *pp, uint32_t b) {
  PLayout y;
  y.L = pp->L; y.lK = pp->lK; y.lM = pp->lM; y.b = b;
  y.N = pp->N; y.K = pp->K; y.M = pp->M;
  y.nb = (pp->K + b - 1) / b;
  y.t_last = (uint32_t)(pp->K - (y.nb - 1) * b);
  y.len_full = vc_proof_len(pp->L, b);
  y.len_last = vc_proof_len(pp->L, y.t_last);
  return y;
}
static uint64_t proofs_total(const PLayout &y) {
  return (y.nb - 1) * y.b * y.M * y.len_full + (uint64_t)y.t_last * y.M * y.len_last;
}
static uint64_t proof_offset(const PLayout &y, uint64_t i) {
  uint64_t bm = (uint64_t)y.b * y.M, k = i / bm;
  return k * bm * y.len_full + (i - k * bm) * (k == y.nb - 1 ? y.len_last : y.len_full);
}

VC_API int vc_proofs_serialize(const vc_proofs *pr, void *dst, uint64_t cap, uint64_t *len) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!pr || !len || !pr->step2) return VC_EINVAL;
  const vc_params *pp = pr->pp;
  PLayout y = proof_layout(pp, pr->b);
  *len = proofs_total(y);
  if (!dst) return VC_OK;
  if (cap < *len) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  hipStream_t st = pp->ex->side[0];
  PSCtx c;
  c.y = y;
  void *bm = pr->mem;
  c.Cj = at<g1_aff>(bm, pr->o_Cj); c.Lg1 = at<g1_aff>(bm, pr->o_Lg1); c.Rg1 = at<g1_aff>(bm, pr->o_Rg1);
  c.Al = at<g1_aff>(bm, pr->o_Al); c.D = at<g1_aff>(bm, pr->o_D); c.W = at<g1_aff>(bm, pr->o_W);
  c.Lgt = at<fp12>(bm, pr->o_Lgt); c.Rgt = at<fp12>(bm, pr->o_Rgt);
  c.vl = at<g2_aff>(bm, pr->o_vl); c.piv = at<g2_aff>(bm, pr->o_piv);
  c.Y = at<fe>(bm, pr->o_Y); c.tree = at<uint32_t>(bm, pr->o_tree);
  c.out = static_cast<uint8_t *>(dst);
  kva::serialize(c, st);
  CKL("vc_proofs_serialize launch");
  CK(hipStreamSynchronize(st));
  return VC_OK;
}

VC_API int vc_verify_all(const vc_params *pp, const uint8_t C[384], uint32_t b, const void *m, const void *proofs,
                         uint64_t len, const uint8_t seed[32], uint64_t *n_single) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (n_single) *n_single = 0;
  if (!pp || !C || !m || !proofs || !seed || b < 1 || b > pp->K) return VC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(proofs) & 15) != 0) return VC_EINVAL;
  PLayout y = proof_layout(pp, b);
  if (len != proofs_total(y)) return VC_EINVAL;
  CK(hipSetDevice(pp->device));
  vc_exec *ex = pp->ex;
  hipStream_t st = ex->main;
  const uint64_t N = y.N, K = y.K, M = y.M;
  VACtx c;
  c.y = y;
  c.proofs = static_cast<const uint8_t *>(proofs);
  c.m = static_cast<const uint8_t *>(m);
  c.vk = pp->vk;
  Carve w;
  size_t o_Cb = w.take<uint8_t>(384), o_seed = w.take<uint8_t>(32), o_Cj = w.take<g1_aff>(K), o_Dn = w.take<g1_aff>(2 * K),
         o_Wn = w.take<g1_aff>(M), o_C = w.take<fp12>(1), o_root = w.take<uint32_t>(8 * N), o_rho = w.take<fe>(K),
         o_delta = w.take<fe>(N), o_dy = w.take<fe>(N), o_odd = w.take<uint8_t>(N), o_ol = w.take<uint64_t>(N),
         o_oc = w.take<uint32_t>(1), o_row = w.take<fe>(K), o_col = w.take<fe>(M), o_sy = w.take<fe>(1);
  const uint64_t T = 3 * K + 2 * M - 3;
  size_t o_bases = w.take<g1_aff>(T), o_scal = w.take<fe>(T), o_prod = w.take<g1_aff>(T), o_pp = w.take<g1_aff>(y.lM + 1),
         o_pq = w.take<g2_aff>(y.lM + 1), o_F = w.take<fp12>(y.lM + 1), o_E = w.take<fp12>(1), o_fl = w.take<int>(1);
  if (int rc = ensure_cnt(ex, tree_counters(y.lM + 1), st)) return rc;
  void *d = nullptr;
  CK(hipMalloc(&d, w.off));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } free_d{d};
  c.Cb = at<uint8_t>(d, o_Cb); c.seed = at<uint8_t>(d, o_seed);
  c.Cj = at<g1_aff>(d, o_Cj); c.Dn = at<g1_aff>(d, o_Dn); c.Wn = at<g1_aff>(d, o_Wn); c.C = at<fp12>(d, o_C);
  c.root = at<uint32_t>(d, o_root); c.rho = at<fe>(d, o_rho); c.delta = at<fe>(d, o_delta); c.dy = at<fe>(d, o_dy);
  c.odd = at<uint8_t>(d, o_odd); c.oddlist = at<uint64_t>(d, o_ol); c.oddcnt = at<uint32_t>(d, o_oc);
  c.rowsum = at<fe>(d, o_row); c.colsum = at<fe>(d, o_col); c.sy = at<fe>(d, o_sy);
  c.bases = at<g1_aff>(d, o_bases); c.scal = at<fe>(d, o_scal); c.prod = at<g1_aff>(d, o_prod);
  c.pp = at<g1_aff>(d, o_pp); c.pq = at<g2_aff>(d, o_pq); c.E = at<fp12>(d, o_E); c.flags = at<int>(d, o_fl);
  fp12 *F = at<fp12>(d, o_F);
  CK(hipMemcpyAsync(at<void>(d, o_Cb), C, 384, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(at<void>(d, o_seed), seed, 32, hipMemcpyHostToDevice, st));
  CK(hipMemsetAsync(c.flags, 0, sizeof(int), st));
  CK(hipMemsetAsync(c.oddcnt, 0, sizeof(uint32_t), st));
  kva::decode(c, st);
  kva::roots(c, st);
  kva::rho(c, st);
  kva::same(c, st);
  kva::proof(c, st);
  kva::sums(c, st);
  kva::terms(c, st);
  klw::g1_mul(c.bases, 0, c.scal, T, c.prod, st);
  kva::segsum(c, st);
  ks::miller(c.pp, 1, c.pq, 1, y.lM + 1, F, st);
  ks::f12_reduce(F, 1, y.lM + 1, y.lM + 1, ex->cnt, st);
  ks::final_exp(F, 1, 1, c.E, nullptr, 1, st);
  kva::check(c, st);
  int flags = 0;
  uint32_t nodd = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, c.flags, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nodd, c.oddcnt, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    ex->cnt_dirty = true;
    return hip_fail(e, "vc_verify_all");
  }
  if (flags & VFLAG_BAD_INPUT) return VC_EINVAL;
  if (flags & VFLAG_BAD_PROOF) return 0;
  // the combined check covers every proof that is not left to the one-proof verifier
  if (nodd < N && !(flags & VFLAG_ACCEPT)) return 0;
  // one proof per batch (its FC part) and the proofs that differ from their representatives,
  // in index order, one at a time; the first rejection ends the call
  std::vector<uint64_t> single;
  for (uint64_t k = 0; k < y.nb; k++) single.push_back(k * y.b * M);
  if (nodd) {
    std::vector<uint64_t> ol(nodd);
    CK(hipMemcpy(ol.data(), c.oddlist, nodd * sizeof(uint64_t), hipMemcpyDeviceToHost));
    single.insert(single.end(), ol.begin(), ol.end());
  }
  std::sort(single.begin(), single.end());
  single.erase(std::unique(single.begin(), single.end()), single.end());
  // (device copy of C for the one-proof checks)
  std::vector<const uint8_t *> pfs(single.size()), mis(single.size());
  for (size_t q = 0; q < single.size(); q++) {
    pfs[q] = c.proofs + proof_offset(y, single[q]);
    mis[q] = c.m + 32 * single[q];
  }
  std::vector<int> v(single.size(), 0);
  const uint32_t chunk = 4096;  // bounded working memory per pass
  for (size_t q0 = 0; q0 < single.size(); q0 += chunk) {
    uint32_t nq = (uint32_t)std::min<size_t>(chunk, single.size() - q0);
    if (int rc = verify_many(pp, c.Cb, b, nq, single.data() + q0, pfs.data() + q0, mis.data() + q0, st, v.data() + q0))
      return rc;
    if (n_single) *n_single += nq;
    for (uint32_t q = 0; q < nq; q++) {
      if (v[q0 + q] < 0) return v[q0 + q];
      if (v[q0 + q] != 1) return 0;
    }
  }
  return 1;
}

// (host buffers) in the 8-lanes-per-element layout: op 0 mul, 1 add, 2 sub, 3 half,
// 4 inverse, 5 square; which 0 = F_p, 1 = F_r.
VC_API int vc_diag_field(int which, int op, uint64_t n, const void *a, const void *b, void *out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!a || !b || !out || n == 0) return VC_EINVAL;
  void *d = nullptr;
  CK(hipMalloc(&d, 3 * n * 32));
  hipError_t e = hipMemcpy(d, a, n * 32, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(static_cast<char *>(d) + n * 32, b, n * 32, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    klw::diag_field(which, op, d, static_cast<char *>(d) + n * 32, n, static_cast<char *>(d) + 2 * n * 32, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, static_cast<char *>(d) + 2 * n * 32, n * 32, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "vc_diag_field");
  return VC_OK;
}

VC_API int vc_diag_fold(const vc_commitment *cm, double *ms_out) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!cm || !ms_out) return VC_EINVAL;
  const vc_params *pp = cm->pp;
  CK(hipSetDevice(pp->device));
  const uint64_t K = pp->K, M = pp->M;
  Carve t;
  size_t o_rho = t.take<fe>(K), o_Y = t.take<fe>((2 * K - 1) * M), o_J = t.take<S2Job>(1);
  void *d = nullptr;
  CK(hipMalloc(&d, t.off));
  // rho_j = 1 (Montgomery form R mod r): the passes read the entries and write every node
  std::vector<fe> one(K);
  for (auto &v : one) v = fe_const(bn::R_ONE);
  S2Job j = {cm->m, cm->Cj, cm->C, nullptr, at<fe>(d, o_rho), at<fe>(d, o_Y), nullptr, nullptr};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemcpy(at<fe>(d, o_rho), one.data(), K * sizeof(fe), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(at<S2Job>(d, o_J), &j, sizeof j, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = 0;
  for (int rep = 0; rep < 6 && e == hipSuccess; rep++) {
    e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) {
      kl::ytree(at<S2Job>(d, o_J), 1, M, K, pp->lK, nullptr);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best == 0 || ms < best)) best = ms;  // rep 0 warms up
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "vc_diag_fold");
  *ms_out = best;
  return VC_OK;
}

VC_API int vc_diag_mad_rate(int device, double *tera_per_s) {
  (void)hipGetLastError();  // errors left by other HIP clients are not ours
  if (!tera_per_s) return VC_EINVAL;
  CK(hipSetDevice(device));
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, device));
  // 8 workgroups of 4 waves per compute unit: 8 waves per SIMD
  const unsigned blocks = 8u * (unsigned)prop.multiProcessorCount;
  const uint32_t iters = 8192;
  uint64_t *d = nullptr;
  CK(hipMalloc(&d, (size_t)blocks * 256 * sizeof(uint64_t)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 0;
  for (int rep = 0; rep < 6 && e == hipSuccess; rep++) {
    e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) {
      kl::diag_mad(0x9e3779b9u + rep, iters, blocks, d, nullptr);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    double mads = (double)blocks * 256.0 * 8.0 * iters;
    if (e == hipSuccess && rep > 0 && ms > 0) best = std::max(best, mads / (ms * 1e-3) / 1e12);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "vc_diag_mad_rate");
  *tera_per_s = best;
  return VC_OK;
}
