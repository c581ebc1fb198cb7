"""FlexProofs on MI355X: Python binding of the C ABI in include/vc.h.

Argument marshalling only: every step of commit / open-all runs in the HIP
kernels of lib/libvc.so.  PyTorch supplies device memory and streams.  The
library must have been built (``python -m paper_2601_03031_amd.build``); if it is
missing, every call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libvc.so")

# open-all runs on the caller's stream and five side streams, and batches run several jobs
# at once on executors of their own; HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues
# per process (default 4), and streams that share a queue run one after the other.  Raised
# to 16 here (one job's six streams, or sixteen one-stream jobs, on queues of their own;
# more queues than that slowed single jobs down in measurements); takes effect only before
# the process first uses the device.
HW_QUEUES = 16


def _raise_hw_queues() -> None:
    try:
        cur = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    except ValueError:
        cur = 4
    if cur < HW_QUEUES:
        os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)
        # too late if torch has already started HIP in this process: say so (an open-all at
        # N = 2^16, b = 256 measured 25.5 ms on 4 queues against 17.5 ms on 16)
        import sys
        torch = sys.modules.get("torch")
        try:
            started = torch is not None and torch.cuda.is_initialized()
        except Exception:
            started = False
        if started:
            import warnings
            warnings.warn("paper_2601_03031_amd imported after the device was first used: HIP keeps "
                          "GPU_MAX_HW_QUEUES=%d, so the open-all's side streams share hardware queues "
                          "and run partly in sequence (same results, longer latency); import the "
                          "package, or set the variable, before the first device use" % cur,
                          RuntimeWarning, stacklevel=3)


_raise_hw_queues()

VC_OK, VC_EINVAL, VC_ENOMEM, VC_EDEVICE, VC_ENOTIMPL, VC_ECHALLENGE = 0, -1, -2, -3, -4, -5

_lib = None


class VCError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().vc_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s failed: %s (%d)" % (where, msg, code))


def lib():
    """Load lib/libvc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("FlexProofs HIP library not built: %s is missing "
                               "(run python -m paper_2601_03031_amd.build)" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, u8p, u64, u32, sz = C.c_void_p, C.c_char_p, C.c_uint64, C.c_uint32, C.c_size_t
        L.vc_setup.argtypes = [u32, u8p, C.c_int, C.POINTER(vp)]
        L.vc_commit.argtypes = [vp, vp, u64, u32, vp, C.POINTER(vp), vp]
        L.vc_open_all.argtypes = [vp, vp, u32, vp, C.POINTER(vp)]
        L.vc_commit_noalloc.argtypes = [vp, vp, u64, u32, vp, vp, vp]
        L.vc_params_load.argtypes = [u8p, sz, C.c_int, C.POINTER(vp)]
        L.vc_commit_batch.argtypes = [u32, C.POINTER(vp), C.POINTER(vp), C.POINTER(u32), vp, vp, C.POINTER(vp), vp]
        L.vc_tune_msm.argtypes = [C.c_int, u32, u32, C.c_char_p]
        L.vc_tune_load.argtypes = [C.c_char_p]
        L.vc_diag_fold.argtypes = [vp, C.POINTER(C.c_double)]
        L.vc_diag_mad_rate.argtypes = [C.c_int, C.POINTER(C.c_double)]
        L.vc_exec_create.argtypes = [C.c_int, u32, C.POINTER(vp)]
        L.vc_exec_free.argtypes = [vp]
        L.vc_exec_set_graphs.argtypes = [vp, C.c_int]
        L.vc_exec_set_ahead.argtypes = [vp, u64]
        L.vc_exec_graph_stats.argtypes = [vp, vp]
        L.vc_open_all_ex.argtypes = [vp, vp, u32, vp, vp, C.POINTER(vp)]
        L.vc_open_all_footprint.argtypes = [vp, u32, C.POINTER(u64)]
        L.vc_server_create.argtypes = [C.c_int, u32, u32, u64, C.POINTER(vp)]
        L.vc_server_submit.argtypes = [vp, vp, vp, u32, C.POINTER(u64)]
        L.vc_server_wait.argtypes = [vp, u64, C.POINTER(vp), C.POINTER(C.c_double)]
        L.vc_server_free.argtypes = [vp]
        L.vc_server_stats.argtypes = [vp, C.POINTER(u64)]
        L.vc_proofs_serialize.argtypes = [vp, vp, u64, C.POINTER(u64)]
        L.vc_open_subarrays.argtypes = [vp, vp, u32, vp, C.POINTER(vp)]
        L.vc_eval_proof_len.restype = u64
        L.vc_eval_proof_len.argtypes = [u32]
        L.vc_eval_proof.argtypes = [vp, vp, u8p, vp, vp, sz, C.POINTER(sz)]
        L.vc_verify_eval.argtypes = [vp, u8p, u8p, u8p, sz]
        L.vc_subarray_proof_len.restype = u64
        L.vc_subarray_proof_len.argtypes = [u32, u32]
        L.vc_subarray_proof_get.argtypes = [vp, u64, vp, sz, C.POINTER(sz)]
        L.vc_verify_subarray.argtypes = [vp, u8p, u32, u64, u8p, u8p, sz]
        L.vc_verify_subarrays_all.argtypes = [vp, u8p, u32, vp, vp, u64, C.POINTER(u64)]
        L.vc_verify_all.argtypes = [vp, u8p, u32, vp, vp, u64, u8p, C.POINTER(u64)]
        L.vc_open_all_batch.argtypes = [u32, C.POINTER(vp), C.POINTER(vp), C.POINTER(u32), u32, C.POINTER(vp),
                                        C.POINTER(vp)]
        L.vc_open_all_grouped.argtypes = [u32, C.POINTER(vp), C.POINTER(vp), C.POINTER(u32), u32, u32,
                                          C.POINTER(vp), C.POINTER(vp)]
        L.vc_proof_len.restype = u64
        L.vc_proof_len.argtypes = [u32, u32]
        L.vc_proof_get.argtypes = [vp, u64, vp, sz, C.POINTER(sz)]
        L.vc_verify.argtypes = [vp, u8p, u64, u32, u64, u8p, u8p, sz]
        L.vc_params_export.argtypes = [vp, C.c_int, u32, vp, sz, C.POINTER(sz)]
        L.vc_commitment_export.argtypes = [vp, C.c_int, vp, sz, C.POINTER(sz)]
        L.vc_proofs_export.argtypes = [vp, C.c_int, u64, vp, sz, C.POINTER(sz)]
        for f in ("vc_params_free", "vc_commitment_free", "vc_proofs_free"):
            getattr(L, f).argtypes = [vp]
        L.vc_profile_enable.argtypes = [C.c_int]
        L.vc_profile_only.argtypes = [C.c_char_p]
        L.vc_profile_read.argtypes = [C.c_char_p, sz]
        L.vc_test_zero_challenge.argtypes = [u32]
        L.vc_strerror.restype = C.c_char_p
        L.vc_strerror.argtypes = [C.c_int]
        _lib = L
    return _lib


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise VCError(rc, where)
    return rc


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(getattr(stream, "cuda_stream", stream))


class _Handle:
    _free = ""

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            getattr(_lib, self._free)(self.ptr)
            self.ptr = None


class Params(_Handle):
    _free = "vc_params_free"

    def __init__(self, ptr, log_n, device=0):
        super().__init__(ptr)
        self.log_n, self.device = log_n, device
        self.lK = log_n // 2
        self.lM = log_n - self.lK
        self.N, self.K, self.M = 1 << log_n, 1 << self.lK, 1 << self.lM

    def export(self, what: str, idx: int = 0) -> bytes:
        codes = {"ek": 0, "vk": 1, "h": 2, "g1beta": 3}
        n = C.c_size_t(0)
        lib().vc_params_export(self.ptr, codes[what], idx, None, 0, C.byref(n))
        buf = C.create_string_buffer(n.value)
        _check(lib().vc_params_export(self.ptr, codes[what], idx, buf, n.value, C.byref(n)), "vc_params_export")
        return buf.raw

    def srs_bytes(self) -> bytes:
        """The keys in vc_params_load's layout: ek_0..ek_{log M}, vk, h, beta g1."""
        return b"".join([self.export("ek", k) for k in range(self.lM + 1)] +
                        [self.export("vk"), self.export("h"), self.export("g1beta")])


class Commitment(_Handle):
    _free = "vc_commitment_free"

    def __init__(self, ptr, pp, C_bytes):
        super().__init__(ptr)
        self.pp, self.C = pp, C_bytes

    def export(self, what: str) -> bytes:
        codes = {"Cj": 0, "C": 1}
        n = C.c_size_t(0)
        lib().vc_commitment_export(self.ptr, codes[what], None, 0, C.byref(n))
        buf = C.create_string_buffer(n.value)
        _check(lib().vc_commitment_export(self.ptr, codes[what], buf, n.value, C.byref(n)), "vc_commitment_export")
        return buf.raw


class Proofs(_Handle):
    _free = "vc_proofs_free"

    def __init__(self, ptr, pp, b):
        super().__init__(ptr)
        self.pp, self.b = pp, b
        self.nb = (pp.K + b - 1) // b

    def export(self, what: str, idx: int = 0) -> bytes:
        codes = {"fc_rounds": 0, "fc_tail": 1, "fc_x": 2, "merkle": 3, "rho": 4, "y": 5, "D": 6, "W": 7}
        n = C.c_size_t(0)
        lib().vc_proofs_export(self.ptr, codes[what], idx, None, 0, C.byref(n))
        buf = C.create_string_buffer(n.value)
        _check(lib().vc_proofs_export(self.ptr, codes[what], idx, buf, n.value, C.byref(n)), "vc_proofs_export")
        return buf.raw


def vc_setup(log_n: int, seed: bytes, device: int = 0) -> Params:
    out = C.c_void_p()
    _check(lib().vc_setup(log_n, seed, device, C.byref(out)), "vc_setup")
    return Params(out, log_n, device)


def vc_params_load(srs: bytes, device: int = 0) -> Params:
    """Parameters from an externally made SRS (the layout of Params.srs_bytes)."""
    out = C.c_void_p()
    _check(lib().vc_params_load(srs, len(srs), device, C.byref(out)), "vc_params_load")
    log_n = next(L for L in range(2, 31) if _srs_len(L) == len(srs))
    return Params(out, log_n, device)


def _srs_len(L: int) -> int:
    lK = L // 2
    lM = L - lK
    return 64 * (2 * (1 << lM) - 1) + 128 * lM + 128 * (2 * (1 << lK) - 1) + 64


def _check_entries(pp: Params, m, entry_bits: int) -> None:
    if m.numel() * m.element_size() < pp.N * (4 if entry_bits == 32 else 32):
        raise ValueError("the entry tensor holds fewer than N entries of %d bits" % entry_bits)


def vc_commit(pp: Params, m, entry_bits: int = 256, stream=None) -> Commitment:
    """m: a device tensor holding N x 32 little-endian bytes (entry_bits=256) or
    N 32-bit integers (entry_bits=32)."""
    _check_entries(pp, m, entry_bits)
    out = C.c_void_p()
    cbuf = C.create_string_buffer(384)
    _check(lib().vc_commit(pp.ptr, C.c_void_p(m.data_ptr()), pp.N, entry_bits, _stream_ptr(stream),
                           C.byref(out), cbuf), "vc_commit")
    return Commitment(out, pp, cbuf.raw)


def vc_commit_batch(jobs, ex=None, stream=None) -> list:
    """jobs: a list of (Params, device tensor of entries, entry_bits).  All commitments in fused
    launches; returns the Commitment of every job, in order."""
    n = len(jobs)
    VP = C.c_void_p
    for pp, m, bits in jobs:
        _check_entries(pp, m, bits)
    pps = (VP * max(n, 1))(*[pp.ptr for pp, _, _ in jobs])
    ms = (VP * max(n, 1))(*[m.data_ptr() for _, m, _ in jobs])
    bits = (C.c_uint32 * max(n, 1))(*[b for _, _, b in jobs])
    outs = (VP * max(n, 1))()
    Cb = C.create_string_buffer(384 * max(n, 1))
    _check(lib().vc_commit_batch(n, pps, ms, bits, ex.ptr if ex else None, _stream_ptr(stream), outs, Cb),
           "vc_commit_batch")
    return [Commitment(VP(outs[i]), jobs[i][0], Cb.raw[384 * i:384 * i + 384]) for i in range(n)]


def vc_tune_msm(lo: int, hi: int, path=None, device: int = 0) -> None:
    """Autotune the commit MSM's slice length for log2 N in [lo, hi] (and write the table)."""
    _check(lib().vc_tune_msm(device, lo, hi, path.encode() if path else None), "vc_tune_msm")


def vc_tune_load(path=None) -> None:
    """Load a tuned MSM schedule table (None: back to the default schedule)."""
    _check(lib().vc_tune_load(path.encode() if path else None), "vc_tune_load")


def vc_commit_noalloc(pp: Params, m, entry_bits: int, Cj_out, stream=None) -> bytes:
    """m as for vc_commit; Cj_out: a device uint8 tensor of K x 64 bytes that receives the
    encoded C_j.  Returns C (384 bytes)."""
    _check_entries(pp, m, entry_bits)
    if Cj_out.numel() * Cj_out.element_size() < 64 * pp.K:
        raise ValueError("Cj_out holds fewer than K x 64 bytes")
    cbuf = C.create_string_buffer(384)
    _check(lib().vc_commit_noalloc(pp.ptr, C.c_void_p(m.data_ptr()), pp.N, entry_bits, _stream_ptr(stream),
                                   C.c_void_p(Cj_out.data_ptr()), cbuf), "vc_commit_noalloc")
    return cbuf.raw


def vc_open_all(pp: Params, cm: Commitment, b: int, stream=None) -> Proofs:
    out = C.c_void_p()
    _check(lib().vc_open_all(pp.ptr, cm.ptr, b, _stream_ptr(stream), C.byref(out)), "vc_open_all")
    return Proofs(out, pp, b)


class Exec(_Handle):
    """Streams, events and workspace of one open-all job at a time."""
    _free = "vc_exec_free"

    def set_graphs(self, on: bool = True) -> None:
        """Capture and replay batched commits on this executor as HIP graphs."""
        _check(lib().vc_exec_set_graphs(self.ptr, 1 if on else 0), "vc_exec_set_graphs")

    def set_ahead(self, max_pairs: int) -> None:
        """Take Step 1's terms one round ahead while batches x K <= max_pairs (0: never)."""
        _check(lib().vc_exec_set_ahead(self.ptr, max_pairs), "vc_exec_set_ahead")

    def graph_stats(self) -> tuple:
        """(captures, replays) of batched-commit graphs on this executor."""
        st = (C.c_uint64 * 2)()
        _check(lib().vc_exec_graph_stats(self.ptr, st), "vc_exec_graph_stats")
        return int(st[0]), int(st[1])


def vc_exec_create(device: int = 0, nstreams: int = 6) -> Exec:
    out = C.c_void_p()
    _check(lib().vc_exec_create(device, nstreams, C.byref(out)), "vc_exec_create")
    return Exec(out)


def vc_open_all_ex(pp: Params, cm: Commitment, b: int, ex: Exec, stream=None) -> Proofs:
    out = C.c_void_p()
    _check(lib().vc_open_all_ex(pp.ptr, cm.ptr, b, ex.ptr, _stream_ptr(stream), C.byref(out)), "vc_open_all_ex")
    return Proofs(out, pp, b)


def vc_open_all_batch(jobs, execs) -> list:
    """jobs: a list of (Params, Commitment, b); execs: the executors that run them, one job
    at a time each.  Returns the Proofs of every job, in order."""
    n = len(jobs)
    VP = C.c_void_p
    pps = (VP * max(n, 1))(*[pp.ptr for pp, _, _ in jobs])
    cms = (VP * max(n, 1))(*[cm.ptr for _, cm, _ in jobs])
    bs = (C.c_uint32 * max(n, 1))(*[b for _, _, b in jobs])
    exs = (VP * max(len(execs), 1))(*[ex.ptr for ex in execs])
    outs = (VP * max(n, 1))()
    _check(lib().vc_open_all_batch(n, pps, cms, bs, len(execs), exs, outs), "vc_open_all_batch")
    return [Proofs(outs[i], jobs[i][0], jobs[i][2]) for i in range(n)]


def vc_open_all_grouped(jobs, execs, max_group: int) -> list:
    """As vc_open_all_batch, with the jobs on the same Params and b opened together in fused
    groups of at most max_group jobs."""
    n = len(jobs)
    VP = C.c_void_p
    pps = (VP * max(n, 1))(*[pp.ptr for pp, _, _ in jobs])
    cms = (VP * max(n, 1))(*[cm.ptr for _, cm, _ in jobs])
    bs = (C.c_uint32 * max(n, 1))(*[b for _, _, b in jobs])
    exs = (VP * max(len(execs), 1))(*[ex.ptr for ex in execs])
    outs = (VP * max(n, 1))()
    _check(lib().vc_open_all_grouped(n, pps, cms, bs, max_group, len(execs), exs, outs), "vc_open_all_grouped")
    return [Proofs(outs[i], jobs[i][0], jobs[i][2]) for i in range(n)]


def vc_open_all_footprint(pp: Params, b: int) -> int:
    n = C.c_uint64(0)
    _check(lib().vc_open_all_footprint(pp.ptr, b, C.byref(n)), "vc_open_all_footprint")
    return n.value


class Server(_Handle):
    """Serving loop: open-all requests queued in arrival order, run on a pool of executors
    under a device-memory budget."""
    _free = "vc_server_free"

    def __init__(self, ptr, device):
        super().__init__(ptr)
        self.device = device
        self._jobs = {}  # ticket -> (params, commitment, b), kept alive until collected

    def submit(self, pp: Params, cm: Commitment, b: int) -> int:
        t = C.c_uint64(0)
        _check(lib().vc_server_submit(self.ptr, pp.ptr, cm.ptr, b, C.byref(t)), "vc_server_submit")
        self._jobs[t.value] = (pp, cm, b)
        return t.value

    def stats(self):
        """(bytes held now, most bytes held at any time, budget)"""
        v = (C.c_uint64 * 3)()
        _check(lib().vc_server_stats(self.ptr, v), "vc_server_stats")
        return v[0], v[1], v[2]

    def wait(self, ticket: int):
        """(Proofs, [ms waiting before start, ms from submission to completion])"""
        out = C.c_void_p()
        times = (C.c_double * 2)()
        pp, cm, b = self._jobs.pop(ticket)
        _check(lib().vc_server_wait(self.ptr, ticket, C.byref(out), times), "vc_server_wait")
        return Proofs(out, pp, b), [times[0], times[1]]


def vc_server_create(device: int = 0, nexec: int = 16, nstreams: int = 1, hbm_budget: int = 64 << 30) -> Server:
    out = C.c_void_p()
    _check(lib().vc_server_create(device, nexec, nstreams, hbm_budget, C.byref(out)), "vc_server_create")
    return Server(out, device)


def vc_eval_proof(pp: Params, cm: Commitment, r: list, stream=None) -> bytes:
    """evaluation proof of f_m at r = [r_0, ..., r_{L-1}] (integers below the group order)"""
    cap = int(lib().vc_eval_proof_len(pp.log_n))
    buf = C.create_string_buffer(cap)
    n = C.c_size_t(0)
    rb = b"".join(int(x).to_bytes(32, "little") for x in r)
    if len(r) != pp.log_n:
        raise ValueError("the point has log N coordinates")
    _check(lib().vc_eval_proof(pp.ptr, cm.ptr, rb, _stream_ptr(stream), buf, cap, C.byref(n)), "vc_eval_proof")
    return buf.raw[:n.value]


def vc_verify_eval(pp: Params, C_bytes: bytes, r: list, proof: bytes) -> int:
    rb = b"".join(int(x).to_bytes(32, "little") for x in r)
    if len(r) != pp.log_n:
        raise ValueError("the point has log N coordinates")
    return _check(lib().vc_verify_eval(pp.ptr, C_bytes, rb, proof, len(proof)), "vc_verify_eval")


def vc_open_subarrays(pp: Params, cm: Commitment, b: int, stream=None) -> Proofs:
    out = C.c_void_p()
    _check(lib().vc_open_subarrays(pp.ptr, cm.ptr, b, _stream_ptr(stream), C.byref(out)), "vc_open_subarrays")
    return Proofs(out, pp, b)


def vc_subarray_proof_get(pr: Proofs, j: int) -> bytes:
    cap = int(lib().vc_subarray_proof_len(pr.pp.log_n, pr.b))
    buf = C.create_string_buffer(cap)
    n = C.c_size_t(0)
    _check(lib().vc_subarray_proof_get(pr.ptr, j, buf, cap, C.byref(n)), "vc_subarray_proof_get")
    return buf.raw[:n.value]


def vc_verify_subarray(pp: Params, C_bytes: bytes, b: int, j: int, m_j: bytes, proof: bytes) -> int:
    """m_j: the M entries of sub-array j, 32 little-endian bytes each."""
    return _check(lib().vc_verify_subarray(pp.ptr, C_bytes, b, j, m_j, proof, len(proof)), "vc_verify_subarray")


def vc_verify_subarrays_all(pp: Params, C_bytes: bytes, b: int, m, proofs):
    """m: device tensor of N x 32 little-endian bytes; proofs: device uint8 tensor holding the K
    sub-array proofs in order.  Returns (1 all accepted / 0, proofs checked by the verifier)."""
    ns = C.c_uint64(0)
    v = _check(lib().vc_verify_subarrays_all(pp.ptr, C_bytes, b, C.c_void_p(m.data_ptr()), C.c_void_p(proofs.data_ptr()),
                                             proofs.numel(), C.byref(ns)), "vc_verify_subarrays_all")
    return v, ns.value


def vc_proofs_serialize(pr: Proofs):
    """All N serialized proofs in index order, as one uint8 device tensor."""
    import torch
    n = C.c_uint64(0)
    _check(lib().vc_proofs_serialize(pr.ptr, None, 0, C.byref(n)), "vc_proofs_serialize")
    out = torch.empty(n.value, dtype=torch.uint8, device="cuda:%d" % pr.pp.device)
    _check(lib().vc_proofs_serialize(pr.ptr, C.c_void_p(out.data_ptr()), n.value, C.byref(n)), "vc_proofs_serialize")
    return out


def proof_offsets(pp: Params, b: int) -> list:
    """Byte offset of every proof in the serialized layout (N + 1 entries)."""
    K, M = pp.K, pp.M
    nb = (K + b - 1) // b
    offs, o = [0], 0
    for k in range(nb):
        ln = vc_proof_len(pp.log_n, min(b, K - k * b))
        for _ in range(min(b, K - k * b) * M):
            o += ln
            offs.append(o)
    return offs


def vc_verify_all(pp: Params, C_bytes: bytes, b: int, m, proofs, seed: bytes):
    """m: device tensor of N x 32 little-endian bytes; proofs: device tensor from
    vc_proofs_serialize (or the same layout).  Returns (1 all accepted / 0, proofs checked alone)."""
    ns = C.c_uint64(0)
    v = _check(lib().vc_verify_all(pp.ptr, C_bytes, b, C.c_void_p(m.data_ptr()), C.c_void_p(proofs.data_ptr()),
                                   proofs.numel(), seed, C.byref(ns)), "vc_verify_all")
    return v, ns.value


def vc_proof_len(log_n: int, t: int) -> int:
    return int(lib().vc_proof_len(log_n, t))


def vc_proof_get(pr: Proofs, i: int) -> bytes:
    cap = vc_proof_len(pr.pp.log_n, pr.b)
    buf = C.create_string_buffer(cap)
    n = C.c_size_t(0)
    _check(lib().vc_proof_get(pr.ptr, i, buf, cap, C.byref(n)), "vc_proof_get")
    return buf.raw[:n.value]


def vc_verify(pp: Params, C_bytes: bytes, b: int, i: int, m_i: int, proof: bytes) -> int:
    return _check(lib().vc_verify(pp.ptr, C_bytes, pp.N, b, i, int(m_i).to_bytes(32, "little"), proof, len(proof)),
                  "vc_verify")


def vc_diag_fold(cm) -> float:
    """Milliseconds of the y-tree passes over cm's entries, alone on the device."""
    ms = C.c_double(0)
    _check(lib().vc_diag_fold(cm.ptr, C.byref(ms)), "vc_diag_fold")
    return ms.value


def vc_diag_mad_rate(device: int = 0) -> float:
    """measured 32 x 32 -> 64-bit multiply-add throughput of the device (10^12 per second)"""
    r = C.c_double(0)
    _check(lib().vc_diag_mad_rate(device, C.byref(r)), "vc_diag_mad_rate")
    return r.value


def vc_profile_enable(on: bool = True) -> None:
    lib().vc_profile_enable(1 if on else 0)


def vc_test_zero_challenge(round_: int) -> None:
    """Test hook: later open-alls force batch 0's challenge x_round to zero and fail with
    VC_ECHALLENGE (0 turns it off)."""
    lib().vc_test_zero_challenge(round_)


def vc_profile_only(kernel=None) -> None:
    """Restrict profiling to launches of one kernel (None: every kernel)."""
    lib().vc_profile_only(kernel.encode() if kernel else None)


def vc_profile_read() -> dict:
    """{kernel name: (launches, total_ms)} for launches since vc_profile_enable(True)."""
    n = lib().vc_profile_read(None, 0)
    buf = C.create_string_buffer(n)
    lib().vc_profile_read(buf, n)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.rsplit(" ", 2)
        out[name] = (int(cnt), float(ms))
    return out
