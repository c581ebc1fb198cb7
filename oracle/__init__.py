"""FlexProofs CPU oracle (plain C, BN254) -- ctypes wrapper.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously-correct reference the
GPU library is checked against; only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it.  It shares no code with the GPU
library (``paper_2601_03031_amd``) and imports nothing from it.

The C sources follow the paper's algorithms: FC.Setup/Commit/BOpen/BVerify
(section 3), VC.Setup/Commit (section 4.1, Eq. vcpp, genCi, genC), OpenAll
(section 4.2, Protocol 1 and its Sub-protocol, made non-interactive with a Merkle
tree) and the verifier of the correctness proof (appendix C).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["field.c", "curve.c", "hash.c", "flexproofs.c", "api.c"]

P = 0x30644E72E131A029B85045B68181585D97816A916871CA8D3C208C16D87CFD47
R = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP over independent units)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O3", "-std=gnu11", "-fPIC", "-fopenmp", "-fvisibility=hidden", "-shared",
           "-Wall", "-o", LIB_PATH + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, u8p, u64, u32 = C.c_void_p, C.c_char_p, C.c_uint64, C.c_uint32
        L.or_setup.restype = vp
        L.or_setup.argtypes = [u32, u8p]
        L.or_params_free.argtypes = [vp]
        L.or_params_export.argtypes = [vp, C.c_int, u32, C.c_void_p]
        L.or_commit.restype = vp
        L.or_commit.argtypes = [vp, u8p, u64]
        L.or_commit_free.argtypes = [vp]
        L.or_commit_export.argtypes = [vp, C.c_void_p, C.c_void_p]
        L.or_open_all.restype = vp
        L.or_open_all.argtypes = [vp, u32]
        L.or_open_free.argtypes = [vp]
        L.or_open_export.argtypes = [vp, C.c_int, u64, C.c_void_p]
        L.or_proof_len.restype = u64
        L.or_proof_len.argtypes = [u32, u32]
        L.or_proof.argtypes = [vp, u64, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.or_verify.argtypes = [vp, u8p, u64, u32, u64, u8p, u8p, C.c_size_t]
        L.or_open_blocks.argtypes = [vp, u32, C.POINTER(C.c_uint64), u64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_naive_proof.argtypes = [vp, u8p, u64, u32, u64, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.or_two_step_pst.argtypes = [vp, u64, C.c_void_p, C.c_void_p]
        L.or_eval_proof_len.restype = u64
        L.or_eval_proof_len.argtypes = [u32]
        L.or_eval_proof.argtypes = [vp, u8p, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.or_eval_verify.argtypes = [vp, u8p, u8p, u8p, C.c_size_t]
        L.or_pst_commit.argtypes = [vp, u8p, C.c_void_p]
        L.or_two_step_fc.argtypes = [vp, u64]
        L.or_fc_roundtrip.argtypes = [vp, C.POINTER(C.c_uint64), u32, C.c_int]
        L.or_set_invariant_check.argtypes = [C.c_int]
        L.or_invariant_checks.restype = C.c_long
        L.or_invariant_failures.restype = C.c_long
        L.or_field_op.argtypes = [C.c_int, C.c_int, u8p, u8p, C.c_void_p]
        L.or_fp2_op.argtypes = [C.c_int, u8p, u8p, C.c_void_p]
        L.or_fp12_op.argtypes = [C.c_int, u8p, u8p, C.c_void_p]
        L.or_g1_op.argtypes = [C.c_int, u8p, u8p, C.c_void_p]
        L.or_g2_op.argtypes = [C.c_int, u8p, u8p, C.c_void_p]
        L.or_g1_check.argtypes = [u8p]
        L.or_g2_check.argtypes = [u8p]
        L.or_generators.argtypes = [C.c_void_p, C.c_void_p]
        L.or_pairing.argtypes = [u8p, u8p, u64, C.c_void_p]
        L.or_compress.argtypes = [C.c_int, u8p, C.c_void_p]
        L.or_sha256.argtypes = [u8p, u64, C.c_void_p]
        L.or_xmd.argtypes = [u8p, u64, u8p, u64, C.c_void_p, u64]
        L.or_h2f.argtypes = [u8p, u8p, u64, C.c_void_p]
        L.or_init_api()
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle uses for its independent units."""
    os.environ["OMP_NUM_THREADS"] = str(n)
    try:
        gomp = C.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(C.c_int(n))
    except OSError:
        pass


def max_threads() -> int:
    try:
        gomp = C.CDLL("libgomp.so.1")
        return int(gomp.omp_get_max_threads())
    except OSError:
        return 1


def _buf(n: int):
    return C.create_string_buffer(n)


def be32(x: int) -> bytes:
    return int(x).to_bytes(32, "big")


def le32(x: int) -> bytes:
    return int(x).to_bytes(32, "little")


# ----------------------------------------------------------------- primitives
def field_op(which: str, op: str, a: int, b: int = 0):
    ops = {"add": 0, "sub": 1, "mul": 2, "inv": 3, "neg": 4, "sqrt": 5}
    out = _buf(32)
    rc = lib().or_field_op(1 if which == "r" else 0, ops[op], be32(a), be32(b), out)
    if rc < 0:
        raise ValueError("bad field input")
    val = int.from_bytes(out.raw, "big")
    return (val, rc == 1) if op == "sqrt" else val


def fp2_op(op: str, a: tuple, b: tuple = (0, 0)):
    ops = {"mul": 0, "inv": 1, "sqrt": 2}
    out = _buf(64)
    rc = lib().or_fp2_op(ops[op], be32(a[0]) + be32(a[1]), be32(b[0]) + be32(b[1]), out)
    if rc < 0:
        raise ValueError("bad fp2 input")
    v = (int.from_bytes(out.raw[:32], "big"), int.from_bytes(out.raw[32:], "big"))
    return (v, rc == 1) if op == "sqrt" else v


def fp12_op(op: str, a: bytes, b: bytes = bytes(384)) -> bytes:
    ops = {"mul": 0, "inv": 1, "final_exp": 2, "pow": 3}
    out = _buf(384)
    if len(b) < 384:
        b = b + bytes(384 - len(b))
    if lib().or_fp12_op(ops[op], a, b, out) < 0:
        raise ValueError("bad fp12 input")
    return out.raw


def g1_op(op: str, P: bytes, Q: bytes = bytes(64)) -> bytes:
    ops = {"add": 0, "mul": 1, "neg": 2, "mul_int": 3}
    out = _buf(64)
    if len(Q) < 64:
        Q = Q + bytes(64 - len(Q))
    if lib().or_g1_op(ops[op], P, Q, out) < 0:
        raise ValueError("bad g1 input")
    return out.raw


def g2_op(op: str, P: bytes, Q: bytes = bytes(128)) -> bytes:
    ops = {"add": 0, "mul": 1, "neg": 2, "frobenius": 3, "mul_int": 4}
    out = _buf(128)
    if len(Q) < 128:
        Q = Q + bytes(128 - len(Q))
    if lib().or_g2_op(ops[op], P, Q, out) < 0:
        raise ValueError("bad g2 input")
    return out.raw


def g1_valid(P: bytes) -> bool:
    return bool(lib().or_g1_check(P))


def g2_valid(P: bytes) -> bool:
    return bool(lib().or_g2_check(P))


def generators():
    a, b = _buf(64), _buf(128)
    lib().or_generators(a, b)
    return a.raw, b.raw


def pairing(Ps, Qs) -> bytes:
    """prod_i e(P_i, Q_i) for lists of 64-byte G1 and 128-byte G2 encodings."""
    out = _buf(384)
    if lib().or_pairing(b"".join(Ps), b"".join(Qs), len(Ps), out) < 0:
        raise ValueError("bad pairing input")
    return out.raw


def compress(kind: int, data: bytes) -> bytes:
    n = {1: 32, 2: 64, -1: 64, -2: 128}[kind]
    out = _buf(n)
    if lib().or_compress(kind, data, out) < 0:
        raise ValueError("bad point encoding")
    return out.raw


def sha256(msg: bytes) -> bytes:
    out = _buf(32)
    lib().or_sha256(msg, len(msg), out)
    return out.raw


def expand_message_xmd(msg: bytes, dst: bytes, n: int) -> bytes:
    out = _buf(n)
    lib().or_xmd(msg, len(msg), dst, len(dst), out, n)
    return out.raw


def hash_to_fr(dst: str, msg: bytes) -> int:
    out = _buf(32)
    lib().or_h2f(dst.encode(), msg, len(msg), out)
    return int.from_bytes(out.raw, "big")


GT_ONE = (1).to_bytes(32, "big") + bytes(352)


# ----------------------------------------------------------------- scheme
def proof_len(log_n: int, t: int) -> int:
    return int(lib().or_proof_len(log_n, t))


class Params:
    """VC.Setup with a seeded test trapdoor."""

    def __init__(self, log_n: int, seed: bytes):
        assert len(seed) == 32
        self.log_n = log_n
        self.lK = log_n // 2
        self.lM = log_n - self.lK
        self.N, self.K, self.M = 1 << log_n, 1 << self.lK, 1 << self.lM
        self.h = lib().or_setup(log_n, seed)
        if not self.h:
            raise ValueError("setup failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_params_free(self.h)
            self.h = None

    def export(self, what: str, idx: int = 0) -> bytes:
        codes = {"ek": 0, "vk": 1, "h": 2, "g1beta": 3, "trapdoor": 4}
        sizes = {"ek": 64 << idx, "vk": 128 * self.lM, "h": 128 * (2 * self.K - 1), "g1beta": 64,
                 "trapdoor": 32 * (self.lM + 1)}
        out = _buf(sizes[what])
        if lib().or_params_export(self.h, codes[what], idx, out) < 0:
            raise ValueError(what)
        return out.raw


class Commitment:
    def __init__(self, pp: Params, m_le: bytes):
        self.pp = pp
        self.m_le = m_le
        self.h = lib().or_commit(pp.h, m_le, len(m_le) // 32)
        if not self.h:
            raise ValueError("commit failed (size or entry >= r)")
        cj, c = _buf(64 * pp.K), _buf(384)
        lib().or_commit_export(self.h, cj, c)
        self.Cj = [cj.raw[64 * j:64 * j + 64] for j in range(pp.K)]
        self.C = c.raw

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_commit_free(self.h)
            self.h = None

    def eval_proof(self, r: list) -> bytes:
        """evaluation proof of f_m at r = [r_0, ..., r_{L-1}] (section 4.3)"""
        cap = eval_proof_len(self.pp.log_n)
        out, ln = _buf(cap), C.c_size_t(0)
        if lib().or_eval_proof(self.h, b"".join(le32(x) for x in r), out, cap, C.byref(ln)) < 0:
            raise ValueError("eval proof")
        return out.raw[:ln.value]

    def open_blocks(self, b: int, ks) -> list:
        """Step 1 of OpenAll(b) for blocks ks only: per block the byte strings of
        Opening.export's "fc_rounds", "fc_tail" and "fc_x"."""
        ks = [int(k) for k in ks]
        lK, n = self.pp.lK, len(ks)
        arr = (C.c_uint64 * n)(*ks)
        rounds, tail, xs = _buf(896 * lK * n), _buf(320 * n), _buf(32 * lK * n)
        rc = lib().or_open_blocks(self.h, b, arr, n, rounds, tail, xs)
        if rc < 0:
            raise ValueError("open_blocks rc=%d" % rc)
        out = []
        for q in range(n):
            out.append({"fc_rounds": rounds.raw[896 * lK * q:896 * lK * (q + 1)],
                        "fc_tail": tail.raw[320 * q:320 * (q + 1)],
                        "fc_x": xs.raw[32 * lK * q:32 * lK * (q + 1)]})
        return out

    def two_step_pst(self, i: int):
        w, y = _buf(64 * self.pp.lM), _buf(32)
        ok = lib().or_two_step_pst(self.h, i, w, y)
        return [w.raw[64 * d:64 * d + 64] for d in range(self.pp.lM)], int.from_bytes(y.raw, "big"), ok == 1

    def two_step_fc(self, j: int) -> bool:
        return lib().or_two_step_fc(self.h, j) == 1

    def fc_roundtrip(self, idx, bad_slot: int = -1) -> int:
        arr = (C.c_uint64 * len(idx))(*idx)
        return int(lib().or_fc_roundtrip(self.h, arr, len(idx), bad_slot))


class Opening:
    def __init__(self, cm: Commitment, b: int):
        self.cm, self.pp, self.b = cm, cm.pp, b
        self.h = lib().or_open_all(cm.h, b)
        if not self.h:
            raise ValueError("open_all failed")
        self.nb = (self.pp.K + b - 1) // b

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_open_free(self.h)
            self.h = None

    def export(self, what: str, idx: int = 0) -> bytes:
        pp = self.pp
        codes = {"fc_rounds": 0, "fc_tail": 1, "fc_x": 2, "merkle": 3, "rho": 4, "y": 5, "D": 6, "W": 7}
        sizes = {"fc_rounds": 896 * pp.lK, "fc_tail": 320, "fc_x": 32 * pp.lK, "merkle": 64 * pp.N,
                 "rho": 32 * pp.K, "y": 32 * (2 * pp.K - 1) * pp.M, "D": 64 * (2 * pp.K - 1),
                 "W": 64 * (pp.M - 1)}
        out = _buf(sizes[what])
        if lib().or_open_export(self.h, codes[what], idx, out) < 0:
            raise ValueError(what)
        return out.raw

    def proof(self, i: int) -> bytes:
        cap = proof_len(self.pp.log_n, self.b)
        out, ln = _buf(cap), C.c_size_t(0)
        if lib().or_proof(self.h, i, out, cap, C.byref(ln)) < 0:
            raise ValueError("proof")
        return out.raw[:ln.value]


def verify(pp: Params, C_gt: bytes, b: int, i: int, m_i: int, proof: bytes) -> int:
    return int(lib().or_verify(pp.h, C_gt, pp.N, b, i, le32(m_i), proof, len(proof)))


def eval_proof_len(log_n: int) -> int:
    return int(lib().or_eval_proof_len(log_n))


def eval_verify(pp: Params, C_gt: bytes, r: list, proof: bytes) -> int:
    return int(lib().or_eval_verify(pp.h, C_gt, b"".join(le32(x) for x in r), proof, len(proof)))


def pst_commit(pp: Params, table: list) -> bytes:
    """PST commitment (x || y, 64 bytes) of a table of M values with ek_{lM}"""
    out = _buf(64)
    if lib().or_pst_commit(pp.h, b"".join(le32(x) for x in table), out) < 0:
        raise ValueError("pst commit")
    return out.raw


def naive_proof(pp: Params, m_le: bytes, b: int, i: int) -> bytes:
    cap = proof_len(pp.log_n, b)
    out, ln = _buf(cap), C.c_size_t(0)
    if lib().or_naive_proof(pp.h, m_le, pp.N, b, i, out, cap, C.byref(ln)) < 0:
        raise ValueError("naive proof")
    return out.raw[:ln.value]


def set_invariant_check(on: bool) -> None:
    lib().or_set_invariant_check(1 if on else 0)


def invariant_counts():
    return int(lib().or_invariant_checks()), int(lib().or_invariant_failures())
