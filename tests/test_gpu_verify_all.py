"""Every proof at once: device serialization of all N proofs equals vc_proof_get's bytes, and
vc_verify_all accepts exactly when every proof is valid (the oracle's one-proof verifier
decides the tampered ones)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2601_03031_amd import inputs as I

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SEED = I.TRAPDOOR_SEED
VSEED = bytes(range(32))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_03031_amd as V
    V.lib()
    return V


def dev_u32(v):
    return torch.from_numpy(v.astype(np.uint32).view(np.int32).copy()).cuda()


def dev_bytes(b: bytes):
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).cuda()


class Job:
    def __init__(self, V, L, b, seed, bits=32, zero=False):
        say("job L=%d b=%d seed=%d bits=%d zero=%s" % (L, b, seed, bits, zero))
        N = 1 << L
        self.L, self.b = L, b
        self.limbs = np.zeros((N, 4), dtype=np.uint64) if zero else I.entries(N, seed, bits)
        self.ints = I.limbs_to_ints(self.limbs)
        self.pp = V.vc_setup(L, SEED, 0)
        if bits == 32:
            self.cm = V.vc_commit(self.pp, dev_u32(self.limbs[:, 0]), 32)
        else:
            self.cm = V.vc_commit(self.pp, dev_bytes(I.limbs_to_bytes(self.limbs)), 256)
        self.pr = V.vc_open_all(self.pp, self.cm, b)
        self.ser = V.vc_proofs_serialize(self.pr)
        self.offs = V.proof_offsets(self.pp, b)
        self.m = dev_bytes(I.limbs_to_bytes(self.limbs))
        assert self.ser.numel() == self.offs[-1]

    def proof(self, i, data=None):
        src = self.ser if data is None else data
        return bytes(src[self.offs[i]:self.offs[i + 1]].cpu().numpy())

    def layout(self, i):
        """byte offsets inside proof i: (t, start of the Step 2 part)"""
        K, M, lK = self.pp.K, self.pp.M, self.pp.lK
        k = i // (self.b * M)
        t = min(self.b, K - k * self.b)
        return t, 32 * t + 832 * lK + 160


def test_serialize_matches_proof_get(vc):
    for L, b, seed in ((6, 3, 51), (7, 2, 52), (10, 4, 53)):
        jb = Job(vc, L, b, seed)
        N = 1 << L
        idx = range(N) if L <= 7 else sorted({0, 1, 31, 32, 33, 500, 511, 512, 513, N - 1})
        for i in idx:
            assert jb.proof(i) == vc.vc_proof_get(jb.pr, i), (L, b, i)


def test_verify_all_accepts(vc):
    for L, b, seed, bits, zero in ((6, 3, 61, 32, False), (7, 1, 62, 256, False), (10, 4, 63, 32, False),
                                   (6, 8, 0, 32, True)):
        jb = Job(vc, L, b, seed, bits, zero)
        v, ns = vc.vc_verify_all(jb.pp, jb.cm.C, b, jb.m, jb.ser, VSEED)
        nb = (jb.pp.K + b - 1) // b
        say("  verify_all = %d, %d checked alone (batches %d)" % (v, ns, nb))
        assert v == 1 and ns == nb


def tampered(jb, edits):
    """copy of the serialized proofs with (proof, byte offset, xor mask) edits"""
    d = jb.ser.clone()
    for i, off, mask in edits:
        q = jb.offs[i] + off
        d[q] = int(d[q].item()) ^ mask
    return d


def test_verify_all_rejects(vc):
    jb = Job(vc, 6, 3, 71)
    pp, K, M, lK, lM = jb.pp, jb.pp.K, jb.pp.M, jb.pp.lK, jb.pp.lM
    O_pp = O.Params(6, SEED)

    def check(data, m=None, bad=(), label=""):
        v, ns = vc.vc_verify_all(pp, jb.cm.C, jb.b, jb.m if m is None else m, data, VSEED)
        say("  %s: verify_all = %d (%d checked alone)" % (label, v, ns))
        assert v == 0, label
        # the oracle rejects the altered proofs
        for i, mi in bad:
            assert O.verify(O_pp, jb.cm.C, jb.b, i, mi, jb.proof(i, data)) == 0, (label, i)

    i = 13  # batch 0, subvector 1: represents nothing
    t, s2 = jb.layout(i)
    # 1. a y sibling of one proof (stays < r): only the combined check sees it
    check(tampered(jb, [(i, s2 + 32 + 31, 1)]), bad=[(i, jb.ints[i])], label="y sibling")
    # 2. a wrong entry given to the verifier: its Merkle root differs, it is checked alone
    m2 = jb.m.clone()
    m2[32 * i] ^= 1
    check(jb.ser, m=m2, bad=[], label="entry")
    assert O.verify(O_pp, jb.cm.C, jb.b, i, jb.ints[i] ^ 1, jb.proof(i)) == 0
    # 3. W of depth 1 replaced, in every proof that carries it, by another valid point
    #    (the same proof's W of depth 0): consistent, so only the combined check sees it
    edits = []
    for q in range(pp.N):
        a = q % M
        if a >> (lM - 1) == 1:
            tq, sq = jb.layout(q)
            w0 = jb.proof(q)[sq + 64 * lK: sq + 64 * lK + 32]
            w1 = jb.proof(q)[sq + 64 * lK + 32: sq + 64 * lK + 64]
            edits += [(q, sq + 64 * lK + 32 + z, w0[z] ^ w1[z]) for z in range(32) if w0[z] != w1[z]]
    d3 = tampered(jb, edits)
    check(d3, bad=[(M // 2, jb.ints[M // 2])], label="W group")
    # 4. a D-tree sibling of one proof: it differs from its representative, checked alone
    check(tampered(jb, [(i, s2 + 5, 0x10)]), bad=[(i, jb.ints[i])], label="D sibling")
    # 5. the FC proof of batch 1 (a G_T coefficient of round 1) in every proof of the batch
    lo, hi = 3 * M, 6 * M
    tb, _ = jb.layout(lo)
    d5 = tampered(jb, [(q, 32 * tb + 31, 1) for q in range(lo, hi)])
    check(d5, bad=[(lo, jb.ints[lo])], label="FC proof of a batch")
    # 6. the block of one proof (not the batch's representative): checked alone
    check(tampered(jb, [(i, 7, 0x01)]), bad=[(i, jb.ints[i])], label="block of one proof")
    # the untouched set is still accepted
    assert vc.vc_verify_all(pp, jb.cm.C, jb.b, jb.m, jb.ser, VSEED)[0] == 1


def test_verify_all_n16_b256(vc):
    """the benchmark workload: all 2^16 proofs (1.07 GB serialized)"""
    jb = Job(vc, 16, 256, 2, 32)
    v, ns = vc.vc_verify_all(jb.pp, jb.cm.C, 256, jb.m, jb.ser, VSEED)
    say("  2^16: verify_all = %d, %d checked alone" % (v, ns))
    assert v == 1 and ns == 1
    for i in (0, 1, 255, 256, 40000, (1 << 16) - 1):
        assert jb.proof(i) == vc.vc_proof_get(jb.pr, i), i
    d = tampered(jb, [(40000, jb.layout(40000)[1] + 32 + 31, 1)])
    assert vc.vc_verify_all(jb.pp, jb.cm.C, 256, jb.m, d, VSEED)[0] == 0
