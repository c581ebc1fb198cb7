"""OpenAll for consecutive sub-arrays: Step 1 alone.  Each sub-array proof equals the first
part of the full proof (and the oracle's), and vc_verify_subarray accepts exactly the honest
sub-arrays."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2601_03031_amd import inputs as I

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SEED = I.TRAPDOOR_SEED


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


def dev_entries(limbs, bits):
    if bits == 32:
        return torch.from_numpy(limbs[:, 0].astype(np.uint32).view(np.int32).copy()).cuda()
    return torch.from_numpy(np.ascontiguousarray(limbs).view(np.uint8).reshape(-1).copy()).cuda()


def flip(b: bytes, pos: int, mask: int = 1) -> bytes:
    a = bytearray(b)
    a[pos] ^= mask
    return bytes(a)


@pytest.mark.parametrize("L,b,bits,seed", [(6, 3, 32, 81), (7, 1, 256, 82), (8, 16, 32, 83)])
def test_subarrays_match_and_verify(vc, L, b, bits, seed):
    say("sub-arrays L=%d b=%d bits=%d" % (L, b, bits))
    limbs = I.entries(1 << L, seed, bits)
    ints = I.limbs_to_ints(limbs)
    m_le = I.limbs_to_bytes(limbs)
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(limbs, bits), bits)
    sub = vc.vc_open_subarrays(pp, cm, b)
    full = vc.vc_open_all(pp, cm, b)
    opp = O.Params(L, SEED)
    oop = O.Opening(O.Commitment(opp, m_le), b)
    K, M = pp.K, pp.M
    for j in range(K):
        p = vc.vc_subarray_proof_get(sub, j)
        t = min(b, K - (j // b) * b)
        assert len(p) == vc.lib().vc_subarray_proof_len(L, t)
        assert p == vc.vc_subarray_proof_get(full, j), j
        assert p == vc.vc_proof_get(full, j * M)[:len(p)], j
        assert p == oop.proof(j * M)[:len(p)], j
        mj = m_le[32 * M * j: 32 * M * (j + 1)]
        assert vc.vc_verify_subarray(pp, cm.C, b, j, mj, p) == 1, j
    # FC exports agree; Step 2 is absent
    for k in range((K + b - 1) // b):
        for w in ("fc_x", "fc_rounds", "fc_tail"):
            assert sub.export(w, k) == full.export(w, k), (w, k)
    for w in ("merkle", "y", "W"):
        with pytest.raises(vc.VCError) as e:
            sub.export(w)
        assert e.value.code == vc.VC_EINVAL
    with pytest.raises(vc.VCError) as e:
        vc.vc_proof_get(sub, 0)
    assert e.value.code == vc.VC_EINVAL
    # rejections (the oracle's verifier rejects the same alterations in full proofs)
    j = K - 1
    p = vc.vc_subarray_proof_get(sub, j)
    mj = m_le[32 * M * j: 32 * M * (j + 1)]
    i = j * M + 1
    bad_m = flip(mj, 32 * 1)  # entry j M + 1, low byte
    assert vc.vc_verify_subarray(pp, cm.C, b, j, bad_m, p) == 0
    assert O.verify(opp, cm.C, b, i, ints[i] ^ 1, oop.proof(i)) == 0
    if j >= 1:
        prev = m_le[32 * M * (j - 1): 32 * M * j]
        assert vc.vc_verify_subarray(pp, cm.C, b, j, prev, p) == 0  # another sub-array under j
    t = min(b, K - (j // b) * b)
    fc_byte = 32 * t + 31  # round 1, first G_T coefficient
    assert vc.vc_verify_subarray(pp, cm.C, b, j, mj, flip(p, fc_byte)) == 0
    assert O.verify(opp, cm.C, b, i, ints[i], flip(oop.proof(i), fc_byte)) == 0
    if t > 1:
        other = (j - (j // b) * b + 1) % t  # another entry of the block
        blk_byte = 32 * other + 5
        assert vc.vc_verify_subarray(pp, cm.C, b, j, mj, flip(p, blk_byte, 0x04)) == 0
        assert O.verify(opp, cm.C, b, i, ints[i], flip(oop.proof(i), blk_byte, 0x04)) == 0
    with pytest.raises(vc.VCError) as e:
        vc.vc_verify_subarray(pp, cm.C, b, j, mj, p[:-1])
    assert e.value.code == vc.VC_EINVAL


def test_subarrays_n16_b256(vc):
    L, b = 16, 256
    limbs = I.entries(1 << L, 2, 32)
    m_le = I.limbs_to_bytes(limbs)
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(limbs, 32), 32)
    sub = vc.vc_open_subarrays(pp, cm, b)
    full = vc.vc_open_all(pp, cm, b)
    M = pp.M
    for j in (0, 1, 128, 255):
        p = vc.vc_subarray_proof_get(sub, j)
        assert p == vc.vc_proof_get(full, j * M)[:len(p)], j
        assert vc.vc_verify_subarray(pp, cm.C, b, j, m_le[32 * M * j: 32 * M * (j + 1)], p) == 1, j


def _subarray_set(vc, sub, K):
    return b"".join(vc.vc_subarray_proof_get(sub, j) for j in range(K))


def _dev(b: bytes):
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).cuda()


def test_verify_subarrays_all(vc):
    L, b = 7, 3  # K = 8: batches of 3, 3, 2
    limbs = I.entries(1 << L, 84, 256)
    m_le = I.limbs_to_bytes(limbs)
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(limbs, 256), 256)
    sub = vc.vc_open_subarrays(pp, cm, b)
    K, M = pp.K, pp.M
    blob = _subarray_set(vc, sub, K)
    offs = [0]
    for j in range(K):
        offs.append(offs[-1] + len(vc.vc_subarray_proof_get(sub, j)))
    m = _dev(m_le)
    v, ns = vc.vc_verify_subarrays_all(pp, cm.C, b, m, _dev(blob))
    say("  sub-arrays all: %d (%d checked by the verifier)" % (v, ns))
    assert v == 1 and ns == 3

    def flip(data, pos, mask=1):
        a = bytearray(data)
        a[pos] ^= mask
        return bytes(a)

    # an entry of sub-array 4: its recomputed C_4 is not in the block
    assert vc.vc_verify_subarrays_all(pp, cm.C, b, _dev(flip(m_le, 32 * (4 * M + 2))), _dev(blob))[0] == 0
    # the FC proof of sub-array 4 alone (not its batch's first): checked by the verifier, rejected
    fc_byte = 32 * 3 + 31
    v, ns = vc.vc_verify_subarrays_all(pp, cm.C, b, m, _dev(flip(blob, offs[4] + fc_byte)))
    assert v == 0 and ns == 4
    opp = O.Params(L, SEED)
    oop = O.Opening(O.Commitment(opp, m_le), b)
    i = 4 * M
    assert O.verify(opp, cm.C, b, i, I.limbs_to_ints(limbs)[i], flip(oop.proof(i), fc_byte)) == 0
    # the FC proof of batch 1 in all its proofs (3, 4, 5): its first proof is rejected
    bad = blob
    for j in (3, 4, 5):
        bad = flip(bad, offs[j] + fc_byte)
    assert vc.vc_verify_subarrays_all(pp, cm.C, b, m, _dev(bad))[0] == 0
    # entry 5 of the block in proof 5 only
    assert vc.vc_verify_subarrays_all(pp, cm.C, b, m, _dev(flip(blob, offs[5] + 32 * 2 + 5, 0x04)))[0] == 0
    with pytest.raises(vc.VCError) as e:
        vc.vc_verify_subarrays_all(pp, cm.C, b, m, _dev(blob[:-32]))
    assert e.value.code == vc.VC_EINVAL


def test_verify_subarrays_all_n16_b256(vc):
    L, b = 16, 256
    limbs = I.entries(1 << L, 2, 32)
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(limbs, 32), 32)
    sub = vc.vc_open_subarrays(pp, cm, b)
    v, ns = vc.vc_verify_subarrays_all(pp, cm.C, b, _dev(I.limbs_to_bytes(limbs)), _dev(_subarray_set(vc, sub, pp.K)))
    assert v == 1 and ns == 1
