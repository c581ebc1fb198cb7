"""Evaluation proof at a point (section 4.3): the HIP path's bytes equal the oracle's, and the
oracle's verifier accepts them."""
import random
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


@pytest.mark.parametrize("L,bits,seed", [(4, 256, 101), (5, 32, 102), (6, 256, 103), (11, 32, 104), (16, 32, 2)])
def test_eval_proof_matches_oracle(vc, L, bits, seed):
    say("eval proof L=%d bits=%d" % (L, bits))
    limbs = I.entries(1 << L, seed, bits)
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(limbs, bits), bits)
    opp = O.Params(L, SEED)
    ocm = O.Commitment(opp, I.limbs_to_bytes(limbs))
    rng = random.Random(seed)
    points = [[rng.randrange(O.R) for _ in range(L)], [rng.randrange(2) for _ in range(L)],
              [0] * L, [O.R - 1] + [1] * (L - 1)]
    if L > 11:
        points = points[:1]
    for r in points:
        p = vc.vc_eval_proof(pp, cm, r)
        assert len(p) == O.eval_proof_len(L)
        assert p == ocm.eval_proof(r), r[:2]
        assert O.eval_verify(opp, cm.C, r, p) == 1
    say("  equal at %d points" % len(points))


def test_eval_proof_rejects_bad_point(vc):
    L = 5
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(I.entries(1 << L, 105, 32), 32), 32)
    with pytest.raises(vc.VCError) as e:
        vc.vc_eval_proof(pp, cm, [O.R] + [0] * (L - 1))
    assert e.value.code == vc.VC_EINVAL
    # the library stays usable
    r = [3] * L
    opp = O.Params(L, SEED)
    assert O.eval_verify(opp, cm.C, r, vc.vc_eval_proof(pp, cm, r)) == 1


@pytest.mark.parametrize("L,seed", [(5, 111), (6, 112), (10, 113)])
def test_verify_eval_matches_oracle(vc, L, seed):
    say("verify eval L=%d" % L)
    limbs = I.entries(1 << L, seed, 256)
    pp = vc.vc_setup(L, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(limbs, 256), 256)
    opp = O.Params(L, SEED)
    rng = random.Random(seed)
    r = [rng.randrange(O.R) for _ in range(L)]
    p = vc.vc_eval_proof(pp, cm, r)
    assert vc.vc_verify_eval(pp, cm.C, r, p) == 1
    rb = [rng.randrange(2) for _ in range(L)]
    assert vc.vc_verify_eval(pp, cm.C, rb, vc.vc_eval_proof(pp, cm, rb)) == 1
    lK, lM = L // 2, L - L // 2
    y_off = 32 + 832 * lK + 160

    def flip(pos, mask=1):
        a = bytearray(p)
        a[pos] ^= mask
        return bytes(a)

    r2 = list(r)
    r2[0] = (r2[0] + 1) % O.R
    cm2 = vc.vc_commit(pp, dev_entries(I.entries(1 << L, seed + 50, 256), 256), 256)
    cases = [("value", cm.C, r, flip(y_off + 31)), ("W", cm.C, r, flip(y_off + 32 + 32 * (lM - 1) + 7, 0x04)),
             ("FC byte", cm.C, r, flip(32 + 31)), ("C_F", cm.C, r, flip(5, 0x04)), ("point", cm.C, r2, p),
             ("commitment", cm2.C, r, p)]
    for label, Cb, rr, pf in cases:
        v = vc.vc_verify_eval(pp, Cb, rr, pf)
        assert v == 0, label
        assert O.eval_verify(opp, Cb, rr, pf) == 0, label
    with pytest.raises(vc.VCError) as e:
        vc.vc_verify_eval(pp, cm.C, [O.R] + r[1:], p)
    assert e.value.code == vc.VC_EINVAL
    with pytest.raises(vc.VCError) as e:
        vc.vc_verify_eval(pp, cm.C, r, p[:-1])
    assert e.value.code == vc.VC_EINVAL
