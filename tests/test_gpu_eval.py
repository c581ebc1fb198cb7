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
