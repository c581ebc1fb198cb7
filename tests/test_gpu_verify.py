"""vc_verify on the GPU against the oracle's VC.Verify: honest proofs are accepted,
and for every tampered proof, wrong value and malformed input the device verifier
returns exactly what the oracle returns."""
import random
import sys

import numpy as np
import pytest

import oracle as O
from paper_2601_03031_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_03031_amd as V
    V.lib()
    return V


def setup_case(V, L, b, seed):
    N = 1 << L
    limbs = I.entries(N, seed, 256)
    ints = I.limbs_to_ints(limbs)
    opp = O.Params(L, I.TRAPDOOR_SEED)
    ocm = O.Commitment(opp, I.limbs_to_bytes(limbs))
    oop = O.Opening(ocm, b)
    gpp = V.vc_setup(L, I.TRAPDOOR_SEED, 0)
    return opp, ocm, oop, gpp, ints


@pytest.mark.parametrize("L,b", [(4, 1), (5, 3), (6, 8)])
def test_verify_matches_oracle(vc, L, b):
    print("verify case L=%d b=%d" % (L, b), flush=True)
    opp, ocm, oop, gpp, ints = setup_case(vc, L, b, 21 + L)
    N = 1 << L
    rng = random.Random(L * 100 + b)
    for i in sorted({0, N - 1, rng.randrange(N)}):
        proof = oop.proof(i)
        assert vc.vc_verify(gpp, ocm.C, b, i, ints[i], proof) == 1, i
        # wrong value
        assert vc.vc_verify(gpp, ocm.C, b, i, (ints[i] + 1) % O.R, proof) == O.verify(opp, ocm.C, b, i, (ints[i] + 1) % O.R, proof) == 0
        # tampered bytes across the proof's fields
        for pos in sorted({0, 5, 32 * 1 + 3, len(proof) // 3, len(proof) // 2, len(proof) - 40, len(proof) - 1}):
            bad = bytearray(proof)
            bad[pos] ^= 0x21
            want = O.verify(opp, ocm.C, b, i, ints[i], bytes(bad))
            got = vc.vc_verify(gpp, ocm.C, b, i, ints[i], bytes(bad))
            assert got == want, (i, pos, got, want)
    # malformed commitment bytes (a coefficient >= p) and out-of-range m_i
    badC = b"\xff" * 32 + ocm.C[32:]
    assert O.verify(opp, badC, b, 0, ints[0], oop.proof(0)) < 0
    with pytest.raises(vc.VCError):
        vc.vc_verify(gpp, badC, b, 0, ints[0], oop.proof(0))


def test_gpu_proofs_verify_on_gpu(vc):
    """proofs produced by the HIP path verify on the device verifier"""
    L, b = 6, 3
    N = 1 << L
    limbs = I.entries(N, 31, 256)
    ints = I.limbs_to_ints(limbs)
    gpp = vc.vc_setup(L, I.TRAPDOOR_SEED, 0)
    m = torch.from_numpy(np.ascontiguousarray(limbs).view(np.uint8).reshape(-1).copy()).cuda()
    gcm = vc.vc_commit(gpp, m, 256)
    gpr = vc.vc_open_all(gpp, gcm, b)
    for i in (1, 17, N - 2):
        assert vc.vc_verify(gpp, gcm.C, b, i, ints[i], vc.vc_proof_get(gpr, i)) == 1
