"""Batched jobs: OpenAll over several independent vectors at once (executors on host
threads) gives, job by job, exactly the proofs of the one-job call, and the oracle's for the
small ones."""
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


def dev_u32(v: np.ndarray):
    return torch.from_numpy(v.astype(np.uint32).view(np.int32).copy()).cuda()


def same_proofs(V, pp, a, b_, idx):
    K = pp.K
    nb = (K + a.b - 1) // a.b
    for k in range(nb):
        for w in ("fc_x", "fc_rounds", "fc_tail"):
            assert a.export(w, k) == b_.export(w, k), (w, k)
    for w in ("merkle", "rho", "y", "D", "W"):
        assert a.export(w) == b_.export(w), w
    for i in idx:
        assert V.vc_proof_get(a, i) == V.vc_proof_get(b_, i), ("proof", i)


def test_batch_matches_single_jobs_and_oracle(vc):
    # (L, b, seed): rounds taken ahead (most), direct then ahead (2^12, b=1), all direct
    # (2^14, b=2), ragged last batches, two jobs on one params, more jobs than executors
    spec = [(4, 1, 11), (6, 8, 12), (10, 3, 13), (5, 3, 14), (12, 36, 15), (6, 2, 16), (10, 20, 17),
            (12, 1, 18), (14, 2, 19)]
    params = {}
    jobs, ints = [], []
    for L, b, seed in spec:
        say("batch job L=%d b=%d seed=%d" % (L, b, seed))
        if L not in params:
            params[L] = vc.vc_setup(L, SEED, 0)
        limbs = I.entries(1 << L, seed, 32)
        cm = vc.vc_commit(params[L], dev_u32(limbs[:, 0]), 32)
        jobs.append((params[L], cm, b))
        ints.append(limbs)
    # executors of six, two and one streams
    execs = [vc.vc_exec_create(0, ns) for ns in (6, 2, 1)]
    say("  batch of %d jobs on %d executors" % (len(jobs), len(execs)))
    out = vc.vc_open_all_batch(jobs, execs)
    torch.cuda.synchronize()
    say("  batch done; single jobs")
    for (pp, cm, b), pr, limbs, (L, _, seed) in zip(jobs, out, ints, spec):
        one = vc.vc_open_all(pp, cm, b)
        N, M = pp.N, pp.M
        idx = sorted({0, 1, M - 1, M, N - 1, N // 2 + 3})
        same_proofs(vc, pp, pr, one, idx)
        if L <= 6:
            opp = O.Params(L, SEED)
            oop = O.Opening(O.Commitment(opp, I.limbs_to_bytes(limbs)), b)
            for i in range(N):
                assert vc.vc_proof_get(pr, i) == oop.proof(i), (L, b, i)
        say("  job L=%d b=%d seed=%d equal" % (L, b, seed))


def test_batch_on_one_executor_and_errors(vc):
    pp = vc.vc_setup(6, SEED, 0)
    cms = [vc.vc_commit(pp, dev_u32(I.entries(64, s, 32)[:, 0]), 32) for s in (21, 22)]
    ex = vc.vc_exec_create(0, 3)
    say("batch on one executor")
    out = vc.vc_open_all_batch([(pp, cms[0], 4), (pp, cms[1], 5)], [ex])
    ref = [vc.vc_open_all_ex(pp, cms[0], 4, ex), vc.vc_open_all(pp, cms[1], 5)]
    for a, r in zip(out, ref):
        same_proofs(vc, pp, a, r, range(64))
    assert vc.vc_open_all_batch([], [ex]) == []
    say("batch with an invalid batch size")
    with pytest.raises(vc.VCError) as e:
        vc.vc_open_all_batch([(pp, cms[0], 4), (pp, cms[1], 0)], [ex, vc.vc_exec_create(0)])
    assert e.value.code == vc.VC_EINVAL
    with pytest.raises(vc.VCError) as e:
        vc.vc_open_all_batch([(pp, cms[0], 4)], [])
    assert e.value.code == vc.VC_EINVAL
    for ns in (0, 7):
        with pytest.raises(vc.VCError) as e:
            vc.vc_exec_create(0, ns)
        assert e.value.code == vc.VC_EINVAL
