"""Serving loop: requests queued in arrival order on a pool of executors under a device-memory
budget give, request by request, exactly the proofs of the one-job call (and the oracle's for
the small ones)."""
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


def test_footprint(vc):
    pp = vc.vc_setup(10, SEED, 0)
    f = [vc.vc_open_all_footprint(pp, b) for b in (1, 2, 5, 32)]
    say("footprints at 2^10, b = 1, 2, 5, 32: %s" % f)
    assert all(x > 0 for x in f)
    assert f[0] > f[1] > f[2] > f[3]  # fewer batches, smaller workspace
    # the proof bundle alone (y-tree, Merkle heap) is a lower bound
    assert f[3] > (2 * 32 - 1) * 32 * 32 + 2 * 1024 * 32
    for b in (0, 33):
        with pytest.raises(vc.VCError) as e:
            vc.vc_open_all_footprint(pp, b)
        assert e.value.code == vc.VC_EINVAL


def test_server_matches_single_jobs_and_oracle(vc):
    # (L, b, bits, seed); submitted all at once, so that the budget decides what runs together
    spec = [(10, 1, 256, 31), (4, 2, 32, 32), (12, 12, 32, 33), (6, 8, 256, 34), (8, 1, 32, 35), (5, 3, 256, 36),
            (12, 1, 256, 37), (10, 10, 32, 38), (6, 1, 32, 39)]
    params, jobs = {}, []
    for L, b, bits, seed in spec:
        if L not in params:
            params[L] = vc.vc_setup(L, SEED, 0)
        limbs = I.entries(1 << L, seed, bits)
        jobs.append((params[L], vc.vc_commit(params[L], dev_entries(limbs, bits), bits), b, limbs))
    foot = [vc.vc_open_all_footprint(pp, b) for pp, _, b, _ in jobs]
    budget = max(foot) + min(foot)  # the largest runs with at most the smallest beside it
    say("server: 3 executors x 2 streams, budget %d bytes (largest request %d)" % (budget, max(foot)))
    sv = vc.vc_server_create(0, 3, 2, budget)
    tickets = [sv.submit(pp, cm, b) for pp, cm, b, _ in jobs]
    got = [sv.wait(t) for t in tickets]
    held, peak, bud = sv.stats()
    say("  served; the server held at most %d bytes (budget %d); single jobs" % (peak, bud))
    assert bud == budget and 0 < peak <= budget
    for (pp, cm, b, limbs), (pr, (waited, total)), (L, _, bits, seed) in zip(jobs, got, spec):
        assert 0 <= waited <= total
        one = vc.vc_open_all(pp, cm, b)
        nb = (pp.K + b - 1) // b
        for k in range(nb):
            for w in ("fc_x", "fc_rounds", "fc_tail"):
                assert pr.export(w, k) == one.export(w, k), (L, b, w, k)
        for w in ("merkle", "rho", "y", "D", "W"):
            assert pr.export(w) == one.export(w), (L, b, w)
        idx = range(pp.N) if L <= 6 else sorted({0, 1, pp.M, pp.N // 2 + 5, pp.N - 1})
        for i in idx:
            assert vc.vc_proof_get(pr, i) == vc.vc_proof_get(one, i), (L, b, i)
        if L <= 6:
            opp = O.Params(L, SEED)
            oop = O.Opening(O.Commitment(opp, I.limbs_to_bytes(limbs)), b)
            for i in range(pp.N):
                assert vc.vc_proof_get(pr, i) == oop.proof(i), (L, b, i)
        say("  request L=%d b=%d bits=%d equal (waited %.1f ms of %.1f ms)" % (L, b, bits, waited, total))
    del sv


def test_server_errors(vc):
    pp = vc.vc_setup(6, SEED, 0)
    cm = vc.vc_commit(pp, dev_entries(I.entries(64, 41, 32), 32), 32)
    f = vc.vc_open_all_footprint(pp, 2)
    sv = vc.vc_server_create(0, 1, 1, f - 1)
    with pytest.raises(vc.VCError) as e:
        sv.submit(pp, cm, 2)
    assert e.value.code == vc.VC_ENOMEM
    with pytest.raises(vc.VCError) as e:
        sv.submit(pp, cm, 9)
    assert e.value.code == vc.VC_EINVAL
    del sv
    for args in ((0, 0, 1, 1 << 30), (0, 1, 0, 1 << 30), (0, 1, 7, 1 << 30), (0, 1, 1, 0)):
        with pytest.raises(vc.VCError) as e:
            vc.vc_server_create(*args)
        assert e.value.code == vc.VC_EINVAL
    # released with requests still waiting: the running one finishes, the others are dropped
    sv = vc.vc_server_create(0, 1, 1, 1 << 30)
    for s in range(3):
        sv.submit(pp, cm, 1 + s)
    del sv
    torch.cuda.synchronize()


def test_server_budget_counts_kept_workspace(vc):
    """A budget that fits one large request but not a large request beside another executor's
    kept workspace: the server stays within it (its accounting is exact), by releasing idle
    executors' workspaces, and every request still equals the one-job call.  Device memory in
    use, sampled while it serves, rises by at most the budget plus the one bundle the caller
    holds, plus the runtime's queue allocations for an executor's first launches."""
    import threading
    spec = [(18, 1, 256, 51), (14, 1, 32, 52), (18, 2, 256, 53), (16, 1, 256, 54), (18, 1, 32, 55), (12, 2, 32, 56)]
    params, jobs = {}, []
    for L, b, bits, seed in spec:
        if L not in params:
            params[L] = vc.vc_setup(L, SEED, 0)
        limbs = I.entries(1 << L, seed, bits)
        jobs.append((params[L], vc.vc_commit(params[L], dev_entries(limbs, bits), bits), b))
    foot = [vc.vc_open_all_footprint(pp, b) for pp, _, b in jobs]
    budget = max(foot) + max(foot) // 8
    sv = vc.vc_server_create(0, 3, 1, budget)
    # warm-up: three small requests at once, so that every executor has launched (its queues
    # exist) before the baseline is taken
    pw = vc.vc_setup(10, SEED, 0)
    cw = vc.vc_commit(pw, dev_entries(I.entries(1 << 10, 57, 32), 32), 32)
    for t in [sv.submit(pw, cw, 1) for _ in range(3)]:
        sv.wait(t)
    torch.cuda.synchronize()
    f0, tot = torch.cuda.mem_get_info()
    used0 = tot - f0 - sv.stats()[0]  # without what the server holds now
    seen = [0]
    done = threading.Event()

    def sample():
        while not done.is_set():
            f, t = torch.cuda.mem_get_info()
            seen[0] = max(seen[0], t - f - used0)
            done.wait(0.002)

    th = threading.Thread(target=sample)
    th.start()
    tickets = [sv.submit(pp, cm, b) for pp, cm, b in jobs]
    results = []
    for t in tickets:
        pr, _ = sv.wait(t)
        results.append(pr.export("fc_x", 0) + pr.export("W"))
        del pr  # the caller holds one bundle at a time
    held, peak, bud = sv.stats()
    done.set()
    th.join()
    say("  budget %d: the server held at most %d; device use rose by at most %d" % (budget, peak, seen[0]))
    assert peak <= budget
    assert seen[0] <= budget + max(foot) + (64 << 20)
    del sv
    for (pp, cm, b), got in zip(jobs, results):
        one = vc.vc_open_all(pp, cm, b)
        assert got == one.export("fc_x", 0) + one.export("W")
