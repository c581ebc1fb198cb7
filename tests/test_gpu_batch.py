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
    say("batch with one executor given twice")
    with pytest.raises(vc.VCError) as e:
        vc.vc_open_all_batch([(pp, cms[0], 4), (pp, cms[1], 5)], [ex, ex])
    assert e.value.code == vc.VC_EINVAL
    for ns in (0, 7):
        with pytest.raises(vc.VCError) as e:
            vc.vc_exec_create(0, ns)
        assert e.value.code == vc.VC_EINVAL


def test_grouped_matches_single_jobs_and_oracle(vc):
    """Fused groups (vc_open_all_grouped): jobs on the same params with the same b run as one
    Step 1 over all their batches.  Every job's arrays and sampled proofs equal its one-job
    call's, and the oracle's at L <= 6; groups cut at 2 and at 8 jobs; rounds taken ahead
    (small groups), direct rounds where the group's batches fill the device but the single
    job's do not (four 2^12, b = 1 jobs), ragged last batches, u32 and full-width entries in
    one group, a job with no partner."""
    spec = [(6, 2, 31, 32), (6, 2, 32, 256), (6, 2, 33, 32), (5, 3, 34, 256), (5, 3, 35, 256),
            (9, 3, 36, 32), (9, 3, 37, 256), (9, 3, 38, 32), (12, 1, 39, 32), (12, 1, 40, 256),
            (12, 1, 41, 32), (12, 1, 42, 32), (14, 2, 43, 256), (14, 2, 44, 32), (10, 32, 45, 256),
            (10, 32, 46, 256), (8, 16, 47, 32), (8, 16, 48, 256), (7, 4, 49, 256)]
    params, jobs, ints = {}, [], []
    for L, b, seed, bits in spec:
        if L not in params:
            params[L] = vc.vc_setup(L, SEED, 0)
        limbs = I.entries(1 << L, seed, bits)
        m = dev_u32(limbs[:, 0]) if bits == 32 else \
            torch.from_numpy(np.ascontiguousarray(limbs).view(np.uint8).reshape(-1).copy()).cuda()
        jobs.append((params[L], vc.vc_commit(params[L], m, bits), b))
        ints.append(limbs)
    singles = [vc.vc_open_all(pp, cm, b) for pp, cm, b in jobs]
    execs = [vc.vc_exec_create(0, ns) for ns in (6, 2)]
    for gmax in (8, 2):
        say("grouped: %d jobs, groups of at most %d" % (len(jobs), gmax))
        out = vc.vc_open_all_grouped(jobs, execs, gmax)
        torch.cuda.synchronize()
        for (pp, cm, b), pr, one, limbs, (L, _, seed, bits) in zip(jobs, out, singles, ints, spec):
            N, M = pp.N, pp.M
            same_proofs(vc, pp, pr, one, sorted({0, 1, M - 1, M, N - 1, N // 2 + 3}))
            if L <= 6:
                opp = O.Params(L, SEED)
                oop = O.Opening(O.Commitment(opp, I.limbs_to_bytes(limbs)), b)
                for i in range(N):
                    assert vc.vc_proof_get(pr, i) == oop.proof(i), (L, b, seed, i)
        say("  every job equal")
        del out
    say("grouped: zero challenge in a group")
    try:
        vc.vc_test_zero_challenge(2)
        with pytest.raises(vc.VCError) as e:
            vc.vc_open_all_grouped(jobs[:3], execs, 8)
        assert e.value.code == vc.VC_ECHALLENGE
    finally:
        vc.vc_test_zero_challenge(0)
    again = vc.vc_open_all_grouped(jobs[:3], execs[:1], 8)
    for pr, one, (pp, _, _) in zip(again, singles[:3], jobs[:3]):
        same_proofs(vc, pp, pr, one, range(pp.N))
    with pytest.raises(vc.VCError) as e:
        vc.vc_open_all_grouped(jobs[:2], execs, 0)
    assert e.value.code == vc.VC_EINVAL


def _dev_entries(limbs, bits):
    if bits == 32:
        return dev_u32(limbs[:, 0])
    return torch.from_numpy(np.ascontiguousarray(limbs).view(np.uint8).reshape(-1).copy()).cuda()


def test_commit_batch_matches_single_and_oracle(vc, tmp_path):
    """vc_commit_batch (all jobs' MSMs in one persistent launch, FC.Commit of all jobs in fused
    launches): every job's C_j and C equal vc_commit's and the oracle's (L <= 8); jobs of uneven
    N and entry width, some on shared params; open-all from a batch-made commitment equals the
    one from vc_commit's; the autotuned schedule gives the same bytes; an entry >= r fails the
    batch."""
    spec = [(4, 256, 51), (8, 32, 52), (12, 256, 53), (6, 32, 54), (8, 256, 55), (14, 32, 56), (10, 256, 57),
            (12, 32, 58), (5, 256, 59), (16, 256, 60)]
    params = {}
    jobs, limbs_all = [], []
    for L, bits, seed in spec:
        if L not in params:
            params[L] = vc.vc_setup(L, SEED, 0)
        limbs = I.entries(1 << L, seed, bits)
        jobs.append((params[L], _dev_entries(limbs, bits), bits))
        limbs_all.append(limbs)
    say("commit batch of %d jobs" % len(jobs))
    got = vc.vc_commit_batch(jobs)
    singles = [vc.vc_commit(pp, m, bits) for pp, m, bits in jobs]
    for (L, bits, seed), g, s, limbs in zip(spec, got, singles, limbs_all):
        assert g.C == s.C and g.export("C") == s.C, (L, bits, seed)
        assert g.export("Cj") == s.export("Cj"), (L, bits, seed)
        if L <= 8:
            ocm = O.Commitment(O.Params(L, SEED), I.limbs_to_bytes(limbs))
            assert g.C == ocm.C and g.export("Cj") == b"".join(ocm.Cj), (L, bits, seed)
    for i in (2, 5):
        pp = jobs[i][0]
        a = vc.vc_open_all(pp, got[i], 3)
        b_ = vc.vc_open_all(pp, singles[i], 3)
        same_proofs(vc, pp, a, b_, [0, pp.N - 1, pp.N // 3])
    say("autotuned schedule")
    path = str(tmp_path / "msm.txt")
    vc.vc_tune_msm(4, 16, path)
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    assert {(int(a), int(b)) for a, b, _ in rows} == {(L, w) for L in range(4, 17) for w in (32, 256)}
    try:
        vc.vc_tune_load(path)
        tuned = vc.vc_commit_batch(jobs)
        for g, s in zip(tuned, singles):
            assert g.C == s.C and g.export("Cj") == s.export("Cj")
        for (pp, m, bits), s in zip(jobs, singles):
            t1 = vc.vc_commit(pp, m, bits)
            assert t1.C == s.C and t1.export("Cj") == s.export("Cj")
        bad = tmp_path / "bad.txt"
        bad.write_text("16 256 1000\n")  # 1000 x 32 digits: more than a workgroup sorts
        with pytest.raises(vc.VCError) as e:
            vc.vc_tune_load(str(bad))
        assert e.value.code == vc.VC_EINVAL
    finally:
        vc.vc_tune_load(None)
    say("commit batch with an entry >= r")
    limbs = I.entries(64, 61)
    r_limbs = [(I.R >> (64 * k)) & (2**64 - 1) for k in range(4)]
    limbs[7] = np.array(r_limbs, dtype=np.uint64)
    with pytest.raises(vc.VCError) as e:
        vc.vc_commit_batch([jobs[3], (params[6], _dev_entries(limbs, 256), 256)])
    assert e.value.code == vc.VC_EINVAL
    assert vc.vc_commit_batch([]) == []


def test_commit_batch_graph_replays(vc):
    """Batched commits through a captured HIP graph (vc_exec_set_graphs): the first call of a
    shape captures the fused chain, later calls of that shape replay it with new entries (with
    other device work between the replays); every replay equals the eager batch and vc_commit,
    a new shape captures again, and the old shape after it too."""
    shapes = {"A": [(8, 256), (12, 32), (10, 256), (6, 32)], "B": [(14, 256), (9, 32)]}
    params = {}

    def jobs_for(shape, seed):
        out = []
        for k, (L, bits) in enumerate(shapes[shape]):
            if L not in params:
                params[L] = vc.vc_setup(L, SEED, 0)
            out.append((params[L], _dev_entries(I.entries(1 << L, 1000 * seed + k, bits), bits), bits))
        return out

    gex = vc.vc_exec_create(0, 2)
    gex.set_graphs(True)
    eex = vc.vc_exec_create(0, 2)
    order = [("A", 71), ("A", 72), ("A", 73), ("B", 74), ("B", 75), ("A", 76)]
    for shape, seed in order:
        say("graph batch %s seed %d" % (shape, seed))
        jobs = jobs_for(shape, seed)
        got = vc.vc_commit_batch(jobs, ex=gex)
        # other device work between replays: an eager batch, single commits, a torch op
        ref = vc.vc_commit_batch(jobs, ex=eex)
        x = torch.arange(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert int(x) == (1 << 20) * ((1 << 20) - 1) // 2
        for g, r, (pp, m, bits) in zip(got, ref, jobs):
            one = vc.vc_commit(pp, m, bits)
            assert g.C == r.C == one.C and g.export("Cj") == r.export("Cj") == one.export("Cj")
    caps, reps = gex.graph_stats()
    assert reps == len(order) and caps == 3, (caps, reps)  # A, B, then A again
    assert eex.graph_stats() == (0, 0)
    gex.set_graphs(False)
