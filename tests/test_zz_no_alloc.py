"""vc_commit_noalloc (the commit that allocates no device memory, its scratch in one static
device array per GPU) against vc_commit, byte for byte: two calls in a row, the second with a
smaller input, and its error paths."""
import sys

import numpy as np
import pytest

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


def check_against_commit(V, L, bits, seed):
    say("no-alloc commit L=%d bits=%d seed=%d" % (L, bits, seed))
    pp = V.vc_setup(L, SEED, 0)
    m = dev_entries(I.entries(1 << L, seed, bits), bits)
    cj = torch.full((64 * pp.K,), 0xA5, dtype=torch.uint8, device="cuda")
    c = V.vc_commit_noalloc(pp, m, bits, cj)
    torch.cuda.synchronize()
    ref = V.vc_commit(pp, m, bits)
    assert c == ref.C
    assert bytes(cj.cpu().numpy()) == ref.export("Cj")


def test_two_calls_second_smaller(vc):
    # the second call reuses the array the first one filled (larger N, full-width entries)
    check_against_commit(vc, 16, 256, 21)
    check_against_commit(vc, 10, 32, 22)


def test_largest_size_then_small(vc):
    check_against_commit(vc, 20, 256, 23)
    check_against_commit(vc, 6, 256, 24)


def test_errors(vc):
    pp = vc.vc_setup(4, SEED, 0)
    cj = torch.zeros(64 * pp.K, dtype=torch.uint8, device="cuda")
    bad = np.zeros((16, 4), dtype=np.uint64)
    bad[5] = np.array([(I.R >> (64 * k)) & (2**64 - 1) for k in range(4)], dtype=np.uint64)  # entry == r
    with pytest.raises(vc.VCError) as e:
        vc.vc_commit_noalloc(pp, dev_entries(bad, 256), 256, cj)
    assert e.value.code == vc.VC_EINVAL
    # a good call right after the failed one
    good = I.entries(16, 25, 256)
    c = vc.vc_commit_noalloc(pp, dev_entries(good, 256), 256, cj)
    ref = vc.vc_commit(pp, dev_entries(good, 256), 256)
    assert c == ref.C and bytes(cj.cpu().numpy()) == ref.export("Cj")


def test_rejects_beyond_its_scratch(vc):
    # N = 2^21 is past the array's stated maximum (N <= 2^20): refused before any launch
    pp = vc.vc_setup(21, SEED, 0)
    m = torch.zeros(32 << 21, dtype=torch.uint8, device="cuda")
    cj = torch.zeros(64 * pp.K, dtype=torch.uint8, device="cuda")
    with pytest.raises(vc.VCError) as e:
        vc.vc_commit_noalloc(pp, m, 256, cj)
    assert e.value.code == vc.VC_EINVAL
