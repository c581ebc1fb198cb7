"""GPU self-test of the base-field layer the proof rounds run on (8 lanes per
element), against Python integers, through the C ABI."""
import ctypes as C
import os
import random

import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vlib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_03031_amd as V
    L = V.lib()
    L.vc_diag_field.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_char_p, C.c_char_p, C.c_void_p]
    return L


@pytest.mark.parametrize("which,mod", [(0, O.P), (1, O.R)])
def test_wide_field_ops(vlib, which, mod):
    rng = random.Random(17 + which)
    edge = [0, 1, 2, mod - 1, mod - 2, (1 << 32) - 1, 1 << 32, (1 << 224) + 5, mod >> 1]
    a = edge + [rng.randrange(mod) for _ in range(300)]
    b = [rng.randrange(mod) for _ in range(len(edge))] + [rng.randrange(mod) for _ in range(300)]
    b[3] = mod - 1
    n = len(a)
    A = b"".join(x.to_bytes(32, "little") for x in a)
    B = b"".join(x.to_bytes(32, "little") for x in b)
    want = {0: lambda x, y: x * y % mod, 1: lambda x, y: (x + y) % mod, 2: lambda x, y: (x - y) % mod,
            3: lambda x, y: x * pow(2, -1, mod) % mod, 4: lambda x, y: pow(x, -1, mod) if x else 0,
            5: lambda x, y: x * x % mod}
    for op, f in want.items():
        out = C.create_string_buffer(32 * n)
        assert vlib.vc_diag_field(which, op, n, A, B, out) == 0
        got = [int.from_bytes(out.raw[32 * i:32 * i + 32], "little") for i in range(n)]
        bad = [i for i in range(n) if got[i] != f(a[i], b[i])]
        assert not bad, (op, bad[:5], [hex(got[i]) for i in bad[:2]])


@pytest.mark.parametrize("which,mod", [(0, O.P), (1, O.R)])
def test_wide_raw_matches_lane_model(vlib, which, mod):
    """Raw Montgomery limbs through the 8-lane layout's mul/add/sub on the device, bit for bit
    against the host lane model of the same layout, over the whole 256-bit input range
    (canonical, below twice the modulus, and beyond).  Where the inputs are canonical the
    results are also checked to be canonical and correct, which is the range the wide Miller
    loop's stored coefficients come from."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    HC_PATH = os.path.join(root, "paper_2601_03031_amd", "lib", "libvc_hostcheck.so")
    if not os.path.exists(HC_PATH):
        from paper_2601_03031_amd import build as B
        B.build_hostcheck()
    hc = C.CDLL(HC_PATH)
    rng = random.Random(73 + which)
    canon = [0, 1, mod - 1, mod - 2, mod >> 1, (1 << 32) - 1] + [rng.randrange(mod) for _ in range(120)]
    below2 = [mod, 2 * mod - 1] + [rng.randrange(mod, 2 * mod) for _ in range(60)]
    beyond = [2 * mod, (1 << 256) - 1] + [rng.randrange(2 * mod, 1 << 256) for _ in range(60)]
    a = canon + below2 + beyond
    b = [rng.choice(canon) if i % 3 else rng.choice(a) for i in range(len(a))]
    n = len(a)
    A = b"".join(x.to_bytes(32, "little") for x in a)
    B_ = b"".join(x.to_bytes(32, "little") for x in b)
    rinv = pow(1 << 256, -1, mod)
    for op in (0, 1, 2):
        out = C.create_string_buffer(32 * n)
        assert vlib.vc_diag_field(2 + which, op, n, A, B_, out) == 0
        for i in range(n):
            got = int.from_bytes(out.raw[32 * i:32 * i + 32], "little")
            o = C.create_string_buffer(32)
            assert hc.hc_wide_raw(which, op, a[i].to_bytes(32, "little"), b[i].to_bytes(32, "little"), o) == 0
            assert got == int.from_bytes(o.raw, "little"), (op, i, hex(a[i]), hex(b[i]))
            if a[i] < mod and b[i] < mod:
                want = a[i] * b[i] * rinv % mod if op == 0 else (a[i] + b[i]) % mod if op == 1 else (a[i] - b[i]) % mod
                assert got == want, (op, i)
