"""GPU self-test of the base-field layer the proof rounds run on (8 lanes per
element), against Python integers, through the C ABI."""
import ctypes as C
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
