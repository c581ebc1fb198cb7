"""The index map of the FC rounds' terms taken one round ahead (csrc/oa_terms.hpp), through the
host build: for random arrays over a prime field, with the pairing modelled by the bilinear map
(A, V) -> A V and the G1 sums by b A, the groups U, X, Y weighted by 1, x, 1/x give the L and R
of the arrays folded once (Protocol 1, Eq. folding: A'[i] = A[i] + x A[h+i],
V'[i] = V[i] + x^-1 V[h+i], b likewise).  Every output slot is written by exactly one term."""
import ctypes
import os
import random

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC_PATH = os.path.join(ROOT, "paper_2601_03031_amd", "lib", "libvc_hostcheck.so")
PR = (1 << 61) - 1


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(HC_PATH):
        from paper_2601_03031_amd import build as B
        B.build_hostcheck()
    L = ctypes.CDLL(HC_PATH)
    L.hc_oa_term.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                             ctypes.POINTER(ctypes.c_uint64)]
    return L


def lr(A, V, b, base, n):
    """L and R of one batch's round on arrays of length n at offset base: (G_T part, G1 part)"""
    h = n // 2
    L = sum(A[base + h + i] * V[base + i] for i in range(h)) % PR
    R = sum(A[base + i] * V[base + h + i] for i in range(h)) % PR
    L1 = sum(b[base + i] * A[base + h + i] for i in range(h)) % PR
    R1 = sum(b[base + h + i] * A[base + i] for i in range(h)) % PR
    return (L, L1), (R, R1)


def fold(A, V, b, base, n, x):
    h, xi = n // 2, pow(x, PR - 2, PR)
    for i in range(h):
        A[base + i] = (A[base + i] + x * A[base + h + i]) % PR
        V[base + i] = (V[base + i] + xi * V[base + h + i]) % PR
        b[base + i] = (b[base + i] + xi * b[base + h + i]) % PR


def terms(hc, K, nb, q):
    o = (ctypes.c_uint64 * 3)()
    n = nb * 8 * q
    out = []
    for t in range(n):
        hc.hc_oa_term(t, K, nb, q, o)
        out.append((o[0], o[1], o[2]))
    assert sorted(x[2] for x in out) == list(range(n)), "every output slot exactly once"
    return out


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_one_round_ahead(hc, q):
    rng = random.Random(100 + q)
    K, nb = 64, 3
    A = [rng.randrange(PR) for _ in range(K * nb)]
    V = [rng.randrange(PR) for _ in range(K * nb)]
    b = [rng.randrange(PR) for _ in range(K * nb)]
    ts = terms(hc, K, nb, q)
    gt, g1 = [0] * (nb * 8 * q), [0] * (nb * 8 * q)
    for a, v, out in ts:
        assert a // K == v // K and a % K < 4 * q and v % K < 4 * q
        gt[out], g1[out] = A[a] * V[v] % PR, b[v] * A[a] % PR
    for k in range(nb):
        x = rng.randrange(1, PR)
        xi = pow(x, PR - 2, PR)
        A2, V2, b2 = A[:], V[:], b[:]
        fold(A2, V2, b2, k * K, 4 * q, x)
        want = lr(A2, V2, b2, k * K, 2 * q)
        for side in (0, 1):
            u0 = (2 * k + side) * 2 * q
            got = []
            for arr in (gt, g1):
                U = sum(arr[u0:u0 + 2 * q])
                X = sum(arr[nb * 4 * q + (4 * k + 2 * side) * q:][:q])
                Y = sum(arr[nb * 4 * q + (4 * k + 2 * side + 1) * q:][:q])
                got.append((U + x * X + xi * Y) % PR)
            assert tuple(got) == want[side]

