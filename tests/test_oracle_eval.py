"""Pins of the oracle's evaluation proof at a point (section 4.3, compatibility with
multilinear zkSNARKs): the claimed value against the multilinear extension written out
directly (Eq. f_m), C_F against the PST commitment of the folded table, the Boolean
special cases, and the oracle's verifier against tampering."""
import random

import numpy as np
import pytest

import oracle as O
from paper_2601_03031_amd import inputs as I

SEED = I.TRAPDOOR_SEED
R = O.R


def mle(m, r):
    """f_m(r) = sum_i m_i prod_k (i_k r_k + (1 - i_k)(1 - r_k))"""
    L = len(r)
    tot = 0
    for i, mi in enumerate(m):
        w = 1
        for k in range(L):
            w = w * (r[k] if (i >> k) & 1 else (1 - r[k])) % R
        tot = (tot + mi * w) % R
    return tot


def layout(L):
    lK = L // 2
    lM = L - lK
    y_off = 32 + 832 * lK + 160
    return lK, lM, y_off


def setup(L, seed):
    limbs = I.entries(1 << L, seed, 256)
    m = I.limbs_to_ints(limbs)
    pp = O.Params(L, SEED)
    cm = O.Commitment(pp, I.limbs_to_bytes(limbs))
    return pp, cm, m


@pytest.mark.parametrize("L", [4, 5, 6])
def test_value_and_commitment(L):
    pp, cm, m = setup(L, 90 + L)
    rng = random.Random(L)
    r = [rng.randrange(R) for _ in range(L)]
    proof = cm.eval_proof(r)
    lK, lM, y_off = layout(L)
    assert len(proof) == O.eval_proof_len(L) == y_off + 32 + 32 * lM
    # the claimed value is the multilinear extension at r
    assert int.from_bytes(proof[y_off:y_off + 32], "big") == mle(m, r)
    # C_F = sum_j T_j C_j equals the PST commitment of F's table g[a] = sum_j T_j m[jM + a]
    K, M = 1 << lK, 1 << lM
    T = []
    for j in range(K):
        w = 1
        for c in range(lK):
            w = w * (r[lM + c] if (j >> c) & 1 else (1 - r[lM + c])) % R
        T.append(w)
    g = [sum(T[j] * m[j * M + a] for j in range(K)) % R for a in range(M)]
    assert proof[:32] == O.compress(1, O.pst_commit(pp, g))
    assert O.eval_verify(pp, cm.C, r, proof) == 1


def test_boolean_points():
    L = 6
    pp, cm, m = setup(L, 97)
    lK, lM, y_off = layout(L)
    M = 1 << lM
    for i in (0, 5, 37, 63):
        r = [(i >> k) & 1 for k in range(L)]
        proof = cm.eval_proof(r)
        assert int.from_bytes(proof[y_off:y_off + 32], "big") == m[i]
        # T(r_L) is the unit vector of j: C_F is C_j
        assert proof[:32] == O.compress(1, cm.Cj[i // M])
        assert O.eval_verify(pp, cm.C, r, proof) == 1


def test_verifier_rejects():
    L = 5
    pp, cm, m = setup(L, 98)
    rng = random.Random(5)
    r = [rng.randrange(R) for _ in range(L)]
    proof = cm.eval_proof(r)
    lK, lM, y_off = layout(L)

    def flip(pos, mask=1):
        a = bytearray(proof)
        a[pos] ^= mask
        return bytes(a)

    assert O.eval_verify(pp, cm.C, r, proof) == 1
    assert O.eval_verify(pp, cm.C, r, flip(y_off + 31)) == 0                  # claimed value
    assert O.eval_verify(pp, cm.C, r, flip(y_off + 32 + 32 * (lM - 1) + 7, 0x04)) == 0  # a W
    assert O.eval_verify(pp, cm.C, r, flip(32 + 31)) == 0                     # a G_T coefficient of round 1
    assert O.eval_verify(pp, cm.C, r, flip(5, 0x04)) == 0                     # C_F
    r2 = list(r)
    r2[0] = (r2[0] + 1) % R
    assert O.eval_verify(pp, cm.C, r2, proof) == 0                            # another point
    # another commitment to the same point
    _, cm2, _ = setup(L, 99)
    assert O.eval_verify(pp, cm2.C, r, proof) == 0
