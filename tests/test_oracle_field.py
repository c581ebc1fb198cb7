"""Pins for the oracle's prime fields and F_p2 against Python integers."""
import random

import pytest

import oracle as O

P, R = O.P, O.R
EDGE = [0, 1, 2, P - 1, P - 2, (P - 1) // 2, 1 << 253]


@pytest.mark.parametrize("which,mod", [("p", P), ("r", R)])
def test_field_ops_match_python_ints(which, mod):
    rng = random.Random(7)
    vals = [v % mod for v in EDGE] + [rng.randrange(mod) for _ in range(200)]
    for a in vals:
        b = vals[rng.randrange(len(vals))]
        assert O.field_op(which, "add", a, b) == (a + b) % mod
        assert O.field_op(which, "sub", a, b) == (a - b) % mod
        assert O.field_op(which, "mul", a, b) == (a * b) % mod
        assert O.field_op(which, "neg", a) == (-a) % mod
        if a:
            assert O.field_op(which, "inv", a) == pow(a, -1, mod)


def test_field_rejects_noncanonical():
    with pytest.raises(ValueError):
        O.field_op("p", "add", P, 1)
    with pytest.raises(ValueError):
        O.field_op("r", "mul", R, 1)


def test_fp_sqrt():
    rng = random.Random(3)
    for _ in range(50):
        x = rng.randrange(P)
        s, ok = O.field_op("p", "sqrt", x * x % P)
        assert ok and s * s % P == x * x % P
        y = rng.randrange(P)
        s, ok = O.field_op("p", "sqrt", y)
        assert ok == (pow(y, (P - 1) // 2, P) in (0, 1))


def _f2mul(a, b):
    return ((a[0] * b[0] - a[1] * b[1]) % P, (a[0] * b[1] + a[1] * b[0]) % P)


def test_fp2_mul_inv_sqrt():
    rng = random.Random(5)
    for _ in range(50):
        a = (rng.randrange(P), rng.randrange(P))
        b = (rng.randrange(P), rng.randrange(P))
        assert O.fp2_op("mul", a, b) == _f2mul(a, b)
        ai = O.fp2_op("inv", a)
        assert _f2mul(a, ai) == (1, 0)
        sq = _f2mul(a, a)
        s, ok = O.fp2_op("sqrt", sq)
        assert ok and _f2mul(s, s) == sq
    # i^2 = -1: i itself is not a square root of 1
    assert O.fp2_op("mul", (0, 1), (0, 1)) == (P - 1, 0)


def test_fp12_inverse_and_order():
    rng = random.Random(11)
    a = b"".join(O.be32(rng.randrange(P)) for _ in range(12))
    ai = O.fp12_op("inv", a)
    assert O.fp12_op("mul", a, ai) == O.GT_ONE
    # the final exponent maps into the order-r subgroup: FE(a)^r = 1
    f = O.fp12_op("final_exp", a)
    assert O.fp12_op("pow", f, O.be32(0)) == O.GT_ONE
    # homomorphism: FE(a b) = FE(a) FE(b)
    b = b"".join(O.be32(rng.randrange(P)) for _ in range(12))
    assert O.fp12_op("final_exp", O.fp12_op("mul", a, b)) == O.fp12_op(
        "mul", f, O.fp12_op("final_exp", b))
