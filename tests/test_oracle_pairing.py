"""Pins for the oracle's pairing: bilinearity, non-degeneracy, order r, and that the
multi-pairing A*B equals the product of single pairings."""
import random

import oracle as O

R = O.R
G1, G2 = O.generators()


def test_bilinear_nondegenerate_order_r():
    rng = random.Random(9)
    e = O.pairing([G1], [G2])
    assert e != O.GT_ONE
    assert O.fp12_op("pow", e, O.be32(0)) == O.GT_ONE  # exponent r = 0 mod r would be trivial;
    # e^r = 1 checked by e^(r-1) * e = 1
    assert O.fp12_op("mul", O.fp12_op("pow", e, O.be32(R - 1)), e) == O.GT_ONE
    for _ in range(3):
        a, b = rng.randrange(1, R), rng.randrange(1, R)
        lhs = O.pairing([O.g1_op("mul", G1, O.be32(a))], [O.g2_op("mul", G2, O.be32(b))])
        assert lhs == O.fp12_op("pow", e, O.be32(a * b % R))


def test_multi_pairing_is_product_and_identity_pairs():
    rng = random.Random(10)
    Ps = [O.g1_op("mul", G1, O.be32(rng.randrange(R))) for _ in range(3)]
    Qs = [O.g2_op("mul", G2, O.be32(rng.randrange(R))) for _ in range(3)]
    prod = O.GT_ONE
    for p_, q_ in zip(Ps, Qs):
        prod = O.fp12_op("mul", prod, O.pairing([p_], [q_]))
    assert O.pairing(Ps, Qs) == prod
    assert O.pairing([bytes(64)], [G2]) == O.GT_ONE
    assert O.pairing([G1], [bytes(128)]) == O.GT_ONE
    # e(-P, Q) e(P, Q) = 1
    assert O.pairing([O.g1_op("neg", G1), G1], [G2, G2]) == O.GT_ONE
