"""Pins for the oracle's G1/G2 group law: curve equations, group orders, the
chord-tangent law in affine coordinates (Python integers), scalar-multiplication
identities, the Frobenius eigenvalue on G2 and point compression."""
import random

import oracle as O

P, R = O.P, O.R
G1, G2 = O.generators()


def xy(b):
    return int.from_bytes(b[:32], "big"), int.from_bytes(b[32:64], "big")


def enc(pt):
    if pt is None:
        return bytes(64)
    return O.be32(pt[0]) + O.be32(pt[1])


def aff_add(A, B):
    """textbook affine group law on y^2 = x^3 + 3"""
    if A is None:
        return B
    if B is None:
        return A
    if A[0] == B[0]:
        if (A[1] + B[1]) % P == 0:
            return None
        lam = 3 * A[0] * A[0] * pow(2 * A[1], -1, P) % P
    else:
        lam = (B[1] - A[1]) * pow(B[0] - A[0], -1, P) % P
    x3 = (lam * lam - A[0] - B[0]) % P
    return (x3, (lam * (A[0] - x3) - A[1]) % P)


def aff_mul(A, k):
    out = None
    while k:
        if k & 1:
            out = aff_add(out, A)
        A = aff_add(A, A)
        k >>= 1
    return out


def test_generators_on_curve_and_order_r():
    assert xy(G1) == (1, 2)
    assert O.g1_valid(G1) and O.g2_valid(G2)
    assert O.g1_op("mul_int", G1, O.be32(R)) == bytes(64)
    assert O.g2_op("mul_int", G2, O.be32(R)) == bytes(128)
    # r - 1 gives -G
    assert O.g1_op("mul_int", G1, O.be32(R - 1)) == O.g1_op("neg", G1)


def test_g1_matches_affine_chord_tangent():
    rng = random.Random(1)
    for k in [1, 2, 3, 5, 255, 2**64 + 3] + [rng.randrange(R) for _ in range(10)]:
        assert O.g1_op("mul", G1, O.be32(k)) == enc(aff_mul((1, 2), k))
    A = O.g1_op("mul", G1, O.be32(12345))
    B = O.g1_op("mul", G1, O.be32(999))
    assert O.g1_op("add", A, B) == enc(aff_add(xy(A), xy(B)))
    assert O.g1_op("add", A, A) == enc(aff_add(xy(A), xy(A)))
    assert O.g1_op("add", A, O.g1_op("neg", A)) == bytes(64)
    assert O.g1_op("add", A, bytes(64)) == A


def test_scalar_mul_identities():
    rng = random.Random(2)
    for gen, op in ((G1, O.g1_op), (G2, O.g2_op)):
        a, b = rng.randrange(R), rng.randrange(R)
        aG, bG = op("mul", gen, O.be32(a)), op("mul", gen, O.be32(b))
        assert op("add", aG, bG) == op("mul", gen, O.be32((a + b) % R))
        assert op("mul", aG, O.be32(b)) == op("mul", gen, O.be32(a * b % R))
        assert op("add", aG, aG) == op("mul", gen, O.be32(2 * a % R))
        assert op("add", aG, op("neg", aG)) == bytes(len(gen))


def test_g2_frobenius_is_multiplication_by_p():
    Q = O.g2_op("mul", G2, O.be32(777))
    assert O.g2_op("frobenius", Q) == O.g2_op("mul", Q, O.be32(P % R))


def test_compression_roundtrip_and_rejection():
    rng = random.Random(4)
    for _ in range(10):
        A = O.g1_op("mul", G1, O.be32(rng.randrange(R)))
        c = O.compress(1, A)
        assert len(c) == 32 and O.compress(-1, c) == A
        B = O.g2_op("mul", G2, O.be32(rng.randrange(R)))
        c2 = O.compress(2, B)
        assert len(c2) == 64 and O.compress(-2, c2) == B
    assert O.compress(-1, O.compress(1, bytes(64))) == bytes(64)
    assert O.compress(-2, O.compress(2, bytes(128))) == bytes(128)
    # x = 0 has no point on y^2 = x^3 + 3 with 3 a non-residue? (3 is a QR mod p iff ...)
    bad = 0
    for x in range(1, 40):
        rhs = (x ** 3 + 3) % P
        if pow(rhs, (P - 1) // 2, P) != 1:
            bad = x
            break
    assert bad
    try:
        O.compress(-1, O.be32(bad))
        raise AssertionError("accepted an x with no curve point")
    except ValueError:
        pass
