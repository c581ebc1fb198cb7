"""The library's field, tower, curve, pairing and hash formulas, compiled for the host
(lib/libvc_hostcheck.so: the same headers the gfx950 kernels use, one lane per
element), checked against the CPU oracle on seeded random inputs.  This runs without
a GPU and catches formula mistakes before any kernel is launched."""
import ctypes as C
import hashlib
import os
import random

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC_PATH = os.path.join(ROOT, "paper_2601_03031_amd", "lib", "libvc_hostcheck.so")
P, R = O.P, O.R


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(HC_PATH):
        from paper_2601_03031_amd import build as B
        B.build_hostcheck()
    L = C.CDLL(HC_PATH)
    L.hc_h2f.argtypes = [C.c_char_p, C.c_char_p, C.c_uint64, C.c_void_p]
    L.hc_sha256.argtypes = [C.c_char_p, C.c_uint64, C.c_void_p]
    L.hc_sha256_coop.argtypes = [C.c_char_p, C.c_uint64, C.c_void_p]
    L.hc_h2f_coop.argtypes = [C.c_char_p, C.c_char_p, C.c_uint64, C.c_void_p]
    L.hc_count.restype = C.c_uint64
    return L


def buf(n):
    return C.create_string_buffer(n)


@pytest.mark.parametrize("which,mod", [(0, P), (1, R)])
def test_field_ops(hc, which, mod):
    rng = random.Random(100 + which)
    vals = [0, 1, 2, mod - 1, mod - 2, (mod + 1) // 2] + [rng.randrange(mod) for _ in range(150)]
    for a in vals:
        b = rng.randrange(mod)
        want = {0: (a + b) % mod, 1: (a - b) % mod, 2: a * b % mod, 5: a * pow(2, -1, mod) % mod}
        if a:
            want[3] = want[4] = pow(a, -1, mod)
        for op, w in want.items():
            o = buf(32)
            assert hc.hc_field(which, op, O.be32(a), O.be32(b), o) == 0
            assert int.from_bytes(o.raw, "big") == w, (which, op, a, b)


def test_fp2_ops(hc):
    rng = random.Random(7)
    for _ in range(40):
        a = (rng.randrange(P), rng.randrange(P))
        b = (rng.randrange(P), rng.randrange(P))
        want = {0: O.fp2_op("mul", a, b), 1: O.fp2_op("mul", a, a), 2: O.fp2_op("inv", a),
                3: O.fp2_op("mul", a, (9, 1))}  # xi = 9 + i
        for op, w in want.items():
            o = buf(64)
            assert hc.hc_fp2(op, O.be32(a[0]) + O.be32(a[1]), O.be32(b[0]) + O.be32(b[1]), o) == 0
            assert (int.from_bytes(o.raw[:32], "big"), int.from_bytes(o.raw[32:], "big")) == w, oop


def rand12(rng):
    return b"".join(O.be32(rng.randrange(P)) for _ in range(12))


def frob(f):
    """f^p by generic powers: p = (r - 1) + 1 + 6u^2, each exponent below r"""
    u = 0x44E992B44A6909F1
    t = O.fp12_op("mul", O.fp12_op("pow", f, O.be32(R - 1)), f)
    return O.fp12_op("mul", t, O.fp12_op("pow", f, O.be32(6 * u * u)))


def test_fp12_ops(hc):
    rng = random.Random(8)
    for _ in range(4):
        f, g = rand12(rng), rand12(rng)
        f1 = frob(f)
        f2 = frob(f1)
        want = {0: O.fp12_op("mul", f, g), 2: O.fp12_op("inv", f), 4: f1, 5: f2, 6: frob(f2)}
        for op, w in want.items():
            o = buf(384)
            assert hc.hc_fp12(op, f, g, o) == 0
            assert o.raw == w, op
        o = buf(384)
        hc.hc_fp12(1, f, g, o)
        assert o.raw == O.fp12_op("mul", f, f)
    f = rand12(rng)
    o = buf(384)
    hc.hc_fp12(3, f, f, o)
    assert o.raw == O.fp12_op("final_exp", f)


def test_cyclotomic_ops(hc):
    """Granger-Scott squaring and f^u agree with generic arithmetic on cyclotomic elements."""
    rng = random.Random(9)
    g = O.fp12_op("final_exp", rand12(rng))  # an element of order r lies in the cyclotomic subgroup
    o = buf(384)
    hc.hc_fp12(7, g, g, o)
    assert o.raw == O.fp12_op("mul", g, g)
    o = buf(384)
    hc.hc_fp12(8, g, g, o)
    u = 0x44E992B44A6909F1
    assert o.raw == O.fp12_op("pow", g, O.be32(u))


def test_group_ops(hc):
    rng = random.Random(10)
    g1, g2 = O.generators()
    for _ in range(4):
        k = rng.randrange(R)
        o = buf(64)
        hc.hc_g1(2, g1, O.be32(k), o)
        assert o.raw == O.g1_op("mul", g1, O.be32(k))
        o = buf(128)
        hc.hc_g2(2, g2, O.be32(k), o)
        assert o.raw == O.g2_op("mul", g2, O.be32(k))
    A, B = O.g1_op("mul", g1, O.be32(5)), O.g1_op("mul", g1, O.be32(7))
    A2, B2 = O.g2_op("mul", g2, O.be32(5)), O.g2_op("mul", g2, O.be32(7))
    for op in (0, 3):
        for X, Y in ((A, B), (A, A), (A, O.g1_op("neg", A))):
            o = buf(64)
            hc.hc_g1(op, X, Y, o)
            assert o.raw == O.g1_op("add", X, Y)
        for X, Y in ((A2, B2), (A2, A2), (A2, O.g2_op("neg", A2))):
            o = buf(128)
            hc.hc_g2(op, X, Y, o)
            assert o.raw == O.g2_op("add", X, Y)
    o = buf(64)
    hc.hc_g1(1, A, A, o)
    assert o.raw == O.g1_op("add", A, A)
    o = buf(128)
    hc.hc_g2(4, A2, A2, o)
    assert o.raw == O.g2_op("frobenius", A2)


def test_pairing(hc):
    g1, g2 = O.generators()
    A = O.g1_op("mul", g1, O.be32(1234567))
    B = O.g2_op("mul", g2, O.be32(7654321))
    o = buf(384)
    hc.hc_pairing(A, B, o)
    assert o.raw == O.pairing([A], [B])


def test_hashes(hc):
    rng = random.Random(11)
    for n in (0, 1, 3, 55, 56, 63, 64, 65, 200, 1000):
        msg = bytes(rng.randrange(256) for _ in range(n))
        o = buf(32)
        hc.hc_sha256(msg, len(msg), o)
        assert o.raw == hashlib.sha256(msg).digest()
        o = buf(32)
        hc.hc_sha256_coop(msg, len(msg), o)
        assert o.raw == hashlib.sha256(msg).digest()
        for dst in ("FLEXPROOFS-V1-FC-X", "FLEXPROOFS-V1-RHO"):
            o = buf(32)
            hc.hc_h2f(dst.encode(), msg, len(msg), o)
            assert int.from_bytes(o.raw, "big") == O.hash_to_fr(dst, msg)
    # the cooperative form of the challenge kernels, over lengths that put the suffix and
    # padding in one or two final blocks
    for n in list(range(0, 80)) + [896, 928, 960, 992, 1000, 1024]:
        msg = bytes(rng.randrange(256) for _ in range(n))
        for dst in ("FLEXPROOFS-V1-FC-X", "FLEXPROOFS-V1-FC-Z"):
            o = buf(32)
            hc.hc_h2f_coop(dst.encode(), msg, len(msg), o)
            assert int.from_bytes(o.raw, "big") == O.hash_to_fr(dst, msg), (n, dst)
    m, c = bytes(range(32)), bytes(range(64, 128))
    o = buf(32)
    hc.hc_merkle_leaf(m, c, o)
    assert o.raw == hashlib.sha256(b"\x00" + m + c).digest()
    o = buf(32)
    hc.hc_merkle_node(m, c[:32], o)
    assert o.raw == hashlib.sha256(b"\x01" + m + c[:32]).digest()


def test_engine_programs_on_host(hc):
    """The engine's generated programs, run through the host model of its interpreter
    (same operation decoder and arithmetic as the GPU kernels): Miller loop then the
    oracle's final exponentiation equals the oracle's pairing; the engine's final
    exponentiation and F_p12 product equal the oracle's."""
    rng = random.Random(12)
    g1, g2 = O.generators()
    for _ in range(2):
        A = O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))
        B = O.g2_op("mul", g2, O.be32(rng.randrange(1, R)))
        f = buf(384)
        assert hc.hc_slp_miller(A, B, f) == 0
        assert O.fp12_op("final_exp", f.raw) == O.pairing([A], [B])
    for _ in range(3):
        x, y = rand12(rng), rand12(rng)
        o = buf(384)
        hc.hc_slp_f12(1, x, y, o)
        assert o.raw == O.fp12_op("mul", x, y)
        hc.hc_slp_f12(0, x, y, o)
        assert o.raw == O.fp12_op("final_exp", x)


def test_engine_lane_arithmetic(hc):
    """Radix-2^29 lane arithmetic of the engine on edge and random inputs below 2p
    (slot values are almost reduced): linear combinations with coefficients up to the
    product-operand scale (32 x 15) and Montgomery products with R = 2^261."""
    rng = random.Random(13)
    edge = [0, 1, P - 1, P, P + 1, 2 * P - 1, (1 << 254) - 1 if (1 << 254) - 1 < 2 * P else 2 * P - 2]
    for trial in range(3000):
        n = rng.randrange(1, 7)
        kmax = 480 if trial % 2 else 15
        ks = [rng.randrange(-kmax, kmax + 1) for _ in range(n)]
        if trial % 7 == 0:
            ks = [rng.choice([-kmax, kmax]) for _ in range(n)]
        xs = [rng.choice(edge) if rng.random() < 0.3 else rng.randrange(2 * P) for _ in range(n)]
        karr = (C.c_int * 6)(*ks)
        blob = b"".join(x.to_bytes(32, "big") for x in xs)
        o = buf(32)
        hc.hc_slp_lane(0, n, karr, blob, o)
        assert int.from_bytes(o.raw, "big") == sum(k * x for k, x in zip(ks, xs)) % P, (ks, xs)
        hc.hc_slp_lane(2, n, karr, blob, o)
        raw = int.from_bytes(o.raw, "big")
        assert raw < 2 * P and raw % P == sum(k * x for k, x in zip(ks, xs)) % P
    # full-width sums: up to 16 terms, coefficient magnitudes summing to the encoder's limit
    # (32767), the columns started at one offset (a product factor) or at two (a 16-term sum)
    for trial in range(3000):
        n = rng.randrange(1, 17)
        budget = 32767
        ks = []
        for i in range(n):
            c = rng.randrange(0, min(budget, 127 * 32) + 1) if trial % 3 else min(budget, 127 * 32)
            budget -= c
            ks.append(c if rng.random() < 0.5 else -c)
        xs = [rng.choice(edge) if rng.random() < 0.3 else rng.randrange(2 * P) for _ in range(n)]
        karr = (C.c_int * n)(*ks)
        blob = b"".join(x.to_bytes(32, "big") for x in xs)
        want = sum(k * x for k, x in zip(ks, xs)) % P
        for op in (2, 4):
            o = buf(32)
            hc.hc_slp_lane(op, n, karr, blob, o)
            raw = int.from_bytes(o.raw, "big")
            assert raw < 2 * P and raw % P == want, (op, ks, xs)
        o = buf(32)
        hc.hc_slp_lane(3, n, karr, blob, o)
        assert int.from_bytes(o.raw, "big") == want
    rinv = pow(1 << 261, -1, P)
    for trial in range(2000):
        a = rng.choice(edge) if trial % 5 == 0 else rng.randrange(2 * P)
        b = rng.choice(edge) if trial % 3 == 0 else rng.randrange(2 * P)
        o = buf(32)
        hc.hc_slp_lane(1, 2, None, a.to_bytes(32, "big") + b.to_bytes(32, "big"), o)
        assert int.from_bytes(o.raw, "big") == a * b * rinv % P, (a, b)


def test_gls_decomposition(hc):
    """k = sum_j k_j lam^j (mod r) with lam = p mod r (the eigenvalue of the twist
    Frobenius on G2, pinned against the oracle's Frobenius) and |k_j| < 2^65."""
    g1, g2 = O.generators()
    lam = P % R
    Q = O.g2_op("mul", g2, O.be32(777))
    assert O.g2_op("frobenius", Q) == O.g2_op("mul", Q, O.be32(lam))
    rng = random.Random(14)
    for k in [0, 1, 2, R - 1, R - 2, (R - 1) // 2, 1 << 200] + [rng.randrange(R) for _ in range(3000)]:
        o = buf(64)
        nb = C.c_uint32()
        hc.hc_gls(k.to_bytes(32, "big"), o, C.byref(nb))
        kj = [int.from_bytes(o.raw[16 * j:16 * j + 16], "little", signed=True) for j in range(4)]
        assert (sum(kj[j] * pow(lam, j, R) for j in range(4)) - k) % R == 0, k
        assert max(abs(x) for x in kj) < 2**65
        assert nb.value == max(abs(x) for x in kj).bit_length()


def test_g2_scalar_mul_engine(hc):
    """k Q + A through the engine's host model (GLS split, signed table, exact handling
    of equal and opposite points) against the oracle's group law."""
    g1, g2 = O.generators()
    rng = random.Random(15)
    ident = bytes(128)
    cases = []
    for _ in range(4):
        Q = O.g2_op("mul", g2, O.be32(rng.randrange(1, R)))
        A = O.g2_op("mul", g2, O.be32(rng.randrange(1, R)))
        cases.append((Q, rng.randrange(R), A))
    Q = O.g2_op("mul", g2, O.be32(12345))
    k = rng.randrange(1, R)
    kQ = O.g2_op("mul", Q, O.be32(k))
    cases += [(Q, 0, None), (Q, 1, None), (Q, R - 1, None), (ident, 5, None), (Q, k, ident),
              (Q, k, kQ), (Q, k, O.g2_op("neg", kQ)), (Q, 0, kQ), (Q, k, None)]
    for Qb, k, Ab in cases:
        o = buf(128)
        assert hc.hc_g2_mul(Qb, k.to_bytes(32, "big"), Ab, o) == 0
        want = O.g2_op("mul", Qb, O.be32(k)) if Qb != ident else ident
        if Ab is not None:
            want = O.g2_op("add", want, Ab)
        assert o.raw == want, (k,)


def test_g1_glv(hc):
    """phi(x, y) = (beta x, y) is multiplication by the chosen cube root of unity lam on
    G1 (pinned against the oracle); k = k_0 + k_1 lam with |k_j| < 2^128; k P through the
    split equals the oracle's k P, including k = 0, 1, r - 1 and the identity."""
    g1, g2 = O.generators()
    beta = 0x59E26BCEA0D48BACD4F263F1ACDB5C4F5763473177FFFFFE
    lam = 0xB3C4D79D41A917585BFC41088D8DAAA78B17EA66B99C90DD
    x, y = int.from_bytes(g1[:32], "big"), int.from_bytes(g1[32:], "big")
    assert O.g1_op("mul", g1, O.be32(lam)) == O.be32(beta * x % P) + O.be32(y)
    rng = random.Random(16)
    for k in [0, 1, 2, R - 1, R - 2, (R - 1) // 2] + [rng.randrange(R) for _ in range(60)]:
        Pt = O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))
        o, dec = buf(64), buf(40)
        hc.hc_g1_mul_glv(Pt, k.to_bytes(32, "big"), o, dec)
        assert o.raw == O.g1_op("mul", Pt, O.be32(k)), k
        w = [int.from_bytes(dec.raw[4 * i:4 * i + 4], "little") for i in range(10)]
        k0 = w[0] | w[1] << 32 | w[2] << 64 | w[3] << 96
        k1 = w[4] | w[5] << 32 | w[6] << 64 | w[7] << 96
        k0 = -k0 if w[8] & 1 else k0
        k1 = -k1 if w[8] & 2 else k1
        assert (k0 + k1 * lam - k) % R == 0 and max(abs(k0), abs(k1)) < 2**128
    o = buf(64)
    hc.hc_g1_mul_glv(bytes(64), (12345).to_bytes(32, "big"), o, None)
    assert o.raw == bytes(64)


@pytest.mark.parametrize("which,mod", [(0, P), (1, R)])
def test_bingcd_inverse(hc, which, mod):
    """The batched binary GCD itself (without the exponentiation fallback) against
    Python's modular inverse, with its round count within the 2 len(m) - 1 step bound."""
    rng = random.Random(300 + which)
    vals = [1, 2, 3, mod - 1, mod - 2, (mod + 1) // 2, 1 << 200, (1 << 253) + 1, (1 << 64) - 1, 1 << 64]
    vals += [rng.randrange(1, mod) for _ in range(400)] + [rng.randrange(1, 1 << 70) for _ in range(50)]
    rounds = C.c_int(0)
    worst = 0
    for x in vals:
        o = buf(32)
        assert hc.hc_bingcd(which, O.be32(x), o, C.byref(rounds)) == 1, x
        assert int.from_bytes(o.raw, "big") == pow(x, -1, mod), x
        worst = max(worst, rounds.value)
    assert worst <= -(-(2 * mod.bit_length() - 1) // 30), worst


def test_gt_pow_cyc(hc):
    """g^k on the engine through k = sum_j k_j lam^j and the Frobenius powers of g equals
    the oracle's g^k for pairing values g (of order r), including k = 0, 1, r - 1."""
    g1, g2 = O.generators()
    rng = random.Random(23)
    for trial in range(4):
        Pt = O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))
        Qt = O.g2_op("mul", g2, O.be32(rng.randrange(1, R)))
        g = O.pairing([Pt], [Qt])
        ks = [0, 1, R - 1, 2] if trial == 0 else [rng.randrange(R) for _ in range(5)]
        for k in ks:
            o = buf(384)
            assert hc.hc_gt_pow_cyc(g, k.to_bytes(32, "big"), o) == 0
            assert o.raw == O.fp12_op("pow", g, O.be32(k)), k


def test_g1_scalar_mul_engine(hc):
    """k P + A through the engine's host model (GLV split, signed table, exact handling of
    equal and opposite points, also inside the window loop) against the oracle's group law."""
    g1, g2 = O.generators()
    rng = random.Random(25)
    ident = bytes(64)
    cases = []
    for _ in range(6):
        Pt = O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))
        A = O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))
        cases.append((Pt, rng.randrange(R), A))
        cases.append((Pt, rng.randrange(R), None))
    Pt = O.g1_op("mul", g1, O.be32(777))
    k = rng.randrange(1, R)
    kP = O.g1_op("mul", Pt, O.be32(k))
    cases += [(Pt, 0, None), (Pt, 1, None), (Pt, 2, None), (Pt, R - 1, None), (ident, 5, None), (Pt, k, ident),
              (Pt, k, kP), (Pt, k, O.g1_op("neg", kP)), (Pt, 0, kP), (Pt, 5, None), (Pt, 16, None)]
    for Pb, k, Ab in cases:
        o = buf(64)
        assert hc.hc_g1_mul_engine(Pb, k.to_bytes(32, "big"), Ab, o) == 0
        want = O.g1_op("mul", Pb, O.be32(k)) if Pb != ident else ident
        if Ab is not None:
            want = O.g1_op("add", want, Ab)
        assert o.raw == want, (k,)


def test_split_multiplications(hc):
    """The time-split forms used to run a multiplication in parallel parts: k P as
    sum_t chunk_t(k) (2^{32 t} P) over the GLV split, and g^k as prod_t of the Frobenius-split
    chunks of g^{2^{16 t}}; both equal the oracle's k P and g^k."""
    g1, g2 = O.generators()
    rng = random.Random(27)
    for k in [0, 1, R - 1, 2**32, 2**64 + 5] + [rng.randrange(R) for _ in range(12)]:
        Pt = O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))
        o = buf(64)
        assert hc.hc_g1_mul_split(Pt, k.to_bytes(32, "big"), o) == 0
        assert o.raw == O.g1_op("mul", Pt, O.be32(k)), k
    for trial in range(2):
        g = O.pairing([O.g1_op("mul", g1, O.be32(rng.randrange(1, R)))], [g2])
        for k in ([0, 1, R - 1, 2**16] if trial == 0 else [rng.randrange(R) for _ in range(4)]):
            o = buf(384)
            assert hc.hc_gt_pow_split(g, k.to_bytes(32, "big"), o) == 0
            assert o.raw == O.fp12_op("pow", g, O.be32(k)), k


@pytest.mark.parametrize("grp", ["g1", "g2"])
def test_split_fold(hc, grp):
    """The split fold exactly as the kernels run it (multiples by the engine's doublings,
    four chunked multiplications, their sum and A through the engine's Jacobian and
    mixed additions): A + k P against the oracle, including the cases where partial
    sums meet (A = k P doubles, A = -k P gives the identity) and identity inputs."""
    g1, g2 = O.generators()
    op, gen, size = (O.g1_op, g1, 64) if grp == "g1" else (O.g2_op, g2, 128)
    fn = hc.hc_fold_split_g1 if grp == "g1" else hc.hc_fold_split_g2
    rng = random.Random(41 if grp == "g1" else 42)
    inf = bytes(size)
    cases = []
    for _ in range(5):
        Pt = op("mul", gen, O.be32(rng.randrange(1, R)))
        cases.append((Pt, rng.randrange(R), op("mul", gen, O.be32(rng.randrange(1, R)))))
    Pt = op("mul", gen, O.be32(rng.randrange(1, R)))
    k = rng.randrange(R)
    kP = op("mul", Pt, O.be32(k))
    cases += [(Pt, k, kP), (Pt, k, op("neg", kP)), (Pt, 0, kP), (Pt, k, inf), (inf, k, kP), (Pt, 1, inf),
              (Pt, R - 1, Pt), (Pt, 2**16 + 1, inf), (Pt, 2**64, inf)]
    for Pt, k, A in cases:
        o = buf(size)
        assert fn(Pt, k.to_bytes(32, "big"), A, o) == 0
        assert o.raw == op("add", op("mul", Pt, O.be32(k)), A), (k,)


def wide_raw(hc, which, op, a, b):
    o = buf(32)
    assert hc.hc_wide_raw(which, op, a.to_bytes(32, "little"), b.to_bytes(32, "little"), o) == 0
    return int.from_bytes(o.raw, "little")


@pytest.mark.parametrize("which,mod", [(0, P), (1, R)])
def test_wide_layout_output_range(hc, which, mod):
    """The 8-lane field layout's operations (lane model of field_wide.hpp: limb broadcasts, limb
    shifts, ballot carry-lookahead) on raw Montgomery limbs at the extremes of their inputs.
    With canonical inputs (below the modulus) every result is canonical and correct; products
    stay canonical and correct for inputs up to twice the modulus.  So values built only from
    these operations on canonical inputs (the wide Miller loop's F_p12 coefficients from
    canonical affine points) are canonical."""
    rng = random.Random(41 + which)
    rinv = pow(1 << 256, -1, mod)
    canon = [0, 1, 2, mod - 1, mod - 2, mod >> 1, (1 << 32) - 1, 1 << 32, (1 << 224) + 5] + \
        [rng.randrange(mod) for _ in range(200)]
    for i, a in enumerate(canon):
        b = canon[(7 * i + 3) % len(canon)]
        m = wide_raw(hc, which, 0, a, b)
        assert m < mod and m == a * b * rinv % mod, (a, b)
        s = wide_raw(hc, which, 1, a, b)
        assert s < mod and s == (a + b) % mod, (a, b)
        d = wide_raw(hc, which, 2, a, b)
        assert d < mod and d == (a - b) % mod, (a, b)
    below2 = [mod, mod + 1, 2 * mod - 1, 2 * mod - 2] + [rng.randrange(mod, 2 * mod) for _ in range(200)]
    for i, a in enumerate(below2):
        for b in (below2[(5 * i + 1) % len(below2)], canon[i % len(canon)]):
            m = wide_raw(hc, which, 0, a, b)
            assert m < mod and m == a * b * rinv % mod, (a, b)
