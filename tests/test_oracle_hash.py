"""Pins for the oracle's SHA-256 (hashlib), expand_message_xmd (RFC 9380 vectors)
and hash-to-field reduction."""
import hashlib
import os

import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("n", [0, 1, 3, 55, 56, 57, 63, 64, 65, 119, 120, 128, 1000, 4097])
def test_sha256_matches_hashlib(n):
    msg = bytes((i * 131 + 7) & 0xFF for i in range(n))
    assert O.sha256(msg) == hashlib.sha256(msg).digest()


def _golden_msg(text):
    # "q128_*128" stands for the prefix "q128_" followed by 128 copies of its first letter
    if "*" in text:
        prefix, count = text.split("*")
        return (prefix + prefix[0] * int(count)).encode()
    return text.encode()


def test_expand_message_xmd_rfc9380_vectors():
    dst = b"QUUX-V01-CS02-with-expander-SHA256-128"
    rows = [ln.strip() for ln in open(os.path.join(HERE, "golden", "rfc9380_xmd_sha256.txt"))
            if ln.strip() and not ln.startswith("#")]
    lens = set()
    for row in rows:
        len_hex, msg, out_hex = row.split("|")
        n = int(len_hex, 16)
        lens.add(n)
        assert O.expand_message_xmd(_golden_msg(msg), dst, n).hex() == out_hex
    # both the one-block branch and the chained multi-block branch are pinned
    assert lens == {0x20, 0x80}


def test_expand_message_xmd_prefix_property():
    # the 48-byte output of hash-to-field is the chained branch with two blocks; its blocks are
    # those of no other length (len_in_bytes is hashed into b_0), so check it is not a prefix
    dst = b"QUUX-V01-CS02-with-expander-SHA256-128"
    u48 = O.expand_message_xmd(b"abc", dst, 48)
    u128 = O.expand_message_xmd(b"abc", dst, 128)
    assert len(u48) == 48 and u48 != u128[:48]


def test_hash_to_field_is_48_byte_reduction():
    for msg in [b"", b"abc", bytes(range(200))]:
        u = O.expand_message_xmd(msg, b"FLEXPROOFS-V1-FC-X", 48)
        assert O.hash_to_fr("FLEXPROOFS-V1-FC-X", msg) == int.from_bytes(u, "big") % O.R
    # distinct domain tags give independent outputs
    assert O.hash_to_fr("A", b"x") != O.hash_to_fr("B", b"x")
