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


def test_expand_message_xmd_rfc9380_vectors():
    dst = b"QUUX-V01-CS02-with-expander-SHA256-128"
    rows = [ln.strip() for ln in open(os.path.join(HERE, "golden", "rfc9380_xmd_sha256.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert rows
    for row in rows:
        msg_hex, out_hex = row.split("|")
        assert O.expand_message_xmd(bytes.fromhex(msg_hex), dst, 32).hex() == out_hex


def test_hash_to_field_is_48_byte_reduction():
    for msg in [b"", b"abc", bytes(range(200))]:
        u = O.expand_message_xmd(msg, b"FLEXPROOFS-V1-FC-X", 48)
        assert O.hash_to_fr("FLEXPROOFS-V1-FC-X", msg) == int.from_bytes(u, "big") % O.R
    # distinct domain tags give independent outputs
    assert O.hash_to_fr("A", b"x") != O.hash_to_fr("B", b"x")
