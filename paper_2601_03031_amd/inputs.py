"""Seeded synthetic inputs for FlexProofs commit/open-all workloads.

This module only draws random numbers; it holds none of the scheme's arithmetic and
is the one piece shared by the GPU path's tests, the oracle's tests and the
benchmark.  The paper states no input distribution, so the workloads use:

* full-width entries: uniform in [0, r) by rejection sampling of 254-bit draws
  (numpy PCG64, four 64-bit words per draw, top word masked to 62 bits);
* 32-bit entries: uniform uint32, read as field elements m_i < 2^32.

Entries are returned as little-endian 32-byte canonical encodings (N x 32 bytes),
the layout the library and the oracle both take.
"""
from __future__ import annotations

import numpy as np

# BN254 scalar field order (also the group order of G1, G2, G_T)
R = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
_R_WORDS = np.array([(R >> (64 * k)) & (2**64 - 1) for k in range(4)], dtype=np.uint64)

TRAPDOOR_SEED = b"FP-trapdoor-v1".ljust(32, b"\0")


def _below_r(words: np.ndarray) -> np.ndarray:
    """words: (n, 4) little-endian uint64 limbs; True where the value is < r."""
    lt = np.zeros(len(words), dtype=bool)
    eq = np.ones(len(words), dtype=bool)
    for k in (3, 2, 1, 0):
        lt |= eq & (words[:, k] < _R_WORDS[k])
        eq &= words[:, k] == _R_WORDS[k]
    return lt


def field_entries(n: int, seed: int) -> np.ndarray:
    """n uniform elements of [0, r) as an (n, 4) uint64 little-endian limb array."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((0, 4), dtype=np.uint64)
    while len(out) < n:
        need = max(16, int((n - len(out)) * 1.4))
        w = rng.integers(0, 2**64, size=(need, 4), dtype=np.uint64)
        w[:, 3] &= np.uint64((1 << 62) - 1)
        out = np.concatenate([out, w[_below_r(w)]])
    return np.ascontiguousarray(out[:n])


def u32_entries(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2**32, size=n, dtype=np.uint32)


def u32_to_limbs(v: np.ndarray) -> np.ndarray:
    out = np.zeros((len(v), 4), dtype=np.uint64)
    out[:, 0] = v.astype(np.uint64)
    return out


def limbs_to_bytes(w: np.ndarray) -> bytes:
    return np.ascontiguousarray(w, dtype="<u8").tobytes()


def limbs_to_ints(w: np.ndarray) -> list:
    return [int(a) | (int(b) << 64) | (int(c) << 128) | (int(d) << 192) for a, b, c, d in w]


def entries(n: int, seed: int, bits: int = 256) -> np.ndarray:
    """(n, 4) limb array: full-width (bits=256) or 32-bit entries (bits=32)."""
    if bits == 32:
        return u32_to_limbs(u32_entries(n, seed))
    return field_entries(n, seed)


def device_entries(n: int, seed: int, device: str = "cuda", chunk: int = 1 << 22):
    """n full-width entries drawn on the device (for sizes where drawing on the host is slow):
    a seeded torch generator, eight 32-bit words per entry with the top word below 2^29, so
    the entries are uniform in [0, 2^253), all below r.  Drawn in chunks of `chunk` entries.
    Returns an (n * 32)-byte uint8 tensor of little-endian encodings."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((n, 8), dtype=torch.int32, device=device)
    for lo in range(0, n, chunk):
        c = min(chunk, n - lo)
        w = torch.randint(0, 2**32, (c, 8), generator=g, device=device, dtype=torch.int64)
        w[:, 7] &= (1 << 29) - 1
        out[lo:lo + c] = w.to(torch.int32)  # the low 32 bits of each word
        del w
    return out.view(torch.uint8).reshape(-1)
