"""A second Salsa20 oracle in pure Python (test infrastructure only).

Written separately from the C oracle's Salsa20, from Bernstein's definition
("The Salsa20 family of stream ciphers", 2008): the engine's second cipher,
behind the same page interface as ChaCha (the paper's modular cipher,
sections 1 and 6).  Block j of a page uses the 64-bit nonce = page nonce
bytes 0..7 and the 64-bit block counter = page nonce word 2 * 2^32 + j.
Far too slow for anything but a few pages.
"""
from __future__ import annotations

MASK = 0xFFFFFFFF

# positions of the four constant words, the eight key words, the two nonce
# words and the two counter words in the 4x4 state
CONST_AT = (0, 5, 10, 15)
KEY_AT = (1, 2, 3, 4, 11, 12, 13, 14)
NONCE_AT = (6, 7)
COUNTER_AT = (8, 9)

# each quarter round updates its second, third, fourth, then first word
COLUMNS = ((0, 4, 8, 12), (5, 9, 13, 1), (10, 14, 2, 6), (15, 3, 7, 11))
ROWS = ((0, 1, 2, 3), (5, 6, 7, 4), (10, 11, 8, 9), (15, 12, 13, 14))


def _rotl(v: int, n: int) -> int:
    v &= MASK
    return ((v << n) & MASK) | (v >> (32 - n))


def _quarter(s: list, y0: int, y1: int, y2: int, y3: int) -> None:
    s[y1] ^= _rotl(s[y0] + s[y3], 7)
    s[y2] ^= _rotl(s[y1] + s[y0], 9)
    s[y3] ^= _rotl(s[y2] + s[y1], 13)
    s[y0] ^= _rotl(s[y3] + s[y2], 18)


def _le(b: bytes, i: int) -> int:
    return int.from_bytes(b[4 * i:4 * i + 4], "little")


def block(key: bytes, nonce8: bytes, counter: int, rounds: int = 20) -> bytes:
    assert len(key) == 32 and len(nonce8) == 8 and rounds % 2 == 0
    init = [0] * 16
    sigma = b"expand 32-byte k"
    for i, at in enumerate(CONST_AT):
        init[at] = _le(sigma, i)
    for i, at in enumerate(KEY_AT):
        init[at] = _le(key, i)
    for i, at in enumerate(NONCE_AT):
        init[at] = _le(nonce8, i)
    init[COUNTER_AT[0]] = counter & MASK
    init[COUNTER_AT[1]] = (counter >> 32) & MASK
    s = list(init)
    for _ in range(rounds // 2):
        for q in COLUMNS:
            _quarter(s, *q)
        for q in ROWS:
            _quarter(s, *q)
    return b"".join(((x + y) & MASK).to_bytes(4, "little")
                    for x, y in zip(s, init))


def cipher_page(key: bytes, nonce12: bytes, page: bytes,
                rounds: int = 20) -> bytes:
    """Page XOR with Salsa20 blocks j = 0..63 (counter = word 2 * 2^32 + j)."""
    assert len(page) == 4096 and len(nonce12) == 12
    high = int.from_bytes(nonce12[8:12], "little") << 32
    out = bytearray(4096)
    for j in range(64):
        ks = block(key, nonce12[:8], high + j, rounds)
        for i in range(64):
            out[64 * j + i] = page[64 * j + i] ^ ks[i]
    return bytes(out)
