"""A second ChaCha oracle in pure Python (test infrastructure only).

Written separately from ``chacha20_oracle.c`` from the same definition (the
cipher the paper selects in section 4.4; state layout and rounds as in
Bernstein 2008 / RFC 8439 sections 2.1-2.3).  Far too slow for anything but
a few pages; it exists so that the C oracle is checked by code that does not
share its mistakes.
"""
from __future__ import annotations

MASK = 0xFFFFFFFF


def _rotl(v: int, n: int) -> int:
    return ((v << n) & MASK) | (v >> (32 - n))


def _qr(s: list, a: int, b: int, c: int, d: int) -> None:
    s[a] = (s[a] + s[b]) & MASK
    s[d] = _rotl(s[d] ^ s[a], 16)
    s[c] = (s[c] + s[d]) & MASK
    s[b] = _rotl(s[b] ^ s[c], 12)
    s[a] = (s[a] + s[b]) & MASK
    s[d] = _rotl(s[d] ^ s[a], 8)
    s[c] = (s[c] + s[d]) & MASK
    s[b] = _rotl(s[b] ^ s[c], 7)


def _words(b: bytes) -> list:
    return [int.from_bytes(b[i:i + 4], "little") for i in range(0, len(b), 4)]


def block(key: bytes, counter: int, nonce: bytes, rounds: int = 20) -> bytes:
    assert len(key) == 32 and len(nonce) == 12 and rounds % 2 == 0
    init = _words(b"expand 32-byte k") + _words(key) + [counter & MASK] + \
        _words(nonce)
    s = list(init)
    for _ in range(rounds // 2):
        for a, b, c, d in ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14),
                           (3, 7, 11, 15)):
            _qr(s, a, b, c, d)
        for a, b, c, d in ((0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13),
                           (3, 4, 9, 14)):
            _qr(s, a, b, c, d)
    return b"".join(((x + y) & MASK).to_bytes(4, "little")
                    for x, y in zip(s, init))


def cipher_page(key: bytes, nonce: bytes, page: bytes,
                rounds: int = 20) -> bytes:
    """Page XOR with counters 0..63 (section 4.4)."""
    assert len(page) == 4096
    out = bytearray(4096)
    for j in range(64):
        ks = block(key, j, nonce, rounds)
        for i in range(64):
            out[64 * j + i] = page[64 * j + i] ^ ks[i]
    return bytes(out)
