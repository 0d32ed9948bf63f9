"""Per-page nonces of the oracle (test infrastructure only).

The paper (section 4.4) builds the 128-bit seed value of every keystream
block from the page's virtual address, the client's PID and the block counter
0..63, without fixing an order or byte layout.  The reading used throughout
this project: word 12 of the state is the block counter, and the 96-bit page
nonce (words 13..15) is the little-endian 64-bit virtual address followed by
the little-endian 32-bit PID.  For a run of pages that are ``stride`` bytes
apart starting at ``base`` the nonce of page i is therefore
LE64(base + i*stride mod 2**64) || LE32(tag).
"""
from __future__ import annotations

import struct

import numpy as np


def nonce_linear(index: int, base: int, stride: int, tag: int) -> bytes:
    """The 12 nonce bytes of page ``index`` of a linear run."""
    va = (base + index * stride) % (1 << 64)
    return struct.pack("<QI", va, tag % (1 << 32))


def nonces_linear(n_pages: int, base: int, stride: int, tag: int) -> np.ndarray:
    """(n_pages, 12) uint8 array of linear-run nonces, built page by page for
    small runs and with plain numpy integer arithmetic for large ones."""
    out = np.empty((n_pages, 12), dtype=np.uint8)
    if n_pages <= 4096:
        for i in range(n_pages):
            out[i] = np.frombuffer(nonce_linear(i, base, stride, tag),
                                   dtype=np.uint8)
        return out
    idx = np.arange(n_pages, dtype=np.uint64)
    with np.errstate(over="ignore"):
        va = np.uint64(base % (1 << 64)) + idx * np.uint64(stride % (1 << 64))
    out[:, 0:8] = va.astype("<u8").view(np.uint8).reshape(n_pages, 8)
    out[:, 8:12] = np.frombuffer(struct.pack("<I", tag % (1 << 32)),
                                 dtype=np.uint8)
    return out
