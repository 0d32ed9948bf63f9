"""CPU oracle for the MemShield page cipher and its extensions.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP engine and its Python binding) never imports, loads or calls it, and this
package imports nothing from the product package.  Inputs reach both sides
from the seeded generators in ``paper_2004_09252_amd.workloads``, which hold
none of the method's arithmetic.

Contents:
  * ``chacha20_oracle.c`` - scalar C ChaCha block function and page XOR
    (paper section 4.4), and the Salsa20 block function and page XOR of the
    engine's second cipher, built with gcc into ``_build/liboracle_chacha.so``
    and called through ctypes;
  * ``chacha_py`` and ``salsa_py`` - second, pure-Python ChaCha and Salsa20
    written separately, for tiny inputs;
  * ``nonces`` - the page-nonce readings of the paper's 128-bit seed value;
  * ``window_sim`` - the sliding-window decrypt-on-fault model (sections 4.2,
    4.3);
  * ``mlp_ref`` - the numpy float64 reference of the page-access predictor.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

PAGE_BYTES = 4096
BLOCK_BYTES = 64
NONCE_BYTES = 12
KEY_BYTES = 32

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chacha20_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle_chacha.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no intrinsics)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            u8p = ctypes.c_void_p
            lib.oracle_chacha_block.argtypes = [u8p, ctypes.c_uint32, u8p,
                                                ctypes.c_int, u8p]
            lib.oracle_chacha_block.restype = None
            lib.oracle_cipher_pages.argtypes = [u8p, u8p, ctypes.c_int, u8p,
                                                u8p, ctypes.c_uint64]
            lib.oracle_cipher_pages.restype = None
            lib.oracle_cipher_pages_mt.argtypes = [u8p, u8p, ctypes.c_int, u8p,
                                                   u8p, ctypes.c_uint64,
                                                   ctypes.c_int]
            lib.oracle_cipher_pages_mt.restype = ctypes.c_int
            lib.oracle_salsa_block.argtypes = [u8p, u8p, ctypes.c_uint64,
                                               ctypes.c_int, u8p]
            lib.oracle_salsa_block.restype = None
            lib.oracle_cipher_pages_with.argtypes = [
                ctypes.c_int, u8p, u8p, ctypes.c_int, u8p, u8p,
                ctypes.c_uint64]
            lib.oracle_cipher_pages_with.restype = None
            lib.oracle_cipher_pages_mt_with.argtypes = [
                ctypes.c_int, u8p, u8p, ctypes.c_int, u8p, u8p,
                ctypes.c_uint64, ctypes.c_int]
            lib.oracle_cipher_pages_mt_with.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _as_u8(a, shape_tail=None) -> np.ndarray:
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a


def chacha_block(key, counter: int, nonce, rounds: int = 20) -> bytes:
    """One 64-byte keystream block (section 4.4: 384-bit seed -> 512 bits)."""
    k = _as_u8(key)
    n = _as_u8(nonce)
    assert k.size == KEY_BYTES and n.size == NONCE_BYTES
    assert rounds > 0 and rounds % 2 == 0
    out = np.zeros(BLOCK_BYTES, dtype=np.uint8)
    _load().oracle_chacha_block(_ptr(k), counter & 0xFFFFFFFF, _ptr(n),
                                rounds, _ptr(out))
    return out.tobytes()


CIPHERS = {"chacha": 0, "salsa": 1}


def salsa_block(key, nonce8, counter: int, rounds: int = 20) -> bytes:
    """One 64-byte Salsa20 keystream block for a 64-bit nonce and a 64-bit
    block counter (the engine's second cipher)."""
    k = _as_u8(key)
    n = _as_u8(nonce8)
    assert k.size == KEY_BYTES and n.size == 8
    assert rounds > 0 and rounds % 2 == 0
    out = np.zeros(BLOCK_BYTES, dtype=np.uint8)
    _load().oracle_salsa_block(_ptr(k), _ptr(n), counter & (2**64 - 1),
                               rounds, _ptr(out))
    return out.tobytes()


def cipher_pages(key, nonces, data, rounds: int = 20, threads: int = 1,
                 out: np.ndarray | None = None,
                 cipher: str = "chacha") -> np.ndarray:
    """XOR each 4096-byte page with its 64 keystream blocks (section 4.4).

    ``nonces`` is (n_pages, 12) uint8, ``data`` is (n_pages, 4096) uint8 (or
    anything reshapeable to it).  Encryption and decryption are the same call.
    ``cipher`` is "chacha" (the paper's) or "salsa" (Salsa20: nonce = page
    nonce bytes 0..7, block counter = page nonce word 2 * 2^32 + j).
    """
    k = _as_u8(key)
    assert k.size == KEY_BYTES
    d = _as_u8(data).reshape(-1, PAGE_BYTES)
    n = _as_u8(nonces).reshape(-1, NONCE_BYTES)
    assert n.shape[0] == d.shape[0], "one nonce per page"
    assert rounds > 0 and rounds % 2 == 0
    if out is None:
        out = np.empty_like(d)
    else:
        assert out.dtype == np.uint8 and out.flags.c_contiguous
        assert out.size == d.size
    lib = _load()
    cid = CIPHERS[cipher]
    if threads <= 1:
        lib.oracle_cipher_pages_with(cid, _ptr(k), _ptr(n), rounds, _ptr(d),
                                     _ptr(out), d.shape[0])
    else:
        lib.oracle_cipher_pages_mt_with(cid, _ptr(k), _ptr(n), rounds,
                                        _ptr(d), _ptr(out), d.shape[0],
                                        int(threads))
    return out.reshape(d.shape)


def cipher_pages_timed(key, nonces, data, rounds: int = 20,
                       threads: int = 1,
                       cipher: str = "chacha") -> tuple[np.ndarray, int]:
    """Like ``cipher_pages`` but also returns the thread count actually used."""
    k = _as_u8(key)
    d = _as_u8(data).reshape(-1, PAGE_BYTES)
    n = _as_u8(nonces).reshape(-1, NONCE_BYTES)
    out = np.empty_like(d)
    used = _load().oracle_cipher_pages_mt_with(
        CIPHERS[cipher], _ptr(k), _ptr(n), rounds, _ptr(d), _ptr(out),
        d.shape[0], int(threads))
    return out, used


from .nonces import nonces_linear, nonce_linear  # noqa: E402

__all__ = ["build", "chacha_block", "salsa_block", "cipher_pages",
           "cipher_pages_timed",
           "nonces_linear", "nonce_linear", "PAGE_BYTES", "BLOCK_BYTES",
           "NONCE_BYTES", "KEY_BYTES"]
