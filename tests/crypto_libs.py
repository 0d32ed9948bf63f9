"""Black-box access to two system ChaCha20 implementations for pinning the
oracle: OpenSSL's libcrypto (EVP_chacha20, 16-byte IV = LE32 counter ||
96-bit nonce) and libgcrypt (ChaCha20 in stream mode, 12-byte IV = 96-bit
nonce, counter starting at 0).  Only their public C APIs are called."""
from __future__ import annotations

import ctypes
import ctypes.util


def _load(names):
    for n in names:
        try:
            return ctypes.CDLL(n)
        except OSError:
            continue
    return None


_crypto = _load(["libcrypto.so.3", ctypes.util.find_library("crypto") or ""])
_gcrypt = _load(["libgcrypt.so.20", ctypes.util.find_library("gcrypt") or ""])

if _crypto is not None:
    _crypto.EVP_CIPHER_CTX_new.restype = ctypes.c_void_p
    _crypto.EVP_CIPHER_CTX_free.argtypes = [ctypes.c_void_p]
    _crypto.EVP_chacha20.restype = ctypes.c_void_p
    _crypto.EVP_EncryptInit_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_char_p,
                                           ctypes.c_char_p]
    _crypto.EVP_EncryptUpdate.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.c_char_p, ctypes.c_int]

if _gcrypt is not None:
    _gcrypt.gcry_check_version.restype = ctypes.c_char_p
    _gcrypt.gcry_check_version.argtypes = [ctypes.c_char_p]
    _gcrypt.gcry_check_version(None)
    _gcrypt.gcry_cipher_map_name.argtypes = [ctypes.c_char_p]
    _gcrypt.gcry_cipher_open.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.c_int, ctypes.c_int,
                                         ctypes.c_uint]
    _gcrypt.gcry_cipher_setkey.argtypes = [ctypes.c_void_p, ctypes.c_char_p,
                                           ctypes.c_size_t]
    _gcrypt.gcry_cipher_setiv.argtypes = [ctypes.c_void_p, ctypes.c_char_p,
                                          ctypes.c_size_t]
    _gcrypt.gcry_cipher_encrypt.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_char_p,
                                            ctypes.c_size_t]
    _gcrypt.gcry_cipher_close.argtypes = [ctypes.c_void_p]

HAVE_OPENSSL = _crypto is not None
HAVE_GCRYPT = _gcrypt is not None
GCRY_MODE_STREAM = 4


def openssl_chacha20(key: bytes, counter: int, nonce: bytes,
                     data: bytes) -> bytes:
    ctx = _crypto.EVP_CIPHER_CTX_new()
    try:
        iv = counter.to_bytes(4, "little") + nonce
        assert _crypto.EVP_EncryptInit_ex(ctx, _crypto.EVP_chacha20(), None,
                                          key, iv) == 1
        out = ctypes.create_string_buffer(len(data))
        outl = ctypes.c_int(0)
        assert _crypto.EVP_EncryptUpdate(ctx, out, ctypes.byref(outl), data,
                                         len(data)) == 1
        assert outl.value == len(data)
        return out.raw
    finally:
        _crypto.EVP_CIPHER_CTX_free(ctx)


def gcrypt_chacha20(key: bytes, nonce: bytes, data: bytes) -> bytes:
    algo = _gcrypt.gcry_cipher_map_name(b"CHACHA20")
    hd = ctypes.c_void_p()
    assert _gcrypt.gcry_cipher_open(ctypes.byref(hd), algo, GCRY_MODE_STREAM,
                                    0) == 0
    try:
        assert _gcrypt.gcry_cipher_setkey(hd, key, 32) == 0
        assert _gcrypt.gcry_cipher_setiv(hd, nonce, 12) == 0
        out = ctypes.create_string_buffer(len(data))
        assert _gcrypt.gcry_cipher_encrypt(hd, out, len(data), data,
                                           len(data)) == 0
        return out.raw
    finally:
        _gcrypt.gcry_cipher_close(hd)


# --- Salsa20 (the engine's second cipher) -------------------------------
# libgcrypt: SALSA20 / SALSA20R12 in stream mode, 8-byte IV, block counter
# from 0.  libnettle: salsa20_256_set_key, salsa20_set_nonce (8 bytes,
# counter 0), salsa20_crypt / salsa20r12_crypt; its context is the 16-word
# input state (nettle's struct salsa20_ctx), so a test may set the 64-bit
# block counter words 8 and 9 itself before ciphering.

_nettle = _load(["libnettle.so.8", ctypes.util.find_library("nettle") or ""])
if _nettle is not None:
    for _f in ("nettle_salsa20_256_set_key", "nettle_salsa20_set_nonce"):
        getattr(_nettle, _f).argtypes = [ctypes.c_void_p, ctypes.c_char_p]
        getattr(_nettle, _f).restype = None
    for _f in ("nettle_salsa20_crypt", "nettle_salsa20r12_crypt"):
        getattr(_nettle, _f).argtypes = [ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p, ctypes.c_char_p]
        getattr(_nettle, _f).restype = None

HAVE_NETTLE = _nettle is not None


def gcrypt_salsa20(key: bytes, nonce8: bytes, data: bytes,
                   rounds: int = 20) -> bytes:
    name = {20: b"SALSA20", 12: b"SALSA20R12"}[rounds]
    algo = _gcrypt.gcry_cipher_map_name(name)
    assert algo != 0
    hd = ctypes.c_void_p()
    assert _gcrypt.gcry_cipher_open(ctypes.byref(hd), algo, GCRY_MODE_STREAM,
                                    0) == 0
    try:
        assert _gcrypt.gcry_cipher_setkey(hd, key, 32) == 0
        assert _gcrypt.gcry_cipher_setiv(hd, nonce8, 8) == 0
        out = ctypes.create_string_buffer(len(data))
        assert _gcrypt.gcry_cipher_encrypt(hd, out, len(data), data,
                                           len(data)) == 0
        return out.raw
    finally:
        _gcrypt.gcry_cipher_close(hd)


def nettle_salsa20(key: bytes, nonce8: bytes, counter: int, data: bytes,
                   rounds: int = 20) -> bytes:
    """Salsa20 from 64-bit block counter `counter` (words 8, 9 of nettle's
    input state, set after salsa20_set_nonce)."""
    ctx = (ctypes.c_uint32 * 64)()   # the 16-word state, with room to spare
    _nettle.nettle_salsa20_256_set_key(ctx, key)
    _nettle.nettle_salsa20_set_nonce(ctx, nonce8)
    ctx[8] = counter & 0xFFFFFFFF
    ctx[9] = (counter >> 32) & 0xFFFFFFFF
    out = ctypes.create_string_buffer(len(data))
    fn = {20: _nettle.nettle_salsa20_crypt,
          12: _nettle.nettle_salsa20r12_crypt}[rounds]
    fn(ctx, len(data), out, data)
    return out.raw
