"""Pins of the CPU oracle against things other than itself.

The paper (section 4.4) fixes the cipher (ChaCha with 20 rounds), the unit of
work (a 4096-byte page XORed with 64 keystream blocks whose counter is the
block index 0..63) and that encryption and decryption are one operation.  It
prints no test vector, so the oracle is pinned here by

  * two independent system implementations of the same cipher, called as
    black boxes through their public APIs (OpenSSL EVP_chacha20 and
    libgcrypt's ChaCha20 stream mode): a page under nonce N is exactly the
    RFC 8439 ChaCha20 stream with counter 0 over the page's 4096 bytes;
  * a second oracle written separately in pure Python;
  * the invariants the paper states (XOR stream, same function both ways,
    blocks independent of each other);
  * mutation checks: plausible mistakes planted in a copy of the C oracle
    must each be caught by the library pins.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import chacha_py
from paper_2004_09252_amd import workloads
from tests import crypto_libs as cl

pytestmark = pytest.mark.skipif(not cl.HAVE_OPENSSL,
                                reason="libcrypto not present")

RNG = np.random.default_rng(12345)


def _rand(n):
    return RNG.bytes(n)


@pytest.mark.parametrize("counter", [0, 1, 2, 31, 62, 63, 64, 1000,
                                     0x7FFFFFFF, 0xFFFFFFFF])
def test_block_matches_openssl(counter):
    for _ in range(8):
        key, nonce = _rand(32), _rand(12)
        want = cl.openssl_chacha20(key, counter, nonce, bytes(64))
        assert oracle.chacha_block(key, counter, nonce) == want


def test_block_special_inputs_match_openssl():
    for key in (bytes(32), b"\xff" * 32, bytes(range(32))):
        for nonce in (bytes(12), b"\xff" * 12, bytes(range(12))):
            for ctr in (0, 63):
                want = cl.openssl_chacha20(key, ctr, nonce, bytes(64))
                assert oracle.chacha_block(key, ctr, nonce) == want


def test_page_matches_openssl_stream():
    key = _rand(32)
    nonces = np.frombuffer(_rand(12 * 9), np.uint8).reshape(9, 12)
    data = np.frombuffer(_rand(4096 * 9), np.uint8).reshape(9, 4096)
    got = oracle.cipher_pages(key, nonces, data)
    for p in range(9):
        want = cl.openssl_chacha20(key, 0, bytes(nonces[p]), bytes(data[p]))
        assert got[p].tobytes() == want


@pytest.mark.skipif(not cl.HAVE_GCRYPT, reason="libgcrypt not present")
def test_page_matches_gcrypt_stream():
    key = _rand(32)
    nonces = np.frombuffer(_rand(12 * 5), np.uint8).reshape(5, 12)
    data = np.frombuffer(_rand(4096 * 5), np.uint8).reshape(5, 4096)
    got = oracle.cipher_pages(key, nonces, data)
    for p in range(5):
        want = cl.gcrypt_chacha20(key, bytes(nonces[p]), bytes(data[p]))
        assert got[p].tobytes() == want


def test_python_oracle_agrees_with_c_oracle():
    key, nonce = _rand(32), _rand(12)
    page = _rand(4096)
    c_out = oracle.cipher_pages(key, np.frombuffer(nonce, np.uint8),
                                np.frombuffer(page, np.uint8))
    assert chacha_py.cipher_page(key, nonce, page) == c_out.tobytes()
    for ctr in (0, 7, 63):
        assert chacha_py.block(key, ctr, nonce) == \
            oracle.chacha_block(key, ctr, nonce)


@pytest.mark.parametrize("rounds", [8, 12])
def test_reduced_round_oracles_agree(rounds):
    """ChaCha12 and ChaCha8 (the cipher variants) have no library
    reference here: the C and the independent Python oracle must agree on
    blocks and whole pages, and the round count must matter (each variant
    differs from the others and from ChaCha20)."""
    key, nonce = _rand(32), _rand(12)
    page = _rand(4096)
    c_out = oracle.cipher_pages(key, np.frombuffer(nonce, np.uint8),
                                np.frombuffer(page, np.uint8), rounds=rounds)
    assert chacha_py.cipher_page(key, nonce, page, rounds) == c_out.tobytes()
    for ctr in (0, 9, 63):
        assert chacha_py.block(key, ctr, nonce, rounds) == \
            oracle.chacha_block(key, ctr, nonce, rounds)
    outs = {r: oracle.chacha_block(key, 5, nonce, r) for r in (8, 12, 20)}
    assert len(set(outs.values())) == 3


def test_python_oracle_matches_openssl():
    key, nonce = _rand(32), _rand(12)
    assert chacha_py.block(key, 3, nonce) == \
        cl.openssl_chacha20(key, 3, nonce, bytes(64))


def test_round_trip_and_same_function_both_ways():
    w = workloads.tiny(seed=1)
    enc = oracle.cipher_pages(w.key, w.nonces, w.data)
    assert not np.array_equal(enc, w.data)
    dec = oracle.cipher_pages(w.key, w.nonces, enc)
    assert np.array_equal(dec, w.data)


def test_xor_stream_linearity():
    key = _rand(32)
    nonces = np.frombuffer(_rand(12 * 3), np.uint8).reshape(3, 12)
    x = np.frombuffer(_rand(4096 * 3), np.uint8).reshape(3, 4096)
    y = np.frombuffer(_rand(4096 * 3), np.uint8).reshape(3, 4096)
    ex = oracle.cipher_pages(key, nonces, x)
    ey = oracle.cipher_pages(key, nonces, y)
    ks = oracle.cipher_pages(key, nonces, np.zeros_like(x))
    assert np.array_equal(ex ^ ey, x ^ y)
    assert np.array_equal(ex, x ^ ks)


def test_blocks_are_counter_indexed_and_independent():
    key, nonce = _rand(32), _rand(12)
    ks = oracle.cipher_pages(key, np.frombuffer(nonce, np.uint8),
                             np.zeros((1, 4096), np.uint8)).reshape(-1)
    for j in (0, 1, 17, 63):
        assert ks[64 * j:64 * j + 64].tobytes() == \
            oracle.chacha_block(key, j, nonce)
        # a stream started at counter j yields block j first
        assert cl.openssl_chacha20(key, j, nonce, bytes(64)) == \
            ks[64 * j:64 * j + 64].tobytes()


def test_page_permutation_permutes_outputs():
    w = workloads.tiny(seed=7, n_pages=16)
    perm = np.random.default_rng(3).permutation(16)
    a = oracle.cipher_pages(w.key, w.nonces, w.data)
    b = oracle.cipher_pages(w.key, w.nonces[perm], w.data[perm])
    assert np.array_equal(a[perm], b)


def _bit_fraction(a: bytes, b: bytes) -> float:
    x = np.frombuffer(a, np.uint8) ^ np.frombuffer(b, np.uint8)
    return np.unpackbits(x).mean()


def test_distinct_keystreams_per_key_nonce_page():
    key, nonce = bytearray(_rand(32)), bytearray(_rand(12))
    zero = np.zeros((1, 4096), np.uint8)

    def ks(k, n):
        return oracle.cipher_pages(bytes(k), np.frombuffer(bytes(n), np.uint8),
                                   zero).tobytes()

    base = ks(key, nonce)
    # 4096 B = 32768 bits; 5 sigma of a fair coin is 5*sqrt(32768)/2/32768
    tol = 5 * 0.5 / np.sqrt(32768)
    for bit in (0, 77, 255):
        k2 = bytearray(key)
        k2[bit // 8] ^= 1 << (bit % 8)
        assert abs(_bit_fraction(base, ks(k2, nonce)) - 0.5) < tol
    for bit in (0, 50, 95):
        n2 = bytearray(nonce)
        n2[bit // 8] ^= 1 << (bit % 8)
        assert abs(_bit_fraction(base, ks(key, n2)) - 0.5) < tol
    # different pages of a linear run have different keystreams
    n = oracle.nonces_linear(4, 0x7F0000000000, 4096, 1234)
    k = oracle.cipher_pages(bytes(key), n, np.zeros((4, 4096), np.uint8))
    for i in range(4):
        for j in range(i + 1, 4):
            assert abs(_bit_fraction(k[i].tobytes(), k[j].tobytes()) - 0.5) \
                < tol


def test_linear_nonces_layout():
    n = oracle.nonces_linear(3, 0x7F0000001000, 4096, 4321)
    assert n[0].tobytes() == (0x7F0000001000).to_bytes(8, "little") + \
        (4321).to_bytes(4, "little")
    assert n[2].tobytes()[:8] == (0x7F0000003000).to_bytes(8, "little")
    big = oracle.nonces_linear(5000, 2**64 - 3, 1, 7)
    small = np.stack([np.frombuffer(oracle.nonce_linear(i, 2**64 - 3, 1, 7),
                                    np.uint8) for i in range(5000)])
    assert np.array_equal(big, small)
    assert big[3].tobytes()[:8] == bytes(8)   # wraps mod 2**64


def test_threaded_oracle_equals_single_thread():
    w = workloads.tiny(seed=9, n_pages=37)
    a = oracle.cipher_pages(w.key, w.nonces, w.data, threads=1)
    b = oracle.cipher_pages(w.key, w.nonces, w.data, threads=5)
    assert np.array_equal(a, b)


MUTATIONS = [
    ("rotate_left(x[d] ^ x[a], 16)", "rotate_left(x[d] ^ x[a], 15)"),
    ("rotate_left(x[b] ^ x[c], 7)", "rotate_left(x[b] ^ x[c], 8)"),
    ("quarter_round(work, 1, 6, 11, 12)", "quarter_round(work, 1, 6, 11, 13)"),
    ("quarter_round(work, 3, 7, 11, 15)", "quarter_round(work, 3, 7, 15, 11)"),
    ("x[c] = x[c] + x[d];", "x[c] = x[c] ^ x[d];"),
    ("write_le32(out + 4 * i, work[i] + input[i]);",
     "write_le32(out + 4 * i, work[i]);"),
    ("input[12] = counter;", "input[12] = counter + 1;"),
    ("input[13 + i] = read_le32(nonce + 4 * i);",
     "input[13 + i] = read_le32(nonce + 4 * (2 - i));"),
    ("for (i = 0; i < rounds; i += 2) {", "for (i = 2; i < rounds; i += 2) {"),
    ("input[4 + i] = read_le32(key + 4 * i);",
     "input[4 + i] = read_le32(key + 4 * (i ^ 1));"),
]


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_pins_catch_planted_mistakes(tmp_path, old, new):
    import ctypes
    src = open(os.path.join(os.path.dirname(oracle.__file__),
                            "chacha20_oracle.c")).read()
    assert old in src
    mutated = src.replace(old, new, 1)
    c = tmp_path / "m.c"
    so = tmp_path / "m.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread",
                           str(c), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_chacha_block.argtypes = [ctypes.c_char_p, ctypes.c_uint32,
                                        ctypes.c_char_p, ctypes.c_int,
                                        ctypes.c_void_p]
    caught = False
    rng = np.random.default_rng(99)
    for ctr in (0, 1, 63):
        key, nonce = rng.bytes(32), rng.bytes(12)
        out = ctypes.create_string_buffer(64)
        lib.oracle_chacha_block(key, ctr, nonce, 20, out)
        if out.raw != cl.openssl_chacha20(key, ctr, nonce, bytes(64)):
            caught = True
    assert caught, "library pin missed a planted mistake"


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "page_cipher_digests.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, seed, n, digest = line.split()
        out[name] = (int(seed), int(n), digest)
    return out


def test_golden_tiny_digest_reproduces():
    import hashlib
    seed, n, digest = _golden()["tiny"]
    t = workloads.tiny(seed=seed, n_pages=n)
    enc = oracle.cipher_pages(t.key, t.nonces, t.data)
    assert hashlib.sha256(enc.tobytes()).hexdigest() == digest


# --- Salsa20, the engine's second cipher ---------------------------------
# A Salsa20 page under the 12-byte page nonce N is the Salsa20 stream with
# the 8-byte nonce N[0:8] from block counter LE32(N[8:12]) * 2^32 over the
# page's 4096 bytes.  Pinned by libgcrypt (whose stream starts at counter 0:
# pages whose third nonce word is 0) and libnettle (any starting counter),
# by the pure-Python Salsa20 and by planted mistakes.

salsa_libs = pytest.mark.skipif(not (cl.HAVE_GCRYPT and cl.HAVE_NETTLE),
                                reason="libgcrypt or libnettle not present")


@salsa_libs
@pytest.mark.parametrize("rounds", [20, 12])
def test_salsa_page_matches_gcrypt_stream(rounds):
    key = _rand(32)
    nonces = np.frombuffer(_rand(12 * 6), np.uint8).reshape(6, 12).copy()
    nonces[:, 8:] = 0
    data = np.frombuffer(_rand(4096 * 6), np.uint8).reshape(6, 4096)
    got = oracle.cipher_pages(key, nonces, data, rounds=rounds,
                              cipher="salsa")
    for p in range(6):
        want = cl.gcrypt_salsa20(key, nonces[p, :8].tobytes(),
                                 data[p].tobytes(), rounds)
        assert got[p].tobytes() == want


@salsa_libs
@pytest.mark.parametrize("rounds", [20, 12])
def test_salsa_page_matches_nettle_from_high_counter(rounds):
    key = _rand(32)
    nonces = np.frombuffer(_rand(12 * 6), np.uint8).reshape(6, 12).copy()
    nonces[0, 8:] = 255      # counter high word 0xffffffff
    data = np.frombuffer(_rand(4096 * 6), np.uint8).reshape(6, 4096)
    got = oracle.cipher_pages(key, nonces, data, rounds=rounds,
                              cipher="salsa")
    for p in range(6):
        high = int.from_bytes(nonces[p, 8:].tobytes(), "little") << 32
        want = cl.nettle_salsa20(key, nonces[p, :8].tobytes(), high,
                                 data[p].tobytes(), rounds)
        assert got[p].tobytes() == want


@salsa_libs
def test_salsa_libraries_agree_and_nettle_counter_words():
    """The two libraries agree from counter 0, and nettle started at counter
    1 equals libgcrypt's second block: words 8 and 9 of nettle's state are
    the block counter, as the high-counter pin assumes."""
    key, n8 = _rand(32), _rand(8)
    a = cl.gcrypt_salsa20(key, n8, bytes(4096))
    assert cl.nettle_salsa20(key, n8, 0, bytes(4096)) == a
    assert cl.nettle_salsa20(key, n8, 1, bytes(64)) == a[64:128]
    assert cl.nettle_salsa20(key, n8, 63, bytes(64)) == a[4032:]


@pytest.mark.parametrize("rounds", [20, 12, 8])
def test_salsa_python_oracle_agrees_with_c_oracle(rounds):
    from oracle import salsa_py
    key = _rand(32)
    nonces = np.frombuffer(_rand(12 * 2), np.uint8).reshape(2, 12)
    data = np.frombuffer(_rand(4096 * 2), np.uint8).reshape(2, 4096)
    got = oracle.cipher_pages(key, nonces, data, rounds=rounds,
                              cipher="salsa")
    for p in range(2):
        want = salsa_py.cipher_page(key, nonces[p].tobytes(),
                                    data[p].tobytes(), rounds)
        assert got[p].tobytes() == want
    for ctr in (0, 63, 2**32 - 1, 2**32, 2**64 - 1):
        n8 = _rand(8)
        assert oracle.salsa_block(key, n8, ctr, rounds) == \
            salsa_py.block(key, n8, ctr, rounds)


def test_salsa_invariants():
    """Same function both ways, a distinct keystream from ChaCha's under the
    same key and nonce, and different keystreams for nonces that differ only
    in the word that becomes the counter's high half."""
    w = workloads.tiny(seed=13, n_pages=4)
    enc = oracle.cipher_pages(w.key, w.nonces, w.data, cipher="salsa")
    assert np.array_equal(oracle.cipher_pages(w.key, w.nonces, enc,
                                              cipher="salsa"), w.data)
    cha = oracle.cipher_pages(w.key, w.nonces, w.data)
    assert abs(_bit_fraction(enc.tobytes(), cha.tobytes()) - 0.5) < 0.02
    n2 = w.nonces.copy()
    n2[:, 8] ^= 1
    other = oracle.cipher_pages(w.key, n2, w.data, cipher="salsa")
    assert abs(_bit_fraction(enc.tobytes(), other.tobytes()) - 0.5) < 0.02
    # blocks are independent: block j of a page is the block at counter j
    ks = oracle.cipher_pages(w.key, w.nonces[:1], np.zeros((1, 4096),
                                                           np.uint8),
                             cipher="salsa")[0]
    high = int.from_bytes(w.nonces[0, 8:].tobytes(), "little") << 32
    for j in (0, 1, 37, 63):
        assert ks[64 * j:64 * j + 64].tobytes() == oracle.salsa_block(
            w.key, w.nonces[0, :8], high + j)


SALSA_MUTATIONS = [
    ("x[b] ^= rotate_left(x[a] + x[d], 7);",
     "x[b] ^= rotate_left(x[a] + x[d], 8);"),
    ("x[a] ^= rotate_left(x[d] + x[c], 18);",
     "x[a] ^= rotate_left(x[d] + x[c], 16);"),
    ("x[c] ^= rotate_left(x[b] + x[a], 9);",
     "x[c] += rotate_left(x[b] + x[a], 9);"),
    ("salsa_quarter(work, 5, 9, 13, 1);", "salsa_quarter(work, 5, 9, 1, 13);"),
    ("salsa_quarter(work, 10, 11, 8, 9);",
     "salsa_quarter(work, 10, 11, 9, 8);"),
    ("input[8] = (uint32_t)(counter & 0xffffffffu);",
     "input[8] = (uint32_t)(counter & 0xffffffffu) + 1;"),
    ("input[9] = (uint32_t)(counter >> 32);", "input[9] = 0;"),
    ("input[11 + i] = read_le32(key + 16 + 4 * i);",
     "input[11 + i] = read_le32(key + 4 * i);"),
    ("input[6] = read_le32(nonce8);", "input[6] = read_le32(nonce8 + 4);"),
    ("input[5] = read_le32((const uint8_t *)sigma + 4);",
     "input[5] = read_le32((const uint8_t *)sigma + 8);"),
    ("write_le32(out + 4 * i, work[i] + input[i]);\n}\n\n/* One page with "
     "Salsa20", "write_le32(out + 4 * i, work[i] ^ input[i]);\n}\n\n/* One "
     "page with Salsa20"),
]


@salsa_libs
@pytest.mark.parametrize("old,new", SALSA_MUTATIONS)
def test_salsa_pins_catch_planted_mistakes(tmp_path, old, new):
    import ctypes
    src = open(os.path.join(os.path.dirname(oracle.__file__),
                            "chacha20_oracle.c")).read()
    assert src.count(old) == 1, old
    mutated = src.replace(old, new, 1)
    c = tmp_path / "m.c"
    so = tmp_path / "m.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread",
                           str(c), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_salsa_block.argtypes = [ctypes.c_char_p, ctypes.c_char_p,
                                       ctypes.c_uint64, ctypes.c_int,
                                       ctypes.c_void_p]
    caught = False
    rng = np.random.default_rng(98)
    for ctr in (0, 1, 63, (7 << 32) + 5):
        key, n8 = rng.bytes(32), rng.bytes(8)
        out = ctypes.create_string_buffer(64)
        lib.oracle_salsa_block(key, n8, ctr, 20, out)
        if out.raw != cl.nettle_salsa20(key, n8, ctr, bytes(64)):
            caught = True
    assert caught, "library pin missed a planted mistake"
