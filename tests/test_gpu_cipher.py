"""GPU parity of the page cipher: HIP engine vs the CPU oracle, bit-exact.

Every case draws its inputs from the seeded generators, runs them through the
C ABI (via the ctypes binding) on the GPU and compares every byte with the
oracle's output for the same inputs (the paper's section 4.4 cipher: 4096-
byte pages, 64 ChaCha20 blocks per page with counter = block index, the same
XOR for both directions).
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2004_09252_amd import workloads

pytestmark = pytest.mark.gpu

HOST_THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _note(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ms():
    from paper_2004_09252_amd import memshield
    return memshield


@pytest.fixture(scope="module")
def eng(ms):
    e = ms.Engine(0)
    yield e
    e.close()


def _dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda")


def _host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_tiny_array_nonces_bit_exact(ms, eng):
    _note("tiny seed=1 array nonces")
    w = workloads.tiny(seed=1)
    key = eng.key_load(w.key)
    src, nonces = _dev(w.data), _dev(w.nonces)
    dst = src.clone().zero_()
    eng.encrypt_pages(key, src, dst, ms.array_nonce(nonces))
    enc = _host(dst).reshape(64, 4096)
    want = oracle.cipher_pages(w.key, w.nonces, w.data)
    assert np.array_equal(enc, want)
    back = src.clone().zero_()
    eng.decrypt_pages(key, dst, back, ms.array_nonce(nonces))
    assert np.array_equal(_host(back).reshape(64, 4096), w.data)
    eng.key_destroy(key)


@pytest.mark.parametrize("n_pages", [1, 2, 3, 4, 5, 7, 63, 64, 65, 255, 257,
                                     1023, 4097])
@pytest.mark.parametrize("in_place", [False, True])
def test_linear_nonces_sizes(ms, eng, n_pages, in_place):
    _note("linear n_pages=%d in_place=%s" % (n_pages, in_place))
    rng = np.random.default_rng(1000 + n_pages)
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n_pages)
    base, stride, tag = 0x7F0000000000 + 4096 * 17, 4096, 4242
    key = eng.key_load(key_b)
    src = _dev(data)
    dst = src if in_place else src.clone().zero_()
    eng.encrypt_pages(key, src, dst, ms.linear_nonce(base, stride, tag))
    got = _host(dst).reshape(n_pages, 4096)
    n = oracle.nonces_linear(n_pages, base, stride, tag)
    want = oracle.cipher_pages(key_b, n, data, threads=HOST_THREADS)
    assert np.array_equal(got, want)
    eng.key_destroy(key)


def test_encrypt_equals_decrypt_and_round_trip(ms, eng):
    _note("encrypt == decrypt")
    rng = np.random.default_rng(77)
    data = workloads.random_pages(rng, 100)
    key = eng.key_generate()
    src = _dev(data)
    a = src.clone().zero_()
    b = src.clone().zero_()
    nonce = ms.linear_nonce(5, 1, 9)
    eng.encrypt_pages(key, src, a, nonce)
    eng.decrypt_pages(key, src, b, nonce)
    assert np.array_equal(_host(a), _host(b))
    c = src.clone().zero_()
    eng.decrypt_pages(key, a, c, nonce)
    assert np.array_equal(_host(c), data.reshape(-1))
    eng.key_destroy(key)


def test_nonce_wraps_mod_2_64(ms, eng):
    _note("nonce wrap")
    rng = np.random.default_rng(5)
    data = workloads.random_pages(rng, 8)
    kb = rng.bytes(32)
    key = eng.key_load(kb)
    src = _dev(data)
    dst = src.clone()
    base = 2**64 - 3
    eng.encrypt_pages(key, src, dst, ms.linear_nonce(base, 1, 0xFFFFFFFF))
    want = oracle.cipher_pages(kb, oracle.nonces_linear(8, base, 1,
                                                        0xFFFFFFFF), data)
    assert np.array_equal(_host(dst).reshape(8, 4096), want)
    eng.key_destroy(key)


def test_many_keys_distinct_slots(ms, eng):
    _note("many keys")
    rng = np.random.default_rng(9)
    data = workloads.random_pages(rng, 3)
    src = _dev(data)
    handles, kbs = [], []
    for i in range(20):
        kb = rng.bytes(32)
        kbs.append(kb)
        handles.append(eng.key_load(kb))
    for i in (0, 7, 19):
        dst = src.clone()
        eng.encrypt_pages(handles[i], src, dst, ms.linear_nonce(i, 1, 0))
        want = oracle.cipher_pages(kbs[i], oracle.nonces_linear(3, i, 1, 0),
                                   data)
        assert np.array_equal(_host(dst).reshape(3, 4096), want)
    for h in handles:
        eng.key_destroy(h)


def test_bulk_1gib_full_parity(ms, eng):
    """The 1 GiB plain workload: 262144 pages, nonce = page index."""
    _note("bulk 1GiB seed=2")
    import torch
    b = workloads.bulk(seed=2)
    n = b.data.shape[0]
    key = eng.key_load(b.key)
    src = _dev(b.data)
    dst = torch.empty_like(src)
    nonce = ms.linear_nonce(b.nonce_base, b.nonce_stride, b.nonce_tag)
    eng.encrypt_pages(key, src, dst, nonce)
    enc = _host(dst).reshape(n, 4096)
    golden = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden",
                                  "page_cipher_digests.txt")):
        if line.strip() and not line.startswith("#"):
            name, _, _, digest = line.split()
            golden[name] = digest
    assert hashlib.sha256(enc.tobytes()).hexdigest() == golden["bulk"]
    nonces = oracle.nonces_linear(n, b.nonce_base, b.nonce_stride,
                                  b.nonce_tag)
    want = oracle.cipher_pages(b.key, nonces, b.data, threads=HOST_THREADS)
    assert np.array_equal(enc, want)
    # decrypt pass back to the plaintext, in place
    eng.decrypt_pages(key, dst, dst, nonce)
    assert torch.equal(dst, src)
    del dst, src
    eng.key_destroy(key)


def test_split_launch_beyond_2_24_pages(ms, eng):
    """One call of 2^24 + 3 pages (64 GiB + 12 KiB, in place): the engine
    splits it into launches of at most 2^24 pages, each starting at its own
    page offset (section 4.4: page p's nonce and its 64 block counters).
    Pages on both sides of the split, the first and last page and a seeded
    sample are compared with the oracle byte for byte, with linear nonces
    (encrypt) and then with an array of random nonces (decrypt)."""
    import torch
    n = (1 << 24) + 3
    _note("split launch n_pages=%d (64 GiB in place)" % n)
    rng = np.random.default_rng(2424)
    key_b = rng.bytes(32)
    buf = torch.empty(n * 4096, dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(2424)
    chunk = 1 << 30
    for off in range(0, buf.numel(), chunk):
        buf[off:off + chunk].random_(0, 256, generator=gen)
    split = 1 << 24
    idx = sorted(set([0, 1, split - 2, split - 1, split, split + 1,
                      split + 2, n - 1] +
                     rng.integers(0, n, 16).tolist()))
    pages = buf.view(n, 4096)
    sel = torch.tensor(idx, dtype=torch.int64, device="cuda")
    plain = pages[sel].cpu().numpy()
    key = eng.key_load(key_b)
    base, stride, tag = 0x7F0000000000, 4096, 77
    eng.encrypt_pages(key, buf, buf, ms.linear_nonce(base, stride, tag))
    enc = pages[sel].cpu().numpy()
    lin = np.stack([np.frombuffer(oracle.nonce_linear(i, base, stride, tag),
                                  np.uint8) for i in idx])
    want = oracle.cipher_pages(key_b, lin, plain)
    bad = [idx[r] for r in range(len(idx)) if not np.array_equal(enc[r],
                                                                  want[r])]
    assert not bad, "linear nonces: pages %s differ from the oracle" % bad
    nonces = np.frombuffer(rng.bytes(12 * n), np.uint8).reshape(n, 12)
    dn = torch.from_numpy(nonces.reshape(-1)).to("cuda")
    eng.decrypt_pages(key, buf, buf, ms.array_nonce(dn))
    got = pages[sel].cpu().numpy()
    want2 = oracle.cipher_pages(key_b, nonces[idx], enc)
    bad = [idx[r] for r in range(len(idx)) if not np.array_equal(got[r],
                                                                 want2[r])]
    assert not bad, "array nonces: pages %s differ from the oracle" % bad
    eng.key_destroy(key)
    del buf, pages, sel, dn
    torch.cuda.empty_cache()


def test_rejects_bad_arguments(ms, eng):
    _note("argument validation")
    import torch
    key = eng.key_generate()
    buf = torch.zeros(8 * 4096, dtype=torch.uint8, device="cuda")
    ctx = eng.ctx
    lin = ms.linear_nonce(0, 1, 0)
    p = buf.data_ptr()
    # zero pages: no-op
    assert ms.ms_encrypt_pages(ctx, key, p, p, 0, lin) == ms.MS_OK
    # run past the end of the allocation
    assert ms.ms_encrypt_pages(ctx, key, p, p, 1 << 20, lin) == ms.MS_EINVAL
    # misaligned
    assert ms.ms_encrypt_pages(ctx, key, p + 4, p + 4, 1, lin) == ms.MS_EINVAL
    # partial overlap
    assert ms.ms_encrypt_pages(ctx, key, p, p + 4096, 2, lin) == ms.MS_EINVAL
    # host pointer
    host = np.zeros(4096 * 2, np.uint8)
    assert ms.ms_encrypt_pages(ctx, key, host.ctypes.data, p, 1, lin) == \
        ms.MS_EINVAL
    # null
    assert ms.ms_encrypt_pages(ctx, key, 0, p, 1, lin) == ms.MS_EINVAL
    # bad nonce kind and short nonce array
    bad = ms.ms_nonce(7, 0, None, 0, 0)
    assert ms.ms_encrypt_pages(ctx, key, p, p, 1, bad) == ms.MS_EINVAL
    small = torch.zeros(12, dtype=torch.uint8, device="cuda")
    arr = ms.array_nonce(small)
    assert ms.ms_encrypt_pages(ctx, key, p, p, 1, arr) == ms.MS_OK
    # a misaligned nonce array
    arr_odd = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, small.data_ptr() + 1, 0, 0)
    assert ms.ms_encrypt_pages(ctx, key, p, p, 1, arr_odd) == ms.MS_EINVAL
    # unknown / destroyed / stale handles
    assert ms.ms_encrypt_pages(ctx, 0, p, p, 1, lin) == ms.MS_ENOKEY
    assert ms.ms_encrypt_pages(ctx, key + (1 << 32), p, p, 1, lin) == \
        ms.MS_ENOKEY
    eng.key_destroy(key)
    assert ms.ms_encrypt_pages(ctx, key, p, p, 1, lin) == ms.MS_ENOKEY
    assert ms.ms_key_destroy(ctx, key) == ms.MS_ENOKEY
    torch.cuda.synchronize()


def test_key_purged_from_host_staging(ms, eng):
    _note("key purge")
    assert ms.ms_debug_staging_is_zero(eng.ctx) == 1
    h = eng.key_load(b"\x5a" * 32)
    assert ms.ms_debug_staging_is_zero(eng.ctx) == 1
    g = eng.key_generate()
    assert ms.ms_debug_staging_is_zero(eng.ctx) == 1
    eng.key_destroy(h)
    eng.key_destroy(g)


def test_key_table_full(ms):
    _note("key table full")
    e = ms.Engine(0, max_keys=3)
    try:
        hs = [e.key_generate() for _ in range(3)]
        st, _ = ms.ms_key_generate(e.ctx)
        assert st == ms.MS_ENOMEM
        e.key_destroy(hs[1])
        h = e.key_generate()          # slot reused with a new generation
        assert h != hs[1]
        assert ms.ms_key_destroy(e.ctx, hs[1]) == ms.MS_ENOKEY
    finally:
        e.close()


@pytest.mark.parametrize("rounds", [12, 8])
def test_reduced_round_variants(ms, rounds):
    _note("rounds=%d" % rounds)
    e = ms.Engine(0, rounds=rounds)
    try:
        rng = np.random.default_rng(rounds)
        data = workloads.random_pages(rng, 65)
        kb = rng.bytes(32)
        key = e.key_load(kb)
        src = _dev(data)
        dst = src.clone()
        e.encrypt_pages(key, src, dst, ms.linear_nonce(3, 4096, 11))
        want = oracle.cipher_pages(kb, oracle.nonces_linear(65, 3, 4096, 11),
                                   data, rounds=rounds)
        assert np.array_equal(_host(dst).reshape(65, 4096), want)
    finally:
        e.close()


@pytest.mark.parametrize("rounds", [20, 12, 8])
@pytest.mark.parametrize("n_pages,in_place,kind", [
    (1, False, "linear"), (63, True, "linear"), (257, False, "array"),
    (4097, True, "array"), (3000, False, "linear")])
def test_salsa20_pages_bit_exact(ms, rounds, n_pages, in_place, kind):
    """The second cipher behind the same ABI (ms_config.cipher = Salsa20):
    every page equals the Salsa20 oracle (nonce = page nonce bytes 0..7,
    block counter = page nonce word 2 * 2^32 + j), and decrypting gives the
    data back."""
    _note("salsa20 rounds=%d n_pages=%d in_place=%s %s" % (
        rounds, n_pages, in_place, kind))
    import torch
    e = ms.Engine(0, rounds=rounds, cipher=ms.MS_CIPHER_SALSA)
    try:
        rng = np.random.default_rng(5000 + rounds + n_pages)
        data = workloads.random_pages(rng, n_pages)
        kb = rng.bytes(32)
        key = e.key_load(kb)
        src = _dev(data)
        dst = src if in_place else torch.zeros_like(src)
        if kind == "array":
            nonces = np.frombuffer(rng.bytes(12 * n_pages),
                                   np.uint8).reshape(n_pages, 12)
            nd = _dev(nonces)
            nonce = ms.array_nonce(nd)
        else:
            base, stride, tag = 0x7F0000000000 + 4096 * 9, 4096, 0xDEADBEEF
            nonces = oracle.nonces_linear(n_pages, base, stride, tag)
            nonce = ms.linear_nonce(base, stride, tag)
        e.encrypt_pages(key, src, dst, nonce)
        got = _host(dst).reshape(n_pages, 4096)
        want = oracle.cipher_pages(kb, nonces, data, rounds=rounds,
                                   cipher="salsa", threads=HOST_THREADS)
        assert np.array_equal(got, want)
        back = torch.zeros_like(src)
        e.decrypt_pages(key, dst, back, nonce)
        assert np.array_equal(_host(back).reshape(n_pages, 4096), data)
        e.key_destroy(key)
    finally:
        e.close()


def test_salsa20_bulk_1gib_sampled(ms):
    """The bulk workload under Salsa20/20 (262144 pages, nonce = page
    index): the first, last and a seeded sample of pages against the
    oracle, and the round trip in full."""
    _note("salsa20 bulk 1GiB")
    import torch
    b = workloads.bulk(seed=2)
    n = b.data.shape[0]
    e = ms.Engine(0, cipher=ms.MS_CIPHER_SALSA)
    try:
        key = e.key_load(b.key)
        src = _dev(b.data)
        dst = torch.empty_like(src)
        nonce = ms.linear_nonce(b.nonce_base, b.nonce_stride, b.nonce_tag)
        e.encrypt_pages(key, src, dst, nonce)
        idx = sorted(set([0, 1, n - 1] + np.random.default_rng(2).integers(
            0, n, 64).tolist()))
        got = _host(dst).reshape(n, 4096)[idx]
        nn = oracle.nonces_linear(n, b.nonce_base, b.nonce_stride,
                                  b.nonce_tag)[idx]
        want = oracle.cipher_pages(b.key, nn, b.data[idx], cipher="salsa")
        assert np.array_equal(got, want)
        e.decrypt_pages(key, dst, dst, nonce)
        assert torch.equal(dst, src)
        e.key_destroy(key)
        del src, dst
    finally:
        e.close()


def test_plain_launch_info_names_the_launch(ms, eng):
    """ms_plain_launch_info describes what a call launches: the kernel's
    template arguments, one launch per 2^24 pages, a grid of the resident
    waves (or one wave per page below that)."""
    st, i = ms.ms_plain_launch_info(eng.ctx, 262144, ms.MS_NONCE_LINEAR)
    assert st == 0
    assert i.kernel.decode() == "plain_pages_kernel<0u, 20, 1, 1u>"
    assert i.launches == 1 and i.block_threads == 256 and i.unroll == 1
    cus = ms.ms_device_cu_count(eng.ctx)
    assert i.grid_blocks == cus * i.waves_per_cu // 4
    st, i = ms.ms_plain_launch_info(eng.ctx, (1 << 24) + 3, ms.MS_NONCE_ARRAY)
    assert st == 0 and i.launches == 2
    assert i.kernel.decode() == "plain_pages_kernel<0u, 20, 1, 0u>"
    st, i = ms.ms_plain_launch_info(eng.ctx, 10, ms.MS_NONCE_LINEAR)
    assert st == 0 and i.grid_blocks == 3
    e = ms.Engine(0, cipher=ms.MS_CIPHER_SALSA, rounds=12)
    try:
        st, i = ms.ms_plain_launch_info(e.ctx, 5, ms.MS_NONCE_LINEAR)
        assert i.kernel.decode() == "plain_pages_kernel<1u, 12, 1, 1u>"
    finally:
        e.close()
    assert ms.ms_plain_launch_info(eng.ctx, 0, 1)[0] == ms.MS_EINVAL
