"""GPU parity of the host-resident page calls (include/memshield_host.h):
pages in pinned host memory ciphered through each transfer mode, compared
byte for byte with the CPU oracle on the same seeded inputs.  The staged
modes run with a small chunk (64 pages) and two staging slots so that short
runs, ragged last chunks and slot reuse within and across calls are all
exercised."""
import sys
import threading

import numpy as np
import pytest

import oracle
from paper_2004_09252_amd import workloads

pytestmark = pytest.mark.gpu

CHUNK = 64
MODES = {"auto": 0, "mapped": 1, "dma": 2, "dma_in": 3}
BASE, STRIDE, TAG = 0x7F0000000000 + 4096 * 33, 4096, 777


def _note(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ms():
    from paper_2004_09252_amd import memshield
    return memshield


@pytest.fixture(scope="module")
def eng(ms):
    e = ms.Engine(0, host_chunk_pages=CHUNK, host_stage_slots=2)
    yield e
    e.close()


def _want(key_b, data, base=BASE, stride=STRIDE, tag=TAG):
    n = data.shape[0]
    return oracle.cipher_pages(key_b, oracle.nonces_linear(n, base, stride,
                                                           tag), data)


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("n_pages", [1, 3, CHUNK - 1, CHUNK, CHUNK + 1,
                                     3 * CHUNK + 17])
def test_host_to_host_bit_exact(ms, eng, mode, n_pages):
    _note("host->host mode=%s n_pages=%d" % (mode, n_pages))
    rng = np.random.default_rng(3000 + n_pages)
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n_pages)
    key = eng.key_load(key_b)
    src = eng.host_alloc(n_pages * 4096)
    dst = eng.host_alloc(n_pages * 4096)
    src.array[:] = data.reshape(-1)
    eng.encrypt_host_pages(key, src, dst, ms.linear_nonce(BASE, STRIDE, TAG),
                           mode=MODES[mode])
    _sync()
    assert np.array_equal(dst.array.reshape(n_pages, 4096),
                          _want(key_b, data))
    assert np.array_equal(src.array.reshape(n_pages, 4096), data)
    # decrypt in place returns the plaintext
    eng.decrypt_host_pages(key, dst, dst, ms.linear_nonce(BASE, STRIDE, TAG),
                           mode=MODES[mode])
    _sync()
    assert np.array_equal(dst.array.reshape(n_pages, 4096), data)
    src.free()
    dst.free()
    eng.key_destroy(key)


@pytest.mark.parametrize("mode", list(MODES))
def test_torch_pinned_tensors_in_place(ms, eng, mode):
    _note("torch pinned in place mode=%s" % mode)
    import torch
    rng = np.random.default_rng(31)
    n = 2 * CHUNK + 5
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n)
    key = eng.key_load(key_b)
    buf = torch.from_numpy(data.reshape(-1).copy()).pin_memory()
    eng.encrypt_host_pages(key, buf, buf, ms.linear_nonce(BASE, STRIDE, TAG),
                           mode=MODES[mode])
    _sync()
    assert np.array_equal(buf.numpy().reshape(n, 4096), _want(key_b, data))
    eng.key_destroy(key)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("direction", ["host->dev", "dev->host"])
def test_mixed_host_and_device(ms, eng, mode, direction):
    _note("mixed %s mode=%s" % (direction, mode))
    import torch
    rng = np.random.default_rng(41)
    n = 2 * CHUNK + 9
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n)
    key = eng.key_load(key_b)
    host = eng.host_alloc(n * 4096)
    dev = torch.zeros(n * 4096, dtype=torch.uint8, device="cuda")
    nonce = ms.linear_nonce(BASE, STRIDE, TAG)
    if direction == "host->dev":
        host.array[:] = data.reshape(-1)
        eng.encrypt_host_pages(key, host, dev, nonce, mode=MODES[mode])
        _sync()
        got = dev.cpu().numpy()
    else:
        dev.copy_(torch.from_numpy(data.reshape(-1)))
        _sync()
        eng.encrypt_host_pages(key, dev, host, nonce, mode=MODES[mode])
        _sync()
        got = host.array.copy()
    assert np.array_equal(got.reshape(n, 4096), _want(key_b, data))
    host.free()
    eng.key_destroy(key)


@pytest.mark.parametrize("mode", ["mapped", "dma", "dma_in"])
def test_array_nonces(ms, eng, mode):
    _note("array nonces mode=%s" % mode)
    import torch
    rng = np.random.default_rng(51)
    n = CHUNK * 2 + 3
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n)
    nonces = np.frombuffer(rng.bytes(12 * n), dtype=np.uint8).reshape(n, 12)
    key = eng.key_load(key_b)
    src = eng.host_alloc(n * 4096)
    dst = eng.host_alloc(n * 4096)
    src.array[:] = data.reshape(-1)
    nd = torch.from_numpy(nonces.reshape(-1).copy()).to("cuda")
    eng.encrypt_host_pages(key, src, dst, ms.array_nonce(nd), mode=MODES[mode])
    _sync()
    want = oracle.cipher_pages(key_b, nonces, data)
    assert np.array_equal(dst.array.reshape(n, 4096), want)
    src.free()
    dst.free()
    eng.key_destroy(key)


def test_same_bytes_as_device_path(ms, eng):
    _note("host modes == device path")
    import torch
    rng = np.random.default_rng(61)
    n = 5 * CHUNK + 11
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n)
    key = eng.key_load(key_b)
    nonce = ms.linear_nonce(2**64 - 7, 4096, 0xFFFFFFFF)  # wraps mod 2^64
    d_src = torch.from_numpy(data.reshape(-1).copy()).to("cuda")
    d_dst = torch.zeros_like(d_src)
    eng.encrypt_pages(key, d_src, d_dst, nonce)
    ref = d_dst.cpu().numpy()
    src = eng.host_alloc(n * 4096)
    src.array[:] = data.reshape(-1)
    for mode in (1, 2, 3):
        dst = eng.host_alloc(n * 4096)
        eng.encrypt_host_pages(key, src, dst, nonce, mode=mode)
        _sync()
        assert np.array_equal(dst.array, ref), mode
        dst.free()
    want = oracle.cipher_pages(key_b, oracle.nonces_linear(n, 2**64 - 7, 4096,
                                                           0xFFFFFFFF), data)
    assert np.array_equal(ref.reshape(n, 4096), want)
    src.free()
    eng.key_destroy(key)


@pytest.mark.parametrize("mode", ["dma", "dma_in", "mapped"])
def test_stream_order_on_caller_stream(ms, eng, mode):
    """Work the caller enqueues before the call is seen by it, and work
    enqueued after it sees its output, on a non-default stream."""
    _note("stream order mode=%s" % mode)
    import torch
    rng = np.random.default_rng(71)
    n = 3 * CHUNK
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n)
    key = eng.key_load(key_b)
    host = eng.host_alloc(n * 4096)
    host.array[:] = data.reshape(-1)
    dev = torch.empty(n * 4096, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dev.fill_(0xA5)  # overwritten by the call, which must come after
        eng.encrypt_host_pages(key, host, dev,
                               ms.linear_nonce(BASE, STRIDE, TAG),
                               mode=MODES[mode], stream=s)
        after = dev.clone()  # must see the call's output
    s.synchronize()
    assert np.array_equal(after.cpu().numpy().reshape(n, 4096),
                          _want(key_b, data))
    host.free()
    eng.key_destroy(key)


def test_concurrent_staged_callers(ms, eng):
    _note("concurrent staged callers")
    import torch
    rng = np.random.default_rng(81)
    key_b = rng.bytes(32)
    key = eng.key_load(key_b)
    jobs = []
    for t in range(4):
        n = CHUNK * (t + 1) + 7 * t + 1
        data = workloads.random_pages(rng, n)
        src = eng.host_alloc(n * 4096)
        dst = eng.host_alloc(n * 4096)
        src.array[:] = data.reshape(-1)
        jobs.append((n, data, src, dst, 1000 + 4096 * n * t))
    errors = []

    def work(j):
        n, data, src, dst, base = j
        try:
            s = torch.cuda.Stream()
            for rep in range(3):
                eng.encrypt_host_pages(key, src, dst,
                                       ms.linear_nonce(base, STRIDE, TAG),
                                       mode=2 if rep % 2 == 0 else 3,
                                       stream=s)
            s.synchronize()
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(j,)) for j in jobs]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for n, data, src, dst, base in jobs:
        assert np.array_equal(dst.array.reshape(n, 4096),
                              _want(key_b, data, base=base))
        src.free()
        dst.free()
    eng.key_destroy(key)


def test_invalid_arguments_rejected(ms, eng):
    _note("host-path rejections")
    import torch
    rng = np.random.default_rng(91)
    key = eng.key_load(rng.bytes(32))
    n = 8
    host = eng.host_alloc(n * 4096)
    other = eng.host_alloc(n * 4096)
    nonce = ms.linear_nonce(0, 1, 0)
    ctx = eng.ctx
    pageable = np.zeros(n * 4096, dtype=np.uint8)
    # pageable memory
    assert ms.ms_encrypt_host_pages(ctx, key, pageable.ctypes.data,
                                    other.ptr, n, nonce, 1) == ms.MS_EINVAL
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, pageable.ctypes.data,
                                    n, nonce, 2) == ms.MS_EINVAL
    # range beyond the pinned allocation
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, other.ptr, n + 1,
                                    nonce, 1) == ms.MS_EINVAL
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr + 4096, other.ptr, n,
                                    nonce, 2) == ms.MS_EINVAL
    # misaligned, partial overlap, bad mode, bad key, bad nonce kind
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr + 8, other.ptr, 1,
                                    nonce, 1) == ms.MS_EINVAL
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, host.ptr + 4096, 2,
                                    nonce, 1) == ms.MS_EINVAL
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, other.ptr, 1, nonce,
                                    4) == ms.MS_EINVAL
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, other.ptr, 1, nonce,
                                    -1) == ms.MS_EINVAL
    assert ms.ms_encrypt_host_pages(ctx, key ^ (1 << 40), host.ptr,
                                    other.ptr, 1, nonce, 1) == ms.MS_ENOKEY
    bad = ms.linear_nonce(0, 1, 0)
    bad.kind = 5
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, other.ptr, 1, bad,
                                    1) == ms.MS_EINVAL
    # nonce arrays must be device memory
    host_nonce = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, other.ptr, 0, 0)
    assert ms.ms_encrypt_host_pages(ctx, key, host.ptr, host.ptr, 1,
                                    host_nonce, 1) == ms.MS_EINVAL
    # zero pages is a no-op, even with a null pointer
    assert ms.ms_encrypt_host_pages(ctx, key, None, None, 0, nonce, 1) == \
        ms.MS_OK
    # frees: unknown pointer, double free
    assert ms.ms_host_free(ctx, pageable.ctypes.data) == ms.MS_EINVAL
    p = host.ptr
    host.free()
    assert ms.ms_host_free(ctx, p) == ms.MS_EINVAL
    assert ms.ms_host_alloc(ctx, 0)[0] == ms.MS_EINVAL
    # the engine still works afterwards
    d = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    eng.encrypt_host_pages(key, other, d, nonce, n_pages=1)
    _sync()
    other.free()
    eng.key_destroy(key)


def test_host_alloc_is_zeroed_and_mapped(ms, eng):
    _note("host alloc")
    import torch
    b = eng.host_alloc(3 * 4096 + 16)
    assert not b.array.any()
    b.array[:] = 7
    # the copy kernel reads it through the GPU mapping
    d = torch.zeros(3 * 4096 + 16, dtype=torch.uint8, device="cuda")
    assert ms.ms_probe_link(eng.ctx, b.ptr, d.data_ptr(), 3 * 4096 + 16, 0,
                            torch.cuda.current_stream().cuda_stream) == \
        ms.MS_OK
    _sync()
    assert bool((d == 7).all())
    d.fill_(9)
    assert ms.ms_probe_link(eng.ctx, d.data_ptr(), b.ptr, 3 * 4096 + 16, 1,
                            torch.cuda.current_stream().cuda_stream) == \
        ms.MS_OK
    _sync()
    assert (b.array == 9).all()
    b.free()


def test_large_run_sampled_against_oracle(ms):
    """512 MiB of host pages (8 default staging chunks) through every mode,
    one call each, with a deterministic sample of pages checked against the
    oracle."""
    _note("large host run 131072 pages")
    n = 131072
    with ms.Engine(0) as e:
        rng = np.random.default_rng(101)
        key_b = rng.bytes(32)
        key = e.key_load(key_b)
        src = e.host_alloc(n * 4096)
        dst = e.host_alloc(n * 4096)
        data = src.array.reshape(n, 4096)
        data[:] = rng.integers(0, 256, size=(n, 4096), dtype=np.uint8)
        for mode in (0, 1, 2, 3):
            dst.array[:] = 0
            e.encrypt_host_pages(key, src, dst,
                                 ms.linear_nonce(BASE, STRIDE, TAG), mode=mode)
            _sync()
            idx = np.unique(np.concatenate([[0, 1, n - 2, n - 1],
                                            rng.integers(0, n, 60)]))
            got = dst.array.reshape(n, 4096)[idx]
            nonces = oracle.nonces_linear(n, BASE, STRIDE, TAG)[idx]
            want = oracle.cipher_pages(key_b, nonces, data[idx])
            assert np.array_equal(got, want), mode
        src.free()
        dst.free()
        e.key_destroy(key)
