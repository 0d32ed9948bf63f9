"""GPU tests of the resident-key engine (include/memshield_resident.h), the
paper's own design: a kernel that keeps the key in registers and takes pages
from a ring in mapped host memory.  Outputs are compared byte for byte with
the CPU oracle.  Every engine here runs with a short idle limit, so the
kernel ends by itself within seconds even if a test fails half-way."""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2004_09252_amd import workloads

pytestmark = pytest.mark.gpu

IDLE_MS = 3000
BASE, STRIDE, TAG = 0x7F0000000000 + 4096 * 91, 4096, 4321


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


def _want(key_b, data, base=BASE, stride=STRIDE, tag=TAG):
    return oracle.cipher_pages(
        key_b, oracle.nonces_linear(data.shape[0], base, stride, tag), data)


def _start(eng, key_b, **cfg):
    cfg.setdefault("idle_limit_ms", IDLE_MS)
    return eng.resident(key=key_b, **cfg)


@pytest.mark.parametrize("n_pages", [1, 2, 15, 16, 17, 100, 1000])
@pytest.mark.parametrize("in_place", [False, True])
def test_bit_exact_against_oracle(ms, eng, n_pages, in_place):
    _note("resident n_pages=%d in_place=%s" % (n_pages, in_place))
    rng = np.random.default_rng(5000 + n_pages)
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n_pages)
    src = eng.host_alloc(n_pages * 4096)
    dst = src if in_place else eng.host_alloc(n_pages * 4096)
    src.array[:] = data.reshape(-1)
    r = _start(eng, key_b, workers=64, desc_pages=16)
    try:
        t = r.submit(src, dst, ms.linear_nonce(BASE, STRIDE, TAG))
        r.wait([t])
        assert np.array_equal(dst.array.reshape(n_pages, 4096),
                              _want(key_b, data))
        # the same call decrypts
        t = r.submit(dst, dst, ms.linear_nonce(BASE, STRIDE, TAG))
        r.wait([t])
        assert np.array_equal(dst.array.reshape(n_pages, 4096), data)
    finally:
        r.stop()
    src.free()
    if not in_place:
        dst.free()


def test_key_lives_only_in_registers(ms, eng):
    _note("resident key purge")
    rng = np.random.default_rng(11)
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, 40)
    buf = eng.host_alloc(40 * 4096)
    buf.array[:] = data.reshape(-1)
    r = _start(eng, key_b)
    try:
        assert r.alive()
        # device copy zeroed by the kernel, host staging wiped by the library
        assert r.key_wiped() == 1
        t = r.submit(buf, buf, ms.linear_nonce(BASE, STRIDE, TAG))
        r.wait([t])
        assert np.array_equal(buf.array.reshape(40, 4096), _want(key_b, data))
        assert r.key_wiped() == 1
    finally:
        r.stop()
    buf.free()


def test_generated_keys_round_trip_and_differ(ms, eng):
    _note("resident generated keys")
    rng = np.random.default_rng(12)
    data = workloads.random_pages(rng, 8)
    a = eng.host_alloc(8 * 4096)
    b = eng.host_alloc(8 * 4096)
    c = eng.host_alloc(8 * 4096)
    a.array[:] = data.reshape(-1)
    r1 = eng.resident(idle_limit_ms=IDLE_MS)
    r2 = eng.resident(idle_limit_ms=IDLE_MS)
    try:
        n = ms.linear_nonce(BASE, STRIDE, TAG)
        r1.wait([r1.submit(a, b, n)])
        r2.wait([r2.submit(a, c, n)])
        assert not np.array_equal(b.array, c.array)
        assert not np.array_equal(b.array, a.array)
        r1.wait([r1.submit(b, b, n)])
        assert np.array_equal(b.array, a.array)
    finally:
        r1.stop()
        r2.stop()
    for x in (a, b, c):
        x.free()


def test_same_bytes_as_launch_path(ms, eng):
    _note("resident == launch path")
    rng = np.random.default_rng(13)
    key_b = rng.bytes(32)
    n = 300
    data = workloads.random_pages(rng, n)
    src = eng.host_alloc(n * 4096)
    d1 = eng.host_alloc(n * 4096)
    d2 = eng.host_alloc(n * 4096)
    src.array[:] = data.reshape(-1)
    nonce = ms.linear_nonce(2**64 - 4096 * 5, 4096, 0xFFFFFFFF)  # wraps
    key = eng.key_load(key_b)
    import torch
    s = torch.cuda.Stream()
    eng.encrypt_host_pages(key, src, d1, nonce, mode=ms.MS_HOST_MAPPED,
                           stream=s)
    s.synchronize()
    eng.key_destroy(key)
    r = _start(eng, key_b, desc_pages=7)
    try:
        r.wait([r.submit(src, d2, nonce)])
    finally:
        r.stop()
    assert np.array_equal(d1.array, d2.array)
    assert np.array_equal(d2.array.reshape(n, 4096),
                          _want(key_b, data, 2**64 - 4096 * 5, 4096,
                                0xFFFFFFFF))
    for x in (src, d1, d2):
        x.free()


def test_many_producers(ms, eng):
    """8 host threads submit 40 requests each (1..40 pages, own buffers)."""
    _note("resident many producers")
    rng = np.random.default_rng(14)
    key_b = rng.bytes(32)
    jobs = []
    for t in range(8):
        for i in range(40):
            n = int(rng.integers(1, 41))
            data = workloads.random_pages(rng, n)
            src = eng.host_alloc(n * 4096)
            src.array[:] = data.reshape(-1)
            dst = eng.host_alloc(n * 4096)
            base = BASE + 4096 * 100000 * (t * 40 + i)
            jobs.append((t, n, data, src, dst, base))
    r = _start(eng, key_b, workers=128, ring_depth=64, desc_pages=4)
    errors = []
    tickets = {}

    def producer(t):
        try:
            for j in [j for j in jobs if j[0] == t]:
                _, n, data, src, dst, base = j
                while True:
                    try:
                        tickets[id(j)] = r.submit(
                            src, dst, ms.linear_nonce(base, STRIDE, TAG))
                        break
                    except ms.MemShieldError as e:
                        if e.status != ms.MS_EAGAIN:
                            raise
                        time.sleep(0.0002)
        except Exception as e:  # reported below
            errors.append(e)

    try:
        th = [threading.Thread(target=producer, args=(t,)) for t in range(8)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors
        r.wait(list(tickets.values()))
    finally:
        r.stop()
    for _, n, data, src, dst, base in jobs:
        assert np.array_equal(dst.array.reshape(n, 4096),
                              _want(key_b, data, base=base))
        src.free()
        dst.free()


def test_ring_wraps_many_times(ms, eng):
    _note("resident ring wrap")
    rng = np.random.default_rng(15)
    key_b = rng.bytes(32)
    n = 3
    data = workloads.random_pages(rng, n)
    src = eng.host_alloc(n * 4096)
    dst = eng.host_alloc(n * 4096)
    src.array[:] = data.reshape(-1)
    r = _start(eng, key_b, ring_depth=16, desc_pages=1, workers=8)
    try:
        for i in range(200):
            base = BASE + 4096 * 7 * i
            r.wait([r.submit(src, dst, ms.linear_nonce(base, STRIDE, TAG))])
            if i % 37 == 0:
                assert np.array_equal(dst.array.reshape(n, 4096),
                                      _want(key_b, data, base=base))
        # a request needing more descriptors than the ring holds can never fit
        big = eng.host_alloc(17 * 4096)
        st, _ = ms.ms_resident_submit(r.handle, big.ptr, big.ptr, 17,
                                      ms.linear_nonce(0, 1, 0))
        assert st == ms.MS_EINVAL
        big.free()
    finally:
        r.stop()
    src.free()
    dst.free()


def test_rejections(ms, eng):
    _note("resident rejections")
    import torch
    rng = np.random.default_rng(16)
    host = eng.host_alloc(4 * 4096)
    dev = torch.zeros(4 * 4096, dtype=torch.uint8, device="cuda")
    pageable = np.zeros(4 * 4096, dtype=np.uint8)
    bad = ms.ms_resident_config_default()
    bad.ring_depth = 1000
    assert ms.ms_resident_start(eng.ctx, bad, None)[0] == ms.MS_EINVAL
    bad = ms.ms_resident_config_default()
    bad.workers = 1 << 20
    assert ms.ms_resident_start(eng.ctx, bad, None)[0] == ms.MS_EINVAL
    r = _start(eng, rng.bytes(32), workers=16)
    try:
        h = r.handle
        lin = ms.linear_nonce(0, 1, 0)
        assert ms.ms_resident_submit(h, dev.data_ptr(), host.ptr, 1,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, pageable.ctypes.data, host.ptr, 1,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 5,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, host.ptr + 4096, 2,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 0,
                                     lin)[0] == ms.MS_EINVAL
        arr = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, dev.data_ptr(), 0, 0)
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 1,
                                     arr)[0] == ms.MS_ENOTSUP
        assert ms.ms_resident_poll(h, [12345 << 24 | 1])[0] == ms.MS_EINVAL
        t = r.submit(host, host, lin, n_pages=1)
        r.wait([t])
    finally:
        r.stop()
    host.free()


def test_idle_limit_ends_the_kernel(ms, eng):
    """Forced from the host: a 150 ms idle limit ends the kernel by itself;
    the key is gone and submissions report it."""
    _note("resident idle limit")
    rng = np.random.default_rng(17)
    buf = eng.host_alloc(4096)
    r = _start(eng, rng.bytes(32), idle_limit_ms=150, workers=8)
    try:
        assert r.alive()
        t0 = time.time()
        while r.alive() and time.time() - t0 < 10:
            time.sleep(0.05)
        assert not r.alive()
        st, _ = ms.ms_resident_submit(r.handle, buf.ptr, buf.ptr, 1,
                                      ms.linear_nonce(0, 1, 0))
        assert st == ms.MS_ECLOSED
    finally:
        r.stop()
    buf.free()


def test_other_device_work_runs_beside_it(ms, eng):
    """Launch-path work and torch kernels on other streams finish while the
    resident kernel holds its share of the device."""
    _note("resident beside other work")
    import torch
    rng = np.random.default_rng(18)
    key_b = rng.bytes(32)
    # load the matrix-product libraries before the timed region
    w = torch.randn(512, 512, device="cuda")
    float((w @ w).sum().cpu())
    r = _start(eng, key_b, idle_limit_ms=5000)
    try:
        key = eng.key_load(key_b)
        data = workloads.random_pages(rng, 256)
        s = torch.cuda.Stream()
        t0 = time.time()
        with torch.cuda.stream(s):
            src = torch.from_numpy(data.reshape(-1).copy()).to("cuda",
                                                               non_blocking=False)
            dst = torch.empty_like(src)
            eng.encrypt_pages(key, src, dst, ms.linear_nonce(BASE, STRIDE, TAG),
                              stream=s)
            x = torch.randn(512, 512, device="cuda")
            y = (x @ x).sum()
        s.synchronize()
        torch.cuda.synchronize()  # device-wide: must not wait for the kernel
        elapsed = time.time() - t0
        assert elapsed < 2.5, elapsed   # not held until the idle limit
        assert np.isfinite(float(y.cpu()))
        assert np.array_equal(dst.cpu().numpy().reshape(256, 4096),
                              _want(key_b, data))
        assert r.alive()
        buf = eng.host_alloc(256 * 4096)
        buf.array[:] = data.reshape(-1)
        r.wait([r.submit(buf, buf, ms.linear_nonce(BASE, STRIDE, TAG))])
        assert np.array_equal(buf.array, dst.cpu().numpy())
        buf.free()
    finally:
        r.stop()
    eng.key_destroy(key)


def test_shutdown_stops_running_engines(ms):
    """ms_shutdown itself stops engines the caller left running."""
    _note("resident stopped by shutdown")
    e = ms.Engine(0)
    r = e.resident(idle_limit_ms=20000, workers=32)
    assert r.alive()
    e._residents.clear()  # leave it to the native shutdown
    t0 = time.time()
    assert ms.ms_shutdown(e.ctx) == ms.MS_OK
    e.ctx = None
    assert time.time() - t0 < 5.0


@pytest.mark.parametrize("rounds", [12, 8])
def test_reduced_round_resident_kernels(ms, rounds):
    """The engine dispatches the kernel of its context's round count."""
    _note("resident rounds=%d" % rounds)
    rng = np.random.default_rng(40 + rounds)
    key_b = rng.bytes(32)
    n = 37
    data = workloads.random_pages(rng, n)
    e = ms.Engine(0, rounds=rounds)
    try:
        buf = e.host_alloc(n * 4096)
        buf.array[:] = data.reshape(-1)
        r = e.resident(key=key_b, workers=32, idle_limit_ms=IDLE_MS)
        try:
            r.wait([r.submit(buf, buf, ms.linear_nonce(BASE, STRIDE, TAG))])
        finally:
            r.stop()
        want = oracle.cipher_pages(
            key_b, oracle.nonces_linear(n, BASE, STRIDE, TAG), data,
            rounds=rounds)
        assert np.array_equal(buf.array.reshape(n, 4096), want)
        buf.free()
    finally:
        e.close()
