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
        assert ms.ms_resident_submit(h, pageable.ctypes.data, host.ptr, 1,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, pageable.ctypes.data, 1,
                                     lin)[0] == ms.MS_EINVAL
        # device memory beyond its allocation, or misaligned
        assert ms.ms_resident_submit(h, dev.data_ptr(), host.ptr, 5,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, dev.data_ptr() + 8, host.ptr, 1,
                                     lin)[0] == ms.MS_EINVAL
        # a one-key engine holds key index 0 only
        assert ms.ms_resident_submit_keyed(h, 1, host.ptr, host.ptr, 1,
                                           lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 5,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, host.ptr + 4096, 2,
                                     lin)[0] == ms.MS_EINVAL
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 0,
                                     lin)[0] == ms.MS_EINVAL
        # a nonce array in pageable memory, or not 4-byte aligned
        arr = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, pageable.ctypes.data, 0, 0)
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 1,
                                     arr)[0] == ms.MS_EINVAL
        arr = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, dev.data_ptr() + 2, 0, 0)
        assert ms.ms_resident_submit(h, host.ptr, host.ptr, 1,
                                     arr)[0] == ms.MS_EINVAL
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


@pytest.mark.parametrize("rounds", [20, 12, 8])
def test_salsa20_resident_kernels(ms, rounds):
    """A Salsa20 context's engine dispatches the Salsa20 kernel of its round
    count: host pages with one key in registers, and device pages with two
    keys from the key table, both equal to the Salsa20 oracle."""
    _note("resident salsa20 rounds=%d" % rounds)
    import torch
    rng = np.random.default_rng(60 + rounds)
    key_b = [rng.bytes(32), rng.bytes(32)]
    n = 37
    data = workloads.random_pages(rng, n)
    e = ms.Engine(0, cipher=ms.MS_CIPHER_SALSA, rounds=rounds)
    try:
        buf = e.host_alloc(n * 4096)
        buf.array[:] = data.reshape(-1)
        r = e.resident(key=key_b[0], workers=32, idle_limit_ms=IDLE_MS)
        try:
            r.wait([r.submit(buf, buf, ms.linear_nonce(BASE, STRIDE, TAG))])
        finally:
            r.stop()
        want = [oracle.cipher_pages(
            k, oracle.nonces_linear(n, BASE, STRIDE, TAG), data,
            rounds=rounds, cipher="salsa") for k in key_b]
        assert np.array_equal(buf.array.reshape(n, 4096), want[0])
        buf.free()
        handles = [e.key_load(k) for k in key_b]
        src = _dev(torch, data)
        out = [torch.zeros_like(src) for _ in key_b]
        r = e.resident(keys=handles, workers=64, desc_pages=1,
                       idle_limit_ms=IDLE_MS)
        try:
            r.wait([r.submit(src, o, ms.linear_nonce(BASE, STRIDE, TAG),
                             key_index=i) for i, o in enumerate(out)])
        finally:
            r.stop()
        for i, o in enumerate(out):
            assert np.array_equal(o.cpu().numpy().reshape(n, 4096),
                                  want[i]), i
    finally:
        e.close()


def _dev(torch, data):
    return torch.from_numpy(data.reshape(-1).copy()).to("cuda")


@pytest.mark.parametrize("n_pages", [1, 17, 300])
@pytest.mark.parametrize("in_place", [False, True])
def test_device_pages_bit_exact(ms, eng, n_pages, in_place):
    """Pages in HBM go through the same ring: no launch per request."""
    _note("resident device n_pages=%d in_place=%s" % (n_pages, in_place))
    import torch
    rng = np.random.default_rng(7000 + n_pages)
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, n_pages)
    src = _dev(torch, data)
    dst = src if in_place else torch.zeros_like(src)
    r = _start(eng, key_b, workers=128, desc_pages=4)
    try:
        r.wait([r.submit(src, dst, ms.linear_nonce(BASE, STRIDE, TAG))])
        torch.cuda.synchronize()
        got = dst.cpu().numpy().reshape(n_pages, 4096)
        assert np.array_equal(got, _want(key_b, data))
        r.wait([r.submit(dst, dst, ms.linear_nonce(BASE, STRIDE, TAG))])
        assert np.array_equal(dst.cpu().numpy().reshape(n_pages, 4096), data)
    finally:
        r.stop()


def test_host_to_device_and_back(ms, eng):
    """A host page can be ciphered into HBM and an HBM page out to the
    host: each direction matches the oracle."""
    _note("resident host<->device")
    import torch
    rng = np.random.default_rng(71)
    key_b = rng.bytes(32)
    n = 40
    data = workloads.random_pages(rng, n)
    host = eng.host_alloc(n * 4096)
    host.array[:] = data.reshape(-1)
    dev = torch.zeros(n * 4096, dtype=torch.uint8, device="cuda")
    r = _start(eng, key_b, workers=64, desc_pages=16)
    try:
        r.wait([r.submit(host, dev, ms.linear_nonce(BASE, STRIDE, TAG))])
        want = _want(key_b, data)
        assert np.array_equal(dev.cpu().numpy().reshape(n, 4096), want)
        host.array[:] = 0
        r.wait([r.submit(dev, host, ms.linear_nonce(BASE, STRIDE, TAG))])
        assert np.array_equal(host.array.reshape(n, 4096), data)
    finally:
        r.stop()
    host.free()


def test_many_keys_from_the_key_table(ms):
    """An engine started from key handles: key index i ciphers with the
    i-th handle's key, in any interleaving; its device copy of the keys is
    wiped; destroying a handle afterwards does not reach the engine."""
    _note("resident 64 keys")
    import torch
    eng = ms.Engine(0)   # a key table of its own: all 64 rows are used
    rng = np.random.default_rng(72)
    key_bs = [rng.bytes(32) for _ in range(64)]
    handles = [eng.key_load(k) for k in key_bs]
    n = 6
    picks = [0, 63, 1, 31, 32, 62, 5, 5, 17]
    data = [workloads.random_pages(rng, n) for _ in picks]
    src = [_dev(torch, d) for d in data]
    dst = [torch.zeros_like(s) for s in src]
    r = eng.resident(keys=handles, workers=96, desc_pages=2,
                     idle_limit_ms=IDLE_MS)
    try:
        assert r.key_wiped() == 1
        tks = [r.submit(s, o, ms.linear_nonce(BASE + 4096 * 64 * j, STRIDE,
                                              TAG + j), key_index=k)
               for j, (k, s, o) in enumerate(zip(picks, src, dst))]
        r.wait(tks)
        for j, (k, d, o) in enumerate(zip(picks, data, dst)):
            want = _want(key_bs[k], d, base=BASE + 4096 * 64 * j,
                         tag=TAG + j)
            assert np.array_equal(o.cpu().numpy().reshape(n, 4096), want), j
        # the same bytes as the launch path with the context's key
        ref = torch.zeros_like(src[1])
        eng.encrypt_pages(handles[63], src[1], ref,
                          ms.linear_nonce(BASE + 4096 * 64, STRIDE, TAG + 1))
        torch.cuda.synchronize()
        assert torch.equal(ref, dst[1])
        assert ms.ms_resident_submit_keyed(r.handle, 64, src[0].data_ptr(),
                                           src[0].data_ptr(), 1,
                                           ms.linear_nonce(0, 1, 0))[0] \
            == ms.MS_EINVAL
        eng.key_destroy(handles[5])
        out = torch.zeros_like(src[6])
        r.wait([r.submit(src[6], out, ms.linear_nonce(BASE + 4096 * 64 * 6,
                                                      STRIDE, TAG + 6),
                         key_index=5)])
        assert torch.equal(out, dst[6])
    finally:
        r.stop()
        eng.close()


def test_key_table_start_rejections(ms, eng):
    _note("resident key table rejections")
    rng = np.random.default_rng(73)
    hs = [eng.key_load(rng.bytes(32)) for _ in range(2)]
    cfg = ms.ms_resident_config_default()
    cfg.idle_limit_ms = IDLE_MS
    try:
        assert ms.ms_resident_start_keys(eng.ctx, cfg, [])[0] == ms.MS_EINVAL
        assert ms.ms_resident_start_keys(eng.ctx, cfg, hs * 33)[0] == \
            ms.MS_EINVAL
        bad = hs[1] ^ (1 << 40)   # a stale generation
        assert ms.ms_resident_start_keys(eng.ctx, cfg, [hs[0], bad])[0] == \
            ms.MS_ENOKEY
    finally:
        for h in hs:
            eng.key_destroy(h)


def test_device_pages_producers_small_ring(ms):
    """4 host threads, 200 requests of 1..64 device pages, one descriptor
    per page, a 128-slot ring and 3 client keys: requests finish out of
    order, counters and completion slots are reused many times over, and
    every output matches the oracle."""
    _note("resident device producers small ring")
    import torch
    eng = ms.Engine(0)
    rng = np.random.default_rng(74)
    key_bs = [rng.bytes(32) for _ in range(3)]
    handles = [eng.key_load(k) for k in key_bs]
    jobs = []
    for t in range(4):
        for i in range(50):
            n = int(rng.integers(1, 65))
            data = workloads.random_pages(rng, n)
            k = int(rng.integers(0, 3))
            base = BASE + 4096 * 100000 * (t * 50 + i)
            jobs.append((t, n, data, k, base, _dev(torch, data)))
    outs = {id(j): torch.zeros(j[1] * 4096, dtype=torch.uint8, device="cuda")
            for j in jobs}
    torch.cuda.synchronize()
    r = eng.resident(keys=handles, workers=256, ring_depth=128, desc_pages=1,
                     idle_limit_ms=IDLE_MS)
    errors, tickets = [], {}

    def producer(t):
        try:
            for j in [j for j in jobs if j[0] == t]:
                _, n, data, k, base, src = j
                while True:
                    try:
                        tickets[id(j)] = r.submit(
                            src, outs[id(j)], ms.linear_nonce(base, STRIDE, TAG),
                            key_index=k)
                        break
                    except ms.MemShieldError as e:
                        if e.status != ms.MS_EAGAIN:
                            raise
                        time.sleep(0.0001)
        except Exception as e:  # reported below
            errors.append(e)

    try:
        th = [threading.Thread(target=producer, args=(t,)) for t in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors
        r.wait(list(tickets.values()))
        for j in jobs:
            _, n, data, k, base, _ = j
            got = outs[id(j)].cpu().numpy().reshape(n, 4096)
            assert np.array_equal(got, _want(key_bs[k], data, base=base)), \
                (n, k, base)
    finally:
        r.stop()
        eng.close()


@pytest.mark.parametrize("where", ["device", "host"])
def test_array_nonces_bit_exact(ms, eng, where):
    """Nonces from an array of 12-byte values (in HBM with device pages, in
    pinned host memory with host pages), as for the launch paths."""
    _note("resident array nonces %s" % where)
    import torch
    rng = np.random.default_rng(75)
    key_b = rng.bytes(32)
    n = 37
    data = workloads.random_pages(rng, n)
    nonces = np.frombuffer(rng.bytes(12 * n), dtype=np.uint8).reshape(n, 12)
    want = oracle.cipher_pages(key_b, nonces, data)
    r = _start(eng, key_b, workers=64, desc_pages=4)
    try:
        if where == "device":
            src = _dev(torch, data)
            dst = torch.zeros_like(src)
            arr = torch.from_numpy(nonces.reshape(-1).copy()).to("cuda")
            torch.cuda.synchronize()
            nonce = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, arr.data_ptr(), 0, 0)
            r.wait([r.submit(src, dst, nonce)])
            got = dst.cpu().numpy().reshape(n, 4096)
        else:
            src = eng.host_alloc(n * 4096)
            dst = eng.host_alloc(n * 4096)
            arr = eng.host_alloc(12 * n)
            src.array[:] = data.reshape(-1)
            arr.array[:] = nonces.reshape(-1)
            nonce = ms.ms_nonce(ms.MS_NONCE_ARRAY, 0, arr.ptr, 0, 0)
            r.wait([r.submit(src, dst, nonce)])
            got = dst.array.reshape(n, 4096).copy()
            for b in (src, dst, arr):
                b.free()
        assert np.array_equal(got, want)
    finally:
        r.stop()


def test_resident_holds_tensors_of_requests_in_flight(ms, eng):
    """Device tensors given to the ring stay alive while their ticket is in
    flight even when the caller drops them; poll reporting the ticket
    finished releases them."""
    _note("resident tensors held while in flight")
    import gc
    import weakref

    import torch
    rng = np.random.default_rng(77)
    key_b = rng.bytes(32)
    data = workloads.random_pages(rng, 40)
    src = torch.from_numpy(data.reshape(-1)).to("cuda")
    dst = torch.zeros_like(src)
    torch.cuda.synchronize()
    refs = [weakref.ref(src), weakref.ref(dst)]
    r = _start(eng, key_b, workers=64, desc_pages=4)
    try:
        t = r.submit(src, dst, ms.linear_nonce(BASE, STRIDE, TAG))
        out = dst  # one tensor kept to check the bytes
        del src, dst
        gc.collect()
        assert all(w() is not None for w in refs)
        r.wait([t])
        gc.collect()
        assert refs[0]() is None
        assert np.array_equal(out.cpu().numpy().reshape(40, 4096),
                              _want(key_b, data))
    finally:
        r.stop()
