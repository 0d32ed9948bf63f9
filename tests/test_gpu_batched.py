"""GPU parity of the fused batched launch (many requests, many keys, one
persistent launch replayed from a captured hipGraph) against the CPU oracle,
request by request, bit-exact.  Each page's output depends only on its key,
nonce and bytes (paper section 4.4: blocks and pages are independent), so a
request's output in any batch must equal the oracle run on that request
alone."""
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


def _layout(ms, eng, w, keys, src, dst, rng=None, array_every=0,
            nonce_arrays=None):
    """ms_request array for workload `w` laid out back to back in src/dst."""
    reqs, off = [], 0
    for i, r in enumerate(w.requests):
        if array_every and i % array_every == 0:
            nonce = ms.array_nonce(nonce_arrays[i])
        else:
            nonce = ms.linear_nonce(r.va, 4096, r.pid)
        reqs.append(ms.request(keys[r.client], src, dst, r.n_pages, nonce,
                               op=r.op, client=r.client,
                               src_offset_pages=off, dst_offset_pages=off))
        off += r.n_pages
    return (ms.ms_request * len(reqs))(*reqs)


def _expected(w, inputs, nonce_host):
    """Per request: the oracle on that request alone."""
    out = []
    for i, r in enumerate(w.requests):
        out.append(oracle.cipher_pages(w.keys[r.client], nonce_host[i],
                                       inputs[i], threads=HOST_THREADS))
    return out


def _linear_nonces(w):
    return [oracle.nonces_linear(r.n_pages, r.va, 4096, r.pid)
            for r in w.requests]


def test_batched_512_requests_full_config(ms, eng):
    """512 requests from 32 clients, page counts log-uniform in [1, 4096],
    50/50 encrypt/decrypt; decrypt inputs are oracle ciphertexts."""
    _note("batched seed=3 512 requests")
    import torch
    w = workloads.batched(seed=3)
    nh = _linear_nonces(w)
    inputs = []
    for i, r in enumerate(w.requests):
        if r.op == 1:   # decrypt: input is the oracle's ciphertext
            inputs.append(oracle.cipher_pages(w.keys[r.client], nh[i],
                                              w.plain[i],
                                              threads=HOST_THREADS))
        else:
            inputs.append(w.plain[i])
    flat = np.concatenate([x.reshape(-1) for x in inputs])
    keys = [eng.key_load(k) for k in w.keys]
    src = torch.from_numpy(flat).to("cuda")
    dst = torch.zeros_like(src)
    arr = _layout(ms, eng, w, keys, src, dst)
    eng.process_batch(arr)
    got = dst.cpu().numpy()
    off = 0
    for i, r in enumerate(w.requests):
        n = r.n_pages * 4096
        want = w.plain[i] if r.op == 1 else oracle.cipher_pages(
            w.keys[r.client], nh[i], w.plain[i], threads=HOST_THREADS)
        assert np.array_equal(got[off:off + n], want.reshape(-1)), \
            "request %d (client %d, %d pages, op %d)" % (i, r.client,
                                                         r.n_pages, r.op)
        off += n
    for k in keys:
        eng.key_destroy(k)


def _small(seed, n_requests=40, max_pages=64):
    return workloads.batched(seed=seed, n_requests=n_requests, n_clients=5,
                             max_pages=max_pages)


@pytest.mark.parametrize("ppw,unroll,wpc", [(1, 1, 8), (1, 2, 32), (3, 2, 16),
                                            (8, 1, 24), (64, 2, 4),
                                            (4096, 1, 1)])
def test_batched_any_tiling_same_bytes(ms, eng, ppw, unroll, wpc):
    _note("tiling ppw=%d unroll=%d wpc=%d" % (ppw, unroll, wpc))
    import torch
    w = _small(11)
    nh = _linear_nonces(w)
    keys = [eng.key_load(k) for k in w.keys]
    flat = np.concatenate([x.reshape(-1) for x in w.plain])
    src = torch.from_numpy(flat).to("cuda")
    dst = torch.zeros_like(src)
    arr = _layout(ms, eng, w, keys, src, dst)
    assert ms.ms_set_tuning(eng.ctx, ms.ms_tuning(ppw, unroll, wpc, 0,
                                                  0.0)) == 0
    try:
        eng.process_batch(arr)
        got = dst.cpu().numpy()
    finally:
        ms.ms_set_tuning(eng.ctx, None)
    want = np.concatenate([x.reshape(-1) for x in _expected(w, w.plain, nh)])
    assert np.array_equal(got, want)
    for k in keys:
        eng.key_destroy(k)


def test_graph_replays_with_eager_work_between(ms, eng):
    """The captured graph is replayed several times; between replays the
    program does its own eager GPU work and synchronizes; every replay must
    reproduce the eager (plain-launch) result."""
    _note("graph replays")
    import torch
    w = _small(12, n_requests=30, max_pages=200)
    nh = _linear_nonces(w)
    keys = [eng.key_load(k) for k in w.keys]
    flat = np.concatenate([x.reshape(-1) for x in w.plain])
    src = torch.from_numpy(flat).to("cuda")
    dst = torch.empty_like(src)
    arr = _layout(ms, eng, w, keys, src, dst)
    # eager reference: one plain launch per request
    ref = torch.zeros_like(src)
    off = 0
    for i, r in enumerate(w.requests):
        eng.encrypt_pages(keys[r.client], src[off * 4096:], ref[off * 4096:],
                          ms.linear_nonce(r.va, 4096, r.pid),
                          n_pages=r.n_pages)
        off += r.n_pages
    torch.cuda.synchronize()
    for rep in range(5):
        dst.fill_(rep)
        scratch = torch.randn(1 << 20, device="cuda").sum()  # eager work
        eng.process_batch(arr)
        torch.cuda.synchronize()
        assert torch.equal(dst, ref), "replay %d differs" % rep
        del scratch
    want = np.concatenate([x.reshape(-1) for x in _expected(w, w.plain, nh)])
    assert np.array_equal(ref.cpu().numpy(), want)
    for k in keys:
        eng.key_destroy(k)


def test_batches_of_changing_size_reuse_every_buffer(ms):
    """Calls of 1024, 3 and 200 requests in an order that reuses each of
    the context's batch buffers with a different size, so the descriptor
    copy (a graph node, or a direct launch) changes size and grid from call
    to call: every call's output equals the oracle, request by request, in
    both launch forms."""
    import torch
    sizes = [1024, 3, 200, 3, 1024, 200, 3, 1024, 200]
    ws = {n: _small(60 + n % 7, n_requests=n, max_pages=3)
          for n in sorted(set(sizes))}
    want = {n: np.concatenate([x.reshape(-1) for x in
                               _expected(w, w.plain, _linear_nonces(w))])
            for n, w in ws.items()}
    stream = torch.cuda.current_stream()
    for use_graphs in (1, 0):
        _note("changing batch sizes, use_graphs=%d" % use_graphs)
        e = ms.Engine(0, use_graphs=use_graphs)
        try:
            data = {}
            for n, w in ws.items():
                keys = [e.key_load(k) for k in w.keys]
                flat = np.concatenate([x.reshape(-1) for x in w.plain])
                src = torch.from_numpy(flat).to("cuda")
                dst = torch.zeros_like(src)
                data[n] = (src, dst, _layout(ms, e, w, keys, src, dst))
            for i, n in enumerate(sizes):
                src, dst, arr = data[n]
                dst.fill_(i + 1)
                e.process_batch(arr, stream=stream)
                torch.cuda.synchronize()
                assert np.array_equal(dst.cpu().numpy(), want[n]), \
                    (use_graphs, i, n)
        finally:
            e.close()


def test_batched_mixed_nonce_kinds_empty_and_in_place(ms, eng):
    _note("mixed nonce kinds, empty requests, in place")
    import torch
    w = _small(13, n_requests=25, max_pages=40)
    rng = np.random.default_rng(13)
    nonce_arrays, nh = [], _linear_nonces(w)
    for i, r in enumerate(w.requests):
        a = np.frombuffer(rng.bytes(12 * r.n_pages), np.uint8).reshape(-1, 12)
        nonce_arrays.append(torch.from_numpy(a.copy().reshape(-1)).to("cuda"))
        if i % 3 == 0:
            nh[i] = a
    keys = [eng.key_load(k) for k in w.keys]
    flat = np.concatenate([x.reshape(-1) for x in w.plain])
    buf = torch.from_numpy(flat).to("cuda")
    arr = _layout(ms, eng, w, keys, buf, buf, array_every=3,
                  nonce_arrays=nonce_arrays)     # in place
    # add two empty requests: they are skipped
    empty = ms.request(keys[0], buf, buf, 0, ms.linear_nonce(0, 1, 0))
    full = (ms.ms_request * (len(arr) + 2))(empty, *arr, empty)
    eng.process_batch(full)
    got = buf.cpu().numpy()
    want = np.concatenate([x.reshape(-1) for x in _expected(w, w.plain, nh)])
    assert np.array_equal(got, want)
    for k in keys:
        eng.key_destroy(k)


def test_graphs_off_equals_graphs_on(ms):
    _note("use_graphs=0")
    import torch
    w = _small(14)
    e1 = ms.Engine(0, use_graphs=0)
    try:
        keys = [e1.key_load(k) for k in w.keys]
        flat = np.concatenate([x.reshape(-1) for x in w.plain])
        src = torch.from_numpy(flat).to("cuda")
        dst = torch.zeros_like(src)
        e1.process_batch(_layout(ms, e1, w, keys, src, dst))
        got = dst.cpu().numpy()
    finally:
        e1.close()
    want = np.concatenate([x.reshape(-1) for x in
                           _expected(w, w.plain, _linear_nonces(w))])
    assert np.array_equal(got, want)


def test_batched_rejects_overlaps_and_oversize(ms, eng):
    _note("batched validation")
    import torch
    key = eng.key_generate()
    buf = torch.zeros(64 * 4096, dtype=torch.uint8, device="cuda")
    lin = ms.linear_nonce(0, 1, 0)
    a = ms.request(key, buf, buf, 8, lin, src_offset_pages=0,
                   dst_offset_pages=16)
    b = ms.request(key, buf, buf, 8, lin, src_offset_pages=32,
                   dst_offset_pages=20)            # dst overlaps a's dst
    arr = (ms.ms_request * 2)(a, b)
    assert ms.ms_process_batch(eng.ctx, arr) == ms.MS_EINVAL
    c = ms.request(key, buf, buf, 8, lin, src_offset_pages=12,
                   dst_offset_pages=40)            # src overlaps a's dst
    arr = (ms.ms_request * 2)(a, c)
    assert ms.ms_process_batch(eng.ctx, arr) == ms.MS_EINVAL
    d = ms.request(key, buf, buf, 8, lin, src_offset_pages=40,
                   dst_offset_pages=40)            # in place: fine
    arr = (ms.ms_request * 2)(a, d)
    assert ms.ms_process_batch(eng.ctx, arr) == ms.MS_OK
    many = (ms.ms_request * 1025)(*([d] * 1025))
    assert ms.ms_process_batch(eng.ctx, many) == ms.MS_EINVAL
    torch.cuda.synchronize()
    eng.key_destroy(key)


def test_autotune_returns_valid_tiling(ms, eng):
    _note("autotune")
    t = eng.autotune(4096)
    assert t.pages_per_wave >= 1 and t.unroll in (1, 2)
    assert t.waves_per_cu >= 1 and t.us_per_launch > 0
    st, t2 = ms.ms_get_tuning(eng.ctx, 4000)
    assert st == 0 and t2.pages_per_wave == t.pages_per_wave


@pytest.mark.parametrize("rounds", [20, 8])
def test_batched_salsa20_per_request(ms, rounds):
    """The fused launch of a Salsa20 context: each request equals the
    Salsa20 oracle run on that request alone."""
    _note("batched salsa20 rounds=%d" % rounds)
    import torch
    e = ms.Engine(0, cipher=ms.MS_CIPHER_SALSA, rounds=rounds)
    try:
        w = _small(13, n_requests=60, max_pages=256)
        nh = _linear_nonces(w)
        keys = [e.key_load(k) for k in w.keys]
        flat = np.concatenate([x.reshape(-1) for x in w.plain])
        src = torch.from_numpy(flat).to("cuda")
        dst = torch.zeros_like(src)
        arr = _layout(ms, e, w, keys, src, dst)
        e.process_batch(arr)
        got = dst.cpu().numpy()
        off = 0
        for i, r in enumerate(w.requests):
            n = r.n_pages * 4096
            want = oracle.cipher_pages(w.keys[r.client], nh[i], w.plain[i],
                                       rounds=rounds, cipher="salsa")
            assert np.array_equal(got[off:off + n], want.reshape(-1)), i
            off += n
        for k in keys:
            e.key_destroy(k)
    finally:
        e.close()


def test_static_batch_at_its_request_limit(ms):
    """ms_process_batch_static with MS_STATIC_BATCH_MAX_REQUESTS one-page
    requests (the largest descriptor array, so the largest descriptor copy)
    equals the oracle page for page; one request more is MS_EINVAL and
    writes nothing."""
    _note("static batch at its limit")
    import torch
    n = ms.MS_STATIC_BATCH_MAX_REQUESTS
    rng = np.random.default_rng(52)
    kb = [rng.bytes(32) for _ in range(3)]
    e = ms.Engine(0)
    try:
        keys = [e.key_load(k) for k in kb]
        host = workloads.random_pages(rng, n + 1)
        src = torch.from_numpy(host.reshape(-1).copy()).to("cuda")
        dst = torch.zeros_like(src)
        kidx = rng.integers(0, 3, size=n + 1)
        va = 0x7F0000000000 + 4096 * rng.integers(0, 1 << 24, size=n + 1)
        reqs = [ms.request(keys[int(kidx[i])], src, dst, 1,
                           ms.linear_nonce(int(va[i]), 4096, 2000 + i),
                           client=int(kidx[i]), src_offset_pages=i,
                           dst_offset_pages=i) for i in range(n + 1)]
        over = (ms.ms_request * (n + 1))(*reqs)
        assert ms.ms_process_batch_static(e.ctx, over) == ms.MS_EINVAL
        torch.cuda.synchronize()
        assert int(dst.count_nonzero()) == 0
        e.process_batch_static((ms.ms_request * n)(*reqs[:n]),
                               stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        got = dst.cpu().numpy().reshape(n + 1, 4096)
        nonces = np.empty((n, 12), np.uint8)
        nonces[:, 0:8] = va[:n].astype("<u8").view(np.uint8).reshape(n, 8)
        nonces[:, 8:12] = (2000 + np.arange(n)).astype("<u4").view(
            np.uint8).reshape(n, 4)
        for k in range(3):
            sel = np.nonzero(kidx[:n] == k)[0]
            want = oracle.cipher_pages(kb[k], nonces[sel], host[sel],
                                       threads=HOST_THREADS)
            assert np.array_equal(got[sel], want), k
        assert not got[n].any()
    finally:
        e.close()


def test_batch_validation_after_a_valid_request(ms, eng):
    """A call remembers the allocations its earlier requests were checked
    against; a later request that runs past the end of the same allocation,
    or names host memory, is still refused (MS_EINVAL) by ms_process_batch
    and by ms_submit, before anything runs."""
    _note("batch validation after a valid request")
    import torch
    key = eng.key_generate()
    n = 16384
    # a fresh 64 MiB allocation that ends where the tensor ends (torch's
    # cache could otherwise hand out the front of a larger one, and the
    # check is against the runtime's allocation, not the tensor)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    buf = torch.zeros(n * 4096, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    p = buf.data_ptr()
    seg = [s for s in torch.cuda.memory_snapshot()
           if s["address"] <= p < s["address"] + s["total_size"]]
    assert len(seg) == 1 and \
        seg[0]["address"] + seg[0]["total_size"] == p + buf.numel(), seg
    lin = ms.linear_nonce(0, 1, 0)
    good = ms.request(key, buf, buf, 8, lin)
    past_src = ms.request(key, buf, buf, 2, lin, src_offset_pages=n - 1,
                          dst_offset_pages=100)
    past_dst = ms.request(key, buf, buf, 2, lin, src_offset_pages=200,
                          dst_offset_pages=n - 1)
    host = np.zeros(3 * 4096 + 16, np.uint8)
    hp = host.ctypes.data + (-host.ctypes.data) % 16
    on_host = ms.ms_request(ms.MS_ENCRYPT, 0, key, hp, hp, 2, lin, 0, 0)
    for bad in (past_src, past_dst, on_host):
        for pair in ((good, bad), (bad, good)):
            arr = (ms.ms_request * 2)(*pair)
            assert ms.ms_process_batch(eng.ctx, arr) == ms.MS_EINVAL
            assert ms.ms_submit(eng.ctx, arr)[0] == ms.MS_EINVAL
    torch.cuda.synchronize()
    assert int(buf.count_nonzero()) == 0
    eng.key_destroy(key)


def test_static_batch_small_calls(ms):
    """ms_process_batch_static with 5 and then 15 requests (the most that
    travel in the kernel arguments) and then 16 (through the device array):
    each call equals the oracle, request by request."""
    import torch
    e = ms.Engine(0)
    try:
        for n in (5, 15, 16):
            _note("static batch of %d requests" % n)
            w = _small(70 + n, n_requests=n, max_pages=5)
            keys = [e.key_load(k) for k in w.keys]
            flat = np.concatenate([x.reshape(-1) for x in w.plain])
            src = torch.from_numpy(flat).to("cuda")
            dst = torch.zeros_like(src)
            e.process_batch_static(_layout(ms, e, w, keys, src, dst),
                                   stream=torch.cuda.current_stream())
            torch.cuda.synchronize()
            want = np.concatenate([x.reshape(-1) for x in
                                   _expected(w, w.plain, _linear_nonces(w))])
            assert np.array_equal(dst.cpu().numpy(), want), n
            for k in keys:
                e.key_destroy(k)
    finally:
        e.close()
