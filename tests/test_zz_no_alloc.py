"""The allocation-free fused batch (ms_process_batch_static) against the
allocating one (ms_process_batch), through the C ABI, bit-exact.

Two calls in a row on one stream, the second with fewer requests than the
first (so the device array still holds the first call's later records), then
both checked against ms_process_batch on the same requests and, on a sample
of requests, against the CPU oracle (each page depends only on its key,
nonce and bytes: paper section 4.4).  Pages of requests the second call does
not name must stay untouched.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ms():
    from paper_2004_09252_amd import memshield
    return memshield


def _requests(ms, rng, keys, n, src, dst, nonce_dev):
    """n requests back to back: 1..64 pages log-uniform, keys and ops mixed,
    every 3rd with an array of nonces, every 5th in place."""
    out, meta, off = [], [], 0
    for i in range(n):
        pages = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(65)))),
                            1, 64))
        k = int(rng.integers(0, len(keys)))
        in_place = i % 5 == 0
        if i % 3 == 0:
            nonce = ms.array_nonce(nonce_dev[off * 12:(off + pages) * 12])
            kind = ("array", off)
        else:
            va = 0x7F0000000000 + 4096 * int(rng.integers(0, 1 << 24))
            nonce = ms.linear_nonce(va, 4096, 1000 + k)
            kind = ("linear", va, 1000 + k)
        out.append(ms.request(keys[k], src, src if in_place else dst, pages,
                              nonce, op=i % 2, client=k,
                              src_offset_pages=off, dst_offset_pages=off))
        meta.append((off, pages, k, in_place, kind))
        off += pages
    return out, meta, off


def test_static_batch_matches_process_batch(ms):
    import torch
    # the allocating entry point takes up to max_batch_requests requests
    eng = ms.Engine(0, max_batch_requests=ms.MS_STATIC_BATCH_MAX_REQUESTS)
    try:
        rng = np.random.default_rng(77)
        key_bytes = [rng.bytes(32) for _ in range(8)]
        keys = [eng.key_load(k) for k in key_bytes]
        cap = 1200 * 64
        gen = torch.Generator(device="cuda").manual_seed(77)
        data = torch.randint(0, 256, (cap * 4096,), dtype=torch.uint8,
                             device="cuda", generator=gen)
        nonce_host = np.frombuffer(rng.bytes(cap * 12), np.uint8)
        nonce_dev = torch.from_numpy(nonce_host.copy()).to("cuda")

        def run(fn, reqs_of, sizes):
            """Call fn once per size back to back on the current stream, each
            call on fresh copies of the inputs; returns the source and
            destination buffers of each call after one synchronize."""
            outs = []
            for n in sizes:
                src = data.clone()
                dst = torch.full_like(data, 0xA5)
                reqs, meta, _ = reqs_of(n, src, dst)
                fn(reqs)
                outs.append((src, dst, meta))
            torch.cuda.synchronize()
            return outs

        plan = np.random.default_rng(78)
        seeds = {}

        def reqs_of(n, src, dst):
            # the same requests for the same n on every path
            r = np.random.default_rng(seeds.setdefault(n, int(
                plan.integers(1 << 30))))
            return _requests(ms, r, keys, n, src, dst, nonce_dev)

        sizes = [1100, 37]
        _note("static batch: %s requests, two calls in a row" % sizes)
        got = run(eng.process_batch_static, reqs_of, sizes)
        _note("process_batch on the same requests")
        want = run(eng.process_batch, reqs_of, sizes)
        for (gs, gd, meta), (ws, wd, _) in zip(got, want):
            assert torch.equal(gs, ws), "in-place pages differ (%d requests)" \
                % len(meta)
            assert torch.equal(gd, wd), "out-of-place pages differ (%d " \
                "requests)" % len(meta)
        # the second (smaller) call touched only its own requests' pages
        gs, gd, meta = got[1]
        end = meta[-1][0] + meta[-1][1]
        assert bool((gd[end * 4096:] == 0xA5).all())
        assert torch.equal(gs[end * 4096:], data[end * 4096:])
        # a sample of requests against the oracle
        host_in = None
        for call, (gs, gd, meta) in enumerate(got):
            for i in range(0, len(meta), 23 if call == 0 else 5):
                off, pages, k, in_place, kind = meta[i]
                lo, hi = off * 4096, (off + pages) * 4096
                if host_in is None:
                    host_in = data.cpu().numpy()
                if kind[0] == "array":
                    nn = nonce_host[kind[1] * 12:(kind[1] + pages) * 12]
                else:
                    nn = oracle.nonces_linear(pages, kind[1], 4096, kind[2])
                exp = oracle.cipher_pages(key_bytes[k], nn, host_in[lo:hi])
                out = (gs if in_place else gd)[lo:hi].cpu().numpy()
                assert np.array_equal(out.reshape(exp.shape), exp), \
                    "call %d request %d differs from the oracle" % (call, i)
        # sizes beyond the array are refused; an empty call is a no-op
        src = data.clone()
        one = ms.request(keys[0], src, src, 1, ms.linear_nonce(0, 1, 0))
        too_many = (ms.ms_request * (ms.MS_STATIC_BATCH_MAX_REQUESTS + 1))(
            *([one] * (ms.MS_STATIC_BATCH_MAX_REQUESTS + 1)))
        assert ms.ms_process_batch_static(eng.ctx, too_many) == ms.MS_EINVAL
        assert ms.ms_process_batch_static(eng.ctx, []) == 0
        for k in keys:
            eng.key_destroy(k)
    finally:
        eng.close()
