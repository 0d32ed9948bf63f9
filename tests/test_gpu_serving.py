"""GPU tests of the serving path: continuous batching through ms_submit /
ms_poll, admission by device memory, back-pressure, cancellation, prefetch
hints, and the native load generator, on both serving stages (fused
launches formed by the scheduler, and the ring: a resident kernel on the
context's own HSA queue that reads one descriptor per page from mapped
memory).  Every output checked here is compared with the CPU oracle on that
request alone (tolerance 0: the cipher is integer arithmetic)."""
import os
import sys
import threading
import time

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


# serving stages: MS_SERVE_STAGE_LAUNCH (1) and MS_SERVE_STAGE_RING (2)
STAGES = pytest.mark.parametrize("stage", [1, 2], ids=["launch", "ring"])


def _oracle_req(key, va, pid, data):
    n = data.size // 4096
    return oracle.cipher_pages(key, oracle.nonces_linear(n, va, 4096, pid),
                               data.reshape(n, 4096),
                               threads=HOST_THREADS).reshape(-1)


class _Reqs:
    """n requests from several clients over one device input pool, each with
    its own slot in each of two output buffers."""

    def __init__(self, ms, eng, seed, n, max_pages=256, n_clients=8):
        import torch
        rng = np.random.default_rng(seed)
        self.kbytes = [rng.bytes(32) for _ in range(n_clients)]
        self.keys = [eng.key_load(k) for k in self.kbytes]
        self.pages = workloads.log_uniform_pages(rng, max_pages, size=n)
        self.client = rng.integers(0, n_clients, size=n)
        self.va = workloads.VA_BASE + 4096 * rng.integers(0, 1 << 20, size=n)
        self.pid = 1000 + self.client
        self.off = np.concatenate([[0], np.cumsum(self.pages)[:-1]])
        total = int(self.pages.sum())
        self.host = workloads.random_pages(rng, total).reshape(-1)
        self.src = torch.from_numpy(self.host).to("cuda")
        self.dst_a = torch.zeros_like(self.src)
        self.dst_b = torch.zeros_like(self.src)
        # submitted work does not wait for torch's stream
        torch.cuda.synchronize()
        self.ms = ms

    def req(self, i, dst):
        ms = self.ms
        return ms.request(self.keys[self.client[i]], self.src, dst,
                          int(self.pages[i]),
                          ms.linear_nonce(int(self.va[i]), 4096,
                                          int(self.pid[i])),
                          op=int(i % 2), client=int(self.client[i]),
                          src_offset_pages=int(self.off[i]),
                          dst_offset_pages=int(self.off[i]))

    def expect(self, i):
        s = int(self.off[i]) * 4096
        e = s + int(self.pages[i]) * 4096
        return _oracle_req(self.kbytes[self.client[i]], int(self.va[i]),
                           int(self.pid[i]), self.host[s:e])

    def slice(self, t, i):
        s = int(self.off[i]) * 4096
        return t[s:s + int(self.pages[i]) * 4096].cpu().numpy()


@STAGES
def test_alone_equals_mix_equals_oracle(ms, stage):
    """Each request's result is the same submitted alone (one at a time,
    waiting for each) and in the mix (submitted concurrently from 8
    threads, 12 requests per call, batched by the scheduler).  A call's
    requests are queued together, so every launch serves at least one
    call's worth: the batching does not depend on how fast the device
    finishes a request before the next call arrives."""
    _note("alone vs mix, 96 requests, stage %d" % stage)
    eng = ms.Engine(0, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=41, n=96)
        for i in range(96):
            t = eng.submit([r.req(i, r.dst_a)])
            st, done = eng.poll(t, timeout_s=30)
            assert st == 0 and done == [1]
        before = eng.stats()
        tickets = [None] * 96

        def submitter(k):
            mine = list(range(k, 96, 8))
            got = eng.submit([r.req(i, r.dst_b) for i in mine])
            for i, t in zip(mine, got):
                tickets[i] = t

        th = [threading.Thread(target=submitter, args=(k,)) for k in range(8)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        st, done = eng.poll(tickets, timeout_s=60)
        assert st == 0 and all(d == 1 for d in done)
        after = eng.stats()
        if stage == ms.MS_SERVE_STAGE_LAUNCH:
            # the mix was served by fused launches of at least one call each
            assert after.batches - before.batches <= 8
            assert after.max_batch_requests > 1
        for i in range(96):
            a = r.slice(r.dst_a, i)
            b = r.slice(r.dst_b, i)
            assert np.array_equal(a, b), "request %d alone != mix" % i
            assert np.array_equal(a, r.expect(i)), "request %d != oracle" % i
    finally:
        eng.close()


def test_batches_overlap_on_device(ms):
    """Requests that arrive while a large batch runs are launched as their
    own batches on other streams and complete before the large one.  This
    needs the engine's serving streams on distinct hardware queues, which
    the HIP runtime does not promise in a process that already holds many
    streams (it shares its few queues among them); the scenario therefore
    runs in a fresh child process whose first streams are the engine's."""
    _note("overlap (child process)")
    import json
    import subprocess
    child = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                         "serving_overlap_child.py")
    r = subprocess.run([sys.executable, "-u", child], capture_output=True,
                       text=True, timeout=180)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["small_exact"]
    assert out["max_inflight_batches"] >= 2
    assert out["overlapped"] >= 1, out


@STAGES
def test_admission_cap_bounds_inflight_bytes(ms, stage):
    _note("admission cap, stage %d" % stage)
    cap = 64 * 4096
    eng = ms.Engine(0, admission_cap_bytes=cap, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=43, n=60, max_pages=32)
        tickets = eng.submit([r.req(i, r.dst_a) for i in range(60)])
        st, done = eng.poll(tickets, timeout_s=60)
        assert st == 0 and all(d == 1 for d in done)
        s = eng.stats()
        assert 0 < s.max_inflight_bytes <= cap
        for i in (0, 17, 59):
            assert np.array_equal(r.slice(r.dst_a, i), r.expect(i))
        # a single request larger than the cap can never be admitted
        import torch
        big = torch.zeros(65 * 4096, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        bad = ms.request(r.keys[0], big, big, 65, ms.linear_nonce(0, 1, 0))
        st, _ = ms.ms_submit(eng.ctx, [bad])
        assert st == ms.MS_EINVAL
    finally:
        eng.close()


@STAGES
def test_queue_full_is_eagain_and_all_or_nothing(ms, stage):
    _note("eagain, stage %d" % stage)
    eng = ms.Engine(0, queue_depth=4, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=44, n=5, max_pages=4)
        st, _ = ms.ms_submit(eng.ctx, [r.req(i, r.dst_a) for i in range(5)])
        assert st == ms.MS_EAGAIN
        assert eng.stats().submitted == 0
        t = eng.submit([r.req(i, r.dst_a) for i in range(4)])
        st, done = eng.poll(t, timeout_s=30)
        assert st == 0 and done == [1] * 4
    finally:
        eng.close()


@STAGES
def test_cancel_client_keeps_others_exact(ms, stage):
    """Cancelling a client drops its queued requests (their tickets read
    MS_ECANCELED); every other client's results stay bit-exact."""
    _note("cancel client, stage %d" % stage)
    eng = ms.Engine(0, admission_cap_bytes=16 * 4096, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=45, n=120, max_pages=16, n_clients=3)
        tickets = eng.submit([r.req(i, r.dst_a) for i in range(120)])
        st, n_cancel = ms.ms_cancel_client(eng.ctx, 1)
        assert st == 0
        st, done = eng.poll(tickets, timeout_s=60)
        assert st == 0
        cancelled = 0
        for i in range(120):
            if r.client[i] == 1:
                assert done[i] in (1, ms.MS_ECANCELED)
                cancelled += done[i] == ms.MS_ECANCELED
            else:
                assert done[i] == 1
                assert np.array_equal(r.slice(r.dst_a, i), r.expect(i))
        assert cancelled == n_cancel and cancelled > 0
    finally:
        eng.close()


@STAGES
def test_key_destroy_while_queued_is_ebusy(ms, stage):
    _note("destroy busy, stage %d" % stage)
    eng = ms.Engine(0, admission_cap_bytes=4 * 4096, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=46, n=400, max_pages=4, n_clients=1)
        tickets = eng.submit([r.req(i, r.dst_a) for i in range(400)])
        # 400 requests admitted one or two at a time are still queued
        assert ms.ms_key_destroy(eng.ctx, r.keys[0]) == ms.MS_EBUSY
        st, done = eng.poll(tickets, timeout_s=60)
        assert st == 0 and all(d == 1 for d in done)
        eng.drain()
        assert ms.ms_key_destroy(eng.ctx, r.keys[0]) == ms.MS_OK
    finally:
        eng.close()


@STAGES
def test_prefetch_hints_run_or_drop(ms, stage):
    _note("prefetch hints, stage %d" % stage)
    eng = ms.Engine(0, prefetch_depth=4, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=47, n=8, max_pages=8)
        dropped = eng.prefetch_hint([r.req(i, r.dst_a) for i in range(5)])
        assert dropped == [0] * 5         # more than the queue holds
        st, d = eng.poll(dropped)
        assert d == [ms.MS_ECANCELED] * 5
        t = eng.prefetch_hint([r.req(i, r.dst_b) for i in range(4)])
        st, d = eng.poll(t, timeout_s=30)
        assert st == 0
        for i in range(4):
            if d[i] == 1:
                assert np.array_equal(r.slice(r.dst_b, i), r.expect(i))
            else:
                assert d[i] == ms.MS_ECANCELED
        s = eng.stats()
        assert s.prefetch_dropped >= 5
    finally:
        eng.close()


@STAGES
def test_sporadic_request_after_idle_is_reaped_promptly(ms, stage):
    """A request arriving after the scheduler has gone to sleep (spin window
    shortened to 100 us) is launched by the submitting thread; the scheduler
    must wake for it and complete the ticket promptly, not at the end of its
    2 ms sleep.  Median of 7 such requests, each checked against the
    oracle."""
    _note("sporadic request after idle, stage %d" % stage)
    eng = ms.Engine(0, serve_spin_us=100, serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=43, n=7, max_pages=4)
        lat = []
        for i in range(7):
            time.sleep(0.02)   # well past the spin window: the scheduler sleeps
            t0 = time.perf_counter()
            t = eng.submit([r.req(i, r.dst_a)])
            st, done = eng.poll(t, timeout_s=5)
            lat.append(time.perf_counter() - t0)
            assert st == 0 and done == [1]
        lat.sort()
        assert lat[3] < 1e-3, lat
        for i in range(7):
            assert np.array_equal(r.slice(r.dst_a, i), r.expect(i)), i
    finally:
        eng.close()


@pytest.mark.parametrize("mode,stage", [(0, 1), (0, 2), (1, 0), (2, 0)])
def test_loadgen_poisson_sample_exact(ms, mode, stage):
    """Poisson arrivals (20k req/s, 0.5 s) through the native load
    generator (continuous batching on either serving stage, a launch per
    request, the resident-key ring with all 64 client keys); every 25th
    request's output is checked against the oracle."""
    _note("loadgen mode=%d stage=%d" % (mode, stage))
    import torch
    from paper_2004_09252_amd import serving
    pool_pages = 16384
    w = workloads.serving(seed=4, rate_hz=20000, duration_s=0.5,
                          pool_pages=pool_pages)
    eng = ms.Engine(0, serve_stage=stage)
    try:
        keys = [eng.key_load(k) for k in w.keys]
        src = torch.empty(pool_pages * 4096, dtype=torch.uint8, device="cuda")
        serving.fill_pool(src, seed=4)
        lay = serving.layout(w, ring_pages=8192, sample_every=25)
        dst = torch.zeros(lay.dst_pages * 4096, dtype=torch.uint8,
                          device="cuda")
        res, lat = serving.run(eng, lay, keys, src, dst, mode)
        assert res.completed == lay.trace.n
        assert res.failed == 0, "%d failed, first: request %d state %d" % (
            res.failed, res.first_failed - 1, res.first_failed_state)
        assert res.p50_us > 0 and res.p99_us >= res.p50_us
        assert np.all(lat > 0)
        a = lay.arrays
        for i, inp, out in serving.sampled_outputs(lay, src, dst):
            c = int(a["client"][i])
            want = _oracle_req(w.keys[c], int(a["va"][i]), int(a["pid"][i]),
                               inp)
            assert np.array_equal(out, want), "request %d" % i
        if mode == 0:
            s = eng.stats()
            assert s.batches <= s.submitted
    finally:
        eng.close()


@pytest.mark.parametrize("tiling", [None, (8, 1, 28), (1, 1, 1), (8, 2, 28),
                                    (64, 2, 2)])
def test_large_submitted_request_every_tiling(ms, tiling):
    """One request of 65536 pages (256 MiB) through ms_submit, under the
    default and forced tilings with one and several chunks per wave."""
    _note("large submit tiling=%s" % (tiling,))
    import torch
    eng = ms.Engine(0)
    try:
        kb = bytes(range(32))
        key = eng.key_load(kb)
        n = 65536
        g = torch.Generator("cuda").manual_seed(7)
        src = torch.randint(0, 256, (n * 4096,), dtype=torch.uint8,
                            device="cuda", generator=g)
        dst = torch.zeros_like(src)
        torch.cuda.synchronize()   # submitted work does not wait for torch
        if tiling:
            assert ms.ms_set_tuning(eng.ctx, ms.ms_tuning(*tiling, 0,
                                                          0.0)) == 0
        t = eng.submit([ms.request(key, src, dst, n,
                                   ms.linear_nonce(7, 4096, 99))])
        st, d = eng.poll(t, timeout_s=60)
        assert st == 0 and d == [1]
        got = dst.cpu().numpy().reshape(n, 4096)
        want = _oracle_req(kb, 7, 99, src.cpu().numpy()).reshape(n, 4096)
        bad = np.where(~np.all(got == want, axis=1))[0]
        assert bad.size == 0, "%d bad pages, first %s" % (bad.size, bad[:5])
    finally:
        ms.ms_set_tuning(eng.ctx, None)
        eng.close()


def test_ring_requests_overlap_a_running_launch(ms):
    """On the ring stage, small requests submitted while a large request
    (above the ring's page limit, so a fused launch, here on a narrow grid)
    runs are served by the resident kernel on its own HSA queue and finish
    before it: overlap on the device does not depend on the process's
    streams.  Their outputs equal the oracle."""
    _note("ring overlap with a running launch")
    import torch
    eng = ms.Engine(0, serve_stage=ms.MS_SERVE_STAGE_RING)
    try:
        rng = np.random.default_rng(48)
        kb = [rng.bytes(32) for _ in range(2)]
        keys = [eng.key_load(k) for k in kb]
        small = workloads.random_pages(rng, 12)
        src = torch.from_numpy(small.reshape(-1).copy()).to("cuda")
        dst = torch.zeros_like(src)
        big_pages = 65536
        big = torch.zeros(big_pages * 4096, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()

        def small_req(i):
            return ms.request(keys[1], src, dst, 2,
                              ms.linear_nonce(4096 * i, 1, 7),
                              src_offset_pages=2 * i, dst_offset_pages=2 * i)

        t = eng.submit([small_req(0)])   # the ring is up
        assert eng.poll(t, timeout_s=30)[0] == 0
        assert ms.ms_set_tuning(eng.ctx, ms.ms_tuning(64, 1, 2, 0, 0.0)) == 0
        tb = eng.submit([ms.request(keys[0], big, big, big_pages,
                                    ms.linear_nonce(0, 1, 0))])
        overlapped = 0
        for i in range(6):
            ts = eng.submit([small_req(i)])
            st, d = eng.poll(ts, timeout_s=30)
            assert st == 0 and d == [1]
            overlapped += eng.poll(tb, timeout_s=0)[1] == [0]
        assert eng.poll(tb, timeout_s=60)[0] == 0
        assert overlapped >= 3, overlapped
        got = dst.cpu().numpy().reshape(12, 4096)
        for i in range(6):
            want = oracle.cipher_pages(kb[1], oracle.nonces_linear(
                2, 4096 * i, 1, 7), small[2 * i:2 * i + 2])
            assert np.array_equal(got[2 * i:2 * i + 2], want), i
    finally:
        ms.ms_set_tuning(eng.ctx, None)
        eng.close()


def test_ring_stage_serves_clients_round_robin(ms):
    """On the ring stage, requests that wait for ring positions queue per
    client and are published round robin.  Client A submits a burst of 160
    requests of 1024 pages (163,840 pages against a ring of 65,536
    positions, so most of the burst waits); client B then submits 8
    one-page requests.  B's requests take turns with A's, so all of them
    finish while a quarter or more of A's burst is still pending (in one
    FIFO they would finish after all of it).  Every output equals the
    oracle (a sample of A's, all of B's)."""
    _note("ring stage round robin: burst of 160 x 1024 pages + 8 x 1 page")
    import torch
    eng = ms.Engine(0, serve_stage=ms.MS_SERVE_STAGE_RING)
    try:
        rng = np.random.default_rng(49)
        kb = [rng.bytes(32) for _ in range(2)]
        keys = [eng.key_load(k) for k in kb]
        na, pa, nb = 160, 1024, 8
        a_src = torch.randint(0, 256, (na * pa * 4096,), dtype=torch.uint8,
                              device="cuda")
        a_dst = torch.zeros_like(a_src)
        b_host = workloads.random_pages(rng, nb)
        b_src = torch.from_numpy(b_host.reshape(-1).copy()).to("cuda")
        b_dst = torch.zeros_like(b_src)
        torch.cuda.synchronize()
        t0 = eng.submit([ms.request(keys[1], b_src, b_dst, 1,
                                    ms.linear_nonce(0, 1, 9))])
        assert eng.poll(t0, timeout_s=30)[0] == 0   # the ring is up
        ta = eng.submit([ms.request(keys[0], a_src, a_dst, pa,
                                    ms.linear_nonce(pa * i, 1, 1), client=0,
                                    src_offset_pages=pa * i,
                                    dst_offset_pages=pa * i)
                         for i in range(na)])
        tb = eng.submit([ms.request(keys[1], b_src, b_dst, 1,
                                    ms.linear_nonce(i, 1, 2), client=1,
                                    src_offset_pages=i, dst_offset_pages=i)
                         for i in range(nb)])
        tickets = list(ta) + list(tb)
        stats = eng.stats()
        # the first ring's worth of the burst went straight onto the ring,
        # the rest of it and all of B's requests waited in client queues
        assert stats.ring_direct >= 60, stats.ring_direct
        assert stats.ring_queued >= na - 64 + nb, stats.ring_queued
        assert stats.ring_max_queued >= na - 64, stats.ring_max_queued
        seen = [None] * len(tickets)
        it = 0
        deadline = time.time() + 60
        while any(x is None for x in seen):
            assert time.time() < deadline, "requests did not finish"
            st, d = ms.ms_poll(eng.ctx, tickets, 0)
            assert st in (0, ms.MS_ETIMEDOUT)
            for k, v in enumerate(d):
                assert v >= 0, (k, v)
                if v == 1 and seen[k] is None:
                    seen[k] = it
            it += 1
        assert eng.poll(tickets, timeout_s=10)[0] == 0
        b_last = max(seen[na:])
        a_done = sum(1 for x in seen[:na] if x <= b_last)
        assert a_done <= 3 * na // 4, (a_done, b_last, it)
        got = b_dst.cpu().numpy().reshape(nb, 4096)
        for i in range(nb):
            want = oracle.cipher_pages(kb[1], oracle.nonces_linear(
                1, i, 1, 2), b_host[i:i + 1])
            assert np.array_equal(got[i:i + 1], want), i
        for i in (0, 1, na // 2, na - 1):
            s0 = pa * i * 4096
            src_h = a_src[s0:s0 + pa * 4096].cpu().numpy().reshape(pa, 4096)
            want = oracle.cipher_pages(kb[0], oracle.nonces_linear(
                pa, pa * i, 1, 1), src_h, threads=HOST_THREADS)
            got_a = a_dst[s0:s0 + pa * 4096].cpu().numpy().reshape(pa, 4096)
            assert np.array_equal(got_a, want), i
    finally:
        eng.close()


def test_plain_launches_leave_room_for_the_ring(ms):
    """Once a context's serving ring runs (one wave on every SIMD), plain
    launches size their grid to the wave slots left: ms_plain_launch_info
    reports 4 fewer waves per compute unit, a 1 GiB pass takes at most 1.35x
    its time on an idle device (a grid sized for an idle device would leave
    an eighth of its workgroups to start after the rest, about 2x), and its
    output equals the oracle on sampled pages."""
    _note("plain launch beside the serving ring")
    import torch
    eng = ms.Engine(0, serve_stage=ms.MS_SERVE_STAGE_RING)
    try:
        rng = np.random.default_rng(51)
        kb = rng.bytes(32)
        key = eng.key_load(kb)
        n = 262144
        src = torch.randint(0, 256, (n * 4096,), dtype=torch.uint8,
                            device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        nonce = ms.linear_nonce(0, 1, 0)
        s = torch.cuda.Stream()

        def best():
            ts = []
            for _ in range(10):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                eng.encrypt_pages(key, src, dst, nonce, stream=s)
                e1.record(s)
                s.synchronize()
                ts.append(e0.elapsed_time(e1))
            return min(ts[3:])

        st, idle = ms.ms_plain_launch_info(eng.ctx, n, ms.MS_NONCE_LINEAR)
        assert st == 0
        t_idle = best()
        one = torch.zeros(4096, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t = eng.submit([ms.request(key, one, one, 1, nonce)])
        assert eng.poll(t, timeout_s=30)[0] == 0   # the ring is up
        st, busy = ms.ms_plain_launch_info(eng.ctx, n, ms.MS_NONCE_LINEAR)
        assert st == 0 and busy.waves_per_cu == idle.waves_per_cu - 4
        assert busy.grid_blocks == idle.grid_blocks - eng_cus(ms, eng)
        t_ring = best()
        assert t_ring < 1.35 * t_idle, (t_ring, t_idle)
        for p in (0, 1, n // 3, n - 1):
            got = dst[p * 4096:(p + 1) * 4096].cpu().numpy().reshape(1, 4096)
            inp = src[p * 4096:(p + 1) * 4096].cpu().numpy().reshape(1, 4096)
            want = oracle.cipher_pages(kb, oracle.nonces_linear(1, p, 1, 0),
                                       inp)
            assert np.array_equal(got, want), p
    finally:
        eng.close()


def eng_cus(ms, eng):
    return ms.ms_device_cu_count(eng.ctx)


@STAGES
@pytest.mark.parametrize("rounds", [20, 8])
def test_salsa20_context_serves_on_both_stages(ms, stage, rounds):
    """A Salsa20 context's submissions run on either serving stage (the
    ring's resident kernel runs the context's cipher and rounds) and equal
    the Salsa20 oracle request by request."""
    _note("salsa20/%d served, stage %d" % (rounds, stage))
    eng = ms.Engine(0, cipher=ms.MS_CIPHER_SALSA, rounds=rounds,
                    serve_stage=stage)
    try:
        r = _Reqs(ms, eng, seed=49, n=20, max_pages=16)
        t = eng.submit([r.req(i, r.dst_a) for i in range(20)])
        st, done = eng.poll(t, timeout_s=30)
        assert st == 0 and all(d == 1 for d in done)
        for i in range(20):
            s0 = int(r.off[i]) * 4096
            e0 = s0 + int(r.pages[i]) * 4096
            n = int(r.pages[i])
            want = oracle.cipher_pages(
                r.kbytes[r.client[i]],
                oracle.nonces_linear(n, int(r.va[i]), 4096, int(r.pid[i])),
                r.host[s0:e0].reshape(n, 4096), rounds=rounds,
                cipher="salsa").reshape(-1)
            assert np.array_equal(r.slice(r.dst_a, i), want), i
    finally:
        eng.close()


@STAGES
def test_engine_holds_tensors_of_requests_in_flight(ms, stage):
    """A request's tensors stay alive while it is in flight even when the
    caller drops them, and are released once poll reports it finished."""
    _note("tensors held while in flight, stage %d" % stage)
    import gc
    import weakref

    import torch
    eng = ms.Engine(0, serve_stage=stage)
    try:
        key = eng.key_generate()
        src = torch.randint(0, 256, (256 * 4096,), dtype=torch.uint8,
                            device="cuda")
        dst = torch.zeros_like(src)
        arr = torch.zeros(256 * 12, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        refs = [weakref.ref(t) for t in (src, dst, arr)]
        t = eng.submit([ms.request(key, src, dst, 256, ms.array_nonce(arr))])
        del src, dst, arr
        gc.collect()
        assert all(w() is not None for w in refs)
        st, done = eng.poll(t, timeout_s=30)
        assert st == 0 and done == [1]
        gc.collect()
        assert all(w() is None for w in refs)
    finally:
        eng.close()


def test_ring_stage_size_boundary(ms):
    """On the ring stage, requests of 1, 1023 and 1024 pages (the ring's
    limit) go to the ring and one of 1025 pages to a fused launch; all of
    them, submitted in one call, equal the oracle page for page, and the
    context's counters place each where its size says."""
    _note("ring stage size boundary: 1, 1023, 1024, 1025 pages")
    import torch
    eng = ms.Engine(0, serve_stage=ms.MS_SERVE_STAGE_RING)
    try:
        r = _Reqs(ms, eng, seed=50, n=4, max_pages=2)
        r.pages[:] = [1, 1023, 1024, 1025]
        r.off = np.concatenate([[0], np.cumsum(r.pages)[:-1]])
        rng = np.random.default_rng(51)
        total = int(r.pages.sum())
        r.host = workloads.random_pages(rng, total).reshape(-1)
        r.src = torch.from_numpy(r.host).to("cuda")
        r.dst_a = torch.zeros_like(r.src)
        torch.cuda.synchronize()
        t0 = eng.submit([r.req(0, r.dst_a)])       # the ring is up
        assert eng.poll(t0, timeout_s=30)[0] == 0
        before = eng.stats()
        t = eng.submit([r.req(i, r.dst_a) for i in range(4)])
        st, done = eng.poll(t, timeout_s=60)
        assert st == 0 and done == [1, 1, 1, 1]
        after = eng.stats()
        on_ring = ((after.ring_direct - before.ring_direct) +
                   (after.ring_queued - before.ring_queued))
        assert on_ring == 3, on_ring
        assert after.batches - before.batches == 1
        for i in range(4):
            assert np.array_equal(r.slice(r.dst_a, i), r.expect(i)), i
    finally:
        eng.close()


@pytest.mark.parametrize("n", [2, 15, 16, 40])
def test_launch_stage_one_batch_per_submission(ms, n):
    """On the launch stage, one submission of n requests with nothing in
    flight becomes one fused launch: up to 15 requests with their records
    in the kernel arguments, more through the descriptor copy.  Every
    request equals the oracle, and each submission counts one batch."""
    _note("launch stage, one batch of %d requests" % n)
    eng = ms.Engine(0, serve_stage=ms.MS_SERVE_STAGE_LAUNCH)
    try:
        r = _Reqs(ms, eng, seed=60 + n, n=n, max_pages=6)
        for rep, dst in enumerate((r.dst_a, r.dst_b)):
            eng.drain(timeout_s=30)
            before = eng.stats()
            t = eng.submit([r.req(i, dst) for i in range(n)])
            st, done = eng.poll(t, timeout_s=30)
            assert st == 0 and done == [1] * n
            after = eng.stats()
            assert after.batches - before.batches == 1, rep
            for i in range(n):
                assert np.array_equal(r.slice(dst, i), r.expect(i)), (rep, i)
    finally:
        eng.close()
