"""The decrypt-on-fault simulation with its page data on the GPU, with and
without the learned predictor: counters equal the reference model's, and
the ciphertext store at the end is bit-exact against the oracle (every
touched page = ChaCha20 of its final plaintext under its client's key and
the page's (virtual address, PID) nonce)."""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import window_sim
from paper_2004_09252_amd import workloads

pytestmark = pytest.mark.gpu

HOST_THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _note(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _keys(tr, seed):
    rng = np.random.default_rng(seed)
    return [rng.bytes(32) for _ in range(tr.clients)]


def _check_store(mem, tr, key_bytes, stop):
    n = tr.pages_per_client
    store = mem.store.cpu().numpy().reshape(tr.clients, n, 4096)
    for c in range(tr.clients):
        plain = window_sim.final_plaintext(n, tr.page[c, :stop],
                                           tr.word[c, :stop],
                                           tr.value[c, :stop])
        touched = np.zeros(n, bool)
        touched[np.unique(tr.page[c, :stop])] = True
        nonces = oracle.nonces_linear(n, workloads.VA_BASE, 4096, 1000 + c)
        want = oracle.cipher_pages(key_bytes[c], nonces, plain,
                                   threads=HOST_THREADS)
        assert np.array_equal(store[c][touched], want[touched]), \
            "client %d ciphertext store" % c
        assert not store[c][~touched].any()


def _oracle_counts(tr, window, start, stop, decisions=None, slots=0,
                   bg_threshold=0):
    tot = {}
    for c in range(tr.clients):
        pf = None
        if decisions is not None:
            pf = {t: q for (cc, t), q in decisions.items() if cc == c}
        o, _ = window_sim.simulate(tr.page[c, :stop], window, prefetch=pf,
                                   prefetch_slots=slots, start=start,
                                   writes=tr.value[c, :stop] != 0,
                                   bg_threshold=bg_threshold)
        for k, v in o.items():
            tot[k] = tot.get(k, 0) + v
    return tot


def test_baseline_store_bit_exact():
    _note("prefetch baseline")
    from paper_2004_09252_amd import memshield as ms
    from paper_2004_09252_amd import prefetch
    tr = workloads.access_trace(seed=21, total_pages=16 * 256,
                                accesses=16 * 1500, clients=16)
    kb = _keys(tr, 21)
    eng = ms.Engine(0)
    try:
        keys = [eng.key_load(k) for k in kb]
        mem = prefetch.PagedMemory(eng, keys, tr.pages_per_client, slots=40)
        cnt, _, _, cl = prefetch.run(tr, 6, mem=mem)
        prefetch.finish(mem, cl)
        ref = _oracle_counts(tr, 6, 0, tr.steps)
        for k, v in ref.items():
            assert cnt[k] == v, k
        assert mem.launches < cnt["decrypts"] + cnt["encrypts"]
        _check_store(mem, tr, kb, tr.steps)
    finally:
        eng.close()


def test_predictor_run_counts_and_store_bit_exact():
    """Train briefly on the fault events of the first 60% and prefetch in
    the rest; the oracle replays the same prefetch decisions."""
    _note("prefetch with predictor")
    from paper_2004_09252_amd import memshield as ms
    from paper_2004_09252_amd import prefetch
    from paper_2004_09252_amd.predictor import Predictor
    tr = workloads.access_trace(seed=22, total_pages=16 * 256,
                                accesses=16 * 3000, clients=16)
    kb = _keys(tr, 22)
    W, P = 6, 8
    split = int(tr.steps * 0.6)
    _, events, _, _ = prefetch.run(tr, W, stop=split, record_events=True)
    vocab = prefetch.DeltaVocab([d for ev in events for d in np.diff(ev)])
    xs, ys = prefetch.training_examples(events, vocab, 16)
    pred = Predictor(max_batch=1024)
    prefetch.train(pred, xs, ys, steps=150, batch=512, lr=2e-3)
    eng = ms.Engine(0)
    try:
        keys = [eng.key_load(k) for k in kb]
        mem = prefetch.PagedMemory(eng, keys, tr.pages_per_client,
                                   slots=W + P + 24)
        cnt, _, dec, cl = prefetch.run(tr, W, mem=mem, prefetch_slots=P,
                                       predictor=pred, vocab=vocab, k=8,
                                       predict_from=split, count_from=split)
        prefetch.finish(mem, cl)
        ref = _oracle_counts(tr, W, split, tr.steps, decisions=dec, slots=P)
        for k, v in ref.items():
            assert cnt[k] == v, k
        assert cnt["prefetch_issued"] > 0 and cnt["prefetch_hits"] > 0
        _check_store(mem, tr, kb, tr.steps)
    finally:
        eng.close()


@pytest.mark.parametrize("threshold", [1, 3])
def test_background_pre_encryption_store_bit_exact(threshold):
    """Background pre-encryption on GPU-resident page data: the counters
    equal the oracle's, evictions of clean pages skip the fault-path
    encryption, and the final ciphertext store is the oracle's, bit for
    bit (a background encryption followed by a write is redone at
    eviction)."""
    _note("background pre-encryption threshold=%d" % threshold)
    from paper_2004_09252_amd import memshield as ms
    from paper_2004_09252_amd import prefetch
    tr = workloads.access_trace(seed=23, total_pages=16 * 256,
                                accesses=16 * 1500, clients=16)
    kb = _keys(tr, 23)
    eng = ms.Engine(0)
    try:
        keys = [eng.key_load(k) for k in kb]
        mem = prefetch.PagedMemory(eng, keys, tr.pages_per_client, slots=40)
        cnt, _, _, cl = prefetch.run(tr, 6, mem=mem, bg_threshold=threshold)
        prefetch.finish(mem, cl)
        ref = _oracle_counts(tr, 6, 0, tr.steps, bg_threshold=threshold)
        for k, v in ref.items():
            assert cnt[k] == v, k
        assert cnt["evict_clean"] > 0 and cnt["encrypts_bg"] > 0
        _check_store(mem, tr, kb, tr.steps)
    finally:
        eng.close()


def _trained(tr, W, split, steps=300, seed=24):
    from paper_2004_09252_amd import prefetch
    from paper_2004_09252_amd.predictor import Predictor
    _, events, _, _ = prefetch.run(tr, W, stop=split, record_events=True)
    vocab = prefetch.DeltaVocab([d for ev in events for d in np.diff(ev)])
    xs, ys = prefetch.training_examples(events, vocab, 16)
    pred = Predictor(max_batch=1024, seed=seed)
    prefetch.train(pred, xs, ys, steps=steps, batch=512, lr=2e-3, seed=seed)
    return pred, vocab


def test_predictor_gain_at_equal_budget_with_hints():
    """What the trained network gains over decrypt-on-fault alone (sections
    4.2-4.3), at an equal clear-page budget: a window of W + P pages against
    a window of W pages plus P pre-decrypted pages, the pre-decryptions sent
    as prefetch hints (ms_prefetch_hint) with the predictor's default
    confidence gate.  The gated predictor must remove at least a quarter of
    the decrypt faults, its total decrypt work must stay within 1.5 times
    the baseline's, and both ciphertext stores must be the oracle's."""
    _note("predictor gain at equal budget, hints")
    from paper_2004_09252_amd import memshield as ms
    from paper_2004_09252_amd import prefetch
    tr = workloads.access_trace(seed=24, total_pages=16 * 1024,
                                accesses=16 * 8000, clients=16)
    kb = _keys(tr, 24)
    W, P = 6, 8
    split = int(tr.steps * 0.8)
    pred, vocab = _trained(tr, W, split)
    assert pred.min_prob == pred.DEFAULT_MIN_PROB == 0.1
    eng = ms.Engine(0)
    try:
        keys = [eng.key_load(k) for k in kb]
        base_mem = prefetch.PagedMemory(eng, keys, tr.pages_per_client,
                                        slots=W + P + 24)
        base, _, _, cl = prefetch.run(tr, W + P, mem=base_mem,
                                      count_from=split)
        prefetch.finish(base_mem, cl)
        ref = _oracle_counts(tr, W + P, split, tr.steps)
        for k, v in ref.items():
            assert base[k] == v, k
        _check_store(base_mem, tr, kb, tr.steps)
        del base_mem
        mem = prefetch.PagedMemory(eng, keys, tr.pages_per_client,
                                   slots=W + P + 24)
        got, _, dec, cl = prefetch.run(tr, W, mem=mem, prefetch_slots=P,
                                       predictor=pred, vocab=vocab, k=8,
                                       predict_from=split, count_from=split,
                                       hints=True)
        prefetch.finish(mem, cl)
        ref = _oracle_counts(tr, W, split, tr.steps, decisions=dec, slots=P)
        for k, v in ref.items():
            assert got[k] == v, k
        assert got["prefetch_dropped"] == 0
        assert mem.hints_issued == got["prefetch_issued"] > 0
        _check_store(mem, tr, kb, tr.steps)
        print("baseline faults %d decrypts %d; predictor faults %d "
              "decrypts %d hits %d issued %d" % (
                  base["faults"], base["decrypts"], got["faults"],
                  got["decrypts"], got["prefetch_hits"],
                  got["prefetch_issued"]), flush=True)
        assert got["faults"] <= 0.75 * base["faults"]
        assert got["decrypts"] <= 1.5 * base["decrypts"]
    finally:
        eng.close()


def test_hints_and_fused_prefetch_store_the_same():
    """Pre-decryptions as prefetch hints on the engine's streams or inside
    the fused demand launches: the same decisions, the same counters as the
    oracle's replay, and bit-exact ciphertext stores."""
    _note("hints vs fused pre-decryption")
    from paper_2004_09252_amd import memshield as ms
    from paper_2004_09252_amd import prefetch
    tr = workloads.access_trace(seed=25, total_pages=16 * 256,
                                accesses=16 * 3000, clients=16)
    kb = _keys(tr, 25)
    W, P = 6, 8
    split = int(tr.steps * 0.6)
    pred, vocab = _trained(tr, W, split, steps=150, seed=25)
    eng = ms.Engine(0)
    try:
        keys = [eng.key_load(k) for k in kb]
        out = []
        for hints in (False, True):
            mem = prefetch.PagedMemory(eng, keys, tr.pages_per_client,
                                       slots=W + P + 24)
            cnt, _, dec, cl = prefetch.run(
                tr, W, mem=mem, prefetch_slots=P, predictor=pred,
                vocab=vocab, k=8, predict_from=split, count_from=split,
                min_prob=0.0, hints=hints)
            prefetch.finish(mem, cl)
            ref = _oracle_counts(tr, W, split, tr.steps, decisions=dec,
                                 slots=P)
            for k, v in ref.items():
                assert cnt[k] == v, (hints, k)
            _check_store(mem, tr, kb, tr.steps)
            out.append((cnt, dec))
            del mem
        assert out[0][1] == out[1][1]
        assert out[0][0] == out[1][0]
    finally:
        eng.close()
