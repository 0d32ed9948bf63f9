"""Pins of the sliding-window model (oracle/window_sim.py) against hand-
worked cases of the paper's policy (sections 4.2 and 4.3): FIFO eviction of
the oldest clear page, first touch served with zeros and no decrypt, a fault
on a known page decrypted; and of the prefetch accounting readings."""
import numpy as np

from oracle import window_sim
from paper_2004_09252_amd import prefetch, workloads


def test_fifo_window_hand_case():
    # window 2: 0 1 2 (evict 0) 0 (fault, evict 1) 2 (hit) 1 (fault, evict 2)
    cnt, log = window_sim.simulate([0, 1, 2, 0, 2, 1], window=2)
    assert cnt["first_touch"] == 3
    assert cnt["faults"] == 2 and [p for _, p in log] == [0, 1]
    assert cnt["encrypts"] == 3   # 0 at t=2, 1 at t=3, 2 at t=5
    assert cnt["decrypts"] == 2


def test_fifo_not_lru():
    # FIFO evicts the oldest admitted page even if it was just used
    cnt, log = window_sim.simulate([0, 1, 0, 2, 0], window=2)
    # admit 0, 1; hit 0; admit 2 evicts 0 (oldest); access 0 faults
    assert cnt["faults"] == 1 and log == [(4, 0)]


def test_scan_larger_than_window_always_faults():
    pages = list(range(10)) * 3
    cnt, _ = window_sim.simulate(pages, window=4)
    assert cnt["first_touch"] == 10 and cnt["faults"] == 20


def test_prefetch_hit_and_waste_accounting():
    pages = [0, 1, 2, 3, 0, 1]
    # after access 3 (page 3), prefetch pages 0 and 2 with one slot
    cnt, _ = window_sim.simulate(pages, window=2, prefetch={3: [0, 2]},
                                 prefetch_slots=1)
    # 2 is still in the window? window after t=3 holds {2, 3}: 2 ignored
    assert cnt["prefetch_issued"] == 1 and cnt["prefetch_hits"] == 1
    assert cnt["faults"] == 1          # page 1 at t=5
    assert cnt["prefetch_wasted"] == 0


def test_untouched_pages_are_never_prefetched():
    cnt, _ = window_sim.simulate([0, 1, 2], window=1, prefetch={0: [5]},
                                 prefetch_slots=4)
    assert cnt["prefetch_issued"] == 0


def test_final_plaintext_xor_of_writes():
    pages = [3, 3, 1]
    words = [0, 0, 511]
    vals = [0x0102030405060708, 0x0102030405060708 ^ 0xFF, 7]
    mem = window_sim.final_plaintext(4, pages, words, vals)
    assert mem[3, 0] == 0xFF and mem[3, 1:8].sum() == 0
    assert mem[1, 511 * 8] == 7 and mem[0].sum() == 0


def test_product_host_logic_matches_oracle_counts():
    tr = workloads.access_trace(seed=9, accesses=16 * 2000, clients=16,
                                total_pages=16 * 256)
    cnt, events, _, _ = prefetch.run(tr, 6, record_events=True,
                                     count_from=500)
    tot = {}
    for c in range(tr.clients):
        o, log = window_sim.simulate(tr.page[c], 6, start=500)
        for k, v in o.items():
            tot[k] = tot.get(k, 0) + v
    for k, v in tot.items():
        assert cnt[k] == v, k
    # fault events = window misses: faults + first touches (no prefetching)
    assert cnt["events"] == cnt["faults"] + cnt["first_touch"]


def test_delta_vocab_and_examples():
    vocab = prefetch.DeltaVocab([1, 1, 1, 2, 2, -5], size=4)
    assert vocab.n_known == 3 and vocab.oov == 3
    assert vocab.ids([1, 2, -5, 99]).tolist() == [0, 1, 2, 3]
    ev = [[0, 1, 2, 3, 4, 6, 8]]
    x, y = prefetch.training_examples(ev, vocab, context=3)
    assert x.tolist() == [[0, 0, 0], [0, 0, 0], [0, 0, 1]]
    assert y.tolist() == [0, 1, 1]


def test_background_pre_encryption_hand_cases():
    """Background pre-encryption (the paper's conclusions suggest it): after
    each window miss, while free slots + clean pages < threshold, the oldest
    page that is not clean is encrypted in the background."""
    # W=2, threshold 1, no writes: every eviction finds its page clean
    cnt, _ = window_sim.simulate([0, 1, 2, 0], window=2, bg_threshold=1,
                                 writes=[0, 0, 0, 0])
    # t1: {0,1} full, 0 encrypted in background; t2: 0 evicted clean, 1
    # encrypted; t3 (fault on 0): 1 evicted clean, 2 encrypted
    assert cnt["encrypts"] == 0 and cnt["evict_clean"] == 2
    assert cnt["encrypts_bg"] == 3 and cnt["bg_wasted"] == 0
    assert cnt["faults"] == 1 and cnt["first_touch"] == 3
    # a write to a clean page undoes its background encryption
    cnt, _ = window_sim.simulate([0, 1, 0, 2], window=2, bg_threshold=1,
                                 writes=[0, 0, 1, 0])
    # t1: 0 encrypted in background; t2: 0 written (wasted); t3: 0 evicted
    # dirty (encrypted on the fault path), 1 encrypted in background
    assert cnt["encrypts"] == 1 and cnt["evict_clean"] == 0
    assert cnt["encrypts_bg"] == 2 and cnt["bg_wasted"] == 1
    # a write to a page that is not clean costs nothing extra
    cnt, _ = window_sim.simulate([0, 1, 1, 2], window=2, bg_threshold=1,
                                 writes=[0, 0, 1, 0])
    assert cnt["encrypts"] == 0 and cnt["evict_clean"] == 1
    assert cnt["encrypts_bg"] == 2 and cnt["bg_wasted"] == 0


def test_background_pre_encryption_invariants():
    """On a mixed trace, for several thresholds: the window's behaviour
    (faults, first touches, decrypts, evictions) does not change; every
    eviction is either clean or encrypted on the fault path; every
    background encryption ends clean-evicted, wasted by a write, or still
    clean in the window at the end."""
    tr = workloads.access_trace(seed=12, accesses=8 * 3000, clients=8,
                                total_pages=8 * 256)
    for c in range(tr.clients):
        pages = tr.page[c]
        writes = tr.value[c] != 0
        base, _ = window_sim.simulate(pages, 6)
        assert base["encrypts_bg"] == 0 and base["evict_clean"] == 0
        same, _ = window_sim.simulate(pages, 6, writes=writes, bg_threshold=0)
        assert same == base
        for thr in (1, 2, 4, 6, 9):
            cnt, log = window_sim.simulate(pages, 6, writes=writes,
                                           bg_threshold=thr)
            for k in ("faults", "first_touch", "decrypts", "accesses"):
                assert cnt[k] == base[k], (thr, k)
            assert cnt["encrypts"] + cnt["evict_clean"] == base["encrypts"]
            left = cnt["encrypts_bg"] - cnt["evict_clean"] - cnt["bg_wasted"]
            assert 0 <= left <= 6, (thr, left)
            # a larger threshold never puts more encryptions on the fault path
            if thr > 1:
                assert cnt["encrypts"] <= prev["encrypts"], thr
            prev = cnt


def test_product_host_logic_matches_oracle_with_background():
    tr = workloads.access_trace(seed=13, accesses=8 * 2000, clients=8,
                                total_pages=8 * 256)
    for thr in (1, 3):
        cnt, _, _, _ = prefetch.run(tr, 6, count_from=300, bg_threshold=thr)
        tot = {}
        for c in range(tr.clients):
            o, _ = window_sim.simulate(tr.page[c], 6, start=300,
                                       writes=tr.value[c] != 0,
                                       bg_threshold=thr)
            for k, v in o.items():
                tot[k] = tot.get(k, 0) + v
        for k, v in tot.items():
            assert cnt[k] == v, (thr, k)
