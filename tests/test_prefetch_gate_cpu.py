"""Host logic of the learned pre-decryption (CPU, no GPU): the predictor's
default confidence gate and how the decrypt-on-fault replay applies it.

A stub predictor stands in for the network: it names fixed deltas with
fixed probabilities, so which pages are pre-decrypted follows from the gate
alone."""
import torch

from paper_2004_09252_amd import prefetch, workloads
from paper_2004_09252_amd.predictor import Predictor


class _Stub:
    context = 16

    def __init__(self, probs, min_prob=Predictor.DEFAULT_MIN_PROB):
        self.probs = probs
        self.min_prob = min_prob

    def predict(self, ids, k, exclude, with_prob=False):
        rows = ids.shape[0]
        top = torch.arange(k, dtype=torch.int32).repeat(rows, 1)
        prob = torch.tensor(self.probs[:k], dtype=torch.float32).repeat(
            rows, 1)
        return top, prob


def _vocab():
    # ids 0..7 are deltas +1..+8
    return prefetch.DeltaVocab([d for d in range(1, 9) for _ in range(20 - d)])


def _trace():
    return workloads.access_trace(seed=31, total_pages=4 * 256,
                                  accesses=4 * 600, clients=4)


def test_default_gate_is_a_tenth():
    assert Predictor.DEFAULT_MIN_PROB == 0.1


def test_replay_uses_the_predictors_gate_by_default():
    tr = _trace()
    v = _vocab()
    assert list(v.delta_of[:8]) == list(range(1, 9))
    # deltas +1..+8 with falling probabilities: 0.5, 0.2, 0.12, 0.09, ...
    probs = [0.5, 0.2, 0.12, 0.09, 0.05, 0.02, 0.01, 0.01]
    _, _, gated, _ = prefetch.run(tr, 4, prefetch_slots=8,
                                  predictor=_Stub(probs), vocab=v, k=8)
    _, _, explicit, _ = prefetch.run(tr, 4, prefetch_slots=8,
                                     predictor=_Stub(probs), vocab=v, k=8,
                                     min_prob=0.1)
    assert gated == explicit and gated
    # only deltas +1..+3 pass a gate of 0.1
    for (c, t), pages in gated.items():
        last = int(tr.page[c, t])
        assert {p - last for p in pages} <= {1, 2, 3}
    _, _, ungated, _ = prefetch.run(tr, 4, prefetch_slots=8,
                                    predictor=_Stub(probs, min_prob=0.0),
                                    vocab=v, k=8)
    assert sum(map(len, ungated.values())) > sum(map(len, gated.values()))


def test_gate_keeps_exactly_the_confident_deltas():
    """Every pre-decrypted page is the last fault page plus one of the
    deltas whose probability reaches the gate."""
    tr = _trace()
    v = _vocab()
    probs = [0.05, 0.3, 0.05, 0.25, 0.05, 0.05, 0.1, 0.05]
    cnt, _, dec, _ = prefetch.run(tr, 4, prefetch_slots=8,
                                  predictor=_Stub(probs), vocab=v, k=8)
    allowed = {2, 4, 7}   # deltas of ids 1, 3 and 6
    for (c, t), pages in dec.items():
        # the fault event at step t is the client's last one up to t
        last = int(tr.page[c, t])
        assert {p - last for p in pages} <= allowed
    assert cnt["prefetch_issued"] == sum(map(len, dec.values())) > 0
