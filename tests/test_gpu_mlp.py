"""GPU predictor kernels vs the float64 reference network fed the same
bf16-rounded tensors (oracle/mlp_ref.py).  Tolerance for float32-accumulated
bf16 products against the float64 reference, per tensor: max|diff| <=
2^-6 * max|ref| and cosine similarity >= 0.999.  Integer decisions (top-k)
are compared exactly, both sides deciding on the GPU's own float32 logits."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu

SHAPE = dict(vocab=1024, context=16, embed=64, hidden=256)


def _note(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _close(got, ref, what):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    cos = float(got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref) +
                             1e-300))
    assert err <= 2**-6 * scale, "%s: max err %g vs scale %g" % (what, err,
                                                                   scale)
    assert cos >= 0.999, "%s: cosine %f" % (what, cos)


@pytest.fixture(scope="module")
def pred():
    from paper_2004_09252_amd.predictor import Predictor
    return Predictor(max_batch=1024, **SHAPE)


def _load(pred, seed):
    rng = np.random.default_rng(seed)
    p = mlp_ref.init_params(rng, **SHAPE)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    blob = np.concatenate([p[k].reshape(-1) for k in mlp_ref.PARAMS])
    pred.load_master(blob.astype(np.float32))
    pb = {k: mlp_ref.bf16_round(v.astype(np.float32)) for k, v in p.items()}
    return pb, rng


def test_bf16_blob_is_round_to_nearest_even(pred):
    _note("bf16 blob")
    import torch
    _load(pred, 1)
    want = pred.master.cpu().to(torch.bfloat16)
    assert torch.equal(pred.params.cpu().view(torch.int16),
                       want.view(torch.int16))


@pytest.mark.parametrize("batch", [1, 7, 64, 200, 1024])
def test_forward_matches_reference(pred, batch):
    _note("forward batch=%d" % batch)
    pb, rng = _load(pred, 2)
    ids = rng.integers(0, SHAPE["vocab"], size=(batch, SHAPE["context"]))
    got = pred.forward(ids).cpu().numpy()
    ref, _ = mlp_ref.forward(pb, ids, round_fn=mlp_ref.bf16_round)
    _close(got, ref, "logits")


def test_backward_matches_reference(pred):
    _note("backward")
    pb, rng = _load(pred, 3)
    B = 1024
    ids = rng.integers(0, SHAPE["vocab"], size=(B, SHAPE["context"]))
    # skewed ids so that embedding rows collect many contributions
    ids[: B // 2] = rng.integers(0, 8, size=(B // 2, SHAPE["context"]))
    tgt = rng.integers(0, SHAPE["vocab"], size=B)
    loss = float(pred.backward(ids, tgt).cpu().numpy()[0])
    ref_loss, g = mlp_ref.loss_and_grads(pb, ids, tgt,
                                         round_fn=mlp_ref.bf16_round,
                                         grad_round_fn=mlp_ref.bf16_round)
    assert abs(loss - ref_loss) <= 1e-3 * abs(ref_loss)
    gg = pred.unpack(pred.grads.cpu())
    for k in mlp_ref.PARAMS:
        _close(gg[k].numpy(), g[k], "grad " + k)


def test_adam_step_matches_reference(pred):
    """Three GPU Adam steps against oracle.mlp_ref.adam_step (which
    tests/test_mlp_oracle.py pins to torch.optim.Adam), same gradient each
    step, parameters compared tensor by tensor."""
    _note("adam")
    import torch
    _load(pred, 4)
    rng = np.random.default_rng(44)
    g = rng.normal(0, 1e-2, pred.n_params).astype(np.float32)
    w0 = pred.master.cpu()
    pred.grads.copy_(torch.from_numpy(g))
    for _ in range(3):
        pred.adam(lr=1e-3)
    got = pred.unpack(pred.master.cpu())
    p = {k: t.numpy().astype(np.float64) for k, t in pred.unpack(w0).items()}
    gd = {k: t.numpy().astype(np.float64)
          for k, t in pred.unpack(torch.from_numpy(g)).items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    for t in range(1, 4):
        mlp_ref.adam_step(p, gd, m, v, t, lr=1e-3)
    for k in mlp_ref.PARAMS:
        assert np.max(np.abs(got[k].numpy() - p[k])) < 1e-6, k
    want = pred.master.cpu().to(torch.bfloat16)
    assert torch.equal(pred.params.cpu().view(torch.int16),
                       want.view(torch.int16))


def test_topk_exact_on_gpu_logits(pred):
    _note("topk")
    pb, rng = _load(pred, 5)
    ids = rng.integers(0, SHAPE["vocab"], size=(300, SHAPE["context"]))
    logits = pred.forward(ids)
    host = logits.cpu().numpy()
    # plant ties: across lanes at the top of row 0; everywhere in row 1
    # (values on a coarse grid, so positions 64 apart, which one lane scans,
    # tie too); row 2 all equal (the answer is then ids 0..k-1)
    host[0, 10] = host[0, 20] = host[0, 30] = host[0].max() + 1.0
    host[1] = np.floor(host[1] * 2.0) / 2.0
    host[2] = 0.25
    logits.copy_(__import__("torch").from_numpy(host))
    got, prob = pred.topk(logits, 8, SHAPE["vocab"] - 1, with_prob=True)
    got = got.cpu().numpy()
    want = mlp_ref.topk_ids(host, 8, exclude=SHAPE["vocab"] - 1)
    assert np.array_equal(got, want)
    assert got[0, :3].tolist() == [10, 20, 30]
    assert got[2].tolist() == list(range(8))
    got16 = pred.topk(logits, 16, 3)
    assert np.array_equal(got16.cpu().numpy(),
                          mlp_ref.topk_ids(host, 16, exclude=3))
    h64 = host.astype(np.float64)
    sm = np.exp(h64 - h64.max(axis=1, keepdims=True))
    sm /= sm.sum(axis=1, keepdims=True)
    want_p = np.take_along_axis(sm, want, axis=1)
    assert np.max(np.abs(prob.cpu().numpy() - want_p)) < 1e-5


def test_training_learns_a_simple_rule(pred):
    """Target = the last input id: the loss must fall far below log(V)."""
    _note("training")
    _load(pred, 6)
    rng = np.random.default_rng(66)
    from paper_2004_09252_amd import prefetch
    xs = rng.integers(0, 64, size=(8192, SHAPE["context"])).astype(np.int32)
    ys = xs[:, -1].copy()
    losses = prefetch.train(pred, xs, ys, steps=300, batch=256, lr=3e-3)
    assert losses[0] > 5.0
    assert losses[-20:].mean() < 0.5, losses[-20:]


def test_save_load_round_trip(pred, tmp_path):
    _note("save/load")
    import torch
    _load(pred, 7)
    before = pred.params.clone()
    path = str(tmp_path / "pred.npz")
    pred.save(path)
    pred.init_random(123)
    assert not torch.equal(pred.params, before)
    pred.load(path)
    assert torch.equal(pred.params.view(torch.int16), before.view(torch.int16))


ODD = dict(vocab=192, context=17, embed=32, hidden=96)


def test_ragged_split_k_matches_reference_and_repeats_exactly():
    """A shape whose long-K GEMMs split K into slices that end inside a K
    step (K = 544 -> 384 + 160; batch 777 -> 384 + 384 + 9) over ragged
    output tiles (hidden 96): logits and gradients match the reference, and
    a second backward pass gives bit-identical gradients (a second kernel
    adds the slices' partial products in slice order)."""
    _note("ragged split-K shape %s batch 777" % ODD)
    from paper_2004_09252_amd.predictor import Predictor
    pred = Predictor(max_batch=1024, **ODD)
    rng = np.random.default_rng(21)
    p = mlp_ref.init_params(rng, **ODD)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    pred.load_master(np.concatenate(
        [p[k].reshape(-1) for k in mlp_ref.PARAMS]).astype(np.float32))
    pb = {k: mlp_ref.bf16_round(v.astype(np.float32)) for k, v in p.items()}
    B = 777
    ids = rng.integers(0, ODD["vocab"], size=(B, ODD["context"]))
    tgt = rng.integers(0, ODD["vocab"], size=B)
    got = pred.forward(ids).cpu().numpy()
    ref, _ = mlp_ref.forward(pb, ids, round_fn=mlp_ref.bf16_round)
    _close(got, ref, "logits")
    pred.backward(ids, tgt)
    first = pred.grads.cpu().clone()
    _, g = mlp_ref.loss_and_grads(pb, ids, tgt, round_fn=mlp_ref.bf16_round,
                                  grad_round_fn=mlp_ref.bf16_round)
    gg = pred.unpack(first)
    for k in mlp_ref.PARAMS:
        _close(gg[k].numpy(), g[k], "grad " + k)
    pred.backward(ids, tgt)
    assert np.array_equal(pred.grads.cpu().numpy(), first.numpy())


WIDE = dict(vocab=128, context=20, embed=96, hidden=64)


def test_embedding_gradient_over_several_id_chunks():
    """Batch 1000 x context 20 = 20000 ids: the embedding-gradient kernel
    stages them in two chunks (16384, then a ragged 3616), and embed 96
    takes two column passes (64, then a ragged 32).  Two rows collect 3000
    contributions each, across both chunks (their position lists fill and
    are added many times over), and one row none.  The gradients match the
    reference, and a second pass is bit-identical."""
    _note("embedding gradient shape %s batch 1000" % WIDE)
    from paper_2004_09252_amd.predictor import Predictor
    pred = Predictor(max_batch=1024, **WIDE)
    rng = np.random.default_rng(23)
    p = mlp_ref.init_params(rng, **WIDE)
    pred.load_master(np.concatenate(
        [p[k].reshape(-1) for k in mlp_ref.PARAMS]).astype(np.float32))
    pb = {k: mlp_ref.bf16_round(v.astype(np.float32)) for k, v in p.items()}
    B = 1000
    ids = rng.integers(2, WIDE["vocab"] - 1, size=(B, WIDE["context"]))
    ids[:300] = rng.integers(0, 2, size=(300, WIDE["context"]))
    ids[-1, -1] = 0  # the last position of the ragged chunk
    tgt = rng.integers(0, WIDE["vocab"], size=B)
    pred.backward(ids, tgt)
    first = pred.grads.cpu().clone()
    _, g = mlp_ref.loss_and_grads(pb, ids, tgt, round_fn=mlp_ref.bf16_round,
                                  grad_round_fn=mlp_ref.bf16_round)
    gg = pred.unpack(first)
    dE = gg["E"].numpy().reshape(WIDE["vocab"], WIDE["embed"])
    assert not np.any(dE[WIDE["vocab"] - 1])
    for k in mlp_ref.PARAMS:
        _close(gg[k].numpy(), g[k], "grad " + k)
    pred.backward(ids, tgt)
    assert np.array_equal(pred.grads.cpu().numpy(), first.numpy())


def test_topk_ragged_vocab_over_several_chunks():
    """A vocabulary of 2500 (three 1024-wide chunks, the last ragged), an
    excluded id, a row that is -inf but for one value, ties, and rows with
    NaN (ranked as -inf): ids equal the reference's exactly, probabilities
    the float64 softmax within 1e-5."""
    _note("topk V=2500")
    import torch
    from paper_2004_09252_amd import memshield as ms
    rng = np.random.default_rng(31)
    B, V, k, exclude = 37, 2500, 16, 1234
    host = rng.normal(0, 3, (B, V)).astype(np.float32)
    host[0, :] = -np.inf
    host[0, 2499] = 1.0
    host[1] = np.floor(host[1])           # ties within and across lanes
    host[2, 2040:2060] = host[2].max() + 1.0   # ties across a chunk edge
    host[3, exclude] = host[3].max() + 5.0     # the best is excluded
    stream = torch.cuda.current_stream().cuda_stream

    def run(h, with_prob):
        logits = torch.from_numpy(h).to("cuda")
        ids = torch.empty(B * k, dtype=torch.int32, device="cuda")
        pr = torch.empty(B * k, dtype=torch.float32, device="cuda")
        st = ms.ms_mlp_topk(logits.data_ptr(), B, V, k, exclude,
                            ids.data_ptr(),
                            pr.data_ptr() if with_prob else None, stream)
        assert st == ms.MS_OK
        torch.cuda.synchronize()
        return ids.view(B, k).cpu().numpy(), pr.view(B, k).cpu().numpy()

    got, prob = run(host, True)
    want = mlp_ref.topk_ids(host, k, exclude=exclude)
    assert np.array_equal(got, want)
    h64 = host.astype(np.float64)
    sm = np.exp(h64 - h64.max(axis=1, keepdims=True))
    sm /= sm.sum(axis=1, keepdims=True)
    assert np.max(np.abs(prob - np.take_along_axis(sm, want, axis=1))) < 1e-5
    nan = host.copy()
    nan[5:9, ::7] = np.nan
    got, _ = run(nan, False)
    ranked = np.where(np.isnan(nan), -np.inf, nan)
    assert np.array_equal(got, mlp_ref.topk_ids(ranked, k, exclude=exclude))
