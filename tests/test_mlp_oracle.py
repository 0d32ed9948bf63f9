"""Pins of the predictor's reference network (oracle/mlp_ref.py) against
things other than itself: central finite differences in float64, torch's
own bfloat16 conversion, cross-entropy and Adam (library routines), and
hand-made top-k cases."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref


def _tiny(seed=0):
    rng = np.random.default_rng(seed)
    p = mlp_ref.init_params(rng, vocab=12, context=3, embed=4, hidden=5)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.3, p[k].shape)
    ids = rng.integers(0, 12, size=(6, 3))
    tgt = rng.integers(0, 12, size=6)
    return p, ids, tgt


def test_gradients_match_central_differences():
    p, ids, tgt = _tiny()
    _, g = mlp_ref.loss_and_grads(p, ids, tgt)
    rng = np.random.default_rng(1)
    h = 1e-6
    for name in mlp_ref.PARAMS:
        flat = p[name].reshape(-1)
        for i in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp_ref.loss_and_grads(p, ids, tgt)
            flat[i] = old - h
            lm, _ = mlp_ref.loss_and_grads(p, ids, tgt)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            ana = g[name].reshape(-1)[i]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(num)), (name, i)


def test_embedding_gradient_sums_repeated_ids():
    p, ids, tgt = _tiny(2)
    ids[:, :] = 5          # every slot uses the same row
    _, g = mlp_ref.loss_and_grads(p, ids, tgt)
    nz = np.nonzero(np.abs(g["E"]).sum(axis=1))[0]
    assert list(nz) == [5]


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-30, 100),
                        [1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, -2.5, 0.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(
        torch.float64).numpy()
    assert np.array_equal(mlp_ref.bf16_round(x), want)
    assert mlp_ref.bf16_round(np.array([1.0 + 2**-8]))[0] == 1.0  # tie->even


def test_loss_matches_torch_cross_entropy():
    p, ids, tgt = _tiny(4)
    logits, _ = mlp_ref.forward(p, ids)
    loss, _ = mlp_ref.loss_and_grads(p, ids, tgt)
    want = torch.nn.functional.cross_entropy(
        torch.tensor(logits), torch.tensor(tgt)).item()
    assert abs(loss - want) < 1e-12


def test_adam_matches_torch_optimizer():
    p, ids, tgt = _tiny(5)
    tp = {k: torch.tensor(v.copy(), requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999),
                           eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    for step in range(1, 4):
        _, g = mlp_ref.loss_and_grads(p, ids, tgt)
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        mlp_ref.adam_step(p, g, m, v, step)
        for k in tp:
            assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-12,
                               atol=1e-15), (k, step)


def test_topk_tie_break_and_exclude():
    logits = np.array([[1.0, 3.0, 3.0, 2.0, 3.0, 0.5]])
    assert mlp_ref.topk_ids(logits, 3).tolist() == [[1, 2, 4]]
    assert mlp_ref.topk_ids(logits, 3, exclude=2).tolist() == [[1, 4, 3]]


def test_rounded_network_close_to_exact_one():
    rng = np.random.default_rng(6)
    p = mlp_ref.init_params(rng, vocab=64, context=4, embed=8, hidden=32)
    ids = rng.integers(0, 64, size=(16, 4))
    pb = {k: mlp_ref.bf16_round(v) for k, v in p.items()}
    exact, _ = mlp_ref.forward(pb, ids)
    rounded, _ = mlp_ref.forward(pb, ids, round_fn=mlp_ref.bf16_round)
    assert np.max(np.abs(exact - rounded)) < 2**-5 * np.max(np.abs(exact))
