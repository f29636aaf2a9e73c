"""Pins of the surrogate MLP oracle."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_definition_and_torch():
    # 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1.0)
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -9) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-(1.0 + 2.0 ** -7 + 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    x = np.random.default_rng(0).normal(size=10000) * 10.0 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_backward_matches_central_differences_float64():
    g = np.random.default_rng(3)
    p = mlp.init_params(seed=1)
    X = g.normal(size=(16, mlp.D_PAD))
    X[:, mlp.D_IN:] = 0
    t = g.uniform(0.05, 0.95, size=16)
    _, grads = mlp.loss_and_grads(X, t, p, bf16_points=False)
    eps = 1e-6
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = p[k].reshape(-1)
        for idx in g.choice(flat.size, size=min(6, flat.size), replace=False):
            if k == "W1" and idx // mlp.D_H >= mlp.D_IN:
                continue
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = mlp.loss_and_grads(X, t, p, bf16_points=False)
            flat[idx] = old - eps
            lm, _ = mlp.loss_and_grads(X, t, p, bf16_points=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[k].reshape(-1)[idx]
            # rounding of the two losses (~0.1, ulp ~1.4e-17, a few ulps each)
            # divided by 2 eps = 2e-6 gives an absolute floor of about 5e-11
            assert abs(fd - an) <= 1e-7 * max(abs(fd), abs(an)) + 5e-11, (k, idx, fd, an)


def test_adam_reduces_loss_on_a_smooth_target():
    g = np.random.default_rng(4)
    p = mlp.init_params(seed=2)
    X = g.normal(size=(256, mlp.D_PAD)) * 0.5
    X[:, 15:mlp.D_IN] = g.uniform(0, 1, size=(256, mlp.D_IN - 15))
    X[:, mlp.D_IN:] = 0
    h = 1.0 - X[:, 15:mlp.D_IN].mean(axis=1)
    t = np.clip(h + 0.2 * np.tanh(X[:, 0] - 0.5 * X[:, 1]), 0, 1)
    st = {}
    l0, _ = mlp.loss_and_grads(X, t, p)
    for _ in range(60):
        _, gr = mlp.loss_and_grads(X, t, p)
        mlp.adam_step(p, gr, st, lr=1e-3)
    l1, _ = mlp.loss_and_grads(X, t, p)
    assert l1 < 0.5 * l0


def test_feature_row_layout():
    occ = np.arange(512) / 512.0
    x = mlp.box_features([1, 2, 3], np.eye(3), [0.5, 1.0, 2.0], np.array([1.0, 1.0, 1.0]), 2.0, occ)
    assert x.shape == (544,)
    assert np.allclose(x[:3], [0, 0.5, 1.0]) and np.allclose(x[3:12], np.eye(3).reshape(-1))
    assert np.allclose(x[12:15], np.log([0.25, 0.5, 1.0]))
    assert np.array_equal(x[15:527], occ) and not x[527:].any()


def test_adam_first_step_is_a_signed_learning_rate_step():
    """Kingma and Ba (2015): after one step from zero moments the bias-corrected
    update is lr * g / (|g| + eps) per parameter."""
    g = np.random.default_rng(9)
    p = {"a": g.normal(size=7), "b": g.normal(size=(2, 3))}
    grads = {"a": g.normal(size=7), "b": g.normal(size=(2, 3)) * 1e-3}
    ref = {k: v - 0.01 * grads[k] / (np.abs(grads[k]) + 1e-8) for k, v in p.items()}
    out = mlp.adam_step({k: v.copy() for k, v in p.items()}, grads, {}, lr=0.01)
    for k in p:
        assert np.allclose(out[k], ref[k], rtol=1e-12, atol=1e-15)
