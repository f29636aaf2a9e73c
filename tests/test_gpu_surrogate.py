"""HIP ranker features and MLP vs the CPU oracle (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import raygrid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def test_box_features_match_oracle_occupancy(api):
    import torch
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(8, seed=31, center_range=0.9, half_range=(0.2, 0.7))
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    B = torch.from_numpy(synth.boxes_to_array(c, a, h)).cuda()
    frame = api.mesh_frame(Vt)
    X = api.box_features(B, seed=17, meshes=[(Vt, Ft)]).cpu().numpy()
    fr = frame.cpu().numpy().astype(np.float64)
    for b in range(8):
        occ = raygrid.occupancy(V, F, c[b], a[b], h[b], 17, b)
        ref = omlp.box_features(c[b], a[b], h[b], fr[:3], fr[3], occ)
        assert np.allclose(X[b, :15], ref[:15], atol=2e-6)
        assert np.abs(X[b, 15:527] - ref[15:527]).max() <= 1e-4, b
        assert not X[b, 527:].any()


def _rand_problem(n, seed):
    g = np.random.default_rng(seed)
    p = omlp.init_params(seed=seed)
    for k in ("b1", "b2", "b3"):
        p[k] = g.normal(0, 0.05, size=p[k].shape)
    X = g.normal(0, 1.0, size=(n, omlp.D_PAD))
    X[:, omlp.D_IN:] = 0
    t = g.uniform(0.05, 0.95, size=n)
    return p, X, t


def test_mlp_forward_and_gradients_match_oracle(api):
    """Same bfloat16 rounding points, float32 vs float64 accumulation:
    gradients within 1e-3 relative (per tensor, in norm), outputs within 1e-4."""
    import torch
    p, X, t = _rand_problem(96, 5)
    # the GPU keeps float32 master weights: give the oracle the same float32 values
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    X = X.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    P = torch.from_numpy(api.mlp_pack(p)).cuda()
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    tt = torch.from_numpy(t.astype(np.float32)).cuda()
    f = api.mlp_forward(P, Xt).cpu().numpy()
    f_ref, _ = omlp.forward(X, p)
    assert np.abs(f - f_ref).max() <= 1e-4
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    loss, grad = api.mlp_train_step(P, m, v, 1, Xt, tt, lr=0.0, want_grad=True)
    l_ref, g_ref = omlp.loss_and_grads(X, t, p)
    assert abs(loss.item() - l_ref) <= 1e-4 * l_ref
    g = api.mlp_unpack(grad.cpu().numpy())
    for k in g_ref:
        num = np.linalg.norm(g[k] - g_ref[k])
        den = np.linalg.norm(g_ref[k])
        assert num <= 1e-3 * den + 1e-12, (k, num / max(den, 1e-30))


def test_mlp_adam_step_matches_oracle(api):
    import torch
    p, X, t = _rand_problem(64, 6)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    P = torch.from_numpy(api.mlp_pack(p)).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    tt = torch.from_numpy(t.astype(np.float32)).cuda()
    _, grad = api.mlp_train_step(P, m, v, 1, Xt, tt, lr=1e-3, want_grad=True)
    g = api.mlp_unpack(grad.cpu().numpy())
    ref = omlp.adam_step(dict(p), g, {}, lr=1e-3)
    got = api.mlp_unpack(P.cpu().numpy())
    for k in ref:
        assert np.abs(got[k] - ref[k]).max() <= 2e-6, k


def test_mlp_training_reduces_loss(api):
    import torch
    g = np.random.default_rng(8)
    n = 512
    X = g.normal(0, 1.0, size=(n, omlp.D_PAD)).astype(np.float32)
    X[:, 15:omlp.D_IN] = g.uniform(0, 1, size=(n, omlp.D_IN - 15))
    X[:, omlp.D_IN:] = 0
    h = 1.0 - X[:, 15:omlp.D_IN].mean(axis=1)
    t = np.clip(h + 0.2 * np.tanh(X[:, 0] - 0.5 * X[:, 5] + 0.3 * X[:, 10]), 0, 1).astype(np.float32)
    P = torch.from_numpy(api.mlp_pack(omlp.init_params(seed=1))).cuda()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    Xt, tt = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    losses = []
    for step in range(1, 201):
        loss, _ = api.mlp_train_step(P, m, v, step, Xt, tt, lr=1e-3)
        losses.append(loss.item())
    assert losses[-1] < 0.2 * losses[0]
