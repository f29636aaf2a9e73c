"""HIP ranker features and MLP vs the CPU oracle (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import raygrid
from conftest import record_parity

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


def _dyadic_problem(n, seed):
    """Inputs on the 2^-4 grid in [-4, 4], W1 on the 2^-8 grid, b1 on 2^-12: every
    product of the first layer is a multiple of 2^-12 of size at most 1, so every
    partial sum of its 544 terms (below 2^10) is exact in float32, in any order."""
    p, X, t = _rand_problem(n, seed)
    X = np.clip(np.round(X * 16) / 16, -4, 4)
    X[:, omlp.D_IN:] = 0
    p["W1"] = np.round(p["W1"] * 256) / 256
    p["b1"] = np.round(p["b1"] * 4096) / 4096
    return p, X, t


def _rand_problem(n, seed):
    g = np.random.default_rng(seed)
    p = omlp.init_params(seed=seed)
    for k in ("b1", "b2", "b3"):
        p[k] = g.normal(0, 0.05, size=p[k].shape)
    X = g.normal(0, 1.0, size=(n, omlp.D_PAD))
    X[:, omlp.D_IN:] = 0
    t = g.uniform(0.05, 0.95, size=n)
    return p, X, t


def _grad_error_bounds(X, t, p, exact_first_layer=False):
    """First-order bound on |g_device - g_oracle| for every gradient entry.

    Both sides round to bfloat16 at the same points: inputs and weights from
    the same float32 values (identical), hidden activations and
    back-propagated gradients after float32 (device) vs float64 (oracle)
    accumulation.  Rounding is monotone, so a value known to lie within +-e of
    the oracle's v rounds to within bf16(v + e) - bf16(v - e) of the oracle's
    rounded value: zero unless a rounding boundary falls inside the interval.
    Each product adds the float32 accumulation error gamma_n = n 2^-24 times its
    absolute-value product; a ReLU is monotone too, and its derivative mask may
    differ where |Z| is within its error of 0.  The errors are carried through
    the network in absolute value.  With ``exact_first_layer`` the inputs,
    W1 and b1 lie on dyadic grids on which every float32 partial sum of the
    first layer is exact (its error term is zero)."""
    u = 2.0 ** -24
    r = omlp.bf16

    def spread(v, e):
        return r(v + e) - r(v - e)

    f, c = omlp.forward(X, p)
    n = X.shape[0]
    Xb, W1, W2, w3 = r(X), r(p["W1"]), r(p["W2"]), r(p["w3"])
    aX, aW1, aW2, aw3 = np.abs(Xb), np.abs(W1), np.abs(W2), np.abs(w3)
    eZ1 = 0.0 * aX[:, :1] if exact_first_layer else omlp.D_PAD * u * (aX @ aW1)
    eH1 = spread(np.maximum(c["Z1"], 0.0), 0.0) + (r(np.maximum(c["Z1"] + eZ1, 0.0))
                                                  - r(np.maximum(c["Z1"] - eZ1, 0.0)))
    aH1 = np.abs(c["H1b"])
    eZ2 = omlp.D_H * u * (aH1 @ aW2) + eH1 @ aW2
    eH2 = r(np.maximum(c["Z2"] + eZ2, 0.0)) - r(np.maximum(c["Z2"] - eZ2, 0.0))
    aH2 = np.abs(c["H2b"])
    ez = omlp.D_H * u * (aH2 @ aw3) + eH2 @ aw3
    sig = c["sig"]
    ds = sig * (1 - sig)
    dz = 2.0 * (f - t) * ds / n
    edz = 2.0 / n * (ds * ds * ez + np.abs(f - t) * 0.1 * ez) + 8 * u * np.abs(dz)
    dzb = r(dz)
    adzb = np.abs(dzb)
    edzb = spread(dz, edz)
    g = {"w3": n * u * (aH2.T @ adzb) + eH2.T @ adzb + aH2.T @ edzb,
         "b3": np.array([edz.sum() + n * u * np.abs(dz).sum()])}
    live2, edge2 = c["Z2"] > 0, np.abs(c["Z2"]) <= eZ2
    dH2 = np.outer(dzb, w3) * live2
    edH2 = np.outer(edzb, aw3) * (live2 | edge2) + np.abs(np.outer(dzb, w3)) * edge2
    adH2b = np.abs(r(dH2))
    edH2b = spread(dH2, edH2)
    g["W2"] = n * u * (aH1.T @ adH2b) + eH1.T @ adH2b + aH1.T @ edH2b
    g["b2"] = edH2.sum(0) + n * u * np.abs(dH2).sum(0)
    live1, edge1 = c["Z1"] > 0, np.abs(c["Z1"]) <= eZ1
    back = r(dH2) @ W2.T
    dH1 = back * live1
    eback = omlp.D_H * u * (adH2b @ aW2.T) + edH2b @ aW2.T
    edH1 = eback * (live1 | edge1) + np.abs(back) * edge1
    edH1b = spread(dH1, edH1)
    g["W1"] = n * u * (aX.T @ np.abs(r(dH1))) + aX.T @ edH1b
    g["b1"] = edH1.sum(0) + n * u * np.abs(dH1).sum(0)
    return g


def test_mlp_forward_and_gradients_match_oracle(api):
    """Same bfloat16 rounding points, float32 vs float64 accumulation:
    gradients within 1e-3 relative (per tensor, in norm) and every entry within
    1e-3 relative or within the rounding-point bound; outputs within 1e-4.  The
    first layer's inputs and weights lie on dyadic grids that make its float32
    sums exact, so its rounding points agree on both sides."""
    import torch
    p, X, t = _dyadic_problem(96, 5)
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
    bound = _grad_error_bounds(X, t, p, exact_first_layer=True)
    floored = 0
    for k in g_ref:
        num = np.linalg.norm(g[k] - g_ref[k])
        den = np.linalg.norm(g_ref[k])
        assert num <= 1e-3 * den + 1e-12, (k, num / max(den, 1e-30))
        # every entry: within 1e-3 relative, or within the bound of the rounding points
        err = np.abs(g[k] - g_ref[k])
        rel_ok = err <= 1e-3 * np.abs(g_ref[k])
        assert np.all(rel_ok | (err <= bound[k])), (k, float((err - bound[k]).max()))
        floored += int((~rel_ok).sum())
    record_parity({"test": "mlp_gradients_elementwise", "entries": int(sum(v.size for v in g_ref.values())),
                   "entries_within_rounding_bound_only": floored})


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
