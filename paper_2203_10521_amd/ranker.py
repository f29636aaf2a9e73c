"""Training and evaluation of the candidate-box ranker (learned part of the flood).

Orchestration only: the training targets are outer fractions OBV / V_box from
the exact kernel (obbv_outer_volume), the inputs come from obbv_sample_features,
and every forward, backward and Adam step runs in the library's MFMA kernels.
"""
import math

import numpy as np
import torch

from . import api

PARAMS = 544 * 256 + 256 + 256 * 256 + 256 + 256 + 1


def init_params(seed=0):
    """He-uniform hidden weights (first-layer rows past the 527 real inputs zero),
    zero biases and a zero output layer: the untrained network predicts exactly
    the occupancy estimate 1 - mean occupancy, and training learns the correction."""
    g = np.random.default_rng(seed)

    def he(n_in, n_out):
        lim = math.sqrt(6.0 / n_in)
        return g.uniform(-lim, lim, size=(n_in, n_out))
    W1 = he(544, 256)
    W1[527:] = 0.0
    return {"W1": W1, "b1": np.zeros(256), "W2": he(256, 256), "b2": np.zeros(256),
            "w3": np.zeros(256), "b3": np.zeros(1)}


def occupancy_params(seed=0):
    """A ranker whose network output is 0 for every input (output layer zero, as
    before training): through the same machinery it predicts the occupancy
    estimate 1 - mean occupancy, the heuristic the learned ranker must beat."""
    return torch.from_numpy(api.mlp_pack(init_params(seed))).cuda()


def make_dataset(meshes, boxes, R=64, seed=0, nb=16):
    """Ranker inputs and targets for every (mesh, box set) pair.

    meshes: list of (V, F) device tensors; boxes: list of float32 [n, 15] device
    tensors.  Returns (X [N, 544], t [N]) on the device and the per-mesh
    (volume, frame) used for the features.
    """
    Xs, ts, vols = [], [], []
    for (Vt, Ft), B in zip(meshes, boxes):
        vol, frame = api.occupancy_volume(Vt, Ft, nb=nb, seed=seed)
        obv = api.outer_volume(Vt, Ft, B, R, seed=seed)
        vb = 8.0 * B[:, 12].double() * B[:, 13].double() * B[:, 14].double()
        ok = vb > 0
        t = torch.zeros_like(obv)
        t[ok] = (obv[ok] / vb[ok]).clamp(0.0, 1.0)
        Xs.append(api.sample_features(vol, frame, B))
        ts.append(t.to(torch.float32))
        vols.append((vol, frame))
    return torch.cat(Xs), torch.cat(ts), vols


def train(X, t, steps=2000, batch=4096, lr=1e-3, seed=0, log_every=0):
    """Adam with a cosine learning-rate decay on random mini-batches; returns
    (float32 parameter vector on the device, list of batch losses)."""
    P = torch.from_numpy(api.mlp_pack(init_params(seed))).to(X.device)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    n = X.shape[0]
    batch = min(batch, n // 32 * 32)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), device=X.device, generator=gen)
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / steps))
        loss, _ = api.mlp_train_step(P, m, v, step, X[idx].contiguous(), t[idx].contiguous(), rate)
        if log_every and (step % log_every == 0 or step == 1):
            losses.append((step, float(loss.item())))
    if not log_every:
        losses.append((steps, float(loss.item())))
    return P, losses


def _kmeans_groups(V, F, k, seed, iters=8):
    """Triangle groups by k-means of the centroids (host, numpy)."""
    cen = V.astype(np.float64)[F].mean(axis=1)
    g = np.random.default_rng(seed)
    C = cen[g.choice(len(cen), size=k, replace=False)]
    for _ in range(iters):
        lab = np.argmin(((cen[:, None, :] - C[None, :, :]) ** 2).sum(-1), axis=1)
        for j in range(k):
            sel = lab == j
            if sel.any():
                C[j] = cen[sel].mean(axis=0)
    return np.argmin(((cen[:, None, :] - C[None, :, :]) ** 2).sum(-1), axis=1).astype(np.int32)


def lloyd_boxes(V, F, R=64, seed=0, n_groups=16, per_group=4, iters=2, cap=8192, pops_per_round=32):
    """Boxes the flood meets in use: a uniform sample of the (box, exact outer
    volume) pairs evaluated by `iters` exact Lloyd iterations of `n_groups`
    k-means triangle groups with `per_group` boxes each (seeded at random
    triangles, axes of the group's covariance box).  V, F are host arrays;
    returns float32 [n, 15] boxes (host)."""
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    grp = _kmeans_groups(V, F, n_groups, seed) if n_groups > 1 else np.zeros(F.shape[0], np.int32)
    fitted, _ = api.fit(Vt, Ft, torch.from_numpy(grp).cuda(), n_groups)
    fitted = fitted.cpu().numpy()
    g = np.random.default_rng(seed + 1)
    cen = V.astype(np.float64)[F].mean(axis=1)
    boxes, box_group = [], []
    for j in range(n_groups):
        tris = np.nonzero(grp == j)[0]
        if len(tris) < per_group:
            continue
        for t in g.choice(tris, size=per_group, replace=False):
            b = fitted[j].copy()
            b[:3] = cen[t]
            b[12:] = 0.0
            boxes.append(b)
            box_group.append(j)
    with api.Lloyd(Vt, Ft, R=R, seed=seed, pops_per_round=pops_per_round) as L:
        L.set_groups(grp, np.array(box_group, np.int32), np.array(boxes, np.float32))
        L.record(cap)
        for _ in range(iters):
            L.step()
        B, _ = L.take_records()
    return B


def predict(P, X):
    """Predicted outer fractions of the rows of X (padded to a multiple of 32)."""
    n = X.shape[0]
    pad = (-n) % 32
    if pad:
        X = torch.cat([X, torch.zeros((pad, X.shape[1]), dtype=X.dtype, device=X.device)])
    return api.mlp_forward(P, X.contiguous())[:n]


def occupancy_heuristic(X):
    """Outer fraction estimated as 1 - mean of the 512 sampled occupancies."""
    return 1.0 - X[:, 15:527].mean(dim=1)


def ranking_metrics(P, X, t, obv, boxes, n_single, n_groups, k=8):
    """Prediction error and ranking quality on one mesh's evaluation set.

    Rows [0, n_single) are single boxes; then n_groups base boxes; then the
    n_groups x k candidates grown from them (in group order).  A candidate's
    change is f V(candidate) - f V(base) with f the predicted outer fraction;
    the exact change uses the exact outer volumes `obv`.  Returns sums over the
    mesh for the network P (None: skipped) and for 1 - mean occupancy:
    absolute errors of all rows and of the candidates, top-1 hits (the
    predicted best candidate of a group is the exact best) and correctly
    ordered candidate pairs."""
    vb = 8.0 * boxes[:, 12].double() * boxes[:, 13].double() * boxes[:, 14].double()
    b0, c0 = n_single, n_single + n_groups
    exact = obv[c0:].reshape(n_groups, k) - obv[b0:c0, None]
    iu = torch.triu_indices(k, k, 1, device=X.device)
    ex_pair = torch.sign(exact[:, iu[0]] - exact[:, iu[1]])
    out = {"rows": int(t.shape[0]), "candidates": int(n_groups * k), "groups": int(n_groups),
           "pairs": int((ex_pair != 0).sum().item())}
    preds = {"occupancy_mean": occupancy_heuristic(X)}
    if P is not None:
        preds["network"] = predict(P, X)
    for name, f in preds.items():
        err = (f - t).abs()
        ch = (f[c0:].double() * vb[c0:]).reshape(n_groups, k) - (f[b0:c0].double() * vb[b0:c0])[:, None]
        pr_pair = torch.sign(ch[:, iu[0]] - ch[:, iu[1]])
        out[name] = {"abs_err": float(err.sum().item()), "cand_abs_err": float(err[c0:].sum().item()),
                     "top1": int((ch.argmin(dim=1) == exact.argmin(dim=1)).sum().item()),
                     "pairs_ok": int(((pr_pair == ex_pair) & (ex_pair != 0)).sum().item())}
    return out


def summarise_metrics(per_mesh):
    """Means over meshes of ranking_metrics sums: MAE, candidate MAE, top-1 rate,
    pair accuracy, for each predictor."""
    tot = {k: sum(m[k] for m in per_mesh) for k in ("rows", "candidates", "groups", "pairs")}
    res = {}
    for name in ("network", "occupancy_mean"):
        if name not in per_mesh[0]:
            continue
        s = {k: sum(m[name][k] for m in per_mesh) for k in ("abs_err", "cand_abs_err", "top1", "pairs_ok")}
        res[name] = {"mae": s["abs_err"] / tot["rows"], "candidate_mae": s["cand_abs_err"] / tot["candidates"],
                     "top1": s["top1"] / tot["groups"], "pair_accuracy": s["pairs_ok"] / max(tot["pairs"], 1)}
    res.update(tot)
    return res
