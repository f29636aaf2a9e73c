"""Surrogate ranker MLP (float64 oracle).

A small network predicts the outer fraction OBV / V_box of a candidate box from
its 15 normalised parameters and an 8 x 8 x 8 occupancy of the box (527 inputs,
zero-padded to 544): 544 -> 256 (ReLU) -> 256 (ReLU) -> 1.  The output is a
correction of the occupancy estimate h = 1 - mean(occupancy):
f = h + sigmoid(z) - 1/2.  The HIP
path multiplies bfloat16 operands with float32 accumulation; this oracle
computes in float64 and, when ``bf16=True``, rounds to bfloat16
(round-to-nearest-even) exactly where the HIP path feeds a matrix product:
the inputs, the weights, the hidden activations, and the back-propagated
gradients entering each product.  Loss: mean squared error on the fraction.
Optimiser: Adam (Kingma and Ba, 2015) with float32 master weights on the GPU.
"""
import numpy as np

D_IN, D_PAD, D_H = 527, 544, 256


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-uniform weights, the output layer scaled by 0.1 so that training starts
    near the occupancy estimate (z close to 0), zero biases (float64); W are [in, out]."""
    g = np.random.default_rng(seed)

    def he(n_in, n_out):
        lim = np.sqrt(6.0 / n_in)
        return g.uniform(-lim, lim, size=(n_in, n_out))
    W1 = he(D_PAD, D_H)
    W1[D_IN:] = 0.0
    return {"W1": W1, "b1": np.zeros(D_H), "W2": he(D_H, D_H), "b2": np.zeros(D_H),
            "w3": 0.1 * he(D_H, 1)[:, 0], "b3": np.zeros(1)}


def forward(X, p, bf16_points=True):
    r = bf16 if bf16_points else (lambda a: np.asarray(a, np.float64))
    Xb = r(X)
    Z1 = Xb @ r(p["W1"]) + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    H1b = r(H1)
    Z2 = H1b @ r(p["W2"]) + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    H2b = r(H2)
    z = H2b @ r(p["w3"]) + p["b3"][0]
    sig = 1.0 / (1.0 + np.exp(-z))
    h = 1.0 - np.asarray(X, np.float64)[:, 15:D_IN].mean(axis=1)
    f = h + sig - 0.5
    return f, {"Xb": Xb, "Z1": Z1, "H1b": H1b, "Z2": Z2, "H2b": H2b, "z": z, "sig": sig}


def loss_and_grads(X, t, p, bf16_points=True):
    """Mean squared error and its gradients with respect to every parameter."""
    r = bf16 if bf16_points else (lambda a: np.asarray(a, np.float64))
    f, c = forward(X, p, bf16_points)
    n = X.shape[0]
    loss = float(np.mean((f - t) ** 2))
    dz = 2.0 * (f - t) * c["sig"] * (1.0 - c["sig"]) / n
    dzb = r(dz)
    g = {"w3": c["H2b"].T @ dzb, "b3": np.array([dz.sum()])}
    dH2 = np.outer(dzb, r(p["w3"])) * (c["Z2"] > 0)
    dH2b = r(dH2)
    g["W2"] = c["H1b"].T @ dH2b
    g["b2"] = dH2.sum(0)
    dH1 = (dH2b @ r(p["W2"]).T) * (c["Z1"] > 0)
    dH1b = r(dH1)
    g["W1"] = c["Xb"].T @ dH1b
    g["b1"] = dH1.sum(0)
    return loss, g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place); state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def box_features(center, axes, half, bbox_center, bbox_diag, occupancy):
    """The 544-wide input row: (c - bbox_centre) / diag, axes (9), log(h / diag),
    the 512 occupancy values (x-major, then y, then z), zero padding."""
    x = np.zeros(D_PAD)
    x[0:3] = (np.asarray(center, np.float64) - bbox_center) / bbox_diag
    x[3:12] = np.asarray(axes, np.float64).reshape(-1)
    x[12:15] = np.log(np.maximum(np.asarray(half, np.float64), 1e-30) / bbox_diag)
    x[15:527] = np.asarray(occupancy, np.float64).reshape(-1)
    return x
