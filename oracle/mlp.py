"""Plain fp64 reference of the learned flip-proposal network.

TEST INFRASTRUCTURE ONLY (tests/, the smoke check): the product never imports
it.  The network is not in the paper (it names reinforcement learning only as
future work); it is this project's flip scorer:

    z1 = X W1 + b1,  h1 = relu(z1) rounded to bf16
    z2 = h1 W2 + b2, h2 = relu(z2) rounded to bf16
    logit = h2 . w3 + b3
    loss = mean over rows of softplus(logit) - y * logit   (binary cross-entropy)

X is M x 512 with entries exactly representable in bf16, W1 is 512 x 256, W2 is
256 x 256, w3 has 256 entries; the weights used for compute are the bf16
roundings of fp32 master weights.  Every function works in fp64 except the
explicit bf16 roundings, which are part of the definition because the GPU
passes activations between layers in bf16.

Each result also returns the L1 mass of the sums that produced it (sum of the
absolute values of the products), used to bound the fp32 accumulation error of
the GPU kernels.
"""
import numpy as np

D_IN, D_H = 512, 256


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as fp64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-style random initialisation (fp32 masters)."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.standard_normal((D_IN, D_H)) * np.sqrt(2.0 / 64.0),
        "b1": np.zeros(D_H),
        "W2": rng.standard_normal((D_H, D_H)) * np.sqrt(2.0 / D_H),
        "b2": np.zeros(D_H),
        "w3": rng.standard_normal(D_H) * np.sqrt(1.0 / D_H),
        "b3": np.zeros(1),
    }
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def forward(p, X, rounding=True):
    """-> dict with z1, h1, z2, h2, logit and the L1 masses m1, m2, m3.
    rounding=False drops the bf16 roundings (a smooth network, used to check
    the analytic gradients by finite differences)."""
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, w3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["w3"])
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + p["b1"]
    m1 = np.abs(X) @ np.abs(W1) + np.abs(p["b1"])
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ W2 + p["b2"]
    m2 = np.abs(h1) @ np.abs(W2) + np.abs(p["b2"])
    h2 = rnd(np.maximum(z2, 0.0))
    logit = h2 @ w3 + p["b3"][0]
    m3 = np.abs(h2) @ np.abs(w3) + abs(p["b3"][0])
    return {"z1": z1, "h1": h1, "z2": z2, "h2": h2, "logit": logit, "m1": m1, "m2": m2,
            "m3": m3}


def loss(p, X, y, rounding=True):
    z = forward(p, X, rounding)["logit"]
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def backward(p, X, y, rounding=True):
    """Gradients of the mean BCE loss with respect to the master weights.
    The bf16 roundings are treated as identity (straight-through), the ReLU
    derivative is 1 where the activation is positive."""
    f = forward(p, X, rounding)
    M = X.shape[0]
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W2, w3 = rnd(p["W2"]), rnd(p["w3"])
    d3 = (1.0 / (1.0 + np.exp(-f["logit"])) - y) / M           # dL/dlogit
    g = {"w3": f["h2"].T @ d3, "b3": np.array([d3.sum()])}
    d2 = np.outer(d3, w3) * (f["z2"] > 0)
    g["W2"] = f["h1"].T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (f["z1"] > 0)
    g["W1"] = np.asarray(X, dtype=np.float64).T @ d1
    g["b1"] = d1.sum(axis=0)
    return g, f


def adam(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on the fp32 masters, in fp64."""
    t = state.get("t", 0) + 1
    state["t"] = t
    out = {}
    for k in p:
        m = b1 * state.get("m_" + k, 0.0) + (1 - b1) * g[k]
        v = b2 * state.get("v_" + k, 0.0) + (1 - b2) * g[k] * g[k]
        state["m_" + k], state["v_" + k] = m, v
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


# Slots of the format one-hot of the feature rows: fifteen small formats with
# sorted dimensions, 15 for every other format (the same table as the
# library's, written out here independently).
FORMAT_SLOTS = {(2, 2, 2): 0, (2, 2, 3): 1, (2, 2, 4): 2, (2, 3, 3): 3, (2, 3, 4): 4,
                (3, 3, 3): 5, (3, 3, 4): 6, (2, 4, 4): 7, (3, 4, 4): 8, (3, 3, 5): 9,
                (4, 4, 4): 10, (3, 4, 5): 11, (4, 4, 5): 12, (4, 5, 5): 13, (5, 5, 5): 14}


def format_slot(m, n, p):
    return FORMAT_SLOTS.get(tuple(sorted((m, n, p))), 15)


def feature_row(factors, slot, rank):
    """factors: six int vectors (x_i, y_i, z_i, x_j, y_j, z_j) with entries in
    {-1,0,1} (length <= 64) -> the 512 feature values (fp64)."""
    row = np.zeros(D_IN)
    for b, vec in enumerate(factors):
        v = np.asarray(vec, dtype=np.float64)
        row[64 * b:64 * b + v.size] = v
    row[384 + slot] = 1.0
    row[400 + min(max(rank, 0), 95)] = 1.0
    return row


def masks_to_vec(d, s, length=64):
    return np.array([0 if not (d >> e) & 1 else (-1 if (s >> e) & 1 else 1) for e in range(length)])
