"""Pins of the fp64 proposal-network oracle (oracle/mlp.py): bf16 rounding
against torch's conversion, analytic gradients against central finite
differences, the linear region against plain matrix products, and Adam's
first step against its closed form."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 3.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0           # tie to even
    assert mlp.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def _small_problem(seed, M=12):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    p["b1"] = rng.standard_normal(mlp.D_H) * 0.1
    p["b2"] = rng.standard_normal(mlp.D_H) * 0.1
    p["b3"] = rng.standard_normal(1) * 0.1
    X = rng.integers(-1, 2, (M, mlp.D_IN)).astype(np.float64) * (rng.random((M, mlp.D_IN)) < 0.05)
    y = (rng.random(M) < 0.3).astype(np.float64)
    return p, X, y


def test_gradients_match_finite_differences():
    p, X, y = _small_problem(1)
    g, _ = mlp.backward(p, X, y, rounding=False)
    rng = np.random.default_rng(2)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, min(12, flat.size), replace=False):
            keep = flat[idx]
            flat[idx] = keep + h
            lp = mlp.loss(p, X, y, rounding=False)
            flat[idx] = keep - h
            lm = mlp.loss(p, X, y, rounding=False)
            flat[idx] = keep
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-4 * abs(fd), (k, idx, fd, an)


def test_linear_region_is_a_matrix_product():
    p, X, _ = _small_problem(3, M=5)
    p["b1"][:] = 1e3  # every unit active: relu is the identity
    p["b2"][:] = 1e5
    f = mlp.forward(p, X, rounding=False)
    want = ((X @ p["W1"] + p["b1"]) @ p["W2"] + p["b2"]) @ p["w3"] + p["b3"][0]
    assert np.allclose(f["logit"], want, rtol=1e-12, atol=1e-9)


def test_adam_first_step_closed_form():
    p, X, y = _small_problem(4)
    g, _ = mlp.backward(p, X, y)
    st = {}
    q = mlp.adam(p, g, st, lr=1e-2)
    for k in p:
        step = q[k] - p[k]
        want = -1e-2 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(step, want, rtol=1e-6, atol=1e-12)
