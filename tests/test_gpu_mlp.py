"""The proposal network's MFMA kernels (tsf_mlp_*) against the fp64 oracle
(oracle/mlp.py).

Tolerances follow from the arithmetic: operands are bf16 (unit roundoff
u = 2^-8 relative to the value), sums are accumulated in fp32, and the GPU
rounds h1, h2 and the backpropagated deltas to bf16 where the oracle keeps
fp64 deltas.  An output whose sum has L1 mass S (sum of |products|) can
therefore differ by about u * S per rounding it passes through; the tests
allow 2^-6 * S for a quantity one rounding away and 2^-5 * S two roundings
away (4x and 8x the unit roundoff), plus 1e-6 absolute."""
import numpy as np
import pytest

from oracle import mlp as ref
from paper_2511_20317_amd import tsf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _problem(seed, M):
    rng = np.random.default_rng(seed)
    p = ref.init_params(seed)
    p["b1"] = rng.standard_normal(ref.D_H) * 0.1
    p["b2"] = rng.standard_normal(ref.D_H) * 0.1
    p["b3"] = rng.standard_normal(1) * 0.1
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    X = (rng.integers(-1, 2, (M, ref.D_IN)) * (rng.random((M, ref.D_IN)) < 0.06)).astype(np.float64)
    X[:, 400 + rng.integers(0, 16, M)] = 1.0     # a format slot
    y = (rng.random(M) < 0.3).astype(np.float64)
    return p, X, y


def _net(torch, p):
    net = tsf.Mlp()
    net.set_params(p["W1"], p["b1"], p["W2"], p["b2"], p["w3"], p["b3"])
    return net


@pytest.mark.parametrize("M", [1, 64, 300, 4096])
def test_forward_matches_oracle(torch, M):
    p, X, _ = _problem(M, M)
    net = _net(torch, p)
    Xd = torch.from_numpy(tsf.bf16_bits(X)).cuda()
    h1, h2, logit = net.forward(Xd)
    torch.cuda.synchronize()
    f = ref.forward(p, X)
    g_h1 = tsf.bf16_to_float(h1.cpu().numpy())
    g_h2 = tsf.bf16_to_float(h2.cpu().numpy())
    g_lg = logit.cpu().numpy().astype(np.float64)
    assert (np.abs(g_h1 - f["h1"]) <= 2 ** -6 * f["m1"] + 1e-6).all()
    m2 = np.abs(f["h1"]) @ np.abs(ref.bf16_round(p["W2"])) + np.abs(p["b2"])
    assert (np.abs(g_h2 - f["h2"]) <= 2 ** -5 * (m2 + f["m1"].max()) + 1e-6).all()
    assert (np.abs(g_lg - f["logit"]) <= 2 ** -5 * (f["m3"] + 1) + 1e-6).all()
    # ReLU pattern: units far from zero agree exactly
    far = np.abs(f["z1"]) > 2 ** -5 * f["m1"]
    assert np.array_equal(g_h1[far] > 0, f["h1"][far] > 0)


@pytest.mark.parametrize("M", [64, 777, 4096])
def test_backward_matches_oracle(torch, M):
    p, X, y = _problem(100 + M, M)
    net = _net(torch, p)
    Xd = torch.from_numpy(tsf.bf16_bits(X)).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    h1, h2, logit = net.forward(Xd)
    loss = net.backward(Xd, yd, h1, h2, logit)
    torch.cuda.synchronize()
    g, f = ref.backward(p, X, y)
    gg = net.unpack(net.grad.cpu().numpy())
    assert abs(float(loss.item()) - ref.loss(p, X, y)) <= 1e-3 * (1 + ref.loss(p, X, y))
    # L1 masses of the gradient sums
    d3 = (1.0 / (1.0 + np.exp(-f["logit"])) - y) / M
    w3 = ref.bf16_round(p["w3"])
    d2 = np.outer(d3, w3) * (f["z2"] > 0)
    d1 = (d2 @ ref.bf16_round(p["W2"]).T) * (f["z1"] > 0)
    ad2 = np.abs(np.outer(d3, w3))
    ad1 = ad2 @ np.abs(ref.bf16_round(p["W2"])).T
    mass = {"w3": np.abs(f["h2"]).T @ np.abs(d3), "b3": np.array([np.abs(d3).sum()]),
            "W2": np.abs(f["h1"]).T @ ad2, "b2": ad2.sum(axis=0),
            "W1": np.abs(X).T @ ad1, "b1": ad1.sum(axis=0)}
    for k in ("w3", "b3", "W2", "b2", "W1", "b1"):
        err = np.abs(gg[k] - g[k])
        bound = 2 ** -5 * mass[k] + 2 ** -5 * np.abs(g[k]) + 1e-6
        assert (err <= bound).all(), (k, float(err.max()), float((err - bound).max()))
    del d1


def test_adam_step_matches_oracle(torch):
    p, X, y = _problem(7, 512)
    net = _net(torch, p)
    Xd = torch.from_numpy(tsf.bf16_bits(X)).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    st = {}
    q = dict(p)
    for step in range(3):
        h1, h2, logit = net.forward(Xd)
        net.backward(Xd, yd, h1, h2, logit)
        gg = net.unpack(net.grad.cpu().numpy())
        net.step(lr=1e-3)
        torch.cuda.synchronize()
        q = ref.adam(q, gg, st, lr=1e-3)   # the same gradients through the fp64 optimiser
        got = net.unpack(net.param.cpu().numpy())
        for k in q:
            assert np.allclose(got[k], q[k], rtol=1e-5, atol=1e-6), (step, k)


def test_training_learns_a_separable_rule(torch):
    """y = 1 iff feature 3 is non-zero: the loss must fall well below log 2."""
    rng = np.random.default_rng(11)
    M = 4096
    X = (rng.integers(-1, 2, (M, ref.D_IN)) * (rng.random((M, ref.D_IN)) < 0.05)).astype(np.float64)
    y = (X[:, 3] != 0).astype(np.float64)
    net = _net(torch, ref.init_params(11))
    Xd = torch.from_numpy(tsf.bf16_bits(X)).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    first = None
    for _ in range(200):
        h1, h2, logit = net.forward(Xd)
        loss = net.backward(Xd, yd, h1, h2, logit)
        if first is None:
            first = float(loss.item())
        net.step(lr=3e-3)
    torch.cuda.synchronize()
    h1, h2, logit = net.forward(Xd)
    acc = float(((logit.cpu().numpy() > 0) == (y > 0.5)).mean())
    assert acc > 0.97 and first > 0.3
