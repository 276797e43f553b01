"""Degenerate and boundary cases of the walk against the oracle: a rank-1
scheme (no flip exists, expand needs two terms: every iteration is a dead
end), formats with a dimension 1, the indexed kernel at its 64-term limit
with no room to expand, Z2 at rank 1; and calls that do nothing (no
iterations, an empty batch, a walk already at its target)."""
import numpy as np
import pytest

from paper_2511_20317_amd import tsf
from tests.gpu_parity import compare, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tsf.Context()


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("fmt,mode,r_cap", [
    ((1, 1, 1), tsf.TSF_TERNARY, 9),
    ((1, 1, 1), tsf.TSF_Z2, 9),
    ((1, 2, 2), tsf.TSF_TERNARY, 12),
    ((2, 1, 3), tsf.TSF_TERNARY, 14),
    ((1, 1, 6), tsf.TSF_Z2, 14),
    ((4, 4, 4), tsf.TSF_TERNARY, 64),
])
def test_degenerate_and_boundary_formats(ctx, fmt, mode, r_cap):
    groups = [(tsf.init_scheme(*fmt, mode=mode), 64, r_cap, 0)]
    prm = tsf.walk_params(base_seed=31, max_iters=3000, plateau=700, t_expand=1 << 28)
    b = tsf.WalkBatch(groups, rec_cap=16)
    b.init(ctx)
    b.walk(ctx, prm, 600)
    b.walk(ctx, prm, 900)
    _sync()
    walks = list(range(0, 64, 9))
    compare(b, run_oracle(groups, prm, walks, 1500), "%s mode %d" % (fmt, mode))
    h = b.headers()
    assert (h["t"] == 1500).all()
    if fmt == (1, 1, 1):
        # no flip and no expand at rank 1: every iteration is a dead end
        assert (h["counters"][:, tsf.COUNTER_NAMES.index("dead_ends")] == 1500).all()
        assert (h["rank"] == 1).all()
    assert (b.verify_device(0).cpu().numpy() == 0).all()


def test_calls_that_do_nothing(ctx):
    s = tsf.init_scheme(3, 3, 3)
    prm = tsf.walk_params(base_seed=2, max_iters=1000, plateau=500)
    b = tsf.WalkBatch([(s, 32, 35, 23)], rec_cap=4)
    b.init(ctx)
    b.walk(ctx, prm, 100)
    _sync()
    h0 = b.headers()
    cur0 = b.cur.cpu().numpy().copy()
    b.walk(ctx, prm, 0)
    _sync()
    assert np.array_equal(b.headers(), h0) and np.array_equal(b.cur.cpu().numpy(), cur0)
    # an empty batch
    e = tsf.WalkBatch.empty(0, 35, tsf.TSF_TERNARY, max_len=9, rec_cap=4)
    e.walk(ctx, prm, 100)
    # a walk whose target is its start rank stops before its first iteration
    t = tsf.WalkBatch([(s, 8, 35, 27)], rec_cap=4)
    t.init(ctx)
    t.walk(ctx, prm, 100)
    _sync()
    h = t.headers()
    assert (h["done"] == 1).all() and (h["t"] == 0).all() and (h["best_rank"] == 27).all()
    # a walk at max_iters is not advanced
    b.walk(ctx, prm, 2000)
    _sync()
    assert (b.headers()["t"] == 1000).all()
    b.walk(ctx, prm, 10)
    _sync()
    assert (b.headers()["t"] == 1000).all()


def test_a_batch_per_format_equals_one_batch_of_all(ctx):
    """Walks split into a batch per format (walk ids continued with
    first_walk_id, each batch sized for its own ranks) end bit-identical to
    the same walks in one batch of all formats (the large-format workload
    runs this way)."""
    import torch
    fmts = [((4, 5, 12), 248), ((5, 6, 10), 308)]
    per = 48
    prm = tsf.walk_params(base_seed=4, max_iters=10 ** 6, plateau=300, t_expand=1 << 28)
    one = tsf.WalkBatch([(tsf.init_scheme(*f), per, cap, 0) for f, cap in fmts], capacity=308,
                        rec_cap=8)
    one.init(ctx)
    one.walk(ctx, prm, 400, 64, 1, 2)
    _sync()
    h1 = one.headers()
    for q, (f, cap) in enumerate(fmts):
        p = tsf.walk_params(base_seed=4, first_walk_id=q * per, max_iters=10 ** 6, plateau=300,
                            t_expand=1 << 28)
        b = tsf.WalkBatch([(tsf.init_scheme(*f), per, cap, 0)], capacity=cap, rec_cap=8)
        b.init(ctx)
        b.walk(ctx, p, 400, 64, 1, 2)
        _sync()
        h = b.headers()
        sl = slice(q * per, (q + 1) * per)
        for k in ("rank", "best_rank", "t", "plateau_start", "n_rec", "best_nnz", "counters"):
            assert np.array_equal(h[k], h1[k][sl]), (f, k)
        assert torch.equal(b.cur[:, :cap], one.cur[sl, :cap]) and torch.equal(b.best[:, :cap],
                                                                             one.best[sl, :cap])
        assert torch.equal(b.rec, one.rec[sl])
