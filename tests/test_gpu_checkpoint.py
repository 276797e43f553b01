"""A batch saved to a checkpoint mid-walk, read back (with the GPU Brent check
of every scheme) and walked on ends bit-identical to the batch that was never
interrupted."""
import numpy as np
import pytest

from paper_2511_20317_amd import tsf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tsf.Context()


@pytest.mark.parametrize("fmt,n,r_cap,cap,first,then", [
    ((3, 3, 3), 1024, 35, None, 700, 900),
    ((6, 7, 9), 64, 386, 386, 100, 150),
])
def test_checkpoint_resume_is_bit_exact(ctx, tmp_path, fmt, n, r_cap, cap, first, then):
    import torch
    groups = [(tsf.init_scheme(*fmt), n, r_cap, 0)]
    prm = tsf.walk_params(base_seed=9, max_iters=10 ** 6, plateau=500)
    a = tsf.WalkBatch(groups, capacity=cap, rec_cap=16)
    a.init(ctx)
    a.walk(ctx, prm, first)
    path = str(tmp_path / "ck.npz")
    a.save(path, prm)
    b = tsf.WalkBatch.load(path, prm=prm)
    a.walk(ctx, prm, then)
    b.walk(ctx, prm, then)
    torch.cuda.synchronize()
    ha, hb = a.headers(), b.headers()
    assert (ha["t"] == first + then).all()
    assert np.array_equal(ha, hb)
    for k in ("cur", "best", "rec"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
