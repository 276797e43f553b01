"""The GPU isotropy-invariant kernel (tsf_invariants_batch) against the exact
oracle (oracle/invariants.py) on schemes found by oracle walks, loaded as the
start schemes of a batch: every factor rank and every rank sum."""
import numpy as np
import pytest

from oracle import invariants as I
from oracle import pyoracle as O
from paper_2511_20317_amd import tsf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tsf.Context()


def _oracle_schemes(fmt, n, z2=False, iters=20000):
    m, n_, p = fmt
    prm = O.make_params(seed=5, max_iters=iters, plateau=8000, target_rank=0,
                        r0=m * n_ * p, t_expand=1 << 29)
    ws = O.run_many(O.standard(m, n_, p, z2=z2), prm, 5, 0, n, iters, 8)
    out = []
    for w in ws:
        d = O.from_c(w.cur)
        out.append(tsf.Scheme(m, n_, p, d["U"], d["V"], d["W"],
                              tsf.TSF_Z2 if z2 else tsf.TSF_TERNARY))
    return out


@pytest.mark.parametrize("z2", [False, True])
def test_invariants_batch_matches_oracle(ctx, z2):
    import torch
    fmts = [(2, 2, 3), (3, 3, 3), (2, 4, 5), (4, 4, 4), (4, 5, 12)]
    schemes = []
    for f in fmts:
        schemes += [(f, s) for s in _oracle_schemes(f, 6, z2, iters=20000 if f != (4, 5, 12) else 300)]
    groups = [(s, 1, s.rank, 0) for _, s in schemes]
    b = tsf.WalkBatch(groups, rec_cap=4)
    b.init(ctx)
    ranks, sums = b.invariants(which=2)
    torch.cuda.synchronize()
    ranks, sums = ranks.cpu().numpy(), sums.cpu().numpy()
    for w, (f, s) in enumerate(schemes):
        U, V, W = s.live()
        rk = I.term_ranks({"U": U, "V": V, "W": W}, *f, z2=z2)
        assert [tuple(int(x) for x in r) for r in ranks[w, :s.rank]] == rk, (w, f)
        assert tuple(sums[w]) == tuple(sum(t[k] for t in rk) for k in range(3))


def test_invariants_batch_after_walks_equal_host(ctx):
    """On the current schemes of GPU walks: the GPU kernel against the host
    routine (the same elimination, compiled for the CPU)."""
    import torch
    b = tsf.WalkBatch([(tsf.init_scheme(3, 3, 3), 256, 35, 23)], rec_cap=4)
    b.init(ctx)
    b.walk(ctx, tsf.walk_params(base_seed=4, max_iters=3000), 3000)
    ranks, sums = b.invariants(which=0)
    torch.cuda.synchronize()
    hdr = b.headers()
    for w in range(0, 256, 17):
        host = tsf.scheme_invariants(b.scheme(w, "cur", hdr))
        assert [tuple(int(x) for x in r) for r in ranks[w, :hdr["rank"][w]].cpu().numpy()] == \
            host["term_ranks"]
        assert tuple(int(x) for x in sums[w].cpu().numpy()) == host["rank_sum"]
