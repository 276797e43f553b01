"""tsf_population_best_noalloc (the population synchronisation with the
library's fixed working memory, for callers that cannot allocate) against
tsf_population_best with a caller workspace: identical tables and counts,
bit for bit, on consecutive calls whose inputs shrink, so that a call finds
the previous call's contents in the fixed array."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2511_20317_amd import tsf

pytestmark = pytest.mark.gpu


def _walked(fmt, seed, iters):
    m, n, p = fmt
    prm = O.make_params(seed=seed, max_iters=iters, plateau=iters, target_rank=0, r0=m * n * p)
    w = O.new_walk(O.standard(m, n, p))
    O.run(w, prm, iters)
    d = O.from_c(w.best)
    return tsf.Scheme(m, n, p, d["U"], d["V"], d["W"])


def _batch(ctx, schemes, cap=96):
    b = tsf.WalkBatch([(s, 1, s.rank, 0) for s in schemes], capacity=cap, rec_cap=4)
    b.max_len = 64
    b.init(ctx)
    return b


def _entries(table, count):
    n = int(count.item())
    return n, table.cpu().numpy().view(tsf.BEST_ENTRY_DTYPE)[:n].tobytes()


def _oracle_table(schemes):
    best = {}
    for w, s in enumerate(schemes):
        key = (s.m, s.n, s.p)
        if key not in best or s.rank < best[key][0]:
            best[key] = (s.rank, w)
    return [(k, best[k][0], best[k][1]) for k in sorted(best)]


def _as_list(table, count):
    n = int(count.item())
    ent = table.cpu().numpy().view(tsf.BEST_ENTRY_DTYPE)[:n]
    return [((int(e["m"]), int(e["n"]), int(e["p"])), int(e["rank"]), int(e["walk"])) for e in ent]


def test_noalloc_population_best_equals_the_workspace_version():
    import torch
    assert torch.cuda.is_available()
    ctx = tsf.Context()
    dev = torch.device("cuda")
    fmts = [(2, 2, 2), (2, 2, 3), (2, 3, 2), (1, 2, 2), (2, 2, 4), (3, 2, 2), (2, 3, 3)]
    big = [_walked(fmts[k % len(fmts)], k, 150 + 29 * k) for k in range(112)]
    small = [_walked(fmts[k % 3], 1000 + k, 120 + 17 * k) for k in range(20)]
    for schemes, slots in ((big, 4096), (small, 16)):
        b = _batch(ctx, schemes)
        want_t, want_c = b.population_best(slots)
        table = torch.full((slots * tsf.BEST_ENTRY_DTYPE.itemsize,), 0xAB, dtype=torch.uint8,
                           device=dev)
        count = torch.full((1,), -7, dtype=torch.int32, device=dev)
        dropped = torch.full((1,), -7, dtype=torch.int32, device=dev)
        b.population_best_noalloc(table, count, slots, dropped)
        torch.cuda.synchronize()
        assert _entries(table, count) == _entries(want_t, want_c)
        assert _as_list(table, count) == _oracle_table(schemes)
        assert int(dropped.item()) == 0
    # more formats than slots: three formats of four walks each in two slots
    # drop one format's four walks, whichever two formats took the slots
    three = [_walked(fmts[k % 3], 2000 + k, 100 + 11 * k) for k in range(12)]
    b = _batch(ctx, three)
    table = torch.zeros(2 * tsf.BEST_ENTRY_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    dropped = torch.zeros(1, dtype=torch.int32, device=dev)
    b.population_best_noalloc(table, count, 2, dropped)
    torch.cuda.synchronize()
    assert int(count.item()) == 2 and int(dropped.item()) == 4
    full = dict((k, (r, w)) for k, r, w in _oracle_table(three))
    got = _as_list(table, count)
    assert got == sorted(got) and all(full[k] == (r, w) for k, r, w in got)
    with pytest.raises(tsf.TsfError):
        b.population_best_noalloc(table, count, 4097, dropped)
