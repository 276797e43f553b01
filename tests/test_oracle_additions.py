"""Pins of the oracle's additions objective (the complexity-minimisation mode
of Sec. 3.9, scored by the naive additions of Sec. 4.5): the metric against
counts made here with numpy and the paper's worked example, and every step of
a walk against what the mode must preserve -- the rank, the matmul tensor,
non-zero factors -- and against a best-scheme rule recomputed from the
trajectory."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests.golden_io import load_formula_scheme, load_scheme, matmul_tensor, scheme_tensor


def _nnz(d):
    return int(np.count_nonzero(d["U"]) + np.count_nonzero(d["V"]) + np.count_nonzero(d["W"]))


def _rank_walk_best(fmt, target, seed=2, iters=100000):
    m, n, p = fmt
    prm = O.make_params(seed=seed, max_iters=iters, plateau=20000, target_rank=target,
                        r0=m * n * p)
    w = O.new_walk(O.standard(m, n, p))
    O.run(w, prm, iters)
    assert w.best_rank == target
    return O.copy(w.best)


def test_nonzeros_and_additions_against_numpy():
    strassen = O.normalise(O.to_c(*load_formula_scheme("strassen_formulas.txt")[3:], 2, 2, 2))
    assert O.nonzeros(strassen) == 36 and O.naive_additions(strassen) == 18
    ex = O.to_c(*load_scheme("paper_2x2x3_rank11.txt")[3:], 2, 2, 3)
    assert O.naive_additions(ex) == 20                       # the example of Sec. 3.1.1
    for fmt in [(2, 2, 2), (2, 3, 4), (3, 3, 3)]:
        s = O.standard(*fmt)
        m, n, p = fmt
        assert O.nonzeros(s) == 3 * m * n * p
        assert O.naive_additions(s) == m * p * (n - 1)
    s = _rank_walk_best((2, 2, 3), 11)
    d = O.from_c(s)
    assert O.nonzeros(s) == _nnz(d)
    assert O.naive_additions(s) == _nnz(d) - 2 * s.r - 2 * 3


@pytest.mark.parametrize("fmt,target,z2", [((2, 2, 3), 11, False), ((2, 3, 3), 18, False),
                                           ((2, 2, 3), 11, True)])
def test_additions_walk_step_by_step(fmt, target, z2):
    """Every iteration keeps the rank and the matmul tensor, leaves no zero
    factor, changes at most two terms; the best scheme always has the fewest
    non-zeros seen since the walk began (strictly fewer replaces it, equal
    may), and each strict improvement is recorded with its naive additions."""
    m, n, p = fmt
    if z2:
        prm = O.make_params(seed=4, max_iters=100000, plateau=20000, target_rank=target,
                            r0=m * n * p)
        w = O.new_walk(O.standard(m, n, p, z2=True))
        O.run(w, prm, 100000)
        start = O.copy(w.best)
    else:
        start = _rank_walk_best(fmt, target)
    r = start.r
    T = matmul_tensor(m, n, p)
    prm = O.make_params(seed=7, max_iters=3000, plateau=0, target_rank=0, r0=r, objective=1)
    w = O.new_walk(start)
    prev = O.from_c(w.cur)
    lowest = _nnz(prev)
    rec_seen = 0
    for t in range(1, 3001):
        O.run(w, prm, 1)
        cur = O.from_c(w.cur)
        assert w.cur.r == r and w.best.r == r
        if z2:
            assert O.brent_violations(w.cur) == 0
        else:
            assert np.array_equal(scheme_tensor(cur["U"], cur["V"], cur["W"]), T)
        for X in "UVW":
            assert (np.abs(cur[X]).sum(axis=1) > 0).all()
        changed = [l for l in range(r)
                   if any(not np.array_equal(cur[X][l], prev[X][l]) for X in "UVW")]
        assert len(changed) in (0, 2)
        nnz = _nnz(cur)
        if nnz < lowest:
            lowest = nnz
            recs = O.records(w)
            assert len(recs) == rec_seen + 1 and recs[-1] == (t, nnz - 2 * r - m * p)
            rec_seen += 1
        assert w.best_nnz == lowest == _nnz(O.from_c(w.best))
        prev = cur
    assert w.c.flips > 0 and w.c.merges == 0 and w.c.expands == 0 and w.c.zero_removed == 0
    adds = [a for _, a in O.records(w)]
    assert all(b < a for a, b in zip(adds, adds[1:]))


def test_additions_walk_from_the_paper_example_never_worse():
    """From the (2,2,3:11) scheme of Sec. 3.1.1 (20 naive additions) the best
    scheme never has more additions, and restarts return to it."""
    ex = O.normalise(O.to_c(*load_scheme("paper_2x2x3_rank11.txt")[3:], 2, 2, 3))
    prm = O.make_params(seed=1, max_iters=20000, plateau=3000, target_rank=0, r0=11, objective=1)
    ws = O.run_many(ex, prm, 1, 0, 16, 20000, 8)
    for w in ws:
        assert O.naive_additions(w.best) <= 20
        assert w.best.r == 11 and O.brent_violations(w.best) == 0 and O.is_normalised(w.best)
        assert w.c.restarts > 0


def test_additions_stop_rule_and_improvement():
    start = _rank_walk_best((2, 2, 3), 11)
    a0 = O.naive_additions(start)
    prm = O.make_params(seed=0, max_iters=20000, plateau=5000, target_rank=a0 - 6, r0=11,
                        objective=1)
    ws = O.run_many(start, prm, 0, 0, 16, 20000, 8)
    hit = [w for w in ws if w.done]
    assert hit, "no walk reached %d additions" % (a0 - 6)
    for w in hit:
        assert O.naive_additions(w.best) <= a0 - 6
        assert O.records(w)[-1] == (w.t, O.naive_additions(w.best))
