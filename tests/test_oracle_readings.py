"""Pins of the oracle's walk and Resize steps against an independent numpy
restatement of the readings (tests/np_reading.py), predicted from the Philox
words alone.

Stepping oracle walks one iteration at a time, every iteration's current and
best scheme, best rank, plateau start, records and counters must equal the
prediction.  This pins what the paper leaves open and the earlier pins did
not reach: the order and slot placement of the reduction cascade (reduction
operator of Sec. 3.3.1, reduce() of Algorithm 1), the zero-term removal, the
exact plateau-restart iteration (t - plateau_start >= plateau), the restart
source, and the dead-end path.  The Resize step (Algorithm 2, Sec. 3.4.3) is
predicted in the same way: the swap, the merge partner and its axis order,
and the 5/50/30/15 % choice of project / product / double / extend."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import np_reading as R
from tests.golden_io import load_formula_scheme


def _F(s):
    d = O.from_c(s)
    return [d["U"].astype(np.int64), d["V"].astype(np.int64), d["W"].astype(np.int64)]


def _same(F, G):
    return all(a.shape == b.shape and np.array_equal(a, b) for a, b in zip(F, G))


def _strassen():
    return O.normalise(O.to_c(*load_formula_scheme("strassen_formulas.txt")[3:], 2, 2, 2))


# (format, z2, params): plateau short enough for many restarts in the window
WALKS = [
    ((3, 3, 3), False, dict(plateau=150)),
    ((3, 3, 3), False, dict(plateau=90, restart_from_best=1)),
    ((2, 2, 3), False, dict(plateau=300, t_expand=int(0.2 * 2 ** 32))),
    ((2, 3, 3), False, dict(plateau=400, t_expand=int(0.05 * 2 ** 32), flip_tries=2)),
    ((3, 3, 3), True, dict(plateau=200)),
    # from Strassen's scheme, which has no flip: dead ends and their expands
    ("strassen", False, dict(plateau=10 ** 6, r_cap=10)),
]


@pytest.mark.parametrize("fmt,z2,extra", WALKS)
def test_walk_iterations_follow_the_readings(fmt, z2, extra):
    if fmt == "strassen":
        m, n, p = 2, 2, 2
        start = _strassen()
    else:
        m, n, p = fmt
        start = O.standard(m, n, p, z2)
    r0 = start.r
    prm = dict(flip_tries=7, t_eq=42949673, t_reduce=1 << 32, t_expand=0, plateau=150,
               restart_from_best=0, r_cap=r0 + 8)
    prm.update(extra)
    events = dict(restarts=0, cascades=0, moved_merges=0, dead_ends=0, zero_removed=0,
                  expands=0, fallbacks=0)
    for seed in (11, 12):
        cp = O.make_params(seed=seed, max_iters=10 ** 6, plateau=prm["plateau"], target_rank=0,
                           r_cap=prm["r_cap"], flip_tries=prm["flip_tries"],
                           restart_from_best=prm["restart_from_best"], t_eq=prm["t_eq"],
                           t_reduce=prm["t_reduce"], t_expand=prm["t_expand"])
        w = O.new_walk(start)
        nw = R.Walk(_F(w.start), z2)
        key = (seed & R.M32, seed >> 32)
        last_reset = 0
        for _ in range(1200):
            c0 = O.counters(w)
            O.run(w, cp, 1)
            nw.iteration(O.philox, key, prm)
            c1 = O.counters(w)
            d = {k: c1[k] - c0[k] for k in c1}
            t = w.t
            assert t == nw.t
            assert _same(_F(w.cur), nw.cur), (fmt, seed, t)
            assert w.best_rank == nw.best_rank and _same(_F(w.best), nw.best), (fmt, seed, t)
            assert w.plateau_start == nw.plateau_start, (fmt, seed, t)
            for k in nw.c:
                assert c1[k] == nw.c[k], (fmt, seed, t, k)
            # the restart fires exactly `plateau` iterations after the last
            # strict improvement or restart, never earlier or later
            if d["improvements"]:
                last_reset = t
            if d["restarts"]:
                assert t - last_reset == prm["plateau"], (fmt, seed, t)
                last_reset = t
                events["restarts"] += 1
            else:
                assert t - last_reset < prm["plateau"]
            events["cascades"] += d["merges"] >= 2
            for k in ("dead_ends", "zero_removed", "expands", "fallbacks"):
                events[k] += d[k]
        assert O.records(w) == nw.records
        assert O.brent_violations(w.cur) == 0 and O.brent_violations(w.best) == 0
    # the window reaches the steps these readings are about
    if prm["plateau"] < 10 ** 6:
        assert events["restarts"] >= 2, events
    if fmt == "strassen":
        assert events["dead_ends"] >= 5 and events["expands"] >= 5, events
    if fmt == (2, 2, 3):
        assert events["cascades"] >= 1 and events["expands"] >= 20, events


def _walked(fmt, seed, iters, z2=False):
    m, n, p = fmt
    prm = O.make_params(seed=seed, max_iters=iters, plateau=10 ** 6, target_rank=0,
                        r0=m * n * p, t_expand=1 << 28)
    w = O.new_walk(O.standard(m, n, p, z2))
    O.run(w, prm, iters)
    return O.copy(w.cur)


def _resize_cases():
    """(scheme, best list, cap): partners that never merge with the scheme
    (so Algorithm 2's operator choice runs every time), partners that do
    merge, along p or only along m, and a tight capacity."""
    small = [O.standard(1, 1, 2), O.standard(1, 1, 1), O.standard(1, 2, 1)]
    mergeable = [_strassen(), _walked((2, 2, 3), 5, 300), _walked((3, 2, 2), 6, 300)]
    cases = []
    for seed in range(160):
        fmt = [(2, 2, 3), (2, 3, 2), (3, 2, 2), (2, 2, 2)][seed % 4]
        s = _walked(fmt, seed, 40 + seed % 50)
        if seed % 3 == 2:
            cases.append((s, mergeable, 512, seed))
        elif seed % 7 == 5:
            cases.append((s, small, s.r + 1, seed))
        else:
            cases.append((s, small, 512, seed))
    z2 = [O.standard(1, 1, 2, True), O.standard(2, 1, 1, True)]
    for seed in range(24):
        cases.append((_walked((2, 2, 3), seed, 60, z2=True), z2, 512, 1000 + seed))
    return cases


def test_resize_follows_algorithm_2():
    """Every Resize result (operators applied, format, and every coefficient in
    term order) equals the numpy prediction from blocks (round, 0, 3) and
    (round, 1, 3); the run covers every operator, the merge along p and
    along m, refusals past the capacity, and draws that fall between the
    50 % and 55 % points (product, not double)."""
    seen = {}
    near = 0
    for s, best, cap, seed in _resize_cases():
        for rnd in (1, 2, 7):
            bits, t = O.resize(s, best, seed, rnd, 1 << 32, cap)
            z2 = bool(s.z2)
            pb = [(_F(b), (b.m, b.n, b.p)) for b in best]
            pbits, F, dims = R.resize(_F(s), (s.m, s.n, s.p), pb, O.philox, (seed & R.M32, seed >> 32),
                                      rnd, 1 << 32, cap, z2)
            assert bits == pbits, (seed, rnd)
            assert (t.m, t.n, t.p) == dims and _same(_F(t), F), (seed, rnd, bits)
            assert O.brent_violations(t) == 0
            for b in range(6):
                if bits >> b & 1:
                    seen[b] = seen.get(b, 0) + 1
            q = O.philox((rnd, 0, 0, 3), (seed & R.M32, seed >> 32))[3]
            if not bits & 2 and R.T_PRODUCT - int(0.05 * 2 ** 32) <= q < R.T_PRODUCT:
                near += 1
    assert all(seen.get(b, 0) >= 3 for b in range(6)), seen
    assert near >= 5, near


def test_resize_merge_axis_order():
    """A partner that merges along p and along m: Algorithm 2's merge is taken
    along p first; a partner that merges only along m is merged along m."""
    a = O.standard(2, 2, 2)
    for seed in range(200):
        b0 = O.philox((1, 0, 0, 3), (seed, 0))
        if b0[0] >= 2 ** 31:  # no swap, so the format stays (2,2,2)
            bits, t = O.resize(a, [O.standard(2, 2, 2)], seed, 1, 0, 512)
            assert bits == 2 and (t.m, t.n, t.p) == (2, 2, 4)
            bits, t = O.resize(a, [O.standard(1, 2, 2)], seed, 1, 0, 512)
            assert bits == 2 and (t.m, t.n, t.p) == (3, 2, 2)
            return
    pytest.fail("no round without a swap")
