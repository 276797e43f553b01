"""Pins of the oracle's meta operators for the Resize kernel (Sec. 3.3.2,
Algorithm 2): every result satisfies the Brent equations of its format (the
verifier is pinned by the paper's example and Strassen), merges and products
of standard schemes are the standard schemes of the result, swapping twice
is the identity, Strassen (x) Strassen is a (4,4,4:49) scheme, and a resize
step changes format and rank exactly as the operators it reports."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests.golden_io import load_formula_scheme, load_scheme


def _terms(s):
    d = O.from_c(s)
    return sorted(tuple(d["U"][l]) + tuple(d["V"][l]) + tuple(d["W"][l]) for l in range(s.r))


def _strassen():
    return O.normalise(O.to_c(*load_formula_scheme("strassen_formulas.txt")[3:], 2, 2, 2))


def _walked(fmt, seed=1, iters=20000):
    m, n, p = fmt
    prm = O.make_params(seed=seed, max_iters=iters, plateau=8000, target_rank=0, r0=m * n * p,
                        t_expand=1 << 28)
    w = O.new_walk(O.standard(m, n, p))
    O.run(w, prm, iters)
    return O.copy(w.cur)


def test_swap_sizes_valid_and_an_involution():
    ex = O.normalise(O.to_c(*load_scheme("paper_2x2x3_rank11.txt")[3:], 2, 2, 3))
    for s in (_strassen(), ex, _walked((2, 3, 4)), _walked((3, 3, 4))):
        t = O.swap_sizes(s)
        assert (t.m, t.n, t.p, t.r) == (s.m, s.p, s.n, s.r)
        assert O.brent_violations(t) == 0 and O.is_normalised(t)
        assert _terms(O.swap_sizes(t)) == _terms(s)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_merge_of_standard_schemes_is_standard(axis):
    a, b = O.standard(2, 3, 2), O.standard(2, 3, 2)
    dims = [2, 3, 2]
    dims[axis] *= 2
    got = O.merge(a, b, axis)
    assert _terms(got) == _terms(O.standard(*dims))
    # unequal sizes along the merge axis
    sizes = [[2, 3, 4], [2, 3, 4]]
    sizes[1][axis] = 1
    got = O.merge(O.standard(*sizes[0]), O.standard(*sizes[1]), axis)
    want = list(sizes[0])
    want[axis] += 1
    assert _terms(got) == _terms(O.standard(*want))


def test_merge_of_walked_schemes_valid_and_refused_when_incompatible():
    a, b = _walked((2, 3, 3)), _walked((2, 3, 2), seed=2)
    got = O.merge(a, b, 2)
    assert (got.m, got.n, got.p, got.r) == (2, 3, 5, a.r + b.r)
    assert O.brent_violations(got) == 0
    assert O.merge(a, b, 0) is None and O.merge(a, b, 1) is None
    assert O.brent_violations(O.merge(_strassen(), _strassen(), 2)) == 0


def test_product_strassen_squared_and_standard():
    s2 = O.product(_strassen(), _strassen())
    assert (s2.m, s2.n, s2.p, s2.r) == (4, 4, 4, 49)
    assert O.brent_violations(s2) == 0 and O.is_normalised(s2)
    assert _terms(O.product(O.standard(2, 1, 3), O.standard(1, 2, 2))) == _terms(O.standard(2, 2, 6))
    one = O.standard(1, 1, 1)
    w = _walked((2, 2, 3))
    assert _terms(O.product(w, one)) == _terms(w)
    assert O.brent_violations(O.product(_walked((2, 2, 2)), _walked((1, 2, 2)))) == 0
    assert O.product(O.standard(4, 4, 4), O.standard(2, 2, 3)) is None  # 96-entry factors


def test_resize_steps_follow_their_operators():
    best = [_strassen(), _walked((2, 2, 3)), _walked((2, 3, 2), seed=3), O.standard(1, 2, 2)]
    seen = 0
    for seed in range(200):
        s = _walked((2, 2, 3), seed=seed % 7, iters=500)
        bits, t = O.resize(s, best, seed, 1, 1 << 32, 128)
        assert bits >= 0
        seen |= bits
        assert O.brent_violations(t) == 0 and O.is_normalised(t)
        m, n, p = (s.m, s.p, s.n) if bits & 1 else (s.m, s.n, s.p)
        if bits & 2:
            assert t.r > s.r and (t.m, t.n, t.p) != (m, n, p)
        elif bits & 8:
            assert t.r % s.r == 0 and t.r > s.r
        elif bits & 16:
            assert t.r == 2 * s.r
        elif bits & 32:
            assert t.r > s.r
        elif bits & 4:
            assert t.r <= s.r and t.m * t.n * t.p < m * n * p
        else:
            assert (t.m, t.n, t.p, t.r) == (m, n, p, s.r)
    assert seen & 1 and seen & 2 and seen & 16 and seen & 32
