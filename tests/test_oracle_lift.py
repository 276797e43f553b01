"""Pins of the oracle's ternary lifting (Sec. 3.10.1, exhaustive search in a
fixed order): the lifting of Strassen's scheme reduced mod 2 is a valid
ternary scheme with the same support; a scheme reduced mod 2 from a valid
ternary scheme always has a lifting (the original signs are a witness); and
the first lifting in the stated order equals the one found by enumerating
every sign pattern in that order without pruning (small cases)."""
import itertools

import numpy as np
import pytest

from oracle import pyoracle as O
from tests.golden_io import load_formula_scheme, matmul_tensor, scheme_tensor


def _z2_of(s):
    d = O.from_c(s)
    return O.to_c(np.abs(d["U"]), np.abs(d["V"]), np.abs(d["W"]), s.m, s.n, s.p, z2=True)


def _check_lifting(z, t):
    dz, dt = O.from_c(z), O.from_c(t)
    assert O.brent_violations(t) == 0 and not t.z2 and O.is_normalised(t)
    for X in "UVW":
        assert np.array_equal(np.abs(dt[X]), dz[X])


def test_strassen_mod_2_lifts():
    U, V, W = load_formula_scheme("strassen_formulas.txt")[3:]
    z = O.to_c(np.abs(U), np.abs(V), np.abs(W), 2, 2, 2, z2=True)
    st, t, _ = O.lift(z)
    assert st == 1
    _check_lifting(z, t)


@pytest.mark.parametrize("fmt,iters", [((2, 2, 2), 3000), ((2, 2, 3), 3000), ((2, 3, 3), 300)])
def test_reductions_of_ternary_schemes_lift(fmt, iters):
    """A lifting exists, so the search never reports none; within its budget
    it finds one for most of them."""
    m, n, p = fmt
    found = 0
    for seed in range(6):
        prm = O.make_params(seed=seed, max_iters=iters, plateau=10 ** 6, target_rank=0,
                            r0=m * n * p)
        w = O.new_walk(O.standard(m, n, p))
        O.run(w, prm, iters)
        z = _z2_of(w.cur)
        assert O.brent_violations(z) == 0
        st, t, _ = O.lift(z, 10 ** 7)
        assert st != 0, (fmt, seed)
        if st == 1:
            _check_lifting(z, t)
            found += 1
    assert found >= 4


def _brute_first(z):
    """Every sign pattern in the search order (term 0 most significant,
    patterns ascending), checked on the whole tensor; the first valid one."""
    d = O.from_c(z)
    m, n, p = z.m, z.n, z.p
    T = matmul_tensor(m, n, p)
    free = []
    for l in range(z.r):
        ent = []
        for X in "UVW":
            nz = list(np.flatnonzero(d[X][l]))
            ent += [(X, e) for e in (nz[1:] if X != "W" else nz)]
        free.append(ent)
    for pats in itertools.product(*[range(1 << len(f)) for f in free]):
        U, V, W = d["U"].astype(np.int64), d["V"].astype(np.int64), d["W"].astype(np.int64)
        M = {"U": U, "V": V, "W": W}
        for l, x in enumerate(pats):
            for i, (X, e) in enumerate(free[l]):
                if (x >> i) & 1:
                    M[X][l, e] = -1
        if np.array_equal(scheme_tensor(U, V, W), T):
            return U, V, W
    return None


def test_first_lifting_equals_unpruned_enumeration():
    checked = 0
    for seed in range(40):
        prm = O.make_params(seed=seed, max_iters=2 + seed % 5, plateau=10 ** 6, target_rank=0,
                            r0=8, t_expand=1 << 30)
        w = O.new_walk(O.standard(2, 2, 2, z2=True))
        O.run(w, prm, 2 + seed % 5)
        z = O.copy(w.cur)
        d = O.from_c(z)
        nfree = sum(np.count_nonzero(d["U"][l]) + np.count_nonzero(d["V"][l]) - 2 +
                    np.count_nonzero(d["W"][l]) for l in range(z.r))
        if nfree > 12:
            continue
        st, t, _ = O.lift(z)
        want = _brute_first(z)
        if want is None:
            assert st == 0
        else:
            assert st == 1
            dt = O.from_c(t)
            for got, w_ in zip((dt["U"], dt["V"], dt["W"]), want):
                assert np.array_equal(got, w_)
        checked += 1
    assert checked >= 5
