"""Pins of the isotropy-invariant oracle (oracle/invariants.py, Sec. 3.7):
exact ranks against numpy's SVD rank and matrices of known rank, a matrix
whose rank differs over GF(2) and over Q, the standard scheme, Strassen's
scheme (whose factor ranks follow from the textbook formulas: M1 has three
rank-2 factors, every other product three rank-1 factors), and invariance of
all three polynomials under the isotropy group acting on schemes found by
walks (each transformed scheme is checked against the Brent equations)."""
import numpy as np
import pytest

from oracle import invariants as I
from oracle import pyoracle as O
from tests.golden_io import load_formula_scheme


def test_rank_against_numpy_and_known_matrices():
    rng = np.random.default_rng(0)
    for _ in range(300):
        r, c = rng.integers(1, 9, 2)
        M = rng.integers(-1, 2, (r, c)) * (rng.random((r, c)) < 0.6)
        assert I.rank_q(M.tolist()) == np.linalg.matrix_rank(M.astype(float))
    assert I.rank_q(np.eye(5, dtype=int).tolist()) == 5
    assert I.rank_q(np.outer([1, -1, 0, 1], [0, 1, 1]).tolist()) == 1
    assert I.rank_q([[0, 0], [0, 0]]) == 0
    # det = 2: full rank over Q, rank 2 over GF(2)
    M = [[1, 1, 0], [0, 1, 1], [1, 0, 1]]
    assert I.rank_q(M) == 3 and I.rank_gf2(M) == 2


@pytest.mark.parametrize("fmt", [(2, 2, 2), (2, 3, 4), (3, 3, 3)])
def test_standard_scheme_invariants(fmt):
    m, n, p = fmt
    rk = I.term_ranks(O.from_c(O.standard(m, n, p)), m, n, p)
    assert I.type_polynomial(rk) == {(1, 1, 1): m * n * p}
    assert I.symmetric_polynomial(rk) == {(1, 1, 1): 6 * m * n * p}
    assert I.rank_sum_polynomial(rk) == {m * n * p: 3}


def test_strassen_invariants():
    U, V, W = load_formula_scheme("strassen_formulas.txt")[3:]
    rk = I.term_ranks({"U": U, "V": V, "W": W}, 2, 2, 2)
    assert I.type_polynomial(rk) == {(2, 2, 2): 1, (1, 1, 1): 6}
    assert I.symmetric_polynomial(rk) == {(2, 2, 2): 6, (1, 1, 1): 36}
    assert I.rank_sum_polynomial(rk) == {8: 3}
    assert I.term_ranks({"U": U, "V": V, "W": W}, 2, 2, 2, z2=True) == rk


def _signed_perm(k, rng):
    P = np.zeros((k, k), dtype=np.int64)
    P[np.arange(k), rng.permutation(k)] = rng.choice([-1, 1], k)
    return P


def _isotropy(d, m, n, p, rng):
    """Scheme for A B from one for (P A Q)(Q^-1 B R) = P A B R: with signed
    permutation matrices the coefficients stay ternary."""
    P, Q, R = _signed_perm(m, rng), _signed_perm(n, rng), _signed_perm(p, rng)
    U2, V2, W2 = [], [], []
    for u, v, w in zip(d["U"], d["V"], d["W"]):
        Um = np.asarray(u, np.int64).reshape(m, n)
        Vm = np.asarray(v, np.int64).reshape(n, p)
        Wm = np.asarray(w, np.int64).reshape(p, m).T          # c_ik at [i, k]
        U2.append((P.T @ Um @ Q.T).reshape(-1))
        V2.append((Q @ Vm @ R.T).reshape(-1))
        W2.append((P.T @ Wm @ R.T).T.reshape(-1))
    return {"U": np.array(U2), "V": np.array(V2), "W": np.array(W2)}


@pytest.mark.parametrize("fmt,target", [((2, 2, 3), 11), ((2, 3, 3), 16), ((3, 3, 3), 25)])
def test_invariants_unchanged_by_isotropies(fmt, target):
    m, n, p = fmt
    prm = O.make_params(seed=0, max_iters=100000, plateau=30000, target_rank=target,
                        r0=m * n * p)
    w = O.new_walk(O.standard(m, n, p))
    O.run(w, prm, 100000)
    d = O.from_c(w.best)
    rk = I.term_ranks(d, m, n, p)
    rng = np.random.default_rng(sum(fmt))
    for _ in range(5):
        d2 = _isotropy(d, m, n, p, rng)
        s2 = O.to_c(d2["U"], d2["V"], d2["W"], m, n, p)
        assert O.brent_violations(s2) == 0
        rk2 = I.term_ranks(d2, m, n, p)
        assert I.type_polynomial(rk2) == I.type_polynomial(rk)
        assert I.symmetric_polynomial(rk2) == I.symmetric_polynomial(rk)
        assert I.rank_sum_polynomial(rk2) == I.rank_sum_polynomial(rk)
