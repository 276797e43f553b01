"""Isotropy invariants of a matrix multiplication scheme (Sec. 3.7).

TEST INFRASTRUCTURE ONLY: the oracle of the library's invariant routines.
Plain, slow and exact.  Each factor of a term is reshaped into its matrix in
the layout of Sec. 3.1 (u: m x n with a_ij at row i, column j; v: n x p with
b_jk at row j, column k; w: p x m with c_ik at row k, column i, the C^T
layout) and its rank is found by Gaussian elimination over the rationals
(fractions.Fraction) for ternary schemes and over GF(2) for Z2 schemes.
Then, with (a_l, b_l, c_l) the ranks of the three factors of term l:
  type polynomial       sum_l X^a_l Y^b_l Z^c_l
  symmetric polynomial  sum over the six permutations pi of (x, y, z) of
                        pi(sum_l x^a_l y^b_l z^c_l)
  rank-sum polynomial   w^(sum_l a_l) + w^(sum_l b_l) + w^(sum_l c_l)
Polynomials are dicts from exponent tuples to coefficients.
"""
from fractions import Fraction
from itertools import permutations


def rank_q(M):
    """Rank over Q of a list of rows of integers."""
    A = [[Fraction(x) for x in row] for row in M]
    rows = len(A)
    cols = len(A[0]) if rows else 0
    rank = 0
    for c in range(cols):
        piv = next((r for r in range(rank, rows) if A[r][c] != 0), None)
        if piv is None:
            continue
        A[rank], A[piv] = A[piv], A[rank]
        for r in range(rows):
            if r != rank and A[r][c] != 0:
                f = A[r][c] / A[rank][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[rank])]
        rank += 1
    return rank


def rank_gf2(M):
    """Rank over GF(2) of a list of rows of 0/1 integers."""
    A = [[x & 1 for x in row] for row in M]
    rows = len(A)
    cols = len(A[0]) if rows else 0
    rank = 0
    for c in range(cols):
        piv = next((r for r in range(rank, rows) if A[r][c]), None)
        if piv is None:
            continue
        A[rank], A[piv] = A[piv], A[rank]
        for r in range(rows):
            if r != rank and A[r][c]:
                A[r] = [x ^ y for x, y in zip(A[r], A[rank])]
        rank += 1
    return rank


def factor_matrices(u, v, w, m, n, p):
    U = [[int(u[i * n + j]) for j in range(n)] for i in range(m)]
    V = [[int(v[j * p + k]) for k in range(p)] for j in range(n)]
    W = [[int(w[k * m + i]) for i in range(m)] for k in range(p)]
    return U, V, W


def term_ranks(d, m, n, p, z2=False):
    """[(rank U_l, rank V_l, rank W_l)] for the rows of d['U'], d['V'], d['W']."""
    rk = rank_gf2 if z2 else rank_q
    out = []
    for u, v, w in zip(d["U"], d["V"], d["W"]):
        out.append(tuple(rk(M) for M in factor_matrices(u, v, w, m, n, p)))
    return out


def type_polynomial(ranks):
    poly = {}
    for t in ranks:
        poly[t] = poly.get(t, 0) + 1
    return poly


def symmetric_polynomial(ranks):
    poly = {}
    for t in ranks:
        for q in permutations(range(3)):
            e = (t[q[0]], t[q[1]], t[q[2]])
            poly[e] = poly.get(e, 0) + 1
    return poly


def rank_sum_polynomial(ranks):
    poly = {}
    for k in range(3):
        e = sum(t[k] for t in ranks)
        poly[e] = poly.get(e, 0) + 1
    return poly
