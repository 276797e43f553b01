"""Readers for the text fixtures under tests/golden/ (no method arithmetic)."""
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_scheme(name):
    """-> (m, n, p, U, V, W) from a 'format/rank/U/V/W' text fixture"""
    rows = {"U": [], "V": [], "W": []}
    cur = None
    m = n = p = r = None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("format"):
                m, n, p = (int(x) for x in line.split()[1:4])
            elif line.startswith("rank"):
                r = int(line.split()[1])
            elif line in rows:
                cur = line
            else:
                rows[cur].append([int(x) for x in line.split()])
    U, V, W = (np.array(rows[k], dtype=np.int8) for k in "UVW")
    assert U.shape == (r, m * n) and V.shape == (r, n * p) and W.shape == (r, p * m)
    return m, n, p, U, V, W


def load_formula_scheme(name, m=2, n=2, p=2):
    """Parse 'Mk = (sum of +-Aij) * (sum of +-Bjk)' and 'Cik = sum of +-Mk'
    lines into U, V, W in the paper's flattening (1-based indices in text)."""
    prods, outs = {}, {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            lhs, rhs = (x.strip() for x in line.split("="))
            if lhs.startswith("M"):
                a, b = rhs.split("*")
                prods[int(lhs[1:])] = (_linear(a, "A"), _linear(b, "B"))
            else:
                outs[(int(lhs[1]) - 1, int(lhs[2]) - 1)] = _linear(rhs, "M")
    r = len(prods)
    U = np.zeros((r, m * n), np.int8)
    V = np.zeros((r, n * p), np.int8)
    W = np.zeros((r, p * m), np.int8)
    for k in range(1, r + 1):
        for (i, j), c in prods[k][0].items():
            U[k - 1, (i - 1) * n + (j - 1)] = c
        for (j, kk), c in prods[k][1].items():
            V[k - 1, (j - 1) * p + (kk - 1)] = c
    for (i, kk), lin in outs.items():
        for idx, c in lin.items():
            W[idx - 1, kk * m + i] = c
    return m, n, p, U, V, W


def _linear(text, sym):
    text = text.replace("(", "").replace(")", "").replace(" ", "")
    out = {}
    for sign, name in re.findall(r"([+-]?)(" + sym + r"\d+)", text):
        c = -1 if sign == "-" else 1
        digits = name[1:]
        key = int(digits) if sym == "M" else (int(digits[0]), int(digits[1]))
        out[key] = c
    return out


def matmul_tensor(m, n, p):
    """T[a, b, c] of <m,n,p> in the C^T convention, straight from C = A B:
    c_ik = sum_j a_ij b_jk, with a = i*n+j, b = j*p+k, c = k*m+i."""
    T = np.zeros((m * n, n * p, p * m), dtype=np.int64)
    for i in range(m):
        for j in range(n):
            for k in range(p):
                T[i * n + j, j * p + k, k * m + i] = 1
    return T


def scheme_tensor(U, V, W):
    """sum over terms of u (x) v (x) w, exact int64"""
    U, V, W = (np.asarray(x, dtype=np.int64) for x in (U, V, W))
    return np.einsum("la,lb,lc->abc", U, V, W)
