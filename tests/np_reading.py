"""An independent numpy restatement of the walk's readings, used only to
predict what the oracle does from the Philox words alone.

The paper fixes the operators (Sec. 3.3.1 flip, plus, split, reduction;
Sec. 3.3.2 project, extend, swap, merge, product), the sign normalisation
(Sec. 3.6) and the order of the steps of Algorithm 1 (Sec. 3.4.2) and
Algorithm 2 (Sec. 3.4.3).  Where it is silent the readings below are the
ones the walk implements; each function states the reading it restates.
Schemes are lists [U, V, W] of int64 arrays (one row per term), in the
flattening of Sec. 3.1.1: u[i*n+j] <-> a_ij, v[j*p+k] <-> b_jk,
w[k*m+i] <-> c_ik.  Nothing here shares code with the oracle: the Philox
words come from the oracle's generator (pinned separately by published
known-answer vectors), everything else is numpy.
"""
import itertools

import numpy as np

M32 = 0xFFFFFFFF
PERMS = list(itertools.permutations(range(3)))  # (X, Y, Z) in lexicographic order


def below(word, n):
    """uniform integer in [0, n) from a 32-bit word: floor(word * n / 2^32)"""
    return (int(word) * int(n)) >> 32


def words(philox, key, t, a, dom):
    """the four words of the Philox block (iteration t, attempt a, domain dom)"""
    return philox((t & M32, t >> 32, a, dom), key)


def add(x, y, sign, z2):
    """x + sign*y; ternary: None when an entry leaves {-1,0,1}; Z2: mod 2"""
    if z2:
        return (x + y) % 2
    o = x + sign * y
    return None if np.abs(o).max(initial=0) > 1 else o


def normalise_term(F, l, z2):
    """Sec. 3.6 on term l: the first non-zero of u, then of v, made positive;
    w absorbs each sign change."""
    if z2:
        return
    for X in (0, 1):
        nz = np.flatnonzero(F[X][l])
        if nz.size and F[X][l][nz[0]] < 0:
            F[X][l] = -F[X][l]
            F[2][l] = -F[2][l]


def other_kinds(X, role):
    """the kinds other than X in u < v < w order, swapped for role 1"""
    a, b = [k for k in range(3) if k != X]
    return (a, b) if role == 0 else (b, a)


def sign_between(F, i, j, X, z2):
    """+1 if x_j = x_i, -1 if x_j = -x_i (w only, ternary only), else 0"""
    if np.array_equal(F[X][j], F[X][i]):
        return 1
    if not z2 and X == 2 and np.array_equal(F[X][j], -F[X][i]):
        return -1
    return 0


def candidates(F, i, X, z2):
    """Valid flip partners of attempt (term i, kind X): (j, role, sigma) with
    x_j = sigma x_i, y_i + sigma y_j and z_j - z_i in the coefficient set;
    role 0 first, j ascending (reading of try_flip)."""
    eq = (F[X] == F[X][i]).all(1)
    neg = (F[X] == -F[X][i]).all(1) if (X == 2 and not z2) else np.zeros_like(eq)
    sig = np.where(eq, 1, np.where(neg, -1, 0))
    sig[i] = 0
    out = []
    for role in (0, 1):
        Y, Z = other_kinds(X, role)
        if z2:
            ok = sig != 0
        else:
            ny = F[Y][i][None, :] + sig[:, None] * F[Y]
            nz = F[Z] - F[Z][i][None, :]
            ok = (sig != 0) & (np.abs(ny).max(1) <= 1) & (np.abs(nz).max(1) <= 1)
        out += [(int(j), role, int(sig[j])) for j in np.flatnonzero(ok)]
    return out


def choose_flip(F, philox, key, t, flip_tries, z2):
    """try_flip: attempt a uses block (t, a, 0): i = U(w0, r), X = U(w1, 3),
    pick U(w2, n) among its candidates; the first attempt with candidates
    wins.  If none has any: pairs p = 3i + X visited cyclically from
    U(w3 of (t,0,0), 3r), the first with candidates yields U(w3 of (t,1,0), n).
    None at all (or fewer than two terms): a dead end.
    -> ((i, j, X, role, sigma) or None, whether the cyclic search ran)"""
    r = F[0].shape[0]
    if r < 2:
        return None, False
    for a in range(flip_tries):
        w0, w1, w2, _ = words(philox, key, t, a, 0)
        i, X = below(w0, r), below(w1, 3)
        c = candidates(F, i, X, z2)
        if c:
            j, role, s = c[below(w2, len(c))]
            return (i, j, X, role, s), False
    f0 = words(philox, key, t, 0, 0)[3]
    f1 = words(philox, key, t, 1, 0)[3]
    n_pairs = 3 * r
    p0 = below(f0, n_pairs)
    for q in range(n_pairs):
        i, X = divmod((p0 + q) % n_pairs, 3)
        c = candidates(F, i, X, z2)
        if c:
            j, role, s = c[below(f1, len(c))]
            return (i, j, X, role, s), True
    return None, True


def apply_flip(F, i, j, X, role, s, z2):
    """Sec. 3.3.1: y_i += s y_j, z_j -= z_i, then terms i and j normalised"""
    Y, Z = other_kinds(X, role)
    ny = add(F[Y][i], F[Y][j], s, z2)
    nz = add(F[Z][j], F[Z][i], -1, z2)
    F[Y][i], F[Z][j] = ny, nz
    normalise_term(F, i, z2)
    normalise_term(F, j, z2)


def has_zero_factor(F, l):
    return any(not F[X][l].any() for X in range(3))


def swap_remove(F, h, track):
    """the last term moves into slot h; tracked indices follow (h -> -1)"""
    last = F[0].shape[0] - 1
    track[:] = [-1 if q == h else q for q in track]
    if h != last:
        for X in range(3):
            F[X][h] = F[X][last]
        track[:] = [h if q == last else q for q in track]
    for X in range(3):
        F[X] = F[X][:last].copy()


def merge_of(F, t, k, z2):
    """Reduction (Sec. 3.3.1) between terms t and k: the shared pairs tried in
    the order (u,v) -> w_t + w_k, (u, w = s w') -> v_t + s v_k,
    (v, w = s w') -> u_t + s u_k; the first ternary-valid one, or None."""
    eu = np.array_equal(F[0][t], F[0][k])
    ev = np.array_equal(F[1][t], F[1][k])
    sw = sign_between(F, t, k, 2, z2)
    if eu and ev:
        o = add(F[2][t], F[2][k], 1, z2)
        if o is not None:
            return 2, o
    if eu and sw:
        o = add(F[1][t], F[1][k], sw, z2)
        if o is not None:
            return 1, o
    if ev and sw:
        o = add(F[0][t], F[0][k], sw, z2)
        if o is not None:
            return 0, o
    return None


def reduce_tracked(F, track, z2):
    """reduce() of Algorithm 1 on the terms modified by the flip.  Reading:
    for each tracked term in order, the first k (ascending, k != t) that
    merges with it; the merged term is written at slot min(t, k) and slot
    max(t, k) is swap-removed; the merge repeats on the merged term until it
    has no partner (a cascade).  A merged factor of zero removes both terms,
    the higher slot first.  Returns the number of merges."""
    merges = 0
    for q in range(len(track)):
        while track[q] >= 0:
            t = track[q]
            found = None
            # terms sharing two factors with t (w up to sign): only those can merge
            eu = (F[0] == F[0][t]).all(1)
            ev = (F[1] == F[1][t]).all(1)
            ew = (F[2] == F[2][t]).all(1)
            if not z2:
                ew |= (F[2] == -F[2][t]).all(1)
            two = (eu & ev) | (eu & ew) | (ev & ew)
            two[t] = False
            for k in np.flatnonzero(two):
                mk = merge_of(F, t, int(k), z2)
                if mk is not None:
                    found = (int(k),) + mk
                    break
            if found is None:
                break
            k, kind, o = found
            merges += 1
            lo, hi = min(t, k), max(t, k)
            track[:] = [-1 if (p != q and v == k) else v for p, v in enumerate(track)]
            if not o.any():
                track[q] = -1
                swap_remove(F, hi, track)
                swap_remove(F, lo, track)
                break
            for X in range(3):
                F[X][lo] = F[X][t]
            F[kind][lo] = o
            normalise_term(F, lo, z2)
            track[q] = lo
            swap_remove(F, hi, track)
    return merges


def expand(F, philox, key, t, r_cap, z2):
    """expand of Algorithm 1 (plus or split, Sec. 3.3.1).  Reading: up to eight
    attempts, block (t, a, 2): i = U(w0, r), j = U(w1, r-1) shifted past i,
    roles (X, Y, Z) = the U(w2, 6)-th permutation, the top bit of w3 picks
    plus (0) or split (1).  Plus needs x_i != x_j, y_i != y_j, z_i != z_j and
    y_i + y_j non-zero and valid, z_j - z_i and x_j - x_i valid; split needs
    x_i != x_j and x_i - x_j valid.  Refused at r_cap.  The new term is
    appended; terms i, j and the new one are normalised."""
    r = F[0].shape[0]
    if r >= r_cap or r < 2:
        return False
    for a in range(8):
        w0, w1, w2, w3 = words(philox, key, t, a, 2)
        i = below(w0, r)
        j = below(w1, r - 1)
        j += j >= i
        X, Y, Z = PERMS[below(w2, 6)]
        if (w3 >> 31) == 0:
            if any(np.array_equal(F[k][i], F[k][j]) for k in (X, Y, Z)):
                continue
            sy = add(F[Y][i], F[Y][j], 1, z2)
            sz = add(F[Z][j], F[Z][i], -1, z2)
            sx = add(F[X][j], F[X][i], -1, z2)
            if sy is None or sz is None or sx is None or not sy.any():
                continue
            new = [None, None, None]
            new[X], new[Y], new[Z] = sx, F[Y][j].copy(), F[Z][j].copy()
            F[X][j], F[Z][j], F[Y][i] = F[X][i].copy(), sz, sy
        else:
            if np.array_equal(F[X][i], F[X][j]):
                continue
            sx = add(F[X][i], F[X][j], -1, z2)
            if sx is None:
                continue
            new = [F[0][i].copy(), F[1][i].copy(), F[2][i].copy()]
            new[X] = sx
            F[X][i] = F[X][j].copy()
        for k in range(3):
            F[k] = np.vstack([F[k], new[k][None, :]])
        for l in (i, j, r):
            normalise_term(F, l, z2)
        return True
    return False


class Walk:
    """State of one walk as Algorithm 1 and the readings define it."""

    def __init__(self, start, z2):
        self.z2 = z2
        self.start = [x.copy() for x in start]
        self.cur = [x.copy() for x in start]
        self.best = [x.copy() for x in start]
        self.best_rank = start[0].shape[0]
        self.plateau_start = 0
        self.t = 0
        self.records = []
        self.c = dict(flips=0, dead_ends=0, zero_removed=0, merges=0, expands=0,
                      restarts=0, eq_accepts=0, improvements=0, fallbacks=0)

    def iteration(self, philox, key, prm):
        """one iteration t = self.t + 1 of Algorithm 1 (rank objective):
        try_flip, else expand and continue; zero-term removal (higher slot
        first); the best update (strictly lower rank always; equal rank iff
        w0 of block (t,0,1) < t_eq); reduce iff w1 < t_reduce; expand iff
        w2 < t_expand and r <= best + 2 and r < r_cap; then the plateau
        restart: t - plateau_start >= plateau -> current := start (or best),
        plateau_start := t."""
        t = self.t + 1
        F = self.cur
        ch, fb = choose_flip(F, philox, key, t, prm["flip_tries"], self.z2)
        self.c["fallbacks"] += fb
        if ch is None:
            self.c["dead_ends"] += 1
            if expand(F, philox, key, t, prm["r_cap"], self.z2):
                self.c["expands"] += 1
        else:
            i, j, X, role, s = ch
            apply_flip(F, i, j, X, role, s, self.z2)
            self.c["flips"] += 1
            track = [i, j]
            zi, zj = has_zero_factor(F, i), has_zero_factor(F, j)
            for h in sorted([l for l, z in ((i, zi), (j, zj)) if z], reverse=True):
                swap_remove(F, h, track)
                self.c["zero_removed"] += 1
            g0, g1, g2, _ = words(philox, key, t, 0, 1)
            r = F[0].shape[0]
            if r < self.best_rank:
                self.best = [x.copy() for x in F]
                self.best_rank = r
                self.plateau_start = t
                self.records.append((t, r))
                self.c["improvements"] += 1
            elif r == self.best_rank and g0 < prm["t_eq"]:
                self.best = [x.copy() for x in F]
                self.c["eq_accepts"] += 1
            if g1 < prm["t_reduce"]:
                self.c["merges"] += reduce_tracked(F, track, self.z2)
            r = F[0].shape[0]
            if g2 < prm["t_expand"] and r <= self.best_rank + 2 and r < prm["r_cap"]:
                if expand(F, philox, key, t, prm["r_cap"], self.z2):
                    self.c["expands"] += 1
        if prm["plateau"] > 0 and t - self.plateau_start >= prm["plateau"]:
            src = self.best if prm["restart_from_best"] else self.start
            self.cur = [x.copy() for x in src]
            self.plateau_start = t
            self.c["restarts"] += 1
        self.t = t


# ------------------------------------------------------- meta operators
def _mats(F, l, m, n, p):
    """term l as matrices: u (m x n), v (n x p), w (p x m)"""
    return F[0][l].reshape(m, n), F[1][l].reshape(n, p), F[2][l].reshape(p, m)


def _scheme(terms, z2):
    """[U, V, W] from a list of (u, v, w) matrices, each term normalised"""
    F = [np.array([t[k].reshape(-1) for t in terms], dtype=np.int64) for k in range(3)]
    for l in range(len(terms)):
        normalise_term(F, l, z2)
    return F


def swap_sizes(F, dims, z2):
    """(m,n,p) -> (m,p,n): u' = w^T, v' = v^T, w' = u^T (Sec. 3.3.2; the
    transpose C^T = B^T A^T in the C^T layout)"""
    m, n, p = dims
    terms = []
    for l in range(F[0].shape[0]):
        u, v, w = _mats(F, l, m, n, p)
        terms.append((w.T, v.T, u.T))
    return _scheme(terms, z2), (m, p, n)


def merge(Fa, da, Fb, db, axis, z2):
    """Sec. 3.3.2 merge along axis (0: [A1; A2] B, 1: [A1 A2][B1; B2],
    2: A [B1 B2]); the terms of a first.  None when the other two sizes
    differ or a factor exceeds 64 entries or the rank 512."""
    others = [k for k in range(3) if k != axis]
    if any(da[k] != db[k] for k in others):
        return None
    D = list(da)
    D[axis] = da[axis] + db[axis]
    M, N, P = D
    if M * N > 64 or N * P > 64 or P * M > 64 or Fa[0].shape[0] + Fb[0].shape[0] > 512:
        return None
    terms = []
    for q, (F, d) in enumerate(((Fa, da), (Fb, db))):
        off = [0, 0, 0]
        if q:
            off[axis] = da[axis]
        oi, oj, ok = off
        for l in range(F[0].shape[0]):
            u, v, w = _mats(F, l, *d)
            U = np.zeros((M, N), np.int64)
            V = np.zeros((N, P), np.int64)
            W = np.zeros((P, M), np.int64)
            U[oi:oi + d[0], oj:oj + d[1]] = u
            V[oj:oj + d[1], ok:ok + d[2]] = v
            W[ok:ok + d[2], oi:oi + d[0]] = w
            terms.append((U, V, W))
    return _scheme(terms, z2), tuple(D)


def product(Fa, da, Fb, db, z2):
    """tensor product (Sec. 3.3.2): factors are Kronecker products of the
    matrices, term l1 * r2 + l2"""
    M, N, P = (da[k] * db[k] for k in range(3))
    ra, rb = Fa[0].shape[0], Fb[0].shape[0]
    if M * N > 64 or N * P > 64 or P * M > 64 or ra * rb > 512:
        return None
    terms = []
    for l1 in range(ra):
        a = _mats(Fa, l1, *da)
        for l2 in range(rb):
            b = _mats(Fb, l2, *db)
            terms.append(tuple(np.kron(a[k], b[k]) for k in range(3)))
    return _scheme(terms, z2), (M, N, P)


def extend(F, dims, axis, z2):
    """Sec. 3.3.2 extend: one more row of A (axis 0), column of A (axis 1) or
    column of B (axis 2), covered by appending the naive products of the new
    index in (j,k), (i,k) or (i,j) order.  None past 64 entries or rank 512."""
    m, n, p = dims
    D = [m, n, p]
    D[axis] += 1
    M, N, P = D
    extra = [n * p, m * p, m * n][axis]
    if M * N > 64 or N * P > 64 or P * M > 64 or F[0].shape[0] + extra > 512:
        return None
    terms = []
    for l in range(F[0].shape[0]):
        u, v, w = _mats(F, l, m, n, p)
        U = np.zeros((M, N), np.int64)
        V = np.zeros((N, P), np.int64)
        W = np.zeros((P, M), np.int64)
        U[:m, :n], V[:n, :p], W[:p, :m] = u, v, w
        terms.append((U, V, W))

    def unit(a, b, shape):
        e = np.zeros(shape, np.int64)
        e[a, b] = 1
        return e

    if axis == 2:
        new = [(i, j, p) for i in range(m) for j in range(n)]
    elif axis == 0:
        new = [(m, j, k) for j in range(n) for k in range(p)]
    else:
        new = [(i, n, k) for i in range(m) for k in range(p)]
    for i, j, k in new:
        terms.append((unit(i, j, (M, N)), unit(j, k, (N, P)), unit(k, i, (P, M))))
    return _scheme(terms, z2), tuple(D)


def project(F, dims, axis, index, z2):
    """Sec. 3.3.2 project: drop index `index` of axis, then drop the terms
    with a zero factor (the others keep their order)"""
    m, n, p = dims
    keep = [np.arange(d) != (index if a == axis else -1) for a, d in enumerate(dims)]
    terms = []
    for l in range(F[0].shape[0]):
        u, v, w = _mats(F, l, m, n, p)
        u = u[keep[0]][:, keep[1]]
        v = v[keep[1]][:, keep[2]]
        w = w[keep[2]][:, keep[0]]
        if u.any() and v.any() and w.any():
            terms.append((u, v, w))
    D = list(dims)
    D[axis] -= 1
    return _scheme(terms, z2), tuple(D)


# Algorithm 2 (Sec. 3.4.3): with probability p_resize, project 5%, product
# 50%, double 30%, extend 15%; as cumulative 32-bit thresholds
P_PROJECT, P_PRODUCT, P_DOUBLE = 0.05, 0.50, 0.30
T_PROJECT = round(P_PROJECT * 2 ** 32)
T_PRODUCT = round((P_PROJECT + P_PRODUCT) * 2 ** 32)
T_DOUBLE = round((P_PROJECT + P_PRODUCT + P_DOUBLE) * 2 ** 32)


def resize(F, dims, best, philox, key, rnd, t_resize, cap, z2):
    """Algorithm 2 for one scheme.  Reading of its random choices: blocks
    b0 = (round, 0, 3) and b1 = (round, 1, 3); swap sizes iff b0.w0 < 2^31;
    merge partner best[U(b0.w1, K)], axes tried p, m, n, the first that
    exists and fits (rank <= cap) is taken; without a merge and
    b0.w2 < t_resize, b0.w3 picks project / product / double / extend by the
    thresholds above, axis U(b1.w1, 3), product partner best[U(b1.w0, K)],
    project index U(b1.w2, size of the axis); an operator that does not exist
    or fit leaves the scheme as it is.  best: list of (F, dims).
    -> (bits: 1 swap, 2 merge, 4 project, 8 product, 16 double, 32 extend,
        F, dims)"""
    b0 = words(philox, key, rnd, 0, 3)
    b1 = words(philox, key, rnd, 1, 3)
    bits = 0
    if b0[0] < 2 ** 31:
        F, dims = swap_sizes(F, dims, z2)
        bits |= 1
    if best:
        Fb, db = best[below(b0[1], len(best))]
        for axis in (2, 0, 1):
            got = merge(F, dims, Fb, db, axis, z2)
            if got is not None and got[0][0].shape[0] <= cap:
                F, dims = got
                bits |= 2
                break
    if not bits & 2 and b0[2] < t_resize:
        axis = below(b1[1], 3)
        q = b0[3]
        got = None
        if q < T_PROJECT:
            bit = 4
            if dims[axis] >= 2:
                got = project(F, dims, axis, below(b1[2], dims[axis]), z2)
        elif q < T_PRODUCT:
            bit = 8
            if best:
                Fb, db = best[below(b1[0], len(best))]
                got = product(F, dims, Fb, db, z2)
        elif q < T_DOUBLE:
            bit = 16
            got = merge(F, dims, F, dims, axis, z2)
        else:
            bit = 32
            got = extend(F, dims, axis, z2)
        if got is not None and got[0][0].shape[0] <= cap:
            F, dims = got
            bits |= bit
    return bits, F, dims
