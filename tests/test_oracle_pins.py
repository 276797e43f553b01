"""Pins of the CPU oracle against things other than itself: the paper's worked
examples, Strassen's textbook formulas, published Philox known-answer
vectors, the matmul tensor written from C = AB, exact tensor invariance of
every operator, brute-force enumeration and known lower bounds on rank."""
import itertools

import numpy as np
import pytest

from oracle import pyoracle as O
from tests.golden_io import (load_formula_scheme, load_scheme, matmul_tensor,
                             scheme_tensor)


# ---------------------------------------------------------------- Philox
# Known-answer vectors published with the Random123 library (kat_vectors,
# philox4x32 with 10 rounds): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(O.philox(ctr, key)) == want


@pytest.mark.gpu
def test_philox_against_rocrand_host_generator():
    """rocRAND's blocking host Philox4x32-10 generator: output 4k..4k+3 is the block
    with counter (k,0,0,0) and key = the 64-bit seed.  Marked gpu: the
    generator initialises the HIP runtime, which aborts without a device."""
    import ctypes as C
    try:
        L = C.CDLL("/opt/rocm/lib/librocrand.so")
    except OSError:
        pytest.skip("rocRAND not installed")
    gen = C.c_void_p()
    if L.rocrand_create_generator_host_blocking(C.byref(gen), 404) != 0:
        pytest.skip("rocRAND host generator unavailable")
    try:
        seed = 0x0123456789ABCDEF
        assert L.rocrand_set_seed(gen, C.c_ulonglong(seed)) == 0
        buf = (C.c_uint32 * 32)()
        if L.rocrand_generate(gen, buf, C.c_size_t(32)) != 0:
            pytest.skip("rocRAND host generator cannot run here (no HIP device)")
        want = []
        for k in range(8):
            want += O.philox((k, 0, 0, 0), (seed & 0xFFFFFFFF, seed >> 32))
        assert list(buf) == want
    finally:
        L.rocrand_destroy_generator(gen)


# ---------------------------------------------------------------- verifier
def test_paper_2x2x3_example_is_valid():
    m, n, p, U, V, W = load_scheme("paper_2x2x3_rank11.txt")
    s = O.to_c(U, V, W, m, n, p)
    assert O.brent_violations(s) == 0
    assert np.array_equal(scheme_tensor(U, V, W), matmul_tensor(m, n, p))
    # spot checks printed with the example: m1 = (a11+a22)(b11+b22),
    # c11 = m1 - m3 + m4 + m5
    assert list(U[0]) == [1, 0, 0, 1]
    assert list(V[0]) == [1, 0, 0, 0, 1, 0]
    assert list(W[:, 0]) == [1, 0, -1, 1, 1, 0, 0, 0, 0, 0, 0]
    # naive additive complexity nnz - 2r - mp (Sec. 4.5)
    assert O.naive_additions(s) == 20


def test_paper_example_needs_the_transposed_c_index():
    """The printed W columns are (c11,c21,c12,c22,c13,c23), i.e. c_ik at
    k*m+i.  Reading the same matrix as c_ik at i*p+k is not a scheme."""
    m, n, p, U, V, W = load_scheme("paper_2x2x3_rank11.txt")
    Wwrong = np.zeros_like(W)
    for i in range(m):
        for k in range(p):
            Wwrong[:, k * m + i] = W[:, i * p + k]
    assert O.brent_violations(O.to_c(U, V, Wwrong, m, n, p)) > 0


def test_strassen_textbook_is_valid_with_18_additions():
    m, n, p, U, V, W = load_formula_scheme("strassen_formulas.txt")
    s = O.to_c(U, V, W, m, n, p)
    assert O.brent_violations(s) == 0
    assert np.array_equal(scheme_tensor(U, V, W), matmul_tensor(2, 2, 2))
    assert O.naive_additions(s) == 18
    assert s.r == 7


def test_strassen_every_single_mutation_fails():
    m, n, p, U, V, W = load_formula_scheme("strassen_formulas.txt")
    for which in range(3):
        mats = [U.copy(), V.copy(), W.copy()]
        M = mats[which]
        for l in range(M.shape[0]):
            for e in range(M.shape[1]):
                for val in (-1, 0, 1):
                    if M[l, e] == val:
                        continue
                    mm = [x.copy() for x in mats]
                    mm[which][l, e] = val
                    assert O.brent_violations(O.to_c(*mm, m, n, p)) > 0


@pytest.mark.parametrize("fmt", [(1, 1, 1), (1, 2, 2), (2, 2, 2), (2, 2, 3), (2, 3, 4),
                                 (3, 3, 3), (3, 3, 4), (3, 4, 5), (4, 4, 4), (4, 4, 5)])
def test_standard_scheme(fmt):
    m, n, p = fmt
    s = O.standard(m, n, p)
    d = O.from_c(s)
    assert s.r == m * n * p
    assert O.brent_violations(s) == 0
    assert np.array_equal(scheme_tensor(d["U"], d["V"], d["W"]), matmul_tensor(m, n, p))
    assert O.naive_additions(s) == m * p * (n - 1)
    assert O.is_normalised(s)


def test_verifier_counts_exactly_the_wrong_equations():
    rng = np.random.default_rng(7)
    for fmt in [(2, 2, 2), (2, 3, 2), (3, 2, 4)]:
        m, n, p = fmt
        T = matmul_tensor(m, n, p)
        for _ in range(20):
            r = int(rng.integers(1, 12))
            U = rng.integers(-1, 2, size=(r, m * n)).astype(np.int8)
            V = rng.integers(-1, 2, size=(r, n * p)).astype(np.int8)
            W = rng.integers(-1, 2, size=(r, p * m)).astype(np.int8)
            want = int(np.count_nonzero(scheme_tensor(U, V, W) - T))
            assert O.brent_violations(O.to_c(U, V, W, m, n, p)) == want
            want2 = int(np.count_nonzero((scheme_tensor(U, V, W) - T) % 2))
            assert O.brent_violations(O.to_c(U % 2, V % 2, W % 2, m, n, p, z2=True)) == want2


def test_large_standard_schemes_verify():
    for fmt in [(4, 5, 12), (5, 6, 10), (6, 7, 9)]:
        s = O.standard(*fmt)
        assert O.brent_violations(s) == 0
        assert s.r == fmt[0] * fmt[1] * fmt[2]


# ---------------------------------------------------------------- normalisation
def test_paper_normalisation_example():
    m, n, p, U, V, W = load_scheme("paper_normalisation_2x2x2_before.txt")
    _, _, _, U2, V2, W2 = load_scheme("paper_normalisation_2x2x2_after.txt")
    before = O.to_c(U, V, W, m, n, p)
    assert O.brent_violations(before) == 0
    assert not O.is_normalised(before)
    after = O.to_c(U2, V2, W2, m, n, p)
    assert O.brent_violations(after) == 0
    got = O.from_c(O.normalise(before))
    assert np.array_equal(got["U"], U2)
    assert np.array_equal(got["V"], V2)
    assert np.array_equal(got["W"], W2)


# ---------------------------------------------------------------- operators
def _np_normalise(U, V, W):
    U, V, W = U.copy(), V.copy(), W.copy()
    for l in range(U.shape[0]):
        for M in (U, V):
            nz = np.flatnonzero(M[l])
            if len(nz) and M[l, nz[0]] < 0:
                M[l] *= -1
                W[l] *= -1
    return U, V, W


def _np_flip(d, i, j, X, sigma, role):
    """Flip written independently from the paper's formula on numpy arrays."""
    F = [d["U"].astype(np.int64), d["V"].astype(np.int64), d["W"].astype(np.int64)]
    others = [k for k in range(3) if k != X]
    Y, Z = (others[1], others[0]) if role else (others[0], others[1])
    if not np.array_equal(F[X][j], sigma * F[X][i]):
        return None
    ny = F[Y][i] + sigma * F[Y][j]
    nz = F[Z][j] - F[Z][i]
    if np.abs(ny).max() > 1 or np.abs(nz).max() > 1:
        return None
    F[Y][i] = ny
    F[Z][j] = nz
    return _np_normalise(*(x.astype(np.int8) for x in F))


@pytest.mark.parametrize("start", ["standard", "strassen"])
def test_brute_force_all_flips_2x2x2(start):
    if start == "standard":
        s0 = O.standard(2, 2, 2)
    else:
        s0 = O.normalise(O.to_c(*load_formula_scheme("strassen_formulas.txt")[3:], 2, 2, 2))
    d = O.from_c(s0)
    T = matmul_tensor(2, 2, 2)
    n_valid = 0
    for i, j in itertools.permutations(range(s0.r), 2):
        for X in range(3):
            for role in (0, 1):
                for sigma in (1, -1):
                    want = _np_flip(d, i, j, X, sigma, role)
                    same = np.array_equal(d["UVW"[X]][j], sigma * d["UVW"[X]][i])
                    ok = O.flip_valid(s0, i, j, X, sigma, role) and same
                    assert ok == (want is not None)
                    if want is None:
                        continue
                    n_valid += 1
                    s = O.copy(s0)
                    assert O.flip(s, i, j, X, sigma, role)
                    got = O.from_c(s)
                    for k, M in enumerate(want):
                        assert np.array_equal(got["UVW"[k]], M)
                    assert np.array_equal(scheme_tensor(*want), T)
    if start == "standard":
        # every ordered pair sharing a factor: pairs of E_ij(x)E_jk(x)E_ki
        # sharing u differ in k only, etc.; each gives 2 roles
        assert n_valid > 0


def _all_valid_flips(s):
    out = []
    d = O.from_c(s)
    for i, j in itertools.permutations(range(s.r), 2):
        for X in range(3):
            for sigma in ((1,) if s.z2 else (1, -1)):
                if not np.array_equal(d["UVW"[X]][j], sigma * d["UVW"[X]][i]):
                    continue
                for role in (0, 1):
                    if O.flip_valid(s, i, j, X, sigma, role):
                        out.append((i, j, X, sigma, role))
    return out


@pytest.mark.parametrize("fmt", [(2, 2, 2), (2, 2, 3), (3, 3, 3)])
def test_operator_tensor_invariance_random_trajectories(fmt):
    rng = np.random.default_rng(sum(fmt))
    m, n, p = fmt
    T = matmul_tensor(m, n, p)
    s = O.standard(m, n, p)
    for step in range(150):
        moves = _all_valid_flips(s)
        kind = rng.integers(0, 10)
        if kind < 7 and moves:
            i, j, X, sigma, role = moves[rng.integers(0, len(moves))]
            assert O.flip(s, i, j, X, sigma, role)
            O.remove_zero_terms(s)
        elif kind < 8:
            i, j = rng.choice(s.r, 2, replace=False)
            O.plus(s, i, j, rng.integers(0, 6))
        elif kind < 9:
            i, j = rng.choice(s.r, 2, replace=False)
            O.split(s, i, j, rng.integers(0, 6))
        else:
            O.full_reduce(s)
        d = O.from_c(s)
        assert np.array_equal(scheme_tensor(d["U"], d["V"], d["W"]), T), step
        assert O.is_normalised(s)
        assert np.abs(d["U"]).max() <= 1 and np.abs(d["V"]).max() <= 1 and np.abs(d["W"]).max() <= 1
        for M in (d["U"], d["V"], d["W"]):
            assert (np.abs(M).sum(axis=1) > 0).all()


def test_reduction_merges_shared_pairs_and_cancels():
    # two copies of one term with opposite w cancel completely (rank -2)
    U = np.array([[1, 0, 0, 0], [1, 0, 0, 0]], np.int8)
    V = np.array([[0, 1, 0, 0], [0, 1, 0, 0]], np.int8)
    W = np.array([[0, 0, 1, 0], [0, 0, -1, 0]], np.int8)
    s = O.to_c(U, V, W, 2, 2, 2)
    O.full_reduce(s)
    assert s.r == 0
    # shared (u, w) up to sign merges v: u(x)v1(x)w + u(x)v2(x)(-w) = u(x)(v1-v2)(x)w
    U = np.array([[1, 0, 0, 0], [1, 0, 0, 0]], np.int8)
    V = np.array([[1, 0, 0, 0], [0, 1, 0, 0]], np.int8)
    W = np.array([[0, 0, 1, 0], [0, 0, -1, 0]], np.int8)
    s = O.to_c(U, V, W, 2, 2, 2)
    T = scheme_tensor(U, V, W)
    assert O.full_reduce(s) == 1
    d = O.from_c(s)
    assert s.r == 1 and np.array_equal(scheme_tensor(d["U"], d["V"], d["W"]), T)
    assert list(d["V"][0]) == [1, -1, 0, 0]
    # a merge that would leave Z_T is refused: u(x)v(x)w + u(x)v(x)w = u(x)v(x)2w
    s = O.to_c(U[:1].repeat(2, 0), V[:1].repeat(2, 0), W[:1].repeat(2, 0), 2, 2, 2)
    assert O.full_reduce(s) == 0 and s.r == 2
    # ... but in Z2 the same pair cancels (2w = 0 mod 2)
    s = O.to_c(U[:1].repeat(2, 0), V[:1].repeat(2, 0), np.abs(W[:1]).repeat(2, 0), 2, 2, 2,
               z2=True)
    O.full_reduce(s)
    assert s.r == 0


# ---------------------------------------------------------------- meta operators
def _term_set(d):
    return sorted(tuple(d["U"][l]) + tuple(d["V"][l]) + tuple(d["W"][l]) for l in range(d["r"]))


@pytest.mark.parametrize("fmt", [(2, 2, 2), (2, 3, 4), (3, 3, 4), (4, 5, 12)])
def test_project_standard_is_standard(fmt):
    for axis in range(3):
        if fmt[axis] < 2:
            continue
        for index in (0, fmt[axis] - 1):
            got = O.from_c(O.project(O.standard(*fmt), axis, index))
            small = list(fmt)
            small[axis] -= 1
            want = O.from_c(O.standard(*small))
            assert _term_set(got) == _term_set(want)


@pytest.mark.parametrize("fmt", [(2, 2, 2), (2, 3, 4), (3, 4, 5)])
def test_extend_then_project_is_identity(fmt):
    m, n, p = fmt
    s = O.normalise(O.to_c(*load_formula_scheme("strassen_formulas.txt")[3:], 2, 2, 2)) \
        if fmt == (2, 2, 2) else O.standard(*fmt)
    for axis in range(3):
        e = O.extend(s, axis)
        extra = [n * p, m * p, m * n][axis]
        assert e.r == s.r + extra
        assert O.brent_violations(e) == 0
        back = O.project(e, axis, fmt[axis])
        assert _term_set(O.from_c(back)) == _term_set(O.from_c(s))


def test_project_of_strassen_is_valid():
    s = O.normalise(O.to_c(*load_formula_scheme("strassen_formulas.txt")[3:], 2, 2, 2))
    for axis in range(3):
        for index in range(2):
            q = O.project(s, axis, index)
            assert O.brent_violations(q) == 0
            assert q.r <= 7


# ---------------------------------------------------------------- walks
def _check_walk(w, low):
    for sch in (w.cur, w.best):
        assert O.brent_violations(sch) == 0
        assert O.is_normalised(sch)
    assert w.best_rank == w.best.r
    assert w.best_rank >= low


def test_walk_2x2x2_reaches_strassen_rank_never_below():
    start = O.standard(2, 2, 2)
    prm = O.make_params(max_iters=100000, plateau=20000, target_rank=7, r0=8)
    ws = O.run_many(start, prm, 0, 0, 64, 100000, 8)
    for w in ws:
        _check_walk(w, 7)  # rank of <2,2,2> is 7 (Winograd 1971)
        assert w.best_rank == 7 and w.done
        recs = O.records(w)
        assert recs and recs[-1][1] == 7 and recs[-1][0] == w.t


def test_walk_z2_2x2x2():
    start = O.standard(2, 2, 2, z2=True)
    prm = O.make_params(max_iters=100000, plateau=20000, target_rank=7, r0=8)
    ws = O.run_many(start, prm, 0, 0, 32, 100000, 8)
    for w in ws:
        _check_walk(w, 7)  # 7 is also the rank over GF(2) (Hopcroft-Kerr 1971)
    assert sum(w.best_rank == 7 for w in ws) >= 28


def test_walk_1xnxp_never_below_np():
    start = O.standard(1, 2, 3)
    prm = O.make_params(max_iters=20000, plateau=5000, target_rank=0, r0=6, t_expand=1 << 30)
    ws = O.run_many(start, prm, 5, 0, 16, 20000, 8)
    for w in ws:
        _check_walk(w, 6)  # <1,n,p> has rank n*p


def test_walk_3x3x3_short_is_valid():
    start = O.standard(3, 3, 3)
    prm = O.make_params(max_iters=20000, plateau=50000, target_rank=23, r0=27)
    ws = O.run_many(start, prm, 0, 0, 8, 20000, 8)
    for w in ws:
        _check_walk(w, 23)
        assert w.c.flips == w.t  # (3,3,3) from the standard scheme never dead-ends early


@pytest.mark.parametrize("fmt,expand", [((2, 2, 2), 0), ((2, 2, 3), 1 << 29), ((3, 3, 3), 1 << 28)])
def test_round_split_invariance(fmt, expand):
    """A walk run in uneven chunks equals the uninterrupted walk (checkpoint/resume)."""
    import ctypes
    m, n, p = fmt
    start = O.standard(m, n, p)
    prm = O.make_params(seed=99, max_iters=6000, plateau=1500, target_rank=0, r0=m * n * p,
                        t_expand=expand)
    a = O.new_walk(start)
    O.run(a, prm, 6000)
    b = O.new_walk(start)
    for chunk in (1, 7, 500, 1234, 6000):
        O.run(b, prm, chunk)
    assert ctypes.string_at(ctypes.addressof(a), ctypes.sizeof(a)) == \
        ctypes.string_at(ctypes.addressof(b), ctypes.sizeof(b))
    assert a.t == 6000 and a.c.restarts > 0
    if expand:
        assert a.c.expands > 0


# ---------------------------------------------------------- flip sampling
def _numpy_candidates(F, i, X):
    """Valid partners (j, role) of attempt (term i, kind X), written from the
    flip of Sec. 3.3.1 in numpy: x_j = s x_i (s = -1 only for w), then
    y_i + s y_j and z_j - z_i must stay in {-1, 0, 1}; (Y, Z) are the other
    kinds in u < v < w order, swapped for role 1; role 0 first, j ascending."""
    A = 1 if X == 0 else 0
    B = 1 if X == 2 else 2
    out = []
    for role in (0, 1):
        Y, Z = (A, B) if role == 0 else (B, A)
        for j in range(F[0].shape[0]):
            if j == i:
                continue
            if np.array_equal(F[X][j], F[X][i]):
                s = 1
            elif X == 2 and np.array_equal(F[X][j], -F[X][i]):
                s = -1
            else:
                continue
            ny = F[Y][i] + s * F[Y][j]
            nz = F[Z][j] - F[Z][i]
            if np.abs(ny).max() <= 1 and np.abs(nz).max() <= 1:
                out.append((j, role, Y, Z))
    return out


def _bits(v):
    d = sum(1 << e for e, x in enumerate(v) if x != 0)
    s = sum(1 << e for e, x in enumerate(v) if x < 0)
    return d, s


@pytest.mark.parametrize("flip_tries", [1, 7])
def test_flip_sampling_reading(flip_tries):
    """The flip each oracle iteration applies is the one the sampling reading
    predicts from the Philox words alone: attempt a uses block (t, a, 0), term
    U(w0, r), kind U(w1, 3), candidate U(w2, n) of the first attempt with
    candidates; when none has one, the cyclic search starts at pair
    U(w3 of (t,0,0), 3r) and picks U(w3 of (t,1,0), n).  The candidate lists
    come from the independent numpy enumeration above; one attempt
    (flip_tries 1) makes the fallback frequent."""
    M32 = 0xFFFFFFFF
    fallbacks = 0
    for k in range(4):
        seed = 4242 + k
        prm = O.make_params(seed=seed, max_iters=10 ** 6, plateau=10 ** 6, r0=27,
                            flip_tries=flip_tries)
        w = O.new_walk(O.standard(3, 3, 3))
        O.run(w, prm, 150 + 61 * k)
        key = (seed & M32, seed >> 32)
        for _ in range(40):
            d = O.from_c(w.cur)
            F = [d["U"].astype(np.int64), d["V"].astype(np.int64), d["W"].astype(np.int64)]
            r = F[0].shape[0]
            t = w.t + 1
            pred = None
            for a in range(flip_tries):
                w0, w1, w2, _ = O.philox((t & M32, t >> 32, a, 0), key)
                i, X = (w0 * r) >> 32, (w1 * 3) >> 32
                c = _numpy_candidates(F, i, X)
                if c:
                    pred = (i, X) + c[(w2 * len(c)) >> 32]
                    break
            if pred is None:
                fallbacks += 1
                f0 = O.philox((t & M32, t >> 32, 0, 0), key)[3]
                f1 = O.philox((t & M32, t >> 32, 1, 0), key)[3]
                p0 = (f0 * 3 * r) >> 32
                for q in range(3 * r):
                    i, X = divmod((p0 + q) % (3 * r), 3)
                    c = _numpy_candidates(F, i, X)
                    if c:
                        pred = (i, X) + c[(f1 * len(c)) >> 32]
                        break
            assert pred is not None  # (3,3,3) walks from the standard scheme never dead-end here
            i, X, j, role, Y, Z = pred
            logs = O.run_logged(w, prm, 1, t, 0)
            lg = logs[t - 1]
            assert lg.rank_before == r
            want = [_bits(F[X][i]), _bits(F[Y][i]), _bits(F[Z][i]),
                    _bits(F[X][j]), _bits(F[Y][j]), _bits(F[Z][j])]
            got = [(lg.f[2 * q], lg.f[2 * q + 1]) for q in range(6)]
            assert got == want, (seed, t, pred)
    if flip_tries == 1:
        assert fallbacks > 10


# ------------------------------------------------------------------ expand
def _numpy_normalise(u, v, w):
    """Sec. 3.6 on one term: the first non-zero of u, then of v, made
    positive; w absorbs each sign change."""
    u, v, w = u.copy(), v.copy(), w.copy()
    for x in (u, v):
        nz = np.flatnonzero(x)
        if nz.size and x[nz[0]] < 0:
            x *= -1
            w *= -1
    return u, v, w


def _numpy_expand(F, key, t):
    """The expand the reading R10 predicts from the Philox words: up to eight
    attempts, block (t, a, 2): i = U(w0, r), j = U(w1, r-1) shifted past i,
    roles = the U(w2, 6)-th permutation of (u, v, w) in lexicographic order,
    plus when the top bit of w3 is 0, else split (Sec. 3.3.1)."""
    perms = list(itertools.permutations(range(3)))
    r = F[0].shape[0]
    ok = lambda x: np.abs(x).max() <= 1
    for a in range(8):
        w0, w1, w2, w3 = O.philox((t & 0xFFFFFFFF, t >> 32, a, 2), key)
        i = (w0 * r) >> 32
        j = (w1 * (r - 1)) >> 32
        j += j >= i
        X, Y, Z = perms[(w2 * 6) >> 32]
        G = [f.copy() for f in F]
        new = [None, None, None]
        if (w3 >> 31) == 0:
            # plus: x_i (y_i + y_j) z_i + x_i y_j (z_j - z_i) + (x_j - x_i) y_j z_j
            if any(np.array_equal(F[k][i], F[k][j]) for k in (X, Y, Z)):
                continue
            sy, sz, sx = F[Y][i] + F[Y][j], F[Z][j] - F[Z][i], F[X][j] - F[X][i]
            if not (ok(sy) and ok(sz) and ok(sx)) or not sy.any():
                continue
            new[X], new[Y], new[Z] = sx, F[Y][j].copy(), F[Z][j].copy()
            G[X][j], G[Z][j], G[Y][i] = F[X][i], sz, sy
            kind = "plus"
        else:
            # split: x_j y_i z_i + (x_i - x_j) y_i z_i
            if np.array_equal(F[X][i], F[X][j]):
                continue
            sx = F[X][i] - F[X][j]
            if not ok(sx):
                continue
            new = [F[0][i].copy(), F[1][i].copy(), F[2][i].copy()]
            new[X] = sx
            G[X][i] = F[X][j]
            kind = "split"
        G = [np.vstack([G[k], new[k][None, :]]) for k in range(3)]
        for k in (i, j, r):
            G[0][k], G[1][k], G[2][k] = _numpy_normalise(G[0][k], G[1][k], G[2][k])
        return kind, G
    return None, None


def test_expand_sampling_reading():
    """Strassen's scheme has no flip at all (checked here with the numpy
    enumeration), so the first iteration of a walk from it is a dead end and
    Algorithm 1 expands: the oracle's new scheme equals the plus or split the
    reading predicts, and it stays a valid scheme."""
    U, V, W = load_formula_scheme("strassen_formulas.txt")[3:]
    start = O.normalise(O.to_c(U, V, W, 2, 2, 2))
    d0 = O.from_c(start)
    F = [d0["U"].astype(np.int64), d0["V"].astype(np.int64), d0["W"].astype(np.int64)]
    assert not any(_numpy_candidates(F, i, X) for i in range(7) for X in range(3))
    kinds = set()
    for seed in range(64):
        prm = O.make_params(seed=seed, max_iters=10, plateau=10 ** 6, r0=7, r_cap=12)
        w = O.new_walk(start)
        O.run(w, prm, 1)
        kind, G = _numpy_expand(F, (seed & 0xFFFFFFFF, seed >> 32), 1)
        c = O.counters(w)
        assert c["dead_ends"] == 1 and c["flips"] == 0
        if kind is None:
            assert c["expands"] == 0 and w.cur.r == 7
            continue
        kinds.add(kind)
        d = O.from_c(w.cur)
        assert c["expands"] == 1 and d["r"] == 8
        for got, want in zip((d["U"], d["V"], d["W"]), G):
            assert np.array_equal(got, want), (seed, kind)
        assert O.brent_violations(w.cur) == 0
    assert kinds == {"plus", "split"}


# ------------------------------------------------------- best-scheme gates
def test_equal_rank_acceptance_reading():
    """Algorithm 1 keeps the current scheme as the best one when it merely
    equals the best rank with probability 0.01: reading R11/R12, accepted iff
    word w0 of block (t, 0, 1) is below round(0.01 * 2^32).  Stepping walks one
    iteration at a time (iterations without a merge, whose state at the check
    is the final one), every acceptance and every refusal is predicted."""
    t_eq = 42949673
    M32 = 0xFFFFFFFF
    accepted = refused = 0
    for seed in range(3):
        prm = O.make_params(seed=777 + seed, max_iters=10 ** 6, plateau=10 ** 6, r0=27,
                            t_eq=t_eq)
        w = O.new_walk(O.standard(3, 3, 3))
        O.run(w, prm, 300)
        key = ((777 + seed) & M32, (777 + seed) >> 32)
        for _ in range(1500):
            best_rank = w.best_rank
            best = O.from_c(w.best)
            c0 = O.counters(w)
            t = w.t + 1
            O.run(w, prm, 1)
            c1 = O.counters(w)
            if c1["merges"] != c0["merges"] or c1["flips"] == c0["flips"]:
                continue
            cur = O.from_c(w.cur)
            if cur["r"] < best_rank:
                continue  # a strict improvement
            g0 = O.philox((t & M32, t >> 32, 0, 1), key)[0]
            same_best = all(np.array_equal(best[k], O.from_c(w.best)[k]) for k in "UVW")
            if cur["r"] == best_rank and g0 < t_eq:
                accepted += 1
                assert c1["eq_accepts"] == c0["eq_accepts"] + 1
                assert all(np.array_equal(cur[k], O.from_c(w.best)[k]) for k in "UVW")
            else:
                refused += cur["r"] == best_rank
                assert c1["eq_accepts"] == c0["eq_accepts"] and same_best
    assert accepted >= 5 and refused >= 100
