"""CPU tests of libtsf's host side: exported symbols, the one-bit ternary
arithmetic (exhaustive against integers), and the host scheme operations
against the oracle and the paper's examples."""
import ctypes as C
import itertools
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2511_20317_amd import tsf
from tests.golden_io import load_formula_scheme, load_scheme, matmul_tensor, scheme_tensor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tsf.LIB_PATH):
        from paper_2511_20317_amd import build
        build.build()
    return tsf.lib()


def test_library_exports_every_declared_symbol(lib):
    text = open(os.path.join(ROOT, "include", "tsf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(tsf_[a-z_]+)\s*\(", text))
    assert "tsf_walk" in names and "tsf_verify" in names
    for name in sorted(names):
        assert hasattr(lib, name), name


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "libshim.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out),
                           os.path.join(ROOT, "tests", "bits_shim.cpp")])
    L = C.CDLL(str(out))
    u64 = C.c_uint64
    for name in ("shim_add", "shim_sub"):
        getattr(L, name).argtypes = [u64, u64, u64, u64, C.POINTER(u64), C.POINTER(u64)]
    L.shim_neg_eq.argtypes = [u64, u64, u64, u64]
    L.shim_philox.argtypes = [u64, C.c_int64, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32)]
    return L


def _enc(vec):
    d = s = 0
    for e, x in enumerate(vec):
        if x:
            d |= 1 << e
        if x < 0:
            s |= 1 << e
    return d, s


def _dec(d, s, n):
    return [0 if not (d >> e) & 1 else (-1 if (s >> e) & 1 else 1) for e in range(n)]


def test_ternary_bit_formulas_exhaustive(shim):
    """Sec. 3.5.2 formulas vs integer arithmetic on all pairs of length-4 vectors
    (plus random length-64 pairs)."""
    n = 4
    vecs = list(itertools.product((-1, 0, 1), repeat=n))
    d, s = C.c_uint64(), C.c_uint64()
    for a in vecs:
        da, sa = _enc(a)
        for b in vecs:
            db, sb = _enc(b)
            for op, fn in ((1, shim.shim_add), (-1, shim.shim_sub)):
                ok = fn(da, sa, db, sb, C.byref(d), C.byref(s))
                want = [x + op * y for x, y in zip(a, b)]
                valid = all(abs(x) <= 1 for x in want)
                assert bool(ok) == valid
                if valid:
                    assert _dec(d.value, s.value, n) == want
                    assert s.value & ~d.value == 0
            assert bool(shim.shim_neg_eq(da, sa, db, sb)) == (list(a) == [-y for y in b])
    rng = np.random.default_rng(1)
    for _ in range(2000):
        a = rng.integers(-1, 2, 64)
        b = rng.integers(-1, 2, 64)
        da, sa = _enc(a)
        db, sb = _enc(b)
        ok = shim.shim_add(da, sa, db, sb, C.byref(d), C.byref(s))
        assert bool(ok) == bool(np.all(np.abs(a + b) <= 1))
        if ok:
            assert _dec(d.value, s.value, 64) == list(a + b)


def test_library_philox_matches_oracle(shim):
    out = (C.c_uint32 * 4)()
    for seed, t, a, dom in [(0, 1, 0, 0), (123456789, 99999, 7, 2), (2**64 - 1, 2**40 + 3, 8, 1)]:
        shim.shim_philox(seed, t, a, dom, out)
        want = O.philox((t & 0xFFFFFFFF, t >> 32, a, dom), (seed & 0xFFFFFFFF, seed >> 32))
        assert list(out) == want


def _from_oracle(s, mode=tsf.TSF_TERNARY):
    d = O.from_c(s)
    return tsf.Scheme(d["m"], d["n"], d["p"], d["U"], d["V"], d["W"], mode)


def _rows(s):
    U, V, W = s.live()
    return [tuple(U[l]) + tuple(V[l]) + tuple(W[l]) for l in range(s.rank)]


@pytest.mark.parametrize("fmt", [(2, 2, 2), (2, 3, 4), (3, 3, 3), (4, 4, 5), (4, 5, 12), (6, 7, 9)])
def test_init_scheme_equals_oracle_standard(lib, fmt):
    s = tsf.init_scheme(*fmt)
    o = _from_oracle(O.standard(*fmt))
    assert _rows(s) == _rows(o)
    assert tsf.verify(s) == 0


def test_verify_on_paper_examples_and_mutations(lib):
    m, n, p, U, V, W = load_scheme("paper_2x2x3_rank11.txt")
    assert tsf.verify(tsf.Scheme(m, n, p, U, V, W)) == 0
    m, n, p, U, V, W = load_formula_scheme("strassen_formulas.txt")
    assert tsf.verify(tsf.Scheme(m, n, p, U, V, W)) == 0
    rng = np.random.default_rng(3)
    for fmt in [(2, 2, 2), (2, 3, 2), (3, 3, 2)]:
        m, n, p = fmt
        for _ in range(30):
            r = int(rng.integers(1, 10))
            U = rng.integers(-1, 2, (r, m * n))
            V = rng.integers(-1, 2, (r, n * p))
            W = rng.integers(-1, 2, (r, p * m))
            want = O.brent_violations(O.to_c(U, V, W, m, n, p))
            assert tsf.verify(tsf.Scheme(m, n, p, U, V, W)) == want
            want2 = O.brent_violations(O.to_c(U % 2, V % 2, W % 2, m, n, p, z2=True))
            assert tsf.verify(tsf.Scheme(m, n, p, U % 2, V % 2, W % 2, tsf.TSF_Z2)) == want2


def test_not_ternary_is_rejected(lib):
    s = tsf.init_scheme(2, 2, 2)
    s.U[0, 0] = 2
    with pytest.raises(tsf.TsfError) as e:
        tsf.verify(s)
    assert e.value.status == -4
    z = tsf.init_scheme(2, 2, 2, tsf.TSF_Z2)
    z.V[1, 1] = -1
    with pytest.raises(tsf.TsfError):
        tsf.verify(z)
    with pytest.raises(tsf.TsfError) as e:
        tsf.init_scheme(5, 13, 2)
    assert e.value.status == -2


def test_normalise_paper_example(lib):
    m, n, p, U, V, W = load_scheme("paper_normalisation_2x2x2_before.txt")
    _, _, _, U2, V2, W2 = load_scheme("paper_normalisation_2x2x2_after.txt")
    s = tsf.normalise(tsf.Scheme(m, n, p, U, V, W))
    got = s.live()
    assert np.array_equal(got[0], U2) and np.array_equal(got[1], V2) and np.array_equal(got[2], W2)


def test_pack_unpack_round_trip(lib):
    rng = np.random.default_rng(5)
    for fmt, mode in [((2, 2, 3), 0), ((4, 5, 12), 0), ((6, 7, 9), 1), ((3, 3, 3), 1)]:
        m, n, p = fmt
        r = 17
        U = rng.integers(-1, 2, (r, m * n))
        V = rng.integers(-1, 2, (r, n * p))
        W = rng.integers(-1, 2, (r, p * m))
        if mode:
            U, V, W = U % 2, V % 2, W % 2
        s = tsf.Scheme(m, n, p, U, V, W, mode, capacity=20)
        pk = tsf.pack(s)
        assert pk.shape == (20, 6) and not pk[r:].any()
        back = tsf.unpack(pk, m, n, p, r, mode)
        assert all(np.array_equal(a, b) for a, b in zip(back.live(), s.live()))
    bad = tsf.pack(tsf.init_scheme(2, 2, 2))
    bad[0, 1] = 1 << 5  # a sign outside the digits
    with pytest.raises(tsf.TsfError):
        tsf.unpack(bad, 2, 2, 2, 8)


def test_reduce_matches_oracle_on_unique_cases(lib):
    # the worked cases of the oracle pins: cancellation, merge, refusal
    U = np.array([[1, 0, 0, 0], [1, 0, 0, 0]])
    V = np.array([[1, 0, 0, 0], [0, 1, 0, 0]])
    W = np.array([[0, 0, 1, 0], [0, 0, -1, 0]])
    s = tsf.Scheme(2, 2, 2, U, V, W)
    assert tsf.reduce(s) == 1 and s.rank == 1
    assert list(s.live()[1][0]) == [1, -1, 0, 0]
    s = tsf.Scheme(2, 2, 2, U, U * 0 + V[0], W)
    assert tsf.reduce(s) == 1 and s.rank == 0


def test_reduce_keeps_tensor_on_random_expanded_schemes(lib):
    rng = np.random.default_rng(11)
    for fmt in [(2, 2, 2), (2, 2, 3), (3, 3, 3)]:
        s = O.standard(*fmt)
        for _ in range(30):
            i, j = rng.choice(s.r, 2, replace=False)
            (O.plus if rng.integers(2) else O.split)(s, i, j, rng.integers(6))
        T = matmul_tensor(*fmt)
        t = _from_oracle(s)
        tsf.reduce(t)
        assert np.array_equal(scheme_tensor(*t.live()), T)
        assert tsf.verify(t) == 0
        # fixpoint: a second pass merges nothing
        assert tsf.reduce(t) == 0


@pytest.mark.parametrize("fmt", [(2, 2, 2), (2, 3, 4), (3, 4, 5), (4, 5, 12)])
def test_meta_project_extend_match_oracle(lib, fmt):
    s_o = O.standard(*fmt)
    s = tsf.init_scheme(*fmt)
    for axis in range(3):
        if fmt[axis] >= 2:
            for index in (0, fmt[axis] - 1):
                a = tsf.meta_project(s, axis, index)
                b = _from_oracle(O.project(s_o, axis, index))
                assert (a.m, a.n, a.p) == (b.m, b.n, b.p)
                assert _rows(a) == _rows(b)
                assert tsf.verify(a) == 0
        if max(fmt[0] * fmt[1], fmt[1] * fmt[2], fmt[2] * fmt[0]) * 2 <= 64:
            a = tsf.meta_extend(s, axis)
            b = _from_oracle(O.extend(s_o, axis))
            assert _rows(a) == _rows(b)
            assert tsf.verify(a) == 0


def test_meta_on_strassen(lib):
    m, n, p, U, V, W = load_formula_scheme("strassen_formulas.txt")
    s = tsf.normalise(tsf.Scheme(m, n, p, U, V, W))
    e = tsf.meta_extend(s, 2)
    assert e.rank == 7 + 4 and (e.m, e.n, e.p) == (2, 2, 3) and tsf.verify(e) == 0
    back = tsf.meta_project(e, 2, 2)
    assert sorted(_rows(back)) == sorted(_rows(s))


@pytest.mark.parametrize("fmt,target,z2", [((2, 2, 3), 11, False), ((3, 3, 3), 25, False),
                                           ((2, 3, 4), 22, False), ((2, 2, 3), 11, True)])
def test_scheme_invariants_match_oracle(lib, fmt, target, z2):
    """tsf_scheme_invariants (host, the same rank routine as the GPU kernel)
    against the exact oracle on schemes found by oracle walks."""
    from oracle import invariants as I
    m, n, p = fmt
    prm = O.make_params(seed=3, max_iters=60000, plateau=20000, target_rank=target,
                        r0=m * n * p, t_expand=1 << 29)
    ws = O.run_many(O.standard(m, n, p, z2=z2), prm, 3, 0, 6, 60000, 6)
    for w in ws:
        for sch in (w.best, w.cur):
            d = O.from_c(sch)
            got = tsf.scheme_invariants(_from_oracle(sch, tsf.TSF_Z2 if z2 else tsf.TSF_TERNARY))
            rk = I.term_ranks(d, m, n, p, z2=z2)
            assert got["term_ranks"] == rk
            assert got["type"] == I.type_polynomial(rk)
            assert got["symmetric"] == I.symmetric_polynomial(rk)
            sums = tuple(sum(t[k] for t in rk) for k in range(3))
            assert got["rank_sum"] == sums


def _walked_oracle(fmt, seed, iters=5000):
    m, n, p = fmt
    prm = O.make_params(seed=seed, max_iters=iters, plateau=3000, target_rank=0, r0=m * n * p,
                        t_expand=1 << 28)
    w = O.new_walk(O.standard(m, n, p))
    O.run(w, prm, iters)
    return O.copy(w.cur)


def test_meta_swap_merge_product_match_oracle(lib):
    """tsf_meta_swap / merge / product (the packed-term routines the resize
    kernel uses) against the oracle's int8 operators, term by term."""
    cases = [_walked_oracle((2, 3, 4), 1), _walked_oracle((2, 2, 3), 2), _walked_oracle((3, 3, 2), 3)]
    for s in cases:
        want = O.from_c(O.swap_sizes(s))
        got = tsf.meta_swap(_from_oracle(s))
        assert (got.m, got.n, got.p) == (s.m, s.p, s.n)
        assert _rows(got) == [tuple(want["U"][l]) + tuple(want["V"][l]) + tuple(want["W"][l])
                              for l in range(s.r)]
    a, b = _walked_oracle((2, 2, 3), 4), _walked_oracle((2, 2, 2), 5)
    for axis, (x, y) in [(2, (a, b)), (0, (_walked_oracle((1, 2, 3), 6), a)),
                         (1, (a, _walked_oracle((2, 1, 3), 7)))]:
        want = O.from_c(O.merge(x, y, axis))
        got = tsf.meta_merge(_from_oracle(x), _from_oracle(y), axis)
        assert _rows(got) == [tuple(want["U"][l]) + tuple(want["V"][l]) + tuple(want["W"][l])
                              for l in range(want["r"])]
        assert tsf.verify(got) == 0
    x, y = _walked_oracle((2, 2, 2), 8), _walked_oracle((1, 2, 2), 9)
    want = O.from_c(O.product(x, y))
    got = tsf.meta_product(_from_oracle(x), _from_oracle(y))
    assert (got.m, got.n, got.p, got.rank) == (2, 4, 4, x.r * y.r)
    assert _rows(got) == [tuple(want["U"][l]) + tuple(want["V"][l]) + tuple(want["W"][l])
                          for l in range(want["r"])]
    assert tsf.verify(got) == 0
    with pytest.raises(tsf.TsfError):
        tsf.meta_merge(_from_oracle(x), _from_oracle(_walked_oracle((2, 3, 3), 1)), 2)


def test_error_paths_of_the_host_calls(lib):
    """Documented errors of the host calls: null pointers are TSF_E_ARG, a
    factor longer than 64 entries TSF_E_FORMAT, an output too small
    TSF_E_CAPACITY, an axis or index out of range TSF_E_ARG; every error leaves
    a message for tsf_last_error."""
    assert lib.tsf_init_scheme(2, 2, 2, 0, None) == -1
    assert lib.tsf_last_error()
    assert lib.tsf_verify(None, None) == -1
    n = C.c_int64()
    assert lib.tsf_verify(None, C.byref(n)) == -1
    s = tsf.init_scheme(2, 2, 2)
    assert lib.tsf_verify(C.byref(s.c()), None) == -1
    # a factor of 8 x 9 = 72 entries does not fit one 64-bit mask
    with pytest.raises(tsf.TsfError) as e:
        tsf.init_scheme(8, 9, 1)
    assert e.value.status == -2
    # extend of (2,2,2) along p into an output of capacity 9 < 8 + 4
    out = tsf.Scheme.empty(2, 2, 3, 9)
    cs = out.c()
    assert lib.tsf_meta_extend(C.byref(s.c()), 2, C.byref(cs)) == -3
    # axis and index out of range
    out = tsf.Scheme.empty(2, 2, 1, 8)
    cs = out.c()
    assert lib.tsf_meta_project(C.byref(s.c()), 3, 0, C.byref(cs)) == -1
    assert lib.tsf_meta_project(C.byref(s.c()), 2, 2, C.byref(cs)) == -1
    assert b"" != lib.tsf_last_error()
    # the same calls in range succeed
    assert lib.tsf_meta_project(C.byref(s.c()), 2, 1, C.byref(cs)) == 0


def _fnv1a_params(prm):
    """FNV-1a (64-bit) over the little-endian bytes of the resume-relevant
    walk parameters, written out independently of the library."""
    import struct
    h = 0xCBF29CE484222325
    data = struct.pack("<QqqqQQQiii", prm.base_seed, prm.first_walk_id, prm.max_iters,
                       prm.plateau, prm.t_eq, prm.t_reduce, prm.t_expand, prm.flip_tries,
                       prm.restart_from_best, prm.objective)
    for byte in data:
        h ^= byte
        h = (h * 0x100000001B3) % (1 << 64)
    return h or 1


def test_params_hash_and_resume_check(lib):
    """tsf_walk_check (host, no GPU): walks whose headers carry the hash of
    other parameters than the resuming call's are reported as TSF_E_STATE;
    fresh headers (hash 0) and headers of the same parameters pass."""
    a = tsf.walk_params(base_seed=5, max_iters=1000, plateau=300)
    variants = [tsf.walk_params(base_seed=6, max_iters=1000, plateau=300),
                tsf.walk_params(base_seed=5, max_iters=1001, plateau=300),
                tsf.walk_params(base_seed=5, max_iters=1000, plateau=301),
                tsf.walk_params(base_seed=5, max_iters=1000, plateau=300, flip_tries=6),
                tsf.walk_params(base_seed=5, max_iters=1000, plateau=300, restart_from_best=1),
                tsf.walk_params(base_seed=5, max_iters=1000, plateau=300, t_expand=1),
                tsf.walk_params(base_seed=5, max_iters=1000, plateau=300, objective=1),
                tsf.walk_params(base_seed=5, first_walk_id=3, max_iters=1000, plateau=300)]
    ha = tsf.params_hash(a)
    assert ha == _fnv1a_params(a)
    assert len({ha} | {tsf.params_hash(v) for v in variants}) == len(variants) + 1
    hdr = np.zeros(6, tsf.HEADER_DTYPE)
    assert tsf.walk_check(a, hdr) == 0 and tsf.walk_check.mismatched == 0
    hdr["params_hash"] = ha
    assert tsf.walk_check(a, hdr) == 0
    for v in variants:
        assert tsf.walk_check(v, hdr) == tsf.TSF_E_STATE
        assert tsf.walk_check.mismatched == 6
    hdr["params_hash"][2] = 0
    hdr["done"][4] = -3
    assert tsf.walk_check(a, hdr) == tsf.TSF_E_STATE and tsf.walk_check.mismatched == 1
    assert tsf.walk_check(variants[0], hdr) == tsf.TSF_E_STATE
    assert tsf.walk_check.mismatched == 5
