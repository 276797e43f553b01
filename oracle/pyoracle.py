"""ctypes binding of the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark, never by the product library.  Schemes cross
this binding as numpy int8 arrays U (r x m*n), V (r x n*p), W (r x p*m) in the
paper's flattening (Sec. 3.1.1): u[i*n+j] <-> a_ij, v[j*p+k] <-> b_jk,
w[k*m+i] <-> c_ik.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

MAXL = 64
MAXT = 512
MAXREC = 512


class Scheme(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int), ("p", C.c_int), ("r", C.c_int),
                ("z2", C.c_int), ("f", C.c_int8 * (3 * MAXT * MAXL))]


class Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("max_iters", C.c_int64), ("plateau", C.c_int64),
                ("target_rank", C.c_int32), ("r_cap", C.c_int32), ("flip_tries", C.c_int32),
                ("restart_from_best", C.c_int32), ("t_eq", C.c_uint64),
                ("t_reduce", C.c_uint64), ("t_expand", C.c_uint64), ("objective", C.c_int32),
                ("pad", C.c_int32)]


COUNTER_NAMES = ("iters", "flips", "attempts", "fallbacks", "dead_ends", "zero_removed",
                 "merges", "expands", "expand_fails", "restarts", "eq_accepts",
                 "improvements")


class Counters(C.Structure):
    _fields_ = [(name, C.c_int64) for name in COUNTER_NAMES]


class Walk(C.Structure):
    _fields_ = [("cur", Scheme), ("best", Scheme), ("start", Scheme),
                ("best_rank", C.c_int32), ("done", C.c_int32), ("best_nnz", C.c_int32),
                ("pad", C.c_int32), ("t", C.c_int64),
                ("plateau_start", C.c_int64), ("c", Counters), ("n_rec", C.c_int32),
                ("rec_iter", C.c_int64 * MAXREC), ("rec_rank", C.c_int32 * MAXREC)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER
        L.or_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.or_standard.argtypes = [P(Scheme), C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_brent_violations.argtypes = [P(Scheme)]
        L.or_brent_violations.restype = C.c_long
        L.or_naive_additions.argtypes = [P(Scheme)]
        L.or_naive_additions.restype = C.c_long
        L.or_nonzeros.argtypes = [P(Scheme)]
        L.or_nonzeros.restype = C.c_long
        L.or_swap_sizes.argtypes = [P(Scheme), P(Scheme)]
        L.or_merge.argtypes = [P(Scheme), P(Scheme), C.c_int, P(Scheme)]
        L.or_product.argtypes = [P(Scheme), P(Scheme), P(Scheme)]
        L.or_resize.argtypes = [P(Scheme), P(Scheme), C.c_int, C.c_uint64, C.c_int64,
                                C.c_uint64, C.c_int, P(Scheme)]
        L.or_lift.argtypes = [P(Scheme), C.c_int64, P(Scheme), P(C.c_int64)]
        L.or_normalise_term.argtypes = [P(Scheme), C.c_int]
        L.or_is_normalised.argtypes = [P(Scheme)]
        L.or_project.argtypes = [P(Scheme), C.c_int, C.c_int, P(Scheme)]
        L.or_extend.argtypes = [P(Scheme), C.c_int, P(Scheme)]
        L.or_full_reduce.argtypes = [P(Scheme)]
        L.or_walk_init.argtypes = [P(Walk), P(Scheme)]
        L.or_walk_run.argtypes = [P(Walk), P(Params), C.c_int64]
        L.or_run_many.argtypes = [P(Scheme), P(Params), C.c_uint64, C.c_int64, C.c_int,
                                  C.c_int64, C.c_int, P(Walk)]
        L.or_flip.argtypes = [P(Scheme), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_flip_valid.argtypes = [P(Scheme), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_plus.argtypes = [P(Scheme), C.c_int, C.c_int, C.c_int]
        L.or_split.argtypes = [P(Scheme), C.c_int, C.c_int, C.c_int]
        L.or_remove_zero_terms.argtypes = [P(Scheme)]
        L.or_ternary_add.argtypes = [P(C.c_int8), P(C.c_int8), C.c_int, C.c_int, C.c_int,
                                     P(C.c_int8)]
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# conversions
# --------------------------------------------------------------------------
def lengths(m, n, p):
    return m * n, n * p, p * m


def _factor_view(s: Scheme):
    return np.ctypeslib.as_array(s.f).reshape(3, MAXT, MAXL)


def to_c(U, V, W, m, n, p, z2=False) -> Scheme:
    U, V, W = (np.asarray(x, dtype=np.int8) for x in (U, V, W))
    r = U.shape[0]
    assert V.shape[0] == r and W.shape[0] == r and r <= MAXT
    lu, lv, lw = lengths(m, n, p)
    assert U.shape[1] == lu and V.shape[1] == lv and W.shape[1] == lw
    s = Scheme()
    s.m, s.n, s.p, s.r, s.z2 = m, n, p, r, int(bool(z2))
    f = _factor_view(s)
    f[0, :r, :lu] = U
    f[1, :r, :lv] = V
    f[2, :r, :lw] = W
    return s


def from_c(s: Scheme):
    """-> dict(m, n, p, r, z2, U, V, W) with copies of the live rows"""
    f = _factor_view(s)
    lu, lv, lw = lengths(s.m, s.n, s.p)
    r = s.r
    return dict(m=s.m, n=s.n, p=s.p, r=r, z2=bool(s.z2),
                U=f[0, :r, :lu].copy(), V=f[1, :r, :lv].copy(), W=f[2, :r, :lw].copy())


# --------------------------------------------------------------------------
# thin wrappers
# --------------------------------------------------------------------------
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox(c, k, o)
    return [int(x) for x in o]


def standard(m, n, p, z2=False) -> Scheme:
    s = Scheme()
    lib().or_standard(C.byref(s), m, n, p, int(bool(z2)))
    return s


def brent_violations(s: Scheme) -> int:
    return int(lib().or_brent_violations(C.byref(s)))


def naive_additions(s: Scheme) -> int:
    return int(lib().or_naive_additions(C.byref(s)))


def nonzeros(s: Scheme) -> int:
    return int(lib().or_nonzeros(C.byref(s)))


def swap_sizes(s: Scheme) -> Scheme:
    out = Scheme()
    lib().or_swap_sizes(C.byref(s), C.byref(out))
    return out


def merge(a: Scheme, b: Scheme, axis: int):
    out = Scheme()
    return out if lib().or_merge(C.byref(a), C.byref(b), axis, C.byref(out)) == 0 else None


def product(a: Scheme, b: Scheme):
    out = Scheme()
    return out if lib().or_product(C.byref(a), C.byref(b), C.byref(out)) == 0 else None


def lift(z2s: Scheme, max_nodes: int = 10 ** 7):
    """-> (status, ternary Scheme or None, nodes): 1 found, 0 none, -1 budget"""
    out = Scheme()
    nodes = C.c_int64(0)
    st = lib().or_lift(C.byref(z2s), int(max_nodes), C.byref(out), C.byref(nodes))
    return st, (out if st == 1 else None), int(nodes.value)


def resize(s: Scheme, best, seed: int, rnd: int, t_resize: int, cap: int):
    """-> (operators applied as bits, new scheme); best: list of Schemes"""
    arr = (Scheme * max(len(best), 1))(*best) if best else (Scheme * 1)()
    out = Scheme()
    bits = lib().or_resize(C.byref(s), arr, len(best), seed, rnd, t_resize, cap, C.byref(out))
    return bits, out


def is_normalised(s: Scheme) -> bool:
    return bool(lib().or_is_normalised(C.byref(s)))


def normalise(s: Scheme) -> Scheme:
    for l in range(s.r):
        lib().or_normalise_term(C.byref(s), l)
    return s


def project(s: Scheme, axis: int, index: int) -> Scheme:
    out = Scheme()
    rc = lib().or_project(C.byref(s), axis, index, C.byref(out))
    if rc != 0:
        raise ValueError("project refused")
    return out


def extend(s: Scheme, axis: int) -> Scheme:
    out = Scheme()
    rc = lib().or_extend(C.byref(s), axis, C.byref(out))
    if rc != 0:
        raise ValueError("extend refused")
    return out


def full_reduce(s: Scheme) -> int:
    return int(lib().or_full_reduce(C.byref(s)))


def copy(s: Scheme) -> Scheme:
    t = Scheme()
    C.memmove(C.byref(t), C.byref(s), C.sizeof(Scheme))
    return t


def make_params(seed=0, max_iters=100000, plateau=20000, target_rank=0, r_cap=None,
                flip_tries=7, restart_from_best=0, t_eq=42949673, t_reduce=1 << 32,
                t_expand=0, r0=None, objective=0):
    if r_cap is None:
        r_cap = (r0 or 0) + 8
    return Params(seed, max_iters, plateau, target_rank, r_cap, flip_tries,
                  restart_from_best, t_eq, t_reduce, t_expand, objective, 0)


def new_walk(start: Scheme) -> Walk:
    w = Walk()
    lib().or_walk_init(C.byref(w), C.byref(start))
    return w


def run(w: Walk, prm: Params, n_iters: int) -> Walk:
    lib().or_walk_run(C.byref(w), C.byref(prm), int(n_iters))
    return w


def run_many(start: Scheme, prm: Params, base_seed: int, first_walk: int, n_walks: int,
             n_iters: int, n_threads: int = 1):
    out = (Walk * n_walks)()
    lib().or_run_many(C.byref(start), C.byref(prm), base_seed, first_walk, n_walks,
                      n_iters, n_threads, out)
    return out


def counters(w: Walk) -> dict:
    return {name: int(getattr(w.c, name)) for name in COUNTER_NAMES}


def records(w: Walk):
    n = min(w.n_rec, MAXREC)
    return [(int(w.rec_iter[q]), int(w.rec_rank[q])) for q in range(n)]


def flip_valid(s: Scheme, i, j, X, sigma, role) -> bool:
    return bool(lib().or_flip_valid(C.byref(s), i, j, X, sigma, role))


def flip(s: Scheme, i, j, X, sigma, role) -> bool:
    return bool(lib().or_flip(C.byref(s), i, j, X, sigma, role))


def plus(s: Scheme, i, j, perm) -> bool:
    return bool(lib().or_plus(C.byref(s), int(i), int(j), int(perm)))


def split(s: Scheme, i, j, perm) -> bool:
    return bool(lib().or_split(C.byref(s), int(i), int(j), int(perm)))


def remove_zero_terms(s: Scheme) -> int:
    return int(lib().or_remove_zero_terms(C.byref(s)))


class Log(C.Structure):
    _fields_ = [("iter", C.c_int64), ("rank_before", C.c_int32), ("rank_after", C.c_int32),
                ("format_slot", C.c_int32), ("reserved", C.c_int32), ("f", C.c_uint64 * 12),
                ("pad", C.c_uint64)]


def _bind_learned():
    L = lib()
    if not getattr(L, "_learned_bound", False):
        P = C.POINTER
        L.or_walk_run_logged.argtypes = [P(Walk), P(Params), C.c_int64, P(Log), C.c_int64,
                                         C.c_int32]
        L.or_walk_run_choices.argtypes = [P(Walk), P(Params), C.c_int64, P(C.c_uint8), C.c_int64,
                                          P(C.c_int64)]
        L.or_attempt_candidate.argtypes = [P(Scheme), C.c_uint64, C.c_int64, C.c_int,
                                           P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int)]
        L._learned_bound = True
    return L


def run_logged(w: Walk, prm: Params, n_iters: int, log_cap: int, format_slot: int):
    logs = (Log * max(log_cap, 1))()
    _bind_learned().or_walk_run_logged(C.byref(w), C.byref(prm), n_iters, logs, log_cap,
                                       format_slot)
    return logs


def run_choices(w: Walk, prm: Params, n_iters: int, choices):
    arr = np.ascontiguousarray(choices, dtype=np.uint8)
    bad = C.c_int64(0)
    _bind_learned().or_walk_run_choices(C.byref(w), C.byref(prm), n_iters,
                                        arr.ctypes.data_as(C.POINTER(C.c_uint8)), arr.size,
                                        C.byref(bad))
    return int(bad.value)


def attempt_candidate(s: Scheme, seed: int, t: int, a: int):
    """-> None or (n, i, j, X, role)"""
    i, j, X, role = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    n = _bind_learned().or_attempt_candidate(C.byref(s), seed, t, a, C.byref(i), C.byref(j),
                                             C.byref(X), C.byref(role))
    if n == 0:
        return None
    return n, i.value, j.value, X.value, role.value
