"""ctypes binding of libtsf (include/tsf.h): argument marshalling only.

Every step of the walk runs in libtsf's HIP kernels; torch is used for device
memory and streams.  If libtsf.so is missing the import fails loudly: there is
no fallback path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsf.so")

TSF_TERNARY = 0
TSF_Z2 = 1
OBJ_RANK = 0
OBJ_ADDITIONS = 1
ALWAYS = 1 << 32                # Bernoulli threshold of probability 1
EQ_ACCEPT = 42949673            # round(0.01 * 2^32): Algorithm 1's 1% equal-rank acceptance

STATUS = {0: "TSF_OK", -1: "TSF_E_ARG", -2: "TSF_E_FORMAT", -3: "TSF_E_CAPACITY",
          -4: "TSF_E_NOT_TERNARY", -5: "TSF_E_INVALID_SCHEME", -6: "TSF_E_DEVICE",
          -7: "TSF_E_STATE"}
TSF_E_ARG, TSF_E_FORMAT, TSF_E_CAPACITY = -1, -2, -3
TSF_E_NOT_TERNARY, TSF_E_INVALID_SCHEME, TSF_E_DEVICE = -4, -5, -6
TSF_E_STATE = -7
# invariant checks of tsf_walk_checked (bits of the error word in a header's
# `reserved` when done = -4)
CHECK_RANK = 1
CHECK_ZERO_FACTOR = 2
CHECK_CODING = 4
CHECK_NORMALISED = 8
CHECK_INDEX = 16
CHECK_DEAD_SLOTS = 32
DONE_CHECK_FAILED = -4

COUNTER_NAMES = ("iters", "flips", "attempts", "fallbacks", "dead_ends", "zero_removed",
                 "merges", "expands", "expand_fails", "restarts", "eq_accepts",
                 "improvements")


class TsfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Dims(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("p", C.c_int32), ("rank", C.c_int32),
                ("capacity", C.c_int32), ("mode", C.c_int32)]


class CScheme(C.Structure):
    _fields_ = [("d", Dims), ("U", C.POINTER(C.c_int8)), ("V", C.POINTER(C.c_int8)),
                ("W", C.POINTER(C.c_int8))]


class WalkParams(C.Structure):
    _fields_ = [("base_seed", C.c_uint64), ("first_walk_id", C.c_int64),
                ("max_iters", C.c_int64), ("plateau", C.c_int64), ("flip_tries", C.c_int32),
                ("restart_from_best", C.c_int32), ("t_eq", C.c_uint64),
                ("t_reduce", C.c_uint64), ("t_expand", C.c_uint64), ("objective", C.c_int32),
                ("reserved", C.c_int32)]


class WalkBatchC(C.Structure):
    _fields_ = [("n_walks", C.c_int32), ("capacity", C.c_int32), ("rec_cap", C.c_int32),
                ("mode", C.c_int32), ("max_len", C.c_int32), ("reserved", C.c_int32),
                ("hdr", C.c_void_p), ("cur", C.c_void_p), ("best", C.c_void_p),
                ("start", C.c_void_p), ("rec", C.c_void_p), ("log", C.c_void_p),
                ("log_cap", C.c_int32), ("reserved2", C.c_int32)]


class LearnWsC(C.Structure):
    _fields_ = [("cand", C.c_void_p), ("feat", C.c_void_p), ("h1", C.c_void_p),
                ("h2", C.c_void_p), ("logit", C.c_void_p), ("choice", C.c_void_p),
                ("choice_cap", C.c_int32), ("reserved", C.c_int32)]


class InvariantsC(C.Structure):
    _fields_ = [("rank_sum", C.c_int32 * 3), ("type_poly", C.c_int32 * 729),
                ("sym_poly", C.c_int32 * 729)]


class ResizeParams(C.Structure):
    _fields_ = [("base_seed", C.c_uint64), ("first_walk_id", C.c_int64), ("round", C.c_int64),
                ("t_resize", C.c_uint64), ("r_cap_extra", C.c_int32), ("reserved", C.c_int32)]


BEST_ENTRY_DTYPE = np.dtype([("m", "<i4"), ("n", "<i4"), ("p", "<i4"), ("rank", "<i4"),
                             ("walk", "<i8")])


class LiftResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("prefix_terms", C.c_int32), ("subtrees", C.c_int64),
                ("exhausted", C.c_int64), ("subtree", C.c_int64)]


class Launch(C.Structure):
    _fields_ = [("lanes_per_walk", C.c_int32), ("waves_per_block", C.c_int32),
                ("strategy", C.c_int32)]


class MlpC(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("adam_m", C.c_void_p),
                ("adam_v", C.c_void_p), ("wbf", C.c_void_p)]


MLP_IN, MLP_HID, MLP_NPARAM, MLP_NBF16 = 512, 256, 197380, 262400


# numpy view of tsf_walk_header (176 bytes)
HEADER_DTYPE = np.dtype([("m", "<i4"), ("n", "<i4"), ("p", "<i4"), ("mode", "<i4"),
                         ("r_cap", "<i4"), ("target_rank", "<i4"), ("rank", "<i4"),
                         ("best_rank", "<i4"), ("start_rank", "<i4"), ("done", "<i4"),
                         ("n_rec", "<i4"), ("best_nnz", "<i4"), ("t", "<i8"),
                         ("plateau_start", "<i8"), ("counters", "<i8", (12,)),
                         ("params_hash", "<u8"), ("reserved", "<u8")])
assert HEADER_DTYPE.itemsize == 176
HEADER_I32 = HEADER_DTYPE.itemsize // 4   # int32 columns of a header (views of hdr)
RECORD_DTYPE = np.dtype([("iter", "<i8"), ("rank", "<i4"), ("reserved", "<i4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtsf.so is not built (run paper_2511_20317_amd/build.py); "
                              "there is no fallback implementation")
        # torch ships its own HIP runtime; loading it first lets libtsf bind to
        # that same runtime instead of pulling a second copy into the process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.tsf_last_error.restype = C.c_char_p
        for name, args in [
            ("tsf_init_scheme", [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(CScheme)]),
            ("tsf_verify", [P(CScheme), P(C.c_int64)]),
            ("tsf_normalise", [P(CScheme)]),
            ("tsf_reduce", [P(CScheme), P(C.c_int32)]),
            ("tsf_meta_project", [P(CScheme), C.c_int32, C.c_int32, P(CScheme)]),
            ("tsf_meta_extend", [P(CScheme), C.c_int32, P(CScheme)]),
            ("tsf_pack", [P(CScheme), C.c_void_p]),
            ("tsf_unpack", [C.c_void_p, P(Dims), P(CScheme)]),
            ("tsf_ctx_create", [P(C.c_void_p)]),
            ("tsf_ctx_destroy", [C.c_void_p]),
            ("tsf_walk_init", [C.c_void_p, P(WalkBatchC), C.c_void_p]),
            ("tsf_autotune", [C.c_void_p, P(WalkParams), P(WalkBatchC), C.c_int64, P(Launch),
                              C.c_void_p]),
            ("tsf_walk", [C.c_void_p, P(WalkParams), P(WalkBatchC), C.c_int64, P(Launch),
                          C.c_void_p]),
            ("tsf_walk_checked", [C.c_void_p, P(WalkParams), P(WalkBatchC), C.c_int64,
                                  P(Launch), C.c_void_p]),
            ("tsf_verify_batch", [P(WalkBatchC), C.c_int32, C.c_void_p, C.c_void_p]),
            ("tsf_mlp_sync", [P(MlpC), C.c_void_p]),
            ("tsf_mlp_fwd", [P(MlpC), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
            ("tsf_mlp_bwd", [P(MlpC), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
            ("tsf_mlp_step", [P(MlpC), C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32,
                              C.c_void_p]),
            ("tsf_features_from_log", [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
            ("tsf_walk_learned", [C.c_void_p, P(WalkParams), P(WalkBatchC), P(MlpC), P(LearnWsC),
                                  C.c_int64, P(Launch), C.c_void_p]),
            ("tsf_format_slot", [C.c_int32, C.c_int32, C.c_int32]),
            ("tsf_walk_check", [P(WalkParams), C.c_void_p, C.c_int32, P(C.c_int32)]),
            ("tsf_state_check", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_int32, C.c_int32, P(C.c_int32)]),
            ("tsf_scheme_invariants", [P(CScheme), C.c_void_p, P(InvariantsC)]),
            ("tsf_meta_swap", [P(CScheme), P(CScheme)]),
            ("tsf_lift", [P(CScheme), C.c_int64, C.c_int32, P(CScheme), P(LiftResultC)]),
            ("tsf_meta_merge", [P(CScheme), P(CScheme), C.c_int32, P(CScheme)]),
            ("tsf_meta_product", [P(CScheme), P(CScheme), P(CScheme)]),
            ("tsf_population_best", [P(WalkBatchC), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int32, C.c_void_p]),
            ("tsf_population_best_noalloc", [P(WalkBatchC), C.c_void_p, C.c_void_p,
                                             C.c_int32, C.c_void_p, C.c_void_p]),
            ("tsf_resize_batch", [P(WalkBatchC), C.c_int32, C.c_void_p, C.c_void_p,
                                  P(ResizeParams), P(WalkBatchC), C.c_void_p, C.c_void_p]),
            ("tsf_invariants_batch", [P(WalkBatchC), C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
            ("tsf_meta_batch", [P(WalkBatchC), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int32, P(WalkBatchC), C.c_void_p]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.tsf_params_hash.argtypes = [P(WalkParams)]
        L.tsf_params_hash.restype = C.c_uint64
        _lib = L
    return _lib


def check(status):
    if status != 0:
        raise TsfError(status, lib().tsf_last_error().decode())
    return status


# ---------------------------------------------------------------------------
# host schemes
# ---------------------------------------------------------------------------
class Scheme:
    """A scheme (m,n,p:r) in the int8 interchange form of tsf.h."""

    def __init__(self, m, n, p, U, V, W, mode=TSF_TERNARY, capacity=None):
        self.m, self.n, self.p, self.mode = int(m), int(n), int(p), int(mode)
        r = int(np.asarray(U).shape[0])
        self.capacity = max(int(capacity or r), r, 1)
        lu, lv, lw = m * n, n * p, p * m
        self.U = np.zeros((self.capacity, lu), np.int8)
        self.V = np.zeros((self.capacity, lv), np.int8)
        self.W = np.zeros((self.capacity, lw), np.int8)
        self.U[:r] = U
        self.V[:r] = V
        self.W[:r] = W
        self.rank = r

    @classmethod
    def empty(cls, m, n, p, capacity, mode=TSF_TERNARY):
        s = cls(m, n, p, np.zeros((0, m * n)), np.zeros((0, n * p)), np.zeros((0, p * m)),
                mode, capacity)
        return s

    def c(self):
        cs = CScheme()
        cs.d = Dims(self.m, self.n, self.p, self.rank, self.capacity, self.mode)
        cs.U = self.U.ctypes.data_as(C.POINTER(C.c_int8))
        cs.V = self.V.ctypes.data_as(C.POINTER(C.c_int8))
        cs.W = self.W.ctypes.data_as(C.POINTER(C.c_int8))
        return cs

    def _take(self, cs):
        self.m, self.n, self.p = cs.d.m, cs.d.n, cs.d.p
        self.rank, self.mode = cs.d.rank, cs.d.mode

    def live(self):
        """(U, V, W) of the live terms"""
        r = self.rank
        return self.U[:r].copy(), self.V[:r].copy(), self.W[:r].copy()

    def copy(self):
        return Scheme(self.m, self.n, self.p, *self.live(), self.mode, self.capacity)


def init_scheme(m, n, p, mode=TSF_TERNARY, capacity=None):
    s = Scheme.empty(m, n, p, capacity or m * n * p, mode)
    cs = s.c()
    check(lib().tsf_init_scheme(m, n, p, mode, C.byref(cs)))
    s._take(cs)
    return s


def verify(s: Scheme) -> int:
    out = C.c_int64()
    check(lib().tsf_verify(C.byref(s.c()), C.byref(out)))
    return int(out.value)


def normalise(s: Scheme) -> Scheme:
    cs = s.c()
    check(lib().tsf_normalise(C.byref(cs)))
    s._take(cs)
    return s


def reduce(s: Scheme) -> int:
    cs = s.c()
    n = C.c_int32()
    check(lib().tsf_reduce(C.byref(cs), C.byref(n)))
    s._take(cs)
    return int(n.value)


def meta_project(s: Scheme, axis: int, index: int, capacity=None) -> Scheme:
    out = Scheme.empty(1, 1, 1, 1)
    dims = [s.m, s.n, s.p]
    dims[axis] -= 1 if dims[axis] > 1 else 0
    out = Scheme.empty(*dims, capacity or s.capacity, s.mode)
    cs = out.c()
    check(lib().tsf_meta_project(C.byref(s.c()), axis, index, C.byref(cs)))
    out._take(cs)
    return out


def meta_extend(s: Scheme, axis: int, capacity=None) -> Scheme:
    dims = [s.m, s.n, s.p]
    dims[axis] += 1
    extra = [s.n * s.p, s.m * s.p, s.m * s.n][axis]
    out = Scheme.empty(*dims, capacity or (s.rank + extra), s.mode)
    cs = out.c()
    check(lib().tsf_meta_extend(C.byref(s.c()), axis, C.byref(cs)))
    out._take(cs)
    return out


def meta_swap(s: Scheme) -> Scheme:
    """(m,n,p:r) -> (m,p,n:r) (tsf_meta_swap)."""
    out = Scheme.empty(s.m, s.p, s.n, max(s.rank, 1), s.mode)
    cs = out.c()
    check(lib().tsf_meta_swap(C.byref(s.c()), C.byref(cs)))
    out._take(cs)
    return out


def meta_merge(a: Scheme, b: Scheme, axis: int) -> Scheme:
    """Merge along axis 0 (m), 1 (n) or 2 (p) (tsf_meta_merge)."""
    dims = [a.m, a.n, a.p]
    dims[axis] += [b.m, b.n, b.p][axis]
    out = Scheme.empty(*dims, max(a.rank + b.rank, 1), a.mode)
    cs = out.c()
    check(lib().tsf_meta_merge(C.byref(a.c()), C.byref(b.c()), axis, C.byref(cs)))
    out._take(cs)
    return out


def meta_product(a: Scheme, b: Scheme) -> Scheme:
    """Kronecker product of two schemes (tsf_meta_product)."""
    out = Scheme.empty(a.m * b.m, a.n * b.n, a.p * b.p, max(a.rank * b.rank, 1), a.mode)
    cs = out.c()
    check(lib().tsf_meta_product(C.byref(a.c()), C.byref(b.c()), C.byref(cs)))
    out._take(cs)
    return out


def lift(z2: Scheme, max_nodes=1 << 20, max_subtrees=1 << 16):
    """Ternary lifting of a Z2 scheme on the GPU (tsf_lift): returns (result
    dict, ternary Scheme or None)."""
    out = Scheme.empty(z2.m, z2.n, z2.p, max(z2.rank, 1), TSF_TERNARY)
    cs = out.c()
    res = LiftResultC()
    check(lib().tsf_lift(C.byref(z2.c()), int(max_nodes), int(max_subtrees), C.byref(cs),
                         C.byref(res)))
    info = {k: int(getattr(res, k)) for k, _ in LiftResultC._fields_}
    if res.status in (1, 2):
        out._take(cs)
        return info, out
    return info, None


def _poly(arr):
    a = np.ctypeslib.as_array(arr).reshape(9, 9, 9)
    return {tuple(int(x) for x in idx): int(a[idx]) for idx in zip(*np.nonzero(a))}


def scheme_invariants(s: Scheme) -> dict:
    """Isotropy invariants (Sec. 3.7): per-term factor ranks, the type and
    symmetric polynomials ({(a, b, c): coefficient}) and the rank-sum
    exponents."""
    out = InvariantsC()
    ranks = np.zeros((max(s.rank, 1), 3), np.uint8)
    check(lib().tsf_scheme_invariants(C.byref(s.c()), C.c_void_p(ranks.ctypes.data),
                                      C.byref(out)))
    return {"term_ranks": [tuple(int(x) for x in r) for r in ranks[:s.rank]],
            "type": _poly(out.type_poly), "symmetric": _poly(out.sym_poly),
            "rank_sum": tuple(int(x) for x in out.rank_sum)}


def pack(s: Scheme, capacity=None) -> np.ndarray:
    """-> uint64 array (capacity, 6) in the one-bit form"""
    cap = capacity or s.capacity
    if cap < s.rank:
        raise ValueError("capacity below rank")
    tmp = Scheme(s.m, s.n, s.p, *s.live(), s.mode, cap)
    out = np.zeros((cap, 6), np.uint64)
    check(lib().tsf_pack(C.byref(tmp.c()), out.ctypes.data_as(C.c_void_p)))
    return out


def unpack(packed, m, n, p, rank, mode=TSF_TERNARY) -> Scheme:
    packed = np.ascontiguousarray(packed, dtype=np.uint64).reshape(-1, 6)
    cap = max(packed.shape[0], 1)
    out = Scheme.empty(m, n, p, cap, mode)
    d = Dims(m, n, p, rank, cap, mode)
    cs = out.c()
    check(lib().tsf_unpack(packed.ctypes.data_as(C.c_void_p), C.byref(d), C.byref(cs)))
    out._take(cs)
    return out


# ---------------------------------------------------------------------------
# walks on the GPU
# ---------------------------------------------------------------------------
def walk_params(base_seed=0, first_walk_id=0, max_iters=100000, plateau=20000, flip_tries=7,
                restart_from_best=0, t_eq=EQ_ACCEPT, t_reduce=ALWAYS, t_expand=0,
                objective=0):
    """objective: OBJ_RANK (Algorithm 1) or OBJ_ADDITIONS (naive additions at a
    fixed rank; target_rank of the batch is then the target additions)."""
    return WalkParams(base_seed, first_walk_id, max_iters, plateau, flip_tries,
                      restart_from_best, t_eq, t_reduce, t_expand, objective, 0)


def params_hash(prm: WalkParams) -> int:
    return int(lib().tsf_params_hash(C.byref(prm)))


def walk_check(prm: WalkParams, headers: np.ndarray):
    """tsf_walk_check on host headers (HEADER_DTYPE); returns the status
    (0 or TSF_E_STATE) and leaves the count in walk_check.mismatched."""
    h = np.ascontiguousarray(headers, dtype=HEADER_DTYPE)
    n = C.c_int32(0)
    st = lib().tsf_walk_check(C.byref(prm), h.ctypes.data_as(C.c_void_p), int(h.size),
                              C.byref(n))
    walk_check.mismatched = int(n.value)
    return st


def state_check(headers, cur, best, start, capacity, brent=True):
    """tsf_state_check on host copies of a batch's state: returns (status,
    first failing walk or -1)."""
    h = np.ascontiguousarray(headers, dtype=HEADER_DTYPE)
    bufs = [np.ascontiguousarray(x).view(np.uint64) for x in (cur, best, start)]
    first = C.c_int32(-1)
    st = lib().tsf_state_check(h.ctypes.data_as(C.c_void_p),
                               *[b.ctypes.data_as(C.c_void_p) for b in bufs], int(h.size),
                               int(capacity), 1 if brent else 0, C.byref(first))
    return st, int(first.value)


CHECKPOINT_MAGIC = "tsf-walk-batch"
CHECKPOINT_VERSION = 1


class Context:
    def __init__(self):
        self.ptr = C.c_void_p()
        check(lib().tsf_ctx_create(C.byref(self.ptr)))

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.tsf_ctx_destroy(self.ptr)
            self.ptr = None


class WalkBatch:
    """Device buffers of a batch of walks (torch tensors as plain memory).

    groups: list of (start_scheme, n_walks, r_cap, target_rank); walks are laid
    out group after group.  All groups share one mode.
    """

    def __init__(self, groups, capacity=None, rec_cap=64, device="cuda", log_cap=0):
        import torch
        self.torch = torch
        self.log_cap = int(log_cap)
        modes = {g[0].mode for g in groups}
        if len(modes) != 1:
            raise ValueError("one mode per batch")
        self.mode = modes.pop()
        self.n_walks = int(sum(g[1] for g in groups))
        self.capacity = int(capacity or max(g[2] for g in groups))
        self.rec_cap = int(rec_cap)
        self.max_len = max(max(s.m * s.n, s.n * s.p, s.p * s.m) for s, _, _, _ in groups)
        hdr = np.zeros(self.n_walks, HEADER_DTYPE)
        start = np.zeros((self.n_walks, self.capacity, 6), np.uint64)
        w = 0
        self.groups = []
        for s, nw, r_cap, target in groups:
            if r_cap > self.capacity or s.rank > r_cap:
                raise ValueError("need start rank <= r_cap <= capacity")
            ns = normalise(s.copy())
            packed = pack(ns, self.capacity)
            hdr["m"][w:w + nw], hdr["n"][w:w + nw], hdr["p"][w:w + nw] = s.m, s.n, s.p
            hdr["mode"][w:w + nw] = s.mode
            hdr["r_cap"][w:w + nw] = r_cap
            hdr["target_rank"][w:w + nw] = target
            hdr["start_rank"][w:w + nw] = s.rank
            start[w:w + nw] = packed
            self.groups.append((w, nw, (s.m, s.n, s.p), r_cap, target))
            w += nw
        dev = torch.device(device)
        self.hdr = torch.from_numpy(hdr.view(np.uint8).copy()).to(dev)
        self.start = torch.from_numpy(start.view(np.int64)).to(dev)
        self.cur = torch.zeros_like(self.start)
        self.best = torch.zeros_like(self.start)
        self.rec = torch.zeros((self.n_walks, max(self.rec_cap, 1), 2), dtype=torch.int64,
                               device=dev)
        self.log = (torch.zeros((self.n_walks, self.log_cap, 16), dtype=torch.int64, device=dev)
                    if self.log_cap else None)

    @classmethod
    def empty(cls, n_walks, capacity, mode, max_len, rec_cap=64, device="cuda", log_cap=0):
        """Buffers for n_walks walks with no start schemes yet (see meta_from)."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.log_cap = int(log_cap)
        self.mode, self.n_walks, self.capacity = int(mode), int(n_walks), int(capacity)
        self.rec_cap, self.max_len = int(rec_cap), int(max_len)
        self.groups = []
        dev = torch.device(device)
        self.hdr = torch.zeros(self.n_walks * HEADER_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self.start = torch.zeros((self.n_walks, self.capacity, 6), dtype=torch.int64, device=dev)
        self.cur = torch.zeros_like(self.start)
        self.best = torch.zeros_like(self.start)
        self.rec = torch.zeros((self.n_walks, max(self.rec_cap, 1), 2), dtype=torch.int64,
                               device=dev)
        self.log = (torch.zeros((self.n_walks, self.log_cap, 16), dtype=torch.int64, device=dev)
                    if self.log_cap else None)
        return self

    def meta_from(self, src, which, op, axis, index, r_cap_extra=8):
        """Start schemes of this batch := project / extend / copy of src's
        current (which=0) or best (which=1) schemes (tsf_meta_batch); then init."""
        torch = self.torch
        dev = self.hdr.device
        op_d = torch.as_tensor(np.asarray(op, np.int32)).to(dev)
        ax_d = torch.as_tensor(np.asarray(axis, np.int32)).to(dev)
        ix_d = torch.as_tensor(np.asarray(index, np.int32)).to(dev)
        check(lib().tsf_meta_batch(C.byref(src.c()), which, C.c_void_p(op_d.data_ptr()),
                                   C.c_void_p(ax_d.data_ptr()), C.c_void_p(ix_d.data_ptr()),
                                   r_cap_extra, C.byref(self.c()), self._stream()))

    def c(self):
        return WalkBatchC(self.n_walks, self.capacity, self.rec_cap, self.mode, self.max_len, 0,
                          self.hdr.data_ptr(), self.cur.data_ptr(), self.best.data_ptr(),
                          self.start.data_ptr(), self.rec.data_ptr(),
                          self.log.data_ptr() if self.log is not None else None,
                          self.log_cap, 0)

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def init(self, ctx: Context):
        check(lib().tsf_walk_init(ctx.ptr, C.byref(self.c()), self._stream()))

    def walk(self, ctx: Context, prm: WalkParams, n_iters: int, lanes_per_walk=0,
             waves_per_block=0, strategy=0, checked=False):
        """tsf_walk, or tsf_walk_checked with checked=True (invariants checked
        after every iteration; a failing walk stops with done = -4)."""
        la = Launch(lanes_per_walk, waves_per_block, strategy)
        fn = lib().tsf_walk_checked if checked else lib().tsf_walk
        check(fn(ctx.ptr, C.byref(prm), C.byref(self.c()), int(n_iters), C.byref(la),
                 self._stream()))

    def check_resume(self, prm: WalkParams):
        """tsf_walk_check on a host copy of the headers: raises TsfError
        (TSF_E_STATE) if some walk was run with other walk parameters."""
        h = np.ascontiguousarray(self.headers())
        check(walk_check(prm, h))

    def autotune(self, ctx: Context, prm: WalkParams, trial_iters=200):
        """Time every launch configuration on a copy of the state; returns the
        chosen (lanes_per_walk, waves_per_block, strategy)."""
        la = Launch()
        check(lib().tsf_autotune(ctx.ptr, C.byref(prm), C.byref(self.c()), int(trial_iters),
                                 C.byref(la), self._stream()))
        return la.lanes_per_walk, la.waves_per_block, la.strategy

    def walk_learned(self, ctx: Context, prm: WalkParams, net, ws, n_iters: int,
                     lanes_per_walk=0, waves_per_block=0):
        la = Launch(lanes_per_walk, waves_per_block, 1)
        check(lib().tsf_walk_learned(ctx.ptr, C.byref(prm), C.byref(self.c()), C.byref(net.c()),
                                     C.byref(ws.c()), int(n_iters), C.byref(la), self._stream()))

    def invariants(self, which=1):
        """Factor ranks of every live term (uint8, n_walks x capacity x 3; zero
        past a scheme's rank) and their sums (int32, n_walks x 3) of the cur (0),
        best (1) or start (2) scheme of every walk, on the GPU."""
        torch = self.torch
        ranks = torch.zeros((self.n_walks, self.capacity, 3), dtype=torch.uint8,
                            device=self.hdr.device)
        sums = torch.empty((self.n_walks, 3), dtype=torch.int32, device=self.hdr.device)
        check(lib().tsf_invariants_batch(C.byref(self.c()), which, C.c_void_p(ranks.data_ptr()),
                                         C.c_void_p(sums.data_ptr()), self._stream()))
        return ranks, sums

    def population_best(self, slots=4096):
        """Per distinct format, the walk with the best rank (ties: lowest id),
        ascending (m, n, p): (device table of BEST_ENTRY_DTYPE records as a
        uint8 tensor, device int32 count) -- tsf_population_best."""
        torch = self.torch
        dev = self.hdr.device
        table = torch.zeros(slots * BEST_ENTRY_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        count = torch.zeros(1, dtype=torch.int32, device=dev)
        work = torch.empty(2 * slots + 1, dtype=torch.int64, device=dev)
        check(lib().tsf_population_best(C.byref(self.c()), C.c_void_p(table.data_ptr()),
                                        C.c_void_p(count.data_ptr()),
                                        C.c_void_p(work.data_ptr()), slots, self._stream()))
        return table, count

    def population_best_noalloc(self, table, count, slots=4096, dropped=None):
        """tsf_population_best into caller-owned device buffers, with the
        library's fixed working memory instead of a workspace: table (uint8,
        >= slots entries of BEST_ENTRY_DTYPE), count (int32, 1), dropped
        (optional int32, 1)."""
        check(lib().tsf_population_best_noalloc(
            C.byref(self.c()), C.c_void_p(table.data_ptr()), C.c_void_p(count.data_ptr()), slots,
            C.c_void_p(dropped.data_ptr() if dropped is not None else None), self._stream()))
        return table, count

    def resize_into(self, out, table, count, base_seed, rnd, t_resize=ALWAYS, which=1,
                    r_cap_extra=8, first_walk_id=0):
        """Algorithm 2 on every walk into batch `out` (tsf_resize_batch); then
        out.init.  Returns the device tensor of operator bits per walk."""
        torch = self.torch
        applied = torch.empty(self.n_walks, dtype=torch.int32, device=self.hdr.device)
        prm = ResizeParams(base_seed, first_walk_id, rnd, t_resize, r_cap_extra, 0)
        check(lib().tsf_resize_batch(C.byref(self.c()), which, C.c_void_p(table.data_ptr()),
                                     C.c_void_p(count.data_ptr()), C.byref(prm),
                                     C.byref(out.c()), C.c_void_p(applied.data_ptr()),
                                     self._stream()))
        return applied

    def verify_device(self, which=1):
        """Brent check of cur (0), best (1) or start (2) of every walk on the GPU."""
        out = self.torch.empty(self.n_walks, dtype=self.torch.int64, device=self.hdr.device)
        check(lib().tsf_verify_batch(C.byref(self.c()), which, C.c_void_p(out.data_ptr()),
                                     self._stream()))
        return out

    # ------------------------------------------------------------ checkpoints
    def save(self, path, prm: WalkParams = None):
        """Write the batch's whole walk state (headers, current, best and start
        schemes, records) to `path` (a numpy .npz archive, versioned; no
        pickled objects).  With `prm`, its tsf_params_hash is stored too."""
        torch = self.torch
        torch.cuda.synchronize() if self.hdr.is_cuda else None
        np.savez(path, magic=np.array(CHECKPOINT_MAGIC), version=np.int32(CHECKPOINT_VERSION),
                 mode=np.int32(self.mode), capacity=np.int32(self.capacity),
                 rec_cap=np.int32(self.rec_cap), max_len=np.int32(self.max_len),
                 params_hash=np.uint64(params_hash(prm) if prm is not None else 0),
                 hdr=self.headers(), cur=self.cur.cpu().numpy(), best=self.best.cpu().numpy(),
                 start=self.start.cpu().numpy(), rec=self.rec.cpu().numpy())

    @classmethod
    def load(cls, path, prm: WalkParams = None, device="cuda", brent=None):
        """A batch from a checkpoint written by save(), refused (TsfError) when
        it is not one (TSF_E_STATE: magic or version), when its state is
        damaged (tsf_state_check: TSF_E_FORMAT, TSF_E_CAPACITY,
        TSF_E_NOT_TERNARY, TSF_E_INVALID_SCHEME), or, with `prm`, when its
        walks were run with other walk parameters (TSF_E_STATE).  brent: check
        the Brent equations of every scheme -- on the host (default on a CPU
        device) or, on a GPU, with tsf_verify_batch (default there)."""
        z = np.load(path, allow_pickle=False)
        if "magic" not in z or str(z["magic"]) != CHECKPOINT_MAGIC:
            raise TsfError(TSF_E_STATE, "%s is not a walk-batch checkpoint" % path)
        if int(z["version"]) != CHECKPOINT_VERSION:
            raise TsfError(TSF_E_STATE, "checkpoint version %d, expected %d"
                           % (int(z["version"]), CHECKPOINT_VERSION))
        hdr = np.ascontiguousarray(z["hdr"]).view(HEADER_DTYPE)
        cap = int(z["capacity"])
        cur, best, start = (np.ascontiguousarray(z[k]) for k in ("cur", "best", "start"))
        n = int(hdr.size)
        if any(x.shape != (n, cap, 6) for x in (cur, best, start)):
            raise TsfError(TSF_E_STATE, "checkpoint arrays do not match %d walks x %d terms"
                           % (n, cap))
        on_gpu = str(device).startswith("cuda")
        host_brent = (not on_gpu) if brent is None else (brent and not on_gpu)
        st, first = state_check(hdr, cur, best, start, cap, brent=host_brent)
        if st:
            raise TsfError(st, "walk %d of %s: %s" % (first, path,
                                                      lib().tsf_last_error().decode()))
        if prm is not None:
            check(walk_check(prm, hdr))
        b = cls.empty(n, cap, int(z["mode"]), int(z["max_len"]), rec_cap=int(z["rec_cap"]),
                      device=device)
        torch = b.torch
        b.hdr.copy_(torch.from_numpy(hdr.view(np.uint8).reshape(-1).copy()))
        for name, arr in (("cur", cur), ("best", best), ("start", start)):
            getattr(b, name).copy_(torch.from_numpy(arr.view(np.int64)))
        b.rec.copy_(torch.from_numpy(np.ascontiguousarray(z["rec"])))
        if on_gpu and (brent is None or brent):
            live = torch.from_numpy(hdr["done"] >= 0).to(b.hdr.device)
            for which, label in ((0, "current"), (1, "best"), (2, "start")):
                bad = (b.verify_device(which) != 0) & live
                if bool(bad.any()):
                    w = int(torch.nonzero(bad)[0].item())
                    raise TsfError(TSF_E_INVALID_SCHEME, "walk %d of %s: the %s scheme fails "
                                   "the Brent equations" % (w, path, label))
        return b

    # ------------------------------------------------------------ read back
    def headers(self):
        return self.hdr.cpu().numpy().view(HEADER_DTYPE).copy()

    def records(self, walk):
        h = self.headers()[walk]
        n = min(int(h["n_rec"]), self.rec_cap)
        rec = self.rec[walk, :n].cpu().numpy()
        return [(int(a), int(b & 0xFFFFFFFF)) for a, b in rec]

    def scheme(self, walk, which="best", headers=None):
        h = (headers if headers is not None else self.headers())[walk]
        buf = {"cur": self.cur, "best": self.best, "start": self.start}[which]
        rank = {"cur": h["rank"], "best": h["best_rank"], "start": h["start_rank"]}[which]
        packed = buf[walk].cpu().numpy().view(np.uint64)
        return unpack(packed, int(h["m"]), int(h["n"]), int(h["p"]), int(rank), int(h["mode"]))

    def counters(self, walk, headers=None):
        h = (headers if headers is not None else self.headers())[walk]
        return {name: int(h["counters"][k]) for k, name in enumerate(COUNTER_NAMES)}


# ---------------------------------------------------------------------------
# learned proposal network
# ---------------------------------------------------------------------------
class Mlp:
    """Device buffers of the proposal network (see tsf.h)."""

    def __init__(self, device="cuda"):
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.param = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev)
        self.grad = torch.zeros_like(self.param)
        self.adam_m = torch.zeros_like(self.param)
        self.adam_v = torch.zeros_like(self.param)
        self.wbf = torch.zeros(MLP_NBF16, dtype=torch.int16, device=dev)
        self.step_count = 0

    def c(self):
        return MlpC(self.param.data_ptr(), self.grad.data_ptr(), self.adam_m.data_ptr(),
                    self.adam_v.data_ptr(), self.wbf.data_ptr())

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def set_params(self, W1, b1, W2, b2, w3, b3):
        """From the math layout (W1: 512 x 256, W2: 256 x 256) to the packed vector."""
        v = np.concatenate([np.asarray(W1, np.float32).T.reshape(-1), np.asarray(b1, np.float32),
                            np.asarray(W2, np.float32).T.reshape(-1), np.asarray(b2, np.float32),
                            np.asarray(w3, np.float32), np.asarray(b3, np.float32).reshape(-1)[:1],
                            np.zeros(3, np.float32)])
        assert v.size == MLP_NPARAM
        self.param.copy_(self.torch.from_numpy(v))
        self.sync()

    def unpack(self, vec):
        """packed fp32 vector -> dict in the math layout"""
        v = np.asarray(vec, dtype=np.float64)
        H, I = MLP_HID, MLP_IN
        o = 0
        W1 = v[o:o + H * I].reshape(H, I).T; o += H * I
        b1 = v[o:o + H]; o += H
        W2 = v[o:o + H * H].reshape(H, H).T; o += H * H
        b2 = v[o:o + H]; o += H
        w3 = v[o:o + H]; o += H
        b3 = v[o:o + 1]
        return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "w3": w3, "b3": b3}

    def sync(self):
        check(lib().tsf_mlp_sync(C.byref(self.c()), self._stream()))

    def forward(self, X, h1=None, h2=None, logit=None):
        torch = self.torch
        M = X.shape[0]
        h1 = h1 if h1 is not None else torch.empty((M, MLP_HID), dtype=torch.int16, device=X.device)
        h2 = h2 if h2 is not None else torch.empty_like(h1)
        logit = logit if logit is not None else torch.empty(M, dtype=torch.float32, device=X.device)
        check(lib().tsf_mlp_fwd(C.byref(self.c()), C.c_void_p(X.data_ptr()), M,
                                C.c_void_p(h1.data_ptr()), C.c_void_p(h2.data_ptr()),
                                C.c_void_p(logit.data_ptr()), self._stream()))
        return h1, h2, logit

    def backward(self, X, y, h1, h2, logit):
        torch = self.torch
        M = X.shape[0]
        d2 = torch.empty((M, MLP_HID), dtype=torch.int16, device=X.device)
        d1 = torch.empty_like(d2)
        d3 = torch.empty(M, dtype=torch.float32, device=X.device)
        loss = torch.zeros(1, dtype=torch.float32, device=X.device)
        check(lib().tsf_mlp_bwd(C.byref(self.c()), C.c_void_p(X.data_ptr()),
                                C.c_void_p(y.data_ptr()), M, C.c_void_p(h1.data_ptr()),
                                C.c_void_p(h2.data_ptr()), C.c_void_p(logit.data_ptr()),
                                C.c_void_p(d2.data_ptr()), C.c_void_p(d1.data_ptr()),
                                C.c_void_p(d3.data_ptr()), C.c_void_p(loss.data_ptr()),
                                self._stream()))
        return loss

    def step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        check(lib().tsf_mlp_step(C.byref(self.c()), lr, beta1, beta2, eps, self.step_count,
                                 self._stream()))


def bf16_bits(a):
    """float array -> int16 array of bf16 bits (round to nearest even)"""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return r.view(np.int16)


def bf16_to_float(bits):
    b = np.asarray(bits).view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


class LearnWorkspace:
    """Device workspace of tsf_walk_learned for a batch of n_walks walks."""

    def __init__(self, n_walks, choice_cap=0, device="cuda"):
        import torch
        rows = 8 * n_walks
        dev = torch.device(device)
        self.cand = torch.zeros(rows, dtype=torch.int32, device=dev)
        self.feat = torch.zeros((rows, MLP_IN), dtype=torch.int16, device=dev)
        self.h1 = torch.zeros((rows, MLP_HID), dtype=torch.int16, device=dev)
        self.h2 = torch.zeros_like(self.h1)
        self.logit = torch.zeros(rows, dtype=torch.float32, device=dev)
        self.choice_cap = int(choice_cap)
        self.choice = (torch.zeros((n_walks, self.choice_cap), dtype=torch.uint8, device=dev)
                       if self.choice_cap else None)

    def c(self):
        return LearnWsC(self.cand.data_ptr(), self.feat.data_ptr(), self.h1.data_ptr(),
                        self.h2.data_ptr(), self.logit.data_ptr(),
                        self.choice.data_ptr() if self.choice is not None else None,
                        self.choice_cap, 0)


LOG_DTYPE = np.dtype([("iter", "<i8"), ("rank_before", "<i4"), ("rank_after", "<i4"),
                      ("format_slot", "<i4"), ("reserved", "<i4"), ("f", "<u8", (12,)),
                      ("pad", "<u8")])
assert LOG_DTYPE.itemsize == 128


def features_from_log(log_tensor, n=None):
    """Device log records (int64 tensor, 16 words per record) -> bf16 rows (int16 tensor)."""
    import torch
    flat = log_tensor.reshape(-1, 16)
    n = flat.shape[0] if n is None else n
    X = torch.empty((n, MLP_IN), dtype=torch.int16, device=flat.device)
    check(lib().tsf_features_from_log(C.c_void_p(flat.data_ptr()), n, C.c_void_p(X.data_ptr()),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return X


def format_slot(m, n, p):
    return int(lib().tsf_format_slot(m, n, p))
