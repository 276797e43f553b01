"""GPU parity at the events the benchmark reports and at full size:

* the (3,3,3) workload (65,536 walks, seeds 0..65535) in the benchmark's
  launch, compared with the oracle on every walk that reached rank 23 within
  2e4 iterations (the first rank-23 walk among them) and on a sample of the
  rank-24 walks, then continued past the 5e4-iteration plateau restart;
* the GPU Brent verifier's violation counts (Eq. 1) against the oracle's on
  single-coefficient mutations of schemes of every workload format, ternary
  and Z2, and mask bits that encode no coefficient counted one each.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2511_20317_amd import tsf
from tests.gpu_parity import compare, run_oracle

pytestmark = pytest.mark.gpu

FORMATS = [(2, 2, 2), (3, 3, 3), (3, 3, 4), (3, 4, 5), (4, 4, 4), (4, 4, 5), (4, 5, 12),
           (5, 6, 10), (6, 7, 9)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return tsf.Context()


def _sync():
    import torch
    torch.cuda.synchronize()


def test_config2_rank23_walks_and_plateau_restart(ctx):
    groups = [(tsf.init_scheme(3, 3, 3), 65536, 35, 23)]
    prm = tsf.walk_params(base_seed=0, max_iters=1000000, plateau=50000)
    b = tsf.WalkBatch(groups, rec_cap=32)
    b.init(ctx)
    b.walk(ctx, prm, 20000)
    _sync()
    hdr = b.headers()
    at23 = np.flatnonzero(hdr["best_rank"] <= 23)
    at24 = np.flatnonzero(hdr["best_rank"] == 24)
    assert at23.size >= 1, "no walk reached rank 23 within 2e4 iterations"
    rng = np.random.default_rng(23)
    sample24 = rng.choice(at24, min(300, at24.size), replace=False)
    walks = sorted(set(at23.tolist()) | set(sample24.tolist()) | {0, 65535})
    ow = run_oracle(groups, prm, walks, 20000, threads=16)
    compare(b, ow, "cfg2 2e4")
    # the first rank-23 record of the batch, from the oracle's own records
    first = min(min(it for it, rk in O.records(ow[w]) if rk <= 23) for w in at23)
    assert 0 < first <= 20000
    nv = b.verify_device(which=1).cpu().numpy()
    assert (nv == 0).all()
    # a second launch to 6e4 iterations: walks whose last improvement came
    # early cross the 5e4-iteration plateau and restart from the start scheme
    b.walk(ctx, prm, 40000)
    _sync()
    hdr = b.headers()
    restarted = np.flatnonzero(hdr["counters"][:, 9] >= 1)
    assert restarted.size > 0
    pick = sorted(set(rng.choice(restarted, min(16, restarted.size), replace=False).tolist()) |
                  set(at23[:8].tolist()))
    compare(b, run_oracle(groups, prm, pick, 60000, threads=16), "cfg2 6e4")
    assert (b.verify_device(which=1).cpu().numpy() == 0).all()
    assert (b.verify_device(which=0).cpu().numpy()[pick] == 0).all()


def _oracle_scheme(fmt, z2, seed, iters):
    """a scheme reached by the oracle's own walk from the standard scheme"""
    m, n, p = fmt
    r0 = m * n * p
    w = O.new_walk(O.standard(m, n, p, z2=z2))
    O.run(w, O.make_params(seed=seed, max_iters=iters, plateau=10 ** 9, target_rank=0, r0=r0),
          iters)
    d = O.from_c(w.cur)
    return d["U"].copy(), d["V"].copy(), d["W"].copy()


def _mutations(U, V, W, z2, rng, count):
    """single-coefficient changes: a random entry of a random factor takes
    another value of the coefficient set"""
    vals = (0, 1) if z2 else (-1, 0, 1)
    out = []
    for _ in range(count):
        f = [U.copy(), V.copy(), W.copy()]
        X = int(rng.integers(0, 3))
        l = int(rng.integers(0, f[X].shape[0]))
        e = int(rng.integers(0, f[X].shape[1]))
        old = int(f[X][l, e])
        f[X][l, e] = rng.choice([v for v in vals if v != old])
        out.append(tuple(f))
    return out


def _verify_on_gpu(ctx, fmt, mode, schemes, extra=None):
    """the start buffer of a batch holds the given schemes (packed as they
    are; `extra` ORs raw bits into the packed words); returns the GPU counts"""
    import torch
    m, n, p = fmt
    cap = max(s[0].shape[0] for s in schemes)
    hdr = np.zeros(len(schemes), tsf.HEADER_DTYPE)
    start = np.zeros((len(schemes), cap, 6), np.uint64)
    for q, (U, V, W) in enumerate(schemes):
        s = tsf.Scheme(m, n, p, U, V, W, mode=mode)
        start[q] = tsf.pack(s, cap)
        hdr[q]["m"], hdr[q]["n"], hdr[q]["p"], hdr[q]["mode"] = m, n, p, mode
        hdr[q]["start_rank"] = U.shape[0]
        hdr[q]["r_cap"] = cap
    if extra is not None:
        start |= extra
    b = tsf.WalkBatch.empty(len(schemes), cap, mode, max_len=max(m * n, n * p, p * m), rec_cap=1)
    b.hdr.copy_(torch.from_numpy(hdr.view(np.uint8).copy()))
    b.start.copy_(torch.from_numpy(start.view(np.int64)))
    return b.verify_device(which=2).cpu().numpy()


@pytest.mark.parametrize("mode", [tsf.TSF_TERNARY, tsf.TSF_Z2])
@pytest.mark.parametrize("fmt", FORMATS)
def test_verifier_counts_equal_the_oracle(ctx, fmt, mode):
    z2 = mode == tsf.TSF_Z2
    m, n, p = fmt
    rng = np.random.default_rng(hash((fmt, mode)) & 0xFFFF)
    bases = [O.from_c(O.standard(m, n, p, z2=z2))]
    bases = [(bases[0]["U"], bases[0]["V"], bases[0]["W"])]
    bases.append(_oracle_scheme(fmt, z2, 3, 400 if m * n * p <= 80 else 150))
    schemes = []
    for U, V, W in bases:
        schemes.append((U, V, W))
        schemes += _mutations(U, V, W, z2, rng, 12)
    got = _verify_on_gpu(ctx, fmt, mode, schemes)
    want = [O.brent_violations(O.to_c(U, V, W, m, n, p, z2=z2)) for U, V, W in schemes]
    assert got.tolist() == want
    assert want[0] == 0 and want[13] == 0 and max(want) > 0


@pytest.mark.parametrize("mode", [tsf.TSF_TERNARY, tsf.TSF_Z2])
def test_verifier_counts_mask_bits_outside_the_coefficients(ctx, mode):
    z2 = mode == tsf.TSF_Z2
    fmt = (6, 7, 9) if not z2 else (3, 4, 5)
    m, n, p = fmt
    lens = (m * n, n * p, p * m)
    d = O.from_c(O.standard(m, n, p, z2=z2))
    base = (d["U"], d["V"], d["W"])
    r = base[0].shape[0]
    rng = np.random.default_rng(7 + mode)
    schemes, extras, want = [], [], []
    for q in range(12):
        ex = np.zeros((r, 6), np.uint64)
        k = 0
        for _ in range(q % 4 + 1):
            l, X = int(rng.integers(0, r)), int(rng.integers(0, 3))
            if q % 2 == 0:   # a digit past the factor's length
                bit = int(rng.integers(lens[X], 64))
                word = 2 * X
            else:            # a sign without a digit (Z2: any sign)
                packed = tsf.pack(tsf.Scheme(m, n, p, *base, mode=mode))
                free = [e for e in range(lens[X]) if not (int(packed[l, 2 * X]) >> e) & 1]
                bit = free[int(rng.integers(0, len(free)))] if not z2 else \
                    int(rng.integers(0, lens[X]))
                word = 2 * X + 1
            if not (int(ex[l, word]) >> bit) & 1:
                ex[l, word] |= np.uint64(1) << np.uint64(bit)
                k += 1
        schemes.append(base)
        extras.append(ex)
        want.append(k)
    got = _verify_on_gpu(ctx, fmt, mode, schemes, extra=np.stack(extras))
    assert got.tolist() == want
