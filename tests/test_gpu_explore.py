"""Population synchronisation, the Resize kernel (Algorithm 2) and the
exploratory search loop on the GPU against the oracle (or_resize and its walk),
bit for bit: best-scheme tables, resized start schemes, headers and operators,
and whole populations after several rounds of walk + sync + resize."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2511_20317_amd import explore, tsf
from tests.gpu_parity import oracle_start

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tsf.Context()


def _walked(fmt, seed, iters):
    m, n, p = fmt
    prm = O.make_params(seed=seed, max_iters=iters, plateau=iters, target_rank=0, r0=m * n * p)
    w = O.new_walk(O.standard(m, n, p))
    O.run(w, prm, iters)
    d = O.from_c(w.best)
    return tsf.Scheme(m, n, p, d["U"], d["V"], d["W"])


def _oracle_table(schemes):
    """per format: (rank, index) of the lowest rank, ties the lowest index;
    ascending format"""
    best = {}
    for w, s in enumerate(schemes):
        key = (s.m, s.n, s.p)
        if key not in best or s.rank < best[key][0]:
            best[key] = (s.rank, w)
    return [(k, best[k][0], best[k][1]) for k in sorted(best)]


def _gpu_table(table, count):
    n = int(count.item())
    ent = table.cpu().numpy().view(tsf.BEST_ENTRY_DTYPE)[:n]
    return [((int(e["m"]), int(e["n"]), int(e["p"])), int(e["rank"]), int(e["walk"])) for e in ent]


def test_population_best_and_resize_match_oracle(ctx):
    import torch
    fmts = [(2, 2, 2), (2, 2, 3), (2, 3, 2), (1, 2, 2), (2, 2, 4), (3, 2, 2), (2, 3, 3)]
    schemes = [_walked(fmts[k % len(fmts)], k, 200 + 37 * k) for k in range(112)]
    cap = 96
    b = tsf.WalkBatch([(s, 1, s.rank, 0) for s in schemes], capacity=cap, rec_cap=4)
    b.max_len = 64
    b.init(ctx)
    table, count = b.population_best()
    want = _oracle_table(schemes)
    assert _gpu_table(table, count) == want
    out = tsf.WalkBatch.empty(b.n_walks, cap, tsf.TSF_TERNARY, max_len=64, rec_cap=4)
    base = 12345
    for rnd in (0, 1, 5):
        applied = b.resize_into(out, table, count, base, rnd, r_cap_extra=8)
        torch.cuda.synchronize()
        ap = applied.cpu().numpy()
        hdr = out.headers()
        best = [oracle_start(schemes[w]) for _, _, w in want]
        seen = 0
        for w, s in enumerate(schemes):
            bits, t = O.resize(oracle_start(s), best, base + w, rnd, 1 << 32, cap)
            seen |= bits
            assert ap[w] == bits, (rnd, w)
            h = hdr[w]
            assert (int(h["m"]), int(h["n"]), int(h["p"]), int(h["start_rank"])) == \
                (t.m, t.n, t.p, t.r), (rnd, w)
            assert int(h["r_cap"]) == min(t.r + 8, cap)
            packed = out.start[w, :t.r].cpu().numpy().view(np.uint64)
            got = tsf.unpack(packed, t.m, t.n, t.p, t.r)
            d = O.from_c(t)
            for g, o in zip(got.live(), (d["U"], d["V"], d["W"])):
                assert np.array_equal(g, o), (rnd, w, bits)
        assert seen & 1 and seen & 2
        out.init(ctx)
        assert (out.verify_device(which=2).cpu().numpy() == 0).all()
        assert (out.headers()["done"] == 0).all()


def _oracle_explore(groups, rounds, iters, capacity, base_seed, plateau, r_cap_extra):
    pop = []
    for s, nw, r_cap, target in groups:
        pop += [(oracle_start(s), r_cap, target)] * nw
    n = len(pop)
    archive = {}
    for q in range(rounds):
        walks = []
        for w, (st, r_cap, target) in enumerate(pop):
            ow = O.new_walk(st)
            prm = O.make_params(seed=base_seed + q * n + w, max_iters=iters, plateau=plateau,
                                target_rank=target, r_cap=r_cap)
            O.run(ow, prm, iters)
            walks.append(ow)
        best = {}
        for w, ow in enumerate(walks):
            key = (ow.best.m, ow.best.n, ow.best.p)
            if key not in best or ow.best_rank < best[key][0]:
                best[key] = (ow.best_rank, w)
        keys = sorted(best)
        for k in keys:
            if k not in archive or best[k][0] < archive[k]:
                archive[k] = best[k][0]
        table = [walks[best[k][1]].best for k in keys]
        newpop = []
        for w, (ow, (_, _, target)) in enumerate(zip(walks, pop)):
            _, t = O.resize(ow.best, table, base_seed + w, q, 1 << 32, capacity)
            newpop.append((t, min(t.r + r_cap_extra, capacity), target))
        pop = newpop
    return pop, archive


def test_exploratory_rounds_match_oracle(ctx):
    groups = [(tsf.init_scheme(2, 2, 2), 24, 16, 0), (tsf.init_scheme(2, 2, 3), 24, 20, 0),
              (tsf.init_scheme(1, 2, 3), 16, 14, 0)]
    cap = 80
    archive, stats = explore.explore(ctx, groups, rounds=3, iters=400, capacity=cap,
                                     base_seed=77, plateau=300, r_cap_extra=8)
    pop, oarch = _oracle_explore(groups, 3, 400, cap, 77, 300, 8)
    assert {k: v[0] for k, v in archive.items()} == oarch
    for k, (rank, s) in archive.items():
        assert tsf.verify(s) == 0 and s.rank == rank
    assert sum(st["ops"]["merge"] for st in stats) > 0
