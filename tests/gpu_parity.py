"""Helpers shared by the GPU parity tests: run the oracle on the walks a GPU
batch ran and compare every observable bit for bit."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import pyoracle as O
from paper_2511_20317_amd import tsf


def oracle_start(scheme: tsf.Scheme):
    U, V, W = scheme.live()
    return O.to_c(U, V, W, scheme.m, scheme.n, scheme.p, z2=scheme.mode == tsf.TSF_Z2)


def oracle_params(prm: tsf.WalkParams, walk_id: int, r_cap: int, target: int):
    return O.Params(prm.base_seed + prm.first_walk_id + walk_id, prm.max_iters, prm.plateau,
                    target, r_cap, prm.flip_tries, prm.restart_from_best, prm.t_eq,
                    prm.t_reduce, prm.t_expand, prm.objective, 0)


def run_oracle(groups, prm, walks, n_iters, splits=None, threads=8):
    """groups as given to WalkBatch; returns {walk: oracle Walk}"""
    def one(w):
        off = 0
        for s, nw, r_cap, target in groups:
            if w < off + nw:
                break
            off += nw
        ow = O.new_walk(oracle_start(s))
        op = oracle_params(prm, w, r_cap, target)
        for chunk in (splits or [n_iters]):
            O.run(ow, op, chunk)
        return w, ow
    with ThreadPoolExecutor(threads) as ex:
        return dict(ex.map(one, walks))


def rows_of(d):
    return d["U"], d["V"], d["W"]


def compare(batch: tsf.WalkBatch, oracle_walks, label=""):
    hdr = batch.headers()
    mism = []
    for w, ow in oracle_walks.items():
        h = hdr[w]
        tag = "%s walk %d" % (label, w)
        assert h["done"] >= 0, tag + " flagged invalid by the kernel"
        got = {
            "t": int(h["t"]), "rank": int(h["rank"]), "best_rank": int(h["best_rank"]),
            "done": int(h["done"]), "plateau_start": int(h["plateau_start"]),
            "n_rec": int(h["n_rec"]), "best_nnz": int(h["best_nnz"]),
        }
        want = {
            "t": ow.t, "rank": ow.cur.r, "best_rank": ow.best_rank, "done": ow.done,
            "plateau_start": ow.plateau_start, "n_rec": ow.n_rec, "best_nnz": ow.best_nnz,
        }
        if got != want:
            mism.append((tag, "header", got, want))
            continue
        gc = batch.counters(w, hdr)
        oc = O.counters(ow)
        if gc != oc:
            mism.append((tag, "counters", gc, oc))
            continue
        for which, osch in (("cur", ow.cur), ("best", ow.best)):
            g = batch.scheme(w, which, hdr)
            o = O.from_c(osch)
            for a, b, nm in zip(g.live(), rows_of(o), "UVW"):
                if not np.array_equal(a, b):
                    mism.append((tag, which + " " + nm, a.tolist(), b.tolist()))
                    break
        recs = batch.records(w)
        orecs = O.records(ow)[:batch.rec_cap]
        if recs != orecs:
            mism.append((tag, "records", recs, orecs))
    assert not mism, "first mismatches: %r" % (mism[:3],)
