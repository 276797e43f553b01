"""Exploratory search (Sec. 3.4.1 and 3.9): rounds of walks and resizes over
a population whose formats change.  Host driver only: every step runs in
libtsf (tsf_walk, tsf_population_best, tsf_resize_batch, tsf_walk_init);
this module sequences the calls and keeps the archive of the best scheme
found per format.

Round q: the walks of the population run `iters` iterations with walk seeds
base_seed + q * n_walks + walk id; the population's best scheme per format
is synchronised (tsf_population_best); every walk's best scheme is resized
(Algorithm 2, Philox counter `q`, seeds base_seed + walk id) into the other
buffer, which becomes the population of round q + 1.
"""
import numpy as np

from . import tsf


def _archive_update(archive, batch, table, count, hdr):
    n = int(count.item())
    ent = table.cpu().numpy().view(tsf.BEST_ENTRY_DTYPE)[:n]
    for e in ent:
        key = (int(e["m"]), int(e["n"]), int(e["p"]))
        rank = int(e["rank"])
        if key not in archive or rank < archive[key][0]:
            archive[key] = (rank, batch.scheme(int(e["walk"]), "best", hdr))
    return ent


def explore(ctx, groups, rounds, iters, capacity, base_seed=0, t_resize=tsf.ALWAYS, plateau=20000,
            r_cap_extra=8, slots=4096, walk_kw=None, launch=(0, 0, 0)):
    """groups: start schemes as for WalkBatch (one mode).  launch: (lanes per
    walk, wavefronts per workgroup, strategy) of the walk calls, zeros for the
    library's choice.  Returns the archive {format: (best rank, Scheme)} and
    per-round statistics."""
    a = tsf.WalkBatch(groups, capacity=capacity, rec_cap=4)
    a.max_len = 64
    b = tsf.WalkBatch.empty(a.n_walks, capacity, a.mode, max_len=64, rec_cap=4)
    a.init(ctx)
    archive, stats = {}, []
    kw = dict(walk_kw or {})
    for q in range(rounds):
        prm = tsf.walk_params(base_seed=base_seed + q * a.n_walks, max_iters=iters,
                              plateau=plateau, **kw)
        a.walk(ctx, prm, iters, *launch)
        table, count = a.population_best(slots)
        hdr = a.headers()
        ent = _archive_update(archive, a, table, count, hdr)
        applied = a.resize_into(b, table, count, base_seed, q, t_resize=t_resize,
                                r_cap_extra=r_cap_extra)
        b.init(ctx)
        ap = applied.cpu().numpy()
        stats.append({"round": q, "formats": int(len(ent)),
                      "flips": int(hdr["counters"][:, 1].sum()),
                      "ops": {name: int(((ap >= 0) & ((ap >> k) & 1 == 1)).sum())
                              for k, name in enumerate(("swap", "merge", "project", "product",
                                                        "double", "extend"))}})
        a, b = b, a
    return archive, stats
