"""Benchmark: flips/sec of the ternary flip-graph walk on one MI355X, and the
time to reach rank 23 at (3,3,3).

Workload (defaults): format (3,3,3), ternary, 65,536 walks from the standard
rank-27 scheme, walk seeds 0..65535, at most 1e6 iterations per walk, plateau
restart after 5e4 iterations without improvement, target rank 23, uniform
flip proposals.  One step = one walk-kernel launch of every walk followed by
the GPU Brent check of every walk's best scheme; the 1e6-iteration budget is
split evenly over the timed steps (--steps 20: 5e4 iterations per launch), so
every timed launch does work.

After the timed steps (outside the timed region): the time to rank 23 in
rounds of 1,000 iterations on a fresh batch, the learned proposal against
uniform proposals (learned_vs_uniform; --no-learned skips it), and the CPU
oracle on a bounded sample (cpu_baseline; --no-cpu skips it).

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build measures one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_OPS = 256 * 64 * 2.4e9   # CUs x int32 lanes/clk/CU x clock = 39.3e12 op/s
PEAK_HBM = 8.0e12

MAX_ITERS = 1000000

# HBM bytes per walk-kernel launch of the default workload (65,536 walks,
# launches of `iters` iterations each), from two rocprofv3 passes over this
# script: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 per dispatch, the scales read
# off a 1 GiB device copy in the same runs (--calibrate-copy-mib 1024),
# averaged over the timed launches.  Valid only for the kernel sources it was
# measured on (their SHA-1 below) and for launches of the same size;
# otherwise the benchmark reports no traffic.
MEASURED_TRAFFIC = {"sources_sha1": "163039c8ab4c5c97500f7e4dee6f7ccd9a492713",
                    "walks": 65536, "iters": 50000, "bytes_per_launch": 2.7501e+09}
KERNEL_SOURCES = ("walk_kernel.h", "walk_inst.hip", "tsf_bits.h")


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_20317_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def ops_per_flip(mean_rank, attempts_per_iteration, fallback_rate, wd=1):
    """Algorithmic 32-bit integer operations per applied flip, the work model
    A(r, Wd) of the hot path (Wd = 32-bit words per factor mask, r the mean
    rank, T the measured attempts per iteration):
      Philox blocks          100 (T + 1)      (10 rounds x (4 mul + 4 xor + 2 add),
                                               one per attempt and the gate block)
      partner tests          T r (4 Wd + 4)   (equality and negated equality of
                                               the X factor, validity of two roles)
      apply, normalise and   30 r Wd
      the reduction scan
      bookkeeping            80
      cyclic fallback        3 r (4 Wd + 4)   per iteration that needs it
    """
    r, t = mean_rank, attempts_per_iteration
    return (100.0 * (t + 1.0) + t * r * (4 * wd + 4) + 30.0 * r * wd + 80.0 +
            fallback_rate * 3.0 * r * (4 * wd + 4))


def cpu_baseline(n_walks=512, iters=100000, threads=None):
    """The oracle as it stands, on the host cores: (3,3,3) walks from the
    standard scheme with the benchmark's parameters, a bounded sample."""
    from oracle import pyoracle as O
    threads = threads or os.cpu_count() or 1
    start = O.standard(3, 3, 3)
    prm = O.make_params(seed=0, max_iters=1000000, plateau=50000, target_rank=23, r0=27)
    t0 = time.perf_counter()
    ws = O.run_many(start, prm, 0, 0, n_walks, iters, threads)
    dt = time.perf_counter() - t0
    flips = sum(w.c.flips for w in ws)
    its = sum(w.c.iters for w in ws)
    return {"value": flips / dt, "unit": "flips/s", "cores": threads, "kind": "oracle",
            "sample": "%d walks x %d iterations of the (3,3,3) workload (seeds 0..%d), "
                      "%.1f s wall on %d threads, %.3g iterations/s, %.3g flips/s per core"
                      % (n_walks, iters, n_walks - 1, dt, threads, its / dt,
                         flips / dt / threads)}


def _median_or_none(xs):
    """Median of xs, None when it is infinite (most runs did not get there)."""
    m = float(np.median(xs))
    return m if np.isfinite(m) else None


def learned_vs_uniform(ctx, args):
    """The learned proposal: a network (512 -> 256 -> 256 -> 1, bf16 on the
    matrix cores) scores the candidates of an iteration's attempts and the
    walk applies the best scored one.  Trained by the GPU kernels on logged
    flips of uniform (2,2,2) and (3,3,3) walks with 20-flip labels (a quarter
    of every minibatch drawn from the rare positives); reported:
    held-out AUC before and after training; what it gains per iteration (the
    share of walks that reach each rank within a fixed number of iterations,
    for the trained network, an untrained network choosing among the same
    candidates, and uniform proposals, over seed blocks); and learned against
    uniform proposals at equal wall time on (3,3,3) and (4,4,4) (the latter
    skipped with --no-learned-444): medians over R disjoint seed blocks of the time to each
    rank of the ladder (null where the median run does not reach it)."""
    import torch
    from paper_2511_20317_amd import learn, tsf
    s222, s333 = tsf.init_scheme(2, 2, 2), tsf.init_scheme(3, 3, 3)
    t0 = time.perf_counter()
    rec, idx, lab = learn.training_set(ctx, n222=2 * args.learn_walks, n333=args.learn_walks,
                                       n_iters=args.learn_iters, base_seed=10 ** 7)
    held = {"2,2,2": learn.collect(ctx, s222, 1024, args.learn_iters, 16, base_seed=2 * 10 ** 7),
            "3,3,3": learn.collect(ctx, s333, 512, args.learn_iters, 35, base_seed=3 * 10 ** 7)}
    t_collect = time.perf_counter() - t0

    def fresh_net(seed):
        net = tsf.Mlp()
        rng = np.random.default_rng(seed)
        net.set_params(rng.standard_normal((512, 256)) * np.sqrt(2 / 64), np.zeros(256),
                       rng.standard_normal((256, 256)) * np.sqrt(2 / 256), np.zeros(256),
                       rng.standard_normal(256) * np.sqrt(1 / 256), np.zeros(1))
        return net

    net = fresh_net(0)
    ev0 = {k: learn.evaluate(net, *v) for k, v in held.items()}
    t0 = time.perf_counter()
    hist = learn.train(net, rec, idx, lab, args.learn_steps, batch=4096, lr=1e-3,
                       log_every=max(args.learn_steps // 5, 1), pos_share=0.25)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = {k: learn.evaluate(net, *v) for k, v in held.items()}
    n_logged = int(idx.size)
    del rec, held
    out = {"train": {"labelled_flips": n_logged, "positive_rate": float(lab.mean()),
                     "label_window": learn.LABEL_WINDOW, "collect_s": t_collect,
                     "train_s": t_train, "steps": args.learn_steps, "batch": 4096,
                     "positive_share_of_minibatch": 0.25,
                     "loss_history": hist, "held_out_before": ev0, "held_out_after": ev}}
    print("learned: trained, held-out AUC %s" % {k: round(v["auc"], 3) for k, v in ev.items()},
          file=sys.stderr, flush=True)
    # per iteration: the same iterations for every proposal kind
    untrained = fresh_net(7)
    per_it = {}
    for key, s, r_cap, iters, ladder in (("2,2,2", s222, 16, 3000, (7,)),
                                         ("3,3,3", s333, 35, 20000, (26, 25, 24))):
        acc = {}
        for kind, nn in (("trained", net), ("untrained", untrained), ("uniform", None)):
            fr = {str(k): [] for k in ladder}
            walls = []
            for blk in range(3):
                r = learn.reach(ctx, s, r_cap, 2048, iters, ladder, base_seed=(blk + 1) << 21,
                                net=nn)
                walls.append(r["wall_s"])
                for k in ladder:
                    fr[str(k)].append(r["ranks"][str(k)]["fraction"])
            acc[kind] = {"share_reaching": {k: float(np.mean(v)) for k, v in fr.items()},
                         "wall_s_per_run": float(np.mean(walls))}
        per_it[key] = {"walks": 2048, "iterations": iters, "seed_blocks": 3, "by_proposal": acc}
        print("learned: per-iteration %s %s" % (key, {k: v["share_reaching"]
                                                      for k, v in acc.items()}),
              file=sys.stderr, flush=True)
    out["per_iteration"] = per_it
    # equal wall time
    results = {}
    cases = [((3, 3, 3), 35, (26, 25, 24, 23))]
    if not args.no_learned_444:
        cases.append(((4, 4, 4), 64, (63, 62, 61, 60)))
    for fmt, r_cap, ladder in cases:
        s = tsf.init_scheme(*fmt)
        runs = {"uniform": [], "learned": []}
        for rep in range(args.ab_runs):
            seed = 2 ** 20 * (rep + 1)
            for mode in ("uniform", "learned"):
                res = learn.time_to_ranks(ctx, s, args.ab_walks, r_cap, ladder, args.ab_seconds,
                                          seed, net=net if mode == "learned" else None)
                runs[mode].append(res)
        summ = {}
        for mode, rs in runs.items():
            summ[mode] = {
                "median_time_to_rank_s": {str(k): _median_or_none([r["time_to_rank_s"].get(k, np.inf)
                                                                   for r in rs]) for k in ladder},
                "median_iters_to_rank": {str(k): _median_or_none([r["iters_to_rank"].get(k, np.inf)
                                                                  for r in rs]) for k in ladder},
                "iterations_per_s": float(np.median([r["iterations"] / r["wall_s"] for r in rs])),
                "best_rank_median": float(np.median([r["best_rank"] for r in rs])),
            }
        results["%d,%d,%d" % fmt] = summ
        print("learned: equal wall time %s %s" % (fmt, {m: v["median_time_to_rank_s"]
                                                        for m, v in summ.items()}),
              file=sys.stderr, flush=True)
    out["equal_wall_time"] = results
    out["equal_wall_time_setup"] = {"runs": args.ab_runs, "walks": args.ab_walks,
                                    "wall_s": args.ab_seconds}
    return out


def run_mixed(ctx, args):
    """Mixed formats in one launch: 131,072 walks as four blocks of 32,768 over
    (3,3,4), (3,4,5), (4,4,4), (4,4,5) from their standard schemes, r_cap =
    r0 + 8; the same batch walked with ternary and with Z2 coefficients."""
    import torch
    from paper_2511_20317_amd import tsf
    fmts = [(3, 3, 4), (3, 4, 5), (4, 4, 4), (4, 4, 5)]
    per = args.walks // 4
    out = {}
    for mode, name in ((tsf.TSF_TERNARY, "ternary"), (tsf.TSF_Z2, "z2")):
        groups = [(tsf.init_scheme(*f, mode=mode), per, f[0] * f[1] * f[2] + 8, 0) for f in fmts]
        b = tsf.WalkBatch(groups, rec_cap=64)
        prm = tsf.walk_params(base_seed=0, max_iters=1000000, plateau=50000)
        b.init(ctx)
        # tune on the state after a short walk: the first iterations from the
        # standard schemes (many equal factors) are not typical of the run
        b.walk(ctx, prm, 2000)
        tuned = b.autotune(ctx, prm, trial_iters=1000)
        b.init(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kms = 0.0
        for k in range(args.steps):
            ev0.record()
            b.walk(ctx, prm, args.iters)
            ev1.record()
            ev1.synchronize()
            kms += ev0.elapsed_time(ev1)
            print("%s step %d/%d: %.2f s" % (name, k + 1, args.steps, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        nv = b.verify_device(1)
        hdr = b.headers()
        best = {}
        for (w0, nw, fmt, _, _) in b.groups:
            br = hdr["best_rank"][w0:w0 + nw]
            best["%d,%d,%d" % fmt] = {"best": int(br.min()), "median": float(np.median(br))}
        flips = int(hdr["counters"][:, 1].sum())
        out[name] = {"flips_per_s": flips / wall, "walk_kernel_ms": kms, "wall_s": wall,
                     "launch": {"lanes_per_walk": tuned[0], "waves_per_block": tuned[1],
                                "strategy": tuned[2]},
                     "best_rank": best, "best_schemes_failing_brent": int((nv != 0).sum().item())}
    return out


def run_large(ctx, args):
    """Large formats (4,5,12), (5,6,10), (6,7,9), 32,768 walks each from the
    standard schemes (64-bit masks): a round in the format, a device project to
    (m,n,p-1) and a round there, a device extend back to (m,n,p) and a round.
    Each format is its own batch, sized for its own ranks (the term-parallel
    kernel then has as few term slots per lane as the format needs); walk ids
    run on across the formats (first_walk_id), so every walk draws the
    random words it would draw in one batch of all three."""
    import torch
    from paper_2511_20317_amd import tsf
    fmts = [(4, 5, 12), (5, 6, 10), (6, 7, 9)]
    per = args.walks // 3
    rng = np.random.default_rng(5)
    idx_all = [rng.integers(0, f[2], per) for f in fmts]
    flips = 0
    kms = 0.0
    phases = {"start": {"failing_brent": 0}, "projected": {"failing_brent": 0},
              "extended": {"failing_brent": 0}}
    invalid = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def walk_phase(batch, prm, label):
        nonlocal flips, kms
        h0 = batch.headers()["counters"][:, 1].sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            batch.walk(ctx, prm, args.iters, 64, 1, 2)
        e1.record()
        e1.synchronize()
        kms += e0.elapsed_time(e1)
        hdr = batch.headers()
        flips += int(hdr["counters"][:, 1].sum() - h0)
        fm = (int(hdr["m"][0]), int(hdr["n"][0]), int(hdr["p"][0]))
        phases[label]["%d,%d,%d" % fm] = {"best": int(hdr["best_rank"].min()),
                                          "start_median": float(np.median(hdr["start_rank"]))}
        nv = batch.verify_device(1)
        phases[label]["failing_brent"] += int((nv != 0).sum().item())
        print("phase %s %s done: %.1f s" % (label, fm, time.perf_counter() - t0),
              file=sys.stderr, flush=True)

    for q, f in enumerate(fmts):
        r0 = f[0] * f[1] * f[2]
        prm = tsf.walk_params(base_seed=0, first_walk_id=q * per, max_iters=10 ** 9,
                              plateau=50000)
        # capacities: r0 + 8 in the format and after the project (a projected
        # scheme has at most r0 terms); room for the extend back (+ m*n naive
        # terms) in the last phase
        b = tsf.WalkBatch([(tsf.init_scheme(*f), per, r0 + 8, 0)], capacity=r0 + 8, rec_cap=32)
        b.init(ctx)
        walk_phase(b, prm, "start")
        small = tsf.WalkBatch.empty(per, r0 + 8, tsf.TSF_TERNARY, max_len=63, rec_cap=32)
        small.meta_from(b, 1, np.ones(per), np.full(per, 2), idx_all[q], r_cap_extra=8)
        small.init(ctx)
        walk_phase(small, prm, "projected")
        back = tsf.WalkBatch.empty(per, r0 + f[0] * f[1] + 8, tsf.TSF_TERNARY, max_len=63,
                                   rec_cap=32)
        back.meta_from(small, 1, np.full(per, 2), np.full(per, 2), np.zeros(per), r_cap_extra=8)
        back.init(ctx)
        invalid += int((back.headers()["done"] < 0).sum())
        walk_phase(back, prm, "extended")
        del b, small, back
    wall = time.perf_counter() - t0
    return {"flips_per_s": flips / wall, "walk_kernel_ms": kms, "wall_s": wall,
            "phases": phases, "invalid_after_meta": invalid}


def run_additions(ctx, args):
    """The complexity-minimisation mode on (3,3,3): a focused rank search of
    65,536 walks (2e5 iterations, untimed) leaves every walk a best scheme of
    rank 23..26; each is copied on the GPU into a new batch as its start and
    walked with the naive-additions objective (timed): flips/s and the naive
    additions (non-zero coefficients - 2r - mp) before and after, per rank."""
    import torch
    from paper_2511_20317_amd import tsf
    n = args.walks
    focus = tsf.WalkBatch([(tsf.init_scheme(3, 3, 3), n, 35, 23)], rec_cap=8)
    focus.init(ctx)
    prm0 = tsf.walk_params(base_seed=0, max_iters=200000, plateau=50000)
    for _ in range(2):
        focus.walk(ctx, prm0, 100000)
    torch.cuda.synchronize()
    batch = tsf.WalkBatch.empty(n, focus.capacity, tsf.TSF_TERNARY, max_len=9, rec_cap=32)
    batch.meta_from(focus, 1, np.zeros(n), np.zeros(n), np.zeros(n), r_cap_extra=0)
    batch.init(ctx)
    batch.hdr.view(torch.int32).view(n, tsf.HEADER_I32)[:, 5] = 0   # target additions: none
    h0 = batch.headers()
    start_add = h0["best_nnz"] - 2 * h0["start_rank"] - 9
    prm = tsf.walk_params(base_seed=1 << 40, max_iters=10 ** 9, plateau=50000,
                          objective=tsf.OBJ_ADDITIONS)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(args.steps):
        batch.walk(ctx, prm, args.iters)
        print("additions step %d/%d" % (k + 1, args.steps), file=sys.stderr, flush=True)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h = batch.headers()
    nv = batch.verify_device(1).cpu().numpy()
    best_add = h["best_nnz"] - 2 * h["best_rank"] - 9
    per_rank = {}
    for r in sorted(set(h["start_rank"].tolist())):
        sel = h["start_rank"] == r
        per_rank[str(r)] = {"walks": int(sel.sum()),
                            "start_additions_min": int(start_add[sel].min()),
                            "start_additions_median": float(np.median(start_add[sel])),
                            "best_additions_min": int(best_add[sel].min()),
                            "best_additions_median": float(np.median(best_add[sel]))}
    flips = int(h["counters"][:, 1].sum())
    # isotropy invariants (Sec. 3.7) of every best scheme on the GPU, and the
    # number of distinct type polynomials among those of the lowest rank
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    ranks, sums = batch.invariants(which=1)
    e3.record()
    e3.synchronize()
    low = int(h["best_rank"].min())
    sel = np.flatnonzero(h["best_rank"] == low)
    rk = ranks.cpu().numpy()[sel, :low]
    types = {tuple(sorted(map(tuple, r.tolist()))) for r in rk}
    return {"flips_per_s": flips / wall, "walk_kernel_ms": e0.elapsed_time(e1), "wall_s": wall,
            "rank_kept": bool((h["rank"] == h["start_rank"]).all()),
            "best_schemes_failing_brent": int((nv != 0).sum()), "by_start_rank": per_rank,
            "invariants": {"kernel_ms": e2.elapsed_time(e3), "schemes": n,
                           "lowest_rank": low, "schemes_at_lowest_rank": int(sel.size),
                           "distinct_type_polynomials": len(types)}}


def run_explore(ctx, args):
    """Exploratory search: a population of args.walks walks starting from the
    standard schemes of (2,2,2), (2,2,3), (2,3,3), (3,3,3) (a quarter each),
    capacity 128 terms, rounds of args.iters iterations, each followed by the
    population synchronisation and the Resize kernel; reports flips/s over the
    rounds, the time of sync + resize + init per round and the archive of the
    best rank found per format."""
    import torch
    from paper_2511_20317_amd import explore, tsf
    q = args.walks // 4
    groups = [(tsf.init_scheme(*f), q, f[0] * f[1] * f[2] + 8, 0)
              for f in [(2, 2, 2), (2, 2, 3), (2, 3, 3), (3, 3, 3)]]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    archive, stats = explore.explore(ctx, groups, rounds=args.steps, iters=args.iters,
                                     capacity=128, base_seed=0, plateau=20000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flips = sum(s["flips"] for s in stats)
    arch = {"%d,%d,%d" % k: v[0] for k, v in sorted(archive.items())}
    bad = sum(int(tsf.verify(s) != 0) for _, s in archive.values())
    return {"flips_per_s": flips / wall, "wall_s": wall, "rounds": stats,
            "formats_in_archive": len(arch), "archive_best_rank": arch,
            "archive_schemes_failing_brent": bad}


def run_lift(ctx, args):
    """Ternary lifting (Sec. 3.10.1) of Z2 schemes found on the GPU: Z2 walks
    of (2,2,3), (2,3,3) and (3,3,3) from the standard schemes (args.walks each,
    5e4 iterations, untimed); the lowest-rank best schemes (up to 4 distinct
    per format) are lifted with the GPU search (timed per scheme)."""
    import torch
    from paper_2511_20317_amd import tsf
    out = {}
    for fmt in [(2, 2, 3), (2, 3, 3), (3, 3, 3)]:
        m, n, p = fmt
        b = tsf.WalkBatch([(tsf.init_scheme(m, n, p, tsf.TSF_Z2), args.walks, m * n * p + 8, 0)],
                          rec_cap=4)
        b.init(ctx)
        b.walk(ctx, tsf.walk_params(base_seed=5, max_iters=50000, plateau=20000), 50000)
        hdr = b.headers()
        low = int(hdr["best_rank"].min())
        picked, seen = [], set()
        for w in np.flatnonzero(hdr["best_rank"] == low):
            s = b.scheme(int(w), "best", hdr)
            key = s.U.tobytes() + s.V.tobytes() + s.W.tobytes()
            if key not in seen:
                seen.add(key)
                picked.append(s)
            if len(picked) == 4:
                break
        res = []
        for s in picked:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info, t = tsf.lift(s, max_nodes=1 << 16, max_subtrees=1 << 16)
            dt = time.perf_counter() - t0
            res.append({"status": info["status"], "seconds": dt, "subtrees": info["subtrees"],
                        "exhausted": info["exhausted"],
                        "valid": (tsf.verify(t) == 0) if t is not None else None})
            print("lift %s rank %d: status %d in %.2f s" % (fmt, low, info["status"], dt),
                  file=sys.stderr, flush=True)
        out["%d,%d,%d" % fmt] = {"z2_rank": low, "schemes": res}
    return out


def run_learned_walk(ctx, args):
    """Throughput of the learned proposal: 4,096 (3,3,3) walks with a
    random-initialised network (the cost does not depend on the weights),
    learned and uniform proposals for args.ab_seconds each."""
    from paper_2511_20317_amd import learn, tsf
    s = tsf.init_scheme(3, 3, 3)
    rng = np.random.default_rng(0)
    net = tsf.Mlp()
    net.set_params(rng.standard_normal((512, 256)) * np.sqrt(2 / 64), np.zeros(256),
                   rng.standard_normal((256, 256)) * np.sqrt(2 / 256), np.zeros(256),
                   rng.standard_normal(256) * np.sqrt(1 / 256), np.zeros(1))
    out = {}
    for mode in ("learned", "uniform"):
        res = learn.time_to_ranks(ctx, s, args.ab_walks, 35, (26, 25, 24, 23), args.ab_seconds,
                                  1 << 20, net=net if mode == "learned" else None)
        out[mode] = {"iterations_per_s": res["iterations"] / res["wall_s"],
                     "flips_per_s": res["flips"] / res["wall_s"], "wall_s": res["wall_s"],
                     "best_rank": res["best_rank"]}
    return out


def run_222(ctx, args):
    """The (2,2,2) workload: 256 walks from the standard rank-8 scheme, seed
    0, at most 1e5 iterations, plateau 2e4, target rank 7; rounds of
    args.iters iterations until every walk stopped.  Reports flips/s, the
    wall time until the first walk reached 7 (end of that round), the share
    of walks at 7 and the Brent check of every best scheme."""
    import torch
    from paper_2511_20317_amd import tsf
    n = 256
    b = tsf.WalkBatch([(tsf.init_scheme(2, 2, 2), n, 16, 7)], rec_cap=16)
    prm = tsf.walk_params(base_seed=0, max_iters=100000, plateau=20000)
    b.init(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first, done_iters, rounds = None, 0, 0
    while done_iters < 100000:
        b.walk(ctx, prm, args.iters)
        done_iters += args.iters
        rounds += 1
        hdr = b.headers()
        if first is None and (hdr["best_rank"] <= 7).any():
            first = {"s": time.perf_counter() - t0, "iterations": done_iters}
        if (hdr["done"] != 0).all():
            break
    wall = time.perf_counter() - t0
    hdr = b.headers()
    nv = b.verify_device(1).cpu().numpy()
    rec = b.rec.cpu().numpy()
    n_rec = np.minimum(hdr["n_rec"], b.rec_cap)
    first_it = [int(rec[w, :n_rec[w], 0][(rec[w, :n_rec[w], 1] & 0xFFFFFFFF) <= 7].min())
                for w in range(n) if hdr["best_rank"][w] <= 7]
    return {"flips_per_s": int(hdr["counters"][:, 1].sum()) / wall, "wall_s": wall,
            "round_iters": args.iters, "rounds": rounds, "first_rank_7": first,
            "walks_at_7": int((hdr["best_rank"] <= 7).sum()),
            "median_iterations_to_7": float(np.median(first_it)) if first_it else None,
            "max_iterations_to_7": int(max(first_it)) if first_it else None,
            "best_schemes_failing_brent": int((nv != 0).sum())}


def time_to_rank_fine(ctx, args, target=23, round_iters=1000, limit_s=60.0):
    """Time to the target rank with rounds of round_iters iterations: a fresh
    batch of the (3,3,3) workload is walked round by round (the best rank is
    read after each round) until some walk reaches the target; the schemes are
    then Brent-checked on the GPU.  The wall time runs from the first round's
    launch to the end of the round that reached the target."""
    import torch
    from paper_2511_20317_amd import tsf
    b = tsf.WalkBatch([(tsf.init_scheme(3, 3, 3), args.walks, 35, target)], rec_cap=32)
    prm = tsf.walk_params(base_seed=0, max_iters=1000000, plateau=50000)
    b.init(ctx)
    best_col = b.hdr.view(torch.int32).view(args.walks, tsf.HEADER_I32)[:, 7]
    ladder, done = {}, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        b.walk(ctx, prm, round_iters, args.lanes, args.wpb, args.strategy)
        done += round_iters
        best = int(best_col.min().item())
        now = time.perf_counter() - t0
        for rank in (26, 25, 24, 23):
            if best <= rank and rank not in ladder:
                ladder[rank] = {"s": now, "iterations": done}
        if best <= target or now >= limit_s or done >= 1000000:
            break
    hdr = b.headers()
    hit = np.flatnonzero(hdr["best_rank"] <= target)
    nv = b.verify_device(1).cpu().numpy()
    return {"round_iters": round_iters, "time_to_rank_s": {str(k): v["s"] for k, v in ladder.items()},
            "iterations_to_rank": {str(k): v["iterations"] for k, v in ladder.items()},
            "time_to_rank_23_s": ladder[target]["s"] if target in ladder else None,
            "walks_at_target": int(hit.size),
            "walks_at_target_failing_brent": int((nv[hit] != 0).sum()) if hit.size else 0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=0,
                    help="iterations per walk per step (0: the (3,3,3) workload splits its 1e6 "
                         "budget evenly over the steps; the other workloads take 1e5)")
    ap.add_argument("--walks", type=int, default=65536)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per walk (0: library choice)")
    ap.add_argument("--wpb", type=int, default=0, help="waves per workgroup (0: library choice)")
    ap.add_argument("--strategy", type=int, default=0,
                    help="1 attempt-parallel, 2 term-parallel, 3 indexed attempt-parallel "
                         "(0: library choice)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-walks", type=int, default=512)
    ap.add_argument("--cpu-iters", type=int, default=100000)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (HBM counter scale)")
    ap.add_argument("--workload", default="333",
                    choices=["333", "222", "mixed", "large", "additions", "explore", "lift",
                             "learned-walk"],
                    help="333: the (3,3,3) benchmark; mixed / large / additions: the other "
                         "workloads")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training the proposal network and its comparison with uniform "
                         "proposals")
    ap.add_argument("--no-learned-444", action="store_true",
                    help="skip the equal-wall-time comparison on (4,4,4)")
    ap.add_argument("--learn-walks", type=int, default=2048,
                    help="(3,3,3) walks logged for training (twice as many (2,2,2) walks)")
    ap.add_argument("--learn-iters", type=int, default=6000)
    ap.add_argument("--learn-steps", type=int, default=1500)
    ap.add_argument("--ab-runs", type=int, default=9)
    ap.add_argument("--ab-walks", type=int, default=4096)
    ap.add_argument("--ab-seconds", type=float, default=1.5)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (--gpus 1): the walks would shard by walk id "
              "with no communication, and no multi-GPU path is implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_20317_amd import tsf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ctx = tsf.Context()
    if args.workload != "333":
        args.iters = args.iters or 100000
        res = {"mixed": run_mixed, "large": run_large, "additions": run_additions,
               "explore": run_explore, "lift": run_lift, "222": run_222,
               "learned-walk": run_learned_walk}[args.workload](ctx, args)
        if args.workload == "mixed":
            value = res["ternary"]["flips_per_s"]
            desc = ("131,072 walks over (3,3,4), (3,4,5), (4,4,4), (4,4,5) in one launch, "
                    "ternary then Z2")
        elif args.workload == "222":
            value = res["flips_per_s"]
            desc = "256 (2,2,2) walks from the standard rank-8 scheme to rank 7"
        elif args.workload == "explore":
            value = res["flips_per_s"]
            desc = ("exploratory search: 4 x %d walks from (2,2,2), (2,2,3), (2,3,3), (3,3,3), "
                    "rounds of walks, population sync and resize" % (args.walks // 4))
        elif args.workload == "lift":
            value = None
            desc = "ternary lifting of the best Z2 schemes of (2,2,3), (2,3,3), (3,3,3) walks"
        elif args.workload == "learned-walk":
            value = res["learned"]["flips_per_s"]
            desc = ("%d (3,3,3) walks with learned proposals (random-initialised network), "
                    "then uniform proposals, %.0f s each" % (args.ab_walks, args.ab_seconds))
        elif args.workload == "additions":
            value = res["flips_per_s"]
            desc = ("65,536 (3,3,3) walks minimising naive additions at fixed rank from the best "
                    "schemes of a 2e5-iteration rank search")
        else:
            value = res["flips_per_s"]
            desc = ("98,304 walks over (4,5,12), (5,6,10), (6,7,9) (a batch per format) with "
                    "device project to p-1 and extend back between rounds")
        out = {"metric": "flips/sec on 1 GPU", "value": value, "unit": "flips/s", "n_gpus": 1,
               "steps": res["rounds"] if args.workload == "222" else args.steps,
               "warmup": 0, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None,
               "dtype": ("u64" if args.workload in ("large", "explore") else
                         "u32/bf16" if args.workload == "learned-walk" else "u32"),
               "data": "synthetic",
               "config": ({"workload": desc, "walks": args.ab_walks, "seconds": args.ab_seconds}
                          if args.workload == "learned-walk" else
                          {"workload": desc, "walks": 256 if args.workload == "222" else args.walks,
                           "iters_per_step": args.iters}),
               "results": res}
        print(json.dumps(out))
        return
    target = 23
    iters_per_step = args.iters or -(-MAX_ITERS // args.steps)
    groups = [(tsf.init_scheme(3, 3, 3), args.walks, 35, target)]
    prm = tsf.walk_params(base_seed=0, max_iters=MAX_ITERS, plateau=50000)
    batch = tsf.WalkBatch(groups, rec_cap=32)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        batch.init(ctx)
        batch.walk(ctx, prm, iters_per_step, args.lanes, args.wpb, args.strategy)
        batch.verify_device(1)
    torch.cuda.synchronize()

    batch.init(ctx)
    hdr0 = torch.cuda.synchronize() or batch.headers()
    i32 = batch.hdr.view(torch.int32).view(args.walks, tsf.HEADER_I32)
    i64 = batch.hdr.view(torch.int64).view(args.walks, tsf.HEADER_I32 // 2)
    best_col, rank_col, iters_col, flips_col = i32[:, 7], i32[:, 6], i64[:, 8], i64[:, 9]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    ladder = {}
    bad_total = 0
    step_iters, step_flips, mean_ranks = [], [], [float(hdr0["rank"].mean())]
    last_iters, last_flips = 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        batch.walk(ctx, prm, iters_per_step, args.lanes, args.wpb, args.strategy)
        ev[k][1].record(stream)
        nv = batch.verify_device(1)
        bad_total += int((nv != 0).sum().item())
        # one read-back per step (the loop is synchronous at step granularity)
        state = torch.stack([best_col.min().to(torch.int64), iters_col.sum(), flips_col.sum(),
                             rank_col.to(torch.int64).sum()]).tolist()
        best_now = int(state[0])
        step_iters.append(state[1] - last_iters)
        step_flips.append(state[2] - last_flips)
        last_iters, last_flips = state[1], state[2]
        mean_ranks.append(state[3] / args.walks)
        now = time.perf_counter() - t0
        for rank in (26, 25, 24, 23):
            if best_now <= rank and rank not in ladder:
                ladder[rank] = now
        print("step %d/%d: %.2f s, %d iterations, best rank %d" %
              (k + 1, args.steps, now, step_iters[-1], best_now), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.calibrate_copy_mib:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE read the
        # scale of those counters
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    hdr = batch.headers()
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    cnt = {name: int(hdr["counters"][:, k].sum() - hdr0["counters"][:, k].sum())
           for k, name in enumerate(tsf.COUNTER_NAMES)}
    flips = cnt["flips"]
    iters = max(cnt["iters"], 1)
    value = flips / wall
    # launches that did work (all of them unless every walk stopped early)
    working = [k for k in range(args.steps) if step_iters[k] > 0]
    avg_ms = float(np.mean([kernel_ms[k] for k in working])) if working else None
    work_flips = sum(step_flips[k] for k in working)
    # the mean rank over the run: the average of the per-step means
    # (trapezoid over the step boundaries)
    mean_rank = float(np.mean([(a + b) / 2 for a, b in zip(mean_ranks[:-1], mean_ranks[1:])]))
    t_eff = cnt["attempts"] / iters
    a_op = ops_per_flip(mean_rank, t_eff, cnt["fallbacks"] / iters)
    achieved = (a_op * work_flips / len(working)) / (avg_ms * 1e-3) if working else 0.0
    traffic = None
    mt = MEASURED_TRAFFIC
    if (mt["bytes_per_launch"] and mt["sources_sha1"] == kernel_sources_sha1() and
            (args.walks, iters_per_step) == (mt["walks"], mt["iters"])):
        traffic = mt["bytes_per_launch"]
    # first iteration at which some walk recorded the target rank (records
    # are (iteration, rank) of every strict improvement), and its wall time at
    # the measured iteration rate
    first_hit = None
    n_rec = np.minimum(hdr["n_rec"], batch.rec_cap)
    rec = batch.rec.cpu().numpy()
    for w in np.flatnonzero(hdr["best_rank"] <= target):
        its = rec[w, :n_rec[w], 0]
        rks = rec[w, :n_rec[w], 1] & 0xFFFFFFFF
        hit = its[rks <= target]
        if hit.size and (first_hit is None or hit.min() < first_hit):
            first_hit = int(hit.min())
    ranks = np.bincount(hdr["best_rank"], minlength=28)
    fine = time_to_rank_fine(ctx, args, target)
    out = {
        "metric": "flips/sec on 1 GPU and time-to-rank-23 at (3,3,3), learned vs uniform proposal",
        "value": value,
        "unit": "flips/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "(3,3,3) ternary walks from the standard rank-27 scheme, "
                               "uniform proposals", "walks": args.walks,
                   "iters_per_step": iters_per_step, "max_iters": MAX_ITERS, "plateau": 50000,
                   "target_rank": target, "seeds": "0..%d" % (args.walks - 1),
                   "lanes_per_walk": args.lanes or "library", "parallelism": "1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / PEAK_INT32_OPS, "traffic": traffic,
                     "kernel": "walk_kernel", "kernel_avg_ms": avg_ms,
                     "working_launches": len(working), "ops_per_flip": a_op,
                     "mean_rank": mean_rank, "attempts_per_iteration": t_eff},
        "time_to_rank_23_s": fine["time_to_rank_23_s"],
        "time_to_rank_23_fine": fine,
        "time_to_rank_s_at_step_ends": ladder,
        "first_rank_23_iteration": first_hit,
        "walks_at_rank": {str(r): int(ranks[r]) for r in range(20, 28) if ranks[r]},
        "iterations_per_s": iters / wall,
        "attempts_per_iteration": t_eff,
        "fallback_rate": cnt["fallbacks"] / iters,
        "best_schemes_failing_brent": bad_total,
        "learned_vs_uniform": None,
    }
    if not args.no_learned:
        out["learned_vs_uniform"] = learned_vs_uniform(ctx, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_walks, args.cpu_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
