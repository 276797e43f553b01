"""Training and evaluation of the learned flip proposal (host driver).

All arithmetic runs in libtsf's kernels: the walks (with their training
log), the feature rows, and the network's forward, backward and Adam steps.
This module only orchestrates: it labels logged iterations, samples
minibatches and times the comparison with uniform proposals.

Label of a logged iteration t of a walk (a flip was applied): 1 if the walk's
rank after some iteration in (t, t + window] is below its rank after t,
else 0; iterations whose window runs past the end of the log are dropped.
The default window is LABEL_WINDOW = 20 flips: with the 1000-flip window the
labels carry no signal that the network can rank (held-out AUC 0.51 on
(2,2,2) walks, 0.50 on (3,3,3) walks); with 20 flips, trained on the logs
below with a quarter of every minibatch drawn from the rare positives, it
ranks held-out (2,2,2) flips at AUC 0.67-0.69 (0.48-0.49 untrained).

The training set is the one the proposal's workload names: logged flips of
uniform walks of the (2,2,2) and the (3,3,3) workloads (training_set).
"""
import time

import numpy as np

from . import tsf

LABEL_WINDOW = 20


def window_min_after(x, window):
    """m[t] = min(x[t+1 .. t+window]) per row (inf where the window is cut)."""
    L = x.shape[-1]
    big = np.iinfo(np.int32).max
    shifted = np.full(x.shape, big, dtype=np.int64)
    shifted[..., :-1] = x[..., 1:]
    # sliding minimum of width `window` by doubling: mins of widths 1, 2, 4, ...
    res = np.full(x.shape, big, dtype=np.int64)
    cur = shifted.copy()
    width, offset = 1, 0
    w = window
    while w:
        if w & 1:
            part = np.full(x.shape, big, dtype=np.int64)
            if offset < L:
                part[..., :L - offset] = cur[..., offset:]
            res = np.minimum(res, part)
            offset += width
        nxt = np.full(x.shape, big, dtype=np.int64)
        if width < L:
            nxt[..., :L - width] = cur[..., width:]
        cur = np.minimum(cur, nxt)
        width *= 2
        w >>= 1
    return res


def collect(ctx, scheme, n_walks, n_iters, r_cap, base_seed=1000, window=LABEL_WINDOW, prm=None):
    """Run uniform walks with the training log on; returns (records tensor on
    the GPU, int64 indices of usable records, float32 labels)."""
    import torch
    b = tsf.WalkBatch([(scheme, n_walks, r_cap, 0)], rec_cap=4, log_cap=n_iters)
    b.init(ctx)
    prm = prm or tsf.walk_params(base_seed=base_seed, max_iters=n_iters, plateau=50000)
    b.walk(ctx, prm, n_iters)
    torch.cuda.synchronize()
    rec = b.log.reshape(-1, 16)
    words = rec[:, 1].cpu().numpy()  # rank_before | rank_after << 32
    rank_before = (words & 0xFFFFFFFF).astype(np.int64)
    rank_before[rank_before >= 1 << 31] -= 1 << 32
    rank_after = (words >> 32).astype(np.int64)
    ra = rank_after.reshape(n_walks, n_iters)
    later = window_min_after(ra, window)
    label = (later < ra).reshape(-1)
    usable = (rank_before >= 0).reshape(n_walks, n_iters)
    usable[:, n_iters - window:] = False
    idx = np.flatnonzero(usable.reshape(-1))
    return rec, idx, label[idx].astype(np.float32)


def training_set(ctx, n222=4096, n333=2048, n_iters=6000, base_seed=10 ** 7,
                 window=LABEL_WINDOW):
    """Logged flips of uniform (2,2,2) and (3,3,3) walks from the standard
    schemes (r_cap = r0 + 8), labelled: (records of both logs concatenated,
    usable indices into them, labels)."""
    import torch
    r2, i2, l2 = collect(ctx, tsf.init_scheme(2, 2, 2), n222, n_iters, 16, base_seed, window)
    r3, i3, l3 = collect(ctx, tsf.init_scheme(3, 3, 3), n333, n_iters, 35, base_seed + n222,
                         window)
    rec = torch.cat([r2, r3], 0)
    return rec, np.concatenate([i2, i3 + r2.shape[0]]), np.concatenate([l2, l3])


def reach(ctx, scheme, r_cap, n_walks, n_iters, ladder, base_seed, net=None):
    """Walk n_walks walks for n_iters iterations (learned proposals with
    `net`, else uniform); per rung of the ladder, the fraction of walks whose
    best rank reached it and the mean first iteration of those that did
    (from the improvement records), and the wall time."""
    import torch
    b = tsf.WalkBatch([(scheme, n_walks, r_cap, 0)], rec_cap=64)
    b.init(ctx)
    prm = tsf.walk_params(base_seed=base_seed, max_iters=n_iters, plateau=50000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if net is None:
        b.walk(ctx, prm, n_iters)
    else:
        b.walk_learned(ctx, prm, net, tsf.LearnWorkspace(n_walks), n_iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hdr = b.headers()
    rec = b.rec.cpu().numpy()
    n_rec = np.minimum(hdr["n_rec"], b.rec_cap)
    out = {}
    for rank in ladder:
        first = []
        for w in range(n_walks):
            its = rec[w, :n_rec[w], 0]
            rks = rec[w, :n_rec[w], 1] & 0xFFFFFFFF
            hit = its[rks <= rank]
            if hit.size:
                first.append(int(hit.min()))
        out[str(rank)] = {"fraction": len(first) / n_walks,
                          "mean_first_iteration": float(np.mean(first)) if first else None}
    return {"wall_s": wall, "iterations": n_iters, "walks": n_walks, "ranks": out}


def train(net, rec, idx, labels, steps, batch=4096, lr=1e-3, seed=0, log_every=0,
          pos_share=None):
    """Minibatch Adam on the binary cross-entropy; returns the loss history.
    pos_share: draw that share of every minibatch from the positive records
    (the rest from the negatives) instead of uniformly -- positives are rare,
    and only the ranking of candidates is used."""
    import torch
    rng = np.random.default_rng(seed)
    dev = rec.device
    lab = torch.from_numpy(labels).to(dev)
    idx_d = torch.from_numpy(idx).to(dev)
    pos = np.flatnonzero(labels > 0.5)
    neg = np.flatnonzero(labels < 0.5)
    hist = []
    for s in range(steps):
        if pos_share and pos.size and neg.size:
            n_pos = int(round(batch * pos_share))
            sel = np.concatenate([pos[rng.integers(0, pos.size, n_pos)],
                                  neg[rng.integers(0, neg.size, batch - n_pos)]])
        else:
            sel = rng.integers(0, idx.size, batch)
        pick = torch.from_numpy(sel).to(dev)
        rows = rec.index_select(0, idx_d.index_select(0, pick)).contiguous()
        X = tsf.features_from_log(rows)
        y = lab.index_select(0, pick).contiguous()
        h1, h2, logit = net.forward(X)
        loss = net.backward(X, y, h1, h2, logit)
        net.step(lr=lr)
        if log_every and (s % log_every == 0 or s == steps - 1):
            hist.append((s, float(loss.item())))
    return hist


def evaluate(net, rec, idx, labels, n=65536, seed=1):
    """Loss and ranking quality (AUC) of the network on sampled records."""
    import torch
    rng = np.random.default_rng(seed)
    dev = rec.device
    pick = rng.choice(idx.size, min(n, idx.size), replace=False)
    rows = rec.index_select(0, torch.from_numpy(idx[pick]).to(dev)).contiguous()
    X = tsf.features_from_log(rows)
    _, _, logit = net.forward(X)
    z = logit.cpu().numpy().astype(np.float64)
    y = labels[pick].astype(np.float64)
    loss = float(np.mean(np.logaddexp(0.0, z) - y * z))
    pos, neg = z[y > 0.5], z[y < 0.5]
    if pos.size == 0 or neg.size == 0:
        auc = float("nan")
    else:
        order = np.argsort(np.concatenate([pos, neg]))
        ranks = np.empty(order.size)
        ranks[order] = np.arange(1, order.size + 1)
        auc = float((ranks[:pos.size].sum() - pos.size * (pos.size + 1) / 2) / (pos.size * neg.size))
    return {"loss": loss, "auc": auc, "positives": float(y.mean()), "n": int(y.size)}


def time_to_ranks(ctx, scheme, n_walks, r_cap, ladder, wall_s, base_seed, net=None,
                  iters_per_call=None, prm_kw=None):
    """Walk n_walks walks (learned proposals when net is given, else uniform)
    until wall_s seconds have passed; returns the wall time and the iteration at
    which the batch's best rank first reached each rung of the ladder."""
    import torch
    b = tsf.WalkBatch([(scheme, n_walks, r_cap, min(ladder))], rec_cap=64)
    b.init(ctx)
    kw = dict(base_seed=base_seed, max_iters=10 ** 9, plateau=50000)
    kw.update(prm_kw or {})
    prm = tsf.walk_params(**kw)
    ws = tsf.LearnWorkspace(n_walks) if net is not None else None
    best_col = b.hdr.view(torch.int32).view(n_walks, tsf.HEADER_I32)[:, 7]
    iters_per_call = iters_per_call or (20 if net is not None else 2000)
    hit_s = {}
    done_iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        if net is not None:
            b.walk_learned(ctx, prm, net, ws, iters_per_call)
        else:
            b.walk(ctx, prm, iters_per_call)
        done_iters += iters_per_call
        best = int(best_col.min().item())
        now = time.perf_counter() - t0
        for rank in ladder:
            if best <= rank and rank not in hit_s:
                hit_s[rank] = now
        if now >= wall_s or best <= min(ladder):
            break
    hdr = b.headers()
    # the exact first iteration of each rung, from the walks' improvement
    # records (iteration, rank): independent of the call granularity
    rec = b.rec.cpu().numpy()
    n_rec = np.minimum(hdr["n_rec"], b.rec_cap)
    first_it = {}
    for w in range(n_walks):
        its = rec[w, :n_rec[w], 0]
        rks = rec[w, :n_rec[w], 1] & 0xFFFFFFFF
        for rank in ladder:
            hit = its[rks <= rank]
            if hit.size and (rank not in first_it or hit.min() < first_it[rank]):
                first_it[rank] = int(hit.min())
    return {"wall_s": now, "iterations": done_iters, "time_to_rank_s": hit_s,
            "iters_to_rank": first_it, "flips": int(hdr["counters"][:, 1].sum()),
            "best_rank": int(hdr["best_rank"].min())}
