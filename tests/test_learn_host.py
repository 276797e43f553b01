"""CPU checks of the learned-proposal driver's host logic (labelling)."""
import numpy as np

from paper_2511_20317_amd.learn import window_min_after


def test_window_min_matches_brute_force():
    rng = np.random.default_rng(0)
    for L, W in [(1, 1), (7, 3), (50, 1), (50, 13), (64, 64), (100, 1000)]:
        x = rng.integers(0, 30, (4, L))
        got = window_min_after(x, W)
        for r in range(4):
            for t in range(L):
                seg = x[r, t + 1:t + 1 + W]
                want = seg.min() if seg.size else np.iinfo(np.int32).max
                assert got[r, t] == want, (L, W, r, t)
