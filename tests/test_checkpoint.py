"""Checkpoints of a walk batch (WalkBatch.save / WalkBatch.load) and the host
state check behind them (tsf_state_check): a checkpoint reads back bit for
bit, and a damaged one is refused with the status of its first failing
check instead of being walked.  CPU only: the batch lives in host memory and
its state is set up as tsf_walk_init leaves it (current = best = start)."""
import numpy as np
import pytest

from paper_2511_20317_amd import tsf


def _batch():
    groups = [(tsf.init_scheme(2, 2, 2), 4, 12, 7), (tsf.init_scheme(3, 3, 3), 4, 35, 23)]
    b = tsf.WalkBatch(groups, capacity=35, rec_cap=8, device="cpu")
    h = b.headers()
    h["rank"] = h["start_rank"]
    h["best_rank"] = h["start_rank"]
    b.hdr.copy_(b.torch.from_numpy(h.view(np.uint8).reshape(-1).copy()))
    b.cur.copy_(b.start)
    b.best.copy_(b.start)
    return b


def _save(b, tmp_path, name="ck.npz", prm=None):
    path = str(tmp_path / name)
    b.save(path, prm)
    return path


def _rewrite(path, **arrays):
    z = dict(np.load(path, allow_pickle=False))
    z.update(arrays)
    np.savez(path, **z)


def test_checkpoint_reads_back_bit_for_bit(tmp_path):
    b = _batch()
    c = tsf.WalkBatch.load(_save(b, tmp_path), device="cpu")
    assert np.array_equal(c.headers(), b.headers())
    for k in ("cur", "best", "start", "rec"):
        assert np.array_equal(getattr(c, k).numpy(), getattr(b, k).numpy()), k
    assert (c.n_walks, c.capacity, c.mode, c.rec_cap) == (b.n_walks, b.capacity, b.mode, b.rec_cap)


def test_damaged_coefficients_are_refused(tmp_path):
    b = _batch()
    path = _save(b, tmp_path)
    # a sign without its digit in walk 5's current scheme
    cur = b.cur.numpy().copy()
    d = int(cur[5, 3, 0])
    free = (~d) & 0x1FF
    cur[5, 3, 1] = np.int64(int(cur[5, 3, 1]) | (free & -free))
    _rewrite(path, cur=cur)
    st, first = tsf.state_check(np.load(path)["hdr"].view(tsf.HEADER_DTYPE), cur,
                                b.best.numpy(), b.start.numpy(), 35)
    assert (st, first) == (tsf.TSF_E_NOT_TERNARY, 5)
    with pytest.raises(tsf.TsfError) as e:
        tsf.WalkBatch.load(path, device="cpu")
    assert e.value.status == tsf.TSF_E_NOT_TERNARY


def test_a_scheme_off_the_brent_equations_is_refused(tmp_path):
    b = _batch()
    path = _save(b, tmp_path)
    # walk 2's best scheme: one w coefficient changes sign (still well coded)
    best = b.best.numpy().copy()
    best[2, 1, 5] = np.int64(int(best[2, 1, 5]) ^ int(best[2, 1, 4]))
    _rewrite(path, best=best)
    with pytest.raises(tsf.TsfError) as e:
        tsf.WalkBatch.load(path, device="cpu")
    assert e.value.status == tsf.TSF_E_INVALID_SCHEME
    # without the Brent check the coding alone passes
    assert tsf.WalkBatch.load(path, device="cpu", brent=False).n_walks == 8


def test_bad_ranks_and_flagged_walks(tmp_path):
    b = _batch()
    path = _save(b, tmp_path)
    h = b.headers()
    h["rank"][6] = h["r_cap"][6] + 1
    _rewrite(path, hdr=h)
    with pytest.raises(tsf.TsfError) as e:
        tsf.WalkBatch.load(path, device="cpu")
    assert e.value.status == tsf.TSF_E_CAPACITY
    # a walk that a walk call flagged (done < 0) is never advanced again, so
    # its state is not checked
    h["done"][6] = -2
    _rewrite(path, hdr=h)
    assert tsf.WalkBatch.load(path, device="cpu").headers()["done"][6] == -2


def test_not_a_checkpoint_or_other_parameters(tmp_path):
    b = _batch()
    prm = tsf.walk_params(base_seed=3)
    path = _save(b, tmp_path, prm=prm)
    _rewrite(path, version=np.int32(tsf.CHECKPOINT_VERSION + 1))
    with pytest.raises(tsf.TsfError) as e:
        tsf.WalkBatch.load(path, device="cpu")
    assert e.value.status == tsf.TSF_E_STATE
    path = _save(b, tmp_path, "ck2.npz", prm=prm)
    h = b.headers()
    h["params_hash"] = tsf.params_hash(tsf.walk_params(base_seed=4))
    _rewrite(path, hdr=h)
    assert tsf.WalkBatch.load(path, device="cpu").n_walks == 8
    with pytest.raises(tsf.TsfError) as e:
        tsf.WalkBatch.load(path, prm=prm, device="cpu")
    assert e.value.status == tsf.TSF_E_STATE
    tsf.WalkBatch.load(path, prm=tsf.walk_params(base_seed=4), device="cpu")
