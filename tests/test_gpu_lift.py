"""Ternary lifting on the GPU (tsf_lift) against the oracle's exhaustive
search in the same order: where the oracle finishes, the GPU returns the same
first lifting (or also proves there is none); where the oracle runs out of
budget, any lifting the GPU returns is checked for validity."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2511_20317_amd import tsf
from tests.golden_io import load_formula_scheme

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tsf.Context()


def _to_tsf(z):
    d = O.from_c(z)
    return tsf.Scheme(z.m, z.n, z.p, d["U"], d["V"], d["W"], tsf.TSF_Z2 if z.z2 else tsf.TSF_TERNARY)


def _z2_of(s):
    d = O.from_c(s)
    return O.to_c(np.abs(d["U"]), np.abs(d["V"]), np.abs(d["W"]), s.m, s.n, s.p, z2=True)


def _cases():
    U, V, W = load_formula_scheme("strassen_formulas.txt")[3:]
    out = [("strassen", O.to_c(np.abs(U), np.abs(V), np.abs(W), 2, 2, 2, z2=True))]
    for fmt, iters in [((2, 2, 2), 3000), ((2, 2, 3), 3000), ((2, 3, 3), 300)]:
        m, n, p = fmt
        for seed in range(4):
            prm = O.make_params(seed=seed, max_iters=iters, plateau=10 ** 6, target_rank=0,
                                r0=m * n * p)
            w = O.new_walk(O.standard(m, n, p))
            O.run(w, prm, iters)
            out.append(("%s/%d" % (fmt, seed), _z2_of(w.cur)))
    # Z2 walk schemes (rank 7..10); the first two (seed, iterations) pairs end
    # in schemes without a lifting (the oracle proves none)
    for seed, iters in ((92, 60), (138, 150), (3, 300)):
        prm = O.make_params(seed=seed, max_iters=iters, plateau=10 ** 6, target_rank=0, r0=8,
                            t_expand=1 << 30)
        w = O.new_walk(O.standard(2, 2, 2, z2=True))
        O.run(w, prm, iters)
        out.append(("z2walk/%d/%d" % (seed, iters), O.copy(w.cur)))
    return out


def test_lift_matches_oracle(ctx):
    none_seen = 0
    for name, z in _cases():
        ost, ot, _ = O.lift(z, 2 * 10 ** 6)
        info, got = tsf.lift(_to_tsf(z), max_nodes=1 << 20, max_subtrees=1 << 14)
        if ost == 1:
            assert info["status"] == 1, (name, info)
            do = O.from_c(ot)
            for g, o in zip(got.live(), (do["U"], do["V"], do["W"])):
                assert np.array_equal(g, o), name
        elif ost == 0:
            assert info["status"] == 0, (name, info)
            none_seen += 1
        if info["status"] in (1, 2):
            assert tsf.verify(got) == 0, name
            for g, zz in zip(got.live(), _to_tsf(z).live()):
                assert np.array_equal(np.abs(g), zz), name
    assert none_seen >= 1


def test_lift_input_capacity_larger_than_rank(ctx):
    """The output keeps its own capacity when the input has spare rows."""
    U, V, W = load_formula_scheme("strassen_formulas.txt")[3:]
    z = tsf.Scheme(2, 2, 2, np.abs(U), np.abs(V), np.abs(W), tsf.TSF_Z2, capacity=40)
    info, got = tsf.lift(z)
    assert info["status"] == 1 and got.rank == 7 and tsf.verify(got) == 0
