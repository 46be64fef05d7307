"""On-device midplane statistics (paper, Section 3, eqs. (4)-(5)) against the
oracle: the histogram of midplane Tr c accumulated over steps must hold the
oracle's counts bin by bin, except that a sample lying within the two sides'
difference of a bin edge may fall on either side of it (such samples are
counted and bound the allowed difference)."""

import numpy as np
import pytest

from oracle import Grid, Oracle, Params
from oracle import stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import os

    import torch

    import paper_2606_09468_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(P.LIBPATH):
        from paper_2606_09468_amd import build
        build.build()
    return P


def oracle_midplane_samples(g, prm, nsteps, seed, amp):
    """Midplane Tr c after each step, and the largest |Tr c| of the domain
    (the field errors of both sides are relative to that scale)."""
    o = Oracle(g, Params(**prm), seed=seed, amp=amp)
    out, top = [], 0.0
    for _ in range(nsteps):
        o.step(1)
        trc = o.trace_c()
        out.append(trc[o.N // 2].ravel().copy())
        top = max(top, float(np.abs(trc).max()))
    return np.concatenate(out), top


# rel: the field tolerance of the path relative to the largest |Tr c| (FP64:
# 1e-12 at these sizes, with margin; mixed: 2e-5 over the full field, the
# conformation measured near 1e-8)
@pytest.mark.parametrize("dims,precision,rel", [((2, 32, 33, 1), 0, 1e-11), ((3, 16, 17, 16), 0, 1e-11),
                                                ((2, 32, 33, 1), 1, 2e-8)])
def test_midplane_histogram_matches_oracle(P, dims, precision, rel):
    dim, nx, ny, nz = dims
    g = Grid(dim, nx, ny, nz)
    prm = dict(wi=20.0, dt=1e-3)
    nsteps, seed, amp = 12, 6, 1e-2
    ref, top = oracle_midplane_samples(g, prm, nsteps, seed, amp)
    # a range with 3 on a bin edge and some samples outside on both sides
    spread = np.abs(ref - 3.0).max()
    nb = 40
    lo, hi = 3.0 - 0.8 * spread, 3.0 + 0.8 * spread
    print("case histogram %s p%d lo %.6g hi %.6g" % (dims, precision, lo, hi), flush=True)
    sim = P.Sim(P.make_grid(dim, nx, ny, nz), P.make_params(precision=precision, **prm), seed=seed, amp=amp)
    sim.midplane_histogram_setup(lo, hi, nb)
    sim.step(nsteps)
    got = sim.midplane_histogram()
    recs, st = sim.diagnostics()
    sim.close()
    want = stats.histogram(ref, lo, hi, nb)
    assert int(got.sum()) == nsteps * nx * (nz if dim == 3 else 1) == int(want.sum())
    assert got[0] + got[nb + 1] > 0
    # samples within the two sides' difference of an edge may move one bin
    u = (ref - lo) * (nb / (hi - lo))
    ties = int(np.count_nonzero(np.abs(u - np.round(u)) < rel * top * nb / (hi - lo) + 1e-12))
    diff = int(np.abs(got.astype(np.int64) - want.astype(np.int64)).sum())
    print("histogram L1 difference %d, samples near an edge %d" % (diff, ties), flush=True)
    assert diff <= 2 * ties
    # 3 is the edge between bins nb/2 and nb/2 + 1: the counts below it are
    # the step records' midplane counts of Tr c < 3 (same kernel, exact)
    assert int(got[:nb // 2 + 1].sum()) == sum(r["mid_n_lt3"] for r in recs)


def test_midplane_histogram_arguments_and_reset(P):
    sim = P.Sim(P.make_grid(2, 16, 17), P.make_params(wi=20.0, dt=1e-3), seed=1, amp=1e-3)
    with pytest.raises(P.PcsError) as e:
        sim.midplane_histogram()                      # off by default
    assert e.value.status == P.PCS_ERR_ARG
    for lo, hi, nb in ((1.0, 1.0, 8), (2.0, 1.0, 8), (0.0, 1.0, P.PCS_HIST_MAX + 1), (0.0, float("inf"), 8),
                       (0.0, 1.0, -1)):
        with pytest.raises(P.PcsError) as e:
            sim.midplane_histogram_setup(lo, hi, nb)
        assert e.value.status == P.PCS_ERR_ARG
    sim.midplane_histogram_setup(0.0, 10.0, 8)
    sim.step(3)
    assert int(sim.midplane_histogram().sum()) == 3 * 16
    sim.midplane_histogram_setup(0.0, 10.0, 8)        # setup clears the counts
    sim.step(2)
    assert int(sim.midplane_histogram().sum()) == 2 * 16
    sim.midplane_histogram_setup(0.0, 0.0, 0)         # off again
    sim.step(1)
    sim.close()


def test_ensemble_member_histogram_equals_single_run(P):
    """A member's histogram is the single run's (the ensemble advances each
    member exactly as a single run)."""
    grids = [(2, 32, 33, 1), (2, 16, 17, 1)]
    ens = P.Ensemble([P.make_grid(*g) for g in grids], [P.make_params(wi=20.0, dt=1e-3)] * 2, [3, 4], amp=1e-2)
    ens.midplane_histogram_setup(0, 2.9, 3.1, 32)
    ens.step(6)
    got = ens.midplane_histogram(0)
    with pytest.raises(P.PcsError):
        ens.midplane_histogram(1)                     # off for the other member
    ens.close()
    sim = P.Sim(P.make_grid(*grids[0]), P.make_params(wi=20.0, dt=1e-3), seed=3, amp=1e-2)
    sim.midplane_histogram_setup(2.9, 3.1, 32)
    sim.step(6)
    ref = sim.midplane_histogram()
    sim.close()
    assert np.array_equal(got, ref) and int(got.sum()) == 6 * 32
