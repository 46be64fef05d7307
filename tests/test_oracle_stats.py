"""Pins of the oracle's midplane statistics (paper, Section 3, eqs. (4)-(5))
against their definitions: bin membership by construction, the outer
counts, the probability and chi of a hand-counted example, and agreement of
the counts below 3 with the oracle's own per-step midplane count."""

import numpy as np

from oracle import Grid, Oracle, Params
from oracle import stats


def test_histogram_bins_by_construction():
    lo, hi, nb = -2.0, 6.0, 16
    w = (hi - lo) / nb
    centres = lo + (np.arange(nb) + 0.5) * w          # one sample at every bin centre
    edges = lo + np.arange(nb) * w                     # lower edges belong to their bin
    extra = np.array([lo - 1e-9, -np.inf, hi, hi + 1.0, np.inf, np.nan])
    c = stats.histogram(np.concatenate([centres, edges, extra]), lo, hi, nb)
    assert c.dtype == np.uint64 and c.size == nb + 2
    assert c[0] == 2                                   # below lo, -inf
    assert np.all(c[1:nb + 1] == 2)                    # centre and lower edge of each bin
    assert c[nb + 1] == 4                              # hi, above, +inf, NaN
    assert int(c.sum()) == 2 * nb + extra.size


def test_probability_and_chi_hand_counted():
    # two snapshots of a 4 x 1 midplane: samples below 3 are 2.5, 1.0 and -0.5
    snaps = np.array([[2.5, 3.0, 4.0, 1.0], [3.5, -0.5, 3.0, 7.0]])
    assert stats.probability_below(snaps) == 3 / 8          # eq. (4) over 8 samples
    assert stats.chi(snaps, nx=4, nz=1) == 8 * (3 / 8) / 4  # eq. (5): 3 events per 4 points
    assert stats.probability_below([3.0]) == 0.0            # strict inequality


def test_histogram_below_three_matches_midplane_count():
    """With 3 on a bin edge, the counts below 3 are the oracle diagnostics'
    mid_n_lt3 (the same midplane row, y = 0 at Lobatto row N/2)."""
    g = Grid(2, 32, 33)
    o = Oracle(g, Params(wi=20.0, dt=1e-3), seed=5, amp=1e-2)
    lo, hi, nb = 3.0 - 8 * 1e-3, 3.0 + 8 * 1e-3, 16       # edge at 3 between bins 8 and 9
    tot = np.zeros(nb + 2, dtype=np.uint64)
    n3 = 0
    for _ in range(4):
        o.step(1)
        mid = o.trace_c()[o.N // 2]
        assert np.all(np.isfinite(mid)) and mid.size == g.nx
        tot += stats.histogram(mid, lo, hi, nb)
        n3 += o.diagnostics()["mid_n_lt3"]
    assert int(tot[:nb // 2 + 1].sum()) == n3
    assert int(tot.sum()) == 4 * g.nx


def test_midplane_gradients_by_direct_sums():
    """The midplane velocity gradients of oracle.stats (spectral derivatives
    through the oracle's base-grid transform) against direct Fourier sums of
    i kx u-hat and i kz u-hat (and of w) at every base-grid point of the
    midplane, from the Chebyshev series of each mode evaluated at y = 0 with
    numpy.polynomial; the fluctuations u - U(0), w - W(0) likewise."""
    from tests.inputs import random_state
    from tests.test_oracle_assembly_pins import SField
    for dims in ((3, 12, 17, 8), (2, 16, 17, 1)):
        dim, nx, ny, nz = dims
        o = Oracle(Grid(dim, nx, ny, nz), Params(), seed=None)
        o.set_state(random_state(dim, nx, ny, nz, seed=12, amp=1.0))
        got = stats.midplane_quantities(o)
        xs = np.arange(nx) * o.g.lx / nx
        zs = np.arange(nz) * o.g.lz / nz if dim == 3 else np.zeros(1)
        y0 = np.zeros(1)
        u = SField.from_lobatto(o.q["u"], o.kx, o.kz)
        want = {4: u.dx().eval(xs, y0, zs)[0]}
        mean_u = u.coef[:, 0, 0].real
        import numpy.polynomial.chebyshev as npc
        want[1] = u.eval(xs, y0, zs)[0] - npc.chebval(0.0, mean_u)
        if dim == 3:
            w = SField.from_lobatto(o.q["w"], o.kx, o.kz)
            want[5] = u.dz().eval(xs, y0, zs)[0]
            want[6] = w.dx().eval(xs, y0, zs)[0]
            want[7] = w.dz().eval(xs, y0, zs)[0]
            want[3] = w.eval(xs, y0, zs)[0] - npc.chebval(0.0, w.coef[:, 0, 0].real)
        for k, v in want.items():
            g = got[k].reshape(v.shape)
            sc = np.abs(v).max()
            assert sc > 1e-3, (dims, k)
            assert np.abs(g - v).max() <= 1e-12 * sc, (dims, k, np.abs(g - v).max() / sc)
        # moments are the plain sums of the finite samples
        n, s1, s2 = stats.moments(np.array([1.0, 2.0, np.nan, 4.0]))
        assert (n, s1, s2) == (3.0, 7.0, 21.0)
