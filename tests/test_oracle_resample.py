"""Pins of the oracle's state resampling (restart at another resolution)
against facts that do not depend on it:
  * the seeded initial condition is one continuous field, polynomial in y
    (laminar profiles of degree <= 2 at kappa = 0, perturbation of degree
    <= 8) with Fourier modes |m| <= 4; carried between two grids that both
    hold it exactly, it must equal the initial condition built directly on
    the target grid (this fixes the Fourier mode map, the Chebyshev
    interpolant and the header at once);
  * a Chebyshev polynomial T_k of degree above the target's N' is dropped
    (truncation, not re-interpolation), one of degree <= N' is kept exactly;
  * refining then coarsening returns the original state;
  * point values of a random field at arbitrary (x, y, z) survive a
    refinement (evaluated by a direct sum written here)."""

import numpy as np
import pytest

from oracle import Grid, Oracle, Params, state_layout
from oracle.resample import lobatto, resample_state
from tests.inputs import random_state

PRM = Params(kappa=0.0)


def nq(dim):
    return 6 if dim == 2 else 11


def q_part(state, g):
    h, _, per = state_layout(g)
    return state[h: h + nq(g.dim) * per * 2]


@pytest.mark.parametrize("a,b", [
    (Grid(2, 12, 17), Grid(2, 16, 25)),
    (Grid(2, 16, 25), Grid(2, 12, 17)),
    (Grid(3, 10, 13, 10), Grid(3, 12, 17, 16)),
    (Grid(3, 12, 17, 16), Grid(3, 10, 13, 10)),
])
def test_initial_condition_carries_between_grids(a, b):
    sa = Oracle(a, PRM, seed=7, amp=1e-3, cache_lu=False).get_state()
    sb = Oracle(b, PRM, seed=7, amp=1e-3, cache_lu=False).get_state()
    r = resample_state(a, sa, b)
    assert r.size == sb.size
    assert np.array_equal(r[:4], sa[:4])
    qa, qb = q_part(r, b), q_part(sb, b)
    assert np.abs(qa - qb).max() <= 1e-12 * np.abs(qb).max()


def test_chebyshev_truncation_and_exactness():
    N, Np = 24, 16
    g, gd = Grid(2, 4, N + 1), Grid(2, 4, Np + 1)
    h, names, per = state_layout(g)
    y, yd = lobatto(N), lobatto(Np)
    for k, expect in ((20, np.zeros(Np + 1)), (16, np.cos(16 * np.arccos(yd))), (7, np.cos(7 * np.arccos(yd)))):
        s = np.zeros(h + len(names) * per * 2)
        f = np.cos(k * np.arccos(np.clip(y, -1, 1)))
        s[h: h + 2 * per: 2 * (g.nx // 2)] = f          # field u, mode kx = 0, real part
        r = resample_state(g, s, gd)
        hd, _, pd = state_layout(gd)
        got = r[hd: hd + 2 * pd: 2 * (gd.nx // 2)]
        assert np.abs(got - expect).max() <= 1e-13, k
        assert np.count_nonzero(r[hd + 2 * pd:]) == 0


@pytest.mark.parametrize("a,b", [(Grid(2, 12, 17), Grid(2, 20, 33)), (Grid(3, 8, 13, 8), Grid(3, 12, 21, 16))])
def test_refine_then_coarsen_is_identity(a, b):
    s = random_state(a.dim, a.nx, a.ny, a.nz, seed=3, amp=1.0)
    h, names, per = state_layout(a)
    # the source Nyquist slot is not part of the state's content
    if a.dim == 3:
        v = s[h:].reshape(len(names), a.ny, a.nz, a.nx // 2, 2)
        v[:, :, a.nz // 2] = 0
    back = resample_state(b, resample_state(a, s, b), a)
    assert np.abs(back - s).max() <= 1e-13 * np.abs(s).max()


def point_values(g, state, pts):
    """u(x, y, z) by a direct sum over the stored modes: real field =
    sum over kx >= 0 with weight 1 at kx = 0 and 2 above, real part."""
    h, _, per = state_layout(g)
    nzs = 1 if g.dim == 2 else g.nz
    q = (state[h:h + 2 * per:2] + 1j * state[h + 1:h + 2 * per:2]).reshape(g.ny, nzs, g.nx // 2)
    N = g.ny - 1
    yj = lobatto(N)
    out = []
    for x, y, z in pts:
        # Lagrange interpolation through the Lobatto points (barycentric form)
        w = np.ones(N + 1)
        w[1::2] = -1
        w[0] *= 0.5
        w[N] *= 0.5
        lw = w / (y - yj)
        lw /= lw.sum()
        col = np.tensordot(lw, q, axes=(0, 0))              # [slot, kx]
        val = 0.0
        for s in range(nzs):
            if nzs > 1 and s == nzs // 2:
                continue
            mz = 0 if nzs == 1 else (s if s < nzs // 2 else s - nzs)
            for k in range(g.nx // 2):
                ph = 2 * np.pi * (k * x / g.lx + mz * z / g.lz)
                val += (1 if k == 0 else 2) * (col[s, k] * np.exp(1j * ph)).real
        out.append(val)
    return np.array(out)


def test_point_values_survive_refinement():
    a, b = Grid(3, 8, 13, 8), Grid(3, 12, 17, 12)
    s = random_state(3, a.nx, a.ny, a.nz, seed=11, amp=1.0)
    r = resample_state(a, s, b)
    pts = np.random.default_rng(0).uniform([0, -0.99, 0], [a.lx, 0.99, a.lz], size=(8, 3))
    va, vb = point_values(a, s, pts), point_values(b, r, pts)
    assert np.abs(va - vb).max() <= 1e-12 * max(1.0, np.abs(va).max())


def test_rejects_mismatched_boxes():
    s = np.zeros(state_layout(Grid(2, 8, 9))[0] + 10 * 9 * 4 * 2)
    with pytest.raises(ValueError):
        resample_state(Grid(2, 8, 9), s, Grid(2, 8, 9, lx=5.0))
    with pytest.raises(ValueError):
        resample_state(Grid(2, 8, 9), s, Grid(3, 8, 9, 8))
