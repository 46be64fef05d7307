"""pcs_init_static, the allocation-free variant of pcs_init (its workspace is
the library's static device array): runs set up through it must match runs
set up through pcs_init with a caller-allocated workspace, to the parity bars
of the step (FP64: the prognostic and history tolerances; mixed: the mixed
bar), on calls one after another that reuse the same array, each next one
with a smaller input.  Also: the size limit and the one-live-handle rule."""

import numpy as np
import pytest

from oracle import Grid, state_layout
from tests.test_gpu_parity import P, check_counts, fluct_errors, mixed_ok, tol_history, tol_prognostic  # noqa: F401

pytestmark = pytest.mark.gpu


def run(P, g, prm, nsteps, static):
    sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(**prm), seed=3, amp=1e-3,
                static=static)
    sim.step(nsteps)
    recs, st = sim.diagnostics()
    a = sim.get_state()
    sim.close()
    assert st == P.PCS_OK and len(recs) == nsteps
    return a, recs


CALLS = [
    ("2D 256x257 mixed x12", Grid(2, 256, 257), dict(wi=50.0, dt=5e-4, precision=1), 12),
    ("3D 16x17x16 FP64 x12", Grid(3, 16, 17, 16), dict(wi=20.0, dt=1e-3), 12),
    ("2D 32x33 FP64 x12", Grid(2, 32, 33), dict(wi=20.0, dt=1e-3), 12),
]


def test_static_init_matches_workspace_init(P):
    """Three calls in a row on one GPU, each smaller than the one before,
    each against pcs_init with its own workspace."""
    for case, g, prm, n in CALLS:
        print("case static", case, flush=True)
        a, ra = run(P, g, prm, n, static=True)
        b, rb = run(P, g, prm, n, static=False)
        N = g.ny - 1
        hdr, names, per = state_layout(g)
        nq = 6 if g.dim == 2 else 11
        assert a[0] == b[0] and a[1] == b[1] and abs(a[2] - b[2]) <= 1e-9 * abs(b[2])
        if prm.get("precision", 0) == 0:
            o = hdr
            for i, name in enumerate(names):
                x, y = a[o:o + 2 * per], b[o:o + 2 * per]
                sc = np.abs(y).max()
                err = np.abs(x - y).max() / sc if sc > 0 else np.abs(x).max()
                assert err <= (tol_prognostic(N) if i < nq else tol_history(N)), (case, name, err)
                o += 2 * per
        else:
            errs = fluct_errors(a, b, g)
            for name in names[:nq]:
                assert mixed_ok(errs[name]), (case, name, errs[name])
        for x, y in zip(ra, rb):
            assert x["step"] == y["step"] and x["blowup"] == y["blowup"] == 0
            assert abs(x["min_trc"] - y["min_trc"]) <= 2e-5 * abs(y["min_trc"]), (case, x["min_trc"], y["min_trc"])
            assert abs(x["energy"] - y["energy"]) <= 1e-9 * abs(y["energy"])
        # the records' counts: all Tr c values are far above 3 in these runs
        assert all(x["n_lt3"] == y["n_lt3"] == 0 for x, y in zip(ra, rb))


def test_static_init_limits(P):
    """A grid whose workspace exceeds the static array, and a second live
    handle on the same GPU, are refused; destroying the first frees it."""
    print("case static limits", flush=True)
    big = P.make_grid(3, 64, 65, 64)
    prm = P.make_params(wi=20.0, dt=1e-3)
    assert P.pcs_workspace_bytes(big, prm) > P.PCS_STATIC_BYTES
    with pytest.raises(P.PcsError) as e:
        P.Sim(big, prm, static=True)
    assert e.value.status == P.PCS_ERR_WORKSPACE
    g = P.make_grid(2, 16, 17)
    s1 = P.Sim(g, prm, seed=1, static=True)
    with pytest.raises(P.PcsError) as e:
        P.Sim(g, prm, seed=1, static=True)
    assert e.value.status == P.PCS_ERR_WORKSPACE
    s1.step(2)
    s1.close()
    s2 = P.Sim(g, prm, seed=1, static=True)
    s2.step(2)
    recs, st = s2.diagnostics()
    assert st == P.PCS_OK and len(recs) == 2
    s2.close()
