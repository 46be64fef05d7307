"""Ensembles of uneven-size runs (one graph launch per step, every stage one
kernel over all runs) against the FP64 oracle, run by run.

Each member is compared with its own oracle run from the same seeded
initial state, with the single-run tolerances (FP64) or the mixed-precision
bar; the per-step diagnostic records of every member are checked too, so a
member reading another member's data or sizes would fail here.
"""

import numpy as np
import pytest

from oracle import Grid, Oracle, Params
from paper_2606_09468_amd.workloads import ensemble_members
from tests.test_gpu_parity import check_diag, check_state, fluct_errors, mixed_ok, tol_history, tol_prognostic

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


def build(P, members, precision, dt=1e-3):
    grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
    params = [P.make_params(wi=wi, dt=dt, precision=precision) for _, _, wi, _ in members]
    return P.Ensemble(grids, params, [s for _, _, _, s in members], amp=1e-3)


SMALL = ensemble_members(count=6, seed=4, ny_choices=(17, 25, 33), nx_choices=(12, 16, 24, 32))


def test_fp64_ensemble_members_match_oracle(P):
    nsteps = 12
    print("case fp64 ensemble", SMALL, flush=True)
    ens = build(P, SMALL, 0)
    ens.step(nsteps)
    for r, (ny, nx, wi, seed) in enumerate(SMALL):
        g = Grid(2, nx, ny)
        o = Oracle(g, Params(wi=wi, dt=1e-3), seed=seed, amp=1e-3)
        o.step(nsteps)
        recs, st = ens.diagnostics(r)
        assert st == P.PCS_OK and len(recs) == nsteps
        name = "member %d %dx%d Wi%.1f" % (r, nx, ny, wi)
        check_state(ens.get_state(r), o.get_state(), g, tol_prognostic(ny - 1), tol_history(ny - 1), name)
        check_diag(recs, o, o.trace_c(), name)
        for rec, e in zip(recs, o.diag):
            assert rec["step"] == e["step"] and rec["n_lt3"] == e["n_lt3"] and rec["n_lt0"] == e["n_lt0"]
    ens.close()


def test_mixed_ensemble_members_match_oracle(P):
    """Mixed-precision members against the FP64 oracle with the single-run
    mixed bar (mixed_ok: fluctuation 2e-4 of its max, fields with a mean part
    2e-5 of theirs)."""
    nsteps = 20
    members = SMALL[:4]
    print("case mixed ensemble", members, flush=True)
    ens = build(P, members, 1)
    ens.step(nsteps)
    for r, (ny, nx, wi, seed) in enumerate(members):
        g = Grid(2, nx, ny)
        o = Oracle(g, Params(wi=wi, dt=1e-3), seed=seed, amp=1e-3)
        o.step(nsteps)
        errs = fluct_errors(ens.get_state(r), o.get_state(), g)
        print("member", r, {k: "%.1e/%.1e" % v for k, v in errs.items()}, flush=True)
        for name in ("u", "v", "phi", "cxx", "cxy", "cyy"):
            assert mixed_ok(errs[name]), (r, name, errs[name])
    ens.close()


def test_ensemble_equals_single_runs(P):
    """A member advances exactly as the same run on its own would, up to the
    summation order the tile tuner picks for the merged product tables."""
    nsteps = 8
    members = SMALL[:3]
    ens = build(P, members, 0)
    ens.step(nsteps)
    for r, (ny, nx, wi, seed) in enumerate(members):
        sim = P.Sim(P.make_grid(2, nx, ny), P.make_params(wi=wi, dt=1e-3), seed=seed, amp=1e-3)
        sim.step(nsteps)
        a, b = ens.get_state(r), sim.get_state()
        sim.close()
        scale = np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-12 * scale, (r, np.abs(a - b).max() / scale)
    ens.close()


def test_full_size_ensemble_sampled_members(P):
    """The 64-member uneven ensemble (mixed precision) for a few steps; the
    two smallest members are checked against the oracle, and every member's
    records must be finite with the step count advanced."""
    members = ensemble_members()
    nsteps = 5
    print("case full ensemble 64 members", flush=True)
    grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
    params = [P.make_params(wi=wi, dt=5e-4, precision=1) for _, _, wi, _ in members]
    ens = P.Ensemble(grids, params, [s for _, _, _, s in members], amp=1e-3)
    ens.step(nsteps)
    for r in range(len(members)):
        recs, st = ens.diagnostics(r)
        assert st == P.PCS_OK and len(recs) == nsteps and recs[-1]["step"] == nsteps
        assert np.isfinite(recs[-1]["min_trc"]) and recs[-1]["blowup"] == 0
    order = sorted(range(len(members)), key=lambda r: members[r][0] * members[r][1])[:2]
    for r in order:
        ny, nx, wi, seed = members[r]
        g = Grid(2, nx, ny)
        o = Oracle(g, Params(wi=wi, dt=5e-4), seed=seed, amp=1e-3)
        o.step(nsteps)
        errs = fluct_errors(ens.get_state(r), o.get_state(), g)
        print("member", r, nx, ny, {k: "%.1e/%.1e" % v for k, v in errs.items()}, flush=True)
        for name in ("u", "v", "phi", "cxx", "cxy", "cyy"):
            assert mixed_ok(errs[name]), (r, name, errs[name])
    ens.close()


def test_blown_up_member_is_masked_and_isolated(P, monkeypatch):
    """One member of an ensemble runs with an absurd time step (dt = 2,
    CFL far above 1) and blows up numerically within a few steps.  It must be
    flagged (PCS_BLOWUP, then PCS_ERR_STATE from its run status), masked (no
    record or step after the flagged one, its state left where it stopped
    while the others advance), and every other member must stay bitwise
    equal to the same ensemble without the bad time step.  A new state
    through pcs_ensemble_set_state unmasks it, and it then advances as the
    same run on its own does.  Tile shape and product form are forced so
    that both ensembles and the single run evaluate identical products."""
    monkeypatch.setenv("PCS_GEMM_CFG", "4")
    monkeypatch.setenv("PCS_PRODUCT_FORM", "parity")
    members = SMALL[:4]
    bad, nsteps = 1, 16

    def make(dt_bad):
        grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
        params = [P.make_params(wi=wi, dt=(dt_bad if r == bad else 1e-3)) for r, (_, _, wi, _) in enumerate(members)]
        return P.Ensemble(grids, params, [s for _, _, _, s in members], amp=1e-3)

    print("case ensemble blow-up masking", members, flush=True)
    ref = make(1e-3)
    ens = make(2.0)
    ref.step(nsteps)
    ens.step(nsteps)
    recs, st = ens.diagnostics(bad)
    assert st == P.PCS_BLOWUP and 1 <= len(recs) < nsteps
    assert recs[-1]["blowup"] == 1 and all(r["blowup"] == 0 for r in recs[:-1])
    assert recs[-1]["step"] == len(recs)
    assert ens.run_status(bad) == P.PCS_ERR_STATE
    for r in range(len(members)):
        if r == bad:
            continue
        assert ens.run_status(r) == P.PCS_OK
        assert np.array_equal(ens.get_state(r), ref.get_state(r)), r
        ra, sa = ens.diagnostics(r)
        rb, sb = ref.diagnostics(r)
        assert sa == sb == P.PCS_OK and ra == rb and len(ra) == nsteps
    # the masked run stays where it stopped
    frozen = ens.get_state(bad)
    ens.step(3)
    ref.step(3)
    assert np.array_equal(ens.get_state(bad), frozen, equal_nan=True)
    recs, st = ens.diagnostics(bad)
    assert recs == [] and st == P.PCS_BLOWUP
    for r in range(len(members)):
        if r != bad:
            assert np.array_equal(ens.get_state(r), ref.get_state(r)), r
    # recovery: a fresh state for the bad run (its own seeded initial state)
    ny, nx, wi, seed = members[bad]
    sim = P.Sim(P.make_grid(2, nx, ny), P.make_params(wi=wi, dt=2.0), seed=seed, amp=1e-3)
    fresh = sim.get_state()
    ens.set_state(bad, fresh)
    assert ens.run_status(bad) == P.PCS_OK
    ens.step(2)
    sim.step(2)
    recs, st = ens.diagnostics(bad)
    assert st == P.PCS_OK and [x["step"] for x in recs] == [1, 2] and recs[-1]["blowup"] == 0
    a, b = ens.get_state(bad), sim.get_state()
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    sim.close()
    ens.close()
    ref.close()


def test_single_run_stops_at_its_blowup_step(P):
    """A single run with dt = 2 stepped 16 steps in one call: the device
    stops it at the step whose record flags the blow-up (no later records,
    step count frozen), and the host then refuses further steps."""
    print("case single-run blow-up stop", flush=True)
    ny, nx, wi, seed = SMALL[1]
    sim = P.Sim(P.make_grid(2, nx, ny), P.make_params(wi=wi, dt=2.0), seed=seed, amp=1e-3)
    sim.step(16)
    recs, st = sim.diagnostics()
    assert st == P.PCS_BLOWUP and 1 <= len(recs) < 16 and recs[-1]["blowup"] == 1
    state = sim.get_state()
    assert state[0] == recs[-1]["step"]
    with pytest.raises(P.PcsError) as e:
        sim.step(1)
    assert e.value.status == P.PCS_ERR_STATE
    sim.close()


def test_full_ensemble_every_size_class_against_oracle(P):
    """The 64-member uneven ensemble (mixed precision, dt = 5e-4) over 5
    steps: the first member of each of its 19 (Ny, Nx) size classes against
    its own FP64 oracle run with the mixed bar, and every member's records
    finite and advanced.  The Nx = 512 members run the 768-point x
    transforms, the Ny = 97 and 193 members padded wall-normal grids of 145
    and 289 points."""
    members = ensemble_members()
    nsteps = 5
    print("case full ensemble, one member per size class", flush=True)
    grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
    params = [P.make_params(wi=wi, dt=5e-4, precision=1) for _, _, wi, _ in members]
    ens = P.Ensemble(grids, params, [s for _, _, _, s in members], amp=1e-3)
    ens.step(nsteps)
    firsts = {}
    for r, (ny, nx, _, _) in enumerate(members):
        firsts.setdefault((ny, nx), r)
        recs, st = ens.diagnostics(r)
        assert st == P.PCS_OK and len(recs) == nsteps and recs[-1]["blowup"] == 0
    assert len(firsts) == 19
    for (ny, nx), r in sorted(firsts.items()):
        _, _, wi, seed = members[r]
        g = Grid(2, nx, ny)
        o = Oracle(g, Params(wi=wi, dt=5e-4), seed=seed, amp=1e-3)
        o.step(nsteps)
        errs = fluct_errors(ens.get_state(r), o.get_state(), g)
        print("member %d %dx%d: worst fluctuation %.1e, full %.1e" % (
            r, nx, ny, max(v[0] for v in list(errs.values())[:6]), max(v[1] for v in list(errs.values())[:6])),
            flush=True)
        for name in ("u", "v", "phi", "cxx", "cxy", "cyy"):
            assert mixed_ok(errs[name]), (r, nx, ny, name, errs[name])
    ens.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_member_512x193_fifty_steps_against_oracle(P, precision):
    """Member 12 of the ensemble draw (Nx = 512, Ny = 193, Wi = 87.15, seed
    4012) over 50 steps, the full state against its oracle run: FP64 with
    the single-run tolerances (N = 192), mixed with the mixed bar."""
    members = ensemble_members()
    ny, nx, wi, seed = members[12]
    assert (ny, nx) == (193, 512)
    nsteps = 50
    print("case member 12 512x193 p%d x%d" % (precision, nsteps), flush=True)
    g = Grid(2, nx, ny)
    o = Oracle(g, Params(wi=wi, dt=5e-4), seed=seed, amp=1e-3)
    o.step(nsteps)
    sim = P.Sim(P.make_grid(2, nx, ny), P.make_params(wi=wi, dt=5e-4, precision=precision), seed=seed, amp=1e-3)
    sim.step(nsteps)
    recs, st = sim.diagnostics()
    a = sim.get_state()
    sim.close()
    assert st == P.PCS_OK and len(recs) == nsteps
    N = ny - 1
    if precision == 0:
        check_state(a, o.get_state(), g, tol_prognostic(N), tol_history(N), "member 12 FP64")
        check_diag(recs, o, o.trace_c(), "member 12 FP64")
    else:
        errs = fluct_errors(a, o.get_state(), g)
        for name in ("u", "v", "phi", "cxx", "cxy", "cyy"):
            assert mixed_ok(errs[name]), (name, errs[name])
