"""Precision 4: each wall-normal product table (the padded-grid values and
d/dy of the state; the projections of the explicit terms) takes the fastest
of FP32, FP64-operator and error-compensated FP32 arithmetic whose measured
error is within the budget (PCS_Y_ERROR_BUDGET).  Checked through the C ABI
(pcs_y_choice, pcs_ensemble_y_choice): the choice obeys its own measured
errors and times under a generous, a zero and the default budget; a choice
of all-FP32 or all-FP64 steps bit for bit as precision 1 or 2 does; the
compensated variant's measured error is of the order of FP32's (the
rounding inside each FP32 matrix instruction is beyond its reach);
the allocation-free initialisation chooses by error alone.  Parity with the
FP64 oracle at the default budget is part of the mixed-precision tests."""

import numpy as np
import pytest

from tests.test_gpu_parity import P  # noqa: F401

pytestmark = pytest.mark.gpu

FP32, FP64, COMP = 1, 2, 3


def run(P, dims, precision, monkeypatch, budget=None, steps=6, static=False):
    if budget is None:
        monkeypatch.delenv("PCS_Y_ERROR_BUDGET", raising=False)
    else:
        monkeypatch.setenv("PCS_Y_ERROR_BUDGET", repr(budget))
    print("case ychoice %s p%d budget %s static %s" % (dims, precision, budget, static), flush=True)
    sim = P.Sim(P.make_grid(*dims), P.make_params(wi=20.0, dt=1e-3, precision=precision), seed=3, amp=1e-3,
                static=static)
    ch = sim.y_choice()
    sim.step(steps)
    a = sim.get_state()
    recs, st = sim.diagnostics()
    sim.close()
    assert st == P.PCS_OK and len(recs) == steps
    return ch, a


def check_rule(ch, budget, timed=True):
    """The chosen variant of each table is within the budget and no slower
    than any other variant within it."""
    assert ch["budget"] == budget
    for t in range(2):
        errs, times = ch["error"][t], ch["time_us"][t]
        assert errs[FP64 - 1] == 0.0
        v = ch["variant"][t]
        assert errs[v - 1] is not None and errs[v - 1] <= budget, (t, ch)
        if not timed:
            assert all(x is None for x in times)
            continue
        for w in (FP32, FP64, COMP):
            assert errs[w - 1] is not None and times[w - 1] is not None and times[w - 1] > 0
            if errs[w - 1] <= budget:
                assert times[v - 1] <= times[w - 1], (t, w, ch)


DIMS = [(2, 64, 65, 1), (3, 32, 33, 16)]


@pytest.mark.parametrize("dims", DIMS, ids=["2D", "3D"])
def test_generous_budget_takes_fp32(P, dims, monkeypatch):
    ch, a = run(P, dims, 4, monkeypatch, budget=1e30)
    print(ch, flush=True)
    check_rule(ch, 1e30)
    for t in range(2):
        # FP32 is the fastest here (the compensated products take four FP32
        # passes); equal times keep the FP64 operators
        times = ch["time_us"][t]
        if all(times[FP32 - 1] < times[w - 1] for w in (FP64, COMP)):
            assert ch["variant"][t] == FP32
    if ch["variant"] == [FP32, FP32]:
        _, b = run(P, dims, 1, monkeypatch)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dims", DIMS, ids=["2D", "3D"])
def test_zero_budget_takes_exact_variants(P, dims, monkeypatch):
    ch, a = run(P, dims, 4, monkeypatch, budget=0.0)
    print(ch, flush=True)
    check_rule(ch, 0.0)
    assert ch["error"][0][FP32 - 1] > 0 and ch["error"][1][FP32 - 1] > 0
    assert FP32 not in ch["variant"]
    if ch["variant"] == [FP64, FP64]:
        _, b = run(P, dims, 2, monkeypatch)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dims", DIMS, ids=["2D", "3D"])
def test_default_budget_and_error_levels(P, dims, monkeypatch):
    ch, _ = run(P, dims, 4, monkeypatch)
    print(ch, flush=True)
    check_rule(ch, 1e-5)
    # FP32 errors of both tables are of the order of FP32 rounding times the
    # operators' conditioning; the compensated variant cannot recover the
    # rounding inside each FP32 matrix instruction (a chain of four fused
    # multiply-adds), so its error is of the same order, not far below
    for e in ch["error"]:
        assert 1e-9 < e[FP32 - 1] < 1e-2
        assert 0 < e[COMP - 1] <= 4 * e[FP32 - 1]


def test_static_init_chooses_by_error(P, monkeypatch):
    dims = DIMS[0]
    for budget in (1e30, 0.0):
        ch, a = run(P, dims, 4, monkeypatch, budget=budget, static=True)
        print(ch, flush=True)
        check_rule(ch, budget, timed=False)
        assert ch["error"][0][COMP - 1] is None
        want = FP32 if budget > 0 else FP64
        assert ch["variant"] == [want, want]
        _, b = run(P, dims, 1 if budget > 0 else 2, monkeypatch, static=True)
        assert np.array_equal(a, b)


def test_fixed_precisions_report_their_variants(P, monkeypatch):
    for precision, want in ((0, [0, 0]), (1, [FP32, FP32]), (2, [FP64, FP64]), (3, [COMP, COMP])):
        ch, _ = run(P, DIMS[0], precision, monkeypatch, steps=1)
        assert ch["variant"] == want and ch["budget"] is None
        assert all(x is None for row in ch["error"] + ch["time_us"] for x in row)


def test_ensemble_choice(P, monkeypatch):
    monkeypatch.setenv("PCS_Y_ERROR_BUDGET", "1e-5")
    print("case ychoice ensemble", flush=True)
    grids = [P.make_grid(2, 64, 65), P.make_grid(2, 128, 97)]
    params = [P.make_params(wi=20.0, dt=1e-3, precision=4) for _ in grids]
    ens = P.Ensemble(grids, params, [5, 6], amp=1e-3)
    ch = ens.y_choice()
    ens.step(4)
    for r in range(2):
        recs, st = ens.diagnostics(r)
        assert st == P.PCS_OK and len(recs) == 4
    ens.close()
    print(ch, flush=True)
    check_rule(ch, 1e-5)
