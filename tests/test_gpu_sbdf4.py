"""SBDF4 (the paper's 4th-order semi-implicit BDF, Section 2) through the C
ABI against the FP64 oracle: seeded runs long enough to wrap the history
rings and to use both the 8-step and the 1-step graphs, the sPTT relaxation
pin started from an exact history at a nonzero step index, resume / replay
determinism, the stage-timing path (kernels launched repeatedly), mixed
precision, and an ensemble that mixes both schemes."""

import numpy as np
import pytest

from oracle import Grid, Oracle, Params, state_layout
from tests.test_gpu_parity import P, FieldErr, mixed_ok, tol_history, tol_prognostic  # noqa: F401
from tests.test_oracle_sbdf4 import recursion

pytestmark = pytest.mark.gpu


def field_errors(a, b, g):
    hdr, names, per = state_layout(g, 1)
    assert a.size == b.size == hdr + len(names) * per * 2
    out, o = {}, hdr
    for n in names:
        x, y = a[o:o + 2 * per], b[o:o + 2 * per]
        sc = np.abs(y).max()
        out[n] = float(np.abs(x - y).max() / sc) if sc > 0 else float(np.abs(x).max())
        o += 2 * per
    return out


def check(a, b, g, case):
    errs = field_errors(a, b, g)
    nq = 6 if g.dim == 2 else 11
    q_names = set(state_layout(g, 0)[1][:nq])
    N = g.ny - 1
    print(case, "worst q %.1e, worst history %.1e" % (
        max(v for k, v in errs.items() if k.split("@")[0] in q_names),
        max(v for k, v in errs.items() if k.split("@")[0] not in q_names)), flush=True)
    assert a[0] == b[0] and abs(a[1] - b[1]) <= 1e-15 * max(1.0, abs(b[1]))
    assert abs(a[2] - b[2]) <= 1e-9 * abs(b[2]), (a[2], b[2])
    for k, v in errs.items():
        tol = tol_prognostic(N) if k.split("@")[0] in q_names else tol_history(N)
        assert v <= tol, (case, k, v, tol)


CASES = [
    ("2D 32x33 x10", Grid(2, 32, 33), dict(wi=20.0, dt=1e-3), 10),
    ("2D 64x65 eps x10", Grid(2, 64, 65), dict(wi=50.0, dt=5e-4, eps=1e-3), 10),
    ("3D 16x17x16 x10", Grid(3, 16, 17, 16), dict(wi=20.0, dt=1e-3), 10),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_sbdf4_matches_oracle(P, case):
    name, g, prm, n = case
    print("case sbdf4", name, flush=True)
    sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(scheme=1, **prm), seed=2, amp=1e-3)
    sim.step(n)
    a = sim.get_state()
    recs, st = sim.diagnostics()
    sim.close()
    o = Oracle(g, Params(scheme=1, **prm), seed=2, amp=1e-3)
    o.step(n)
    assert st == P.PCS_OK and len(recs) == n
    check(a, o.get_state(), g, name)
    d, e = recs[-1], o.diag[-1]
    for k in ("energy", "mean_trc", "dpdx"):
        assert abs(d[k] - e[k]) <= 1e-11 * max(1.0, abs(e[k])), (k, d[k], e[k])


def test_sbdf4_sptt_relaxation_pin(P):
    """Uniform c_xx = 1 + s with no flow, exact history at step index 5:
    ds/dt = -(s + eps s^2)/Wi follows the scalar SBDF4 recursion."""
    print("case sbdf4 sptt pin", flush=True)
    dt, nsteps, wi, eps, s0 = 0.025, 20, 1.0, 0.5, 1.0
    g = Grid(2, 8, 9)
    prm = dict(re=1.0, wi=wi, beta=0.5, kappa=0.0, eps=eps, dt=dt, forcing=1, q_or_dpdx=0.0)
    o = Oracle(g, Params(scheme=1, **prm), seed=None)

    def exact(t):
        ee = np.exp(-t / wi)
        return s0 * ee / (1.0 + eps * s0 * (1.0 - ee))

    def F(s):
        return -eps * s * s / wi

    s = [exact(-k * dt) for k in range(4)]
    for name in o.q:
        o.q[name][:] = 0
    for suf, k in (("", 0), ("@1", 1), ("@2", 2), ("@3", 3)):
        o.q["cxx" + suf][:, 0, 0] = 1.0 + s[k]
        o.q["cyy" + suf][:, 0, 0] = 1.0
    for suf, k in (("", 1), ("@2", 2), ("@3", 3)):
        o.q["Fxx" + suf][:, 0, 0] = F(s[k])
    o.step_count = 5
    start = o.get_state()
    sim = P.Sim(P.make_grid(2, 8, 9), P.make_params(scheme=1, **prm), seed=0, amp=0.0)
    sim.set_state(start)
    assert np.array_equal(sim.get_state(), start)
    sim.step(nsteps)
    a = sim.get_state()
    sim.close()
    o.step(nsteps)
    b = o.get_state()
    assert a[0] == b[0] == 5 + nsteps
    assert np.abs(a[4:] - b[4:]).max() <= 1e-13
    hdr, names, per = state_layout(g, 1)
    cxx = a[hdr + names.index("cxx") * 2 * per: hdr + (names.index("cxx") + 1) * 2 * per: 2 * (g.nx // 2)]
    rec = recursion(-1.0 / wi, s, F, dt, nsteps, [F(v) for v in s])
    assert np.abs(cxx - 1.0 - rec).max() <= 1e-13


def test_sbdf4_resume_and_stage_path(P):
    """n steps, save, restore into a fresh run (ring slots permuted by the
    step index), n more == 2n steps, bit for bit; the stage-timing path
    (every stage launched three times) advances the state like a step."""
    print("case sbdf4 resume / stage path", flush=True)
    g, p = P.make_grid(3, 16, 17, 16), P.make_params(wi=20.0, dt=1e-3, scheme=1)
    s1 = P.Sim(g, p, seed=5, amp=1e-3)
    s1.step(7)
    mid = s1.get_state()
    s1.step(6)
    end1 = s1.get_state()
    s2 = P.Sim(g, p, seed=9, amp=1e-3)
    s2.set_state(mid)
    s2.step(6)
    assert np.array_equal(end1, s2.get_state())
    s3 = P.Sim(g, p, seed=5, amp=1e-3)
    s4 = P.Sim(g, p, seed=5, amp=1e-3)
    s3.step(5)
    s4.stage_times(5, reps=3)
    assert np.array_equal(s3.get_state(), s4.get_state())
    for s in (s1, s2, s3, s4):
        s.close()


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
def test_sbdf4_mixed_precision(P, precision):
    """Mixed precision with SBDF4 against the FP64 oracle, to the bar of the
    CNAB2 mixed path (mixed_ok): prognostic fluctuation within 2e-4 of its
    own max, every prognostic field with a mean part within 2e-5 of its full
    max."""
    print("case sbdf4 mixed p%d" % precision, flush=True)
    g, prm, n = Grid(2, 64, 65), dict(wi=20.0, dt=1e-3), 40
    sim = P.Sim(P.make_grid(2, 64, 65), P.make_params(precision=precision, scheme=1, **prm), seed=1, amp=1e-3)
    sim.step(n)
    a = sim.get_state()
    sim.close()
    o = Oracle(g, Params(scheme=1, **prm), seed=1, amp=1e-3)
    o.step(n)
    b = o.get_state()
    hdr, names, per = state_layout(g, 1)
    for i, name in enumerate(names[:6]):
        x = a[hdr + i * 2 * per: hdr + (i + 1) * 2 * per].reshape(g.ny, -1, 2).copy()
        y = b[hdr + i * 2 * per: hdr + (i + 1) * 2 * per].reshape(g.ny, -1, 2).copy()
        full = np.abs(x - y).max() / np.abs(y).max()
        zero_mean = not np.any(y[:, 0, :])
        x[:, 0, :] = 0
        y[:, 0, :] = 0
        fl = np.abs(x - y).max() / np.abs(y).max()
        assert mixed_ok(FieldErr(fl, full, zero_mean)), (name, fl, full)


def test_ensemble_mixes_schemes(P):
    """An ensemble of a CNAB2 and an SBDF4 run advances each as on its own."""
    print("case sbdf4 ensemble", flush=True)
    grids = [P.make_grid(2, 32, 33), P.make_grid(2, 16, 33)]
    params = [P.make_params(wi=20.0, dt=1e-3, scheme=0), P.make_params(wi=30.0, dt=1e-3, scheme=1)]
    ens = P.Ensemble(grids, params, [3, 4], amp=1e-3)
    ens.step(10)
    for r in range(2):
        sim = P.Sim(grids[r], params[r], seed=3 + r, amp=1e-3)
        sim.step(10)
        a, b = ens.get_state(r), sim.get_state()
        sim.close()
        assert a.size == b.size
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), (r, np.abs(a - b).max() / np.abs(b).max())
    ens.close()


def test_sbdf4_takes_cnab2_state_with_constant_past(P):
    """An SBDF4 run given a CNAB2-layout state (here a CNAB2 run's, resampled
    to another grid) restarts from a constant past: the same as the full
    SBDF4 state with q^{n-k} := q^n, X^{n-k} := X^{n-1}, and as the oracle."""
    print("case sbdf4 short state", flush=True)
    a, b = (2, 16, 17, 1), (2, 32, 33, 1)
    prm = dict(wi=20.0, dt=1e-3)
    s0 = P.Sim(P.make_grid(*a), P.make_params(**prm), seed=3, amp=1e-3)
    s0.step(5)
    short = P.resample_state(P.make_grid(*a), s0.get_state(), P.make_grid(*b))
    s0.close()
    gb = Grid(*b)
    hdr, names, per = state_layout(gb, 0)
    nq = 6
    base = short[hdr:]
    full = np.concatenate([short, base[:nq * 2 * per], base[:nq * 2 * per], base[:nq * 2 * per],
                           base[nq * 2 * per:], base[nq * 2 * per:]])
    s1 = P.Sim(P.make_grid(*b), P.make_params(scheme=1, **prm), seed=0, amp=0.0)
    s2 = P.Sim(P.make_grid(*b), P.make_params(scheme=1, **prm), seed=0, amp=0.0)
    s1.set_state(short)
    s2.set_state(full)
    assert np.array_equal(s1.get_state(), full)
    s1.step(4)
    s2.step(4)
    x = s1.get_state()
    assert np.array_equal(x, s2.get_state())
    s1.close()
    s2.close()
    o = Oracle(gb, Params(scheme=1, **prm), seed=None)
    o.set_state(full)
    o.step(4)
    check(x, o.get_state(), gb, "sbdf4 short state")
    with pytest.raises(P.PcsError):
        s3 = P.Sim(P.make_grid(*b), P.make_params(scheme=1, **prm), seed=0, amp=0.0)
        try:
            s3.set_state(short[:-2])
        finally:
            s3.close()


@pytest.mark.parametrize("dims,precision", [((2, 24, 25, 1), 0), ((3, 16, 17, 16), 0), ((3, 16, 17, 16), 1)])
def test_sbdf4_branched_graphs_match_single_chain(P, dims, precision, monkeypatch):
    """SBDF4 indexes its history rings with the device step counter that the
    step record advances; in the branched graphs that record runs on a side
    branch beside the next step.  States and records over 20 steps (two
    8-step graphs, four 1-step ones) must be bitwise those of the single
    chain, with the product tiles forced so the tables agree."""
    monkeypatch.setenv("PCS_GEMM_CFG", "4")
    monkeypatch.setenv("PCS_PRODUCT_FORM", "parity")
    out = []
    for br in ("0", "1", "2"):
        monkeypatch.setenv("PCS_GRAPH_BRANCHES", br)
        print("case sbdf4 branches=%s %s p%d" % (br, dims, precision), flush=True)
        sim = P.Sim(P.make_grid(*dims), P.make_params(wi=20.0, dt=1e-3, precision=precision, scheme=1),
                    seed=4, amp=1e-3)
        sim.step(20)
        recs, st = sim.diagnostics()
        assert st == P.PCS_OK and len(recs) == 20
        out.append((sim.get_state(), recs))
        sim.close()
    a, ra = out[0]
    for b, rb in out[1:]:
        assert np.array_equal(a, b)
        for x, y in zip(ra, rb):
            assert x == y, (x, y)
