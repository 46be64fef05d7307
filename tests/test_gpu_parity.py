"""Parity of the HIP step (through the C ABI) with the FP64 oracle.

Every case starts both sides from the same state (the seeded initial
condition built independently on each side, or a random state passed in
through pcs_set_state) and compares the full flat state element by element,
per field, relative to the field's max norm (the oracle's).  Tolerances are
written per case and derived (in the helpers below) from the conditioning
of the wall-normal operators (|D| ~ N^2, |D2| ~ N^4).
Diagnostic counts must lie within the bounds set by the oracle points
within the parity band of a threshold (3 or 0), and agree exactly where no
oracle point lies in that band; dedicated runs whose Tr c crosses 3 and 0 at
many points, away from ties, require exact equality at every step.
"""

import numpy as np
import pytest

from oracle import Grid, Oracle, Params, state_layout
from tests.inputs import random_state

pytestmark = pytest.mark.gpu

TIE_BAND = 1e-9


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


def field_errors(a, b, g):
    hdr, names, per = state_layout(g)
    out, o = {}, hdr
    for n in names:
        x, y = a[o:o + 2 * per], b[o:o + 2 * per]
        sc = np.abs(y).max()
        out[n] = float(np.abs(x - y).max() / sc) if sc > 0 else float(np.abs(x).max())
        o += 2 * per
    return out


def check_state(a, b, g, tol_q, tol_h, case):
    errs = field_errors(a, b, g)
    _, names, _ = state_layout(g)
    nq = 6 if g.dim == 2 else 11
    print(case, " ".join("%s=%.1e" % kv for kv in errs.items()), flush=True)
    assert a[0] == b[0] and abs(a[1] - b[1]) <= 1e-15 * max(1.0, abs(b[1]))
    assert abs(a[2] - b[2]) <= 1e-9 * abs(b[2]), (a[2], b[2])
    for i, n in enumerate(names):
        assert errs[n] <= (tol_q if i < nq else tol_h), (case, n, errs[n])
    return errs


def trc_tol(oracle_trc, N):
    """Pointwise Tr c carries the field error of c, which is relative to the
    field's max norm: tol_prognostic(N) times max |Tr c|."""
    return tol_prognostic(N) * np.abs(oracle_trc).max()


def count_bounds(oracle_trc, N):
    """Bounds on each Tr c count that any evaluation within the parity band
    of the oracle's values can give: lo counts the oracle points below the
    threshold by more than the band, hi those below it plus the band.  Where
    no oracle point lies within the band of a threshold, lo = hi and the
    count is fixed exactly."""
    band = max(TIE_BAND * max(1.0, np.abs(oracle_trc).max()), trc_tol(oracle_trc, N))
    mid = oracle_trc[N // 2]
    out = {}
    for k, vals, thr in (("n_lt3", oracle_trc, 3.0), ("n_lt0", oracle_trc, 0.0),
                         ("mid_n_lt3", mid, 3.0), ("mid_n_lt0", mid, 0.0)):
        out[k] = (int(np.sum(vals < thr - band)), int(np.sum(vals < thr + band)))
    return out


def check_counts(rec, orec, oracle_trc, N, case, exact=False):
    """Every count within the bounds of count_bounds (equal to the oracle's
    where the bounds meet); exact=True requires that they meet."""
    for k, (lo, hi) in count_bounds(oracle_trc, N).items():
        assert lo <= orec[k] <= hi, (case, k, lo, orec[k], hi)
        assert lo <= rec[k] <= hi, (case, k, lo, rec[k], hi)
        if exact:
            assert lo == hi and rec[k] == orec[k], (case, k, lo, hi, rec[k], orec[k])


def check_diag(recs, orc, oracle_trc, case):
    d, e = recs[-1], orc.diag[-1]
    assert d["step"] == e["step"] and d["blowup"] == e["blowup"] == 0
    tmin = trc_tol(oracle_trc, orc.g.ny - 1)
    for k in ("min_trc", "mid_min_trc"):
        assert abs(d[k] - e[k]) <= tmin, (case, k, d[k], e[k], tmin)
    for k in ("energy", "mean_trc", "dpdx", "cfl"):
        assert abs(d[k] - e[k]) <= 1e-11 * max(1.0, abs(e[k])), (case, k, d[k], e[k])
    check_counts(d, e, oracle_trc, orc.g.ny - 1, case)


def run_pair(P, g, prm, seed, amp, nsteps, case, state=None):
    print("case", case, flush=True)
    sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(**prm), seed=seed, amp=amp)
    o = Oracle(g, Params(**prm), seed=None if state is not None else seed, amp=amp)
    if state is not None:
        sim.set_state(state)
        o.set_state(state)
    sim.step(nsteps)
    o.step(nsteps)
    recs, st = sim.diagnostics()
    assert st == P.PCS_OK and len(recs) == nsteps
    a = sim.get_state()
    sim.close()
    return a, o, recs


def tol_prognostic(N):
    """Prognostic fields (u, v, w, phi, g, c): 1e-12 relative up to N = 128
    (the FP64 target); at N = 256 the floor of two correct FP64 evaluations
    of the same discrete step is a few 1e-12 (each wall-normal derivative
    amplifies roundoff by up to |D| ~ N^2), so 1e-11 there."""
    return 1e-12 if N <= 128 else 1e-11


def tol_history(N):
    """History fields h_v, h_g, F hold explicit terms with up to two
    wall-normal derivatives of the state (h_v = -D(i kx H_x + ...) with
    H containing D c): roundoff ~ eps |D|^2 ~ eps N^4."""
    return 1e-16 * N ** 4


CASES = [
    # name, grid, params, steps
    ("C1 2D 64x65 Wi20 dt1e-3 x200", Grid(2, 64, 65), dict(wi=20.0, dt=1e-3), 200),
    ("2D ragged 24x25 Wi20 x40", Grid(2, 24, 25), dict(wi=20.0, dt=1e-3), 40),
    ("2D 128x129 Wi50 kappa0 x30", Grid(2, 128, 129), dict(wi=50.0, dt=5e-4, kappa=0.0), 30),
    ("C2 2D 256x257 Wi50 dt5e-4 x20", Grid(2, 256, 257), dict(wi=50.0, dt=5e-4), 20),
    ("3D 16x17x16 x20", Grid(3, 16, 17, 16), dict(wi=20.0, dt=1e-3), 20),
    ("3D ragged 24x33x12 Wi50 x10", Grid(3, 24, 33, 12), dict(wi=50.0, dt=5e-4), 10),
    ("3D 32x65x32 Wi50 x8", Grid(3, 32, 65, 32), dict(wi=50.0, dt=5e-4), 8),
    # 32 kx columns of length 144 exceed one register pass: z columns in two batches
    ("3D wide-z 64x17x96 x3", Grid(3, 64, 17, 96), dict(wi=50.0, dt=5e-4), 3),
    # padded z columns of the compiled lengths 96 and 192 (the band-folded
    # outer passes) at a small x-y size
    ("3D z columns of 96 16x17x64 x4", Grid(3, 16, 17, 64), dict(wi=20.0, dt=1e-3), 4),
    ("3D z columns of 192 8x17x128 x3", Grid(3, 8, 17, 128), dict(wi=20.0, dt=1e-3), 3),
]


@pytest.mark.parametrize("form", ["plain", "parity"])
def test_both_product_forms_match_oracle(P, form, monkeypatch):
    """The autotuner picks, per product table, the plain or the parity
    (even/odd folded) form; either must reproduce the oracle.  The form is
    forced through PCS_PRODUCT_FORM, read when a simulation is set up.  Odd
    and even padded sizes (N = 24: M + 1 = 37; N = 10: M + 1 = 16) and 3D."""
    monkeypatch.setenv("PCS_PRODUCT_FORM", form)
    for name, g, prm, n in (("2D 24x25", Grid(2, 24, 25), dict(wi=20.0, dt=1e-3), 10),
                            ("2D 16x11", Grid(2, 16, 11), dict(wi=20.0, dt=1e-3), 10),
                            ("3D 16x17x16", Grid(3, 16, 17, 16), dict(wi=20.0, dt=1e-3), 5)):
        case = "%s %s" % (form, name)
        a, o, recs = run_pair(P, g, prm, seed=1, amp=1e-3, nsteps=n, case=case)
        N = g.ny - 1
        check_state(a, o.get_state(), g, tol_prognostic(N), tol_history(N), case)
        check_diag(recs, o, o.trace_c(), case)


_ORACLE_CACHE = {}


def _oracle_run(name, g, prm, n):
    if name not in _ORACLE_CACHE:
        o = Oracle(g, Params(**prm), seed=1, amp=1e-3)
        o.step(n)
        _ORACLE_CACHE[name] = o
    return _ORACLE_CACHE[name]


# tile configurations of the product kernels: 0-3 register-direct (plain
# form only), 4-13 LDS-tiled (plain and parity forms), 14-17 B-stationary
# (parity form only)
GEMM_CFGS = list(range(18))


@pytest.mark.parametrize("cfg", GEMM_CFGS)
def test_every_tile_configuration_matches_oracle(P, cfg, monkeypatch):
    """The autotuner may pick any tile configuration for any table, so each
    one, forced through PCS_GEMM_CFG in both product forms, must reproduce
    the oracle: FP64 2D with odd padded sizes (N = 24: M + 1 = 37) and 3D,
    and a mixed-precision 2D run (FP32 tables mixing FP64 products)."""
    monkeypatch.setenv("PCS_GEMM_CFG", str(cfg))
    forms = ["parity"] if cfg >= 14 else (["plain", "parity"] if cfg >= 4 else ["plain"])
    cases = (("2D 24x25", Grid(2, 24, 25), dict(wi=20.0, dt=1e-3), 10),
             ("3D 16x17x16", Grid(3, 16, 17, 16), dict(wi=20.0, dt=1e-3), 5))
    for form in forms:
        monkeypatch.setenv("PCS_PRODUCT_FORM", form)
        for name, g, prm, n in cases:
            case = "cfg %d %s %s" % (cfg, form, name)
            print("case", case, flush=True)
            sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(**prm), seed=1, amp=1e-3)
            sim.step(n)
            recs, st = sim.diagnostics()
            assert st == P.PCS_OK and len(recs) == n
            a = sim.get_state()
            sim.close()
            o = _oracle_run(name, g, prm, n)
            N = g.ny - 1
            check_state(a, o.get_state(), g, tol_prognostic(N), tol_history(N), case)
            check_diag(recs, o, o.trace_c(), case)
        # mixed precision: the fluctuation bar of the mixed-precision test
        name, g, prm, n = "2D 32x33 mixed", Grid(2, 32, 33), dict(wi=20.0, dt=1e-3), 10
        case = "cfg %d %s %s" % (cfg, form, name)
        print("case", case, flush=True)
        sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(precision=1, **prm),
                    seed=1, amp=1e-3)
        sim.step(n)
        a = sim.get_state()
        sim.close()
        o = _oracle_run(name, g, prm, n)
        errs = fluct_errors(a, o.get_state(), g)
        _, names, _ = state_layout(g)
        for k in names[:6]:
            assert mixed_ok(errs[k]), (case, k, errs[k])


@pytest.mark.parametrize("dims,precision", [((2, 24, 25, 1), 0), ((2, 32, 33, 1), 1), ((3, 16, 17, 16), 1)])
def test_branched_graphs_match_single_chain(P, dims, precision, monkeypatch):
    """The captured steps may run the mean and D2 / D products and the
    previous step's diagnostics on side branches, or the diagnostics only
    (chosen by step size; forced here through PCS_GRAPH_BRANCHES = 1, 2
    against 0): the same launches on the same data,
    so states and every diagnostics record must be bitwise those of the
    single-chain graphs.  20 steps: two 8-step graphs and four 1-step ones.
    The tile configuration and product form are forced, since the branched
    graphs split the state-product table and the autotuner could otherwise
    pick another shape (another summation order) for the parts."""
    monkeypatch.setenv("PCS_GEMM_CFG", "4")
    monkeypatch.setenv("PCS_PRODUCT_FORM", "parity")
    out = []
    for br in ("0", "1", "2"):
        monkeypatch.setenv("PCS_GRAPH_BRANCHES", br)
        print("case branches=%s %s p%d" % (br, dims, precision), flush=True)
        sim = P.Sim(P.make_grid(*dims), P.make_params(wi=20.0, dt=1e-3, precision=precision), seed=4, amp=1e-3)
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


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_seeded_run_matches_oracle(P, case):
    name, g, prm, n = case
    a, o, recs = run_pair(P, g, prm, seed=1, amp=1e-3, nsteps=n, case=name)
    N = g.ny - 1
    check_state(a, o.get_state(), g, tol_prognostic(N), tol_history(N), name)
    check_diag(recs, o, o.trace_c(), name)
    # every per-step record, not only the last
    tmin = trc_tol(o.trace_c(), N)
    for r, e in zip(recs, o.diag):
        assert r["step"] == e["step"] and abs(r["min_trc"] - e["min_trc"]) <= tmin, (r["step"], r["min_trc"], e["min_trc"])


@pytest.mark.parametrize("dim,nx,ny,nz", [(2, 32, 33, 1), (3, 16, 33, 16)])
def test_random_state_one_step(P, dim, nx, ny, nz):
    """A random smooth state (all fields, including history) through one
    step: exercises every term of the explicit products and solves."""
    g = Grid(dim, nx, ny, nz)
    st = random_state(dim, nx, ny, nz, seed=7, amp=0.05)
    o0 = Oracle(g, Params(wi=20.0, dt=1e-3), seed=3, amp=0.0)
    base = o0.get_state()
    st[4:] += base[4:]          # random fields on top of the laminar state and its history
    st[0:4] = [5, 0.005, 200.0, 0.0]
    a, o, _ = run_pair(P, g, dict(wi=20.0, dt=1e-3), seed=3, amp=0.0, nsteps=1, case="random %dD" % dim, state=st)
    check_state(a, o.get_state(), g, tol_prognostic(ny - 1), tol_history(ny - 1), "random %dD" % dim)


@pytest.mark.parametrize("kappa", [0.0, 5e-5])
def test_laminar_state_is_steady_on_gpu(P, kappa):
    """The laminar Oldroyd-B Poiseuille state (kappa = 0: c_xy = Wi U',
    c_xx = 1 + 2 (Wi U')^2, c_yy = 1) stays fixed under the GPU step."""
    print("case laminar kappa=%g" % kappa, flush=True)
    g = P.make_grid(2, 32, 65)
    sim = P.Sim(g, P.make_params(wi=20.0, dt=1e-3, kappa=kappa), seed=0, amp=0.0)
    s0 = sim.get_state()
    y = np.cos(np.pi * np.arange(65) / 64)
    per = 65 * 16 * 2
    U = s0[4:4 + per].reshape(65, 16, 2)[:, 0, 0]
    assert np.abs(U - (1 - y * y)).max() < 1e-15
    if kappa == 0.0:
        cxx = s0[4 + 3 * per:4 + 4 * per].reshape(65, 16, 2)[:, 0, 0]
        assert np.abs(cxx - (1 + 2 * (20.0 * 2 * y) ** 2)).max() <= 1e-15 * 3201
    sim.step(50)
    s1 = sim.get_state()
    recs, _ = sim.diagnostics()
    sim.close()
    # roundoff only: each step applies Ny-term wall-normal sums, so the drift
    # is bounded by steps * Ny * eps relative to the largest field value
    assert np.abs(s1[4:] - s0[4:]).max() / np.abs(s0[4:]).max() < 50 * 65 * 2.3e-16
    assert abs(recs[-1]["dpdx"] - 200.0) < 1e-8


def test_exact_relaxation_counts(P):
    """3D laminar flow with c_zz = 1 + delta: delta_n = delta ((1-a)/(1+a))^n
    exactly (a = dt/(2 Wi)), and the Tr c < 3 count is
    Nx Nz #{j: 8 Wi^2 y_j^2 < -delta_n}: the count kernel against a closed form."""
    print("case exact relaxation counts", flush=True)
    wi, dt, delta = 2.0, 2e-3, -0.37
    g = Grid(3, 8, 33, 8)
    o = Oracle(g, Params(wi=wi, kappa=0.0, dt=dt), seed=1, amp=0.0)
    o.q["czz"][:, 0, 0] += delta
    o.init_history()
    sim = P.Sim(P.make_grid(3, 8, 33, 8), P.make_params(wi=wi, kappa=0.0, dt=dt), seed=1, amp=0.0)
    sim.set_state(o.get_state())
    sim.step(15)
    recs, _ = sim.diagnostics()
    s = sim.get_state()
    sim.close()
    a = dt / (2 * wi)
    y = np.cos(np.pi * np.arange(33) / 32)
    for n, r in enumerate(recs, start=1):
        dn = delta * ((1 - a) / (1 + a)) ** n
        assert r["n_lt3"] == 64 * int(np.sum(8 * wi * wi * y * y < -dn))
        assert r["mid_n_lt3"] == 64 and r["n_lt0"] == 0
        assert abs(r["min_trc"] - (3 + dn)) < 1e-13
    per = 33 * 8 * 4 * 2
    czz = s[4 + 10 * per:4 + 11 * per].reshape(33, 8, 4, 2)[:, 0, 0, 0]
    assert np.abs(czz - (1 + delta * ((1 - a) / (1 + a)) ** 15)).max() < 1e-14


@pytest.mark.parametrize("dims", [(2, 32, 33, 1), (3, 16, 33, 16)])
def test_counts_exact_where_trc_crosses_thresholds(P, dims):
    """FP64 runs whose Tr c crosses 3 and 0 at many base-grid points away
    from ties: a planted c_xx wave of amplitude 5 in the first x mode (and a
    z mode in 3D) on top of the kappa = 0 laminar state with c_yy lowered by
    0.3, so that near the midplane Tr c = 2.7 + 8 Wi^2 y^2 + the wave spans
    values below 0, between 0 and 3 and above 3.  All four counts must equal
    the oracle's exactly at every step (and lie outside any tie band)."""
    g = Grid(*dims)
    prm = dict(wi=5.0, dt=1e-3, kappa=0.0)
    nsteps = 10
    o = Oracle(g, Params(**prm), seed=1, amp=1e-3)
    y = o.op.y
    o.q["cxx"][:, 0, 1] += 2.5 * (1.0 - 0.3 * y * y)
    if g.dim == 3:
        o.q["cxx"][:, 1, 0] += 0.8 * (1.0 - 0.3 * y * y)
        o.q["cxx"][:, g.nz - 1, 0] += 0.8 * (1.0 - 0.3 * y * y)
    o.q["cyy"][:, 0, 0] -= 0.3
    o.init_history()
    st = o.get_state()
    case = "straddling counts %dD" % g.dim
    print("case", case, flush=True)
    sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(**prm), seed=1, amp=1e-3)
    sim.set_state(st)
    traces = []
    for _ in range(nsteps):
        o.step(1)
        traces.append(o.trace_c())
    sim.step(nsteps)
    recs, stt = sim.diagnostics()
    a = sim.get_state()
    sim.close()
    assert stt == P.PCS_OK and len(recs) == nsteps
    N = g.ny - 1
    for r, e, tr in zip(recs, o.diag, traces):
        assert 0 < e["n_lt0"] < e["n_lt3"] < tr.size and 0 < e["mid_n_lt0"] < e["mid_n_lt3"] < tr[N // 2].size
        check_counts(r, e, tr, N, "%s step %d" % (case, r["step"]), exact=True)
    check_state(a, o.get_state(), g, tol_prognostic(N), tol_history(N), case)


def test_blowup_flag_and_recovery(P):
    """A planted NaN is flagged, the run refuses further steps, and a new
    state clears the flag (the error path forced from the host)."""
    print("case blow-up flag", flush=True)
    sim = P.Sim(P.make_grid(2, 16, 17), P.make_params(), seed=1, amp=1e-3)
    good = sim.get_state()
    bad = good.copy()
    bad[4 + 3 * 17 * 8 * 2 + 5] = np.nan       # one c_xx coefficient
    sim.set_state(bad)
    sim.step(1)
    recs, st = sim.diagnostics()
    assert st == P.PCS_BLOWUP and recs[-1]["blowup"] == 1
    with pytest.raises(P.PcsError) as ei:
        sim.step(1)
    assert ei.value.status == P.PCS_ERR_STATE
    sim.set_state(good)
    sim.step(2)
    recs, st = sim.diagnostics()
    assert st == P.PCS_OK and recs[-1]["blowup"] == 0


def test_set_state_rejects_bad_step_index(P):
    """The header's step index picks device ring slots: a negative,
    fractional or huge value is refused and the run is left as it was."""
    print("case set_state step index", flush=True)
    sim = P.Sim(P.make_grid(2, 16, 17), P.make_params(), seed=1, amp=1e-3)
    sim.step(3)
    good = sim.get_state()
    for bad_step in (-1.0, -4096.0, 2.5, 2.0 ** 60, np.inf, np.nan):
        bad = good.copy()
        bad[0] = bad_step
        with pytest.raises(P.PcsError) as ei:
            sim.set_state(bad)
        assert ei.value.status == P.PCS_ERR_ARG
    assert np.array_equal(sim.get_state(), good)
    sim.step(1)
    recs, st = sim.diagnostics()
    assert st == P.PCS_OK and recs[-1]["step"] == 4
    sim.close()
    sim.close()


def test_resume_and_replay_bitwise(P):
    """n steps, save, restore, n steps == 2n steps, bit for bit; two runs of
    the same graph from the same state are bitwise equal."""
    print("case resume / replay determinism", flush=True)
    g, p = P.make_grid(3, 16, 17, 16), P.make_params(wi=20.0, dt=1e-3)
    s1 = P.Sim(g, p, seed=5, amp=1e-3)
    s1.step(6)
    mid = s1.get_state()
    s1.step(6)
    end1 = s1.get_state()
    s2 = P.Sim(g, p, seed=9, amp=1e-3)
    s2.set_state(mid)
    s2.step(6)
    end2 = s2.get_state()
    s1.close()
    s2.close()
    assert np.array_equal(end1, end2)


@pytest.mark.parametrize("dims", [(2, 32, 33, 1), (3, 16, 17, 16)])
def test_stage_times_advance_state_like_step(P, dims):
    print("case stage timing path", dims, flush=True)
    g, p = P.make_grid(*dims), P.make_params(wi=20.0, dt=1e-3)
    s1 = P.Sim(g, p, seed=2, amp=1e-3)
    s2 = P.Sim(g, p, seed=2, amp=1e-3)
    s1.step(3)
    # every stage but the step record is launched three times back to back:
    # they recompute the same outputs, so the state must still match
    t = s2.stage_times(3, reps=3)
    assert set(t) >= {"xpencil", "gemm_state", "finalize"} and all(v >= 0 for v in t.values())
    # stages with no launch report 0: the z transforms in 2D, and the separate
    # mean and D2 / D product launches of small steps (one product launch)
    for k in ("xpencil", "gemm_state", "gemm_proj", "rhs", "gemm_vinv", "gemm_v", "finalize", "diag_rows",
              "diag_final"):
        assert t[k] > 0, (k, t)
    for k in ("gemm_mean", "gemm_d2") + (("zfft_inv", "zfft_fwd", "diag_zfft") if dims[0] == 2 else ()):
        assert t[k] == 0, (k, t)
    if dims[0] == 3:
        assert t["zfft_inv"] > 0 and t["zfft_fwd"] > 0 and t["diag_zfft"] > 0
    assert np.array_equal(s1.get_state(), s2.get_state())
    s1.close()
    s2.close()


def test_ensemble_stage_times(P):
    """pcs_ensemble_stage_times: every stage of a small 2D ensemble timed,
    the state advanced as by pcs_ensemble_step."""
    print("case ensemble stage timing", flush=True)
    grids = [P.make_grid(2, 32, 33), P.make_grid(2, 64, 65)]
    params = [P.make_params(wi=20.0, dt=1e-3) for _ in grids]
    e1 = P.Ensemble(grids, params, [1, 2], amp=1e-3)
    e2 = P.Ensemble(grids, params, [1, 2], amp=1e-3)
    e1.step(3)
    t = e2.stage_times(3, reps=2)
    assert t["gemm_state"] > 0 and t["xpencil"] > 0 and t["zfft_inv"] == 0
    for r in range(2):
        assert np.array_equal(e1.get_state(r), e2.get_state(r))
    e1.close()
    e2.close()


def test_stage_times_bin_each_step_once(P):
    """The row diagnostics also fill the midplane histograms, so the timing
    path runs them once per step: after stage_times(4 steps, reps=5) every
    histogram holds exactly 4 Nx Nz samples, as after 4 ordinary steps."""
    print("case stage timing histograms", flush=True)
    g, p = P.make_grid(3, 16, 17, 8), P.make_params(wi=20.0, dt=1e-3)
    s1 = P.Sim(g, p, seed=2, amp=1e-3)
    s2 = P.Sim(g, p, seed=2, amp=1e-3)
    for s in (s1, s2):
        for q in (P.PCS_PDF_TRC, P.PCS_PDF_U, P.PCS_PDF_V, P.PCS_PDF_W):
            s.midplane_pdf_setup(q, -1.0, 1.0, 16)
    s1.step(4)
    s2.stage_times(4, reps=5)
    for q in (P.PCS_PDF_TRC, P.PCS_PDF_U, P.PCS_PDF_V, P.PCS_PDF_W):
        a, b = s1.midplane_pdf(q), s2.midplane_pdf(q)
        assert int(b.sum()) == 4 * 16 * 8, (q, int(b.sum()))
        assert np.array_equal(a, b), q
    s1.close()
    s2.close()


class FieldErr(tuple):
    """(error relative to the fluctuation's max, error relative to the field's
    max) of one field; zero_mean: the oracle's kx = kz = 0 column is
    identically zero."""

    def __new__(cls, fl, full, zero_mean):
        t = super().__new__(cls, (fl, full))
        t.zero_mean = zero_mean
        return t


# the mixed-precision bar
MIXED_FLUCT, MIXED_FIELD = 2e-4, 2e-5


def mixed_ok(e):
    """The fluctuation (all modes except kx = kz = 0) within MIXED_FLUCT of its
    max norm, and the field within MIXED_FIELD of its max norm.  A field with
    no mean part (its kx = kz = 0 column identically zero: v and phi, whose
    mean vanishes by continuity with impermeable walls, and omega_y in 3D) is
    its own fluctuation, so the fluctuation bar is its only bar."""
    return e[0] <= MIXED_FLUCT and (e.zero_mean or e[1] <= MIXED_FIELD)


def fluct_errors(a, b, g):
    """Per field: error relative to the max of the oracle's fluctuation (all
    modes except kx = kz = 0), and relative to the full field's max."""
    hdr, names, per = state_layout(g)
    out, o = {}, hdr
    for n in names:
        x = a[o:o + 2 * per].reshape(g.ny, -1, 2).copy()
        y = b[o:o + 2 * per].reshape(g.ny, -1, 2).copy()
        full = np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)
        zero_mean = not np.any(y[:, 0, :])
        x[:, 0, :] = 0
        y[:, 0, :] = 0
        fl = np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)
        out[n] = FieldErr(float(fl), float(full), zero_mean)
        o += 2 * per
    return out


MIXED_CASES = [
    ("C1 2D 64x65 x100", Grid(2, 64, 65), dict(wi=20.0, dt=1e-3), 100),
    ("C2 2D 256x257 x50", Grid(2, 256, 257), dict(wi=50.0, dt=5e-4), 50),
    ("3D 32x33x32 x20", Grid(3, 32, 33, 32), dict(wi=50.0, dt=5e-4), 20),
    # FP32 z columns: 32 of length 288 exceed one register pass (two batches)
    ("3D wide-z 64x17x192 x3", Grid(3, 64, 17, 192), dict(wi=50.0, dt=5e-4), 3),
    # padded z columns of 96 (compiled, band-folded) in FP32
    ("3D z columns of 96 16x17x64 x4", Grid(3, 16, 17, 64), dict(wi=20.0, dt=1e-3), 4),
]


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("case", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_precision_against_fp64_oracle(P, case, precision):
    """Mixed path (FP32 transforms and products of the fluctuation, FP64 mean
    mode, solves and diagnostics) against the FP64 oracle.  Stated bar: the
    prognostic fluctuation within 2e-4 of its own max norm and every prognostic
    field with a mean part within 2e-5 of its full max norm (mixed_ok) over the
    case's steps (measured:
    up to 5e-5 and 1e-5 after 100 C2 steps); diagnostics to 1e-8 relative."""
    name, g, prm, n = case
    print("case mixed p%d %s" % (precision, name), flush=True)
    sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(precision=precision, **prm),
                seed=1, amp=1e-3)
    sim.step(n)
    a = sim.get_state()
    recs, st = sim.diagnostics()
    sim.close()
    o = Oracle(g, Params(**prm), seed=1, amp=1e-3)
    o.step(n)
    errs = fluct_errors(a, o.get_state(), g)
    nq = 6 if g.dim == 2 else 11
    _, names, _ = state_layout(g)
    print(name, " ".join("%s=%.1e/%.1e" % (k, v[0], v[1]) for k, v in errs.items() if k in names[:nq]), flush=True)
    for k in names[:nq]:
        assert mixed_ok(errs[k]), (k, errs[k])
    d, e = recs[-1], o.diag[-1]
    for k in ("min_trc", "energy", "mean_trc", "dpdx"):
        assert abs(d[k] - e[k]) <= 1e-8 * max(1.0, abs(e[k])), (k, d[k], e[k])


XFORM_CASES = [
    ("3D 64x33x16 x6", Grid(3, 64, 33, 16), dict(wi=50.0, dt=5e-4, eps=1e-3), 6),     # lines of 96
    ("3D 128x33x8 x6", Grid(3, 128, 33, 8), dict(wi=50.0, dt=5e-4), 6),               # lines of 192
    ("3D 256x17x4 x4", Grid(3, 256, 17, 4), dict(wi=20.0, dt=1e-3, eps=1e-3), 4),     # lines of 384
    # enough lines (25 x 72) for the launch shapes of the large grids (lines
    # of 192 in FP64 and of 384 in both precisions: two workgroups per CU)
    ("3D 128x17x48 x4", Grid(3, 128, 17, 48), dict(wi=50.0, dt=5e-4), 4),             # lines of 192
    ("3D 256x17x48 x3", Grid(3, 256, 17, 48), dict(wi=20.0, dt=1e-3, eps=1e-3), 3),   # lines of 384
    # lines of 768 (whole-line form only): two load batches per wave
    ("3D 512x17x4 x3", Grid(3, 512, 17, 4), dict(wi=20.0, dt=1e-3), 3),
]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", XFORM_CASES, ids=[c[0] for c in XFORM_CASES])
def test_xpencil_forms_match_oracle(P, case, precision, monkeypatch):
    """Both forms of the 3D x pencil (the whole line in LDS, and the chunked
    one that streams the gradients through LDS in field chunks), forced with
    PCS_XPENCIL_FORM, against the FP64 oracle (the FP64 tolerances, or the
    mixed bar), and in FP64 against each other (the same products summed in
    another order) to the same tolerances.  FP64 3D lines of 768 do not fit
    a CU's LDS (18 field pairs of 768 complex values): initialisation
    reports the size unsupported."""
    name, g, prm, n = case
    if precision == 0 and 3 * g.nx // 2 > 384:
        with pytest.raises(P.PcsError) as ex:
            P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(precision=0, **prm), seed=3, amp=1e-3)
        assert ex.value.status == P.PCS_ERR_UNSUPPORTED
        return
    o = Oracle(g, Params(**prm), seed=3, amp=1e-3)
    o.step(n)
    b = o.get_state()
    N = g.ny - 1
    got = {}
    for form in ("whole", "chunked"):
        monkeypatch.setenv("PCS_XPENCIL_FORM", form)
        print("case xpencil %s %s p%d" % (form, name, precision), flush=True)
        sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(precision=precision, **prm),
                    seed=3, amp=1e-3)
        sim.step(n)
        a = sim.get_state()
        recs, st = sim.diagnostics()
        sim.close()
        assert st == P.PCS_OK and len(recs) == n
        if precision == 0:
            check_state(a, b, g, tol_prognostic(N), tol_history(N), name + " " + form)
        else:
            errs = fluct_errors(a, b, g)
            for k in state_layout(g)[1][:11]:
                assert mixed_ok(errs[k]), (form, k, errs[k])
        got[form] = a
    if precision == 0:
        check_state(got["chunked"], got["whole"], g, tol_prognostic(N), tol_history(N), name + " forms")


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
def test_mixed_keeps_laminar_state_exact(P, precision):
    """With no fluctuation the FP32 part contributes nothing: the laminar state
    stays fixed to FP64 roundoff in mixed precision too (measured 5e-13 after
    30 steps, against ~1e-7 for any FP32 contribution)."""
    print("case mixed laminar p%d" % precision, flush=True)
    for dims in ((2, 32, 65, 1), (3, 16, 33, 16)):
        sim = P.Sim(P.make_grid(*dims), P.make_params(wi=20.0, dt=1e-3, precision=precision), seed=0, amp=0.0)
        s0 = sim.get_state()
        sim.step(30)
        s1 = sim.get_state()
        sim.close()
        assert np.abs(s1[4:] - s0[4:]).max() / np.abs(s0[4:]).max() < 1e-11


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("case", [("2D 64x65 eps 0.05 x40", Grid(2, 64, 65), 40),
                                  ("3D 16x33x16 eps 0.05 x20", Grid(3, 16, 33, 16), 20)], ids=["2D", "3D"])
def test_mixed_precision_sptt_against_fp64_oracle(P, case, precision):
    """The sPTT term (eq. (1), eps > 0) in mixed precision: its fluctuation
    part in FP32 ((Tbar + T') C' + T' Cbar with T = Tr(c - I), C = c - I) and
    the mean-profile product in the FP64 mean column, held to the mixed bar
    against the FP64 oracle.  eps = 0.05 makes the term a visible part of F."""
    name, g, n = case
    prm = dict(wi=20.0, dt=1e-3, eps=0.05)
    print("case mixed sptt p%d %s" % (precision, name), flush=True)
    sim = P.Sim(P.make_grid(g.dim, g.nx, g.ny, g.nz, g.lx, g.lz), P.make_params(precision=precision, **prm),
                seed=4, amp=1e-2)
    sim.step(n)
    a = sim.get_state()
    recs, st = sim.diagnostics()
    sim.close()
    o = Oracle(g, Params(**prm), seed=4, amp=1e-2)
    o.step(n)
    b = o.get_state()
    errs = fluct_errors(a, b, g)
    nq = 6 if g.dim == 2 else 11
    names = state_layout(g)[1][:nq]
    print(name, " ".join("%s=%.1e/%.1e" % (k, v[0], v[1]) for k, v in errs.items() if k in names), flush=True)
    for k in names:
        assert mixed_ok(errs[k]), (k, errs[k])
    # the term matters: without it the laminar mean c_xx differs at the 1e-2 level
    o0 = Oracle(g, Params(wi=20.0, dt=1e-3), seed=4, amp=1e-2)
    o0.step(n)
    hdr, _, per = state_layout(g)
    ic = names.index("cxx")
    x = b[hdr + ic * 2 * per: hdr + (ic + 1) * 2 * per]
    y = o0.get_state()[hdr + ic * 2 * per: hdr + (ic + 1) * 2 * per]
    assert np.abs(x - y).max() / np.abs(y).max() > 1e3 * errs["cxx"][1]


@pytest.mark.parametrize("a,b", [((2, 16, 17, 1), (2, 32, 33, 1)), ((2, 32, 33, 1), (2, 16, 17, 1)),
                                 ((3, 16, 17, 16), (3, 8, 33, 8))])
def test_restart_at_another_resolution(P, a, b):
    """Steps on one grid, pcs_resample_state to another, steps there: the
    library end to end against the oracle doing the same with its own
    resampling."""
    print("case restart", a, "->", b, flush=True)
    prm = dict(wi=20.0, dt=1e-3)
    ga, gb = Grid(*a), Grid(*b)
    s1 = P.Sim(P.make_grid(*a), P.make_params(**prm), seed=3, amp=1e-3)
    s1.step(4)
    mid = P.resample_state(P.make_grid(*a), s1.get_state(), P.make_grid(*b))
    s1.close()
    s2 = P.Sim(P.make_grid(*b), P.make_params(**prm), seed=0, amp=0.0)
    s2.set_state(mid)
    s2.step(3)
    got = s2.get_state()
    s2.close()
    from oracle.resample import resample_state
    o1 = Oracle(ga, Params(**prm), seed=3, amp=1e-3)
    o1.step(4)
    o2 = Oracle(gb, Params(**prm), seed=None)
    o2.set_state(resample_state(ga, o1.get_state(), gb))
    o2.step(3)
    N = b[2] - 1
    check_state(got, o2.get_state(), gb, tol_prognostic(N), tol_history(N), "restart %s->%s" % (a, b))
