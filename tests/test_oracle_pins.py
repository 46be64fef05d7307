"""Pins of the oracle's time step against closed forms, invariants and
independent solves (paper, Section 2: eqs. (1)-(3), no-slip walls,
conformation wall rows from eq. (1) with kappa = 0)."""

import json
import os

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import Grid, Oracle, Params
from oracle.initial import laminar_profiles

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("kappa", [0.0, 5e-5])
@pytest.mark.parametrize("dim,nx,ny,nz", [(2, 16, 33, 1), (3, 8, 33, 8)])
def test_laminar_fixed_point(kappa, dim, nx, ny, nz):
    """The laminar Oldroyd-B Poiseuille state is a steady solution of
    eqs. (1)-(3): U = 1 - y^2, c_xy = Wi U', c_yy = c_zz = 1,
    c_xx = 1 + 2 (Wi U')^2 (+ the polymer-diffusion boundary-layer term).
    Ny = 33 resolves the kappa > 0 layer of width sqrt(kappa Wi) = 0.05; at
    Ny = 17 the continuous profile is not the discrete fixed point (drift
    ~7e-10 in 20 steps, spectral truncation, not roundoff)."""
    o = Oracle(Grid(dim, nx, ny, nz), Params(wi=50.0, kappa=kappa, dt=5e-4), seed=5, amp=0.0)
    s0 = o.get_state().copy()
    y = o.op.y
    assert np.allclose(o.q["u"][:, 0, 0].real, 1 - y * y, rtol=0, atol=1e-15)
    if kappa == 0.0:
        assert np.allclose(o.q["cxx"][:, 0, 0].real, 1 + 2 * (50.0 * -2 * y) ** 2, rtol=1e-15)
    o.step(20)
    s1 = o.get_state()
    assert _rel(s1[4:], s0[4:]) < 2e-13
    assert abs(o.pi - 2.0 / 0.01) < 1e-9  # the drive that holds the flux is 2/Re (eq. 2)


def test_laminar_kappa_profile_solves_steady_equation():
    """The kappa > 0 c_xx profile solves kappa f'' - f/Wi = -8 Wi y^2 with
    f(+-1) = 8 Wi^2 (eq. (1), y-only steady state, wall rows at kappa = 0)."""
    wi, kappa = 20.0, 5e-5
    ell = np.sqrt(kappa * wi)
    y = np.linspace(-1, 1, 2001)
    h = 1e-4
    f = lambda s: laminar_profiles(s, wi, kappa)[2] - 1.0
    fpp = (f(y + h) - 2 * f(y) + f(y - h)) / h ** 2
    inner = np.abs(y) < 1 - 5 * h
    res = kappa * fpp - f(y) / wi + 8 * wi * y ** 2
    assert np.max(np.abs(res[inner])) / (8 * wi) < 1e-4
    assert abs(f(np.array([1.0]))[0] - 8 * wi ** 2) < 1e-9
    mid = 16 * kappa * wi ** 3 * (1 - 1 / np.cosh(1 / ell))
    assert abs(f(np.array([0.0]))[0] - mid) < 1e-9


def _poly_v(N, rng, k):
    """v* = (1 - y^2)^2 p(y), deg p <= N - 4: v = Dv = 0 at both walls."""
    p = rng.standard_normal(N - 3) * 0.6 ** np.arange(N - 3)
    w = npc.chebpow([0.5, 0, -0.5], 2)   # (1 - y^2)^2 = ((1 - T_2)/2)^2
    return npc.chebmul(w, p)


@pytest.mark.parametrize("N,k2", [(16, 0.4), (64, 0.4), (64, 40.0), (128, 3.0)])
def test_manufactured_stokes_solve(N, k2):
    """Manufactured solution for the phi-v influence solve: with
    phi* = v*'' - k^2 v* and r = alpha phi* - gamma phi*'' (exact polynomial
    derivatives), the solver returns (phi*, v*)."""
    o = Oracle(Grid(2, 8, N + 1), Params(wi=20.0, dt=1e-3))
    rng = np.random.default_rng(N)
    a = _poly_v(N, rng, k2)
    y = o.op.y
    v = npc.chebval(y, a)
    phi_c = npc.chebsub(npc.chebder(a, 2), k2 * a)
    phi = npc.chebval(y, phi_c)
    nu = o.p.beta / o.p.re
    alpha = 1.0 / o.p.dt + 0.5 * nu * k2
    r = alpha * phi - 0.5 * nu * npc.chebval(y, npc.chebder(phi_c, 2))
    phin, vn = o.solve_phi_v(k2, (1 + 0.5j) * r[1:N])
    tol_v = 2e-16 * N ** 3
    assert _rel(vn, (1 + 0.5j) * v) < tol_v
    assert _rel(phin, (1 + 0.5j) * phi) < tol_v * N


@pytest.mark.parametrize("N,k2", [(32, 1.0), (64, 12.0)])
def test_influence_equals_coupled_solve(N, k2):
    """The influence-matrix solve equals a direct dense solve of the whole
    collocation system (phi interior rows, v interior rows, v = Dv = 0)."""
    o = Oracle(Grid(2, 8, N + 1), Params(wi=20.0, dt=1e-3))
    D, D2 = o.op.D, o.op.D2
    nu = o.p.beta / o.p.re
    alpha, gam = 1.0 / o.p.dt + 0.5 * nu * k2, 0.5 * nu
    n1 = N + 1
    A = np.zeros((2 * n1, 2 * n1))
    rhs = np.zeros(2 * n1, dtype=complex)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(N - 1) + 1j * rng.standard_normal(N - 1)
    row = 0
    for j in range(1, N):
        A[row, :n1] = -gam * D2[j]
        A[row, j] += alpha
        rhs[row] = r[j - 1]
        row += 1
    for j in range(1, N):
        A[row, n1:] = D2[j]
        A[row, n1 + j] -= k2
        A[row, j] = -1.0
        row += 1
    for jb in (0, N):
        A[row, n1 + jb] = 1.0
        row += 1
        A[row, n1:] = D[jb]
        row += 1
    sol = np.linalg.solve(A, rhs)
    phin, vn = o.solve_phi_v(k2, r)
    assert _rel(vn, sol[n1:]) < 1e-11
    assert _rel(phin, sol[:n1]) < 1e-10


@pytest.mark.parametrize("dim,nx,ny,nz", [(2, 16, 33, 1), (3, 16, 17, 16)])
def test_divergence_free_and_no_slip(dim, nx, ny, nz):
    o = Oracle(Grid(dim, nx, ny, nz), Params(wi=20.0, dt=1e-3), seed=3, amp=1e-2)
    o.step(5)
    q = o.q
    Dv = np.tensordot(o.op.D, q["v"], axes=(1, 0))
    div = 1j * o.kx[None, None, :] * q["u"] + Dv
    if dim == 3:
        div = div + 1j * o.kz[None, :, None] * q["w"]
    scale = np.abs(Dv).max()
    assert np.abs(div).max() / scale < 1e-13
    for f in ("u", "v") + (("w",) if dim == 3 else ()):
        assert np.abs(q[f][[0, -1]]).max() < 1e-14
    # flux held (constant-flow-rate drive): sum_j w_j U_j = 4/3
    assert abs(o.op.w @ q["u"][:, 0, 0].real - 4.0 / 3.0) < 1e-13


def test_initial_condition_recipe():
    """Seeded IC: divergence-free, mean flux untouched, amplitude as stated,
    and the same continuous field at two resolutions."""
    o1 = Oracle(Grid(3, 16, 17, 16), Params(wi=50.0), seed=3, amp=1e-3)
    o2 = Oracle(Grid(3, 32, 17, 32), Params(wi=50.0), seed=3, amp=1e-3)
    Dv = np.tensordot(o1.op.D, o1.q["v"], axes=(1, 0))
    div = 1j * o1.kx[None, None, :] * o1.q["u"] + Dv + 1j * o1.kz[None, :, None] * o1.q["w"]
    assert np.abs(div).max() < 1e-15
    assert abs(o1.op.w @ o1.q["u"][:, 0, 0].real - 4 / 3) < 1e-15
    b1 = o1.base_grid(o1.q["v"])
    b2 = o2.base_grid(o2.q["v"])[:, ::2, ::2]
    assert np.abs(b1 - b2).max() < 1e-15
    assert 1e-4 < np.abs(b1).max() < 1.0


def test_exact_relaxation_decay_and_counts():
    """3D laminar flow with c_zz = 1 + delta uniform: the stretching of c_zz
    vanishes, so Crank-Nicolson relaxation gives delta_n = delta
    ((1 - a)/(1 + a))^n exactly, a = dt/(2 Wi).  With delta < 0 the count of
    Tr c < 3 is N_x N_z #{j : 8 Wi^2 y_j^2 < -delta_n} (kappa = 0)."""
    wi, dt = 2.0, 2e-3
    o = Oracle(Grid(3, 8, 33, 8), Params(wi=wi, kappa=0.0, dt=dt), seed=1, amp=0.0)
    delta = -0.37
    o.q["czz"][:, 0, 0] += delta
    o.init_history()
    a = dt / (2 * wi)
    y = o.op.y
    for n in range(1, 16):
        o.step(1)
        dn = delta * ((1 - a) / (1 + a)) ** n
        assert np.abs(o.q["czz"][:, 0, 0].real - (1 + dn)).max() < 1e-14
        d = o.diag[-1]
        expect = 8 * 8 * int(np.sum(8 * wi * wi * y * y < -dn))
        assert d["n_lt3"] == expect
        assert d["mid_n_lt3"] == 64
        assert d["n_lt0"] == 0
        assert abs(d["min_trc"] - (3 + dn)) < 1e-13


def test_time_order_two():
    """CNAB2 is second order: halving dt divides the error by about 4."""
    T = 0.024
    res = {}
    for dt in (4e-3, 2e-3, 1e-3, 1.25e-4):
        o = Oracle(Grid(2, 16, 17), Params(wi=2.0, kappa=0.0, dt=dt, re=1.0, beta=0.5), seed=9, amp=5e-2)
        o.step(int(round(T / dt)))
        # prognostic fields only (the history holds explicit terms at t - dt);
        # phi only inside: its two wall values are auxiliary unknowns of the
        # influence system and converge at about order 1.5
        res[dt] = np.concatenate([o.q[f].ravel() for f in ("u", "v", "cxx", "cxy", "cyy")]
                                 + [o.q["phi"][1:-1].ravel()])
    ref = res[1.25e-4]
    e = [np.abs(res[dt] - ref).max() for dt in (4e-3, 2e-3, 1e-3)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8, (e, r1, r2)


def test_mirror_symmetry_preserved():
    """An IC with the channel's y-mirror symmetry (v, phi, c_xy odd; u, c_xx,
    c_yy even) keeps it: eqs. (1)-(3) are invariant under y -> -y, v -> -v."""
    o = Oracle(Grid(2, 16, 33), Params(wi=20.0, dt=1e-3), seed=4, amp=1e-2)
    q = o.q
    for f in ("u", "cxx", "cyy"):
        q[f] = 0.5 * (q[f] + q[f][::-1])
    for f in ("v", "cxy", "phi"):
        q[f] = 0.5 * (q[f] - q[f][::-1])
    o.init_history()
    o.step(10)
    q = o.q
    for f in ("u", "cxx", "cyy"):
        assert np.abs(q[f] - q[f][::-1]).max() <= 1e-12 * np.abs(q[f]).max()
    for f in ("v", "cxy", "phi"):
        assert np.abs(q[f] + q[f][::-1]).max() <= 1e-12 * np.abs(q[f]).max()


def test_table1_arithmetic():
    """Table 1: M_dof = 10 Nx Ny Nz (6 c + 3 u + 1 p), the ratios to A1, and
    chi/P close to the number of snapshots (Delta(t/Wi) = 0.67 up to ~7.4)."""
    with open(os.path.join(GOLDEN, "table1.json")) as f:
        t = json.load(f)
    a1 = t["runs"]["A1"]["res"]
    m1 = 10 * a1[0] * a1[1] * a1[2]
    assert abs(m1 - t["mdof_A1_approx"]) / t["mdof_A1_approx"] < 0.01
    for name, run in t["runs"].items():
        r = run["res"]
        assert 10 * r[0] * r[1] * r[2] / m1 == run["mdof_ratio"]
        if run["P_1e5"] > 1e-2:
            ratio = run["chi_1e4"] * 10 / run["P_1e5"]
            assert 10.0 < ratio < 11.5
