"""Pins of the oracle's SBDF4 scheme (the paper's 4th-order semi-implicit
BDF, Section 2; Wang and Ruuth 2008) against facts that do not depend on it.
Each case starts from an exact history, so the scheme's own recursion
applies from the first step:
  * a uniform conformation perturbation s = c_xx - 1 with no flow obeys the
    scalar ODE ds/dt = -(s + eps s^2)/Wi (eq. 1: relaxation implicit, the
    sPTT term explicit), solved in closed form; the oracle must follow the
    scalar SBDF4 recursion to roundoff and converge at 4th order;
  * the mean flow with beta = 1 under a constant drive is the linear
    semi-discrete diffusion dU/dt = (1/Re) D2 U + Pi; started on its slowest
    eigenmode it must follow the scalar recursion for that eigenvalue;
  * a single Stokes eigenmode (kx != 0) of the discrete phi-v problem with
    v = Dv = 0 at the walls, found here by a generalised eigen-solve of the
    collocation equations (independent of the influence-matrix method), must
    follow the scalar recursion as well (tiny amplitude: quadratic terms
    cannot feed back into the same Fourier mode at first order)."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import Grid, Oracle, Params
from oracle.channel import SBDF4_A0, SBDF4_ALPHA, SBDF4_BETA, q_h_fields
from oracle.cheb import operators


def recursion(lam, hist, f, dt, nsteps, past_f):
    """Scalar SBDF4 for y' = lam y + f(y): hist = [y^n, y^{n-1}, y^{n-2},
    y^{n-3}], past_f the explicit values at the same times."""
    y, fx = list(hist), list(past_f)
    for _ in range(nsteps):
        rhs = sum(a * v for a, v in zip(SBDF4_ALPHA, y)) / dt + sum(b * v for b, v in zip(SBDF4_BETA, fx))
        yn = rhs / (SBDF4_A0 / dt - lam)
        y = [yn] + y[:3]
        fx = [f(yn)] + fx[:3]
    return y[0]


def sptt_run(dt, T, s0=1.0, wi=1.0, eps=0.5):
    g = Grid(2, 8, 9)
    p = Params(re=1.0, wi=wi, beta=0.5, kappa=0.0, eps=eps, dt=dt, forcing=1, q_or_dpdx=0.0, scheme=1)
    o = Oracle(g, p, seed=None)

    def exact(t):
        e = np.exp(-t / wi)
        return s0 * e / (1.0 + eps * s0 * (1.0 - e))

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
    n = int(round(T / dt))
    o.step(n)
    got = o.q["cxx"][:, 0, 0].real - 1.0
    rec = recursion(-1.0 / wi, s, F, dt, n, [F(v) for v in s])
    return got, rec, exact(n * dt)


def test_sptt_relaxation_follows_recursion_and_converges():
    errs = []
    for dt in (0.025, 0.0125):
        got, rec, ex = sptt_run(dt, 1.0)
        assert np.abs(got - rec).max() <= 1e-13, (dt, got, rec)
        assert np.ptp(got) <= 1e-14          # stays uniform in y
        errs.append(abs(rec - ex))
    ratio = errs[0] / errs[1]
    assert 14.0 < ratio < 20.0, (errs, ratio)   # 2^4 = 16 (17.9 measured)


def test_mean_flow_eigenmode_follows_recursion():
    dt, nsteps = 0.02, 10
    g = Grid(2, 8, 17)
    p = Params(re=1.0, wi=1.0, beta=1.0, kappa=0.0, eps=0.0, dt=dt, forcing=1, q_or_dpdx=2.0, scheme=1)
    o = Oracle(g, p, seed=None)
    N = g.ny - 1
    D2 = operators(N).D2
    lam, V = np.linalg.eig(D2[1:N, 1:N])
    i = np.argmax(lam.real)
    lam1, psi = lam[i].real, V[:, i].real
    Uinf = np.zeros(N + 1)
    Uinf[1:N] = np.linalg.solve(D2[1:N, 1:N], -2.0 * np.ones(N - 1))
    mode = np.zeros(N + 1)
    mode[1:N] = psi / np.abs(psi).max()
    for name in o.q:
        o.q[name][:] = 0
    for suf, k in (("", 0), ("@1", 1), ("@2", 2), ("@3", 3)):
        o.q["u" + suf][:, 0, 0] = Uinf + mode * np.exp(-lam1 * k * dt)
        o.q["cxx" + suf][:, 0, 0] = 1.0
        o.q["cyy" + suf][:, 0, 0] = 1.0
    o.step(nsteps)
    amp = recursion(lam1, [np.exp(-lam1 * k * dt) for k in range(4)], lambda y: 0.0, dt, nsteps, [0.0] * 4)
    want = Uinf + amp * mode
    assert np.abs(o.q["u"][:, 0, 0].real - want).max() <= 1e-13 * np.abs(want).max()
    assert abs(o.pi - 2.0) == 0.0


def stokes_eigenmode(N, k2, nu):
    """Slowest decaying (phi, v, lambda) of lambda phi = nu (D2 - k^2) phi at
    interior rows, (D2 - k^2) v = phi at interior rows, v = Dv = 0 at both
    walls (collocation on the Lobatto points)."""
    op = operators(N)
    D, D2 = op.D, op.D2
    n1 = N + 1
    A = np.zeros((2 * n1, 2 * n1))
    B = np.zeros_like(A)
    L = D2 - k2 * np.eye(n1)
    r = 0
    for i in range(1, N):                  # phi equation
        A[r, :n1] = nu * L[i]
        B[r, i] = 1.0
        r += 1
    for i in range(1, N):                  # v = lap^-1 phi
        A[r, n1:] = L[i]
        A[r, i] = -1.0
        r += 1
    for row in (np.eye(n1)[0], np.eye(n1)[N], D[0], D[N]):
        A[r, n1:] = row
        r += 1
    w, X = sla.eig(A, B)
    ok = np.isfinite(w)
    w, X = w[ok], X[:, ok]
    i = np.argmax(w.real)
    x = X[:, i]
    x = x / x[n1:][np.argmax(np.abs(x[n1:]))]
    return x[:n1], x[n1:], w[i]


def test_stokes_eigenmode_follows_recursion():
    dt, nsteps, amp = 0.01, 8, 1e-7
    g = Grid(2, 8, 17, lx=2 * np.pi)
    p = Params(re=1.0, wi=1.0, beta=1.0, kappa=0.0, eps=0.0, dt=dt, forcing=1, q_or_dpdx=0.0, scheme=1)
    o = Oracle(g, p, seed=None)
    N = g.ny - 1
    kx = 1.0
    phi, v, lam = stokes_eigenmode(N, kx * kx, 1.0)
    assert abs(lam.imag) < 1e-9 * abs(lam.real) and lam.real < 0
    phi, v, lam = phi.real, v.real, lam.real
    D = operators(N).D
    for name in o.q:
        o.q[name][:] = 0
    for suf, k in (("", 0), ("@1", 1), ("@2", 2), ("@3", 3)):
        a = amp * np.exp(-lam * k * dt)
        o.q["phi" + suf][:, 0, 1] = a * phi
        o.q["v" + suf][:, 0, 1] = a * v
        o.q["u" + suf][:, 0, 1] = a * 1j * kx * (D @ v) / (kx * kx)
        o.q["cxx" + suf][:, 0, 0] = 1.0
        o.q["cyy" + suf][:, 0, 0] = 1.0
    o.step(nsteps)
    y = recursion(lam, [amp * np.exp(-lam * k * dt) for k in range(4)], lambda y: 0.0, dt, nsteps, [0.0] * 4)
    for name, ref in (("v", v), ("phi", phi)):
        got = o.q[name][:, 0, 1]
        assert np.abs(got - y * ref).max() <= 1e-9 * abs(y) * np.abs(ref).max(), name


def test_layout_and_cold_start():
    g = Grid(2, 8, 9)
    o = Oracle(g, Params(scheme=1), seed=3, amp=1e-3)
    qn, hn = q_h_fields(2)
    for n in qn:
        for k in (1, 2, 3):
            assert np.array_equal(o.q[n + "@%d" % k], o.q[n])
    for n in hn:
        for k in (2, 3):
            assert np.array_equal(o.q[n + "@%d" % k], o.q[n])
    s = o.get_state()
    assert s.size == 4 + (4 * len(qn) + 3 * len(hn)) * g.ny * (g.nx // 2) * 2
    o2 = Oracle(g, Params(scheme=1), seed=None).set_state(s)
    o.step(2)
    o2.step(2)
    assert np.array_equal(o.get_state(), o2.get_state())
    with pytest.raises(ValueError):
        Oracle(g, Params(scheme=2))


def test_wall_coupled_polymer_diffusion_matches_dense_sbdf4():
    """A mean-mode c_xx = 1 + s(y) with no flow and kappa > 0: the interior
    obeys ds/dt = kappa D2 s - s/Wi, the two wall values the same with
    kappa = 0 (the Section 2 wall condition), so the interior is driven by
    the decaying wall values through the first and last columns of D2.  The
    oracle must equal SBDF4 applied to this linear (N+1)-point system, written
    here as one dense solve per step."""
    dt, nsteps, wi, kappa = 0.01, 9, 1.0, 0.05
    g = Grid(2, 8, 17)
    p = Params(re=1.0, wi=wi, beta=0.5, kappa=kappa, eps=0.0, dt=dt, forcing=1, q_or_dpdx=0.0, scheme=1)
    o = Oracle(g, p, seed=None)
    N = g.ny - 1
    D2 = operators(N).D2
    A = kappa * D2.copy()
    A[0] = 0.0
    A[N] = 0.0
    A -= np.eye(N + 1) / wi
    y = operators(N).y
    rng = np.random.default_rng(5)
    hist = [0.3 * np.cos(1.3 * y + 0.2 * k) + 0.1 * rng.standard_normal(N + 1) for k in range(4)]
    for name in o.q:
        o.q[name][:] = 0
    for suf, k in (("", 0), ("@1", 1), ("@2", 2), ("@3", 3)):
        o.q["cxx" + suf][:, 0, 0] = 1.0 + hist[k]
        o.q["cyy" + suf][:, 0, 0] = 1.0
    o.step(nsteps)
    s = list(hist)
    M = SBDF4_A0 / dt * np.eye(N + 1) - A
    for _ in range(nsteps):
        rhs = sum(a * v for a, v in zip(SBDF4_ALPHA, s)) / dt
        s = [np.linalg.solve(M, rhs)] + s[:3]
    got = o.q["cxx"][:, 0, 0].real - 1.0
    assert np.abs(got - s[0]).max() <= 1e-13 * np.abs(s[0]).max()
    assert np.abs(o.q["u"]).max() < 1e-14      # a mean c_xx drives no flow
