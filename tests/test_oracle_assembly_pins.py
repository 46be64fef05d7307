"""Pins of the oracle's spectral assembly, diagnostics and 3D initial
condition against vector calculus done independently, in physical space.

The oracle writes the momentum terms in velocity-vorticity form (paper,
Section 2, eqs. (2)-(3) with the pressure eliminated): with
H = N + (1 - beta)/(Re Wi) div c,
    h_v = -(curl curl H)_y,   h_g = (curl H)_y,
and the mean-mode slots of h_v and h_g carry the plane means of H_x and
H_z.  Here a spectral field is taken as the continuous function it stands
for (a Chebyshev series in y fitted through the Lobatto values with
numpy.polynomial, Fourier series in x and z summed directly at arbitrary
points), every derivative is taken term by term on that representation, and
H, its curl and the curl of the curl are formed from their component
definitions.  The oracle's discrete operators (Lobatto differentiation
matrices, FFTs) are not used.

The diagnostics (Section 3 observables, with the energy and mean trace as
Clenshaw-Curtis averages) are pinned by the laminar closed forms and, on
random states, by a brute-force evaluation of the fields on the base grid
and exact polynomial integrals in y (the random profiles are of low enough
degree that Clenshaw-Curtis quadrature is exact).  The 3D initial
condition is pinned against the streamfunctions of its recipe:
u = d psi/dy, w = d chi/dy, v = -d psi/dx - d chi/dz, omega_y = du/dz - dw/dx
and phi = lap v.
"""

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import Grid, Oracle, Params
from oracle import fourier as fr
from oracle.initial import perturbation_modes
from tests.inputs import random_state


class SField:
    """A real field given by complex coefficients coef[n, iz, ix]: Chebyshev
    degree n in y, spanwise slot iz (wavenumber kz[iz]) and streamwise
    wavenumber kx[ix] >= 0; the kx < 0 half is the complex conjugate."""

    def __init__(self, coef, kx, kz):
        self.coef, self.kx, self.kz = coef, kx, kz

    @classmethod
    def from_lobatto(cls, vals, kx, kz):
        ny = vals.shape[0]
        y = np.cos(np.pi * np.arange(ny) / (ny - 1))
        flat = vals.reshape(ny, -1)
        cr = npc.chebfit(y, flat.real, ny - 1)
        ci = npc.chebfit(y, flat.imag, ny - 1)
        return cls((cr + 1j * ci).reshape((ny,) + vals.shape[1:]), kx, kz)

    def _new(self, c):
        return SField(c, self.kx, self.kz)

    def dx(self):
        return self._new(1j * self.kx[None, None, :] * self.coef)

    def dz(self):
        return self._new(1j * self.kz[None, :, None] * self.coef)

    def dy(self):
        c = npc.chebder(self.coef, axis=0)
        return self._new(np.concatenate([c, np.zeros((1,) + c.shape[1:], dtype=c.dtype)], axis=0))

    def __add__(self, o):
        return self._new(self.coef + o.coef)

    def __sub__(self, o):
        return self._new(self.coef - o.coef)

    def __neg__(self):
        return self._new(-self.coef)

    def __rmul__(self, s):
        return self._new(s * self.coef)

    def eval(self, x, y, z):
        """Values at every (y, z, x) of the three point lists, [y][z][x]."""
        prof = npc.chebval(y, self.coef.reshape(self.coef.shape[0], -1)).reshape(
            self.coef.shape[1:] + (len(y),))                       # [iz][ix][y]
        ex = np.exp(1j * self.kx[:, None] * x[None, :])             # [ix][x]
        ez = np.exp(1j * self.kz[:, None] * z[None, :])             # [iz][z]
        wgt = np.where(self.kx > 0, 2.0, 1.0)                       # conjugate half
        tot = np.einsum("aby,bx,az,b->yzx", prof, ex, ez, wgt)
        return tot.real


def zero_field(kx, kz, ny):
    return SField(np.zeros((ny, len(kz), len(kx)), dtype=np.complex128), kx, kz)


def oracle_fields(o):
    return {k: SField.from_lobatto(v, o.kx, o.kz) for k, v in o.q.items()}


def points(o, rng, n=7):
    g = o.g
    x = rng.uniform(0.0, g.lx, n)
    z = rng.uniform(0.0, g.lz, n) if g.dim == 3 else np.zeros(1)
    return x, o.op.y.astype(np.float64), z


def c_field(f, a, b, o):
    key = "".join(sorted(a + b))
    if "c" + key in f:
        return f["c" + key]
    s = zero_field(o.kx, o.kz, o.N + 1)
    if key == "zz":
        s.coef[0, 0, 0] = 1.0
    return s


@pytest.mark.parametrize("dims", [(2, 12, 25, 1), (3, 8, 17, 8), (3, 10, 21, 6)])
def test_assemble_is_curl_curl_and_curl_of_H(dims):
    """Oracle.assemble on a random state with random N against h_v =
    -(curl curl H)_y and h_g = (curl H)_y formed in physical space, every
    mode and every Lobatto row, plus the mean-mode slots (plane means of
    H_x, H_z); both the stress divergence G and N enter H."""
    dim, nx, ny, nz = dims
    g = Grid(dim, nx, ny, nz)
    p = Params(re=0.01, wi=20.0, beta=0.8)
    o = Oracle(g, p, seed=None)
    o.set_state(random_state(dim, nx, ny, nz, seed=31, amp=0.7))
    rng = np.random.default_rng(5)
    axes = ("x", "y") if dim == 2 else ("x", "y", "z")
    Nh = {a: o.q["u"].copy() * 0 for a in axes}
    for a in axes:
        r = random_state(dim, nx, ny, nz, seed=40 + len(a) + ord(a), amp=0.9)
        Nh[a] = r[4:4 + o.q["u"].size * 2].view(np.complex128).reshape(o.q["u"].shape)
    hv, hg = o.assemble(Nh)
    f = oracle_fields(o)
    coef = (1.0 - p.beta) / (p.re * p.wi)
    d = {"x": SField.dx, "y": SField.dy, "z": SField.dz}
    zero = zero_field(o.kx, o.kz, ny)
    H = {}
    for a in ("x", "y", "z"):
        if a not in axes:
            H[a] = zero
            continue
        div = zero
        for k in axes:
            div = div + d[k](c_field(f, k, a, o))
        H[a] = SField.from_lobatto(Nh[a], o.kx, o.kz) + coef * div
    # curl H, then the y component of curl (curl H), from the definitions
    wx = H["z"].dy() - H["y"].dz()
    wy = H["x"].dz() - H["z"].dx()
    wz = H["y"].dx() - H["x"].dy()
    cc_y = wx.dz() - wz.dx()
    x, y, z = points(o, rng)
    mean_hx = SField(H["x"].coef * 0, o.kx, o.kz)
    mean_hx.coef[:, 0, 0] = H["x"].coef[:, 0, 0].real
    want_v = (-cc_y).eval(x, y, z) + mean_hx.eval(x, y, z)
    got_v = SField.from_lobatto(hv, o.kx, o.kz).eval(x, y, z)
    scale = np.abs(want_v).max()
    assert scale > 1.0
    assert np.abs(got_v - want_v).max() <= 1e-11 * scale, np.abs(got_v - want_v).max() / scale
    if dim == 3:
        mean_hz = SField(H["z"].coef * 0, o.kx, o.kz)
        mean_hz.coef[:, 0, 0] = H["z"].coef[:, 0, 0].real
        want_g = wy.eval(x, y, z) + mean_hz.eval(x, y, z)
        got_g = SField.from_lobatto(hg, o.kx, o.kz).eval(x, y, z)
        sg = np.abs(want_g).max()
        assert sg > 0.1
        assert np.abs(got_g - want_g).max() <= 1e-11 * sg, np.abs(got_g - want_g).max() / sg


@pytest.mark.parametrize("dim,kappa", [(2, 0.0), (3, 0.0), (2, 5e-5)])
def test_laminar_diagnostics_closed_forms(dim, kappa):
    """Laminar Poiseuille state: E = <(1 - y^2)^2 / 2> = 4/15; at kappa = 0
    <Tr c> = <3 + 8 Wi^2 y^2> = 3 + 8 Wi^2 / 3, min Tr c = 3 at the midplane
    (no point strictly below 3 or 0); CFL = dt Nx / Lx (|U| = 1 at y = 0,
    v = w = 0); the drive of the flux-held state is 2/Re."""
    wi, dt = 20.0, 1e-3
    g = Grid(dim, 16, 33, 8) if dim == 3 else Grid(dim, 16, 33)
    o = Oracle(g, Params(wi=wi, dt=dt, kappa=kappa), seed=1, amp=0.0)
    d = o.diagnostics()
    assert abs(d["energy"] - 4.0 / 15.0) <= 1e-14
    assert abs(d["cfl"] - dt * g.nx / g.lx) <= 1e-15
    if kappa == 0.0:
        assert abs(d["mean_trc"] - (3.0 + 8.0 * wi * wi / 3.0)) <= 1e-12 * (8 * wi * wi)
        assert d["min_trc"] == 3.0 and d["mid_min_trc"] == 3.0
        assert d["n_lt3"] == d["n_lt0"] == d["mid_n_lt3"] == d["mid_n_lt0"] == 0
    o.step(1)
    assert abs(o.diag[-1]["dpdx"] - 2.0 / 0.01) <= 1e-9 * 200
    assert abs(o.diag[-1]["energy"] - 4.0 / 15.0) <= 1e-12


@pytest.mark.parametrize("dims", [(2, 16, 33, 1), (3, 12, 33, 8)])
def test_diagnostics_brute_force_on_random_states(dims):
    """Random state with Tr c crossing 3 and 0 at many points: min Tr c, the
    four counts and CFL against the fields evaluated point by point on the
    base grid from their series; E and <Tr c> against exact integrals
    (Parseval in x, z; numpy.polynomial integration in y; the profiles'
    squares have degree <= 28 <= N, where Clenshaw-Curtis is exact)."""
    dim, nx, ny, nz = dims
    g = Grid(dim, nx, ny, nz)
    dt = 2e-3
    o = Oracle(g, Params(wi=20.0, dt=dt), seed=None)
    st = random_state(dim, nx, ny, nz, seed=77, amp=2.0)
    o.set_state(st)
    # shift the mean traces so that Tr c straddles 3 and 0
    names = ("cxx", "cyy") if dim == 2 else ("cxx", "cyy", "czz")
    for k in names:
        o.q[k][:, 0, 0] += 0.9
    d = o.diagnostics()
    f = oracle_fields(o)
    xs = np.arange(nx) * g.lx / nx
    zs = np.arange(nz) * g.lz / nz if dim == 3 else np.zeros(1)
    y = np.cos(np.pi * np.arange(ny) / (ny - 1))
    trc = sum(f[k].eval(xs, y, zs) for k in names) + (1.0 if dim == 2 else 0.0)
    u = f["u"].eval(xs, y, zs)
    v = f["v"].eval(xs, y, zs)
    w = f["w"].eval(xs, y, zs) if dim == 3 else np.zeros_like(u)
    mid = trc[(ny - 1) // 2]
    assert 0 < (trc < 3).sum() < trc.size and 0 < (trc < 0).sum() < trc.size
    assert 0 < (mid < 3).sum() < mid.size
    # no value so close to a threshold that roundoff could decide it
    assert np.abs(trc - 3).min() > 1e-9 and np.abs(trc).min() > 1e-9
    assert d["n_lt3"] == int((trc < 3).sum()) and d["n_lt0"] == int((trc < 0).sum())
    assert d["mid_n_lt3"] == int((mid < 3).sum()) and d["mid_n_lt0"] == int((mid < 0).sum())
    assert abs(d["min_trc"] - trc.min()) <= 1e-13 * np.abs(trc).max()
    assert abs(d["mid_min_trc"] - mid.min()) <= 1e-13 * np.abs(trc).max()
    # CFL: local Lobatto spacing (y_{j-1} - y_{j+1})/2, one-sided at the walls
    dy = np.array([y[0] - y[1]] + [0.5 * (y[j - 1] - y[j + 1]) for j in range(1, ny - 1)] + [y[-2] - y[-1]])
    brute = 0.0
    for j in range(ny):
        for k in range(len(zs)):
            for i in range(nx):
                c = abs(u[j, k, i]) / (g.lx / nx) + abs(v[j, k, i]) / dy[j]
                if dim == 3:
                    c += abs(w[j, k, i]) / (g.lz / nz)
                brute = max(brute, c)
    assert abs(d["cfl"] - dt * brute) <= 1e-13 * dt * brute
    # exact averages: mean over x, z by Parseval, exact integral in y
    wgt = np.where(o.kx > 0, 2.0, 1.0)[None, :]
    msk = fr.slot_mask(o.nzs)[:, None]

    def mean_square_coef(s):
        tot = np.zeros(1)
        for iz in range(s.coef.shape[1]):
            for ix in range(s.coef.shape[2]):
                if not msk[iz, 0]:
                    continue
                a = s.coef[:, iz, ix]
                # the random velocity profiles have degree <= 14 (degree-12 series
                # times 1 - y^2): drop the fit's roundoff tail
                assert np.abs(a[15:]).max(initial=0.0) <= 1e-12 * max(np.abs(a).max(), 1e-300)
                a = a[:15]
                prod = npc.chebmul(a, np.conj(a)).real * wgt[0, ix]
                tot = npc.chebadd(tot, prod)
        return tot

    e_int = sum(mean_square_coef(f[k]) for k in (("u", "v") if dim == 2 else ("u", "v", "w")))
    assert len(e_int) <= ny   # degree <= N: Clenshaw-Curtis is exact
    E = 0.5 * 0.5 * (npc.chebval(1.0, npc.chebint(e_int)) - npc.chebval(-1.0, npc.chebint(e_int)))
    assert abs(d["energy"] - E) <= 1e-13 * max(1.0, abs(E)), (d["energy"], E)
    t00 = sum(f[k].coef[:, 0, 0].real for k in names)
    T = 0.5 * (npc.chebval(1.0, npc.chebint(t00)) - npc.chebval(-1.0, npc.chebint(t00))) + \
        (1.0 if dim == 2 else 0.0)
    assert abs(d["mean_trc"] - T) <= 1e-13 * max(1.0, abs(T)), (d["mean_trc"], T)


def test_initial_condition_3d_against_streamfunctions():
    """The seeded 3D initial state: every velocity component, phi = lap v and
    g = omega_y = du/dz - dw/dx, evaluated in physical space, against the
    same quantities formed from the recipe's streamfunctions psi and chi
    (phases of the seed, basis (1 - y^2)^2 T_n as a Chebyshev series), plus
    the laminar base state at kappa = 0."""
    g = Grid(3, 12, 17, 12, lx=10.0, lz=5.0)
    wi, amp, seed = 20.0, 1e-3, 9
    o = Oracle(g, Params(wi=wi, kappa=0.0), seed=seed, amp=amp)
    kx, kz = o.kx, o.kz
    ny = g.ny
    slots = fr.mz_of_slot(o.nzs)
    psi = zero_field(kx, kz, ny + 4)
    chi = zero_field(kx, kz, ny + 4)
    w2 = npc.chebpow([0.5, 0.0, -0.5], 2)          # (1 - y^2)^2 = ((1 - T_2)/2)^2
    for pot, mx, mz, th in perturbation_modes(3, seed):
        if mx >= o.nkx or abs(mz) >= g.nz // 2:
            continue
        series = np.zeros(ny + 4, dtype=np.complex128)
        for n in range(5):
            tn = np.zeros(n + 1)
            tn[n] = 1.0
            pn = npc.chebmul(w2, tn)
            series[:len(pn)] += amp * np.exp(1j * th[n]) * pn
        target = psi if pot == "psi" else chi
        iz = int(np.nonzero(slots == mz)[0][0])
        target.coef[:, iz, mx] += series
        if mx == 0:   # the conjugate partner of a kx = 0 mode
            iz2 = int(np.nonzero(slots == -mz)[0][0])
            target.coef[:, iz2, 0] += np.conj(series)
    u = psi.dy()
    w = chi.dy()
    v = -(psi.dx()) - chi.dz()
    gy = u.dz() - w.dx()
    phi = v.dx().dx() + v.dy().dy() + v.dz().dz()
    rng = np.random.default_rng(3)
    x, y, z = points(o, rng)
    f = oracle_fields(o)
    lam_u = (1.0 - y * y)[:, None, None]
    checks = {"u": u.eval(x, y, z) + lam_u, "v": v.eval(x, y, z), "w": w.eval(x, y, z),
              "g": gy.eval(x, y, z), "phi": phi.eval(x, y, z)}
    for k, want in checks.items():
        got = f[k].eval(x, y, z)
        sc = np.abs(want).max()
        assert sc > 0
        assert np.abs(got - want).max() <= 1e-11 * max(sc, 1e-3), (k, np.abs(got - want).max(), sc)
    # the perturbation is divergence-free and vanishes (with du/dy) at the walls
    div = (f["u"].dx() + f["v"].dy() + f["w"].dz()).eval(x, y, z)
    assert np.abs(div).max() <= 1e-13
    cxx = f["cxx"].eval(x, y, z)
    assert np.abs(cxx - (1.0 + 8.0 * wi * wi * y * y)[:, None, None]).max() <= 1e-12 * 8 * wi * wi
    assert np.abs(f["cxy"].eval(x, y, z) + 2.0 * wi * y[:, None, None]).max() <= 1e-12 * wi
