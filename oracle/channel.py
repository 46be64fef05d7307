"""The oracle: one CNAB2 or SBDF4 step of the polymer channel-flow problem, in
float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Equations (paper, Section 2): eq. (1) for the conformation tensor c, eq. (2)
for the momentum, eq. (3) incompressibility; no-slip walls, conformation
wall values from eq. (1) with kappa = 0; Fourier x/z, Chebyshev y, fully
dealiased.  The discrete problem solved here, step by step:

1. Explicit terms at step n, on the padded grid (3/2 rule in x, z; M = 3N/2
   Lobatto intervals in y):
      N_a  = - sum_k u_k d_k u_a                                 (eq. 2)
      F_ab = - sum_k u_k d_k c_ab + sum_k (d_k u_a) c_kb
             + sum_k c_ak (d_k u_b) - (eps/Wi) Tr(c - I)(c_ab - delta_ab)
                                                                 (eq. 1)
   with d_y v taken from continuity, d_y v = -d_x u - d_z w (eq. 3).
   Products are projected back to the retained Fourier modes and to degree
   N in y (P_NM).
2. Spectral assembly on the float64 state:
      G  = (1 - beta)/(Re Wi) div c,   H = N + G                 (eq. 2)
      h_v = -D(i kx H_x + i kz H_z) - k^2 H_y,   h_g = i kz H_x - i kx H_z
   (curl-curl and curl of eq. 2: velocity-vorticity form).
3. CNAB2 (Crank-Nicolson on the implicit terms, 2nd-order Adams-Bashforth
   on the explicit ones; the first step uses X^{-1} := X^0):
      phi = lap v:  (1/dt - nu/2 lap) phi^{n+1} = (1/dt + nu/2 lap) phi^n
                    + 3/2 h_v^n - 1/2 h_v^{n-1}   at interior points,
                    lap v^{n+1} = phi^{n+1}, v = dv/dy = 0 at the walls,
                    solved with two homogeneous solutions and a 2x2
                    influence matrix;
      g = omega_y:  the same Helmholtz operator, g = 0 at the walls;
      mean flow:    (1/dt - nu/2 D^2) U^{n+1} = ... + Pi^{n+1}, U = 0 at the
                    walls, sum_j w_j U_j = Q (flux held, Pi solved for);
      c:            (1/dt + 1/(2Wi) - kappa/2 lap) c^{n+1} = (1/dt - 1/(2Wi)
                    + kappa/2 lap) c^n + 3/2 F^n - 1/2 F^{n-1} + delta/Wi,
                    with kappa = 0 in the two wall rows (Section 2 wall
                    condition).
   nu = beta/Re, lap = D^2 - k^2.  Then u, w follow from continuity and
   omega_y:  u = (i kx Dv - i kz g)/k^2,  w = (i kz Dv + i kx g)/k^2.
3'. SBDF4 (scheme 1; the paper's time integrator, Section 2: the 4th-order
   semi-implicit BDF of Wang and Ruuth 2008), with L the implicit linear part
   of each equation above and X the explicit terms:
      (25/12 q^{n+1} - 4 q^n + 3 q^{n-1} - 4/3 q^{n-2} + 1/4 q^{n-3}) / dt
          = 4 X^n - 6 X^{n-1} + 4 X^{n-2} - X^{n-3} + L q^{n+1},
   i.e. every Helmholtz operator above with 1/dt -> 25/(12 dt) and the
   implicit weight 1/2 -> 1 (no explicit half of L).  The state then also
   carries q^{n-1..n-3} and X^{n-2}, X^{n-3}; a fresh initial condition
   fills them with a constant past (q^{n-k} := q^n, X^{n-k} := X^n).
4. Diagnostics on the base grid (Section 3 observables): min Tr c and counts
   of Tr c < 3 and Tr c < 0 over the volume and on the midplane y = 0
   (eqs. 4-5 use the midplane counts), CFL number, blow-up flag, kinetic
   energy and mean Tr c.

Dirichlet sub-problems are solved by dense LU per wavenumber (scipy), which
is independent of the diagonalisation used by the HIP library.
"""

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
from threadpoolctl import threadpool_limits

from . import fourier as fr
from .cheb import operators
from .initial import _basis, laminar_profiles, perturbation_modes

COMPS = {2: ("xx", "xy", "yy"), 3: ("xx", "xy", "xz", "yy", "yz", "zz")}
BLOWUP_TRC = 1.0e12


@dataclass
class Grid:
    dim: int
    nx: int
    ny: int
    nz: int = 1
    lx: float = 10.0
    lz: float = 5.0


@dataclass
class Params:
    re: float = 0.01
    wi: float = 20.0
    beta: float = 0.8
    kappa: float = 5.0e-5
    eps: float = 0.0
    dt: float = 1.0e-3
    forcing: int = 0          # 0: constant flux Q, 1: constant drive dp/dx
    q_or_dpdx: float = 4.0 / 3.0
    scheme: int = 0           # 0: CNAB2, 1: SBDF4

# SBDF4 (Wang and Ruuth 2008, constant step): leading coefficient, weights of
# q^{n-k} and of the explicit terms X^{n-k}, k = 0..3
SBDF4_A0 = 25.0 / 12.0
SBDF4_ALPHA = (4.0, -3.0, 4.0 / 3.0, -0.25)
SBDF4_BETA = (4.0, -6.0, 4.0, -1.0)


def q_h_fields(dim):
    if dim == 2:
        q = ["u", "v", "phi"] + ["c" + c for c in COMPS[2]]
        h = ["hv"] + ["F" + c for c in COMPS[2]]
    else:
        q = ["u", "v", "w", "phi", "g"] + ["c" + c for c in COMPS[3]]
        h = ["hv", "hg"] + ["F" + c for c in COMPS[3]]
    return q, h


def state_fields(dim, scheme=0):
    """Names of the state fields in the order of the flat state vector: the
    state q^n and the explicit terms X^{n-1} (h); SBDF4 adds q^{n-1..n-3}
    ("name@k") and X^{n-2}, X^{n-3}."""
    q, h = q_h_fields(dim)
    out = q + h
    if scheme == 1:
        out += [f"{n}@{k}" for k in (1, 2, 3) for n in q] + [f"{n}@{k}" for k in (2, 3) for n in h]
    return out


def state_layout(grid, scheme=0):
    """(header length, field names, complex values per field) of the flat
    float64 state vector: header [step, t, Pi, 0] then each field as
    [y (N+1)][kz slot][kx (Nx/2)] complex, real/imag interleaved."""
    nzs = 1 if grid.dim == 2 else grid.nz
    per = (grid.ny) * nzs * (grid.nx // 2)
    return 4, state_fields(grid.dim, scheme), per


def _sym(a, b):
    return "".join(sorted(a + b))


class Oracle:
    """FP64 oracle; see the module docstring for the discrete problem."""

    def __init__(self, grid, params, seed=None, amp=1.0e-3, cache_lu=True):
        g = grid
        if g.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if g.nx % 2 or g.nx < 4:
            raise ValueError("nx must be even and >= 4")
        if (g.ny - 1) % 2 or g.ny < 5:
            raise ValueError("ny must be odd and >= 5")
        if g.dim == 3 and (g.nz % 2 or g.nz < 4):
            raise ValueError("nz must be even and >= 4 in 3D")
        if g.dim == 2:
            g.nz = 1
        self.g, self.p = g, params
        if params.scheme not in (0, 1):
            raise ValueError("scheme must be 0 (CNAB2) or 1 (SBDF4)")
        # Helmholtz coefficients: 1/dt and implicit weight 1/2 (CNAB2) or
        # 25/(12 dt) and 1 (SBDF4)
        self.ia = 1.0 / params.dt if params.scheme == 0 else SBDF4_A0 / params.dt
        self.th = 0.5 if params.scheme == 0 else 1.0
        self.N = g.ny - 1
        self.op = operators(self.N)
        self.M = self.op.M
        self.nkx = g.nx // 2
        self.nzs = 1 if g.dim == 2 else g.nz
        self.px = 3 * g.nx // 2
        self.pz = 1 if g.dim == 2 else 3 * g.nz // 2
        self.kx = fr.kx_values(g.nx, g.lx)
        self.kz = fr.kz_values(self.nzs, g.lz) if g.dim == 3 else np.zeros(1)
        self.k2 = self.kz[:, None] ** 2 + self.kx[None, :] ** 2
        keep = fr.slot_mask(self.nzs)
        self.retained = np.broadcast_to(keep[:, None], (self.nzs, self.nkx)).copy()
        self.nonzero = self.retained.copy()
        self.nonzero[0, 0] = False
        self.comps = COMPS[g.dim]
        self.cache_lu = cache_lu
        self._lu = {}
        self._infl = {}
        self._build_mean_solver()
        shape = (self.N + 1, self.nzs, self.nkx)
        self.q = {name: np.zeros(shape, dtype=np.complex128) for name in state_fields(g.dim, params.scheme)}
        self.step_count = 0
        self.t = 0.0
        self.pi = 2.0 / params.re if params.forcing == 1 else 0.0
        self.diag = []
        if seed is not None:
            self.set_initial(seed, amp)

    # ------------------------------------------------------------------ setup
    def set_initial(self, seed, amp):
        """Laminar base state plus the seeded divergence-free perturbation;
        history set to the explicit terms of this state (CNAB1 start)."""
        g, p, op = self.g, self.p, self.op
        y = op.y
        U, _, cxx, cxy, cyy = laminar_profiles(y, p.wi, p.kappa)
        for name in self.q:
            self.q[name][:] = 0
        self.q["u"][:, 0, 0] = U
        self.q["cxx"][:, 0, 0] = cxx
        self.q["cxy"][:, 0, 0] = cxy
        self.q["cyy"][:, 0, 0] = cyy
        if g.dim == 3:
            self.q["czz"][:, 0, 0] = cyy
        pb, pb1, pb2 = _basis(y)
        psi = {}
        for pot, mx, mz, th in perturbation_modes(g.dim, seed):
            if mx >= self.nkx or (g.dim == 3 and abs(mz) >= self.g.nz // 2):
                continue
            coef = amp * np.exp(1j * np.asarray(th))
            val = (coef[:, None] * pb).sum(0), (coef[:, None] * pb1).sum(0), (coef[:, None] * pb2).sum(0)
            psi[(pot, mx, mz)] = val
            if g.dim == 3 and mx == 0:
                psi[(pot, 0, -mz)] = tuple(np.conj(a) for a in val)
        slots = fr.mz_of_slot(self.nzs)
        for iz in range(self.nzs):
            mz = int(slots[iz]) if g.dim == 3 else 0
            if not self.retained[iz, 0]:
                continue
            kz = self.kz[iz]
            for ix in range(self.nkx):
                if iz == 0 and ix == 0:
                    continue
                kx = self.kx[ix]
                k2 = kx * kx + kz * kz
                z0 = np.zeros(self.N + 1, dtype=np.complex128)
                ps, ps1, ps2 = psi.get(("psi", ix, mz), (z0, z0, z0))
                ch, ch1, ch2 = psi.get(("chi", ix, mz), (z0, z0, z0))
                if not (np.any(ps) or np.any(ch)):
                    continue
                u = ps1
                w = ch1
                v = -1j * kx * ps - 1j * kz * ch
                v2 = -1j * kx * ps2 - 1j * kz * ch2
                self.q["u"][:, iz, ix] = u
                self.q["v"][:, iz, ix] = v
                self.q["phi"][:, iz, ix] = v2 - k2 * v
                if g.dim == 3:
                    self.q["w"][:, iz, ix] = w
                    self.q["g"][:, iz, ix] = 1j * kz * u - 1j * kx * w
        self.step_count = 0
        self.t = 0.0
        self.pi = p.q_or_dpdx if p.forcing == 1 else 2.0 / p.re
        self.init_history()

    def init_history(self):
        """History := explicit terms of the current state (CNAB1 first step);
        SBDF4: a constant past, q^{n-k} := q^n and X^{n-k} := X^n."""
        Nh, Fh = self.explicit()
        hv, hg = self.assemble(Nh)
        self.q["hv"][:] = hv
        if self.g.dim == 3:
            self.q["hg"][:] = hg
        for c in self.comps:
            self.q["F" + c][:] = Fh[c]
        if self.p.scheme == 1:
            qn, hn = q_h_fields(self.g.dim)
            for k in (1, 2, 3):
                for n in qn:
                    self.q[f"{n}@{k}"] = self.q[n].copy()
            for k in (2, 3):
                for n in hn:
                    self.q[f"{n}@{k}"] = self.q[n].copy()

    def _build_mean_solver(self):
        p, op, N = self.p, self.op, self.N
        nu = p.beta / p.re
        D2 = op.D2
        A = self.ia * np.eye(N - 1) - self.th * nu * D2[1:N, 1:N]
        self._lu_mean = sla.lu_factor(A)
        U1 = np.zeros(N + 1)
        U1[1:N] = sla.lu_solve(self._lu_mean, np.ones(N - 1))
        self._U1 = U1
        self._wU1 = float(op.w @ U1)

    def _mode_solvers(self, k2):
        """LU factors and influence data for one wavenumber magnitude k^2 > 0."""
        key = float(k2)
        if key in self._lu:
            return self._lu[key]
        p, op, N = self.p, self.op, self.N
        nu = p.beta / p.re
        D2 = op.D2
        D2ii = D2[1:N, 1:N]
        I = np.eye(N - 1)
        Hphi = (self.ia + self.th * nu * k2) * I - self.th * nu * D2ii
        Lv = D2ii - k2 * I
        lu_phi = sla.lu_factor(Hphi)
        lu_v = sla.lu_factor(Lv)
        # homogeneous solutions: phi = 1 at y = +1 (j = 0) or y = -1 (j = N)
        homo = []
        for jb in (0, N):
            phi = np.zeros(N + 1)
            phi[jb] = 1.0
            phi[1:N] = sla.lu_solve(lu_phi, self.th * nu * D2[1:N, jb])
            v = np.zeros(N + 1)
            v[1:N] = sla.lu_solve(lu_v, phi[1:N])
            homo.append((phi, v))
        (phi1, v1), (phi2, v2) = homo
        Dm = op.D
        A = np.array([[Dm[0] @ v1, Dm[0] @ v2], [Dm[N] @ v1, Dm[N] @ v2]])
        lu_c = None
        if p.kappa > 0:
            Hc = (self.ia + self.th / p.wi + self.th * p.kappa * k2) * I - self.th * p.kappa * D2ii
            lu_c = sla.lu_factor(Hc)
        out = dict(phi=lu_phi, v=lu_v, c=lu_c, phi1=phi1, phi2=phi2, v1=v1, v2=v2, A=A)
        if self.cache_lu:
            self._lu[key] = out
        return out

    def solve_phi_v(self, k2, r_int):
        """Influence-matrix solve of one mode: given the interior right-hand
        side of the phi equation, return (phi, v) on all N+1 points with
        lap v = phi inside and v = Dv = 0 at both walls."""
        N, D = self.N, self.op.D
        S = self._mode_solvers(k2)
        rr = np.stack([np.real(r_int), np.imag(r_int)], axis=1)
        php = sla.lu_solve(S["phi"], rr, check_finite=False)
        vp = sla.lu_solve(S["v"], php, check_finite=False)
        vp_full = np.zeros(N + 1, dtype=np.complex128)
        vp_full[1:N] = vp[:, 0] + 1j * vp[:, 1]
        rhs = -np.array([D[0] @ vp_full, D[N] @ vp_full])
        ab = np.linalg.solve(S["A"], rhs)
        phin = np.zeros(N + 1, dtype=np.complex128)
        phin[1:N] = php[:, 0] + 1j * php[:, 1]
        return phin + ab[0] * S["phi1"] + ab[1] * S["phi2"], vp_full + ab[0] * S["v1"] + ab[1] * S["v2"]

    def _c_solver_mean(self):
        key = ("c00",)
        if key not in self._lu:
            p, N = self.p, self.N
            D2ii = self.op.D2[1:N, 1:N]
            Hc = (self.ia + self.th / p.wi) * np.eye(N - 1) - self.th * p.kappa * D2ii
            self._lu[key] = sla.lu_factor(Hc)
        return self._lu[key]

    # ------------------------------------------------------------ transforms
    def _yI(self, a):
        return np.tensordot(self.op.I_MN, a, axes=(1, 0))

    def _yD(self, a):
        return np.tensordot(self.op.D_MN, a, axes=(1, 0))

    def _phys(self, a):
        return fr.to_physical(a, self.px, self.pz)

    def _spec(self, f):
        s = fr.to_spectral(f, self.nzs, self.nkx)
        return np.tensordot(self.op.P_NM, s, axes=(1, 0))

    def _c(self, a, b, q=None):
        """Spectral component c_ab (2D: c_zz = 1 on the mean mode, c_xz = c_yz = 0)."""
        q = self.q if q is None else q
        key = _sym(a, b)
        if "c" + key in q:
            return q["c" + key]
        out = np.zeros_like(q["u"])
        if key == "zz":
            out[:, 0, 0] = 1.0
        return out

    # -------------------------------------------------------- explicit terms
    def explicit(self):
        """Projected spectral N_a (a = x, y[, z]) and F_ab (stored components)."""
        dim = self.g.dim
        q = self.q
        ikx = 1j * self.kx[None, None, :]
        ikz = 1j * self.kz[None, :, None]
        axes = ("x", "y") if dim == 2 else ("x", "y", "z")
        vel = {"x": q["u"], "y": q["v"]}
        if dim == 3:
            vel["z"] = q["w"]
        U = {a: self._phys(self._yI(vel[a])) for a in axes}
        dU = {}
        for a in axes:
            dU[("x", a)] = self._phys(self._yI(ikx * vel[a]))
            if dim == 3:
                dU[("z", a)] = self._phys(self._yI(ikz * vel[a]))
        dU[("y", "x")] = self._phys(self._yD(vel["x"]))
        if dim == 3:
            dU[("y", "z")] = self._phys(self._yD(vel["z"]))
            dU[("y", "y")] = -dU[("x", "x")] - dU[("z", "z")]
        else:
            dU[("y", "y")] = -dU[("x", "x")]
        C, dC = {}, {}
        for ab in self.comps:
            ch = q["c" + ab]
            C[ab] = self._phys(self._yI(ch))
            dC[("x", ab)] = self._phys(self._yI(ikx * ch))
            dC[("y", ab)] = self._phys(self._yD(ch))
            if dim == 3:
                dC[("z", ab)] = self._phys(self._yI(ikz * ch))

        def cphys(a, b):
            return C[_sym(a, b)]

        Nout = {}
        for a in axes:
            Nout[a] = -sum(U[k] * dU[(k, a)] for k in axes)
        eps, wi = self.p.eps, self.p.wi
        if eps != 0.0:
            tr = sum(cphys(a, a) - 1.0 for a in axes)
        Fout = {}
        for ab in self.comps:
            a, b = ab[0], ab[1]
            f = -sum(U[k] * dC[(k, ab)] for k in axes)
            f = f + sum(dU[(k, a)] * cphys(k, b) for k in axes)
            f = f + sum(cphys(a, k) * dU[(k, b)] for k in axes)
            if eps != 0.0:
                f = f - (eps / wi) * tr * (cphys(a, b) - (1.0 if a == b else 0.0))
            Fout[ab] = f
        Nh = {a: self._spec(Nout[a]) for a in axes}
        Fh = {ab: self._spec(Fout[ab]) for ab in self.comps}
        return Nh, Fh

    def assemble(self, Nh):
        """h_v and h_g (curl-curl / curl of H = N + G); the mean-mode slots
        of h_v and h_g carry the mean streamwise / spanwise H profiles."""
        dim, p, op = self.g.dim, self.p, self.op
        ikx = 1j * self.kx[None, None, :]
        ikz = 1j * self.kz[None, :, None]
        coef = (1.0 - p.beta) / (p.re * p.wi)

        def yd(a):
            return np.tensordot(op.D, a, axes=(1, 0))

        axes = ("x", "y") if dim == 2 else ("x", "y", "z")
        H = {}
        for a in axes:
            div = ikx * self._c("x", a) + yd(self._c("y", a))
            if dim == 3:
                div = div + ikz * self._c("z", a)
            H[a] = Nh[a] + coef * div
        s = ikx * H["x"]
        if dim == 3:
            s = s + ikz * H["z"]
        hv = -yd(s) - self.k2[None] * H["y"]
        hv[:, 0, 0] = H["x"][:, 0, 0].real
        hg = None
        if dim == 3:
            hg = ikz * H["x"] - ikx * H["z"]
            hg[:, 0, 0] = H["z"][:, 0, 0].real
        mask = self.retained[None]
        hv = np.where(mask, hv, 0)
        if hg is not None:
            hg = np.where(mask, hg, 0)
        return hv, hg

    # ------------------------------------------------------------------ step
    def step(self, n=1):
        for _ in range(n):
            self._one_step()
            self.diag.append(self.diagnostics())
        return self

    def _one_step(self):
        g, p, op, N = self.g, self.p, self.op, self.N
        q = self.q
        dt = p.dt
        nu = p.beta / p.re
        Nh, Fh = self.explicit()
        hv, hg = self.assemble(Nh)
        new = {k: np.zeros_like(v) for k, v in q.items()}
        k2 = self.k2[None]

        def d2(a):
            return np.tensordot(op.D2, a, axes=(1, 0))

        sb = p.scheme == 1

        def past(name):
            """SBDF4 history of the state: sum_k alpha_k q^{n-k} / dt."""
            a = SBDF4_ALPHA
            return (a[0] * q[name] + a[1] * q[name + "@1"] + a[2] * q[name + "@2"] + a[3] * q[name + "@3"]) / dt

        def extrap(new_x, name):
            """Explicit terms at n+1: AB2 (CNAB2) or the SBDF4 extrapolation."""
            if not sb:
                return 1.5 * new_x - 0.5 * q[name]
            b = SBDF4_BETA
            return b[0] * new_x + b[1] * q[name] + b[2] * q[name + "@2"] + b[3] * q[name + "@3"]

        # right-hand sides of every mode at once
        if sb:
            r_phi = past("phi") + extrap(hv, "hv")
            if g.dim == 3:
                r_g = past("g") + extrap(hg, "hg")
        else:
            r_phi = (1.0 / dt - 0.5 * nu * k2) * q["phi"] + 0.5 * nu * d2(q["phi"]) \
                + 1.5 * hv - 0.5 * q["hv"]
            if g.dim == 3:
                r_g = (1.0 / dt - 0.5 * nu * k2) * q["g"] + 0.5 * nu * d2(q["g"]) \
                    + 1.5 * hg - 0.5 * q["hg"]
        a_int = 1.0 / dt - 0.5 / p.wi
        a_new = self.ia + self.th / p.wi
        r_c, r_cw = {}, {}
        for ab in self.comps:
            c = q["c" + ab]
            expl = extrap(Fh[ab], "F" + ab)
            if sb:
                r_c[ab] = past("c" + ab) + expl
                r_cw[ab] = r_c[ab].copy()
            else:
                r_c[ab] = (a_int - 0.5 * p.kappa * k2) * c + 0.5 * p.kappa * d2(c) + expl
                r_cw[ab] = a_int * c + expl
            if ab[0] == ab[1]:
                r_c[ab][:, 0, 0] += 1.0 / p.wi
                r_cw[ab][:, 0, 0] += 1.0 / p.wi

        def ri(vec):
            return np.stack([vec.real, vec.imag], axis=1)

        with threadpool_limits(limits=1, user_api="blas"):
            # velocity: phi, v (and g in 3D) for every nonzero retained mode
            for iz in range(self.nzs):
                for ix in range(self.nkx):
                    if not self.nonzero[iz, ix]:
                        continue
                    S = self._mode_solvers(self.k2[iz, ix])
                    phin, vn = self.solve_phi_v(self.k2[iz, ix], r_phi[1:N, iz, ix])
                    new["phi"][:, iz, ix] = phin
                    new["v"][:, iz, ix] = vn
                    if g.dim == 3:
                        gs = sla.lu_solve(S["phi"], ri(r_g[1:N, iz, ix]), check_finite=False)
                        new["g"][1:N, iz, ix] = gs[:, 0] + 1j * gs[:, 1]

            # mean flow (kx = kz = 0): constant flux or constant drive
            U = q["u"][:, 0, 0].real
            if sb:
                r = past("u")[:, 0, 0].real + extrap(hv, "hv")[:, 0, 0].real
            else:
                r = U / dt + 0.5 * nu * (op.D2 @ U) + 1.5 * hv[:, 0, 0].real - 0.5 * q["hv"][:, 0, 0].real
            Up = np.zeros(N + 1)
            Up[1:N] = sla.lu_solve(self._lu_mean, r[1:N], check_finite=False)
            if p.forcing == 0:
                pi = (p.q_or_dpdx - op.w @ Up) / self._wU1
            else:
                pi = p.q_or_dpdx
            new["u"][:, 0, 0] = Up + pi * self._U1
            self.pi = float(pi)
            if g.dim == 3:
                W = q["w"][:, 0, 0].real
                if sb:
                    r = past("w")[:, 0, 0].real + extrap(hg, "hg")[:, 0, 0].real
                else:
                    r = W / dt + 0.5 * nu * (op.D2 @ W) + 1.5 * hg[:, 0, 0].real - 0.5 * q["hg"][:, 0, 0].real
                Wn = np.zeros(N + 1)
                Wn[1:N] = sla.lu_solve(self._lu_mean, r[1:N], check_finite=False)
                new["w"][:, 0, 0] = Wn

            # conformation tensor: interior Helmholtz rows, kappa = 0 wall rows
            for ab in self.comps:
                cn = np.zeros_like(q["c" + ab])
                cn[0] = r_cw[ab][0] / a_new
                cn[N] = r_cw[ab][N] / a_new
                if p.kappa > 0:
                    rin = r_c[ab][1:N] + self.th * p.kappa * (
                        op.D2[1:N, 0][:, None, None] * cn[0][None] + op.D2[1:N, N][:, None, None] * cn[N][None])
                    for iz in range(self.nzs):
                        for ix in range(self.nkx):
                            if not self.retained[iz, ix]:
                                continue
                            if iz == 0 and ix == 0:
                                lu = self._c_solver_mean()
                            else:
                                lu = self._mode_solvers(self.k2[iz, ix])["c"]
                            sol = sla.lu_solve(lu, ri(rin[:, iz, ix]), check_finite=False)
                            cn[1:N, iz, ix] = sol[:, 0] + 1j * sol[:, 1]
                else:
                    cn[1:N] = r_c[ab][1:N] / a_new
                cn[:, 0, 0] = cn[:, 0, 0].real
                cn[:, ~self.retained] = 0
                new["c" + ab] = cn

        # u, w of the nonzero modes from continuity and omega_y
        ikx = 1j * self.kx[None, None, :]
        ikz = 1j * self.kz[None, :, None]
        k2s = np.where(self.nonzero, self.k2, 1.0)[None]
        Dv = np.tensordot(op.D, new["v"], axes=(1, 0))
        nz = self.nonzero[None]
        if g.dim == 3:
            un = (ikx * Dv - ikz * new["g"]) / k2s
            wn = (ikz * Dv + ikx * new["g"]) / k2s
            new["w"] = np.where(nz, wn, new["w"])
        else:
            un = ikx * Dv / k2s
        new["u"] = np.where(nz, un, new["u"])

        # history
        if sb:
            qn, hn = q_h_fields(g.dim)
            for n in qn:
                new[n + "@3"], new[n + "@2"], new[n + "@1"] = q[n + "@2"], q[n + "@1"], q[n]
            for n in hn:
                new[n + "@3"], new[n + "@2"] = q[n + "@2"], q[n]
        new["hv"] = hv
        if g.dim == 3:
            new["hg"] = hg
        for ab in self.comps:
            new["F" + ab] = Fh[ab]
        self.q = new
        self.step_count += 1
        self.t += dt

    # ----------------------------------------------------------- diagnostics
    def base_grid(self, qhat):
        """Spectral field -> values on the base grid [y][z][x]."""
        pz = 1 if self.g.dim == 2 else self.g.nz
        return fr.to_physical(qhat, self.g.nx, pz)

    def trace_c(self):
        q = self.q
        if self.g.dim == 2:
            return self.base_grid(q["cxx"] + q["cyy"]) + 1.0
        return self.base_grid(q["cxx"] + q["cyy"] + q["czz"])

    def diagnostics(self):
        g, p, op, N = self.g, self.p, self.op, self.N
        q = self.q
        trc = self.trace_c()
        u = self.base_grid(q["u"])
        v = self.base_grid(q["v"])
        w = self.base_grid(q["w"]) if g.dim == 3 else np.zeros_like(u)
        allv = np.stack([trc, u, v, w])
        finite = np.isfinite(allv).all()
        blow = (not finite) or bool(np.nanmax(np.abs(trc)) > BLOWUP_TRC)
        mid = trc[N // 2]
        y = op.y
        dy = np.empty(N + 1)
        dy[1:N] = 0.5 * (y[0:N - 1] - y[2:N + 1])
        dy[0] = y[0] - y[1]
        dy[N] = y[N - 1] - y[N]
        dx = g.lx / g.nx
        cfl_f = np.abs(u) / dx + np.abs(v) / dy[:, None, None]
        if g.dim == 3:
            cfl_f = cfl_f + np.abs(w) / (g.lz / g.nz)
        ww = op.w / 2.0
        ke = 0.5 * (u * u + v * v + w * w)
        return dict(
            step=self.step_count, t=self.t,
            min_trc=float(np.nanmin(trc)), mid_min_trc=float(np.nanmin(mid)),
            cfl=float(p.dt * np.nanmax(cfl_f)), dpdx=self.pi,
            energy=float(ww @ ke.mean(axis=(1, 2))), mean_trc=float(ww @ trc.mean(axis=(1, 2))),
            n_lt3=int((trc < 3.0).sum()), n_lt0=int((trc < 0.0).sum()),
            mid_n_lt3=int((mid < 3.0).sum()), mid_n_lt0=int((mid < 0.0).sum()),
            blowup=int(blow),
        )

    # ----------------------------------------------------------- state I/O
    def get_state(self):
        hdr, names, per = state_layout(self.g, self.p.scheme)
        out = np.zeros(hdr + len(names) * per * 2)
        out[0], out[1], out[2] = self.step_count, self.t, self.pi
        o = hdr
        for name in names:
            out[o:o + 2 * per] = self.q[name].view(np.float64).ravel()
            o += 2 * per
        return out

    def set_state(self, flat):
        hdr, names, per = state_layout(self.g, self.p.scheme)
        flat = np.asarray(flat, dtype=np.float64)
        if flat.size != hdr + len(names) * per * 2:
            raise ValueError("state vector has the wrong length")
        self.step_count = int(flat[0])
        self.t = float(flat[1])
        self.pi = float(flat[2])
        o = hdr
        shape = (self.N + 1, self.nzs, self.nkx)
        for name in names:
            self.q[name] = flat[o:o + 2 * per].copy().view(np.complex128).reshape(shape)
            o += 2 * per
        return self

    def fields(self):
        return {k: v.copy() for k, v in self.q.items()}
