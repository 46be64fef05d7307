"""Laminar base state and the seeded initial perturbation (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Laminar state (eqs. (1)-(2) with d/dt = d/dx = d/dz = 0, Section 2 scalings):
the Newtonian-scaled Poiseuille profile U = 1 - y^2 carries, for eps = 0,
    c_xy = Wi U' = -2 Wi y,   c_yy = c_zz = 1,
    c_xx = 1 + 2 (Wi U')^2 + 16 kappa Wi^3 [1 - cosh(y/l)/cosh(1/l)],
with l = sqrt(kappa Wi).  The bracket solves kappa f'' - f/Wi = -8 Wi y^2 for
f = c_xx - 1 with wall values taken from eq. (1) at kappa = 0 (the wall
condition of Section 2); it vanishes for kappa = 0.  The streamwise drive
that holds this state is Pi = 2/Re (eq. (2)).

Perturbation: a divergence-free field from streamfunctions built from
(1 - y^2)^2 T_n(y), n = 0..4 (polynomial degree <= 8, so u = du/dy = 0 at the
walls), with amplitude `amp` per coefficient and phases 2 pi u01 drawn from
SplitMix64 (Steele, Lea and Flood 2014), u01 = (x >> 11) 2^-53.
  2D: psi = sum_{m=1..4} sum_{n=0..4} amp [e^{i(k_m x + th_mn)} + c.c.] p_n(y)
      u' = d psi/dy, v' = -d psi/dx; draw order m outer, n inner.
  3D: psi and chi over m_x = 0..4, m_z = -4..4, (m_x, m_z) != (0, 0), m_z > 0
      when m_x = 0; u' = d psi/dy, w' = d chi/dy, v' = -d psi/dx - d chi/dz;
      draw order psi then chi, then m_x, m_z, n.
Phases are drawn for every listed mode even when a small grid cannot hold it,
so one seed gives the same continuous field at every resolution.
"""

import numpy as np

from .cheb import cheb_poly_values

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea and Flood 2014), one 64-bit word per call."""

    def __init__(self, seed):
        self.s = seed & MASK64

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def u01(self):
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def laminar_profiles(y, wi, kappa):
    """U, U', c_xx, c_xy, c_yy (= c_zz) of the laminar state at points y."""
    y = np.asarray(y, dtype=np.float64)
    U = 1.0 - y * y
    cxy = -2.0 * wi * y
    cxx = 1.0 + 8.0 * wi * wi * y * y
    if kappa > 0.0:
        ell = np.sqrt(kappa * wi)
        a = np.abs(y)
        # cosh(y/l)/cosh(1/l) written without overflow
        ratio = np.exp((a - 1.0) / ell) * (1.0 + np.exp(-2.0 * a / ell)) / (1.0 + np.exp(-2.0 / ell))
        cxx = cxx + 16.0 * kappa * wi ** 3 * (1.0 - ratio)
    cyy = np.ones_like(y)
    return U, -2.0 * y, cxx, cxy, cyy


def _basis(y):
    """p_n = (1 - y^2)^2 T_n(y) and its first two derivatives, n = 0..4."""
    T, T1, T2 = cheb_poly_values(4, y)
    q = 1.0 - y * y
    p = q * q * T
    p1 = -4.0 * y * q * T + q * q * T1
    p2 = (12.0 * y * y - 4.0) * T - 8.0 * y * q * T1 + q * q * T2
    return p, p1, p2


def perturbation_modes(dim, seed):
    """List of (potential, m_x, m_z, [5 phases]) in draw order."""
    rng = SplitMix64(seed)
    out = []
    if dim == 2:
        for m in range(1, 5):
            out.append(("psi", m, 0, [2.0 * np.pi * rng.u01() for _ in range(5)]))
    else:
        for pot in ("psi", "chi"):
            for mx in range(0, 5):
                for mz in range(-4, 5):
                    if (mx, mz) == (0, 0) or (mx == 0 and mz < 0):
                        continue
                    out.append((pot, mx, mz, [2.0 * np.pi * rng.u01() for _ in range(5)]))
    return out
