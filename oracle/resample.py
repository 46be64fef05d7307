"""Resampling a flat state between resolutions: every run of the paper's
Table 1 starts from one snapshot re-interpolated onto its grid (Section 2),
and the conclusions propose fine-grid runs started from coarse-run snapshots.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition followed here, per field and Fourier mode:
  * wall-normal: the unique polynomial of degree <= N through the N+1 source
    Lobatto values, written in the Chebyshev basis; terms above degree
    min(N, N') are dropped; the rest is evaluated at the target Lobatto points
    y'_i = cos(pi i / N').  The coefficients come from solving the Vandermonde
    system V a = f with V[j, n] = T_n(y_j) (numpy.linalg.solve), not from the
    discrete cosine formula, so that the two routes check one another.
  * x and z: the amplitude of mode (m_x, m_z) is a resolution-independent
    Fourier coefficient; modes retained at both resolutions are copied, all
    other target modes are zero (the Nyquist slot is never retained).
  * header [step, t, Pi, 0] is copied.
"""

import numpy as np

from .channel import state_layout
from .cheb import cheb_poly_values
from .fourier import mz_of_slot, slot_mask


def lobatto(N):
    return np.cos(np.pi * np.arange(N + 1) / N)


def cheb_resample_matrix(N, Np):
    """Q[(N'+1) x (N+1)]: source Lobatto values -> target values of the
    truncated (or zero-padded) Chebyshev interpolant."""
    V, _, _ = cheb_poly_values(N, lobatto(N))
    V = V.T                                  # V[j, n] = T_n(y_j)
    A = np.linalg.solve(V, np.eye(N + 1))    # a = A f
    k = min(N, Np)
    E, _, _ = cheb_poly_values(N, lobatto(Np))
    E = E.T[:, : k + 1]                      # E[i, n] = T_n(y'_i), n <= k
    return E @ A[: k + 1]


def resample_state(src, state, dst):
    """Flat state of grid src -> flat state of grid dst (same dim, lx, lz)."""
    if src.dim != dst.dim or src.lx != dst.lx or (src.dim == 3 and src.lz != dst.lz):
        raise ValueError("grids differ in dimension or box")
    h, names, ps = state_layout(src)
    _, _, pd = state_layout(dst)
    state = np.asarray(state, dtype=np.float64)
    if state.size != h + len(names) * ps * 2:
        raise ValueError("state size does not match the source grid")
    nzs = 1 if src.dim == 2 else src.nz
    nzd = 1 if dst.dim == 2 else dst.nz
    nkxs, nkxd = src.nx // 2, dst.nx // 2
    Q = cheb_resample_matrix(src.ny - 1, dst.ny - 1)
    out = np.zeros(h + len(names) * pd * 2)
    out[:h] = state[:h]
    ms, md = mz_of_slot(nzs), mz_of_slot(nzd)
    keep_s, keep_d = slot_mask(nzs), slot_mask(nzd)
    for f in range(len(names)):
        a = state[h + f * ps * 2: h + (f + 1) * ps * 2]
        q = (a[0::2] + 1j * a[1::2]).reshape(src.ny, nzs, nkxs)
        r = np.zeros((dst.ny, nzd, nkxd), dtype=complex)
        for sd in range(nzd):
            if not keep_d[sd]:
                continue
            hit = [s for s in range(nzs) if keep_s[s] and ms[s] == md[sd]]
            if not hit:
                continue
            for k in range(min(nkxs, nkxd)):
                r[:, sd, k] = Q @ q[:, hit[0], k]
        b = out[h + f * pd * 2: h + (f + 1) * pd * 2]
        b[0::2] = r.real.ravel()
        b[1::2] = r.imag.ravel()
    return out
