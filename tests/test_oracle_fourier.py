"""Pins of the oracle's periodic transforms and explicit terms against brute force.

Fourier in x and z with full (3/2-rule) dealiasing (paper, Section 2).  The
brute-force side evaluates every series by direct summation (no FFT) and
every Chebyshev interpolant through numpy.polynomial.chebyshev, so a wrong
sign, index or normalisation in the oracle shows up here.
"""

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import Grid, Oracle, Params
from oracle import fourier as fr
from tests.inputs import random_state, smooth_random_field


def _direct_physical(qhat, nx_pts, nz_pts, lx, lz, dim):
    """q(x, z) = Re[sum_mz qhat(0, mz) e^{i kz z}] + 2 Re[sum_{mx>0, mz} qhat e^{i(kx x + kz z)}]."""
    ny_, nzs, nkx = qhat.shape
    x = np.arange(nx_pts) * lx / nx_pts
    z = np.arange(nz_pts) * lz / nz_pts if dim == 3 else np.zeros(1)
    mz = fr.mz_of_slot(nzs) if dim == 3 else np.zeros(1, dtype=int)
    keep = fr.slot_mask(nzs)
    out = np.zeros((ny_, len(z), nx_pts))
    for iz in range(nzs):
        if not keep[iz]:
            continue
        kz = 2 * np.pi * mz[iz] / lz
        for ix in range(nkx):
            kx = 2 * np.pi * ix / lx
            ph = np.exp(1j * (kz * z[:, None] + kx * x[None, :]))
            term = qhat[:, iz, ix][:, None, None] * ph[None]
            out += (1.0 if ix == 0 else 2.0) * term.real
    return out


def _direct_spectral(q, nzs, nkx, lx, lz, dim):
    ny_, pz, px = q.shape
    x = np.arange(px) * lx / px
    z = np.arange(pz) * lz / pz if dim == 3 else np.zeros(1)
    mz = fr.mz_of_slot(nzs) if dim == 3 else np.zeros(1, dtype=int)
    keep = fr.slot_mask(nzs)
    out = np.zeros((ny_, nzs, nkx), dtype=np.complex128)
    for iz in range(nzs):
        if not keep[iz]:
            continue
        kz = 2 * np.pi * mz[iz] / lz
        for ix in range(nkx):
            kx = 2 * np.pi * ix / lx
            ph = np.exp(-1j * (kz * z[:, None] + kx * x[None, :]))
            out[:, iz, ix] = (q * ph[None]).sum(axis=(1, 2)) / (px * pz)
    return out


@pytest.mark.parametrize("dim,nx,nz", [(2, 8, 1), (2, 16, 1), (3, 8, 8), (3, 12, 16)])
def test_transforms_match_direct_sums(dim, nx, nz):
    rng = np.random.default_rng(3)
    q = smooth_random_field(rng, dim, nx, 9, nz, 1.0)
    lx, lz = 10.0, 5.0
    for px, pz in [(nx, nz), (3 * nx // 2, 3 * nz // 2)]:
        pz_ = 1 if dim == 2 else pz
        phys = fr.to_physical(q, px, pz_)
        ref = _direct_physical(q, px, pz_, lx, lz, dim)
        assert np.max(np.abs(phys - ref)) < 1e-13
        back = fr.to_spectral(phys, q.shape[1], q.shape[2])
        assert np.max(np.abs(back - q)) < 1e-14
        assert np.max(np.abs(_direct_spectral(phys, q.shape[1], q.shape[2], lx, lz, dim) - q)) < 1e-14


@pytest.mark.parametrize("dim,nx,nz", [(2, 16, 1), (3, 8, 8)])
def test_padded_product_is_exact_convolution(dim, nx, nz):
    """3/2 padding makes the truncated product of two retained-mode fields exact."""
    rng = np.random.default_rng(4)
    a = smooth_random_field(rng, dim, nx, 5, nz, 1.0)
    b = smooth_random_field(rng, dim, nx, 5, nz, 1.0)
    px, pz = 3 * nx // 2, (1 if dim == 2 else 3 * nz // 2)
    prod = fr.to_spectral(fr.to_physical(a, px, pz) * fr.to_physical(b, px, pz), a.shape[1], a.shape[2])
    # exact: product on a fine grid (4x, no aliasing possible), then truncation
    fx, fz = 4 * nx, (1 if dim == 2 else 4 * nz)
    exact = _direct_spectral(_direct_physical(a, fx, fz, 10.0, 5.0, dim) * _direct_physical(b, fx, fz, 10.0, 5.0, dim),
                             a.shape[1], a.shape[2], 10.0, 5.0, dim)
    assert np.max(np.abs(prod - exact)) < 1e-13


def _brute_explicit(o):
    """Explicit terms of eqs. (1)-(2) evaluated by direct sums (no FFT, no
    oracle operator matrices): values and derivatives of each Chebyshev
    interpolant from numpy.polynomial, products on the padded grid, direct
    Fourier projection, padded-grid Chebyshev coefficients truncated to N."""
    g, q = o.g, o.q
    dim, N, M = g.dim, o.N, o.M
    y = np.cos(np.pi * np.arange(N + 1) / N)
    yp = np.cos(np.pi * np.arange(M + 1) / M)
    V = npc.chebvander(y, N)
    Vp = npc.chebvander(yp, M)
    px, pz = o.px, o.pz
    kx = 2 * np.pi * np.arange(o.nkx) / g.lx
    kz = (2 * np.pi * fr.mz_of_slot(o.nzs) / g.lz) if dim == 3 else np.zeros(1)

    def ycoef(f):
        sh = f.shape
        return np.linalg.solve(V, f.reshape(N + 1, -1)).reshape(sh)

    def to_pad(f, deriv):
        a = ycoef(f)
        if deriv:
            a = npc.chebder(a, axis=0)
        vals = npc.chebval(yp, a.reshape(a.shape[0], -1)).T.reshape((M + 1,) + f.shape[1:])
        return _direct_physical(vals, px, pz, g.lx, g.lz, dim)

    def from_pad(fp):
        s = _direct_spectral(fp, o.nzs, o.nkx, g.lx, g.lz, dim)
        a = np.linalg.solve(Vp, s.reshape(M + 1, -1))[: N + 1]
        return npc.chebval(y, a).T.reshape((N + 1,) + s.shape[1:])

    ikx = 1j * kx[None, None, :]
    ikz = 1j * kz[None, :, None]
    axes = ("x", "y") if dim == 2 else ("x", "y", "z")
    vel = {"x": q["u"], "y": q["v"]}
    if dim == 3:
        vel["z"] = q["w"]
    U = {a: to_pad(vel[a], False) for a in axes}
    dU = {}
    for a in axes:
        dU[("x", a)] = to_pad(ikx * vel[a], False)
        dU[("y", a)] = to_pad(vel[a], True)
        if dim == 3:
            dU[("z", a)] = to_pad(ikz * vel[a], False)
    comps = o.comps
    C = {ab: to_pad(q["c" + ab], False) for ab in comps}
    dC = {}
    for ab in comps:
        dC[("x", ab)] = to_pad(ikx * q["c" + ab], False)
        dC[("y", ab)] = to_pad(q["c" + ab], True)
        if dim == 3:
            dC[("z", ab)] = to_pad(ikz * q["c" + ab], False)

    def c(a, b):
        return C["".join(sorted(a + b))]

    Nn = {a: from_pad(-sum(U[k] * dU[(k, a)] for k in axes)) for a in axes}
    F = {}
    for ab in comps:
        a, b = ab
        f = -sum(U[k] * dC[(k, ab)] for k in axes)
        for k in axes:
            f = f + dU[(k, a)] * c(k, b) + c(a, k) * dU[(k, b)]
        F[ab] = from_pad(f)
    return Nn, F


@pytest.mark.parametrize("dim,nx,ny,nz", [(2, 8, 9, 1), (3, 8, 9, 8)])
def test_explicit_terms_brute_force(dim, nx, ny, nz):
    o = Oracle(Grid(dim, nx, ny, nz), Params(wi=20.0))
    st = random_state(dim, nx, ny, nz, seed=11, amp=0.3)
    o.set_state(st)
    # the oracle takes d_y v from continuity; make the random state satisfy it
    # so the brute-force side (which differentiates v directly) sees the same field
    if dim == 2:
        k2 = np.where(o.nonzero, o.k2, 1.0)[None]
        o.q["u"] = np.where(o.nonzero[None], 1j * o.kx[None, None, :] * np.tensordot(o.op.D, o.q["v"], axes=(1, 0)) / k2, o.q["u"])
    else:
        ikx = 1j * o.kx[None, None, :]
        ikz = 1j * o.kz[None, :, None]
        k2 = np.where(o.nonzero, o.k2, 1.0)[None]
        Dv = np.tensordot(o.op.D, o.q["v"], axes=(1, 0))
        nzm = o.nonzero[None]
        o.q["u"] = np.where(nzm, (ikx * Dv - ikz * o.q["g"]) / k2, o.q["u"])
        o.q["w"] = np.where(nzm, (ikz * Dv + ikx * o.q["g"]) / k2, o.q["w"])
    o.q["v"][:, 0, 0] = 0
    Nh, Fh = o.explicit()
    Nb, Fb = _brute_explicit(o)
    for a in Nh:
        scale = max(np.abs(Nb[a]).max(), 1e-30)
        assert np.abs(Nh[a] - Nb[a]).max() / scale < 1e-11, a
    for ab in Fh:
        scale = max(np.abs(Fb[ab]).max(), 1e-30)
        assert np.abs(Fh[ab] - Fb[ab]).max() / scale < 1e-11, ab
