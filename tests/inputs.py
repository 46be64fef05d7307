"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Only random numbers arranged in the documented flat-state layout (header
[step, t, Pi, 0], then every field as [y][kz slot][kx] complex): no part of
the method's arithmetic lives here.  Wall-normal profiles are smooth random
Chebyshev series (numpy.polynomial evaluates them) so that derivatives are
well scaled; the kx = 0 column is given conjugate symmetry in kz and the mean
mode is real, as for any real field; the Nyquist kz slot is zero.
"""

import numpy as np
import numpy.polynomial.chebyshev as npc


def n_fields(dim):
    return 10 if dim == 2 else 19


def field_shape(dim, nx, ny, nz):
    return (ny, 1 if dim == 2 else nz, nx // 2)


def state_size(dim, nx, ny, nz=1):
    ny_, nzs, nkx = field_shape(dim, nx, ny, nz)
    return 4 + n_fields(dim) * ny_ * nzs * nkx * 2


def lobatto(ny):
    n = ny - 1
    return np.cos(np.pi * np.arange(ny) / n)


def smooth_random_field(rng, dim, nx, ny, nz, amp, decay=0.6, wall_zero=False):
    """Random complex spectral field [y][kz][kx] with a decaying spectrum."""
    ny_, nzs, nkx = field_shape(dim, nx, ny, nz)
    y = lobatto(ny)
    deg = min(ny - 1, 12)
    out = np.zeros((ny_, nzs, nkx), dtype=np.complex128)
    mz = np.zeros(nzs, dtype=int)
    if dim == 3:
        s = np.arange(nzs)
        mz = np.where(s < nzs // 2, s, s - nzs)
    for iz in range(nzs):
        if dim == 3 and iz == nzs // 2:
            continue
        for ix in range(nkx):
            damp = amp * np.exp(-0.35 * (ix + abs(mz[iz])))
            cr = rng.standard_normal(deg + 1) * decay ** np.arange(deg + 1)
            ci = rng.standard_normal(deg + 1) * decay ** np.arange(deg + 1)
            prof = npc.chebval(y, cr) + 1j * npc.chebval(y, ci)
            if wall_zero:
                prof = prof * (1 - y * y)
            out[:, iz, ix] = damp * prof
    # real-field symmetry of the kx = 0 column
    out[:, 0, 0] = out[:, 0, 0].real
    if dim == 3:
        for iz in range(1, nzs // 2):
            out[:, nzs - iz, 0] = np.conj(out[:, iz, 0])
    return out


def random_state(dim, nx, ny, nz=1, seed=0, amp=1e-3):
    """Flat state vector of random smooth fields (all fields perturbation-like;
    callers add a mean profile where they need one)."""
    rng = np.random.default_rng(seed)
    fields = [smooth_random_field(rng, dim, nx, ny, nz, amp, wall_zero=(k < (3 if dim == 2 else 5)))
              for k in range(n_fields(dim))]
    flat = np.zeros(state_size(dim, nx, ny, nz))
    o = 4
    for f in fields:
        flat[o:o + f.size * 2] = f.view(np.float64).ravel()
        o += f.size * 2
    return flat
