"""Periodic (x, z) directions of the oracle: mode tables and padded transforms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper uses Fourier series in the streamwise and spanwise directions with
full dealiasing (Section 2).  Conventions here:

  * a real field is q(x, z) = sum_k qhat_k exp(i (kx x + kz z)) over all
    retained k (negative kx implied by conjugate symmetry);
  * kx = 2 pi m / Lx, m = 0 .. Nx/2 - 1 (the Nyquist mode is not kept);
  * kz slots follow FFT order at the base size Nz: slot s holds
    m_z = s for s < Nz/2 and m_z = s - Nz for s > Nz/2; slot Nz/2 (Nyquist)
    is always zero.  In 2D there is a single slot (Nz = 1);
  * spectral arrays are laid out [..., kz slot, kx];
  * forward transforms divide by the number of points.

The padded (3/2-rule) transforms evaluate on Px = 3Nx/2 and Pz = 3Nz/2
points; the base-grid transforms use Nx and Nz points.  numpy.fft is used as
the library primitive.
"""

import numpy as np


def kx_values(nx, lx):
    return 2.0 * np.pi * np.arange(nx // 2) / lx


def mz_of_slot(nz):
    """Integer spanwise mode number of each slot (0 for the Nyquist slot)."""
    if nz == 1:
        return np.zeros(1, dtype=np.int64)
    s = np.arange(nz)
    m = np.where(s < nz // 2, s, s - nz)
    m[nz // 2] = 0
    return m


def kz_values(nz, lz):
    if nz == 1:
        return np.zeros(1)
    return 2.0 * np.pi * mz_of_slot(nz) / lz


def slot_mask(nz):
    """True for retained spanwise slots (everything but the Nyquist slot)."""
    m = np.ones(nz, dtype=bool)
    if nz > 1:
        m[nz // 2] = False
    return m


def to_physical(qhat, px, pz):
    """Spectral [..., nz_slots, nkx] -> physical [..., pz, px] (real).

    pz = 1 means a 2D field (single slot).  Zero padding places every retained
    mode at its own frequency in the larger transform.
    """
    nzs, nkx = qhat.shape[-2:]
    lead = qhat.shape[:-2]
    spec = np.zeros(lead + (pz, px // 2 + 1), dtype=np.complex128)
    if pz == 1:
        spec[..., 0, :nkx] = qhat[..., 0, :]
    else:
        m = mz_of_slot(nzs)
        keep = slot_mask(nzs)
        for s in np.nonzero(keep)[0]:
            spec[..., m[s] % pz, :nkx] = qhat[..., s, :]
        spec = np.fft.ifft(spec, axis=-2) * pz
    return np.fft.irfft(spec, n=px, axis=-1) * px


def to_spectral(q, nzs, nkx):
    """Physical [..., pz, px] -> spectral [..., nzs, nkx], truncated to the
    retained modes (the Nyquist slot is left zero)."""
    pz, px = q.shape[-2:]
    spec = np.fft.rfft(q, axis=-1) / px
    lead = q.shape[:-2]
    out = np.zeros(lead + (nzs, nkx), dtype=np.complex128)
    if pz == 1:
        out[..., 0, :] = spec[..., 0, :nkx]
    else:
        spec = np.fft.fft(spec, axis=-2) / pz
        m = mz_of_slot(nzs)
        keep = slot_mask(nzs)
        for s in np.nonzero(keep)[0]:
            out[..., s, :] = spec[..., m[s] % pz, :nkx]
    return out
