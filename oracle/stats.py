"""Midplane statistics of the polymer stretch (paper, Section 3, eqs. (4)-(5)).

TEST INFRASTRUCTURE ONLY (see the package docstring): the check for the HIP
library's on-device midplane histograms (Tr c and the velocity fluctuations).

The paper samples Tr c on the channel midplane y = 0 over many snapshots,
builds the PDF P_c of those samples, and reports the probability of an
unphysical sample, P(Tr c < 3) = integral of P_c below 3 (eq. (4)), and
chi = N_events P(Tr c < 3) / (Nx Nz) (eq. (5)), N_events being the number of
samples: the number of samples below 3 per midplane point.  Here the PDF is
held as counts over nbins uniform bins of [lo, hi) plus two outer counts.
"""

import numpy as np


def histogram(values, lo, hi, nbins):
    """Counts of the samples: counts[0] below lo; counts[b] (1 <= b <= nbins)
    for 1 + floor((v - lo) nbins / (hi - lo)) = b, the scaled offset formed as
    (v - lo) * (nbins / (hi - lo)) in float64; counts[nbins + 1] at or above
    hi and non-finite samples."""
    v = np.asarray(values, dtype=np.float64).ravel()
    u = (v - lo) * (nbins / (hi - lo))
    with np.errstate(invalid="ignore"):
        over = ~(u < nbins)          # also NaN and +inf
        under = ~over & (u < 0.0)    # also -inf
    inside = ~(over | under)
    out = np.zeros(nbins + 2, dtype=np.uint64)
    out[0] = under.sum()
    out[nbins + 1] = over.sum()
    out[1:nbins + 1] = np.bincount(np.floor(u[inside]).astype(np.int64), minlength=nbins)[:nbins]
    return out


def probability_below(values, threshold=3.0):
    """Eq. (4) from the samples: the fraction of samples below the threshold."""
    v = np.asarray(values, dtype=np.float64).ravel()
    return float(np.count_nonzero(v < threshold)) / v.size


def chi(values, nx, nz, threshold=3.0):
    """Eq. (5): N_events P(Tr c < 3) / (Nx Nz)."""
    v = np.asarray(values, dtype=np.float64).ravel()
    return v.size * probability_below(v, threshold) / (nx * nz)


def midplane_quantities(oracle):
    """The midplane samples of the current state of an Oracle, by quantity:
    0 Tr c, 1 u - U(0), 2 v, 3 w - W(0) (3D), 4 du/dx, 5 du/dz (3D),
    6 dw/dx (3D), 7 dw/dz (3D), on the base grid of the row j = N/2 (y = 0),
    with U(0), W(0) the plane means (the kx = kz = 0 mode) of u and w there
    and the gradients as spectral derivatives (i kx, i kz times each mode).
    Section 3 compares the PDFs of the velocity fluctuations and of the
    longitudinal (du/dx, dw/dz) and transverse (du/dz, dw/dx) gradients
    across resolutions."""
    j = oracle.N // 2
    q = oracle.q
    ikx = 1j * oracle.kx[None, None, :]
    ikz = 1j * oracle.kz[None, :, None]
    out = {0: oracle.trace_c()[j].ravel().copy()}
    u = oracle.base_grid(q["u"])[j]
    out[1] = (u - q["u"][j, 0, 0].real).ravel()
    out[2] = oracle.base_grid(q["v"])[j].ravel()
    out[4] = oracle.base_grid(ikx * q["u"])[j].ravel()
    if oracle.g.dim == 3:
        w = oracle.base_grid(q["w"])[j]
        out[3] = (w - q["w"][j, 0, 0].real).ravel()
        out[5] = oracle.base_grid(ikz * q["u"])[j].ravel()
        out[6] = oracle.base_grid(ikx * q["w"])[j].ravel()
        out[7] = oracle.base_grid(ikz * q["w"])[j].ravel()
    return out


def moments(values):
    """(count, sum, sum of squares) of the finite samples: the standardised
    PDFs of Section 3 use mean = sum / count and the standard deviation
    sqrt(sum of squares / count - mean^2)."""
    v = np.asarray(values, dtype=np.float64).ravel()
    v = v[np.isfinite(v)]
    return float(v.size), float(v.sum()), float((v * v).sum())
