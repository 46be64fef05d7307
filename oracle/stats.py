"""Midplane statistics of the polymer stretch (paper, Section 3, eqs. (4)-(5)).

TEST INFRASTRUCTURE ONLY (see the package docstring): the check for the HIP
library's on-device midplane histogram.

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
