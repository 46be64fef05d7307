"""Pins of the oracle's wall-normal operators against the mathematics.

Chebyshev collocation (paper, Section 2: Chebyshev in the wall-normal
direction, fully dealiased).  Each check compares against something outside
the oracle: numpy.polynomial.chebyshev (library evaluation / differentiation /
integration of a Chebyshev series), the textbook closed-form Lobatto
differentiation matrix evaluated in mpmath, or exact identities.
"""

import mpmath
import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle.cheb import operators

NS = [8, 16, 64, 128, 256]


def _rand_coef(rng, deg):
    # decaying coefficients: relative accuracy of derivatives stays meaningful
    return rng.standard_normal(deg + 1) * 0.7 ** np.arange(deg + 1)


@pytest.mark.parametrize("N", NS)
def test_grid_is_lobatto(N):
    op = operators(N)
    with mpmath.workdps(40):
        exact = np.array([float(mpmath.cospi(mpmath.mpf(j) / N)) for j in range(N + 1)])
    assert np.array_equal(op.y, exact)  # correctly rounded cos(pi j / N)
    assert op.y[0] == 1.0 and op.y[N] == -1.0 and op.y[N // 2] == 0.0
    assert np.array_equal(op.y, -op.y[::-1])  # exact antisymmetry


@pytest.mark.parametrize("N", NS)
def test_derivative_exact_on_polynomials(N):
    """D_N and D_MN differentiate any degree <= N polynomial exactly (to roundoff)."""
    op = operators(N)
    rng = np.random.default_rng(N)
    a = _rand_coef(rng, N)
    f = npc.chebval(op.y, a)
    fp = npc.chebval(op.y, npc.chebder(a))
    fpp = npc.chebval(op.y, npc.chebder(a, 2))
    scale = np.max(np.abs(fp))
    tol = 4e-16 * N * N
    assert np.max(np.abs(op.D @ f - fp)) / scale < tol
    assert np.max(np.abs(op.D2 @ f - fpp)) / np.max(np.abs(fpp)) < tol * N
    fpad = npc.chebval(op.ypad, a)
    fppad = npc.chebval(op.ypad, npc.chebder(a))
    assert np.max(np.abs(op.I_MN @ f - fpad)) / np.max(np.abs(fpad)) < 50 * 2.2e-16 * np.sqrt(N)
    assert np.max(np.abs(op.D_MN @ f - fppad)) / scale < tol


@pytest.mark.parametrize("N", [8, 16, 64])
def test_D_matches_closed_form(N):
    """The Lobatto differentiation matrix built from E'_N C_N agrees with the
    textbook closed form (entries (cb_i/cb_j)(-1)^{i+j}/(y_i - y_j), corner
    entries +-(2N^2+1)/6, diagonal -y_j/(2(1-y_j^2))) evaluated in mpmath."""
    op = operators(N)
    with mpmath.workdps(40):
        y = [mpmath.cospi(mpmath.mpf(j) / N) for j in range(N + 1)]
        cb = [2 if j in (0, N) else 1 for j in range(N + 1)]
        D = np.zeros((N + 1, N + 1))
        for i in range(N + 1):
            for j in range(N + 1):
                if i != j:
                    D[i, j] = float(mpmath.mpf(cb[i]) / cb[j] * (-1) ** (i + j) / (y[i] - y[j]))
            if i == 0:
                D[i, i] = float(mpmath.mpf(2 * N * N + 1) / 6)
            elif i == N:
                D[i, i] = -float(mpmath.mpf(2 * N * N + 1) / 6)
            else:
                D[i, i] = float(-y[i] / (2 * (1 - y[i] ** 2)))
    # both are correctly rounded values of the same exact matrix
    assert np.max(np.abs(op.D - D) / np.maximum(np.abs(D), 1e-300)) <= 2.3e-16


@pytest.mark.parametrize("N", NS)
def test_projection_truncates_coefficients(N):
    """P_NM maps padded-grid values of a degree <= M series to the N-grid
    values of the same series truncated to degrees 0..N."""
    op = operators(N)
    M = op.M
    rng = np.random.default_rng(N + 1)
    a = _rand_coef(rng, M)
    fpad = npc.chebval(op.ypad, a)
    expect = npc.chebval(op.y, a[: N + 1])
    assert np.max(np.abs(op.P_NM @ fpad - expect)) < 1e-14 * np.sqrt(N)


@pytest.mark.parametrize("N", NS)
def test_roundtrip_identity(N):
    op = operators(N)
    err = np.max(np.abs(op.P_NM @ op.I_MN - np.eye(N + 1)))
    assert err < 2e-15 * N


@pytest.mark.parametrize("N", [16, 64])
def test_dealiased_product_coefficients(N):
    """Interpolating two degree-N series onto the padded grid, multiplying and
    projecting gives the exact product coefficients for degrees < N; degree N
    carries the alias a_N b_N / 2 (the 3/2 rule on Lobatto points)."""
    op = operators(N)
    rng = np.random.default_rng(7)
    a = _rand_coef(rng, N)
    b = _rand_coef(rng, N)
    fa, fb = npc.chebval(op.y, a), npc.chebval(op.y, b)
    prod = op.P_NM @ ((op.I_MN @ fa) * (op.I_MN @ fb))
    exact = npc.chebmul(a, b)
    coef = op.C_N @ prod
    assert np.max(np.abs(coef[:N] - exact[:N])) < 1e-13
    # the T_N coefficient: exact part plus the alias of the degree-2N term
    # (C_N returns the T_N coefficient with the Lobatto end weight)
    alias = exact[N] + a[N] * b[N] / 2.0
    assert abs(coef[N] - alias) < 1e-13


@pytest.mark.parametrize("N", NS)
def test_clenshaw_curtis_weights(N):
    op = operators(N)
    assert abs(op.w.sum() - 2.0) < 1e-14
    for n in range(0, N + 1):
        e = np.zeros(n + 1)
        e[n] = 1.0
        exact = npc.chebval(1.0, npc.chebint(e)) - npc.chebval(-1.0, npc.chebint(e))
        assert abs(op.w @ npc.chebval(op.y, e) - exact) < 1e-14 * max(1, N / 16)
