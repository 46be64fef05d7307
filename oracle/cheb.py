"""Chebyshev Gauss-Lobatto grid and wall-normal operators of the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper expands the wall-normal direction in Chebyshev polynomials and
dealiases fully (Section 2, numerics paragraph).  The oracle uses collocation
on Gauss-Lobatto points, with N = Ny - 1:

    y_j  = cos(pi j / N),  j = 0..N          (y_0 = +1, y_N = -1, y_{N/2} = 0)
    f(y) = sum_{n=0..N} a_n T_n(y)            (interpolant through f_j)
    a_n  = 2/(N cb_n) sum_j f_j T_n(y_j) / cb_j,   cb_0 = cb_N = 2, else 1

Operators (all plain definitions, no fast transforms):
    C_N       values -> coefficients (the formula above)
    D_N       derivative of the interpolant at y_j        = E'_N C_N
    D2        second derivative                          = D_N D_N
    I_MN      interpolant evaluated on the padded grid     = E_M C_N
    D_MN      its derivative on the padded grid            = E'_M C_N
    P_NM      padded values -> coefficients (C_M), keep degrees 0..N,
              evaluate on y_j                               = E_N C_M[0..N]
    w         Clenshaw-Curtis weights: w_j = sum_n (int_{-1}^{1} T_n) C_N[n, j]
with M = 3N/2 padded intervals, E_K[i, n] = T_n(cos(pi i / K)) and
E'_K[i, n] = T'_n(cos(pi i / K)).

Every matrix is formed in 80-bit extended precision from trigonometric values
computed by mpmath at 40 significant digits, and rounded once to float64.
"""

from functools import lru_cache
from types import SimpleNamespace

import mpmath
import numpy as np

LD = np.longdouble


def _to_ld(x):
    """mpmath number -> long double (hi + lo double split keeps 106 bits)."""
    hi = float(x)
    lo = float(x - mpmath.mpf(hi))
    return LD(hi) + LD(lo)


@lru_cache(maxsize=None)
def _trig(K):
    """cos(pi k / K) and sin(pi k / K) for k = 0..2K-1, in long double."""
    with mpmath.workdps(40):
        c = np.array([_to_ld(mpmath.cospi(mpmath.mpf(k) / K)) for k in range(2 * K)], dtype=LD)
        s = np.array([_to_ld(mpmath.sinpi(mpmath.mpf(k) / K)) for k in range(2 * K)], dtype=LD)
    return c, s


def cheb_eval(K, nmax):
    """E[i, n] = T_n(cos(pi i / K)) = cos(pi n i / K); i = 0..K, n = 0..nmax."""
    c, _ = _trig(K)
    i = np.arange(K + 1)[:, None]
    n = np.arange(nmax + 1)[None, :]
    return c[(i * n) % (2 * K)]


def cheb_eval_deriv(K, nmax):
    """E'[i, n] = T'_n(cos(theta_i)), theta_i = pi i / K.

    T'_n(cos t) = n sin(n t) / sin(t) inside; n^2 at y = +1 and
    (-1)^(n+1) n^2 at y = -1.
    """
    c, s = _trig(K)
    n_int = np.arange(nmax + 1)
    n = n_int.astype(LD)
    E = np.empty((K + 1, nmax + 1), dtype=LD)
    for i in range(1, K):
        E[i] = n * s[(i * n_int) % (2 * K)] / s[i]
    E[0] = n * n
    E[K] = np.where(n_int % 2 == 1, LD(1), LD(-1)) * n * n
    return E


def cheb_coef(N):
    """C_N[n, j] = 2/(N cb_n cb_j) T_n(y_j): Lobatto values -> Chebyshev coefficients."""
    c, _ = _trig(N)
    cb = np.ones(N + 1, dtype=LD)
    cb[0] = cb[N] = 2
    n = np.arange(N + 1)[:, None]
    j = np.arange(N + 1)[None, :]
    return (LD(2) / (LD(N) * cb[:, None] * cb[None, :])) * c[(n * j) % (2 * N)]


@lru_cache(maxsize=None)
def operators(N):
    """All wall-normal operators for N = Ny - 1 (even), rounded to float64."""
    if N < 2 or N % 2:
        raise ValueError("N = Ny - 1 must be even and >= 2")
    M = 3 * N // 2
    C_N = cheb_coef(N)
    C_M = cheb_coef(M)
    D_N = cheb_eval_deriv(N, N) @ C_N
    ops = SimpleNamespace()
    ops.N, ops.M = N, M
    ops.y = cheb_eval(N, 1)[:, 1].astype(np.float64)
    ops.ypad = cheb_eval(M, 1)[:, 1].astype(np.float64)
    ops.D = D_N.astype(np.float64)
    ops.D2 = (D_N @ D_N).astype(np.float64)
    ops.I_MN = (cheb_eval(M, N) @ C_N).astype(np.float64)
    ops.D_MN = (cheb_eval_deriv(M, N) @ C_N).astype(np.float64)
    ops.P_NM = (cheb_eval(N, N) @ C_M[: N + 1, :]).astype(np.float64)
    # int_{-1}^{1} T_n dy = 2/(1 - n^2) for even n, 0 for odd n
    n = np.arange(N + 1)
    integ = np.zeros(N + 1, dtype=LD)
    ev = n[n % 2 == 0]
    integ[ev] = LD(2) / (LD(1) - ev.astype(LD) ** 2)
    ops.w = (integ @ C_N).astype(np.float64)
    ops.C_N = C_N.astype(np.float64)
    return ops


def cheb_poly_values(nmax, y):
    """T_n(y), T'_n(y), T''_n(y) for n = 0..nmax by the three-term recurrence
    T_{n+1} = 2y T_n - T_{n-1} (and its first two derivatives); float64."""
    y = np.asarray(y, dtype=np.float64)
    T = np.zeros((nmax + 1,) + y.shape)
    T1 = np.zeros_like(T)
    T2 = np.zeros_like(T)
    T[0] = 1.0
    if nmax >= 1:
        T[1] = y
        T1[1] = 1.0
    for n in range(1, nmax):
        T[n + 1] = 2 * y * T[n] - T[n - 1]
        T1[n + 1] = 2 * T[n] + 2 * y * T1[n] - T1[n - 1]
        T2[n + 1] = 4 * T1[n] + 2 * y * T2[n] - T2[n - 1]
    return T, T1, T2
