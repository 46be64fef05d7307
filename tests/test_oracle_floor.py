"""The FP64 floor behind the parity tolerances: two correct FP64
evaluations of the same discrete step, measured.

Eqs. (1)-(3) and their discretisation are invariant under the mirror
y -> -y (v -> -v): u, w, omega_y, c_xx, c_yy, c_zz, c_xz and their explicit
terms are even, v, phi, c_xy, c_yz and theirs odd (the mean slot of h_v holds
the even streamwise forcing profile).  Running the oracle on the mirrored
state reverses the order of every wall-normal sum and of the LU solves'
rows; mirrored back, its result differs from the direct run only by
roundoff.  That difference, per field relative to the field's largest
magnitude, is the floor a second correct FP64 implementation (such as the
HIP library) can be expected to reach; the GPU tolerances (1e-12 up to
N = 128, 1e-11 at N = 256) must lie above it.
"""

import numpy as np
import pytest

from oracle import Grid, Oracle, Params

ODD = {"v", "phi", "cxy", "cyz", "hv", "Fxy", "Fyz"}


def mirror(q, dim):
    out = {}
    for k, a in q.items():
        m = -a[::-1].copy() if k in ODD else a[::-1].copy()
        if k == "hv":
            m[:, 0, 0] = a[::-1, 0, 0]   # the streamwise forcing profile is even
        out[k] = m
    return out


def floor(dims, prm, nsteps, seed=1):
    g = Grid(*dims)
    a = Oracle(g, Params(**prm), seed=seed, amp=1e-3)
    b = Oracle(Grid(*dims), Params(**prm), seed=seed, amp=1e-3)
    b.q = mirror(b.q, g.dim)
    a.step(nsteps)
    b.step(nsteps)
    back = mirror(b.q, g.dim)
    nq = 6 if g.dim == 2 else 11
    names = list(a.q)
    errs = {k: float(np.abs(back[k] - a.q[k]).max() / np.abs(a.q[k]).max()) for k in names}
    prog = max(errs[k] for k in names[:nq])
    hist = max(errs[k] for k in names[nq:])
    return prog, hist, errs


@pytest.mark.parametrize("dims,prm,nsteps,tol", [
    ((2, 64, 65, 1), dict(wi=20.0, dt=1e-3), 50, 1e-12),
    ((2, 128, 129, 1), dict(wi=50.0, dt=5e-4), 30, 1e-12),
    ((2, 256, 257, 1), dict(wi=50.0, dt=5e-4), 20, 1e-11),
    ((3, 16, 33, 16), dict(wi=20.0, dt=1e-3), 10, 1e-12),
])
def test_fp64_floor_below_the_parity_tolerance(dims, prm, nsteps, tol):
    prog, hist, errs = floor(dims, prm, nsteps)
    N = dims[2] - 1
    worst = max(errs, key=errs.get)
    print("floor %s %d steps: prognostic %.2e, history %.2e (tolerances %.0e / %.1e), largest in %s"
          % (dims, nsteps, prog, hist, tol, 1e-16 * N ** 4, worst), flush=True)
    assert prog > 0.0                      # a genuine second evaluation, not a copy
    assert prog <= tol and hist <= 1e-16 * N ** 4
