"""The right-hand sides in their two launch forms give the same step.

The assembly of eqs. (1)-(2) needs, at every interior row of a Fourier mode,
the new wall values of c of that mode (the kappa-coupling of the implicit
polymer diffusion to the kappa = 0 wall rows, Sec. 2).  In the fused form
each thread computes them itself; in the split form a first launch over the
two wall rows stores them and the interior launch reads them.  Both evaluate
the same expressions in the same order, and within one process the product
tiles are the same, so the states after several steps are bitwise equal,
for CNAB2 and SBDF4, FP64 and mixed precision, with ragged mode counts
(none a multiple of the 64-thread workgroup) and an ensemble of uneven
members.  Which form a launch takes otherwise depends only on its size.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import os

    import torch

    import paper_2606_09468_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(P.LIBPATH):
        from paper_2606_09468_amd import build
        build.build()
    return P


# (dim, nx, ny, nz, precision, scheme)
CASES = [
    (2, 24, 17, 1, 0, 0),
    (2, 16, 25, 1, 1, 0),
    (2, 24, 17, 1, 0, 1),
    (3, 16, 17, 8, 0, 0),
    (3, 24, 33, 12, 1, 0),
    (3, 16, 17, 16, 0, 1),
]


def run(P, monkeypatch, form, dim, nx, ny, nz, precision, scheme, nsteps=6):
    monkeypatch.setenv("PCS_RHS_FORM", form)
    sim = P.Sim(P.make_grid(dim, nx, ny, nz), P.make_params(wi=20.0, dt=1e-3, precision=precision, scheme=scheme),
                seed=7, amp=1e-3)
    sim.step(nsteps)
    st, (dg, _) = sim.get_state(), sim.diagnostics()
    sim.close()
    return st, dg


@pytest.mark.parametrize("dim,nx,ny,nz,precision,scheme", CASES)
def test_split_and_fused_right_hand_sides_agree(P, monkeypatch, dim, nx, ny, nz, precision, scheme):
    case = (dim, nx, ny, nz, precision, scheme)
    print("rhs forms", case, flush=True)
    a, da = run(P, monkeypatch, "fused", *case)
    b, db = run(P, monkeypatch, "split", *case)
    assert np.isfinite(a).all(), case
    assert np.array_equal(a, b), (case, np.abs(a - b).max())
    assert len(da) == len(db) and len(da) > 0
    for ra, rb in zip(da, db):
        assert ra == rb, (case, ra, rb)


def test_split_and_fused_agree_in_an_ensemble(P, monkeypatch):
    members = [(17, 12, 20.0, 3), (25, 16, 40.0, 4), (33, 24, 60.0, 5)]

    def ens_run(form):
        monkeypatch.setenv("PCS_RHS_FORM", form)
        grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
        params = [P.make_params(wi=wi, dt=1e-3, precision=0) for _, _, wi, _ in members]
        ens = P.Ensemble(grids, params, [s for _, _, _, s in members], amp=1e-3)
        ens.step(6)
        out = [ens.get_state(r) for r in range(len(members))]
        ens.close()
        return out

    a, b = ens_run("fused"), ens_run("split")
    for r in range(len(members)):
        assert np.array_equal(a[r], b[r]), (r, np.abs(a[r] - b[r]).max())
