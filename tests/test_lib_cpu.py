"""Host-side checks of the HIP library that need no GPU: the shared object
loads, exports every function declared in include/pcs.h, and its host logic
(workspace sizing, argument validation) behaves as documented."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2606_09468_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(P.LIBPATH):
        from paper_2606_09468_amd import build
        build.build()
    return P.lib()


def test_exports_match_header(L):
    hdr = open(os.path.join(ROOT, "include", "pcs.h")).read()
    declared = set(re.findall(r"^\s*(?:pcs_status|const char\*)\s+(pcs_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations found"
    assert declared == set(P.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_workspace_bytes_and_validation(L):
    g = P.make_grid(2, 256, 257)
    p = P.make_params(wi=50.0, dt=5e-4)
    n = P.pcs_workspace_bytes(g, p)
    assert 10e6 < n < 100e6
    g3 = P.make_grid(3, 256, 257, 128)
    n3 = P.pcs_workspace_bytes(g3, p)
    assert 1e9 < n3 < 40e9      # resident on one 288 GB device
    sz = ctypes.c_size_t(0)
    bad = [P.make_grid(2, 30, 33), P.make_grid(2, 16, 32), P.make_grid(2, 16, 7), P.make_grid(3, 16, 17, 10),
           P.make_grid(3, 16, 17, 1024)]
    # 3*30/2 = 45 (radix 5), even Ny, Ny < 9, 3*10/2 = 15, FP64 z columns of 1536 beyond one workgroup's LDS
    # (even 8 columns: 209 KB)
    for gb in bad:
        st = L.pcs_workspace_bytes(ctypes.byref(gb), ctypes.byref(p), ctypes.byref(sz))
        assert st == P.PCS_ERR_UNSUPPORTED, (gb.nx, gb.ny, gb.nz)
    # the same z size fits in FP32 (mixed precision: 8 columns, 98 KB), and FP64 columns of 576 fit
    assert P.pcs_workspace_bytes(P.make_grid(3, 16, 17, 1024), P.make_params(precision=1)) > 0
    assert P.pcs_workspace_bytes(P.make_grid(3, 16, 17, 384), p) > 0
    pb = P.make_params(wi=-1.0)
    assert L.pcs_workspace_bytes(ctypes.byref(g), ctypes.byref(pb), ctypes.byref(sz)) == P.PCS_ERR_ARG
    assert L.pcs_workspace_bytes(None, ctypes.byref(p), ctypes.byref(sz)) == P.PCS_ERR_ARG
    assert L.pcs_step(None, 1) == P.PCS_ERR_ARG
    assert L.pcs_status_string(P.PCS_ERR_STATE).decode().startswith("run has blown up")


def test_init_rejects_bad_workspace(L):
    g = P.make_grid(2, 16, 17)
    p = P.make_params()
    h = ctypes.c_void_p(0)
    # too small: rejected before any device call
    st = L.pcs_init(ctypes.byref(g), ctypes.byref(p), 1, 1e-3, ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert st == P.PCS_ERR_WORKSPACE and not h.value
    st = L.pcs_init(ctypes.byref(g), ctypes.byref(p), 1, 1e-3, None, 1 << 30, None, ctypes.byref(h))
    assert st == P.PCS_ERR_ARG


def test_ensemble_workspace_and_validation():
    """Ensemble sizing needs no GPU: it covers every member (at least the
    sum of the single-run workspaces) and rejects mixed dimensions or
    precisions and empty ensembles."""
    import paper_2606_09468_amd as P
    from paper_2606_09468_amd.workloads import ensemble_members
    members = ensemble_members(count=5, seed=4, ny_choices=(17, 25, 33), nx_choices=(12, 16, 24))
    grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
    params = [P.make_params(wi=wi, dt=5e-4) for _, _, wi, _ in members]
    total = P.pcs_ensemble_workspace_bytes(grids, params)
    singles = [P.pcs_workspace_bytes(g, p) for g, p in zip(grids, params)]
    # every member's buffers are there; only the per-launch tables are shared
    assert 0.95 * sum(singles) <= total <= sum(singles)
    assert P.pcs_ensemble_workspace_bytes(grids[:-1], params[:-1]) < total
    with pytest.raises(P.PcsError) as e:
        P.pcs_ensemble_workspace_bytes([P.make_grid(2, 16, 17), P.make_grid(3, 16, 17, 16)], [P.make_params()] * 2)
    assert e.value.status == P.PCS_ERR_UNSUPPORTED
    with pytest.raises(P.PcsError) as e:
        P.pcs_ensemble_workspace_bytes([P.make_grid(2, 16, 17)] * 2,
                                       [P.make_params(), P.make_params(precision=1)])
    assert e.value.status == P.PCS_ERR_UNSUPPORTED
    with pytest.raises(P.PcsError) as e:
        P.pcs_ensemble_workspace_bytes([], [])
    assert e.value.status == P.PCS_ERR_ARG


def test_ensemble_draw_recipe():
    """The uneven-size ensemble draw: sizes from the stated lists, Wi in
    [20, 100], member seeds 4000 + r, reproducible."""
    from paper_2606_09468_amd.workloads import ENSEMBLE_NX, ENSEMBLE_NY, ensemble_members
    a = ensemble_members()
    assert a == ensemble_members() and len(a) == 64
    assert all(ny in ENSEMBLE_NY and nx in ENSEMBLE_NX and 20 <= wi <= 100 and s == 4000 + r
               for r, (ny, nx, wi, s) in enumerate(a))
    assert len({(ny, nx) for ny, nx, _, _ in a}) > 10   # genuinely uneven


@pytest.mark.parametrize("a,b", [
    ((2, 12, 17, 1), (2, 20, 33, 1)),
    ((2, 20, 33, 1), (2, 12, 17, 1)),
    ((3, 8, 13, 8), (3, 12, 21, 16)),
    ((3, 12, 21, 16), (3, 8, 13, 8)),
    ((3, 16, 17, 12), (3, 8, 25, 20)),
])
def test_resample_state_matches_oracle(L, a, b):
    """pcs_resample_state (host code of the library) against the oracle's
    resampling on random states, refining and coarsening each direction."""
    from oracle import Grid
    from oracle.resample import resample_state
    from tests.inputs import random_state
    ga, gb = Grid(*a), Grid(*b)
    s = random_state(a[0], a[1], a[2], a[3], seed=21, amp=1.0)
    s[:4] = [17.0, 0.017, 2.5, 0.0]
    want = resample_state(ga, s, gb)
    got = P.resample_state(P.make_grid(*a), s, P.make_grid(*b))
    assert got.size == want.size == P.state_size(P.make_grid(*b))
    assert np.array_equal(got[:4], want[:4])
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_resample_state_rejects_bad_arguments(L):
    g, s = P.make_grid(2, 8, 9), np.zeros(P.state_size(P.make_grid(2, 8, 9)))
    for dst in (P.make_grid(2, 8, 9, lx=5.0), P.make_grid(3, 8, 9, 8), P.make_grid(2, 7, 9), P.make_grid(2, 8, 10)):
        with pytest.raises(P.PcsError):
            P.resample_state(g, s, dst)
    with pytest.raises(P.PcsError):
        P.resample_state(g, s[:-1], P.make_grid(2, 8, 9))
