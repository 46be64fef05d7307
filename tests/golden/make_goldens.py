"""Writes the sampled oracle goldens of the two large 3D workloads (run from
the repository root: python tests/golden/make_goldens.py [c3|c5]).

Calls only the oracle (oracle/): the FP64 reference of the step, run on the
CPU from the seeded initial condition, stored at a seeded sample of Fourier
columns (every wall-normal point of every state field at those (kz, kx)
modes), together with each field's largest magnitude over all modes and over
its fluctuation (all modes but kx = kz = 0), every per-step diagnostic
record, and the run's FP64 floor: per field, the difference between the
oracle and the same oracle run on the mirrored state (y -> -y, which reverses
the order of every wall-normal sum and solve), mirrored back.  The GPU parity tests compare the HIP
library's state at the same columns, field by field relative to those
magnitudes, and its records.

  c5: 3D channel 256 x 257 x 128, Lx = 10, Lz = 5, Re = 0.01, Wi = 100,
      beta = 0.8, kappa = 5e-5, CNAB2 dt = 2.5e-4, constant flux, seed 5,
      amplitude 1e-3, 8 steps;
  c3: 3D channel 128 x 129 x 64, Wi = 50, dt = 5e-4, seed 3, 100 steps.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Grid, Oracle, Params  # noqa: E402

# fields odd under the mirror y -> -y (with v -> -v); the mean slot of h_v
# holds the even streamwise forcing profile
ODD = {"v", "phi", "cxy", "cyz", "hv", "Fxy", "Fyz"}


def mirror(q):
    out = {}
    for k, a in q.items():
        m = -a[::-1].copy() if k in ODD else a[::-1].copy()
        if k == "hv":
            m[:, 0, 0] = a[::-1, 0, 0]
        out[k] = m
    return out

CASES = {
    "c5": dict(grid=(3, 256, 257, 128), wi=100.0, dt=2.5e-4, seed=5, steps=8, ncols=40),
    "c3": dict(grid=(3, 128, 129, 64), wi=50.0, dt=5e-4, seed=3, steps=100, ncols=48),
}


def sample_columns(nzs, nkx, ncols, seed):
    """(kz slot, kx) pairs: the mean mode, the modes the perturbation fills
    (|m_z| <= 4, m_x <= 4), then modes drawn from the rest; Nyquist slot
    excluded."""
    low = [(0, 0)] + [(iz % nzs, ix) for ix in range(5) for iz in range(-4, 5)
                      if (iz, ix) != (0, 0) and not (ix == 0 and iz < 0)]
    rng = np.random.default_rng(seed)
    pool = [(iz, ix) for iz in range(nzs) for ix in range(nkx) if iz != nzs // 2 and (iz, ix) not in low]
    pick = rng.choice(len(pool), size=ncols - min(ncols, 12), replace=False)
    cols = low[:min(ncols, 12)] + [pool[i] for i in sorted(pick)]
    return np.array(cols, dtype=np.int64)


def make(name):
    c = CASES[name]
    dim, nx, ny, nz = c["grid"]
    g = Grid(dim, nx, ny, nz, 10.0, 5.0)
    t0 = time.time()
    o = Oracle(g, Params(wi=c["wi"], dt=c["dt"]), seed=c["seed"], amp=1e-3)
    for k in range(c["steps"]):
        o.step(1)
        print("%s: step %d of %d (%.0f s)" % (name, k + 1, c["steps"], time.time() - t0), flush=True)
    cols = sample_columns(o.nzs, o.nkx, c["ncols"], seed=c["seed"])
    names = list(o.q.keys())
    vals = np.stack([o.q[n][:, cols[:, 0], cols[:, 1]] for n in names])      # [field][y][col] complex
    scale = np.array([np.abs(o.q[n]).max() for n in names])
    # the FP64 floor of this run: the same oracle on the mirrored state (every
    # wall-normal sum and solve in reverse order), mirrored back
    b = Oracle(Grid(dim, nx, ny, nz, 10.0, 5.0), Params(wi=c["wi"], dt=c["dt"]), seed=c["seed"], amp=1e-3)
    b.q = mirror(b.q)
    for k in range(c["steps"]):
        b.step(1)
        print("%s: mirrored step %d of %d (%.0f s)" % (name, k + 1, c["steps"], time.time() - t0), flush=True)
    back = mirror(b.q)
    floor = np.array([np.abs(back[n] - o.q[n]).max() for n in names]) / scale
    # largest magnitude of each field's fluctuation (every mode but kx = kz = 0)
    fscale = np.array([np.abs(np.where(np.arange(o.nzs)[:, None] * o.nkx + np.arange(o.nkx)[None, :] == 0, 0,
                                       o.q[n])).max() for n in names])
    out = os.path.join(HERE, "%s_oracle_%dsteps.npz" % (name, c["steps"]))
    np.savez_compressed(out, columns=cols, fields=np.array(names), values=vals, scale=scale, fscale=fscale, floor=floor,
                        header=np.array([o.step_count, o.t, o.pi]), records=json.dumps(o.diag),
                        case=json.dumps(c), trc_scale=float(np.abs(o.trace_c()).max()))
    print("wrote", out, os.path.getsize(out), "bytes", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
