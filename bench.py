#!/usr/bin/env python3
"""Throughput of the polymer channel-flow step on one MI355X.

Workload (default): the largest single-GPU workload, a 3D channel, Oldroyd-B,
Lx = 10, Lz = 5, Nx = 256, Ny = 257 Chebyshev points, Nz = 128, Re = 0.01,
Wi = 100, beta = 0.8, kappa = 5e-5, constant flux, CNAB2 with dt = 2.5e-4;
laminar state plus the seeded perturbation (seed 5, amplitude 1e-3), all
state resident in HBM.  A step is one full time step (explicit products,
solves and the per-step diagnostics), replayed from HIP graphs.  The mixed
precision step is the headline value, the FP64 step is timed beside it.

The FP64 oracle is timed on one host thread in a child process started
before anything touches the GPU (it runs while the GPU is timed): one
warm-up step, then the timed sample; the GPU runs of both precisions are
then compared with the oracle's state after those steps.  Prints one JSON
line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time steps/s and grid-point-updates/s, mixed vs FP64 at stated error, 1 GPU"
HBM_PEAK_GBS = 8000.0
# names of the precision settings (pcs_params.precision)
PNAME = {0: "fp64", 1: "mixed", 2: "mixed64y", 3: "mixedcomp", 4: "auto"}
PDESC = {0: "fp64", 1: "mixed", 2: "mixed, FP64 y-transforms", 3: "mixed, error-compensated FP32 y-transforms",
         4: "mixed, each y-transform table the fastest variant within the error budget"}
MFMA_F64_TFS = 78.6
MFMA_F32_TFS = 157.3

from paper_2606_09468_amd.workloads import ENSEMBLE, WORKLOADS, ensemble_members  # noqa: E402


def stage_work(w, precision, split, yvar=None):
    """Algorithmic work of one launch of each stage kernel at this workload:
    {stage: (bound, amount, peak)}.  Products: ('mfma', flops summed over
    the table, peak of the compute precision), each wall-normal product in its
    parity form: an m x k centro(anti)symmetric operator on n columns costs
    2 ceil(m/2) k n (the even and odd halves), the eigenbasis products
    2 (ne^2 + no^2) n with ne, no the even and odd eigenvector counts.  Transform and elementwise
    kernels: ('hbm', bytes), every input field read once and every output
    written once, complex values of the kernel's precision (FP32 in the mixed
    transforms, FP64 elsewhere); small per-mode tables are not counted.
    split: the products of the state run as three launches (mean profiles,
    padded grid, D2 / D) rather than one.  yvar: the wall-normal product
    variants in use (1 FP32, 2 FP64 operators, 3 compensated FP32; for the
    state products and the projections), by default those of the precision."""
    dim, nx, ny, nz = w["dim"], w["nx"], w["ny"], w["nz"]
    N = ny - 1
    n1, m1, ni = N + 1, 3 * N // 2 + 1, N - 1
    nkx = nx // 2
    nzs = 1 if dim == 2 else nz
    pz = 1 if dim == 2 else 3 * nz // 2
    nm = nkx * nzs
    cw = 2 * nm
    nc = 3 if dim == 2 else 6
    nsv = 1 if dim == 2 else 2
    nsolve = nsv + nc
    nout = 5 if dim == 2 else 9
    nyin = 9 if dim == 2 else 17
    nh = 1 + (dim - 2) + nc
    mixed = precision != 0
    if yvar is None:
        yvar = [precision, precision]
    f32_state = yvar[0] in (1, 3)         # the state -> padded-grid products in FP32 (3: compensated)
    f32_proj = yvar[1] in (1, 3)
    tb = 8 if mixed else 16               # bytes per complex value in the transforms
    pk = lambda f32: MFMA_F32_TFS if f32 else MFMA_F64_TFS
    out = {}
    nderiv = 1 if dim == 2 else 2

    def mixed_table(parts):
        """One launch holding FP32 and FP64 products: the peak is the rate at
        which this flop mix would run if every product ran at its own peak."""
        flops = sum(f for f, _ in parts)
        ideal = sum(f / (p * 1e12) for f, p in parts)
        return ("mfma", flops, flops / ideal / 1e12)
    half = lambda r: (r + 1) // 2
    ne, no = half(ni), ni // 2
    eig = 2 * (ne * ne + no * no) * cw      # one product in the eigenbasis (either direction)
    padded = ((dim + nc + nderiv + nc) * 2 * half(m1) * cw * n1, pk(f32_state))                    # to the padded grid
    d2 = ((nsolve + nc) * 2 * half(n1) * cw * n1 + (dim - 1) * 2 * half(n1) * n1, MFMA_F64_TFS)   # D2, D of the state
    mean = ((2 * (dim - 1) + 2 * nc) * 2 * half(m1) * n1, MFMA_F64_TFS)                         # mean profiles (mixed)
    proj = [((nout + dim - 1) * 2 * half(n1) * cw * m1, pk(f32_proj))]                           # P N, (D P) N
    if mixed:
        proj.append((nout * 2 * half(n1) * m1, MFMA_F64_TFS))                              # mean column
    if split:
        # three launches: mean profiles, padded-grid products, D2 / D of the state
        out["gemm_state"] = mixed_table([padded])
        out["gemm_d2"] = mixed_table([d2])
        if mixed:
            out["gemm_mean"] = mixed_table([mean])
    else:
        out["gemm_state"] = mixed_table([padded, d2] + ([mean] if mixed else []))
    if dim == 3:
        out["zfft_inv"] = ("hbm", (nyin * m1 * nzs * nkx + 26 * m1 * pz * nkx) * tb, HBM_PEAK_GBS)
        out["xpencil"] = ("hbm", (26 + nout) * m1 * pz * nkx * tb, HBM_PEAK_GBS)
        out["zfft_fwd"] = ("hbm", (nout * m1 * pz * nkx + nout * m1 * nzs * nkx) * tb, HBM_PEAK_GBS)
        out["diag_zfft"] = ("hbm", (4 * n1 * nzs * nkx + 4 * n1 * nz * nkx) * 16, HBM_PEAK_GBS)
    else:
        out["xpencil"] = ("hbm", (nyin + nout) * m1 * nkx * tb, HBM_PEAK_GBS)
    out["gemm_proj"] = mixed_table(proj)
    out["gemm_vinv"] = ("mfma", nsolve * eig, MFMA_F64_TFS)
    out["gemm_v"] = ("mfma", (2 + (dim - 2) + nc) * eig + 2 * half(n1) * cw * ni + 2 * 2 * ni, MFMA_F64_TFS)
    fld = n1 * nm * 16                     # one FP64 spectral field
    rhs_in = (nsv + nc) + nh + nsolve + nc + nout + (dim - 1)
    rhs_out = nsolve + (dim - 1)
    out["rhs"] = ("hbm", (rhs_in + rhs_out) * fld, HBM_PEAK_GBS)
    fin_in = 3 + (dim - 1) + nc + 3 + nc + (dim - 2)
    fin_out = (2 + 1 + 2 * (dim - 2)) + nh + (3 if dim == 2 else 4)
    out["finalize"] = ("hbm", (fin_in + fin_out) * fld, HBM_PEAK_GBS)
    out["diag_rows"] = ("hbm", (3 if dim == 2 else 4) * n1 * (nz if dim == 3 else 1) * nkx * 16, HBM_PEAK_GBS)
    return out


def ensemble_work(ws, precision, split, yvar=None):
    """stage_work summed over the members of an ensemble (every stage is one
    launch over all of them): bytes and flops add; the peak of a product
    stage is that of its whole flop mix (total flops over the summed time
    each member's flops would take at its own mix's peak)."""
    out = {}
    for w in ws:
        for k, (bound, amount, peak) in stage_work(w, precision, split, yvar).items():
            b, a, t = out.get(k, (bound, 0.0, 0.0))
            out[k] = (bound, a + amount, t + amount / peak)
    return {k: (b, a, a / t if t > 0 else 0.0) for k, (b, a, t) in out.items()}


def roofline_table(stages, work):
    """Per-kernel roofline from the measured per-launch durations."""
    table = {}
    for k, ms in stages.items():
        if k not in work or ms <= 0:
            continue
        bound, amount, peak = work[k]
        t = ms * 1e-3
        if bound == "hbm":
            ach, unit = amount / t / 1e9, "GB/s"
        else:
            ach, unit = amount / t / 1e12, "TFLOP/s"
        table[k] = dict(bound=bound, achieved=ach, peak=peak, unit=unit, frac=ach / peak, avg_ms=ms,
                        **({"algorithmic_bytes": amount} if bound == "hbm" else {"algorithmic_flops": amount}))
    return table


def traffic_for(kernel, workload, precision):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload, if the transform sources have not changed since (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    src = open(os.path.join(ROOT, "paper_2606_09468_amd", "csrc", "fft.hip"), "rb").read() + \
        open(os.path.join(ROOT, "paper_2606_09468_amd", "csrc", "gemm.hip"), "rb").read() + \
        open(os.path.join(ROOT, "paper_2606_09468_amd", "csrc", "elem.hip"), "rb").read()
    digest = hashlib.sha256(src).hexdigest()[:16]
    for line in open(path):
        parts = [x.strip() for x in line.strip().strip("|").split("|")]
        pname = PNAME.get(precision, str(precision))
        if len(parts) >= 6 and parts[0] == kernel and parts[1] == workload and parts[2] == pname:
            if parts[5] != digest:
                return None
            return float(parts[3]) + float(parts[4])
    return None


# timed oracle steps after the warm-up step, per workload (one C5 oracle step
# is about 30 s on one host thread)
CPU_STEPS = {"c1": 60, "c2": 60, "c3": 4, "c5": 1}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_job(workload, sample_steps, scheme, out):
    """Child process: the FP64 oracle of the workload on one host thread
    (BLAS limited to one thread; numpy.fft is single-threaded), one warm-up
    step (it builds the per-wavenumber LU factors) then sample_steps timed
    steps; writes the state, the last record and the timings to out."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import Grid, Oracle, Params
    w = WORKLOADS[workload]
    g = Grid(w["dim"], w["nx"], w["ny"], w["nz"], 10.0, w["lz"])
    prm = Params(wi=w["wi"], dt=w["dt"], scheme=scheme)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = Oracle(g, prm, seed=w["seed"], amp=1e-3)
        t1 = time.perf_counter()
        print("bench oracle: set up in %.1f s" % (t1 - t0), file=sys.stderr, flush=True)
        o.step(1)
        t2 = time.perf_counter()
        print("bench oracle: warm-up step in %.1f s" % (t2 - t1), file=sys.stderr, flush=True)
        for k in range(sample_steps):
            o.step(1)
            print("bench oracle: timed step %d of %d done" % (k + 1, sample_steps), file=sys.stderr, flush=True)
        t3 = time.perf_counter()
    np.savez(out, state=o.get_state(), diag=json.dumps(o.diag[-1]),
             times=np.array([t1 - t0, t2 - t1, t3 - t2]), steps=sample_steps)


def start_oracle(workload, sample_steps, scheme):
    """Starts oracle_job in a child interpreter (before this process uses the
    GPU; it reports its progress on the shared stderr); returns (process,
    output path)."""
    import subprocess
    import tempfile
    fd, out = tempfile.mkstemp(suffix=".npz", prefix="pcs_oracle_")
    os.close(fd)
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-job", workload, str(sample_steps), str(scheme), out]
    proc = subprocess.Popen(cmd, stdout=subprocess.DEVNULL)
    return proc, out


def finish_oracle(job, sample_steps):
    """Waits for the oracle child; returns (state, last record, cpu_baseline)."""
    import numpy as np
    proc, out = job
    rc = proc.wait()
    if rc != 0:
        raise RuntimeError("oracle child failed with status %d (its messages are on stderr)" % rc)
    z = np.load(out)
    setup, warm, timed = (float(x) for x in z["times"])
    state, diag = z["state"].copy(), json.loads(str(z["diag"]))
    try:
        os.remove(out)
    except OSError:
        pass
    cb = dict(value=sample_steps / timed, unit="steps/s", cores=1, kind="oracle",
              cpu_model=cpu_model(), host_threads=os.cpu_count(),
              sample="%d FP64 oracle step(s) of the same workload on one host thread (BLAS limited to one thread, "
                     "single-threaded numpy.fft), timed after one warm-up step (%.1f s) and setup (%.1f s), in a "
                     "child process running beside the GPU timing" % (sample_steps, warm, setup))
    return state, diag, cb


def state_errors(a, b, w):
    import numpy as np

    from oracle import Grid, state_layout
    g = Grid(w["dim"], w["nx"], w["ny"], w["nz"], 10.0, w["lz"])
    hdr, names, per = state_layout(g)
    errs, o = {}, hdr
    for n in names:
        x, y = a[o:o + 2 * per], b[o:o + 2 * per]
        sc = np.abs(y).max()
        errs[n] = float(np.abs(x - y).max() / sc) if sc > 0 else float(np.abs(x).max())
        o += 2 * per
    return errs


def main():
    if len(sys.argv) == 6 and sys.argv[1] == "--oracle-job":
        oracle_job(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), sys.argv[5])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS) + ["c4"],
                    help="c5 (default): 3D 256x257x128, the largest single-GPU workload; "
                         "c4: the 64-member uneven 2D ensemble, one graph launch per step")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed", "mixed64y", "mixedcomp", "auto"],
                    help="both: time mixed (value) and FP64 (reported beside it); mixed64y: FP64 wall-normal "
                         "transforms; mixedcomp: error-compensated FP32 wall-normal transforms")
    ap.add_argument("--stage-steps", type=int, default=10)
    ap.add_argument("--stage-reps", type=int, default=1,
                    help="launches of each stage per profiled step (1: every kernel runs once per step, on the "
                         "inputs the previous stage just wrote, as inside a step)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="timed oracle steps after the warm-up step (default per workload: %s)" % CPU_STEPS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a plain copy kernel of known traffic, the "
                         "reference for HBM counter runs)")
    ap.add_argument("--midplane-bins", type=int, default=0, metavar="N",
                    help="accumulate the on-device midplane Tr c histogram (N bins over [0, 6)) during the timed "
                         "steps; its counts are checked and reported")
    ap.add_argument("--scheme", default="cnab2", choices=["cnab2", "sbdf4"],
                    help="time scheme: CNAB2 (the workloads' scheme) or the paper's SBDF4")
    args = ap.parse_args()
    args.scheme_id = 1 if args.scheme == "sbdf4" else 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (each run, or each ensemble "
              "member, would be sharded across GPUs without communication); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.cpu_steps is None:
        args.cpu_steps = CPU_STEPS.get(args.workload, 1)
    # the oracle child starts before this process touches the GPU
    job = None
    if not args.no_cpu_baseline and args.workload != "c4":
        job = start_oracle(args.workload, args.cpu_steps, args.scheme_id)
        print("bench: oracle child started (1 warm-up + %d timed steps)" % args.cpu_steps, file=sys.stderr,
              flush=True)
    # tile choices of the product tables from the committed tuning file (new
    # table shapes are timed and appended), so that the timed kernels are the
    # ones the committed profiles describe
    os.environ.setdefault("PCS_TUNE_CACHE", os.path.join(ROOT, "paper_2606_09468_amd", "tune_gfx950.txt"))
    import numpy as np
    import torch

    import paper_2606_09468_amd as P
    if not os.path.exists(P.LIBPATH):
        from paper_2606_09468_amd import build
        build.build()
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "c4":
        return bench_ensemble(args, P)
    w = WORKLOADS[args.workload]
    grid = P.make_grid(w["dim"], w["nx"], w["ny"], w["nz"], 10.0, w["lz"])
    precs = {"both": [1, 0], "fp64": [0], "mixed": [1], "mixed64y": [2], "mixedcomp": [3], "auto": [4]}[args.precision]
    timed = {}
    for prec in precs:
        prm = P.make_params(wi=w["wi"], dt=w["dt"], precision=prec, scheme=args.scheme_id)
        sim = P.Sim(grid, prm, seed=w["seed"], amp=1e-3)
        print("bench: %s precision %d, warmup %d" % (args.workload, prec, args.warmup), file=sys.stderr, flush=True)
        sim.step(args.warmup)
        sim.diagnostics()
        if args.midplane_bins > 0:
            sim.midplane_histogram_setup(0.0, 6.0, args.midplane_bins)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        ev0.record(sim.stream)
        sim.step(args.steps)
        ev1.record(sim.stream)
        ev1.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms = ev0.elapsed_time(ev1)
        recs, st = sim.diagnostics()
        assert st == P.PCS_OK and len(recs) == min(args.steps, 4096) and recs[-1]["blowup"] == 0
        hist = None
        if args.midplane_bins > 0:
            counts = sim.midplane_histogram()
            assert int(counts.sum()) == args.steps * w["nx"] * (w["nz"] if w["dim"] == 3 else 1)
            hist = dict(bins=args.midplane_bins, lo=0.0, hi=6.0, samples=int(counts.sum()),
                        below_lo=int(counts[0]), at_or_above_hi=int(counts[-1]))
        print("bench: timed %d steps in %.3f ms (wall %.3f s)" % (args.steps, ms, wall), file=sys.stderr, flush=True)
        # per-stage durations (eager launches, HIP events on the run's stream)
        stages = sim.stage_times(args.stage_steps, reps=args.stage_reps)
        ych = sim.y_choice()
        sim.close()
        timed[prec] = dict(ms=ms, sps=args.steps / (ms / 1e3), stages=stages, prm=prm, hist=hist, ych=ych)
    head = precs[0]
    ms, sps, stages, prm = timed[head]["ms"], timed[head]["sps"], timed[head]["stages"], timed[head]["prm"]
    split = stages.get("gemm_d2", 0.0) > 0.0
    table = roofline_table(stages, stage_work(w, head, split, timed[head]["ych"]["variant"]))
    dom = max(table, key=lambda k: table[k]["avg_ms"])
    roof = dict(kernel=dom, **table[dom])
    roof["traffic"] = traffic_for(dom, args.workload, head)
    points = w["nx"] * w["ny"] * w["nz"]
    line = {
        "metric": METRIC, "value": sps, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if head == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": w["desc"] if args.scheme_id == 0 else w["desc"].replace("CNAB2", "SBDF4"),
                   "grid": [w["nx"], w["ny"], w["nz"]],
                   "precision": PDESC[head],
                   "parallelism": "single GPU"},
        "grid_point_updates_per_s": sps * points,
        "roofline": roof,
        "stage_ms": stages,
        "stage_roofline": {k: {"frac": round(v["frac"], 4), "achieved": round(v["achieved"], 2),
                               "unit": v["unit"], "avg_ms": round(v["avg_ms"], 5)} for k, v in table.items()},
    }
    if len(precs) > 1:
        line["fp64"] = {"value": timed[0]["sps"], "ms_per_step": timed[0]["ms"] / args.steps,
                        "grid_point_updates_per_s": timed[0]["sps"] * points}
        line["speedup_mixed_vs_fp64"] = timed[1]["sps"] / timed[0]["sps"]
    if job is not None:
        # the GPU state of each timed precision after the oracle's steps
        gstates = {}
        for prec in precs:
            sim2 = P.Sim(grid, timed[prec]["prm"], seed=w["seed"], amp=1e-3)
            sim2.step(args.cpu_steps + 1)
            recs2, _ = sim2.diagnostics()
            gstates[prec] = (sim2.get_state(), recs2[-1])
            sim2.close()
        print("bench: waiting for the oracle child", file=sys.stderr, flush=True)
        ostate, odiag, cb = finish_oracle(job, args.cpu_steps)
        line["cpu_baseline"] = cb
        # error of each timed precision against the oracle over the same sample
        line["error_vs_oracle"] = {}
        for prec in precs:
            a, d = gstates[prec]
            errs = state_errors(a, ostate, w)
            e = odiag
            line["error_vs_oracle"][PNAME[prec]] = {
                "steps": args.cpu_steps + 1,
                "max_rel_velocity": max(errs[k] for k in errs if k in ("u", "v", "w", "phi", "g")),
                "max_rel_conformation": max(errs[k] for k in errs if k.startswith("c")),
                "min_trc_abs": abs(d["min_trc"] - e["min_trc"]),
                "counts_equal": all(d[k] == e[k] for k in ("n_lt3", "n_lt0", "mid_n_lt3", "mid_n_lt0")),
            }
    if head == 4:
        line["y_choice"] = timed[head]["ych"]
    if timed[head]["hist"] is not None:
        line["midplane_histogram"] = timed[head]["hist"]
    print(json.dumps(line), flush=True)


def ensemble_cpu_baseline(members, dt, steps=2, scheme=0):
    """Oracle seconds per ensemble step: each distinct member size is timed
    over `steps` steps after one warm-up step, and the members are summed."""
    from threadpoolctl import threadpool_info

    from oracle import Grid, Oracle, Params
    per = {}
    t_all = time.perf_counter()
    for ny, nx, wi, seed in members:
        if (ny, nx) in per:
            continue
        o = Oracle(Grid(2, nx, ny), Params(wi=wi, dt=dt, scheme=scheme), seed=seed, amp=1e-3)
        o.step(1)
        t0 = time.perf_counter()
        o.step(steps)
        per[(ny, nx)] = (time.perf_counter() - t0) / steps
    total = sum(per[(ny, nx)] for ny, nx, _, _ in members)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return dict(value=1.0 / total, unit="steps/s", cores=threads, kind="oracle",
                sample="each of the %d distinct member sizes timed over %d oracle steps after a warm-up step "
                       "(%.1f s in all), summed over the %d members" % (len(per), steps,
                                                                        time.perf_counter() - t_all, len(members)))


def bench_ensemble(args, P):
    """The uneven 64-member ensemble: steps/s of the whole ensemble (every
    member advanced one step per graph launch) and summed point updates."""
    import torch
    members = ensemble_members(ENSEMBLE["count"], ENSEMBLE["seed"])
    prec = {"both": 1, "fp64": 0, "mixed": 1, "mixed64y": 2, "mixedcomp": 3, "auto": 4}[args.precision]
    grids = [P.make_grid(2, nx, ny) for ny, nx, _, _ in members]
    params = [P.make_params(wi=wi, dt=ENSEMBLE["dt"], precision=prec, scheme=args.scheme_id)
              for _, _, wi, _ in members]
    ens = P.Ensemble(grids, params, [s for _, _, _, s in members], amp=1e-3)
    print("bench: ensemble of %d, precision %d, warmup %d" % (len(members), prec, args.warmup),
          file=sys.stderr, flush=True)
    ens.step(args.warmup)
    ens.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(ens.stream)
    ens.step(args.steps)
    ev1.record(ens.stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    for r in range(len(members)):
        recs, st = ens.diagnostics(r)
        assert st == P.PCS_OK and recs[-1]["step"] == args.warmup + args.steps and recs[-1]["blowup"] == 0
    # per-stage durations (eager launches over all members, HIP events on the ensemble's stream)
    stages = ens.stage_times(args.stage_steps, reps=args.stage_reps)
    ych = ens.y_choice()
    ens.close()
    split = stages.get("gemm_d2", 0.0) > 0.0
    work = ensemble_work([dict(dim=2, nx=nx, ny=ny, nz=1) for ny, nx, _, _ in members], prec, split, ych["variant"])
    table = roofline_table(stages, work)
    sps = args.steps / (ms / 1e3)
    points = sum(nx * ny for ny, nx, _, _ in members)
    line = {
        "metric": METRIC, "value": sps, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": ENSEMBLE["desc"] if args.scheme_id == 0 else ENSEMBLE["desc"].replace("CNAB2", "SBDF4"),
                   "members": len(members), "base_points": points,
                   "precision": PDESC[prec],
                   "parallelism": "single GPU, one graph launch per ensemble step"},
        "grid_point_updates_per_s": sps * points,
        "roofline": None,
        "stage_ms": stages,
        "stage_roofline": {k: {"frac": round(v["frac"], 4), "achieved": round(v["achieved"], 2),
                               "unit": v["unit"], "avg_ms": round(v["avg_ms"], 5)} for k, v in table.items()},
    }
    if table:
        dom = max(table, key=lambda k: table[k]["avg_ms"])
        line["roofline"] = dict(kernel=dom, **table[dom], traffic=None)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = ensemble_cpu_baseline(members, ENSEMBLE["dt"], scheme=args.scheme_id)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
