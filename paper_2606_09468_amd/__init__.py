"""Python binding of libpcs: one semi-implicit pseudo-spectral step of
dilute-polymer plane-channel flow on an AMD Instinct MI355X.

Argument marshalling only: every stage of the step runs in the HIP kernels
of libpcs.so; PyTorch provides the device workspace and the HIP stream.
The functions mirror the C ABI in include/pcs.h (same names); ``Sim`` wraps
them for convenience.  Importing works without a GPU; calling anything that
needs the library raises if libpcs.so has not been built, and there is no
fallback path.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libpcs.so")

PCS_OK = 0
PCS_BLOWUP = 1
PCS_ERR_ARG = -1
PCS_ERR_UNSUPPORTED = -2
PCS_ERR_WORKSPACE = -3
PCS_ERR_DEVICE = -4
PCS_ERR_STATE = -5

EXPORTS = ("pcs_workspace_bytes", "pcs_init", "pcs_step", "pcs_diagnostics", "pcs_state_size",
           "pcs_get_state", "pcs_set_state", "pcs_stage_times", "pcs_destroy", "pcs_status_string",
           "pcs_stage_name", "pcs_ensemble_workspace_bytes", "pcs_ensemble_init", "pcs_ensemble_step",
           "pcs_ensemble_diagnostics", "pcs_ensemble_state_size", "pcs_ensemble_get_state",
           "pcs_ensemble_destroy", "pcs_midplane_histogram_setup", "pcs_midplane_histogram",
           "pcs_ensemble_midplane_histogram_setup", "pcs_ensemble_midplane_histogram", "pcs_resample_state",
           "pcs_midplane_pdf_setup", "pcs_midplane_pdf", "pcs_ensemble_midplane_pdf_setup", "pcs_ensemble_midplane_pdf",
           "pcs_init_static", "pcs_ensemble_set_state", "pcs_ensemble_run_status", "pcs_midplane_moments",
           "pcs_ensemble_midplane_moments", "pcs_y_choice", "pcs_ensemble_y_choice", "pcs_ensemble_stage_times")
PCS_NSTAGE = 14
PCS_HIST_MAX = 4096
PCS_STATIC_BYTES = 64 << 20
# midplane PDF quantities (pcs_midplane_pdf_setup)
PCS_PDF_TRC, PCS_PDF_U, PCS_PDF_V, PCS_PDF_W = 0, 1, 2, 3
PCS_PDF_DUDX, PCS_PDF_DUDZ, PCS_PDF_DWDX, PCS_PDF_DWDZ = 4, 5, 6, 7
# wall-normal product variants of the mixed precisions (pcs_y_choice)
PCS_Y_FP32, PCS_Y_FP64, PCS_Y_COMP = 1, 2, 3


class pcs_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("lz", ctypes.c_double)]


class pcs_params(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("wi", ctypes.c_double), ("beta", ctypes.c_double),
                ("kappa", ctypes.c_double), ("eps", ctypes.c_double), ("dt", ctypes.c_double),
                ("forcing", ctypes.c_int32), ("q_or_dpdx", ctypes.c_double), ("precision", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


class pcs_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("min_trc", ctypes.c_double),
                ("mid_min_trc", ctypes.c_double), ("cfl", ctypes.c_double), ("dpdx", ctypes.c_double),
                ("energy", ctypes.c_double), ("mean_trc", ctypes.c_double), ("n_lt3", ctypes.c_uint64),
                ("n_lt0", ctypes.c_uint64), ("mid_n_lt3", ctypes.c_uint64), ("mid_n_lt0", ctypes.c_uint64),
                ("blowup", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pcs_ychoice(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32 * 2), ("budget", ctypes.c_double),
                ("error", (ctypes.c_double * 3) * 2), ("time_us", (ctypes.c_double * 3) * 2)]


_lib = None


def lib():
    """Loads libpcs.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("libpcs.so is not built (run __graft_entry__.build()); no fallback exists")
    L = ctypes.CDLL(LIBPATH)
    vp, sz, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    L.pcs_workspace_bytes.argtypes = [ctypes.POINTER(pcs_grid), ctypes.POINTER(pcs_params), ctypes.POINTER(sz)]
    L.pcs_init.argtypes = [ctypes.POINTER(pcs_grid), ctypes.POINTER(pcs_params), ctypes.c_uint64, ctypes.c_double,
                           vp, sz, vp, ctypes.POINTER(vp)]
    L.pcs_init_static.argtypes = [ctypes.POINTER(pcs_grid), ctypes.POINTER(pcs_params), ctypes.c_uint64,
                                  ctypes.c_double, vp, ctypes.POINTER(vp)]
    L.pcs_step.argtypes = [vp, ctypes.c_int32]
    L.pcs_diagnostics.argtypes = [vp, ctypes.POINTER(pcs_diag), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.pcs_state_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.pcs_get_state.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz]
    L.pcs_set_state.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz]
    L.pcs_stage_times.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.c_int32]
    L.pcs_stage_name.argtypes = [st]
    L.pcs_stage_name.restype = ctypes.c_char_p
    L.pcs_destroy.argtypes = [vp]
    L.pcs_status_string.argtypes = [st]
    L.pcs_status_string.restype = ctypes.c_char_p
    L.pcs_ensemble_workspace_bytes.argtypes = [st, ctypes.POINTER(pcs_grid), ctypes.POINTER(pcs_params),
                                               ctypes.POINTER(sz)]
    L.pcs_ensemble_init.argtypes = [st, ctypes.POINTER(pcs_grid), ctypes.POINTER(pcs_params),
                                    ctypes.POINTER(ctypes.c_uint64), ctypes.c_double, vp, sz, vp, ctypes.POINTER(vp)]
    L.pcs_ensemble_step.argtypes = [vp, st]
    L.pcs_ensemble_diagnostics.argtypes = [vp, st, ctypes.POINTER(pcs_diag), st, ctypes.POINTER(ctypes.c_int32)]
    L.pcs_ensemble_state_size.argtypes = [vp, st, ctypes.POINTER(sz)]
    L.pcs_ensemble_get_state.argtypes = [vp, st, ctypes.POINTER(ctypes.c_double), sz]
    L.pcs_ensemble_destroy.argtypes = [vp]
    L.pcs_ensemble_set_state.argtypes = [vp, st, ctypes.POINTER(ctypes.c_double), sz]
    L.pcs_ensemble_run_status.argtypes = [vp, st]
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.pcs_midplane_histogram_setup.argtypes = [vp, ctypes.c_double, ctypes.c_double, st]
    L.pcs_midplane_histogram.argtypes = [vp, u64p, st]
    L.pcs_ensemble_midplane_histogram_setup.argtypes = [vp, st, ctypes.c_double, ctypes.c_double, st]
    L.pcs_ensemble_midplane_histogram.argtypes = [vp, st, u64p, st]
    L.pcs_midplane_pdf_setup.argtypes = [vp, st, ctypes.c_double, ctypes.c_double, st]
    L.pcs_midplane_pdf.argtypes = [vp, st, u64p, st]
    L.pcs_ensemble_midplane_pdf_setup.argtypes = [vp, st, st, ctypes.c_double, ctypes.c_double, st]
    L.pcs_ensemble_midplane_pdf.argtypes = [vp, st, st, u64p, st]
    L.pcs_midplane_moments.argtypes = [vp, st, ctypes.POINTER(ctypes.c_double)]
    L.pcs_ensemble_midplane_moments.argtypes = [vp, st, st, ctypes.POINTER(ctypes.c_double)]
    dp = ctypes.POINTER(ctypes.c_double)
    L.pcs_y_choice.argtypes = [vp, ctypes.POINTER(pcs_ychoice)]
    L.pcs_ensemble_y_choice.argtypes = [vp, ctypes.POINTER(pcs_ychoice)]
    L.pcs_ensemble_stage_times.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_int32]
    L.pcs_resample_state.argtypes = [ctypes.POINTER(pcs_grid), dp, sz, ctypes.POINTER(pcs_grid), dp, sz]
    for name in EXPORTS:
        if name not in ("pcs_status_string", "pcs_stage_name"):
            getattr(L, name).restype = st
    _lib = L
    return L


class PcsError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().pcs_status_string(status).decode()
        super().__init__("%s: %s (status %d)" % (where, msg, status))
        self.status = status


def _check(status, where, allow=(PCS_OK,)):
    if status not in allow:
        raise PcsError(status, where)
    return status


def make_grid(dim, nx, ny, nz=1, lx=10.0, lz=5.0):
    return pcs_grid(dim, nx, ny, 1 if dim == 2 else nz, lx, lz)


def make_params(re=0.01, wi=20.0, beta=0.8, kappa=5e-5, eps=0.0, dt=1e-3, forcing=0, q_or_dpdx=4.0 / 3.0,
                precision=0, scheme=0):
    return pcs_params(re, wi, beta, kappa, eps, dt, forcing, q_or_dpdx, precision, scheme)


def state_size(grid):
    """Doubles in the flat CNAB2 state of a run on grid (the layout of pcs_get_state)."""
    nf = 10 if grid.dim == 2 else 19
    return 4 + nf * grid.ny * (1 if grid.dim == 2 else grid.nz) * (grid.nx // 2) * 2


def resample_state(src_grid, state, dst_grid):
    """The flat state of another resolution (see pcs_resample_state)."""
    state = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(state_size(dst_grid))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().pcs_resample_state(ctypes.byref(src_grid), state.ctypes.data_as(dp), state.size,
                                    ctypes.byref(dst_grid), out.ctypes.data_as(dp), out.size), "pcs_resample_state")
    return out


def pcs_workspace_bytes(grid, params):
    n = ctypes.c_size_t(0)
    _check(lib().pcs_workspace_bytes(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(n)),
           "pcs_workspace_bytes")
    return n.value


DIAG_FIELDS = [f[0] for f in pcs_diag._fields_ if f[0] != "reserved"]


def _moments(out):
    """(samples, mean, standard deviation) from the device's count, sum and sum of squares."""
    n, s1, s2 = out[0], out[1], out[2]
    if n <= 0:
        return 0, float("nan"), float("nan")
    mean = s1 / n
    return int(n), mean, float(np.sqrt(max(s2 / n - mean * mean, 0.0)))


def _ychoice(out):
    """{"variant": [state products, projections], "budget": b, "error": [[per
    variant FP32, FP64, compensated] per table], "time_us": likewise}, with
    None where not measured."""
    def val(x):
        return None if x < 0 else float(x)
    return {"variant": [int(out.variant[0]), int(out.variant[1])], "budget": val(out.budget),
            "error": [[val(out.error[t][v]) for v in range(3)] for t in range(2)],
            "time_us": [[val(out.time_us[t][v]) for v in range(3)] for t in range(2)]}


def _arrays(grids, params):
    n = len(grids)
    if len(params) != n:
        raise ValueError("grids and params differ in length")
    return n, (pcs_grid * n)(*grids), (pcs_params * n)(*params)


def pcs_ensemble_workspace_bytes(grids, params):
    n, ga, pa = _arrays(grids, params)
    out = ctypes.c_size_t(0)
    _check(lib().pcs_ensemble_workspace_bytes(n, ga, pa, ctypes.byref(out)), "pcs_ensemble_workspace_bytes")
    return out.value


class Sim:
    """One channel-flow run: device workspace and stream from PyTorch, all
    work in libpcs.  Keep the object alive while the run is in use."""

    def __init__(self, grid, params, seed=0, amp=1e-3, device="cuda:0", static=False):
        """static=True: pcs_init_static (the library's static device array as
        workspace, nothing allocated; one live such run per GPU)."""
        import torch
        self.grid, self.params = grid, params
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        nbytes = pcs_workspace_bytes(grid, params)
        self.handle = ctypes.c_void_p(0)
        if static:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib().pcs_init_static(ctypes.byref(grid), ctypes.byref(params), ctypes.c_uint64(seed),
                                             float(amp), ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(self.handle)), "pcs_init_static")
        else:
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.workspace.data_ptr() + 255) & ~255
            _check(lib().pcs_init(ctypes.byref(grid), ctypes.byref(params), ctypes.c_uint64(seed), float(amp),
                                  ctypes.c_void_p(ptr), nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(self.handle)), "pcs_init")
        n = ctypes.c_size_t(0)
        _check(lib().pcs_state_size(self.handle, ctypes.byref(n)), "pcs_state_size")
        self.state_size = n.value
        self.workspace_bytes = nbytes

    def step(self, n=1):
        return _check(lib().pcs_step(self.handle, int(n)), "pcs_step")

    def diagnostics(self, max_records=4096):
        buf = (pcs_diag * max_records)()
        n = ctypes.c_int32(0)
        st = _check(lib().pcs_diagnostics(self.handle, buf, max_records, ctypes.byref(n)), "pcs_diagnostics",
                    allow=(PCS_OK, PCS_BLOWUP))
        recs = [{k: getattr(buf[i], k) for k in DIAG_FIELDS} for i in range(n.value)]
        return recs, st

    def get_state(self):
        out = np.zeros(self.state_size)
        _check(lib().pcs_get_state(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
               "pcs_get_state")
        return out

    def set_state(self, flat):
        """Full state of this run, or (SBDF4 runs) the CNAB2 layout, which
        restarts from a constant past; other sizes raise PcsError."""
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        _check(lib().pcs_set_state(self.handle, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), flat.size),
               "pcs_set_state")

    def midplane_histogram_setup(self, lo, hi, nbins):
        """Starts (nbins > 0, clearing the counts) or stops (nbins = 0) the
        on-device histogram of midplane Tr c (see pcs_midplane_histogram_setup)."""
        _check(lib().pcs_midplane_histogram_setup(self.handle, float(lo), float(hi), int(nbins)),
               "pcs_midplane_histogram_setup")
        self.__dict__.setdefault("pdf_bins", {})[PCS_PDF_TRC] = int(nbins)

    def midplane_histogram(self):
        """The nbins + 2 counts: below lo, the nbins bins, at or above hi (and non-finite)."""
        out = np.zeros(self.__dict__.get("pdf_bins", {}).get(PCS_PDF_TRC, 0) + 2, dtype=np.uint64)
        _check(lib().pcs_midplane_histogram(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                            out.size), "pcs_midplane_histogram")
        return out

    def midplane_pdf_setup(self, quantity, lo, hi, nbins):
        """Histogram of midplane quantity PCS_PDF_TRC / _U / _V / _W (see
        pcs_midplane_pdf_setup)."""
        _check(lib().pcs_midplane_pdf_setup(self.handle, int(quantity), float(lo), float(hi), int(nbins)),
               "pcs_midplane_pdf_setup")
        self.__dict__.setdefault("pdf_bins", {})[int(quantity)] = int(nbins)

    def midplane_pdf(self, quantity):
        out = np.zeros(self.__dict__.get("pdf_bins", {}).get(int(quantity), 0) + 2, dtype=np.uint64)
        _check(lib().pcs_midplane_pdf(self.handle, int(quantity), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      out.size), "pcs_midplane_pdf")
        return out

    def midplane_moments(self, quantity):
        """(samples, mean, standard deviation) of an enabled midplane quantity
        since its setup (pcs_midplane_moments)."""
        out = (ctypes.c_double * 3)()
        _check(lib().pcs_midplane_moments(self.handle, int(quantity), out), "pcs_midplane_moments")
        return _moments(out)

    def y_choice(self):
        """The wall-normal product variants in use and, for precision 4, the
        errors and times they were chosen by (pcs_y_choice)."""
        out = pcs_ychoice()
        _check(lib().pcs_y_choice(self.handle, ctypes.byref(out)), "pcs_y_choice")
        return _ychoice(out)

    def stage_times(self, nsteps, reps=1):
        """Mean milliseconds per launch of each stage over nsteps real steps
        (eager launch, every stage but the last repeated reps times back to
        back, HIP events on this run's stream); returns {stage name: ms}."""
        ms = (ctypes.c_double * PCS_NSTAGE)()
        _check(lib().pcs_stage_times(self.handle, int(nsteps), int(reps), ms, PCS_NSTAGE), "pcs_stage_times")
        return {lib().pcs_stage_name(i).decode(): ms[i] for i in range(PCS_NSTAGE)}

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.handle:
            lib().pcs_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """n independent runs advanced together (one graph launch per step, each
    stage one kernel over all runs); workspace and stream from PyTorch."""

    def __init__(self, grids, params, seeds, amp=1e-3, device="cuda:0"):
        import torch
        n, ga, pa = _arrays(grids, params)
        if len(seeds) != n:
            raise ValueError("need one seed per run")
        sa = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
        self.n = n
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        nbytes = pcs_ensemble_workspace_bytes(grids, params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        self.handle = ctypes.c_void_p(0)
        _check(lib().pcs_ensemble_init(n, ga, pa, sa, float(amp), ctypes.c_void_p(ptr), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)),
               "pcs_ensemble_init")
        self.workspace_bytes = nbytes

    def step(self, n=1):
        return _check(lib().pcs_ensemble_step(self.handle, int(n)), "pcs_ensemble_step")

    def diagnostics(self, run, max_records=4096):
        buf = (pcs_diag * max_records)()
        n = ctypes.c_int32(0)
        st = _check(lib().pcs_ensemble_diagnostics(self.handle, int(run), buf, max_records, ctypes.byref(n)),
                    "pcs_ensemble_diagnostics", allow=(PCS_OK, PCS_BLOWUP))
        recs = [{k: getattr(buf[i], k) for k in DIAG_FIELDS} for i in range(n.value)]
        return recs, st

    def state_size(self, run):
        n = ctypes.c_size_t(0)
        _check(lib().pcs_ensemble_state_size(self.handle, int(run), ctypes.byref(n)), "pcs_ensemble_state_size")
        return n.value

    def midplane_histogram_setup(self, run, lo, hi, nbins):
        _check(lib().pcs_ensemble_midplane_histogram_setup(self.handle, int(run), float(lo), float(hi), int(nbins)),
               "pcs_ensemble_midplane_histogram_setup")
        self.__dict__.setdefault("pdf_bins", {})[(int(run), PCS_PDF_TRC)] = int(nbins)

    def midplane_histogram(self, run):
        out = np.zeros(self.__dict__.get("pdf_bins", {}).get((int(run), PCS_PDF_TRC), 0) + 2, dtype=np.uint64)
        _check(lib().pcs_ensemble_midplane_histogram(self.handle, int(run),
                                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), out.size),
               "pcs_ensemble_midplane_histogram")
        return out

    def midplane_pdf_setup(self, run, quantity, lo, hi, nbins):
        _check(lib().pcs_ensemble_midplane_pdf_setup(self.handle, int(run), int(quantity), float(lo), float(hi),
                                                     int(nbins)), "pcs_ensemble_midplane_pdf_setup")
        self.__dict__.setdefault("pdf_bins", {})[(int(run), int(quantity))] = int(nbins)

    def midplane_pdf(self, run, quantity):
        out = np.zeros(self.__dict__.get("pdf_bins", {}).get((int(run), int(quantity)), 0) + 2, dtype=np.uint64)
        _check(lib().pcs_ensemble_midplane_pdf(self.handle, int(run), int(quantity),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), out.size),
               "pcs_ensemble_midplane_pdf")
        return out

    def set_state(self, run, flat):
        """New state of run `run` (pcs_ensemble_set_state; unmasks a blown-up run)."""
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        _check(lib().pcs_ensemble_set_state(self.handle, int(run), flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            flat.size), "pcs_ensemble_set_state")

    def run_status(self, run):
        """PCS_OK if run `run` is being stepped, PCS_ERR_STATE if it is masked after a blow-up."""
        return _check(lib().pcs_ensemble_run_status(self.handle, int(run)), "pcs_ensemble_run_status",
                      allow=(PCS_OK, PCS_ERR_STATE))

    def stage_times(self, nsteps, reps=1):
        """As Sim.stage_times, for the whole ensemble (pcs_ensemble_stage_times)."""
        ms = (ctypes.c_double * PCS_NSTAGE)()
        _check(lib().pcs_ensemble_stage_times(self.handle, int(nsteps), int(reps), ms, PCS_NSTAGE),
               "pcs_ensemble_stage_times")
        return {lib().pcs_stage_name(i).decode(): ms[i] for i in range(PCS_NSTAGE)}

    def y_choice(self):
        """As Sim.y_choice, for the whole ensemble (pcs_ensemble_y_choice)."""
        out = pcs_ychoice()
        _check(lib().pcs_ensemble_y_choice(self.handle, ctypes.byref(out)), "pcs_ensemble_y_choice")
        return _ychoice(out)

    def midplane_moments(self, run, quantity):
        out = (ctypes.c_double * 3)()
        _check(lib().pcs_ensemble_midplane_moments(self.handle, int(run), int(quantity), out),
               "pcs_ensemble_midplane_moments", "pcs_y_choice", "pcs_ensemble_y_choice", "pcs_ensemble_stage_times")
        return _moments(out)

    def get_state(self, run):
        out = np.zeros(self.state_size(run))
        _check(lib().pcs_ensemble_get_state(self.handle, int(run), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            out.size), "pcs_ensemble_get_state")
        return out

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.handle:
            lib().pcs_ensemble_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
