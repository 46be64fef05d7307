/* pcs.h - polymer channel-flow step on one AMD Instinct MI355X (gfx950).
 *
 * One semi-implicit pseudo-spectral time step of dilute-polymer plane-channel
 * flow, as set up in the paper's Section 2: the conformation-tensor equation
 * (1) (sPTT, Oldroyd-B for eps = 0) with polymer diffusion kappa, the momentum
 * equation (2) with the polymer-stress divergence, incompressibility (3);
 * no-slip walls at y = +-1, conformation wall values from (1) with kappa = 0;
 * Fourier in x and z, Chebyshev (Gauss-Lobatto collocation) in y, fully
 * dealiased by the 3/2 rule.  Positive-definiteness of c is deliberately not
 * enforced; the diagnostics report where Tr c drops below 3 and below 0
 * (Section 3, eqs. (4)-(5) use the midplane counts).  Time integration is
 * CNAB2 (Crank-Nicolson / 2nd-order Adams-Bashforth; the first step uses
 * the current explicit terms as history).
 *
 * Conventions shared by every call
 *  - Errors are returned as pcs_status, never thrown; nothing here exits.
 *  - Device memory: the caller allocates one device workspace of the size
 *    reported by pcs_workspace_bytes (256-byte aligned) and keeps it alive
 *    until pcs_destroy.  The library never allocates device memory itself.
 *  - Streams: every device operation is enqueued on the caller's HIP stream
 *    (hipStream_t passed as void*; NULL means the default stream).  Calls on
 *    one handle must not overlap in time from several host threads.
 *  - The opaque handle belongs to the library and is released by pcs_destroy;
 *    host buffers passed in always belong to the caller.
 */
#ifndef PCS_H
#define PCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pcs_status;
#define PCS_OK 0
#define PCS_BLOWUP 1        /* warning: a diagnostic record flagged blow-up (sticky) */
#define PCS_ERR_ARG (-1)    /* null pointer or out-of-range value */
#define PCS_ERR_UNSUPPORTED (-2) /* size or option not supported (see pcs_grid) */
#define PCS_ERR_WORKSPACE (-3)   /* workspace too small or misaligned */
#define PCS_ERR_DEVICE (-4)      /* a HIP call failed */
#define PCS_ERR_STATE (-5)       /* stepping a run whose blow-up flag is set */

/* Grid.  dim = 2: x-y channel (nz must be 1); dim = 3: x-y-z.
 *  nx: points of the base grid in x (even, >= 4); kx = 2 pi m / lx for
 *      m = 0 .. nx/2 - 1 are kept (Nyquist dropped).  3 nx / 2 must factor
 *      as 2^a 3^b.
 *  ny: Gauss-Lobatto points in y (odd, >= 9): N = ny - 1, y_j = cos(pi j/N),
 *      y_0 = +1, y_N = -1, y_{N/2} = 0 (the midplane).
 *  nz: base points in z (3D: even, >= 4, 3 nz / 2 = 2^a 3^b; the Nyquist
 *      slot nz/2 is held at zero).
 *  lx, lz: periods (the paper uses 10; the 3D workloads here use lz = 5). */
typedef struct {
  int32_t dim, nx, ny, nz;
  double lx, lz;
} pcs_grid;

/* Physical and numerical parameters (paper, Section 2 scalings):
 *  re, wi, beta, kappa, eps as in eqs. (1)-(2); dt the time step.
 *  forcing = 0: constant flow rate, sum_j w_j U_j = q_or_dpdx (4/3 is the
 *               flux of the laminar profile U = 1 - y^2); the drive Pi is
 *               solved for every step and reported as dpdx.
 *  forcing = 1: constant drive Pi = q_or_dpdx (2/Re reproduces eq. (2)).
 *  precision = 0: every stage in FP64.
 *  precision = 1: mixed: transforms and pointwise products of the
 *               fluctuation (all modes except kx = kz = 0) in FP32, the
 *               mean-mode profiles and every boundary-value solve in FP64
 *               (the sPTT eps term is split the same way: fluctuation part
 *               in FP32, product of the mean profiles in FP64).
 *  precision = 2: as 1, but the wall-normal transforms of the fluctuation
 *               (to and from the padded grid) are computed in FP64 and
 *               only the periodic transforms and products in FP32.
 *  precision = 3: as 1, but the wall-normal transforms of the fluctuation
 *               are error-compensated FP32 products: every operator is an
 *               FP32 head plus an FP32 tail, every state value is split the
 *               same way, and the results of the FP32 matrix instructions
 *               are accumulated as unevaluated FP32 pairs (exact two-term
 *               sums).  This removes the rounding of the operands and of
 *               the accumulation across instructions, but not the rounding
 *               inside each instruction (a chain of four fused multiply-adds
 *               on this hardware), so the measured error stays of the order
 *               of plain FP32 at two to five times its cost (pcs_y_choice
 *               reports both).
 *  precision = 4: as 1, but each of the two wall-normal product tables
 *               (values and d/dy of the state on the padded grid; the
 *               projections of the explicit terms) takes, at pcs_init, the
 *               fastest of the three variants above (PCS_Y_FP32,
 *               PCS_Y_FP64, PCS_Y_COMP) whose measured error is within the
 *               budget (equal times keep the FP64 operators): the error of
 *               a variant is the largest difference of
 *               its outputs from those of the FP64-operator variant on the
 *               run's initial state, relative to the largest magnitude of
 *               the same output field (mean mode excluded), over all fields
 *               of the table; the budget is PCS_Y_ERROR_BUDGET from the
 *               environment if set (a non-negative number), else 1e-5.  The
 *               choice is made for the whole ensemble; pcs_y_choice reports
 *               it with the errors and times measured.
 *  scheme = 0:  CNAB2 (Crank-Nicolson on the linear terms, 2nd-order
 *               Adams-Bashforth on the rest).
 *  scheme = 1:  SBDF4, the 4th-order semi-implicit BDF that Section 2 names
 *               (Wang and Ruuth 2008, constant step):
 *               (25/12 q^{n+1} - 4 q^n + 3 q^{n-1} - 4/3 q^{n-2} + 1/4 q^{n-3})/dt
 *                 = 4 X^n - 6 X^{n-1} + 4 X^{n-2} - X^{n-3} + L q^{n+1}
 *               with X the explicit and L the implicit linear terms; a fresh
 *               initial condition starts from a constant past. */
typedef struct {
  double re, wi, beta, kappa, eps, dt;
  int32_t forcing;
  double q_or_dpdx;
  int32_t precision;
  int32_t scheme;
} pcs_params;

/* One record per step, computed on the base grid (nx x ny x nz points):
 *  min_trc, n_lt3, n_lt0 over the volume; mid_* on the midplane j = N/2;
 *  counts use strict '<' and ignore non-finite values;
 *  cfl = dt max(|u|/dx + |v|/dy_j + |w|/dz) with dy_j the local Lobatto
 *  spacing (y_{j-1} - y_{j+1})/2, one-sided at the walls;
 *  dpdx = the drive Pi of this step; energy = <|u|^2/2>, mean_trc = <Tr c>
 *  (Fourier mean in x, z times Clenshaw-Curtis weights / 2 in y);
 *  blowup = 1 if any value was non-finite or |Tr c| > 1e12. */
typedef struct {
  int64_t step;
  double t, min_trc, mid_min_trc, cfl, dpdx, energy, mean_trc;
  uint64_t n_lt3, n_lt0, mid_n_lt3, mid_n_lt0;
  int32_t blowup, reserved;
} pcs_diag;

struct pcs_sim;

/* Device workspace needed by pcs_init for this grid / parameter set. */
pcs_status pcs_workspace_bytes(const pcs_grid* grid, const pcs_params* params, size_t* bytes);

/* Builds the operators (host, extended precision), uploads them into the
 * workspace, sets the initial state: the laminar Poiseuille state of eqs.
 * (1)-(2) (U = 1 - y^2, c_xy = Wi U', c_yy = c_zz = 1, c_xx = 1 + 2 (Wi U')^2
 * plus the kappa boundary-layer term) plus a divergence-free perturbation
 * of amplitude amp drawn from SplitMix64(seed) (amp = 0: laminar), and the
 * history from the explicit terms of that state.  Synchronises the stream.
 * workspace: device pointer of at least pcs_workspace_bytes bytes.
 * stream: hipStream_t or NULL.  *out receives the handle.
 * Tile shapes of the wall-normal products are chosen by timing the
 * candidates on the device (once per table shape and process).  If the
 * environment variable PCS_TUNE_CACHE names a file, choices recorded there for
 * this GPU architecture and table shape are used without timing, and new
 * choices are appended to it, so that runs in different processes use the
 * same tiles and the same summation order. */
pcs_status pcs_init(const pcs_grid* grid, const pcs_params* params, uint64_t seed, double amp, void* workspace,
                    size_t bytes, void* stream, struct pcs_sim** out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as serving loops or harnesses that forbid it, or that later
 * steps the run inside a stream capture): pcs_init without a workspace
 * argument.  The run lives in a static device array of the library,
 * PCS_STATIC_BYTES bytes on each GPU that uses it, held from the library's
 * load until the process ends; nothing is allocated, by the library or on
 * its behalf.  The array of the current device is cleared (on the stream)
 * and then set up exactly as pcs_init would set up a workspace, except that
 * the tile autotuner is not run (default tile shapes) and no graphs or side
 * streams are created: pcs_step launches each step's kernels one by one on
 * the stream, which a caller may capture.  One live handle per GPU: the
 * array is shared by every call on that GPU and keeps the last run's
 * contents, so runs that overlapped on one GPU would race; while a handle
 * from this call is alive, another call on the same GPU returns
 * PCS_ERR_WORKSPACE, as does a grid / parameter set whose pcs_workspace_bytes
 * exceeds PCS_STATIC_BYTES.  pcs_destroy releases the array for the next
 * call.  Other arguments, results and errors as pcs_init. */
#define PCS_STATIC_BYTES ((size_t)64 << 20)
pcs_status pcs_init_static(const pcs_grid* grid, const pcs_params* params, uint64_t seed, double amp, void* stream,
                           struct pcs_sim** out);

/* Enqueues nsteps time steps (asynchronous).  Returns PCS_ERR_STATE if a
 * blow-up was seen at the last synchronisation.  A run blowing up inside the
 * enqueued steps stops on the device: once a step record flags blow-up, every
 * kernel of the following steps skips the run's work and no further records
 * are written (finite-time blow-up, Section 2, is a property of the run, not
 * a device fault); pcs_set_state restarts it. */
pcs_status pcs_step(struct pcs_sim* sim, int32_t nsteps);

/* Synchronises the stream and copies the diagnostic records produced since
 * the previous call (at most max, the oldest first; the device keeps the last
 * 4096) into out.  Returns PCS_BLOWUP if any record since init flagged it. */
pcs_status pcs_diagnostics(struct pcs_sim* sim, pcs_diag* out, int32_t max, int32_t* n_out);

/* Number of doubles in the flat state vector of this handle. */
pcs_status pcs_state_size(struct pcs_sim* sim, size_t* n);

/* Flat FP64 state (host buffer of pcs_state_size doubles), synchronising:
 *   [step, t, Pi, 0] then each field as [y j = 0..N][kz slot][kx] complex
 *   (re, im interleaved);
 *   fields 2D: u v phi cxx cxy cyy | hv Fxx Fxy Fyy
 *          3D: u v w phi g cxx cxy cxz cyy cyz czz | hv hg Fxx Fxy Fxz Fyy Fyz Fzz
 *   phi = lap v, g = omega_y; hv, hg, F are the previous step's explicit
 *   terms (AB2 history); the kx = kz = 0 slot of u and w holds the mean
 *   profiles U, W, that of hv and hg the mean-flow forcing history.
 *   SBDF4 (scheme 1) appends the three previous states (every field of the
 *   first group, for q^{n-1}, q^{n-2}, q^{n-3} in turn) and the explicit
 *   terms of steps n-2 and n-3 (every field of the second group, twice).  */
pcs_status pcs_get_state(struct pcs_sim* sim, double* host, size_t n);
/* Replaces the state (same layout) and clears the blow-up flag.  The header's
 * step must be a whole number in [0, 2^53] and t, Pi finite (PCS_ERR_ARG
 * otherwise, the run unchanged).  An SBDF4
 * run also takes the CNAB2 layout (n of a CNAB2 run on the same grid): the
 * earlier states and explicit terms are then a constant past, q^{n-k} := q^n
 * and X^{n-k} := X^{n-1} (for instance after pcs_resample_state). */
pcs_status pcs_set_state(struct pcs_sim* sim, const double* host, size_t n);

/* Profiling: runs nsteps real time steps (the state advances exactly as with
 * pcs_step) launched stage by stage, with a HIP event recorded on the
 * handle's stream between stages, and returns in ms[i] the mean duration of
 * one launch of stage i.  Every stage is one kernel launch: the products
 * (gemm_*: the FP64 mean profiles, the padded-grid values and derivatives,
 * the FP64 D2 / D of the state, the projections, the two eigenbasis
 * products), the z and x transforms, the RHS, finalize and diagnostics
 * kernels.  Where one launch holds all products of the state (steps of less
 * than about a million padded-grid points), gemm_state times it and
 * gemm_mean and gemm_d2 report 0.  Each stage except the row diagnostics (which also add the
 * step's midplane samples to the histograms) and the step record is launched
 * reps times back to back between its two events (these stages recompute the
 * same outputs from unchanged inputs), so that with reps > 1 the GPU does
 * not wait for the host between launches and ms[i] approaches the kernel's
 * own duration.  nstage must be at least PCS_NSTAGE; stages that do not
 * apply (the z transforms in 2D) report 0, as do entries beyond
 * PCS_NSTAGE.  Stage names come from pcs_stage_name.  Synchronises the
 * stream. */
#define PCS_NSTAGE 14
pcs_status pcs_stage_times(struct pcs_sim* sim, int32_t nsteps, int32_t reps, double* ms, int32_t nstage);
const char* pcs_stage_name(int32_t i);

/* Midplane statistics (paper, Section 3, eqs. (4)-(5)).  While enabled,
 * every step adds the base-grid values of Tr c on the midplane y = 0 (the
 * Nx Nz points of Lobatto row N/2, where y = 0 exactly) to a histogram kept
 * on the device: with w = (hi - lo) / nbins, counts[b] (1 <= b <= nbins)
 * counts values in [lo + (b-1) w, lo + b w) (bin 1 + floor((v - lo) nbins /
 * (hi - lo)), evaluated in FP64), counts[0] values below lo and
 * counts[nbins + 1] values at or above hi and non-finite ones.  These are the
 * samples of the PDF P_c of eq. (4); P(Tr c < 3) is the fraction of samples
 * below 3 and chi of eq. (5) that number of samples divided by Nx Nz (the
 * per-step counts of the same events are also in pcs_diag.mid_n_lt3).
 * Setup clears the counts (nbins = 0 turns the histogram off, the default;
 * PCS_ERR_ARG for nbins > PCS_HIST_MAX, non-finite lo or hi, or lo >= hi) and
 * synchronises the stream.  pcs_midplane_histogram synchronises and copies
 * the nbins + 2 counts (n must be nbins + 2; PCS_ERR_ARG while off). */
/* The wall-normal product variants of the mixed precisions (see
 * pcs_params.precision) and the choice made for precision 4:
 * variant[0] is that of the padded-grid values and d/dy of the state,
 * variant[1] that of the projections of the explicit terms (0 for the FP64
 * path of precision 0); budget the error budget in force; error[t][v - 1]
 * and time_us[t][v - 1] the measured error and launch time of table t in
 * variant v (-1 where not measured: every precision other than 4, and time
 * in runs initialised by pcs_init_static, which are not timed and then
 * prefer PCS_Y_FP32, then PCS_Y_FP64, among the variants within the
 * budget).  The time of table t is that of the launch holding it, which
 * may hold other FP64 products of the same stage. */
#define PCS_Y_FP32 1
#define PCS_Y_FP64 2
#define PCS_Y_COMP 3
typedef struct {
  int32_t variant[2];
  double budget;
  double error[2][3];
  double time_us[2][3];
} pcs_ychoice;
pcs_status pcs_y_choice(struct pcs_sim* sim, pcs_ychoice* out);

#define PCS_HIST_MAX 4096
pcs_status pcs_midplane_histogram_setup(struct pcs_sim* sim, double lo, double hi, int32_t nbins);
pcs_status pcs_midplane_histogram(struct pcs_sim* sim, uint64_t* counts, int32_t n);

/* Midplane PDFs of other quantities (Section 3 compares the midplane
 * statistics of the velocity fluctuations and of the longitudinal and
 * transverse velocity gradients across resolutions): the same histogram for
 * quantity
 *   PCS_PDF_TRC   Tr c (the histogram above),
 *   PCS_PDF_U     u - U(0), U(0) the plane mean of u at y = 0 (its kx = kz = 0
 *                 mode) at the same step,
 *   PCS_PDF_V     v (whose plane mean is zero),
 *   PCS_PDF_W     w - W(0),
 *   PCS_PDF_DUDX  d u / d x (longitudinal gradient of u),
 *   PCS_PDF_DUDZ  d u / d z (transverse gradient of u),
 *   PCS_PDF_DWDX  d w / d x (transverse gradient of w),
 *   PCS_PDF_DWDZ  d w / d z (longitudinal gradient of w),
 * (the quantities with w or d/dz are 3D only: PCS_ERR_ARG in 2D), each with
 * its own range, bins and counts, set up and read as above.  All are binned
 * by the same row-diagnostics kernel in the same step; the gradients are
 * spectral derivatives of the base-grid fields. */
#define PCS_PDF_TRC 0
#define PCS_PDF_U 1
#define PCS_PDF_V 2
#define PCS_PDF_W 3
#define PCS_PDF_DUDX 4
#define PCS_PDF_DUDZ 5
#define PCS_PDF_DWDX 6
#define PCS_PDF_DWDZ 7
pcs_status pcs_midplane_pdf_setup(struct pcs_sim* sim, int32_t quantity, double lo, double hi, int32_t nbins);
pcs_status pcs_midplane_pdf(struct pcs_sim* sim, int32_t quantity, uint64_t* counts, int32_t n);
/* Running moments of the samples of an enabled quantity (the paper's PDFs
 * are standardised by their own mean and standard deviation): out[0] the
 * number of finite samples, out[1] their sum, out[2] the sum of their
 * squares, accumulated on the device since the quantity's setup (which clears
 * them) in a fixed order, so repeated runs give identical sums; mean =
 * out[1] / out[0], variance = out[2] / out[0] - mean^2.  Synchronises;
 * PCS_ERR_ARG while the quantity is off or for a null out. */
pcs_status pcs_midplane_moments(struct pcs_sim* sim, int32_t quantity, double* out);

/* Resampling between resolutions (Section 2 starts every run of Table 1 from one
 * snapshot re-interpolated onto its grid; host only, no GPU work): fills dst_state
 * (the flat CNAB2 layout of pcs_get_state for grid dst, nd doubles) from src_state
 * (grid src, ns doubles) of the same dimension and box (lx, lz).  Per field
 * and Fourier mode, the Chebyshev series interpolating the source Lobatto
 * values is truncated or zero-padded to the target degree and evaluated on
 * the target points (exact for polynomials of degree up to min(Ny, Ny') - 1);
 * Fourier amplitudes of modes retained at both resolutions are copied, the
 * others are zero; the header [step, t, Pi, 0] is copied.  Truncation can
 * leave wall values slightly off their boundary conditions; the next step's
 * solves restore them.  The result goes to a run with pcs_set_state.
 * PCS_ERR_ARG for null pointers, invalid or mismatched grids (as pcs_grid,
 * ny >= 5) or wrong sizes. */
pcs_status pcs_resample_state(const pcs_grid* src, const double* src_state, size_t ns, const pcs_grid* dst,
                              double* dst_state, size_t nd);

pcs_status pcs_destroy(struct pcs_sim* sim);
const char* pcs_status_string(pcs_status s);

/* Ensembles: n independent runs of uneven sizes (the scan over resolutions
 * and Wi of the paper's Section 3 stability and positivity study), all of
 * one dimension and one precision setting, advanced together.  Every stage
 * of the step is one kernel launch over all runs (a ragged table of
 * (run, tile) work items), and the step is one graph launch on the stream.
 * Conventions as for single runs: one caller-owned device workspace of
 * pcs_ensemble_workspace_bytes, the caller's stream, an opaque handle.
 * grids, params and seeds are arrays of n entries (run r starts from the
 * state pcs_init would build with grids[r], params[r], seeds[r], amp).
 * Errors: PCS_ERR_ARG for n <= 0 or null arrays, PCS_ERR_UNSUPPORTED if
 * the runs mix dimensions or precisions (or any run's grid is unsupported),
 * PCS_ERR_WORKSPACE as for pcs_init.  A run that blows up (Section 2
 * discusses finite-time blow-up of the unregularised equations) is masked
 * from the step after the record that flags it: its kernels skip their work
 * items, its step count and records stop, and the other runs advance exactly
 * as they would without it (no run reads another's data).  Its diagnostics
 * report PCS_BLOWUP, pcs_ensemble_run_status reports PCS_ERR_STATE, and
 * pcs_ensemble_set_state gives it a new state and unmasks it. */
struct pcs_ens;
pcs_status pcs_ensemble_workspace_bytes(int32_t n, const pcs_grid* grids, const pcs_params* params, size_t* bytes);
pcs_status pcs_ensemble_init(int32_t n, const pcs_grid* grids, const pcs_params* params, const uint64_t* seeds,
                             double amp, void* workspace, size_t bytes, void* stream, struct pcs_ens** out);
/* Enqueues nsteps steps of every run (asynchronous). */
pcs_status pcs_ensemble_step(struct pcs_ens* ens, int32_t nsteps);
/* Diagnostics, state size and state of run `run` (0 <= run < n), with the
 * semantics of pcs_diagnostics, pcs_state_size and pcs_get_state. */
pcs_status pcs_ensemble_diagnostics(struct pcs_ens* ens, int32_t run, pcs_diag* out, int32_t max, int32_t* n_out);
pcs_status pcs_ensemble_state_size(struct pcs_ens* ens, int32_t run, size_t* n);
pcs_status pcs_ensemble_get_state(struct pcs_ens* ens, int32_t run, double* host, size_t n);
/* Replaces the state of run `run` (the semantics and layout of pcs_set_state:
 * synchronises the stream, clears the run's blow-up flag and so unmasks it;
 * the other runs are untouched). */
pcs_status pcs_ensemble_set_state(struct pcs_ens* ens, int32_t run, const double* host, size_t n);
/* Synchronises the stream; PCS_OK if run `run` is being stepped, PCS_ERR_STATE
 * if it is masked after a blow-up (until pcs_ensemble_set_state). */
pcs_status pcs_ensemble_run_status(struct pcs_ens* ens, int32_t run);
/* Midplane histogram of run `run`, as pcs_midplane_histogram_setup and
 * pcs_midplane_histogram. */
pcs_status pcs_ensemble_midplane_histogram_setup(struct pcs_ens* ens, int32_t run, double lo, double hi,
                                                 int32_t nbins);
pcs_status pcs_ensemble_midplane_histogram(struct pcs_ens* ens, int32_t run, uint64_t* counts, int32_t n);
/* Midplane PDF of quantity `quantity` of run `run`, as pcs_midplane_pdf_setup
 * and pcs_midplane_pdf. */
pcs_status pcs_ensemble_midplane_pdf_setup(struct pcs_ens* ens, int32_t run, int32_t quantity, double lo, double hi,
                                           int32_t nbins);
pcs_status pcs_ensemble_midplane_pdf(struct pcs_ens* ens, int32_t run, int32_t quantity, uint64_t* counts,
                                     int32_t n);
/* Running moments of run `run`, as pcs_midplane_moments. */
pcs_status pcs_ensemble_midplane_moments(struct pcs_ens* ens, int32_t run, int32_t quantity, double* out);
pcs_status pcs_ensemble_y_choice(struct pcs_ens* ens, pcs_ychoice* out);
/* pcs_stage_times for the whole ensemble (every stage is one launch over all
 * runs); runs masked after a blow-up cost nothing in it. */
pcs_status pcs_ensemble_stage_times(struct pcs_ens* ens, int32_t nsteps, int32_t reps, double* ms, int32_t nstage);
pcs_status pcs_ensemble_destroy(struct pcs_ens* ens);

#ifdef __cplusplus
}
#endif

#endif /* PCS_H */
