// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcs {

// Global-memory view of a pointer read from an argument table.  Pointers
// loaded from device memory are generic to the compiler, and generic (flat)
// accesses also count as LDS operations: every wait for an LDS access would
// then wait for all outstanding global loads too, which serialises prefetch
// with compute.  Casting to the global address space yields global_load /
// global_store instructions instead.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// One dense product C = alpha * A * B + beta * C, real.  A (m x k) is stored
// row-major in the compute precision, A[i][kk] at A[i * lda + kk], with
// lda = gemm_lda(k) and gemm_rows(m) rows allocated, all padding zero (the
// kernels read whole 16-wide k blocks and row tiles of A unguarded).
// B (k x n) and C (m x n) are row-major, each in its own precision (see
// GemmType).  Complex fields (re/im interleaved) are multiplied by a real
// operator by treating each complex column as two real columns.
//
// Parity products.  Every wall-normal operator of the step is
// centrosymmetric or centro-antisymmetric (the Lobatto and padded grids are
// symmetric about the midplane): A[mf-1-i][kf-1-j] = sigma A[i][j].  Writing
// B = Be + Bo with Be[j] = B[j] + B[kf-1-j], Bo[j] = B[j] - B[kf-1-j]
// (j < kf-1-j; Be[mid] = B[mid], Bo[mid] = 0), one product becomes two of
// half the size, E = Ae Be and O = Ao Bo over the first ceil(kf/2) rows of
// B, with (A B)[i] = E[i] + O[i] and (A B)[mf-1-i] = sigma (E[i] - O[i]).
// The interior eigenbasis has the same structure (even eigenvectors first),
// which gives the other two kinds: the eigen coefficients of the even and
// odd parts as separate output rows, and a product whose B rows are already
// split into an even and an odd block.
enum {
  PAR_NONE = 0,
  PAR_FOLD_UNFOLD,   // B folded (kf rows), output unfolded (mf rows, sign sigma)
  PAR_FOLD_SPLIT,    // B folded; E to rows [0, m), O to rows [m, mf)
  PAR_SPLIT_UNFOLD,  // Be = B rows [0, k), Bo = B rows [k, kf); output unfolded
};
struct EigScale;
struct GemmJob {
  int type;  // GemmType of this product (a table may mix GEMM_DDD with its own type)
  int kind;  // PAR_*; for the parity kinds m and k are the sizes of E (and of O,
             // whose operator A2 is padded to the same shape) and lda serves both
  const void* A;
  const void* A2;
  const void* Alo;   // error-compensated types: FP32 tails of A and A2 (A = head + tail)
  const void* A2lo;
  const void* B;
  void* C;
  void* C2;  // optional second output: alpha A B scaled by scale2 (no beta term)
  int m, n, k, lda, ldb, ldc;
  int mf, kf, sigma;   // parity kinds: full output rows, full B rows, mirror sign
  double alpha, beta;  // parity kinds: beta must be 0
  int flags;           // GEMM_ZERO_MEAN: B columns 0 and 1 (the kx = kz = 0 mode) read as zero
  int scale, scale2;   // SCALE_*: output row i is eigen coefficient i, scaled per mode
  const EigScale* es;  // per-solve constants for the scaling
  const int* skip;     // the run's blow-up flag (device): nonzero skips the product; null: never
  // B-stationary configurations: 1 when the next job of the table stages the
  // same folded panel (same B, kind, k, kf, ldb, n and flags: the values and
  // d/dy, or D2 and D, of one field), whose product this job's tiles then
  // also compute from the staged panel; 2 for that next job (no tiles of
  // its own there); 0 otherwise.  Other configurations ignore it.
  int pair;
  int tiles_m, tile0;  // filled by gemm_prepare
};
constexpr int GEMM_ZERO_MEAN = 1;

// Diagonal of the Dirichlet Helmholtz operators in the eigenbasis of the
// interior D2 block (D2_II = V diag(lam) V^-1), applied to X = V^-1 R:
//   SCALE_PHI: 1/(1/dt + nu k^2/2 - nu lam/2)       (phi, g; U and W in the mean slot)
//   SCALE_V:   that / (lam - k^2), 0 in the mean slot (v from lap v = phi)
//   SCALE_C:   1/(1/dt + 1/(2Wi) + kappa k^2/2 - kappa lam/2)
enum { SCALE_NONE = 0, SCALE_PHI, SCALE_V, SCALE_C };
struct EigScale {
  const double* lam;
  const double* kx;
  const double* kz;
  int nkx, dim;
  double ia, th;  // Helmholtz coefficients: 1/dt and 1/2 (CNAB2), 25/(12 dt) and 1 (SBDF4)
  double nu, wi, kappa;
};

// compute / B / C precisions: D = double, F = float, C = error-compensated
// FP32 (head and tail products, TwoSum accumulation; parity products in the
// B-stationary configurations only)
enum GemmType { GEMM_DDD = 0, GEMM_FDF, GEMM_FFD, GEMM_DDF, GEMM_DFD, GEMM_CDF, GEMM_CFD, GEMM_NTYPES };
bool gemm_type_comp(GemmType t);

constexpr int MAX_JOBS = 64;
// Tile configurations.  Register-direct kernel (operand fragments loaded
// straight into registers, no LDS in the loop): 0: 32 x 32 with K split over
// the four waves, 1: 64 x 32 and 2: 32 x 64 with K split in two, 3: 64 x 64.
// LDS-tiled kernel (operand chunks shared by the four waves through LDS):
// 4: 32 x 32, 5: 64 x 32, 6: 64 x 64, 7: 128 x 64 (double-buffered chunks),
// 8: 32 x 32, 9: 64 x 32 (one buffer, chunks of 64 k), and for small tables
// deeper parity chunks: 10, 11: 32 x 32, 12, 13: 64 x 64.  B-stationary
// kernel (parity products only; a workgroup stages the whole K range of a
// panel of B once and computes every output row of it): 14: 32, 15: 64
// columns per panel in four waves, 16: 16 and 17: 32 columns in eight.
constexpr int GEMM_NCFG = 18;
constexpr size_t GEMM_LDS_MAX = 160 * 1024;  // LDS a workgroup may take
inline int gemm_lda(int k) { return (k + 15) & ~15; }
inline int gemm_rows(int m) { return (m + 127) & ~127; }

// Fills tiles_m / tile0 for tile configuration cfg and returns the total
// number of workgroups.  Logical tile t belongs to the last job whose tile0
// is <= t; the kernels read that job index from a tile map (one int per
// tile) built by the caller.
int gemm_prepare(GemmJob* jobs, int njobs, int cfg);
// Whether configuration cfg evaluates parity products (the LDS-tiled and
// B-stationary ones), and whether it is B-stationary (one tile per column
// panel of a product, every row; its LDS grows with K).
bool gemm_cfg_parity(int cfg);
bool gemm_cfg_bst(int cfg);
// LDS bytes per workgroup of the LDS-tiled configuration cfg for a table of
// precision combination t (0 for the register-direct ones): the panels of
// the largest product form and compute precision in the table, so that a
// table of parity products, or of FP32 products only, keeps more
// workgroups resident per CU.
size_t gemm_lds_bytes(GemmType t, const GemmJob* jobs, int njobs, int cfg);
// t: the table's precision combination; its jobs are of type t or GEMM_DDD;
// tmap: job index of every logical tile; parity: every job is a parity
// product (else none is; a table holds one form); lds: gemm_lds_bytes of the
// same table and configuration.
void gemm_run(GemmType t, const GemmJob* dev_jobs, const int* tmap, int total_tiles, int cfg, bool parity,
              size_t lds, hipStream_t s);

hipError_t gemm_set_attributes();

// Mixed-radix (8, 4, 2, 3) Stockham plan for a length L = 2^a 3^b.  Per
// pass p: radix, L / radix (lr), product of the earlier radices (ns), the
// twiddle stride L / (ns radix) (ts), and multiply-high reciprocals of lr and
// ns (mlr, mns: floor(n / d) = umulhi(n, m) for the n < 2^16 the passes use;
// 0 when d = 1).
struct FftPlan {
  int L = 0;
  int npass = 0;
  int radix[12] = {0};
  int lr[12] = {0};
  int ns[12] = {0};
  int ts[12] = {0};
  unsigned mlr[12] = {0};
  unsigned mns[12] = {0};
};
// Multiply-high reciprocal of d >= 2 (0 for d = 1), exact for n d < 2^32.
__host__ __device__ inline unsigned fast_div_magic(unsigned d) { return d <= 1 ? 0u : 0xFFFFFFFFu / d + 1u; }
bool make_plan(int L, FftPlan* p);

// Problem description shared by the elementwise kernels.
struct Dims {
  int dim;          // 2 or 3
  int N, M;         // Ny - 1 and 3N/2
  int nkx, nzs;     // retained kx, kz slots (Nz or 1)
  int nm;           // nzs * nkx (complex modes per y row)
  int cw;           // 2 * nm (real columns per y row)
  int px, pz;       // padded x / z points
  int nx, nz;       // base x / z points
  int nc;           // conformation components (3 or 6)
  double lx, lz;
};

struct Phys {
  double re, wi, beta, kappa, eps, dt;
  int forcing;
  double q_or_dpdx;
  double coef;      // (1 - beta)/(Re Wi)
  double nu;        // beta / Re
  int scheme;       // 0: CNAB2, 1: SBDF4
  double ia, th;    // leading coefficient / dt and implicit weight of the scheme
};

// Device-resident scalars advanced by the step itself.  blowup is sticky:
// once a step record flags it, every stage kernel skips the run's work and
// the step record is no longer written (the run is masked until the host
// sets a new state).
struct DevScalars {
  long long step;
  double t;
  double pi;
  int blowup;
  int pad;
};
// the masking test at the start of a stage kernel
__device__ inline bool masked(const int* skip) { return skip != nullptr && *gmem(skip) != 0; }

struct DiagRec {
  long long step;
  double t, min_trc, mid_min_trc, cfl, dpdx, energy, mean_trc;
  unsigned long long n_lt3, n_lt0, mid_n_lt3, mid_n_lt0;
  int blowup, reserved;
};

// Per y-row partial reductions written by the diagnostics kernels.
struct DiagPart {
  double min_trc, cfl, esum, tsum;
  unsigned long long n_lt3, n_lt0;
  int nonfinite, big;
};

// ---- batched stage kernels
// Every stage kernel of the step takes a device table of per-member argument
// blocks (one block per simulation of a batch: a single run is a batch of
// one) and the member count.  blk0 is the first workgroup of the member in
// the launch; a workgroup finds its member by binary search, so members of
// different sizes share one launch (a ragged work list).

// x pencils (fft.hip).  Real FP64 buffers, or FP32 with the mixed
// mean/fluctuation products (mean = [n_means][M+1] FP64 profiles); in mixed
// 2D, mcol receives the FP64-completed kx = 0 column of each output.
struct XArgs {
  const void* in;
  void* out;
  int nrows, nkx, m1, pz;
  FftPlan pl;
  const double* kx;
  const void* tw;
  double eps_wi;
  const double* mean;
  double* mcol;
  const int* skip;  // the run's blow-up flag: nonzero skips its work (as in every stage kernel)
  int blk0;
};
// z columns (fft.hip): workgroups (kx group, row, field) flattened; the
// forward mixed transform writes the FP64-completed kx = kz = 0 value of each
// output into mcol ([nfields][rows]) using the mean profiles.
struct ZArgs {
  const void* in;
  void* out;
  int nkx, nzs, rows, nfields, ngx, inverse;
  FftPlan pl;
  const int* src_field;
  const int* deriv;
  // npair > 0: output fields nfields - npair + k are d/dz of fields k < npair;
  // the two workgroups of a (field, row, kx group) of such a pair are block
  // indices 8 apart (one XCD, dispatched together), so the second reads the
  // shared input from that XCD's L2
  int npair;
  const double* kz;
  const void* tw;
  const double* mean;
  double* mcol;
  double eps_wi;  // sPTT eps / Wi: its mean product enters the FP64 mean column
  const int* skip;
  int blk0;
};
// diagnostics (fft.hip): per (y_j, z) line of the base grid, from the
// spectral Tr c, u, v, w (in: [4][N+1][zrows][kx]), then one workgroup per
// member for the step record.
constexpr int HIST_MAX = 4096;  // largest number of histogram bins
constexpr int HIST_Q = 8;       // histogrammed midplane quantities
struct DRowArgs {
  Dims d;
  const double* in;
  int zrows;
  FftPlan pl;
  const double* tw;
  const double* ydy;
  const double* kx;
  DiagPart* parts;
  // midplane histograms of quantity q = Tr c, u - U(0), v, w - W(0), d_x u,
  // d_z u, d_x w, d_z w (hbins[q] = 0: off), counts at hist + q (HIST_MAX + 2):
  // [0] below hlo, [1 + floor((v - hlo) hscale)] inside, [hbins + 1] at or
  // above the top and non-finite values; umean / wmean: the mean-mode u and w
  // at the midplane; zgrad (3D): d_z u and d_z w of the midplane row,
  // [2][z][kx] (physical in z, spectral in x); mparts: per midplane line z
  // and quantity, the count, sum and sum of squares of its finite samples
  unsigned long long* hist;
  double hlo[HIST_Q], hscale[HIST_Q];
  int hbins[HIST_Q];
  const double *umean, *wmean, *zgrad;
  double* mparts;  // [zrows][HIST_Q][3]
  const int* skip;
  int blk0;
};
struct DFinArgs {
  Dims d;
  Phys p;
  const DiagPart* parts;
  int zrows;
  const double* w;
  DevScalars* sc;
  DiagRec* ring;
  int cap;
  // running moments of the histogrammed midplane quantities: msum[q] +=
  // the sums of mparts over the midplane lines, for q with bit q of mom_mask
  const double* mparts;
  double* msum;  // [HIST_Q][3]: samples, sum, sum of squares
  int mom_mask;
};
// explicit assembly and CNAB2 right-hand sides (elem.hip); smean: mixed
// path only, [nout][N+1] FP64 projection of the kx = kz = 0 column of the
// explicit terms (null in FP64, where S holds it).
struct RhsArgs {
  Dims d;
  Phys p;
  const double *st, *D2buf, *Dc, *S, *smean, *DN, *kx, *kz, *d2i0, *d2in;
  double *R, *hvn, *hgn, *CB;
  double* qring;         // SBDF4: four slots of the state fields, q^k in slot k mod 4
  double* hring;         // SBDF4: four slots of the explicit terms, X^k in slot k mod 4
  const DevScalars* sc;  // step index n of the current state
  int blk0;
};
// rows of a right-hand-side launch (rhs_kernel's template argument): all
// (each thread computes the new wall values of c its row needs), the two
// wall rows (stored into CB), or the interior rows (reading them from CB
// after the wall launch)
enum { RHS_ALL = 0, RHS_WALLS = 1, RHS_INTERIOR = 2 };
// influence correction, flux, velocities, wall rows, history, diagnostics
// inputs (elem.hip)
struct FinArgs {
  Dims d;
  Phys p;
  const double *Zphi, *Zv, *Zg, *ZDv, *flux, *infl, *U1;  // Zg: g (3D) interior rows, else null
  double wU1;
  const double *CB, *hvn, *hgn, *S, *smean, *kx, *kz;
  double *st, *prep;
  DevScalars* sc;
  int blk0;
};

// Member of the current workgroup: the last m with args[m].blk0 <= blockIdx.x.
template <typename Args>
__device__ inline int member_of(const Args* __restrict__ a, int nmem) {
  const int b = blockIdx.x;
  int lo = 0, hi = nmem - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[mid].blk0 <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// precision 0: FP64; otherwise FP32 with the mixed products.  lds: dynamic
// LDS bytes (the largest member's need).  The launch shape is chosen once per
// launch from its largest member: threads per x-pencil workgroup
// (xpencil_threads of that LDS size and the launch's line count).
int xpencil_threads(int precision, size_t lds, int lines);
// 3D lines of the lengths 96, 192 and 384 can take the chunked pencil (the
// nine values and nine explicit terms of each point in registers, the other
// fields through LDS a chunk of field pairs at a time; xpencil_chunked says
// where it is used), with xpencil_chunk_threads() threads per workgroup,
// when every line of the launch has the same such length (chunk_len; 0: the
// whole-line pencil).
bool xpencil_chunked(int dim, int L, int precision);
int xpencil_chunk_threads();
void launch_xpencil(int dim, int precision, int threads, int chunk_len, const XArgs* args, int nmem, int blocks,
                    size_t lds, hipStream_t s);
// group: kx columns per workgroup (zfft_group), the same for every member of the launch
void launch_zfft(int precision, int group, const ZArgs* args, int nmem, int blocks, size_t lds, hipStream_t s);
void launch_diag_rows(const DRowArgs* args, int nmem, int blocks, size_t lds, hipStream_t s);
void launch_diag_final(const DFinArgs* args, int nmem, hipStream_t s);
// the wall rows of every member (walls, wblocks), then the interior rows
// (inner, iblocks); with wblocks == 0, inner covers all rows in one launch
void launch_rhs(const RhsArgs* walls, int wblocks, const RhsArgs* inner, int iblocks, int nmem, hipStream_t s);
void launch_finalize(const FinArgs* args, int nmem, int blocks, hipStream_t s);
// workgroups and dynamic LDS of one member's launch
int xpencil_blocks(const Dims& d);
size_t xpencil_lds_bytes(int dim, int L, int precision, bool chunked = false);
// kx columns per workgroup of z transforms of length L in a precision (0:
// FP64), the workgroups of one member's launch and their LDS
int zfft_group(int L, int precision);
int zfft_blocks(int nkx, int rows, int nfields, int group);
size_t zfft_lds_bytes(int L, int precision, int group);
size_t diag_rows_lds_bytes(int L);
constexpr int ELEM_THREADS = 64;
// Raises the dynamic-LDS limit of the transform kernels (call once, outside capture).
hipError_t fft_set_attributes();

// ---- init-time kernels (elem.hip), one simulation at a time
void launch_homog_rhs(const Dims& d, const Phys& p, const double* d2i0, const double* d2in, double* R,
                      hipStream_t s);
void launch_influence(const Dims& d, const double* Zphi, const double* Zv, const double* ZDv, const double* kz,
                      double* infl, double* U1, hipStream_t s);

}  // namespace pcs
