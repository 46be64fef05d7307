// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcs {

// One dense product C = alpha * A * B + beta * C, real.  A (m x k) is stored
// row-major in the compute precision, A[i][kk] at A[i * lda + kk], with
// lda = gemm_lda(k) and gemm_rows(m) rows allocated, all padding zero (the
// kernels read whole 16-wide k blocks and row tiles of A unguarded).
// B (k x n) and C (m x n) are row-major, each in its own precision (see
// GemmType).  Complex fields (re/im interleaved) are multiplied by a real
// operator by treating each complex column as two real columns.
struct EigScale;
struct GemmJob {
  const void* A;
  const void* B;
  void* C;
  void* C2;  // optional second output: alpha A B scaled by scale2 (no beta term)
  int m, n, k, lda, ldb, ldc;
  double alpha, beta;
  int flags;           // GEMM_ZERO_MEAN: B columns 0 and 1 (the kx = kz = 0 mode) read as zero
  int scale, scale2;   // SCALE_*: output row i is eigen coefficient i, scaled per mode
  const EigScale* es;  // per-solve constants for the scaling
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
  double dt, nu, wi, kappa;
};

// compute / B / C precisions: D = double, F = float
enum GemmType { GEMM_DDD = 0, GEMM_FDF, GEMM_FFD, GEMM_DDF, GEMM_DFD, GEMM_NTYPES };

constexpr int MAX_JOBS = 64;
// Tile configurations.  Register-direct kernel (operand fragments loaded
// straight into registers, no LDS in the loop): 0: 32 x 32 with K split over
// the four waves, 1: 64 x 32 and 2: 32 x 64 with K split in two, 3: 64 x 64.
// LDS-tiled kernel (operand chunks shared by the four waves through LDS):
// 4: 32 x 32, 5: 64 x 32, 6: 64 x 64, 7: 128 x 64.
constexpr int GEMM_NCFG = 8;
inline int gemm_lda(int k) { return (k + 15) & ~15; }
inline int gemm_rows(int m) { return (m + 127) & ~127; }

// Fills tiles_m / tile0 for tile configuration cfg and returns the total
// number of workgroups.
int gemm_prepare(GemmJob* jobs, int njobs, int cfg);
void gemm_run(GemmType t, const GemmJob* dev_jobs, int total_tiles, int njobs, int cfg, hipStream_t s);
hipError_t gemm_set_attributes();

// Mixed-radix (4, 2, 3) Stockham plan for a length L = 2^a 3^b.
struct FftPlan {
  int L = 0;
  int npass = 0;
  int radix[12] = {0};
};
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
};

// Device-resident scalars advanced by the step itself.
struct DevScalars {
  long long step;
  double t;
  double pi;
  int blowup;
  int pad;
};

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

// ---- launchers (fft.hip)
// precision 0: FP64 buffers and products; otherwise FP32 buffers, the mixed
// mean/fluctuation products and `mean` = [n_means][M+1] FP64 profiles.
void launch_xpencil(const Dims& d, const Phys& p, const FftPlan& plan, const void* in, void* out, const double* kx,
                    const void* tw, int precision, const double* mean, double* mcol, hipStream_t s);
// mcol (mixed forward only, else null): [nfields][rows] FP64 kx = kz = 0 column
// of the output plus the product of the mean profiles `mean`.
void launch_zfft(const Dims& d, const FftPlan& plan, const void* in, void* out, int nfields, const int* src_field,
                 const int* deriv, const double* kz, const void* tw, int inverse, int rows, int precision,
                 const double* mean, double* mcol, hipStream_t s);
// prep: [4][N+1][kz][kx] spectral Tr c, u, v, w written by the finalize kernel
void launch_diag_rows(const Dims& d, const FftPlan& planx, const double* prep, double* zbuf, const FftPlan& planz,
                      const double* twx, const double* twz, const double* ydy, DiagPart* parts, hipStream_t s);
void launch_diag_final(const Dims& d, const Phys& p, const DiagPart* parts, const double* w, DevScalars* sc,
                       DiagRec* ring, int ring_cap, hipStream_t s);
// Raises the dynamic-LDS limit of the transform kernels (call once, outside capture).
hipError_t fft_set_attributes();
size_t xpencil_lds_bytes(int dim, int L, int precision);

// ---- launchers (elem.hip)
// smean: mixed path only, [nout][N+1] FP64 projection of the kx = kz = 0
// column of the explicit terms (null in FP64, where S holds it).
void launch_rhs(const Dims& d, const Phys& p, const double* state, const double* D2buf, const double* Dc,
                const double* S, const double* smean, const double* DN, const double* kx, const double* kz,
                const double* d2i0, const double* d2in, double* R, double* hvn, double* hgn, double* CB,
                hipStream_t s);
void launch_finalize(const Dims& d, const Phys& p, const double* Zphi, const double* Zv, const double* ZDv,
                     const double* flux, const double* infl, const double* U1, double wU1, const double* CB,
                     const double* hvn, const double* hgn, const double* S, const double* smean, const double* kx,
                     const double* kz, double* state, double* prep, DevScalars* sc, hipStream_t s);
void launch_homog_rhs(const Dims& d, const Phys& p, const double* d2i0, const double* d2in, double* R,
                      hipStream_t s);
void launch_influence(const Dims& d, const double* Zphi, const double* Zv, const double* ZDv, const double* kz,
                      double* infl, double* U1, hipStream_t s);

}  // namespace pcs
