// State resampling between resolutions (declared in include/pcs.h): the
// spectral re-interpolation of a flat state vector for restarts at another
// resolution.  The paper starts every run of Table 1 from one snapshot
// re-interpolated onto that run's grid (Section 2), and its conclusions
// propose short fine-grid runs started from snapshots of a long coarse run.
//
// Per field and Fourier mode, the values on the source Lobatto points
// y_j = cos(pi j / N) define the interpolating Chebyshev series
//   f(y) = sum_{n=0}^{N} a_n T_n(y),
//   a_n = (2 / (N c_n)) sum_j f_j T_n(y_j) / c_j,   c_0 = c_N = 2, else 1,
// which is truncated (or zero-padded) to degree min(N, N') and evaluated on
// the target Lobatto points.  Fourier modes keep their amplitude (a real
// field is sum_k qhat_k exp(i (kx x + kz z))): modes present at both
// resolutions are copied, the others are zero.  All of this is host work
// done once per restart, in extended precision, rounded once to FP64.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <thread>
#include <vector>

#include "../../include/pcs.h"

namespace {

bool grid_ok(const pcs_grid* g) {
  if (!g || (g->dim != 2 && g->dim != 3)) return false;
  if (g->nx < 4 || (g->nx & 1) || g->ny < 5 || !(g->ny & 1)) return false;
  if (g->dim == 2 && g->nz != 1) return false;
  if (g->dim == 3 && (g->nz < 4 || (g->nz & 1))) return false;
  return g->lx > 0 && (g->dim == 2 || g->lz > 0);
}

int nfields(int dim) { return dim == 2 ? 10 : 19; }
size_t per_field(const pcs_grid* g) { return (size_t)g->ny * (g->dim == 2 ? 1 : g->nz) * (g->nx / 2); }

// spanwise mode number of slot s at base size nz (0 for the Nyquist slot)
int mz_of_slot(int s, int nz) {
  if (nz == 1) return 0;
  if (s == nz / 2) return 0;
  return s < nz / 2 ? s : s - nz;
}
// slot of spanwise mode mz at base size nz, or -1 where it is not retained
int slot_of_mz(int mz, int nz) {
  if (nz == 1) return mz == 0 ? 0 : -1;
  if (mz >= nz / 2 || mz <= -nz / 2) return -1;
  return mz >= 0 ? mz : mz + nz;
}

// cos(pi k / K) for k = 0 .. 2K-1 (T_n at a Lobatto point is cos(pi n j / K),
// read at n j mod 2K)
std::vector<long double> cos_table(int K) {
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<long double> c(2 * (size_t)K);
  for (int k = 0; k < 2 * K; ++k) c[k] = std::cos(pi * (long double)k / K);
  return c;
}

// Q[(N'+1) x (N+1)]: values on the source points -> values of the truncated
// series on the target points
std::vector<double> cheb_resample_matrix(int N, int Np) {
  const int nmax = N < Np ? N : Np;
  const std::vector<long double> cs = cos_table(N), ct = cos_table(Np);
  std::vector<long double> C((size_t)(nmax + 1) * (N + 1));  // a_n = sum_j C[n][j] f_j
  for (int n = 0; n <= nmax; ++n)
    for (int j = 0; j <= N; ++j) {
      const long double cn = (n == 0 || n == N) ? 2.0L : 1.0L, cj = (j == 0 || j == N) ? 2.0L : 1.0L;
      C[(size_t)n * (N + 1) + j] = 2.0L / (N * cn * cj) * cs[((size_t)n * j) % (2 * (size_t)N)];
    }
  std::vector<double> Q((size_t)(Np + 1) * (N + 1));
  std::vector<long double> acc(N + 1);
  for (int i = 0; i <= Np; ++i) {
    std::fill(acc.begin(), acc.end(), 0.0L);
    for (int n = 0; n <= nmax; ++n) {
      const long double e = ct[((size_t)n * i) % (2 * (size_t)Np)];
      const long double* cr = &C[(size_t)n * (N + 1)];
      for (int j = 0; j <= N; ++j) acc[j] += e * cr[j];
    }
    for (int j = 0; j <= N; ++j) Q[(size_t)i * (N + 1) + j] = (double)acc[j];
  }
  return Q;
}

}  // namespace

extern "C" pcs_status pcs_resample_state(const pcs_grid* src, const double* sstate, size_t ns, const pcs_grid* dst,
                                         double* dstate, size_t nd) {
  if (!grid_ok(src) || !grid_ok(dst) || !sstate || !dstate || src->dim != dst->dim) return PCS_ERR_ARG;
  if (src->lx != dst->lx || (src->dim == 3 && src->lz != dst->lz)) return PCS_ERR_ARG;
  const int nf = nfields(src->dim);
  const size_t ps = per_field(src), pd = per_field(dst);
  if (ns != 4 + (size_t)nf * ps * 2 || nd != 4 + (size_t)nf * pd * 2) return PCS_ERR_ARG;
  const int N = src->ny - 1, Np = dst->ny - 1;
  const int nzs = src->dim == 2 ? 1 : src->nz, nzd = dst->dim == 2 ? 1 : dst->nz;
  const int nkxs = src->nx / 2, nkxd = dst->nx / 2;
  const std::vector<double> Q = cheb_resample_matrix(N, Np);
  for (int h = 0; h < 4; ++h) dstate[h] = sstate[h];
  // one field per task on a few host threads (fields are independent)
  auto field = [&](int f) {
    std::vector<double> col(2 * (size_t)(N + 1));
    const double* sf = sstate + 4 + (size_t)f * ps * 2;
    double* df = dstate + 4 + (size_t)f * pd * 2;
    for (int sd = 0; sd < nzd; ++sd) {
      const int ss = (nzd > 1 && sd == nzd / 2) ? -1 : slot_of_mz(mz_of_slot(sd, nzd), nzs);
      for (int k = 0; k < nkxd; ++k) {
        const bool have = ss >= 0 && k < nkxs;
        if (have)
          for (int j = 0; j <= N; ++j) {
            const size_t o = (((size_t)j * nzs + ss) * nkxs + k) * 2;
            col[2 * j] = sf[o];
            col[2 * j + 1] = sf[o + 1];
          }
        for (int i = 0; i <= Np; ++i) {
          double re = 0, im = 0;
          if (have)
            for (int j = 0; j <= N; ++j) {
              const double q = Q[(size_t)i * (N + 1) + j];
              re += q * col[2 * j];
              im += q * col[2 * j + 1];
            }
          const size_t o = (((size_t)i * nzd + sd) * nkxd + k) * 2;
          df[o] = re;
          df[o + 1] = im;
        }
      }
    }
  };
  const unsigned hw = std::thread::hardware_concurrency();
  const int nth = std::max(1, std::min<int>(nf, hw ? (int)std::min(hw, 16u) : 1));
  std::vector<std::thread> pool;
  int started = 1;  // threads 1 .. started-1 run; the calling thread covers the rest
  for (int t = 1; t < nth; ++t) {
    try {
      pool.emplace_back([&, t] {
        for (int f = t; f < nf; f += nth) field(f);
      });
      started = t + 1;
    } catch (...) {
      break;
    }
  }
  for (int f = 0; f < nf; ++f)
    if (f % nth == 0 || f % nth >= started) field(f);
  for (std::thread& th : pool) th.join();
  return PCS_OK;
}
