// Periodic-direction transforms, the fused physical-space products and the
// per-step diagnostics (FP64 path).
//
// Fourier in x and z with full 3/2-rule dealiasing (paper, Section 2): every
// retained mode is placed at its own frequency in a transform of 3/2 the base
// size, products are formed pointwise, and the forward transform is
// truncated back to the retained modes.  Transforms are mixed-radix (4, 2, 3)
// Stockham FFTs in LDS; two real fields share one complex transform
// (z = a + i b), which halves the transform count.
//
// x pencil: one workgroup per padded (y', z') line.  It reads the needed
// spectral fields of that line (kx modes), generates the d/dx variants by
// multiplying with i kx, runs the inverse transforms, evaluates
//   N_a  = - u_k d_k u_a                                       (eq. 2)
//   F_ab = - u_k d_k c_ab + (d_k u_a) c_kb + c_ak (d_k u_b)
//          - (eps/Wi) Tr(c - I)(c_ab - delta_ab)                (eq. 1)
// at every point, and writes the forward transforms of the outputs,
// truncated to the retained modes.  d_y v comes from continuity (eq. 3).
#include "kernels.hpp"

namespace pcs {

bool make_plan(int L, FftPlan* p) {
  p->L = L;
  p->npass = 0;
  int r = L;
  while (r % 4 == 0 && p->npass < 12) {
    p->radix[p->npass++] = 4;
    r /= 4;
  }
  while (r % 2 == 0 && p->npass < 12) {
    p->radix[p->npass++] = 2;
    r /= 2;
  }
  while (r % 3 == 0 && p->npass < 12) {
    p->radix[p->npass++] = 3;
    r /= 3;
  }
  return r == 1 && L >= 2;
}

namespace {

struct c2 {
  double x, y;
};
__device__ inline c2 operator+(c2 a, c2 b) { return c2{a.x + b.x, a.y + b.y}; }
__device__ inline c2 operator-(c2 a, c2 b) { return c2{a.x - b.x, a.y - b.y}; }
__device__ inline c2 cmul(c2 a, c2 b) { return c2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline c2 scal(double s, c2 a) { return c2{s * a.x, s * a.y}; }

// In-LDS R-point DFT, R in {2, 3, 4}; sign -1 forward, +1 inverse.
__device__ inline void butterfly(c2* v, int R, int sign) {
  if (R == 2) {
    c2 t = v[0];
    v[0] = t + v[1];
    v[1] = t - v[1];
  } else if (R == 4) {
    c2 a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = v[1] - v[3];
    c2 sid = sign > 0 ? c2{-d.y, d.x} : c2{d.y, -d.x};  // (sign i) d
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + sid;
    v[3] = b - sid;
  } else {
    const double h = 0.86602540378443864676 * sign;  // sign * sqrt(3)/2
    c2 t1 = v[1] + v[2];
    c2 t2 = v[0] - scal(0.5, t1);
    c2 t3 = scal(h, v[1] - v[2]);
    c2 it3 = c2{-t3.y, t3.x};
    v[0] = v[0] + t1;
    v[1] = t2 + it3;
    v[2] = t2 - it3;
  }
}

// Stockham passes over nseq sequences of length L stored contiguously at a;
// b is the partner buffer.  Returns the buffer holding the result (a after an
// even number of passes, b after an odd one).  tw[m] = exp(-2 pi i m / L).
__device__ c2* lds_fft(c2* a, c2* b, const FftPlan& pl, int nseq, const c2* __restrict__ tw, int sign) {
  const int L = pl.L;
  int Ns = 1;
  c2* in = a;
  c2* out = b;
  for (int ps = 0; ps < pl.npass; ++ps) {
    const int R = pl.radix[ps], LR = L / R, stride = L / (Ns * R);
    for (int idx = threadIdx.x; idx < nseq * LR; idx += blockDim.x) {
      const int s = idx / LR, j = idx - s * LR;
      const c2* src = in + (size_t)s * L;
      c2* dst = out + (size_t)s * L;
      const int k = j % Ns;
      c2 v[4];
      for (int r = 0; r < R; ++r) v[r] = src[j + r * LR];
      if (Ns > 1)
        for (int r = 1; r < R; ++r) {
          c2 w = tw[r * k * stride];
          if (sign > 0) w.y = -w.y;
          v[r] = cmul(v[r], w);
        }
      butterfly(v, R, sign);
      const int base = (j - k) * R + k;
      for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
    }
    __syncthreads();
    c2* t = in;
    in = out;
    out = t;
    Ns *= R;
  }
  return in;
}

// Source table of the real fields fed to the x transforms: field index in
// the [field][row][kx] input buffer and whether d/dx is applied.
struct XTable {
  int nreal, npairs, nout, nopairs;
  short src[36];
  short dx[36];
};

// index of c_ab in the stored list (2D: xx xy yy; 3D: xx xy xz yy yz zz)
__device__ inline int cidx(int dim, int a, int b) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  if (dim == 2) return (a == 0) ? b : 2;
  return (a == 0) ? b : (a == 1 ? 2 + b : 5);
}

// Products of eqs. (1)-(2) at one point.  Real-field order:
//  2D: u v ux uy vx | cxx cxy cyy | dx c (3) | dy c (3)
//  3D: u v w | c (6) | dx u v w | dx c (6) | dy u, dy w | dy c (6) | dz u v w | dz c (6)
// Outputs: N_x N_y (N_z) F_ab (stored components).
template <int DIM>
__device__ inline void pointwise(const double* r, double* o, double eps_wi) {
  double u[3], du[3][3], c[3][3], dc[3][6];
  const int nc = DIM == 2 ? 3 : 6;
  if (DIM == 2) {
    u[0] = r[0];
    u[1] = r[1];
    du[0][0] = r[2];
    du[1][0] = r[3];
    du[0][1] = r[4];
    du[1][1] = -r[2];
    for (int q = 0; q < 3; ++q) {
      dc[0][q] = r[8 + q];
      dc[1][q] = r[11 + q];
    }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) c[a][b] = r[5 + cidx(2, a, b)];
  } else {
    for (int a = 0; a < 3; ++a) {
      u[a] = r[a];
      du[0][a] = r[9 + a];
      du[2][a] = r[26 + a];
    }
    du[1][0] = r[18];
    du[1][2] = r[19];
    du[1][1] = -(r[9] + r[28]);
    for (int q = 0; q < 6; ++q) {
      dc[0][q] = r[12 + q];
      dc[1][q] = r[20 + q];
      dc[2][q] = r[29 + q];
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) c[a][b] = r[3 + cidx(3, a, b)];
  }
  for (int a = 0; a < DIM; ++a) {
    double s = 0;
    for (int k = 0; k < DIM; ++k) s += u[k] * du[k][a];
    o[a] = -s;
  }
  double tr = 0;
  for (int a = 0; a < DIM; ++a) tr += c[a][a] - 1.0;
  for (int a = 0, q = 0; a < DIM; ++a)
    for (int b = a; b < DIM; ++b, ++q) {
      double f = 0;
      for (int k = 0; k < DIM; ++k) f += -u[k] * dc[k][q] + du[k][a] * c[k][b] + c[a][k] * du[k][b];
      if (eps_wi != 0.0) f -= eps_wi * tr * (c[a][b] - (a == b ? 1.0 : 0.0));
      o[DIM + q] = f;
    }
  (void)nc;
}

template <int DIM>
__global__ __launch_bounds__(256) void xpencil_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                      int nrows, int nkx, FftPlan pl, const double* __restrict__ kx,
                                                      const c2* __restrict__ tw, XTable tab, int S, double eps_wi) {
  extern __shared__ double smem_d[];
  c2* P = reinterpret_cast<c2*>(smem_d);
  const int L = pl.L;
  c2* Tm = P + (size_t)tab.npairs * L;
  const int row = blockIdx.x, tid = threadIdx.x;
  const size_t fstride = (size_t)nrows * nkx * 2;
  const double* base = in + (size_t)row * nkx * 2;
  const bool odd = (pl.npass & 1) != 0;
  for (int b0 = 0; b0 < tab.npairs; b0 += S) {
    const int nb = min(S, tab.npairs - b0);
    c2* X = odd ? Tm : P + (size_t)b0 * L;
    c2* Y = odd ? P + (size_t)b0 * L : Tm;
    for (int e = tid; e < nb * L; e += blockDim.x) X[e] = c2{0, 0};
    __syncthreads();
    for (int e = tid; e < nb * nkx; e += blockDim.x) {
      const int q = e / nkx, k = e - q * nkx;
      c2 A{0, 0}, B{0, 0};
      const int fa = 2 * (b0 + q), fb = fa + 1;
      const double kk = kx[k];
      if (fa < tab.nreal) {
        const double* p = base + tab.src[fa] * fstride + 2 * k;
        A = c2{p[0], p[1]};
        if (tab.dx[fa]) A = c2{-kk * A.y, kk * A.x};
      }
      if (fb < tab.nreal) {
        const double* p = base + tab.src[fb] * fstride + 2 * k;
        B = c2{p[0], p[1]};
        if (tab.dx[fb]) B = c2{-kk * B.y, kk * B.x};
      }
      c2* Xq = X + (size_t)q * L;
      if (k == 0) {
        Xq[0] = c2{A.x, B.x};
      } else {
        Xq[k] = c2{A.x - B.y, A.y + B.x};
        Xq[L - k] = c2{A.x + B.y, B.x - A.y};
      }
    }
    __syncthreads();
    lds_fft(X, Y, pl, nb, tw, +1);
  }
  // pointwise products; outputs overwrite the first pairs at the same point
  for (int n = tid; n < L; n += blockDim.x) {
    double r[36], o[10];
    for (int f = 0; f < tab.nreal; ++f) {
      const c2 z = P[(size_t)(f >> 1) * L + n];
      r[f] = (f & 1) ? z.y : z.x;
    }
    pointwise<DIM>(r, o, eps_wi);
    o[tab.nout] = 0.0;
    for (int q = 0; q < tab.nopairs; ++q) P[(size_t)q * L + n] = c2{o[2 * q], o[2 * q + 1]};
  }
  __syncthreads();
  const double inv = 1.0 / L;
  double* obase = out + (size_t)row * nkx * 2;
  for (int q0 = 0; q0 < tab.nopairs; q0 += S) {
    const int nb = min(S, tab.nopairs - q0);
    const c2* res = lds_fft(P + (size_t)q0 * L, Tm, pl, nb, tw, -1);
    for (int e = tid; e < nb * nkx; e += blockDim.x) {
      const int q = e / nkx, k = e - q * nkx;
      const c2* Rq = res + (size_t)q * L;
      const c2 Zk = Rq[k];
      c2 A, B;
      if (k == 0) {
        A = c2{Zk.x, 0};
        B = c2{Zk.y, 0};
      } else {
        const c2 Zc = Rq[L - k];
        A = c2{0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y - Zc.y)};
        B = c2{0.5 * (Zk.y + Zc.y), -0.5 * (Zk.x - Zc.x)};
      }
      const int fa = 2 * (q0 + q), fb = fa + 1;
      double* pa = obase + (size_t)fa * fstride + 2 * k;
      pa[0] = A.x * inv;
      pa[1] = A.y * inv;
      if (fb < tab.nout) {
        double* pb = obase + (size_t)fb * fstride + 2 * k;
        pb[0] = B.x * inv;
        pb[1] = B.y * inv;
      }
    }
    __syncthreads();
  }
}

XTable table2d() {
  XTable t{};
  const short src[14] = {0, 1, 0, 5, 1, 2, 3, 4, 2, 3, 4, 6, 7, 8};
  const short dx[14] = {0, 0, 1, 0, 1, 0, 0, 0, 1, 1, 1, 0, 0, 0};
  t.nreal = 14;
  t.npairs = 7;
  t.nout = 5;
  t.nopairs = 3;
  for (int i = 0; i < 14; ++i) {
    t.src[i] = src[i];
    t.dx[i] = dx[i];
  }
  return t;
}

XTable table3d() {
  XTable t{};
  int n = 0;
  auto add = [&](int s, int d) {
    t.src[n] = (short)s;
    t.dx[n] = (short)d;
    ++n;
  };
  for (int f = 0; f < 9; ++f) add(f, 0);       // u v w c6
  for (int f = 0; f < 9; ++f) add(f, 1);       // dx u v w, dx c6
  add(9, 0);                                   // dy u
  add(10, 0);                                  // dy w
  for (int f = 11; f < 17; ++f) add(f, 0);     // dy c6
  for (int f = 17; f < 26; ++f) add(f, 0);     // dz u v w, dz c6
  t.nreal = n;                                 // 35
  t.npairs = (n + 1) / 2;
  t.nout = 9;
  t.nopairs = 5;
  return t;
}

size_t xpencil_lds(int npairs, int L, int S) { return (size_t)(npairs + S) * L * sizeof(c2); }

int pick_batch(int npairs, int L) {
  const size_t budget = 160 * 1024;
  int S = npairs;
  while (S > 1 && xpencil_lds(npairs, L, S) > budget) --S;
  return S;
}

}  // namespace

void launch_xpencil(const Dims& d, const Phys& p, const FftPlan& plan, const double* yin, double* yout,
                    const double* kx, const double* tw, hipStream_t s) {
  // 2D: rows are the padded y points
  XTable t = table2d();
  const int S = pick_batch(t.npairs, plan.L);
  const size_t lds = xpencil_lds(t.npairs, plan.L, S);
  hipLaunchKernelGGL(xpencil_kernel<2>, dim3(d.M + 1), dim3(256), lds, s, yin, yout, d.M + 1, d.nkx, plan, kx,
                     reinterpret_cast<const c2*>(tw), t, S, p.eps / p.wi);
}

void launch_xpencil3d(const Dims& d, const Phys& p, const FftPlan& plan, const double* zin, double* zout,
                      const double* kx, const double* tw, hipStream_t s) {
  XTable t = table3d();
  const int S = pick_batch(t.npairs, plan.L);
  const size_t lds = xpencil_lds(t.npairs, plan.L, S);
  const int rows = (d.M + 1) * d.pz;
  hipLaunchKernelGGL(xpencil_kernel<3>, dim3(rows), dim3(256), lds, s, zin, zout, rows, d.nkx, plan, kx,
                     reinterpret_cast<const c2*>(tw), t, S, p.eps / p.wi);
}

// ---------------------------------------------------------------- z columns
// Complex transforms along the spanwise index of [field][y][z row][kx] data.
// inverse: kz slots (Nyquist slot skipped, optional i kz factor) are placed at
// their own frequency in a length-Lz transform; forward: length-Lz data is
// transformed, divided by Lz and truncated to the retained slots.
constexpr int ZG = 8;  // kx columns per workgroup

namespace {
__global__ __launch_bounds__(256) void zfft_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                   int nkx, int nzs, int rows_y, FftPlan pl,
                                                   const int* __restrict__ src_field, const int* __restrict__ deriv,
                                                   const double* __restrict__ kz, const c2* __restrict__ tw,
                                                   int inverse) {
  extern __shared__ double smem_z[];
  c2* A = reinterpret_cast<c2*>(smem_z);
  const int L = pl.L;
  c2* B = A + (size_t)ZG * L;
  const int k0 = blockIdx.x * ZG, i = blockIdx.y, f = blockIdx.z;
  const int ng = min(ZG, nkx - k0);
  const int tid = threadIdx.x;
  const int rin = inverse ? nzs : L, rout = inverse ? L : nzs;
  const int sf = src_field ? src_field[f] : f;
  const int dz = deriv ? deriv[f] : 0;
  const double* ib = in + ((size_t)sf * rows_y + i) * rin * nkx * 2;
  double* ob = out + ((size_t)f * rows_y + i) * rout * nkx * 2;
  for (int e = tid; e < ZG * L; e += blockDim.x) A[e] = c2{0, 0};
  __syncthreads();
  if (inverse) {
    for (int e = tid; e < nzs * ng; e += blockDim.x) {
      const int s = e / ng, g = e - s * ng;
      if (nzs > 1 && s == nzs / 2) continue;
      const int mz = (s < nzs / 2) ? s : s - nzs;
      c2 v = c2{ib[((size_t)s * nkx + k0 + g) * 2], ib[((size_t)s * nkx + k0 + g) * 2 + 1]};
      if (dz) {
        const double kk = kz[s];
        v = c2{-kk * v.y, kk * v.x};
      }
      A[(size_t)g * L + ((mz % L) + L) % L] = v;
    }
  } else {
    for (int e = tid; e < L * ng; e += blockDim.x) {
      const int z = e / ng, g = e - z * ng;
      A[(size_t)g * L + z] = c2{ib[((size_t)z * nkx + k0 + g) * 2], ib[((size_t)z * nkx + k0 + g) * 2 + 1]};
    }
  }
  __syncthreads();
  const c2* R = lds_fft(A, B, pl, ng, tw, inverse ? +1 : -1);
  if (inverse) {
    for (int e = tid; e < L * ng; e += blockDim.x) {
      const int z = e / ng, g = e - z * ng;
      const c2 v = R[(size_t)g * L + z];
      ob[((size_t)z * nkx + k0 + g) * 2] = v.x;
      ob[((size_t)z * nkx + k0 + g) * 2 + 1] = v.y;
    }
  } else {
    const double inv = 1.0 / L;
    for (int e = tid; e < nzs * ng; e += blockDim.x) {
      const int s = e / ng, g = e - s * ng;
      c2 v{0, 0};
      if (!(nzs > 1 && s == nzs / 2)) {
        const int mz = (s < nzs / 2) ? s : s - nzs;
        v = scal(inv, R[(size_t)g * L + ((mz % L) + L) % L]);
      }
      ob[((size_t)s * nkx + k0 + g) * 2] = v.x;
      ob[((size_t)s * nkx + k0 + g) * 2 + 1] = v.y;
    }
  }
}
}  // namespace

void launch_zfft(const Dims& d, const FftPlan& plan, const double* in, double* out, int nfields,
                 const int* src_field, const int* deriv, const double* kz, const double* tw, int inverse, int rows,
                 hipStream_t s) {
  const size_t lds = 2 * (size_t)ZG * plan.L * sizeof(c2);
  dim3 grid((d.nkx + ZG - 1) / ZG, rows, nfields);
  hipLaunchKernelGGL(zfft_kernel, grid, dim3(256), lds, s, in, out, d.nkx, d.nzs, rows, plan, src_field, deriv, kz,
                     reinterpret_cast<const c2*>(tw), inverse);
}

// ---------------------------------------------------------------- diagnostics
// Base-grid values of Tr c, u, v, w on every (y_j, z) line: spectral Tr c =
// c_xx + c_yy (+ c_zz) is formed first (2D adds the constant c_zz = 1 after
// the transform), then the inverse x transform.  Per line: min Tr c, counts of
// Tr c < 3 and < 0 (strict), max CFL contribution |u|/dx + |v|/dy_j + |w|/dz,
// sums of |u|^2/2 and Tr c, and non-finite / |Tr c| > 1e12 flags.
namespace {

__global__ void diag_prep_kernel(Dims d, const double* __restrict__ st, double* __restrict__ outb) {
  const int n1 = d.N + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n1 * d.nm) return;
  const size_t fs = (size_t)n1 * d.cw;
  const size_t off = (size_t)(e / d.nm) * d.cw + 2 * (e % d.nm);
  const int FC = d.dim == 2 ? 3 : 5;
  double tr_r, tr_i;
  if (d.dim == 2) {
    tr_r = st[(FC + 0) * fs + off] + st[(FC + 2) * fs + off];
    tr_i = st[(FC + 0) * fs + off + 1] + st[(FC + 2) * fs + off + 1];
  } else {
    tr_r = st[(FC + 0) * fs + off] + st[(FC + 3) * fs + off] + st[(FC + 5) * fs + off];
    tr_i = st[(FC + 0) * fs + off + 1] + st[(FC + 3) * fs + off + 1] + st[(FC + 5) * fs + off + 1];
  }
  outb[off] = tr_r;
  outb[off + 1] = tr_i;
  const int nv = d.dim == 2 ? 2 : 3;
  for (int q = 0; q < nv; ++q) {
    outb[(q + 1) * fs + off] = st[q * fs + off];
    outb[(q + 1) * fs + off + 1] = st[q * fs + off + 1];
  }
}

__global__ __launch_bounds__(256) void diag_rows_kernel(Dims d, Phys p, const double* __restrict__ in, int zrows,
                                                        FftPlan pl, const c2* __restrict__ tw,
                                                        const double* __restrict__ ydy, DiagPart* __restrict__ parts) {
  extern __shared__ double smem_g[];
  c2* A = reinterpret_cast<c2*>(smem_g);
  const int L = pl.L, nkx = d.nkx;
  c2* B = A + 2 * (size_t)L;
  __shared__ double rmin[256], rcfl[256], re[256], rt[256];
  __shared__ unsigned long long c3[256], c0[256];
  __shared__ int rnf[256], rbig[256];
  const int row = blockIdx.x, tid = threadIdx.x;
  const int nrows = (d.N + 1) * zrows;
  const int j = row / zrows;
  const size_t fstride = (size_t)nrows * nkx * 2;
  const double* base = in + (size_t)row * nkx * 2;
  const bool odd = (pl.npass & 1) != 0;
  c2* X = odd ? B : A;
  c2* Y = odd ? A : B;
  for (int e = tid; e < 2 * L; e += blockDim.x) X[e] = c2{0, 0};
  __syncthreads();
  const int nf = d.dim == 2 ? 3 : 4;
  for (int e = tid; e < 2 * nkx; e += blockDim.x) {
    const int q = e / nkx, k = e - q * nkx;
    const int fa = 2 * q, fb = fa + 1;
    c2 Av{0, 0}, Bv{0, 0};
    if (fa < nf) Av = c2{base[fa * fstride + 2 * k], base[fa * fstride + 2 * k + 1]};
    if (fb < nf) Bv = c2{base[fb * fstride + 2 * k], base[fb * fstride + 2 * k + 1]};
    c2* Xq = X + (size_t)q * L;
    if (k == 0) {
      Xq[0] = c2{Av.x, Bv.x};
    } else {
      Xq[k] = c2{Av.x - Bv.y, Av.y + Bv.x};
      Xq[L - k] = c2{Av.x + Bv.y, Bv.x - Av.y};
    }
  }
  __syncthreads();
  lds_fft(X, Y, pl, 2, tw, +1);  // result in A
  const double dx = d.lx / d.nx, dz = d.dim == 3 ? d.lz / d.nz : 1.0;
  const double dyj = ydy[j];
  double mn = 1.0 / 0.0, cf = 0, es = 0, ts = 0;
  unsigned long long n3 = 0, n0 = 0;
  int nfin = 0, big = 0;
  for (int n = tid; n < L; n += blockDim.x) {
    const c2 z0 = A[n], z1 = A[L + n];
    const double trc = z0.x + (d.dim == 2 ? 1.0 : 0.0);
    const double u = z0.y, v = z1.x, w = d.dim == 3 ? z1.y : 0.0;
    mn = fmin(mn, trc);
    n3 += (trc < 3.0);
    n0 += (trc < 0.0);
    double c = fabs(u) / dx + fabs(v) / dyj;
    if (d.dim == 3) c += fabs(w) / dz;
    cf = fmax(cf, c);
    es += 0.5 * (u * u + v * v + w * w);
    ts += trc;
    nfin |= !(isfinite(trc) && isfinite(u) && isfinite(v) && isfinite(w));
    big |= (fabs(trc) > 1.0e12);
  }
  rmin[tid] = mn;
  rcfl[tid] = cf;
  re[tid] = es;
  rt[tid] = ts;
  c3[tid] = n3;
  c0[tid] = n0;
  rnf[tid] = nfin;
  rbig[tid] = big;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (tid < h) {
      rmin[tid] = fmin(rmin[tid], rmin[tid + h]);
      rcfl[tid] = fmax(rcfl[tid], rcfl[tid + h]);
      re[tid] += re[tid + h];
      rt[tid] += rt[tid + h];
      c3[tid] += c3[tid + h];
      c0[tid] += c0[tid + h];
      rnf[tid] |= rnf[tid + h];
      rbig[tid] |= rbig[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    DiagPart q;
    q.min_trc = rmin[0];
    q.cfl = rcfl[0];
    q.esum = re[0];
    q.tsum = rt[0];
    q.n_lt3 = c3[0];
    q.n_lt0 = c0[0];
    q.nonfinite = rnf[0];
    q.big = rbig[0];
    parts[row] = q;
  }
}

__global__ __launch_bounds__(256) void diag_final_kernel(Dims d, Phys p, const DiagPart* __restrict__ parts,
                                                         int zrows, const double* __restrict__ w,
                                                         DevScalars* __restrict__ sc, DiagRec* __restrict__ ring,
                                                         int cap) {
  __shared__ double smin[256], smmin[256], scfl[256], se[256], st_[256];
  __shared__ unsigned long long s3[256], s0[256], sm3[256], sm0[256];
  __shared__ int sb[256];
  const int tid = threadIdx.x;
  const int n1 = d.N + 1, nrows = n1 * zrows, mid = d.N / 2;
  const double norm = 1.0 / ((double)d.nx * (d.dim == 3 ? d.nz : 1));
  double mn = 1.0 / 0.0, mmn = 1.0 / 0.0, cf = 0, es = 0, ts = 0;
  unsigned long long n3 = 0, n0 = 0, m3 = 0, m0 = 0;
  int b = 0;
  for (int r = tid; r < nrows; r += blockDim.x) {
    const DiagPart q = parts[r];
    const int j = r / zrows;
    const double wj = 0.5 * w[j] * norm;
    mn = fmin(mn, q.min_trc);
    cf = fmax(cf, q.cfl);
    es += wj * q.esum;
    ts += wj * q.tsum;
    n3 += q.n_lt3;
    n0 += q.n_lt0;
    if (j == mid) {
      mmn = fmin(mmn, q.min_trc);
      m3 += q.n_lt3;
      m0 += q.n_lt0;
    }
    b |= q.nonfinite | q.big;
  }
  smin[tid] = mn;
  smmin[tid] = mmn;
  scfl[tid] = cf;
  se[tid] = es;
  st_[tid] = ts;
  s3[tid] = n3;
  s0[tid] = n0;
  sm3[tid] = m3;
  sm0[tid] = m0;
  sb[tid] = b;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (tid < h) {
      smin[tid] = fmin(smin[tid], smin[tid + h]);
      smmin[tid] = fmin(smmin[tid], smmin[tid + h]);
      scfl[tid] = fmax(scfl[tid], scfl[tid + h]);
      se[tid] += se[tid + h];
      st_[tid] += st_[tid + h];
      s3[tid] += s3[tid + h];
      s0[tid] += s0[tid + h];
      sm3[tid] += sm3[tid + h];
      sm0[tid] += sm0[tid + h];
      sb[tid] |= sb[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const long long step = sc->step + 1;
    const double t = sc->t + p.dt;
    DiagRec r;
    r.step = step;
    r.t = t;
    r.min_trc = smin[0];
    r.mid_min_trc = smmin[0];
    r.cfl = p.dt * scfl[0];
    r.dpdx = sc->pi;
    r.energy = se[0];
    r.mean_trc = st_[0];
    r.n_lt3 = s3[0];
    r.n_lt0 = s0[0];
    r.mid_n_lt3 = sm3[0];
    r.mid_n_lt0 = sm0[0];
    r.blowup = sb[0] ? 1 : 0;
    r.reserved = 0;
    ring[(step - 1) % cap] = r;
    sc->step = step;
    sc->t = t;
    sc->blowup |= r.blowup;
  }
}

}  // namespace

void launch_diag_rows(const Dims& d, const Phys& p, const FftPlan& planx, const double* st, double* prep,
                      double* zbuf, const FftPlan& planz, const double* twx, const double* twz, const double* ydy,
                      DiagPart* parts, hipStream_t s) {
  const int n1 = d.N + 1;
  const int n = n1 * d.nm;
  hipLaunchKernelGGL(diag_prep_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, st, prep);
  const double* src = prep;
  int zrows = 1;
  if (d.dim == 3) {
    launch_zfft(d, planz, prep, zbuf, 4, nullptr, nullptr, nullptr, twz, 1, n1, s);
    src = zbuf;
    zrows = d.nz;
  }
  const size_t lds = 4 * (size_t)planx.L * sizeof(c2);
  hipLaunchKernelGGL(diag_rows_kernel, dim3(n1 * zrows), dim3(256), lds, s, d, p, src, zrows, planx,
                     reinterpret_cast<const c2*>(twx), ydy, parts);
}

hipError_t fft_set_attributes() {
  const int lim = 160 * 1024;
  hipError_t e = hipFuncSetAttribute((const void*)xpencil_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)xpencil_kernel<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)zfft_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  // the row-diagnostics kernel also holds ~14 KB of static LDS for its reductions
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)diag_rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
  return e;
}

size_t xpencil_lds_bytes(int dim, int L) {
  XTable t = dim == 2 ? table2d() : table3d();
  return xpencil_lds(t.npairs, L, pick_batch(t.npairs, L));
}

void launch_diag_final(const Dims& d, const Phys& p, const DiagPart* parts, const double* w, DevScalars* sc,
                       DiagRec* ring, int ring_cap, hipStream_t s) {
  const int zrows = d.dim == 3 ? d.nz : 1;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, d, p, parts, zrows, w, sc, ring, ring_cap);
}

}  // namespace pcs
