// Spectral elementwise stages of the CNAB2 step (FP64).
//
// Layout of every spectral field: [y row j][kz slot][kx] complex, re/im
// interleaved, i.e. a row-major (rows x cw) real matrix with
// cw = 2 * nzs * nkx.  One thread owns one complex element (j, mode) and all
// fields of it, so consecutive threads touch consecutive modes of one row.
//
// Equations (paper, Section 2): eq. (2) momentum with the polymer-stress
// divergence, handled through its curl-curl and curl (velocity-vorticity
// form, pressure eliminated); eq. (1) conformation update with the
// relaxation -(c - I)/Wi split into an implicit -c/Wi and a constant +I/Wi,
// polymer diffusion implicit in the interior and absent (kappa = 0) in the
// two wall rows (the wall condition of Section 2); eq. (3) exactly, through
// u = (i kx Dv - i kz g)/k^2 and w = (i kz Dv + i kx g)/k^2.
#include "kernels.hpp"

namespace pcs {

namespace {

struct Mode {
  int j, mode, iz, ix;
  double kx, kz, k2;
  bool mean, nyq;
};

template <typename P>
__device__ inline Mode decode(const Dims& d, int e, P kx, P kz) {
  Mode m;
  m.j = e / d.nm;
  m.mode = e - m.j * d.nm;
  m.iz = m.mode / d.nkx;
  m.ix = m.mode - m.iz * d.nkx;
  m.kx = kx[m.ix];
  m.kz = (d.dim == 3) ? kz[m.iz] : 0.0;
  m.k2 = m.kx * m.kx + m.kz * m.kz;
  m.mean = (m.mode == 0);
  m.nyq = (d.dim == 3) && (m.iz == d.nzs / 2);
  return m;
}

struct cd {
  double r, i;
};
template <typename P>
__device__ inline cd ld2(P f, size_t off) {
  return cd{f[off], f[off + 1]};
}
template <typename P>
__device__ inline void st2(P f, size_t off, cd v) {
  f[off] = v.r;
  f[off + 1] = v.i;
}
__device__ inline cd operator+(cd a, cd b) { return cd{a.r + b.r, a.i + b.i}; }
__device__ inline cd operator-(cd a, cd b) { return cd{a.r - b.r, a.i - b.i}; }
__device__ inline cd operator*(double s, cd a) { return cd{s * a.r, s * a.i}; }
__device__ inline cd ik(double k, cd a) { return cd{-k * a.i, k * a.r}; }  // (i k) a

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

struct Layout {
  int nq, nh, F_U, F_V, F_W, F_PHI, F_G, F_C, H_HV, H_HG, H_F, nsv, nsolve, S_F;
  __device__ Layout(int dim, int nc) {
    if (dim == 2) {
      nq = 6; nh = 4; F_U = 0; F_V = 1; F_W = -1; F_PHI = 2; F_G = -1; F_C = 3;
      H_HV = 6; H_HG = -1; H_F = 7; nsv = 1; S_F = 2;
    } else {
      nq = 11; nh = 8; F_U = 0; F_V = 1; F_W = 2; F_PHI = 3; F_G = 4; F_C = 5;
      H_HV = 11; H_HG = 12; H_F = 13; nsv = 2; S_F = 3;
    }
    nsolve = nsv + nc;
  }
};

}  // namespace

// ---------------------------------------------------------------- explicit assembly and RHS
// Per element (j, mode), from the projected explicit terms S = [N_x N_y (N_z)
// F...], DN = [D N_x, (D N_z)], and D c, D2 c of the conformation components:
//   H_a = N_a + (1 - beta)/(Re Wi) (i kx c_xa + D c_ya + i kz c_za)
//   D H_x, D H_z: the same with one more D (D2 on c_y.)
//   h_v = -(i kx D H_x + i kz D H_z) - k^2 H_y,   h_g = i kz H_x - i kx H_z
//   (mean slot: h_v holds Re H_x, h_g holds Re H_z, the mean-flow forcing)
// then the CNAB2 right-hand sides at interior rows (the solve works on rows
// 1..N-1):
//   phi: (1/dt - nu k^2/2) phi + nu/2 D2 phi + 3/2 h_v - 1/2 h_v^old
//   U  : U/dt + nu/2 D2 U + 3/2 H_x - 1/2 H_x^old        (mean slot of phi)
//   g  : as phi with h_g, W in the mean slot (3D)
//   c  : (1/dt - 1/(2Wi) - kappa k^2/2) c + kappa/2 D2 c + 3/2 F - 1/2 F^old
//        + delta/Wi (mean slot) + kappa/2 (D2_i0 c_0^new + D2_iN c_N^new)
// and the new wall rows of c (kappa = 0 there):
//   c_B^new = ((1/dt - 1/(2Wi)) c_B + 3/2 F_B - 1/2 F_B^old + delta/Wi) / (1/dt + 1/(2Wi)).
// ROWS: RHS_ALL, one launch in which each thread computes the two wall
// values of its mode; or RHS_WALLS (rows 0 and N, storing c_B^new into CB)
// and then RHS_INTERIOR (rows 1..N-1, reading them from CB).  Within a
// launch no thread reads what another writes.
// SBDF4 (p.scheme == 1) replaces the CNAB2 combinations by
//   sum_k alpha_k q^{n-k} / dt + sum_k beta_k X^{n-k},
//   alpha = (4, -3, 4/3, -1/4), beta = (4, -6, 4, -1),
// with no explicit half of the linear terms, wall rows divided by
// 25/(12 dt) + 1/Wi and the interior c rows coupled to the new wall values
// by kappa (D2_i0 c_0 + D2_iN c_N).  q^{n-k} comes from ring slot (n-k) mod 4,
// X^{n-1} from the state and X^{n-2}, X^{n-3} from the explicit ring's slots
// (n-k) mod 4.  The thread then stores its element of q^n into slot n mod 4
// and of X^{n-1} into slot (n-1) mod 4 of the two rings: slots no thread of
// this step reads, and the stores repeat the same values if the kernel is
// launched again on the same state.  D2buf = [D2 phi, (D2 g), D2 c...]
// then D2U (N+1) and D2W (N+1); Dc = [D c...].  smean (mixed precision
// only) replaces S in the mean column.  Outputs: R [nsolve][N-1 rows], hvn,
// hgn (3D), CB [nc][2 walls][cw].
template <int ROWS>
__global__ __launch_bounds__(ELEM_THREADS) void rhs_kernel(const RhsArgs* __restrict__ args, int nmem) {
  const RhsArgs& A = args[member_of(args, nmem)];
  if (masked(&A.sc->blowup)) return;
  const Dims d = A.d;
  const Phys p = A.p;
  const auto st = gmem(A.st);
  const auto D2buf = gmem(A.D2buf);
  const auto Dc = gmem(A.Dc);
  const auto S = gmem(A.S);
  const auto smean = gmem(A.smean);
  const auto DN = gmem(A.DN);
  const auto kx = gmem(A.kx);
  const auto kz = gmem(A.kz);
  const auto d2i0 = gmem(A.d2i0);
  const auto d2in = gmem(A.d2in);
  const auto R = gmem(A.R);
  const auto hvn = gmem(A.hvn);
  const auto hgn = gmem(A.hgn);
  const auto CB = gmem(A.CB);
  const int n1 = d.N + 1, N = d.N, ni = d.N - 1;
  const int e = (blockIdx.x - A.blk0) * blockDim.x + threadIdx.x;
  constexpr int rows = ROWS;
  if (e >= (rows == RHS_WALLS ? 2 : rows == RHS_INTERIOR ? ni : n1) * d.nm) return;
  const Layout L(d.dim, d.nc);
  // element (row, mode) of this thread among the launch's rows
  const int el = rows == RHS_WALLS ? (e < d.nm ? e : e + (N - 1) * d.nm) : rows == RHS_INTERIOR ? e + d.nm : e;
  Mode m = decode(d, el, kx, kz);
  const int j = m.j;
  const bool inter = (j > 0 && j < N);
  const size_t fs = (size_t)n1 * d.cw, fsi = (size_t)ni * d.cw;
  const size_t off = (size_t)j * d.cw + 2 * m.mode;
  const size_t offi = (size_t)(j - 1) * d.cw + 2 * m.mode;
  const size_t off0 = 2 * (size_t)m.mode, offN = (size_t)N * d.cw + 2 * m.mode;
  const double dt = p.dt, nu = p.nu;
  if (m.nyq) {
    st2(hvn, off, cd{0, 0});
    if (d.dim == 3) st2(hgn, off, cd{0, 0});
    if (p.scheme == 1) {  // the history rings hold zeros in the Nyquist slot, like the state
      const long long n = A.sc->step;
      const auto qn = gmem(A.qring) + (size_t)(n & 3) * L.nq * fs;
      const auto h1 = gmem(A.hring) + (size_t)((n - 1) & 3) * L.nh * fs;
      for (int f = 0; f < L.nq; ++f) st2(qn, (size_t)f * fs + off, cd{0, 0});
      for (int f = 0; f < L.nh; ++f) st2(h1, (size_t)f * fs + off, cd{0, 0});
    }
    if (inter)
      for (int f = 0; f < L.nsolve; ++f) st2(R, f * fsi + offi, cd{0, 0});
    if (!inter)
      for (int a = 0; a < d.nc; ++a) st2(CB, (size_t)(2 * a + (j == 0 ? 0 : 1)) * d.cw + 2 * m.mode, cd{0, 0});
    return;
  }
  const bool msub = m.mean && smean != nullptr;
  auto Sx = [&](int o, int jj) -> cd {  // explicit term o at row jj of this mode
    if (msub) return cd{smean[(size_t)o * n1 + jj], 0.0};
    return ld2(S, (size_t)o * fs + (size_t)jj * d.cw + 2 * m.mode);
  };
  auto c = [&](int a, int b) { return ld2(st, (size_t)(L.F_C + cidx(d.dim, a, b)) * fs + off); };
  auto Dcv = [&](int a, int b) { return ld2(Dc, (size_t)cidx(d.dim, a, b) * fs + off); };
  auto D2c = [&](int a, int b) { return ld2(D2buf, (size_t)(L.nsv + cidx(d.dim, a, b)) * fs + off); };
  const double coef = p.coef;
  cd hv, hg{0, 0};
  if (d.dim == 2) {
    const cd Hx = Sx(0, j) + coef * (ik(m.kx, c(0, 0)) + Dcv(0, 1));
    const cd Hy = Sx(1, j) + coef * (ik(m.kx, c(0, 1)) + Dcv(1, 1));
    const cd DHx = ld2(DN, off) + coef * (ik(m.kx, Dcv(0, 0)) + D2c(0, 1));
    hv = m.mean ? cd{Hx.r, 0} : cd{0, 0} - ik(m.kx, DHx) - m.k2 * Hy;
  } else {
    const cd Hx = Sx(0, j) + coef * (ik(m.kx, c(0, 0)) + Dcv(0, 1) + ik(m.kz, c(0, 2)));
    const cd Hy = Sx(1, j) + coef * (ik(m.kx, c(0, 1)) + Dcv(1, 1) + ik(m.kz, c(1, 2)));
    const cd Hz = Sx(2, j) + coef * (ik(m.kx, c(0, 2)) + Dcv(1, 2) + ik(m.kz, c(2, 2)));
    const cd DHx = ld2(DN, off) + coef * (ik(m.kx, Dcv(0, 0)) + D2c(0, 1) + ik(m.kz, Dcv(0, 2)));
    const cd DHz = ld2(DN, fs + off) + coef * (ik(m.kx, Dcv(0, 2)) + D2c(1, 2) + ik(m.kz, Dcv(2, 2)));
    hv = m.mean ? cd{Hx.r, 0} : cd{0, 0} - ik(m.kx, DHx) - ik(m.kz, DHz) - m.k2 * Hy;
    hg = m.mean ? cd{Hz.r, 0} : ik(m.kz, Hx) - ik(m.kx, Hz);
    st2(hgn, off, hg);
  }
  st2(hvn, off, hv);
  if (p.scheme == 1) {
    const long long n = A.sc->step;
    const size_t qs = (size_t)L.nq * fs, hs = (size_t)L.nh * fs;
    const auto qr = gmem(A.qring);
    const auto hr = gmem(A.hring);
    const auto q1 = qr + (size_t)((n - 1) & 3) * qs, q2 = qr + (size_t)((n - 2) & 3) * qs;
    const auto q3 = qr + (size_t)((n - 3) & 3) * qs;
    const auto h2 = hr + (size_t)((n - 2) & 3) * hs, h3 = hr + (size_t)((n - 3) & 3) * hs;
    const double idt = 1.0 / dt;
    // field f of the state at element offset o: sum_k alpha_k q^{n-k} / dt
    auto past = [&](int f, size_t o) -> cd {
      const size_t x = (size_t)f * fs + o;
      return idt * (4.0 * ld2(st, x) - 3.0 * ld2(q1, x) + (4.0 / 3.0) * ld2(q2, x) - 0.25 * ld2(q3, x));
    };
    // explicit field f (state index, >= nq) extrapolated from X^n = x0
    auto ext = [&](cd x0, int f, size_t o) -> cd {
      const size_t x = (size_t)(f - L.nq) * fs + o;
      return 4.0 * x0 - 6.0 * ld2(st, (size_t)f * fs + o) + 4.0 * ld2(h2, x) - ld2(h3, x);
    };
    if (inter) {
      cd r = m.mean ? cd{past(L.F_U, off).r + ext(hv, L.H_HV, off).r, 0} : past(L.F_PHI, off) + ext(hv, L.H_HV, off);
      st2(R, 0 * fsi + offi, r);
      if (d.dim == 3) {
        r = m.mean ? cd{past(L.F_W, off).r + ext(hg, L.H_HG, off).r, 0} : past(L.F_G, off) + ext(hg, L.H_HG, off);
        st2(R, 1 * fsi + offi, r);
      }
    }
    const double a_new = p.ia + p.th / p.wi;
    for (int a = 0; a < d.nc; ++a) {
      const bool diag = (d.dim == 2) ? (a == 0 || a == 2) : (a == 0 || a == 3 || a == 5);
      const cd src = cd{(m.mean && diag) ? 1.0 / p.wi : 0.0, 0};
      const int o = L.S_F + a, fc = L.F_C + a, fh = L.H_F + a;
      // new value of component a at wall w (0: row 0, 1: row N)
      auto wall = [&](int w) -> cd {
        if (rows == RHS_INTERIOR) return ld2(CB, (size_t)(2 * a + w) * d.cw + 2 * m.mode);
        const size_t ow = w ? offN : off0;
        return (1.0 / a_new) * (past(fc, ow) + ext(Sx(o, w ? N : 0), fh, ow) + src);
      };
      if (inter) {
        cd r = past(fc, off) + ext(Sx(o, j), fh, off) + src;
        if (p.kappa > 0) r = r + (p.th * p.kappa) * (d2i0[j - 1] * wall(0) + d2in[j - 1] * wall(1));
        st2(R, (size_t)(L.nsv + a) * fsi + offi, r);
      } else {
        st2(CB, (size_t)(2 * a + (j == 0 ? 0 : 1)) * d.cw + 2 * m.mode, wall(j == 0 ? 0 : 1));
      }
    }
    const auto qn = qr + (size_t)(n & 3) * qs;
    for (int f = 0; f < L.nq; ++f) st2(qn, (size_t)f * fs + off, ld2(st, (size_t)f * fs + off));
    const auto h1 = hr + (size_t)((n - 1) & 3) * hs;
    for (int f = 0; f < L.nh; ++f) st2(h1, (size_t)f * fs + off, ld2(st, (size_t)(L.nq + f) * fs + off));
    return;
  }
  const auto D2U = D2buf + (size_t)L.nsolve * fs;
  const auto D2W = D2U + n1;
  if (inter) {
    cd r;
    const cd hvo = ld2(st, (size_t)L.H_HV * fs + off);
    if (m.mean) {
      const double U = st[(size_t)L.F_U * fs + off];
      r = cd{U / dt + 0.5 * nu * D2U[j] + 1.5 * hv.r - 0.5 * hvo.r, 0};
    } else {
      const cd ph = ld2(st, (size_t)L.F_PHI * fs + off);
      r = (1.0 / dt - 0.5 * nu * m.k2) * ph + (0.5 * nu) * ld2(D2buf, 0 * fs + off) + 1.5 * hv - 0.5 * hvo;
    }
    st2(R, 0 * fsi + offi, r);
    if (d.dim == 3) {
      const cd hgo = ld2(st, (size_t)L.H_HG * fs + off);
      if (m.mean) {
        const double W = st[(size_t)L.F_W * fs + off];
        r = cd{W / dt + 0.5 * nu * D2W[j] + 1.5 * hg.r - 0.5 * hgo.r, 0};
      } else {
        const cd g = ld2(st, (size_t)L.F_G * fs + off);
        r = (1.0 / dt - 0.5 * nu * m.k2) * g + (0.5 * nu) * ld2(D2buf, 1 * fs + off) + 1.5 * hg - 0.5 * hgo;
      }
      st2(R, 1 * fsi + offi, r);
    }
  }
  const double a_int = 1.0 / dt - 0.5 / p.wi, a_new = 1.0 / dt + 0.5 / p.wi;
  for (int a = 0; a < d.nc; ++a) {
    const auto cf = st + (size_t)(L.F_C + a) * fs;
    const auto Fo = st + (size_t)(L.H_F + a) * fs;
    const bool diag = (d.dim == 2) ? (a == 0 || a == 2) : (a == 0 || a == 3 || a == 5);
    const cd src = cd{(m.mean && diag) ? 1.0 / p.wi : 0.0, 0};
    const int o = L.S_F + a;
    // new value of component a at wall w (0: row 0, 1: row N)
    auto wall = [&](int w) -> cd {
      if (rows == RHS_INTERIOR) return ld2(CB, (size_t)(2 * a + w) * d.cw + 2 * m.mode);
      const size_t ow = w ? offN : off0;
      return (1.0 / a_new) * (a_int * ld2(cf, ow) + 1.5 * Sx(o, w ? N : 0) - 0.5 * ld2(Fo, ow) + src);
    };
    if (inter) {
      cd r = (a_int - 0.5 * p.kappa * m.k2) * ld2(cf, off) + (0.5 * p.kappa) * ld2(D2buf, (L.nsv + a) * fs + off) +
             1.5 * Sx(o, j) - 0.5 * ld2(Fo, off) + src;
      if (p.kappa > 0) r = r + (0.5 * p.kappa) * (d2i0[j - 1] * wall(0) + d2in[j - 1] * wall(1));
      st2(R, (size_t)(L.nsv + a) * fsi + offi, r);
    } else {
      st2(CB, (size_t)(2 * a + (j == 0 ? 0 : 1)) * d.cw + 2 * m.mode, wall(j == 0 ? 0 : 1));
    }
  }
}

void launch_rhs(const RhsArgs* walls, int wblocks, const RhsArgs* inner, int iblocks, int nmem, hipStream_t s) {
  if (wblocks > 0) {
    hipLaunchKernelGGL(rhs_kernel<RHS_WALLS>, dim3(wblocks), dim3(ELEM_THREADS), 0, s, walls, nmem);
    if (iblocks > 0)
      hipLaunchKernelGGL(rhs_kernel<RHS_INTERIOR>, dim3(iblocks), dim3(ELEM_THREADS), 0, s, inner, nmem);
  } else if (iblocks > 0) {
    hipLaunchKernelGGL(rhs_kernel<RHS_ALL>, dim3(iblocks), dim3(ELEM_THREADS), 0, s, inner, nmem);
  }
}

// ---------------------------------------------------------------- finalize
// Influence-matrix correction, flux constraint, u and w, c wall rows and the
// history update.  Per mode (kx, kz) != 0, with particular solutions phi_p,
// v_p (zero at the walls) and precomputed homogeneous pairs (phi_1, v_1),
// (phi_2, v_2) (phi_1 = 1 at y = +1, phi_2 = 1 at y = -1):
//   [a b]^T = -A^-1 [(D v_p)(+1), (D v_p)(-1)]^T,  A = [[Dv_1, Dv_2] at +1; at -1]
//   phi = phi_p + a phi_1 + b phi_2,  v = v_p + a v_1 + b v_2
//   u = (i kx Dv - i kz g)/k^2,  w = (i kz Dv + i kx g)/k^2
// Mean mode: U = U_p + Pi U_1 with Pi = (Q - w.U_p)/(w.U_1) (constant flux)
// or Pi = dp/dx (constant drive); W = g's mean slot (then cleared).
// infl layout: [phi1 phi2 v1 v2 Dv1 Dv2][N+1][nm], then Ainv [4][nm].
__global__ __launch_bounds__(ELEM_THREADS) void finalize_kernel(const FinArgs* __restrict__ args, int nmem) {
  const FinArgs& A = args[member_of(args, nmem)];
  if (masked(&A.sc->blowup)) return;
  const Dims d = A.d;
  const Phys p = A.p;
  const auto Zphi = gmem(A.Zphi);
  const auto Zv = gmem(A.Zv);
  const auto Zg = gmem(A.Zg);
  const auto ZDv = gmem(A.ZDv);
  const auto flux = gmem(A.flux);
  const auto infl = gmem(A.infl);
  const auto U1 = gmem(A.U1);
  const double wU1 = A.wU1;
  const auto CB = gmem(A.CB);
  const auto hvn = gmem(A.hvn);
  const auto hgn = gmem(A.hgn);
  const auto S = gmem(A.S);
  const auto smean = gmem(A.smean);
  const auto kx = gmem(A.kx);
  const auto kz = gmem(A.kz);
  const auto st = gmem(A.st);
  const auto prep = gmem(A.prep);
  DevScalars* __restrict__ sc = A.sc;
  const int n1 = d.N + 1, N = d.N;
  const int e = (blockIdx.x - A.blk0) * blockDim.x + threadIdx.x;
  if (e >= n1 * d.nm) return;
  const Layout L(d.dim, d.nc);
  Mode m = decode(d, e, kx, kz);
  const int j = m.j;
  const bool inter = (j > 0 && j < N);
  const size_t fs = (size_t)n1 * d.cw;
  const size_t off = (size_t)j * d.cw + 2 * m.mode;
  const size_t offi = (size_t)(j - 1) * d.cw + 2 * m.mode;
  // history: h_v, h_g, F <- this step's explicit terms
  st2(st, (size_t)L.H_HV * fs + off, ld2(hvn, off));
  if (d.dim == 3) st2(st, (size_t)L.H_HG * fs + off, ld2(hgn, off));
  for (int a = 0; a < d.nc; ++a) {
    const cd F = (m.mean && smean) ? cd{smean[(size_t)(L.S_F + a) * n1 + j], 0.0}
                                   : ld2(S, (size_t)(L.S_F + a) * fs + off);
    st2(st, (size_t)(L.H_F + a) * fs + off, F);
  }
  // c wall rows (interior rows were written by the solve product)
  if (!inter)
    for (int a = 0; a < d.nc; ++a)
      st2(st, (size_t)(L.F_C + a) * fs + off, ld2(CB, (size_t)(2 * a + (j == 0 ? 0 : 1)) * d.cw + 2 * m.mode));
  // spectral inputs of the diagnostics: Tr c (c_xx + c_yy (+ c_zz)), u, v, w
  auto diag_prep = [&](cd u, cd v, cd w) {
    cd tr = ld2(st, (size_t)L.F_C * fs + off) + ld2(st, (size_t)(L.F_C + (d.dim == 2 ? 2 : 3)) * fs + off);
    if (d.dim == 3) tr = tr + ld2(st, (size_t)(L.F_C + 5) * fs + off);
    st2(prep, off, tr);
    st2(prep, fs + off, u);
    st2(prep, 2 * fs + off, v);
    if (d.dim == 3) st2(prep, 3 * fs + off, w);
  };
  if (m.nyq) {
    for (int f = 0; f < L.nq; ++f) st2(st, (size_t)f * fs + off, cd{0, 0});
    diag_prep(cd{0, 0}, cd{0, 0}, cd{0, 0});
    return;
  }
  if (m.mean) {
    const double Up = inter ? Zphi[offi] : 0.0;
    const double pi = (p.forcing == 0) ? (p.q_or_dpdx - flux[0]) / wU1 : p.q_or_dpdx;
    if (e == 0) sc->pi = pi;
    const cd U{Up + pi * U1[j], 0};
    st2(st, (size_t)L.F_U * fs + off, U);
    st2(st, (size_t)L.F_V * fs + off, cd{0, 0});
    st2(st, (size_t)L.F_PHI * fs + off, cd{0, 0});
    cd W{0, 0};
    if (d.dim == 3) {
      W = cd{inter ? Zg[offi] : 0.0, 0};  // interior rows from the solve, walls zero
      st2(st, (size_t)L.F_W * fs + off, W);
      st2(st, (size_t)L.F_G * fs + off, cd{0, 0});
    }
    diag_prep(U, cd{0, 0}, W);
    return;
  }
  const size_t pm = (size_t)n1 * d.nm;
  const size_t io = (size_t)j * d.nm + m.mode;
  const auto Ai = infl + 6 * pm;
  const double a00 = Ai[0 * d.nm + m.mode], a01 = Ai[1 * d.nm + m.mode];
  const double a10 = Ai[2 * d.nm + m.mode], a11 = Ai[3 * d.nm + m.mode];
  const cd dp0 = ld2(ZDv, 2 * (size_t)m.mode), dpN = ld2(ZDv, (size_t)N * d.cw + 2 * m.mode);
  const cd a = cd{0, 0} - (a00 * dp0 + a01 * dpN);
  const cd b = cd{0, 0} - (a10 * dp0 + a11 * dpN);
  const double phi1 = infl[0 * pm + io], phi2 = infl[1 * pm + io];
  const double v1 = infl[2 * pm + io], v2 = infl[3 * pm + io];
  const double Dv1 = infl[4 * pm + io], Dv2 = infl[5 * pm + io];
  const cd php = inter ? ld2(Zphi, offi) : cd{0, 0};
  const cd vp = inter ? ld2(Zv, offi) : cd{0, 0};
  const cd phi = php + phi1 * a + phi2 * b;
  const cd v = vp + v1 * a + v2 * b;
  const cd Dv = ld2(ZDv, off) + Dv1 * a + Dv2 * b;
  st2(st, (size_t)L.F_PHI * fs + off, phi);
  st2(st, (size_t)L.F_V * fs + off, v);
  const double ik2 = 1.0 / m.k2;
  if (d.dim == 2) {
    const cd u = ik2 * ik(m.kx, Dv);
    st2(st, (size_t)L.F_U * fs + off, u);
    diag_prep(u, v, cd{0, 0});
  } else {
    // g: interior rows come from the solve product, wall rows are zero
    const cd g = inter ? ld2(Zg, offi) : cd{0, 0};
    st2(st, (size_t)L.F_G * fs + off, g);
    const cd u = ik2 * (ik(m.kx, Dv) - ik(m.kz, g));
    const cd w = ik2 * (ik(m.kz, Dv) + ik(m.kx, g));
    st2(st, (size_t)L.F_U * fs + off, u);
    st2(st, (size_t)L.F_W * fs + off, w);
    diag_prep(u, v, w);
  }
}

void launch_finalize(const FinArgs* args, int nmem, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(ELEM_THREADS), 0, s, args, nmem);
}

// ---------------------------------------------------------------- init: homogeneous solutions
// Right-hand side whose solve yields phi_1 + i phi_2 in every mode's phi slot:
// interior rows of (ia - th nu D2) phi = 0 with phi(+1) = 1 (real part) or
// phi(-1) = 1 (imaginary part) move the wall column to the right:
//   R = th nu (D2_i0 + i D2_iN).   Mean slot: R = 1 (gives U_1).
__global__ void homog_rhs_kernel(Dims d, Phys p, const double* __restrict__ d2i0, const double* __restrict__ d2in,
                                 double* __restrict__ R) {
  const int ni = d.N - 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ni * d.nm) return;
  const int j = e / d.nm, mode = e - j * d.nm;
  const size_t off = (size_t)j * d.cw + 2 * mode;
  if (mode == 0) {
    R[off] = 1.0;
    R[off + 1] = 0.0;
  } else {
    R[off] = p.th * p.nu * d2i0[j];
    R[off + 1] = p.th * p.nu * d2in[j];
  }
}

void launch_homog_rhs(const Dims& d, const Phys& p, const double* d2i0, const double* d2in, double* R,
                      hipStream_t s) {
  const int n = (d.N - 1) * d.nm;
  hipLaunchKernelGGL(homog_rhs_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, p, d2i0, d2in, R);
}

// Splits the homogeneous solves into the per-mode influence data and inverts
// the 2x2 influence matrices.
__global__ void influence_kernel(Dims d, const double* __restrict__ Zphi, const double* __restrict__ Zv,
                                 const double* __restrict__ ZDv, const double* __restrict__ kz,
                                 double* __restrict__ infl, double* __restrict__ U1) {
  const int n1 = d.N + 1, N = d.N;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n1 * d.nm) return;
  const int j = e / d.nm, mode = e - j * d.nm;
  const int iz = mode / d.nkx;
  const bool nyq = (d.dim == 3) && (iz == d.nzs / 2);
  const bool inter = (j > 0 && j < N);
  const size_t pm = (size_t)n1 * d.nm, io = (size_t)j * d.nm + mode;
  const size_t offi = (size_t)(j - 1) * d.cw + 2 * mode, off = (size_t)j * d.cw + 2 * mode;
  if (mode == 0) {
    U1[j] = inter ? Zphi[offi] : 0.0;
    for (int f = 0; f < 6; ++f) infl[f * pm + io] = 0.0;
  } else if (nyq) {
    for (int f = 0; f < 6; ++f) infl[f * pm + io] = 0.0;
  } else {
    infl[0 * pm + io] = (j == 0 ? 1.0 : 0.0) + (inter ? Zphi[offi] : 0.0);
    infl[1 * pm + io] = (j == N ? 1.0 : 0.0) + (inter ? Zphi[offi + 1] : 0.0);
    infl[2 * pm + io] = inter ? Zv[offi] : 0.0;
    infl[3 * pm + io] = inter ? Zv[offi + 1] : 0.0;
    infl[4 * pm + io] = ZDv[off];
    infl[5 * pm + io] = ZDv[off + 1];
  }
  if (j == 0) {
    double* Ai = infl + 6 * pm;
    if (mode == 0 || nyq) {
      Ai[0 * d.nm + mode] = Ai[1 * d.nm + mode] = Ai[2 * d.nm + mode] = Ai[3 * d.nm + mode] = 0.0;
    } else {
      const size_t oN = (size_t)N * d.cw + 2 * mode, o0 = 2 * (size_t)mode;
      const double A00 = ZDv[o0], A01 = ZDv[o0 + 1], A10 = ZDv[oN], A11 = ZDv[oN + 1];
      const double det = A00 * A11 - A01 * A10;
      Ai[0 * d.nm + mode] = A11 / det;
      Ai[1 * d.nm + mode] = -A01 / det;
      Ai[2 * d.nm + mode] = -A10 / det;
      Ai[3 * d.nm + mode] = A00 / det;
    }
  }
}

void launch_influence(const Dims& d, const double* Zphi, const double* Zv, const double* ZDv, const double* kz,
                      double* infl, double* U1, hipStream_t s) {
  const int n = (d.N + 1) * d.nm;
  hipLaunchKernelGGL(influence_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, Zphi, Zv, ZDv, kz, infl, U1);
}

}  // namespace pcs
