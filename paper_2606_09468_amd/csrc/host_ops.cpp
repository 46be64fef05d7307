// Host-side operator builder: wall-normal collocation operators, their
// interior eigendecomposition, Fourier twiddles and the laminar state.
//
// Discretisation of the Chebyshev direction named by the paper (Section 2):
// collocation on Gauss-Lobatto points with 3/2 padding for products.  All
// entries are computed in x87 extended precision (64-bit mantissa) from
// exactly reduced trigonometric arguments and rounded once to double.
//
//   D    : closed-form Lobatto differentiation matrix
//   D2   : D * D (product taken before rounding)
//   IMN  : barycentric interpolation from y_j to the padded points
//   DMN  : IMN * D (derivative of the interpolant on the padded points)
//   PNM  : padded values -> Chebyshev coefficients, keep degrees 0..N,
//          evaluate on y_j; summed in closed form with the Dirichlet kernel
//   w    : Clenshaw-Curtis weights (closed form)
//   V, lam, Vinv : eigendecomposition of the interior block of D2, per
//          parity block (even eigenvectors first, then odd), each from a
//          Hessenberg reduction, shifted QR for the eigenvalues and inverse
//          iteration for the eigenvectors.
#include "host_ops.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>

namespace pcs {

using ld = long double;
static const ld PI_L = 3.141592653589793238462643383279502884L;

// sin(pi num / den) with the argument reduced exactly in integers.
static ld sinpi_frac(long long num, long long den) {
  const long long p = 2 * den;
  num %= p;
  if (num < 0) num += p;
  ld sgn = 1;
  if (num >= den) {
    sgn = -1;
    num -= den;
  }
  if (2 * num > den) num = den - num;
  return sgn * sinl(PI_L * (ld)num / (ld)den);
}

static ld cospi_frac(long long num, long long den) { return sinpi_frac(den - 2 * num, 2 * den); }

// cos(pi a / A) - cos(pi b / B) = -2 sin(pi (aB + bA)/(2AB)) sin(pi (aB - bA)/(2AB))
static ld cos_diff(long long a, long long A, long long b, long long B) {
  const long long den = 2 * A * B;
  return -2 * sinpi_frac(a * B + b * A, den) * sinpi_frac(a * B - b * A, den);
}

// ---------------------------------------------------------------- eigen
// Real nonsymmetric eigendecomposition for a matrix with real, distinct
// eigenvalues: A = V diag(lam) V^-1.  Returns false if QR does not converge.
static bool eig_real(int n, std::vector<ld> A, std::vector<ld>& lam, std::vector<ld>& V) {
  auto at = [n](std::vector<ld>& M, int i, int j) -> ld& { return M[(size_t)i * n + j]; };
  std::vector<ld> Q((size_t)n * n, 0);
  for (int i = 0; i < n; ++i) at(Q, i, i) = 1;
  // Householder reduction to upper Hessenberg form, A <- P A P, Q <- Q P
  std::vector<ld> v(n);
  for (int k = 0; k < n - 2; ++k) {
    ld nrm = 0;
    for (int i = k + 1; i < n; ++i) nrm += at(A, i, k) * at(A, i, k);
    nrm = sqrtl(nrm);
    if (nrm == 0) continue;
    ld x0 = at(A, k + 1, k);
    ld alpha = x0 > 0 ? -nrm : nrm;
    std::fill(v.begin(), v.end(), 0);
    v[k + 1] = x0 - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = at(A, i, k);
    ld vn = 0;
    for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
    if (vn == 0) continue;
    ld inv = 2 / vn;
    for (int j = 0; j < n; ++j) {  // A <- (I - 2vv'/v'v) A
      ld s = 0;
      for (int i = k + 1; i < n; ++i) s += v[i] * at(A, i, j);
      s *= inv;
      for (int i = k + 1; i < n; ++i) at(A, i, j) -= s * v[i];
    }
    for (int i = 0; i < n; ++i) {  // A <- A (I - 2vv'/v'v), Q likewise
      ld s = 0, t = 0;
      for (int j = k + 1; j < n; ++j) {
        s += at(A, i, j) * v[j];
        t += at(Q, i, j) * v[j];
      }
      s *= inv;
      t *= inv;
      for (int j = k + 1; j < n; ++j) {
        at(A, i, j) -= s * v[j];
        at(Q, i, j) -= t * v[j];
      }
    }
    for (int i = k + 2; i < n; ++i) at(A, i, k) = 0;
  }
  const std::vector<ld> H = A;
  // Eigenvalues: explicit single-shift QR (Wilkinson shift) with deflation.
  std::vector<ld> T = H;
  lam.assign(n, 0);
  const ld eps = 1e-20L;
  int hi = n - 1, it = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) {
      lam[0] = at(T, 0, 0);
      break;
    }
    int l = hi;
    while (l > 0 && fabsl(at(T, l, l - 1)) > eps * (fabsl(at(T, l, l)) + fabsl(at(T, l - 1, l - 1)))) --l;
    if (l == hi) {
      lam[hi] = at(T, hi, hi);
      --hi;
      it = 0;
      continue;
    }
    if (++it > 200 || ++total > 60 * n) return false;
    ld a = at(T, hi - 1, hi - 1), b = at(T, hi - 1, hi), c = at(T, hi, hi - 1), d = at(T, hi, hi);
    ld disc = (a - d) * (a - d) / 4 + b * c;
    ld mu = d;
    if (disc >= 0) {
      ld r = sqrtl(disc), m = (a + d) / 2;
      mu = fabsl(m + r - d) < fabsl(m - r - d) ? m + r : m - r;
    }
    if (it % 11 == 10) mu += fabsl(at(T, hi, hi - 1));  // exceptional shift
    for (int i = l; i <= hi; ++i) at(T, i, i) -= mu;
    std::vector<ld> cs(hi - l), sn(hi - l);
    for (int k = l; k < hi; ++k) {
      ld x = at(T, k, k), y = at(T, k + 1, k);
      ld r = hypotl(x, y);
      ld cc = r == 0 ? 1 : x / r, ss = r == 0 ? 0 : y / r;
      cs[k - l] = cc;
      sn[k - l] = ss;
      for (int j = k; j <= hi; ++j) {
        ld t1 = at(T, k, j), t2 = at(T, k + 1, j);
        at(T, k, j) = cc * t1 + ss * t2;
        at(T, k + 1, j) = -ss * t1 + cc * t2;
      }
    }
    for (int k = l; k < hi; ++k) {
      ld cc = cs[k - l], ss = sn[k - l];
      int rmax = std::min(k + 2, hi);
      for (int i = l; i <= rmax; ++i) {
        ld t1 = at(T, i, k), t2 = at(T, i, k + 1);
        at(T, i, k) = cc * t1 + ss * t2;
        at(T, i, k + 1) = -ss * t1 + cc * t2;
      }
    }
    for (int i = l; i <= hi; ++i) at(T, i, i) += mu;
  }
  std::sort(lam.begin(), lam.end());
  // Eigenvectors: inverse iteration on the Hessenberg matrix, then back to A.
  V.assign((size_t)n * n, 0);
  std::vector<ld> B((size_t)n * n), x(n), y(n);
  std::vector<ld> mult(n);
  std::vector<char> swp(n);
  for (int e = 0; e < n; ++e) {
    B = H;
    for (int i = 0; i < n; ++i) at(B, i, i) -= lam[e];
    // LU with partial pivoting restricted to adjacent rows (Hessenberg)
    for (int k = 0; k < n - 1; ++k) {
      swp[k] = fabsl(at(B, k + 1, k)) > fabsl(at(B, k, k));
      if (swp[k])
        for (int j = k; j < n; ++j) std::swap(at(B, k, j), at(B, k + 1, j));
      ld piv = at(B, k, k);
      if (piv == 0) piv = at(B, k, k) = 1e-30L;
      mult[k] = at(B, k + 1, k) / piv;
      for (int j = k + 1; j < n; ++j) at(B, k + 1, j) -= mult[k] * at(B, k, j);
      at(B, k + 1, k) = 0;
    }
    if (at(B, n - 1, n - 1) == 0) at(B, n - 1, n - 1) = 1e-30L;
    std::fill(x.begin(), x.end(), 1);
    for (int iter = 0; iter < 3; ++iter) {
      for (int k = 0; k < n - 1; ++k) {
        if (swp[k]) std::swap(x[k], x[k + 1]);
        x[k + 1] -= mult[k] * x[k];
      }
      for (int i = n - 1; i >= 0; --i) {
        ld s = x[i];
        for (int j = i + 1; j < n; ++j) s -= at(B, i, j) * x[j];
        x[i] = s / at(B, i, i);
      }
      ld mx = 0;
      for (int i = 0; i < n; ++i) mx = std::max(mx, fabsl(x[i]));
      for (int i = 0; i < n; ++i) x[i] /= mx;
    }
    for (int i = 0; i < n; ++i) {
      ld s = 0;
      for (int j = 0; j < n; ++j) s += at(Q, i, j) * x[j];
      y[i] = s;
    }
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (fabsl(y[i]) > fabsl(y[imax])) imax = i;
    ld scale = 1 / y[imax];
    for (int i = 0; i < n; ++i) at(V, i, e) = y[i] * scale;
  }
  return true;
}

static bool invert(int n, std::vector<ld> A, std::vector<ld>& Ai) {
  auto at = [n](std::vector<ld>& M, int i, int j) -> ld& { return M[(size_t)i * n + j]; };
  Ai.assign((size_t)n * n, 0);
  for (int i = 0; i < n; ++i) at(Ai, i, i) = 1;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (fabsl(at(A, i, k)) > fabsl(at(A, p, k))) p = i;
    if (at(A, p, k) == 0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        std::swap(at(A, k, j), at(A, p, j));
        std::swap(at(Ai, k, j), at(Ai, p, j));
      }
    ld inv = 1 / at(A, k, k);
    for (int j = 0; j < n; ++j) {
      at(A, k, j) *= inv;
      at(Ai, k, j) *= inv;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      ld f = at(A, i, k);
      if (f == 0) continue;
      for (int j = 0; j < n; ++j) {
        at(A, i, j) -= f * at(A, k, j);
        at(Ai, i, j) -= f * at(Ai, k, j);
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------- operators
static std::unique_ptr<WallOps> build(int N) {
  auto op = std::make_unique<WallOps>();
  const int M = 3 * N / 2, n1 = N + 1, m1 = M + 1;
  op->N = N;
  op->M = M;
  std::vector<ld> y(n1), yp(m1);
  for (int j = 0; j < n1; ++j) y[j] = sinpi_frac(N - 2 * j, 2 * N);
  for (int i = 0; i < m1; ++i) yp[i] = sinpi_frac(M - 2 * i, 2 * M);
  op->y.assign(y.begin(), y.end());
  op->ypad.assign(yp.begin(), yp.end());

  // Lobatto differentiation matrix, closed form
  std::vector<ld> D((size_t)n1 * n1);
  auto cb = [N](int j) -> ld { return (j == 0 || j == N) ? 2 : 1; };
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      ld v;
      if (i != j) {
        v = cb(i) / cb(j) * (((i + j) & 1) ? -1 : 1) / cos_diff(i, N, j, N);
      } else if (i == 0) {
        v = (2.0L * N * N + 1) / 6;
      } else if (i == N) {
        v = -(2.0L * N * N + 1) / 6;
      } else {
        ld s = sinpi_frac(i, N);
        v = -y[i] / (2 * s * s);
      }
      D[(size_t)i * n1 + j] = v;
    }
  std::vector<ld> D2((size_t)n1 * n1, 0);
  for (int i = 0; i < n1; ++i)
    for (int k = 0; k < n1; ++k) {
      ld a = D[(size_t)i * n1 + k];
      for (int j = 0; j < n1; ++j) D2[(size_t)i * n1 + j] += a * D[(size_t)k * n1 + j];
    }
  op->D.assign(D.begin(), D.end());
  op->D2.assign(D2.begin(), D2.end());

  // Barycentric interpolation to the padded points (weights (-1)^j, halved at the ends)
  std::vector<ld> I((size_t)m1 * n1, 0);
  for (int i = 0; i < m1; ++i) {
    // padded point i coincides with y_j when i N = j M
    if (((long long)i * N) % M == 0) {
      int j = (int)(((long long)i * N) / M);
      I[(size_t)i * n1 + j] = 1;
      continue;
    }
    ld S = 0;
    std::vector<ld> t(n1);
    for (int j = 0; j < n1; ++j) {
      ld lamj = ((j & 1) ? -1 : 1) * ((j == 0 || j == N) ? 0.5L : 1.0L);
      t[j] = lamj / cos_diff(i, M, j, N);
      S += t[j];
    }
    for (int j = 0; j < n1; ++j) I[(size_t)i * n1 + j] = t[j] / S;
  }
  std::vector<ld> DI((size_t)m1 * n1, 0);
  for (int i = 0; i < m1; ++i)
    for (int k = 0; k < n1; ++k) {
      ld a = I[(size_t)i * n1 + k];
      if (a == 0) continue;
      for (int j = 0; j < n1; ++j) DI[(size_t)i * n1 + j] += a * D[(size_t)k * n1 + j];
    }
  op->IMN.assign(I.begin(), I.end());
  op->DMN.assign(DI.begin(), DI.end());

  // Projection: P[j][i] = (2/(M cb'_i)) * (K(a-) + K(a+))/2, with the
  // Dirichlet kernel K(alpha) = 1/2 + sum_{n=1..N} cos(n alpha)
  // = sin((N + 1/2) alpha) / (2 sin(alpha/2)), alpha = pi a/(N M), a = jM -+ iN.
  op->PNM.assign((size_t)n1 * m1, 0);
  const long long NM = (long long)N * M;
  auto K = [&](long long a) -> ld {
    long long r = a % (2 * NM);
    if (r < 0) r += 2 * NM;
    if (r == 0) return N + 0.5L;
    return sinpi_frac((2LL * N + 1) * a, 2 * NM) / (2 * sinpi_frac(a, 2 * NM));
  };
  for (int j = 0; j < n1; ++j)
    for (int i = 0; i < m1; ++i) {
      ld cbi = (i == 0 || i == M) ? 2 : 1;
      long long am = (long long)j * M - (long long)i * N, ap = (long long)j * M + (long long)i * N;
      op->PNM[(size_t)j * m1 + i] = (double)((2.0L / (M * cbi)) * 0.5L * (K(am) + K(ap)));
    }

  // Clenshaw-Curtis weights (N even)
  op->w.assign(n1, 0);
  for (int j = 0; j < n1; ++j) {
    if (j == 0 || j == N) {
      op->w[j] = (double)(1.0L / ((ld)N * N - 1));
      continue;
    }
    ld v = 1;
    for (int k = 1; k < N / 2; ++k) v -= 2 * cospi_frac(2LL * k * j, N) / (4.0L * k * k - 1);
    v -= ((j & 1) ? -1.0L : 1.0L) / ((ld)N * N - 1);
    op->w[j] = (double)(2 * v / N);
  }

  // Interior block of D2 and its eigendecomposition.  The block is
  // centrosymmetric (A[ni-1-i][ni-1-j] = A[i][j]), so it maps even vectors
  // (x_j = x_{ni-1-j}) to even and odd to odd: on the first half of an even
  // vector (j <= mid) it acts as Ke[i][j] = A[i][j] + A[i][ni-1-j] (j < mid),
  // Ke[i][mid] = A[i][mid]; on the first half of an odd one (j < mid, the
  // middle entry being zero) as Ko[i][j] = A[i][j] - A[i][ni-1-j].  The two
  // half-size blocks are diagonalised separately, so every eigenvector is
  // exactly even or odd; the even ones are listed first.
  const int ni = N - 1, mid = ni / 2, ne = mid + 1, no = mid;
  std::vector<ld> A((size_t)ni * ni);
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) A[(size_t)i * ni + j] = D2[(size_t)(i + 1) * n1 + (j + 1)];
  std::vector<ld> Ke((size_t)ne * ne), Ko((size_t)no * no);
  for (int i = 0; i < ne; ++i)
    for (int j = 0; j < ne; ++j)
      Ke[(size_t)i * ne + j] = j < mid ? A[(size_t)i * ni + j] + A[(size_t)i * ni + (ni - 1 - j)] : A[(size_t)i * ni + j];
  for (int i = 0; i < no; ++i)
    for (int j = 0; j < no; ++j) Ko[(size_t)i * no + j] = A[(size_t)i * ni + j] - A[(size_t)i * ni + (ni - 1 - j)];
  std::vector<ld> lame, lamo, We, Wo, Wei, Woi;
  if (!eig_real(ne, Ke, lame, We) || !eig_real(no, Ko, lamo, Wo)) return nullptr;
  if (!invert(ne, We, Wei) || !invert(no, Wo, Woi)) return nullptr;
  // full eigenvectors (columns: even, then odd) and the inverse, whose rows
  // act on the half sums / differences
  std::vector<ld> lam(ni), V((size_t)ni * ni, 0), Vi((size_t)ni * ni, 0);
  for (int p = 0; p < ne; ++p) {
    lam[p] = lame[p];
    for (int j = 0; j <= mid; ++j) {
      V[(size_t)j * ni + p] = V[(size_t)(ni - 1 - j) * ni + p] = We[(size_t)j * ne + p];
      const ld wi = Wei[(size_t)p * ne + j];
      if (j < mid)
        Vi[(size_t)p * ni + j] = Vi[(size_t)p * ni + (ni - 1 - j)] = wi / 2;
      else
        Vi[(size_t)p * ni + j] = wi;
    }
  }
  for (int q = 0; q < no; ++q) {
    lam[ne + q] = lamo[q];
    for (int j = 0; j < mid; ++j) {
      V[(size_t)j * ni + ne + q] = Wo[(size_t)j * no + q];
      V[(size_t)(ni - 1 - j) * ni + ne + q] = -Wo[(size_t)j * no + q];
      Vi[(size_t)(ne + q) * ni + j] = Woi[(size_t)q * no + j] / 2;
      Vi[(size_t)(ne + q) * ni + (ni - 1 - j)] = -Woi[(size_t)q * no + j] / 2;
    }
  }
  // self-check: || V diag(lam) V^-1 - A || relative to ||A||
  ld errmax = 0, amax = 0;
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) {
      ld s = 0;
      for (int k = 0; k < ni; ++k) s += V[(size_t)i * ni + k] * lam[k] * Vi[(size_t)k * ni + j];
      errmax = std::max(errmax, fabsl(s - A[(size_t)i * ni + j]));
      amax = std::max(amax, fabsl(A[(size_t)i * ni + j]));
    }
  if (!(errmax <= 1e-14L * amax)) return nullptr;
  op->ne = ne;
  op->no = no;
  op->V.assign(V.begin(), V.end());
  op->Vinv.assign(Vi.begin(), Vi.end());
  op->lam.assign(lam.begin(), lam.end());
  op->d2_i0.resize(ni);
  op->d2_in.resize(ni);
  for (int i = 0; i < ni; ++i) {
    op->d2_i0[i] = (double)D2[(size_t)(i + 1) * n1 + 0];
    op->d2_in[i] = (double)D2[(size_t)(i + 1) * n1 + N];
  }
  return op;
}

const WallOps* wall_ops(int N) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<WallOps>> cache;
  if (N < 4 || (N & 1)) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(N);
  if (it != cache.end()) return it->second.get();
  auto op = build(N);
  const WallOps* p = op.get();
  if (p) cache[N] = std::move(op);
  return p;
}

std::vector<double> twiddles(int L, int sign) {
  std::vector<double> t(2 * (size_t)L);
  for (int m = 0; m < L; ++m) {
    t[2 * m] = (double)cospi_frac(2LL * m, L);
    t[2 * m + 1] = (double)(sign * sinpi_frac(2LL * m, L));
  }
  return t;
}

void laminar(const double* y, int n, double wi, double kappa, double* U, double* cxx, double* cxy,
             double* cyy) {
  for (int j = 0; j < n; ++j) {
    double yy = y[j];
    U[j] = 1.0 - yy * yy;
    cxy[j] = -2.0 * wi * yy;
    cyy[j] = 1.0;
    double c = 1.0 + 8.0 * wi * wi * yy * yy;
    if (kappa > 0) {
      double ell = std::sqrt(kappa * wi), a = std::fabs(yy);
      double ratio = std::exp((a - 1.0) / ell) * (1.0 + std::exp(-2.0 * a / ell)) / (1.0 + std::exp(-2.0 / ell));
      c += 16.0 * kappa * wi * wi * wi * (1.0 - ratio);
    }
    cxx[j] = c;
  }
}

uint64_t SplitMix64::next() {
  s += 0x9E3779B97F4A7C15ULL;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double SplitMix64::u01() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace pcs
