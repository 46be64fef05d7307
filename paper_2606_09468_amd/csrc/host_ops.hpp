// Host-side construction of the wall-normal operators, Fourier twiddles and
// the initial state of the polymer channel-flow step.
//
// The paper expands the wall-normal direction in Chebyshev polynomials and
// dealiases fully (Section 2, numerics paragraph).  This library discretises
// by collocation on the N+1 Gauss-Lobatto points y_j = sin(pi (N - 2j)/(2N))
// (so y_0 = +1, y_N = -1 and y_{N/2} = 0 exactly) and pads to M = 3N/2
// intervals for products.  Every matrix is formed in x87 extended precision
// and rounded once to double.
#pragma once

#include <cstdint>
#include <vector>

namespace pcs {

struct WallOps {
  int N = 0, M = 0;
  std::vector<double> y, ypad;      // N+1, M+1
  std::vector<double> D;            // (N+1)^2 row-major, first derivative
  std::vector<double> D2;           // (N+1)^2, second derivative (D*D, exact)
  std::vector<double> IMN, DMN;     // (M+1)x(N+1): interpolate / differentiate to the padded grid
  std::vector<double> PNM;          // (N+1)x(M+1): padded values -> degree-N truncation on y_j
  std::vector<double> w;            // N+1 Clenshaw-Curtis weights
  // Interior (j = 1..N-1) block of D2 diagonalised: D2_II = V diag(lam) V^-1,
  // the first ne eigenvectors even about the midplane, the other no odd
  std::vector<double> V, Vinv, lam; // (N-1)^2, (N-1)^2, N-1
  int ne = 0, no = 0;
  std::vector<double> d2_i0, d2_in; // interior rows of the two boundary columns of D2
};

// Builds (and caches per N) the operators.  Returns nullptr for invalid N.
const WallOps* wall_ops(int N);

// exp(sign * 2 pi i m / L), m = 0..L-1, interleaved re/im.
std::vector<double> twiddles(int L, int sign);

// Laminar Poiseuille state of the sPTT/Oldroyd-B channel (eps = 0):
// U = 1 - y^2, c_xy = -2 Wi y, c_yy = c_zz = 1,
// c_xx = 1 + 8 Wi^2 y^2 + 16 kappa Wi^3 [1 - cosh(y/l)/cosh(1/l)], l = sqrt(kappa Wi).
void laminar(const double* y, int n, double wi, double kappa, double* U, double* cxx, double* cxy,
             double* cyy);

// SplitMix64 (Steele, Lea and Flood 2014).
struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next();
  double u01();  // (x >> 11) * 2^-53
};

}  // namespace pcs
