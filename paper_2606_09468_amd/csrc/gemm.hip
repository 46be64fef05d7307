// Batched dense products on the CDNA4 matrix cores.
//
// The wall-normal transforms (interpolation / differentiation to the padded
// grid, projection back), the spectral derivatives and the diagonalised
// Dirichlet solves are all products of a small operator (at most 385 x 385)
// with a wide matrix whose columns are the real and imaginary parts of every
// Fourier mode.  One launch evaluates a table of such products; each 64 x 64
// output tile is one workgroup of four waves, each wave owning a 32 x 32
// sub-tile made of 2 x 2 MFMA 16x16x4 blocks.  Operands are staged through
// LDS in K-chunks of 16.
#include "kernels.hpp"

namespace pcs {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T>
int gemm_prepare(GemmJob<T>* jobs, int njobs) {
  int t = 0;
  for (int j = 0; j < njobs; ++j) {
    jobs[j].tiles_m = (jobs[j].m + GEMM_BM - 1) / GEMM_BM;
    int tn = (jobs[j].n + GEMM_BN - 1) / GEMM_BN;
    jobs[j].tile0 = t;
    t += jobs[j].tiles_m * tn;
  }
  return t;
}
template int gemm_prepare<double>(GemmJob<double>*, int);
template int gemm_prepare<float>(GemmJob<float>*, int);

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline flt4 mfma(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, typename V4>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmJob<T>* __restrict__ jobs, int njobs) {
  __shared__ T As[GEMM_BK][GEMM_BM + 1];
  __shared__ T Bs[GEMM_BK][GEMM_BN + 1];
  const int t = blockIdx.x;
  int jb = 0;
  while (jb + 1 < njobs && jobs[jb + 1].tile0 <= t) ++jb;
  const GemmJob<T> J = jobs[jb];
  const int lt = t - J.tile0;
  const int row0 = (lt % J.tiles_m) * GEMM_BM;
  const int col0 = (lt / J.tiles_m) * GEMM_BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int l16 = lane & 15, lk = lane >> 4;
  V4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

  for (int k0 = 0; k0 < J.k; k0 += GEMM_BK) {
    for (int e = tid; e < GEMM_BM * GEMM_BK; e += 256) {
      const int r = e / GEMM_BK, c = e % GEMM_BK;
      const int gr = row0 + r, gc = k0 + c;
      As[c][r] = (gr < J.m && gc < J.k) ? J.A[(size_t)gr * J.lda + gc] : T(0);
    }
    for (int e = tid; e < GEMM_BK * GEMM_BN; e += 256) {
      const int r = e / GEMM_BN, c = e % GEMM_BN;
      const int gr = k0 + r, gc = col0 + c;
      Bs[r][c] = (gr < J.k && gc < J.n) ? J.B[(size_t)gr * J.ldb + gc] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GEMM_BK; kk += 4) {
      const int kl = kk + lk;
      const T a0 = As[kl][wm + l16], a1 = As[kl][wm + 16 + l16];
      const T b0 = Bs[kl][wn + l16], b1 = Bs[kl][wn + 16 + l16];
      acc[0][0] = mfma(a0, b0, acc[0][0]);
      acc[0][1] = mfma(a0, b1, acc[0][1]);
      acc[1][0] = mfma(a1, b0, acc[1][0]);
      acc[1][1] = mfma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  // Element D[i][j] of a 16x16 block lives in lane j + 16 * (i / 4), register
  // i % 4 for the f32 instruction, and in lane j + 16 * (i % 4), register
  // i / 4 for the f64 one (checked on gfx950 with a one-hot product).
  constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm + bi * 16 + (f64 ? 4 * r + lk : 4 * lk + r);
        const int gc = col0 + wn + bj * 16 + l16;
        if (gr < J.m && gc < J.n) {
          T* cp = J.C + (size_t)gr * J.ldc + gc;
          T v = J.alpha * acc[bi][bj][r];
          if (J.beta != T(0)) v += J.beta * *cp;
          *cp = v;
        }
      }
}

void gemm_f64(const GemmJob<double>* dev_jobs, int total_tiles, int njobs, hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL((gemm_kernel<double, dbl4>), dim3(total_tiles), dim3(256), 0, s, dev_jobs, njobs);
}

void gemm_f32(const GemmJob<float>* dev_jobs, int total_tiles, int njobs, hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL((gemm_kernel<float, flt4>), dim3(total_tiles), dim3(256), 0, s, dev_jobs, njobs);
}

}  // namespace pcs
