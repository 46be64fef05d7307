// Batched dense products on the CDNA4 matrix cores.
//
// The wall-normal transforms (interpolation / differentiation to the padded
// grid, projection back), the spectral derivatives and the diagonalised
// Dirichlet solves are products C = alpha A B + beta C of a small operator A
// (at most 385 x 385, stored K-major so that an MFMA operand fragment is one
// 128-byte read) with a wide matrix B whose columns are the real and
// imaginary parts of every Fourier mode.
//
// One launch evaluates a table of such products.  A workgroup (four waves)
// owns a BM x 32 output tile: it stages the whole K x 32 panel of B in LDS
// (converted to the compute precision) with unrolled loads, then accumulates
// with 16x16x4 MFMAs (f64 or f32), reading A fragments straight from the
// L2-resident operator through a prefetch ring.  BM is chosen per table by
// the host: 16 (the four waves split K) for products too small to fill the
// chip, 64, or 128 for wide products (fewer re-reads of B).
#include "kernels.hpp"

namespace pcs {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

int gemm_prepare(GemmJob* jobs, int njobs, int bm) {
  int t = 0;
  for (int j = 0; j < njobs; ++j) {
    jobs[j].tiles_m = (jobs[j].m + bm - 1) / bm;
    const int tn = (jobs[j].n + GEMM_BN - 1) / GEMM_BN;
    jobs[j].tile0 = t;
    t += jobs[j].tiles_m * tn;
  }
  return t;
}

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline flt4 mfma(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  typedef dbl4 type;
};
template <>
struct Vec4<float> {
  typedef flt4 type;
};

constexpr int LDB = GEMM_BN + 8;  // padded LDS row of the B panel: the four k rows of one read start 16 banks apart

// Tile shapes.  RB: 16-row blocks per wave.  KS = 1: the four waves stack
// their rows (BM = 64 RB); KS = 4: the four waves share BM = 16 RB rows and
// each takes a quarter of K, the partial sums being added through LDS (for
// small products, where otherwise too few workgroups exist).
template <int RB, int KS>
struct Shape {
  static constexpr int BM = (KS == 1 ? 4 : 1) * RB * 16;
};

template <typename T, int RB>
__device__ inline void load_a(T (&a)[4][RB], const T* A, int lda, int K, const int (&arow)[RB],
                              const bool (&aok)[RB], int k0, int lk) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = k0 + 4 * u + lk;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[u][rb] = (k < K && aok[rb]) ? A[(size_t)k * lda + arow[rb]] : T(0);
  }
}

template <typename T, typename V4, int RB>
__device__ inline void mma_block(V4 (&acc)[RB][2], const T (&a)[4][RB], const T* Bs, int k0, int kend, int lk,
                                 int l16) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int kk = k0 + 4 * u;
    if (kk < kend) {
      const T b0 = Bs[(kk + lk) * LDB + l16], b1 = Bs[(kk + lk) * LDB + 16 + l16];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        acc[rb][0] = mfma(a[u][rb], b0, acc[rb][0]);
        acc[rb][1] = mfma(a[u][rb], b1, acc[rb][1]);
      }
    }
  }
}

template <typename T, typename TB, typename TC, int RB, int KS>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmJob* __restrict__ jobs, int njobs) {
  typedef typename Vec4<T>::type V4;
  extern __shared__ double gsm[];
  T* Bs = reinterpret_cast<T*>(gsm);  // [K4][LDB], K rounded up to a multiple of 4
  constexpr int BM = Shape<RB, KS>::BM;
  const int t = blockIdx.x;
  int jb = 0;
  while (jb + 1 < njobs && jobs[jb + 1].tile0 <= t) ++jb;
  const GemmJob J = jobs[jb];
  const T* A = static_cast<const T*>(J.A);
  const TB* B = static_cast<const TB*>(J.B);
  TC* C = static_cast<TC*>(J.C);
  const int lt = t - J.tile0;
  const int row0 = (lt % J.tiles_m) * BM;
  const int col0 = (lt / J.tiles_m) * GEMM_BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int K4 = (J.k + 3) & ~3;
  // stage the K x 32 panel of B (zero outside the matrix, and in the mean
  // columns when asked): 16 loads in flight per thread before any LDS store
  {
    constexpr int UNR = 16, RPP = 256 / GEMM_BN;  // rows per pass of the workgroup
    const int c = tid % GEMM_BN, rr = tid / GEMM_BN;
    const int gc = col0 + c;
    const bool cok = gc < J.n && !((J.flags & GEMM_ZERO_MEAN) && gc < 2);
    if (J.scale == SCALE_NONE) {
      for (int r0 = 0; r0 < K4; r0 += UNR * RPP) {
        T v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = r0 + u * RPP + rr;
          v[u] = (r < J.k && cok) ? T(B[(size_t)r * J.ldb + gc]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = r0 + u * RPP + rr;
          if (r < K4) Bs[r * LDB + c] = v[u];
        }
      }
    } else {
      // B row r is eigen coefficient r of column gc's mode: scale by the
      // inverse of that mode's Helmholtz symbol (see EigScale)
      const EigScale es = *J.es;
      const int mode = cok ? gc >> 1 : 0, iz = mode / es.nkx, ix = mode - iz * es.nkx;
      const double kxv = es.kx[ix], kzv = (es.dim == 3) ? es.kz[iz] : 0.0;
      const double k2 = kxv * kxv + kzv * kzv;
      double a0, a1;  // symbol = a0 - a1 * lam
      if (J.scale == SCALE_C) {
        a0 = 1.0 / es.dt + 0.5 / es.wi + 0.5 * es.kappa * k2;
        a1 = 0.5 * es.kappa;
      } else {
        a0 = 1.0 / es.dt + 0.5 * es.nu * k2;
        a1 = 0.5 * es.nu;
      }
      const bool vz = (J.scale == SCALE_V) && mode == 0;
      for (int r0 = 0; r0 < K4; r0 += UNR * RPP) {
        double v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = r0 + u * RPP + rr;
          v[u] = (r < J.k && cok && !vz) ? double(B[(size_t)r * J.ldb + gc]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = r0 + u * RPP + rr;
          if (r < K4) {
            double f = 0.0;
            if (r < J.k) {
              const double lam = es.lam[r];
              f = 1.0 / (a0 - a1 * lam);
              if (J.scale == SCALE_V) f = f / (lam - k2);
            }
            Bs[r * LDB + c] = T(v[u] * f);
          }
        }
      }
    }
  }
  __syncthreads();
  const int l16 = lane & 15, lk = lane >> 4;
  const int wrow = row0 + (KS == 1 ? wave * RB * 16 : 0);
  int kbeg = 0, kend = K4;
  if (KS > 1) {
    const int kq = ((K4 / 4 + KS - 1) / KS) * 4;
    kbeg = min(wave * kq, K4);
    kend = min(kbeg + kq, K4);
  }
  int arow[RB];
  bool aok[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    arow[rb] = wrow + rb * 16 + l16;
    aok[rb] = arow[rb] < J.m;
  }
  V4 acc[RB][2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb][0] = acc[rb][1] = V4{0, 0, 0, 0};
  // A fragments come straight from the L2-resident operator through a ring of
  // four 16-deep register blocks: block b + 3 is requested while block b is
  // multiplied
  T a0[4][RB], a1[4][RB], a2[4][RB], a3[4][RB];
  const int nblk = (kend - kbeg + 15) / 16;
  auto kb = [&](int b) { return kbeg + 16 * b; };
  if (nblk > 0) load_a(a0, A, J.lda, J.k, arow, aok, kb(0), lk);
  if (nblk > 1) load_a(a1, A, J.lda, J.k, arow, aok, kb(1), lk);
  if (nblk > 2) load_a(a2, A, J.lda, J.k, arow, aok, kb(2), lk);
  for (int b = 0; b < nblk; b += 4) {
    if (b + 3 < nblk) load_a(a3, A, J.lda, J.k, arow, aok, kb(b + 3), lk);
    mma_block<T, V4, RB>(acc, a0, Bs, kb(b), kend, lk, l16);
    if (b + 1 >= nblk) break;
    if (b + 4 < nblk) load_a(a0, A, J.lda, J.k, arow, aok, kb(b + 4), lk);
    mma_block<T, V4, RB>(acc, a1, Bs, kb(b + 1), kend, lk, l16);
    if (b + 2 >= nblk) break;
    if (b + 5 < nblk) load_a(a1, A, J.lda, J.k, arow, aok, kb(b + 5), lk);
    mma_block<T, V4, RB>(acc, a2, Bs, kb(b + 2), kend, lk, l16);
    if (b + 3 >= nblk) break;
    if (b + 6 < nblk) load_a(a2, A, J.lda, J.k, arow, aok, kb(b + 6), lk);
    mma_block<T, V4, RB>(acc, a3, Bs, kb(b + 3), kend, lk, l16);
  }
  if (KS > 1) {
    // add the K-quarters: waves 1..3 park their partial tiles in LDS
    __syncthreads();
    T* red = Bs;
    if (wave > 0) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[(((wave - 1) * RB + rb) * 8 + bj * 4 + r) * 64 + lane] = acc[rb][bj][r];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w2 = 1; w2 < KS; ++w2)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[rb][bj][r] += red[(((w2 - 1) * RB + rb) * 8 + bj * 4 + r) * 64 + lane];
  }
  // Element D[i][j] of a 16x16 block lives in lane j + 16 * (i / 4), register
  // i % 4 for the f32 instruction, and in lane j + 16 * (i % 4), register
  // i / 4 for the f64 one (checked on gfx950 with a one-hot product).
  constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = wrow + rb * 16 + (f64 ? 4 * r + lk : 4 * lk + r);
        const int gc = col0 + bj * 16 + l16;
        if (gr < J.m && gc < J.n) {
          TC* cp = C + (size_t)gr * J.ldc + gc;
          double v = J.alpha * (double)acc[rb][bj][r];
          if (J.beta != 0.0) v += J.beta * (double)*cp;
          *cp = TC(v);
        }
      }
}

size_t gemm_lds_bytes(int kmax, int elem) {
  const size_t panel = (size_t)((kmax + 3) & ~3) * LDB * elem;
  const size_t red = (size_t)3 * 2 * 8 * 64 * elem;  // KS = 4 partial tiles (RB <= 2)
  return panel > red ? panel : red;
}

namespace {

template <typename T, typename TB, typename TC>
hipError_t set_attr3() {
  const int lim = 160 * 1024;
  hipError_t e =
      hipFuncSetAttribute((const void*)gemm_kernel<T, TB, TC, 1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)gemm_kernel<T, TB, TC, 1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)gemm_kernel<T, TB, TC, 2, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim);
  return e;
}

template <typename T, typename TB, typename TC>
void launch3(const GemmJob* dev_jobs, int total_tiles, int njobs, int bm, int kmax, hipStream_t s) {
  const size_t lds = gemm_lds_bytes(kmax, sizeof(T));
  if (bm == 16)
    hipLaunchKernelGGL((gemm_kernel<T, TB, TC, 1, 4>), dim3(total_tiles), dim3(256), lds, s, dev_jobs, njobs);
  else if (bm == 128)
    hipLaunchKernelGGL((gemm_kernel<T, TB, TC, 2, 1>), dim3(total_tiles), dim3(256), lds, s, dev_jobs, njobs);
  else
    hipLaunchKernelGGL((gemm_kernel<T, TB, TC, 1, 1>), dim3(total_tiles), dim3(256), lds, s, dev_jobs, njobs);
}

}  // namespace

hipError_t gemm_set_attributes() {
  hipError_t e = set_attr3<double, double, double>();
  if (e == hipSuccess) e = set_attr3<float, double, float>();
  if (e == hipSuccess) e = set_attr3<float, float, double>();
  if (e == hipSuccess) e = set_attr3<double, double, float>();
  if (e == hipSuccess) e = set_attr3<double, float, double>();
  return e;
}

void gemm_run(GemmType t, const GemmJob* dev_jobs, int total_tiles, int njobs, int bm, int kmax, hipStream_t s) {
  if (total_tiles <= 0 || njobs <= 0) return;
  switch (t) {
    case GEMM_DDD: launch3<double, double, double>(dev_jobs, total_tiles, njobs, bm, kmax, s); break;
    case GEMM_FDF: launch3<float, double, float>(dev_jobs, total_tiles, njobs, bm, kmax, s); break;
    case GEMM_FFD: launch3<float, float, double>(dev_jobs, total_tiles, njobs, bm, kmax, s); break;
    case GEMM_DDF: launch3<double, double, float>(dev_jobs, total_tiles, njobs, bm, kmax, s); break;
    case GEMM_DFD: launch3<double, float, double>(dev_jobs, total_tiles, njobs, bm, kmax, s); break;
    default: break;
  }
}

}  // namespace pcs
