// Batched dense products on the CDNA4 matrix cores.
//
// The wall-normal transforms (interpolation / differentiation to the padded
// grid, projection back), the spectral derivatives and the diagonalised
// Dirichlet solves are products C = alpha A B + beta C of a small operator A
// (a few hundred rows and columns, row-major, padded) with a wide matrix B
// whose columns are the real and imaginary parts of every Fourier mode.  Many
// products of one step share an operator, so one launch evaluates a whole
// table of them.  Two kernel families cover the range of table sizes; the
// host times both on the real tables once and keeps the faster tile shape.
//
// Register-direct kernel (small tables, where a product is short and its
// cost is mostly memory latency): each wave computes a 32 x 32 block with
// 16x16x4 MFMAs (f64 or f32) from operand fragments loaded from global memory
// straight into a three-slot register ring, two 16-wide k blocks ahead of the
// multiply, with no LDS traffic or barriers in the loop.  Within an MFMA
// k-step, lane group g (lanes 16g..16g+15) takes k = 16 b + 4 g + s for step
// s of block b, so the A fragments of a lane are four consecutive elements of
// an operator row (one vector load).  The four waves tile the output
// (TM x TN blocks) and split K (KS ways, k blocks dealt round-robin); the
// partial sums are added through LDS in a fixed order.
//
// LDS-tiled kernel (large tables, where operand reuse matters): the four
// waves (2 x 2) share a BM x BN tile; K is walked in chunks of KC whose A and
// B panels are read into registers as element pairs while the previous chunk
// is multiplied out of LDS, then written to the other LDS buffer (B converted
// to the compute precision and optionally zeroed in the mean columns).  LDS
// rows are padded so that the fragment reads of one MFMA hit distinct banks.
//
// Both deal workgroups to the eight XCDs in contiguous ranges of tiles, so
// the row tiles of one column panel share an L2, and a workgroup finds its
// product through a per-tile job map; both share the epilogue, which can
// scale each output element by the inverse Helmholtz symbol of its eigen
// index (row) and Fourier mode (column) and write a second, differently
// scaled copy.  The LDS-tiled kernel is instantiated once per product form
// (plain or parity) and takes the LDS its table needs (dynamic); the FP64
// products of a mixed-precision table stage half-depth parity chunks so that
// they fit the FP32 panels.  All sums run in a fixed order, so results are
// bitwise reproducible.
#include "kernels.hpp"

#include <type_traits>

namespace pcs {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt2 __attribute__((ext_vector_type(2)));

namespace {

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  typedef dbl4 v4;
  typedef dbl2 v2;
};
template <>
struct Vec<float> {
  typedef flt4 v4;
  typedef flt2 v2;
};

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline flt4 mfma(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Register-direct configurations: TM x TN wave blocks of 32 x 32, K split KS.
template <int CFG>
struct RCfg;
template <>
struct RCfg<0> {
  static constexpr int TM = 1, TN = 1, KS = 4;
};
template <>
struct RCfg<1> {
  static constexpr int TM = 2, TN = 1, KS = 2;
};
template <>
struct RCfg<2> {
  static constexpr int TM = 1, TN = 2, KS = 2;
};
template <>
struct RCfg<3> {
  static constexpr int TM = 2, TN = 2, KS = 1;
};
// LDS-tiled configurations: BM x BN tile, K chunk KC, NBUF LDS buffers (2:
// the next chunk is written to the other buffer while this one is multiplied;
// 1: twice the chunk in the same LDS, one more barrier per chunk).  Parity
// products use K chunks of PKC, so that their panels (B holds both halves)
// fit the LDS of the plain ones and the occupancy stays that of the plain
// kernel (measured: full-size parity chunks gain nothing and cost a
// workgroup per CU).
template <int CFG>
struct LCfg;
template <>
struct LCfg<4> {
  static constexpr int BM = 32, BN = 32, KC = 32, NBUF = 2, PKC = 16;
};
template <>
struct LCfg<5> {
  static constexpr int BM = 64, BN = 32, KC = 32, NBUF = 2, PKC = 16;
};
template <>
struct LCfg<6> {
  static constexpr int BM = 64, BN = 64, KC = 16, NBUF = 2, PKC = 8;
};
template <>
struct LCfg<7> {
  static constexpr int BM = 128, BN = 64, KC = 16, NBUF = 2, PKC = 8;
};
template <>
struct LCfg<8> {
  static constexpr int BM = 32, BN = 32, KC = 64, NBUF = 1, PKC = 32;
};
template <>
struct LCfg<9> {
  static constexpr int BM = 64, BN = 32, KC = 64, NBUF = 1, PKC = 32;
};
// deep parity chunks for small tables, whose time is the chain of chunk loads
template <>
struct LCfg<10> {
  static constexpr int BM = 32, BN = 32, KC = 32, NBUF = 1, PKC = 64;
};
template <>
struct LCfg<11> {
  static constexpr int BM = 32, BN = 32, KC = 32, NBUF = 2, PKC = 32;
};
template <>
struct LCfg<12> {
  static constexpr int BM = 64, BN = 64, KC = 16, NBUF = 2, PKC = 16;
};
template <>
struct LCfg<13> {
  static constexpr int BM = 64, BN = 64, KC = 16, NBUF = 1, PKC = 32;
};
constexpr int CFG_BM[GEMM_NCFG] = {32, 64, 32, 64, 32, 64, 64, 128, 32, 64, 32, 32, 64, 64, 0, 0, 0, 0};
constexpr int CFG_BN[GEMM_NCFG] = {32, 32, 64, 64, 32, 32, 64, 64, 32, 32, 32, 32, 64, 64, 32, 64, 16, 32};
// LDS (in elements of the compute precision) of an LDS-tiled configuration:
// the plain panels, the parity panels (A: BM rows of PKC, B: both halves,
// rows of BN + 4) and the larger of the two.  The kernel takes its LDS
// dynamically, sized for the forms and precisions its table holds.
template <int CFG>
constexpr int lds_plain() {
  return LCfg<CFG>::NBUF * LCfg<CFG>::BM * (LCfg<CFG>::KC + 2) +
         LCfg<CFG>::NBUF * LCfg<CFG>::KC * (LCfg<CFG>::BN + 16);
}
template <int CFG, int KDIV = 1>
constexpr int lds_par() {
  return LCfg<CFG>::NBUF * LCfg<CFG>::BM * (LCfg<CFG>::PKC / KDIV + 2) +
         LCfg<CFG>::NBUF * 2 * (LCfg<CFG>::PKC / KDIV) * (LCfg<CFG>::BN + 4);
}
// FP64 parity products inside a table of FP32 products take chunks of half
// the depth (staged by fewer threads where a panel falls below 512
// elements): their panels then take the bytes of the FP32 panels, and the
// table's LDS stays that of its FP32 products.
// a panel of p elements is staged by 256 threads in element pairs: whole
// pairs for every thread (p >= 512, a multiple of 512) or one pair for the
// first p / 2 threads (p < 512, a divisor of 512)
constexpr bool stageable(int p) { return p >= 512 ? p % 512 == 0 : 512 % p == 0; }
template <int CFG>
constexpr bool ddd_half() {
  constexpr int K = LCfg<CFG>::PKC / 2;
  return K % 4 == 0 && stageable(K * LCfg<CFG>::BM) && stageable(K * LCfg<CFG>::BN);
}
template <int CFG>
constexpr int lds_doubles() {
  return lds_plain<CFG>() > lds_par<CFG>() ? lds_plain<CFG>() : lds_par<CFG>();
}


// Workgroup b runs on XCD b % 8; logical tiles are dealt so that XCD x gets
// one contiguous range (a bijection for any tile count).
__device__ inline int xcd_tile(int b, int total) {
  const int q = total >> 3, r = total & 7;
  const int x = b & 7, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Job of logical tile t, from the table's tile map (one load: a search
// through the job table would be a chain of dependent loads at the start of
// every workgroup, from a table that is cold in a graph-replayed step).
__device__ inline const GemmJob* tile_job(const GemmJob* __restrict__ jobs, const int* __restrict__ tmap, int t) {
  return jobs + gmem(tmap)[t];
}

// Inverse Helmholtz symbol of kind `kind` for eigenvalue lam and wavenumber
// magnitude k2 (mode 0 is the mean slot); ia is the scheme's leading
// coefficient over dt and th its implicit weight.
__device__ inline double eig_factor(const EigScale& es, int kind, double lam, double k2, bool mean) {
  if (kind == SCALE_C) return 1.0 / (es.ia + es.th / es.wi + es.th * es.kappa * (k2 - lam));
  const double f = 1.0 / (es.ia + es.th * es.nu * (k2 - lam));
  if (kind == SCALE_V) return mean ? 0.0 : f / (lam - k2);
  return f;
}

// Stores a lane's RB x CB accumulator blocks whose top-left corner is
// (r0, c0), rows below min(m, mlim) only.  Element D[i][j] of a 16x16 block lives in lane j + 16 * (i / 4),
// register i % 4 for the f32 instruction, and in lane j + 16 * (i % 4),
// register i / 4 for the f64 one (checked on gfx950 with a one-hot product).
// The eigenvalues and wavenumbers the scaling needs are read before the
// first store.
template <typename T, typename TC, int RB, int CB, typename V4>
__device__ inline void store_tile(const GemmJob* __restrict__ jp, const V4 (&acc)[RB][CB], int r0, int c0, int lk,
                                  int l16, int mlim = 1 << 30) {
  constexpr bool f64 = sizeof(T) == 8;
  const GemmJob J = *jp;
  const gptr<TC> C = gmem(static_cast<TC*>(J.C));
  const gptr<TC> C2 = gmem(static_cast<TC*>(J.C2));
  auto row_of = [&](int rb, int r) { return r0 + rb * 16 + (f64 ? 4 * r + lk : 4 * lk + r); };
  auto col_of = [&](int cb) { return c0 + cb * 16 + l16; };
  const bool scaled = J.scale != SCALE_NONE;
  EigScale es{};
  double lam[RB][4], k2[CB];
  bool mean[CB];
  if (scaled) {
    es = *J.es;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int gc = col_of(cb);
      const int mode = gc < J.n ? gc >> 1 : 0, iz = mode / es.nkx, ix = mode - iz * es.nkx;
      const double kxv = gmem(es.kx)[ix], kzv = (es.dim == 3) ? gmem(es.kz)[iz] : 0.0;
      k2[cb] = kxv * kxv + kzv * kzv;
      mean[cb] = mode == 0;
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row_of(rb, r);
        lam[rb][r] = gmem(es.lam)[gr < J.m ? gr : 0];
      }
  }
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row_of(rb, r), gc = col_of(cb);
        if (gr < J.m && gr < mlim && gc < J.n) {
          const double v = J.alpha * (double)acc[rb][cb][r];
          const gptr<TC> cp = C + (size_t)gr * J.ldc + gc;
          double o = scaled ? v * eig_factor(es, J.scale, lam[rb][r], k2[cb], mean[cb]) : v;
          if (J.beta != 0.0) o += J.beta * (double)*cp;
          *cp = TC(o);
          if (C2)
            C2[(size_t)gr * J.ldc + gc] =
                TC(J.scale2 != SCALE_NONE ? v * eig_factor(es, J.scale2, lam[rb][r], k2[cb], mean[cb]) : v);
        }
      }
}

}  // namespace

int gemm_prepare(GemmJob* jobs, int njobs, int cfg) {
  const int bm = CFG_BM[cfg], bn = CFG_BN[cfg];
  int t = 0;
  for (int j = 0; j < njobs; ++j) {
    const int rows = jobs[j].kind != PAR_NONE ? bm / 2 : bm;  // a parity tile: BM/2 rows of E and of O
    // the B-stationary configurations cover every row of a product per tile
    // (and the paired next product's rows: see GemmJob::pair)
    jobs[j].tiles_m = gemm_cfg_bst(cfg) ? 1 : (jobs[j].m + rows - 1) / rows;
    const int tn = (gemm_cfg_bst(cfg) && jobs[j].pair == 2) ? 0 : (jobs[j].n + bn - 1) / bn;
    jobs[j].tile0 = t;
    t += jobs[j].tiles_m * tn;
  }
  return t;
}

// ------------------------------------------------------------ register-direct kernel
template <typename T, typename TB, typename TC, int CFG>
__device__ __attribute__((always_inline)) inline void reg_body(const GemmJob* __restrict__ jp, int t,
                                                               double* smem) {
  constexpr int TM = RCfg<CFG>::TM, TN = RCfg<CFG>::TN, KS = RCfg<CFG>::KS;
  constexpr int BM = 32 * TM, BN = 32 * TN;
  typedef typename Vec<T>::v4 V4;
  T* red = reinterpret_cast<T*>(smem);
  const int lt = t - jp->tile0, tiles_m = jp->tiles_m;
  const int row0 = (lt % tiles_m) * BM, col0 = (lt / tiles_m) * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int ks = wave % KS, tm = (wave / KS) % TM, tn = wave / (KS * TM);
  const int wrow = row0 + 32 * tm, wcol = col0 + 32 * tn;
  const int M = jp->m, N = jp->n, K = jp->k;

  V4 acc[2][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};

  if (wrow < M && wcol < N) {
    const gptr<const T> A = gmem(static_cast<const T*>(jp->A));
    const gptr<const TB> B = gmem(static_cast<const TB*>(jp->B));
    const int lda = jp->lda, ldb = jp->ldb;
    const gptr<const T> ar0 = A + (size_t)(wrow + l16) * lda + 4 * lk;
    const gptr<const T> ar1 = ar0 + (size_t)16 * lda;
    const bool zm = (jp->flags & GEMM_ZERO_MEAN) != 0;
    const int bc0 = wcol + l16, bc1 = bc0 + 16;
    const bool bok0 = bc0 < N && !(zm && bc0 < 2), bok1 = bc1 < N && !(zm && bc1 < 2);
    const int nkb = (K + 15) >> 4;
    const int nb = ks < nkb ? (nkb - ks + KS - 1) / KS : 0;
    V4 a0[2], a1[2], a2[2];
    T b0[2][4], b1[2][4], b2[2][4];
    auto load = [&](V4 (&a)[2], T (&b)[2][4], int i) {
      const int kb = 16 * (ks + KS * i);
      a[0] = *reinterpret_cast<gptr<const V4>>(ar0 + kb);
      a[1] = *reinterpret_cast<gptr<const V4>>(ar1 + kb);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = kb + 4 * lk + s;
        const gptr<const TB> br = B + (size_t)kk * ldb;
        b[0][s] = (kk < K && bok0) ? T(br[bc0]) : T(0);
        b[1][s] = (kk < K && bok1) ? T(br[bc1]) : T(0);
      }
    };
    auto mul = [&](const V4 (&a)[2], const T (&b)[2][4]) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mfma(a[rb][s], b[cb][s], acc[rb][cb]);
    };
    if (nb > 0) load(a0, b0, 0);
    if (nb > 1) load(a1, b1, 1);
    for (int i = 0; i < nb; i += 3) {
      if (i + 2 < nb) load(a2, b2, i + 2);
      mul(a0, b0);
      if (i + 1 >= nb) break;
      if (i + 3 < nb) load(a0, b0, i + 3);
      mul(a1, b1);
      if (i + 2 >= nb) break;
      if (i + 4 < nb) load(a1, b1, i + 4);
      mul(a2, b2);
    }
  }

  if constexpr (KS > 1) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[((wave * 4 + rb * 2 + cb) * 4 + r) * 64 + lane] = acc[rb][cb][r];
    __syncthreads();
    if (ks != 0) return;
#pragma unroll
    for (int w2 = 1; w2 < KS; ++w2)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[rb][cb][r] += red[(((wave + w2) * 4 + rb * 2 + cb) * 4 + r) * 64 + lane];
  }
  if (wrow >= M || wcol >= N) return;
  store_tile<T, TC, 2, 2>(jp, acc, wrow, wcol, lk, l16);
}

// A table may mix FP64 products (type GEMM_DDD) with products of its own
// precision combination; each workgroup branches once on its job's type.
template <typename T, typename TB, typename TC>
constexpr bool dual_type() {
  return !(std::is_same<T, double>::value && std::is_same<TB, double>::value && std::is_same<TC, double>::value);
}

template <typename T, typename TB, typename TC, int CFG>
__global__ __launch_bounds__(256) void gemm_reg_kernel(const GemmJob* __restrict__ jobs, const int* __restrict__ tmap,
                                                       int total) {
  __shared__ double red[RCfg<CFG>::KS > 1 ? 4 * 16 * 64 : 1];
  const int t = xcd_tile(blockIdx.x, total);
  const GemmJob* jp = tile_job(jobs, tmap, t);
  if (masked(jp->skip)) return;
  if (dual_type<T, TB, TC>() && jp->type == GEMM_DDD)
    reg_body<double, double, double, CFG>(jp, t, red);
  else
    reg_body<T, TB, TC, CFG>(jp, t, red);
}

// ------------------------------------------------------------ LDS-tiled kernel
template <typename T, typename TB, typename TC, int CFG>
__device__ __attribute__((always_inline)) inline void lds_body(const GemmJob* __restrict__ jp, int t,
                                                               double* smem) {
  constexpr int BM = LCfg<CFG>::BM, BN = LCfg<CFG>::BN, KC = LCfg<CFG>::KC, NBUF = LCfg<CFG>::NBUF;
  constexpr int WM = BM / 2, WN = BN / 2, RB = WM / 16, CB = WN / 16;
  // A panel row-major [BM][PA] (pitch KC + 2 keeps the 16 rows of a fragment
  // read on distinct banks), B panel [KC][PB]
  constexpr int PA = KC + 2, PB = BN + 16;
  constexpr int NA = KC * BM / 512, NB = KC * BN / 512;  // element pairs per thread and chunk
  constexpr int RA = 512 / KC, SB = 512 / BN;            // row step between a thread's pairs
  static_assert(NA >= 1 && NB >= 1 && KC % 4 == 0, "tile shape");
  typedef typename Vec<T>::v4 V4;
  typedef typename Vec<T>::v2 AP;
  typedef typename Vec<TB>::v2 BP;
  T (*As)[BM * PA] = reinterpret_cast<T (*)[BM * PA]>(smem);  // [NBUF][BM * PA]
  T (*Bs)[KC * PB] = reinterpret_cast<T (*)[KC * PB]>(smem + (NBUF * BM * PA * sizeof(T) + 7) / 8);
  const int lt = t - jp->tile0, tiles_m = jp->tiles_m;
  const int row0 = (lt % tiles_m) * BM, col0 = (lt / tiles_m) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * WM, wc = (wave & 1) * WN;
  const int M = jp->m, N = jp->n, K = jp->k, lda = jp->lda, ldb = jp->ldb;
  const gptr<const T> A = gmem(static_cast<const T*>(jp->A));
  const gptr<const TB> B = gmem(static_cast<const TB*>(jp->B));

  // staging positions: a thread's A pairs are (row ra + u RA, k pair 2 kp);
  // its B pairs share one column pair and step through k
  const int kp = 2 * (tid % (KC / 2)), ra = tid / (KC / 2);
  const int cb2 = 2 * (tid % (BN / 2)), kb = tid / (BN / 2);
  const int gc = col0 + cb2;
  const bool bpair = (((ldb | N) & 1) == 0) && ((reinterpret_cast<uintptr_t>(B) & (2 * sizeof(TB) - 1)) == 0);
  const bool zm = (jp->flags & GEMM_ZERO_MEAN) != 0;
  const bool c0ok = gc < N && !(zm && gc < 2), c1ok = gc + 1 < N && !(zm && gc + 1 < 2);

  AP ar[NA];
  TB br[NB][2];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      // rows up to gemm_rows(m) are allocated and zero; k pairs stop at K
      const int kk = k0 + kp;
      ar[u] = kk < K ? *reinterpret_cast<gptr<const AP>>(A + (size_t)(row0 + ra + u * RA) * lda + kk) : AP{0, 0};
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int kk = k0 + kb + u * SB;
      const gptr<const TB> bp = B + (size_t)kk * ldb + gc;
      if (bpair) {
        if (kk < K && gc < N) {
          const BP v = *reinterpret_cast<gptr<const BP>>(bp);
          br[u][0] = v[0];
          br[u][1] = v[1];
        } else {
          br[u][0] = br[u][1] = TB(0);
        }
      } else {
        br[u][0] = (kk < K && gc < N) ? bp[0] : TB(0);
        br[u][1] = (kk < K && gc + 1 < N) ? bp[1] : TB(0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) *reinterpret_cast<AP*>(&As[buf][(ra + u * RA) * PA + kp]) = ar[u];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      AP v;
      v[0] = c0ok ? T(br[u][0]) : T(0);
      v[1] = c1ok ? T(br[u][1]) : T(0);
      *reinterpret_cast<AP*>(&Bs[buf][(kb + u * SB) * PB + cb2]) = v;
    }
  };

  V4 acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
  const bool active = (row0 + wr < M) && (col0 + wc < N);
  const int nch = (K + KC - 1) / KC;
  auto multiply = [&](int buf) {
    if (!active) return;
    const T* as = &As[buf][(wr + l16) * PA + lk];
    const T* bs = &Bs[buf][lk * PB + wc + l16];
#pragma unroll
    for (int kq = 0; kq < KC / 4; ++kq) {
      T a[RB], b[CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) a[rb] = as[rb * 16 * PA + 4 * kq];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b[cb] = bs[4 * kq * PB + cb * 16];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma(a[rb], b[cb], acc[rb][cb]);
    }
  };
  load(0);
  if constexpr (NBUF == 2) {
    store(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      const int buf = c & 1;
      if (c + 1 < nch) load((c + 1) * KC);
      multiply(buf);
      if (c + 1 < nch) store(buf ^ 1);
      __syncthreads();
    }
  } else {
    for (int c = 0; c < nch; ++c) {
      store(0);
      __syncthreads();
      if (c + 1 < nch) load((c + 1) * KC);
      multiply(0);
      __syncthreads();
    }
  }
  if (!active) return;
  store_tile<T, TC, RB, CB>(jp, acc, row0 + wr, col0 + wc, lk, l16);
}

// ------------------------------------------------------------ parity products (LDS-tiled)
// Writes the E and O blocks of one lane (same layout as store_tile) as the
// outputs of a parity product: E + O at row i and sigma (E - O) at row
// mf-1-i, or E at row i and O at row m + i (eigen coefficients, optionally
// scaled by the inverse Helmholtz symbol of their row).
template <typename T, typename TC, int RB, int CB, typename V4>
__device__ inline void store_par(const GemmJob* __restrict__ jp, const V4 (&accE)[RB][CB], const V4 (&accO)[RB][CB],
                                 int r0, int c0, int lk, int l16) {
  constexpr bool f64 = sizeof(T) == 8;
  const GemmJob J = *jp;
  const gptr<TC> C = gmem(static_cast<TC*>(J.C));
  const gptr<TC> C2 = gmem(static_cast<TC*>(J.C2));
  const bool split = J.kind == PAR_FOLD_SPLIT;
  const bool scaled = split && J.scale != SCALE_NONE;
  EigScale es{};
  if (scaled) es = *J.es;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int gc = c0 + cb * 16 + l16;
    if (gc >= J.n) continue;
    double k2 = 0;
    bool mean = false;
    if (scaled) {
      const int mode = gc >> 1, iz = mode / es.nkx, ix = mode - iz * es.nkx;
      const double kxv = gmem(es.kx)[ix], kzv = (es.dim == 3) ? gmem(es.kz)[iz] : 0.0;
      k2 = kxv * kxv + kzv * kzv;
      mean = mode == 0;
    }
    auto put = [&](int row, double v) {
      if (scaled) {
        const double lam = gmem(es.lam)[row];
        C[(size_t)row * J.ldc + gc] = TC(v * eig_factor(es, J.scale, lam, k2, mean));
        if (C2) C2[(size_t)row * J.ldc + gc] = TC(J.scale2 != SCALE_NONE ? v * eig_factor(es, J.scale2, lam, k2, mean) : v);
      } else {
        C[(size_t)row * J.ldc + gc] = TC(v);
        if (C2) C2[(size_t)row * J.ldc + gc] = TC(v);
      }
    };
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = r0 + rb * 16 + (f64 ? 4 * r + lk : 4 * lk + r);
        if (gi >= J.m) continue;
        const double e = J.alpha * (double)accE[rb][cb][r], o = J.alpha * (double)accO[rb][cb][r];
        if (split) {
          put(gi, e);
          if (J.m + gi < J.mf) put(J.m + gi, o);
        } else {
          put(gi, e + o);
          const int mr = J.mf - 1 - gi;
          if (mr > gi) put(mr, J.sigma * (e - o));
        }
      }
  }
}

// A tile covers BM/2 rows of E and the same rows of O: waves 0, 1 multiply
// the even part (Ae rows, Be panel), waves 2, 3 the odd part (Ao rows, Bo
// panel); at the end the odd waves hand their blocks to the even waves
// through LDS, which write both mirrored output rows.
template <typename T, typename TB, typename TC, int CFG, int KDIV = 1>
__device__ __attribute__((always_inline)) inline void lds_par_body(const GemmJob* __restrict__ jp, int t,
                                                                   double* smem) {
  constexpr int BM = LCfg<CFG>::BM, BN = LCfg<CFG>::BN, KC = LCfg<CFG>::PKC / KDIV, NBUF = LCfg<CFG>::NBUF;
  constexpr int HM = BM / 2, WN = BN / 2, RB = HM / 16, CB = WN / 16;
  constexpr int PA = KC + 2, PB = BN + 4;
  // element pairs per thread and chunk; a panel smaller than 512 elements
  // (half-depth chunks) is staged by the first threads only
  constexpr bool AF = KC * BM >= 512, BF = KC * BN >= 512;
  constexpr int NA = AF ? KC * BM / 512 : 1, NB = BF ? KC * BN / 512 : 1;
  constexpr int RA = 512 / KC, SB = 512 / BN;
  static_assert(KC % 4 == 0 && stageable(KC * BM) && stageable(KC * BN), "tile shape");
  static_assert(lds_doubles<CFG>() * 8 <= 64 * 1024, "LDS");
  // odd -> even hand-over in rounds of XR row blocks (whatever fits the
  // parity panels' LDS)
  constexpr int XR = (2 * RB * CB * 4 * 64 <= lds_par<CFG, KDIV>()) ? RB : 1;
  static_assert(2 * XR * CB * 4 * 64 <= lds_par<CFG, KDIV>() && RB % XR == 0, "exchange area");
  typedef typename Vec<T>::v4 V4;
  typedef typename Vec<T>::v2 AP;
  typedef typename Vec<TB>::v2 BP;
  T (*As)[BM * PA] = reinterpret_cast<T (*)[BM * PA]>(smem);  // [NBUF][BM * PA]: Ae rows, then Ao rows
  T (*Bs)[2][KC * PB] = reinterpret_cast<T (*)[2][KC * PB]>(smem + (NBUF * BM * PA * sizeof(T) + 7) / 8);
  const int lt = t - jp->tile0, tiles_m = jp->tiles_m;
  const int row0 = (lt % tiles_m) * HM, col0 = (lt / tiles_m) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int par = wave >> 1, wc = (wave & 1) * WN;
  const int M = jp->m, N = jp->n, K = jp->k, KF = jp->kf, lda = jp->lda, ldb = jp->ldb;
  const bool fold = jp->kind != PAR_SPLIT_UNFOLD;
  const gptr<const T> A = gmem(static_cast<const T*>(jp->A));
  const gptr<const T> A2 = gmem(static_cast<const T*>(jp->A2));
  const gptr<const TB> B = gmem(static_cast<const TB*>(jp->B));

  const int kp = 2 * (tid % (KC / 2)), ra = tid / (KC / 2);
  const int cb2 = 2 * (tid % (BN / 2)), kb = tid / (BN / 2);
  const bool aon = AF || ra < BM, bon = BF || kb < KC;  // this thread stages A / B pairs
  const int gc = col0 + cb2;
  const bool bpair = (((ldb | N) & 1) == 0) && ((reinterpret_cast<uintptr_t>(B) & (2 * sizeof(TB) - 1)) == 0);
  const bool zm = (jp->flags & GEMM_ZERO_MEAN) != 0;
  const bool c0ok = gc < N && !(zm && gc < 2), c1ok = gc + 1 < N && !(zm && gc + 1 < 2);

  AP ar[NA];
  TB be[NB][2], bo[NB][2];
  auto brow = [&](int kk, TB (&v)[2]) {  // B row kk at this thread's column pair
    const gptr<const TB> bp = B + (size_t)kk * ldb + gc;
    if (bpair) {
      if (gc < N) {
        const BP x = *reinterpret_cast<gptr<const BP>>(bp);
        v[0] = x[0];
        v[1] = x[1];
      } else {
        v[0] = v[1] = TB(0);
      }
    } else {
      v[0] = gc < N ? bp[0] : TB(0);
      v[1] = gc + 1 < N ? bp[1] : TB(0);
    }
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int r = ra + u * RA, kk = k0 + kp;
      const gptr<const T> src = (r < HM ? A : A2) + (size_t)(row0 + (r < HM ? r : r - HM)) * lda + kk;
      ar[u] = (aon && kk < K) ? *reinterpret_cast<gptr<const AP>>(src) : AP{0, 0};
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int kk = k0 + kb + u * SB;
      be[u][0] = be[u][1] = bo[u][0] = bo[u][1] = TB(0);
      if (bon && kk < K) {
        if (fold) {
          const int km = KF - 1 - kk;
          TB x[2];
          brow(kk, x);
          if (km > kk) {
            TB y[2];
            brow(km, y);
            be[u][0] = x[0] + y[0];
            be[u][1] = x[1] + y[1];
            bo[u][0] = x[0] - y[0];
            bo[u][1] = x[1] - y[1];
          } else {
            be[u][0] = x[0];
            be[u][1] = x[1];
          }
        } else {
          brow(kk, be[u]);
          if (K + kk < KF) brow(K + kk, bo[u]);
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u)
      if (aon) *reinterpret_cast<AP*>(&As[buf][(ra + u * RA) * PA + kp]) = ar[u];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (!bon) continue;
      AP v;
      v[0] = c0ok ? T(be[u][0]) : T(0);
      v[1] = c1ok ? T(be[u][1]) : T(0);
      *reinterpret_cast<AP*>(&Bs[buf][0][(kb + u * SB) * PB + cb2]) = v;
      v[0] = c0ok ? T(bo[u][0]) : T(0);
      v[1] = c1ok ? T(bo[u][1]) : T(0);
      *reinterpret_cast<AP*>(&Bs[buf][1][(kb + u * SB) * PB + cb2]) = v;
    }
  };

  V4 acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
  const bool active = (row0 < M) && (col0 + wc < N);
  const int nch = (K + KC - 1) / KC;
  auto multiply = [&](int buf) {
    if (!active) return;
    const T* as = &As[buf][(par * HM + l16) * PA + lk];
    const T* bs = &Bs[buf][par][lk * PB + wc + l16];
#pragma unroll
    for (int kq = 0; kq < KC / 4; ++kq) {
      T a[RB], b[CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) a[rb] = as[rb * 16 * PA + 4 * kq];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b[cb] = bs[4 * kq * PB + cb * 16];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma(a[rb], b[cb], acc[rb][cb]);
    }
  };
  load(0);
  if constexpr (NBUF == 2) {
    store(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      const int buf = c & 1;
      if (c + 1 < nch) load((c + 1) * KC);
      multiply(buf);
      if (c + 1 < nch) store(buf ^ 1);
      __syncthreads();
    }
  } else {
    for (int c = 0; c < nch; ++c) {
      store(0);
      __syncthreads();
      if (c + 1 < nch) load((c + 1) * KC);
      multiply(0);
      __syncthreads();
    }
  }
  // odd waves hand their blocks to the even waves (the panels are no longer read)
  T* xch = reinterpret_cast<T*>(smem) + (size_t)(wave & 1) * XR * CB * 4 * 64;
  V4 accO[RB][CB];
#pragma unroll
  for (int r0 = 0; r0 < RB; r0 += XR) {
    if (par == 1) {
#pragma unroll
      for (int rb = 0; rb < XR; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int r = 0; r < 4; ++r) xch[((rb * CB + cb) * 4 + r) * 64 + lane] = acc[r0 + rb][cb][r];
    }
    __syncthreads();
    if (par == 0) {
#pragma unroll
      for (int rb = 0; rb < XR; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int r = 0; r < 4; ++r) accO[r0 + rb][cb][r] = xch[((rb * CB + cb) * 4 + r) * 64 + lane];
    }
    if (r0 + XR < RB) __syncthreads();
  }
  if (par == 1 || !active) return;
  store_par<T, TC, RB, CB>(jp, acc, accO, row0, col0 + wc, lk, l16);
}

// ------------------------------------------------------------ B-stationary parity kernel
// One workgroup per (product, panel of BN output columns).  The folded (or
// split) B panel of the whole K range is staged into LDS once, converted to
// the compute precision (K padded with zero rows to a multiple of 16); the
// NW waves (four or eight: configurations 14, 15 and 17 are the 32- and
// 64-column panels in four waves and the 32-column ones in eight, 16 the
// 16-column ones in eight; eight waves share one staging among twice the
// waves) sweep the product's 16-row blocks of E and O (block r
// by wave r mod NW), each over all BN columns, with the A fragments streamed from
// global memory (the operators are small and stay in L2) one 16-wide k block
// ahead of the multiply.  Lane group g takes k = 16 b + 4 g + s at MFMA step
// s of block b, so a lane's A fragment of a block is one vector load.  Every
// element of B is read from HBM once per product, where the LDS-tiled kernel
// reads it once per row tile.  Row pitch of the staged panel: BN + 4
// elements in FP32 (the four lane groups' rows of a step fall on disjoint
// banks), BN + 2 in FP64, where both pitches leave two-way conflicts and the
// narrower one lets two 32-column panels of 257-point products share a CU.
template <typename T, int BN>
constexpr int bst_pitch() {
  return BN + (sizeof(T) == 8 ? 2 : 4);
}
template <typename T, typename TB, typename TC, int BN, int NW = 4>
__device__ __attribute__((always_inline)) inline void bst_body(const GemmJob* __restrict__ jp, int t, double* smem) {
  constexpr int CB = BN / 16, PB = bst_pitch<T, BN>();
  typedef typename Vec<T>::v4 V4;
  const int col0 = (t - jp->tile0) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int N = jp->n, K = jp->k, KF = jp->kf, ldb = jp->ldb;
  const int K16 = (K + 15) & ~15;
  const bool fold = jp->kind != PAR_SPLIT_UNFOLD;
  const bool zm = (jp->flags & GEMM_ZERO_MEAN) != 0;
  T* Be = reinterpret_cast<T*>(smem);
  T* Bo = Be + (size_t)K16 * PB;
  const gptr<const TB> B = gmem(static_cast<const TB*>(jp->B));
  // stage the panel, columns fastest (coalesced rows of B): each thread
  // loads runs of VW consecutive columns (16 bytes) of a row and of its
  // mirror row, U runs in flight before their LDS stores (one vector load
  // per run where the row stride and the base keep it aligned)
  constexpr int VW = 16 / sizeof(TB), U = 4;
  typedef TB TBv __attribute__((ext_vector_type(VW)));
  const bool vec = (ldb % VW) == 0 && (reinterpret_cast<uintptr_t>(jp->B) & 15) == 0;
  const int totv = K16 * (BN / VW);
  for (int e0 = 0; e0 < totv; e0 += U * (64 * NW)) {
    TBv x[U], y[U];
    int kk[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = (e0 + u * (64 * NW) + tid) * VW;
      kk[u] = e / BN;
      c[u] = e - kk[u] * BN;
      const int gc = col0 + c[u];
      x[u] = y[u] = TBv{};
      if (e0 + u * (64 * NW) + tid < totv && kk[u] < K && gc < N) {
        const int kr = fold ? KF - 1 - kk[u] : K + kk[u];
        const bool hy = fold ? kr > kk[u] : kr < KF;
        if (vec && gc + VW <= N) {
          x[u] = *reinterpret_cast<gptr<const TBv>>(B + (size_t)kk[u] * ldb + gc);
          if (hy) y[u] = *reinterpret_cast<gptr<const TBv>>(B + (size_t)kr * ldb + gc);
        } else {
#pragma unroll
          for (int i = 0; i < VW; ++i)
            if (gc + i < N) {
              x[u][i] = B[(size_t)kk[u] * ldb + gc + i];
              if (hy) y[u][i] = B[(size_t)kr * ldb + gc + i];
            }
        }
        if (zm && gc < 2) {
#pragma unroll
          for (int i = 0; i < VW; ++i)
            if (gc + i < 2) x[u][i] = y[u][i] = TB(0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u * (64 * NW) + tid >= totv) continue;
      const int o = kk[u] * PB + c[u];
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        if (fold) {
          Be[o + i] = T(x[u][i] + y[u][i]);
          Bo[o + i] = T(x[u][i] - y[u][i]);
        } else {
          Be[o + i] = T(x[u][i]);
          Bo[o + i] = T(y[u][i]);
        }
      }
    }
  }
  __syncthreads();
  const int nkb = K16 >> 4;
  const T* be = Be + (size_t)(4 * lk) * PB + l16;
  const T* bo = Bo + (size_t)(4 * lk) * PB + l16;
  // the row sweep of one product over the staged panel: this job's, then
  // the paired next job's (same panel, its own operator and output)
  for (const GemmJob* q = jp;; ++q) {
    const gptr<const T> A = gmem(static_cast<const T*>(q->A));
    const gptr<const T> A2 = gmem(static_cast<const T*>(q->A2));
    const int nrb = (q->m + 15) >> 4, qlda = q->lda;
    for (int rb = wave; rb < nrb; rb += NW) {
      V4 E[1][CB], O[1][CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) E[0][cb] = O[0][cb] = V4{0, 0, 0, 0};
      // A rows are allocated (zero) up to gemm_rows(m) and lda = K16
      const gptr<const V4> ae = reinterpret_cast<gptr<const V4>>(A + (size_t)(rb * 16 + l16) * qlda + 4 * lk);
      const gptr<const V4> ao = reinterpret_cast<gptr<const V4>>(A2 + (size_t)(rb * 16 + l16) * qlda + 4 * lk);
      V4 xe = ae[0], xo = ao[0];
      for (int b = 0; b < nkb; ++b) {
        const V4 ce = xe, co = xo;
        if (b + 1 < nkb) {
          xe = ae[4 * (b + 1)];
          xo = ao[4 * (b + 1)];
        }
        const T* pe = be + (size_t)(16 * b) * PB;
        const T* po = bo + (size_t)(16 * b) * PB;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            E[0][cb] = mfma(ce[s2], pe[s2 * PB + cb * 16], E[0][cb]);
            O[0][cb] = mfma(co[s2], po[s2 * PB + cb * 16], O[0][cb]);
          }
      }
      store_par<T, TC, 1, CB>(q, E, O, rb * 16, col0, lk, l16);
    }
    if (q != jp || jp->pair != 1) break;
  }
}

// ------------------------------------------------------------ error-compensated FP32 products
// Types GEMM_CDF (B FP64, C FP32) and GEMM_CFD (B FP32, C FP64): the products
// of the B-stationary kernel in FP32 arithmetic with error compensation.
// Every operand is split into an FP32 head and tail, v = hi + lo with
// hi = fp32(v), lo = fp32(v - hi): the operator halves once on the host (A, A2
// the heads, Alo, A2lo the tails), the folded B panel (formed in FP64) while
// it is staged (four LDS panels).  Each MFMA step (four k) computes the head
// product hi*hi into a fresh accumulator and adds it to a running sum with
// Knuth's TwoSum (sum and rounding error kept apart), while the two cross
// products hi*lo and lo*hi, of relative size 2^-24, accumulate in plain FP32.
// The output is hi + lo sum + cross terms, formed in FP64 and rounded once to
// the output precision.  Compared with plain FP32 this removes the rounding of
// the inputs and of the operator and leaves the rounding of four-term FP32
// partial sums (the TwoSum recovers that of their accumulation).  The FP32
// matrix instruction evaluates each output as a chain of fused multiply-adds
// over its four k, starting from the accumulator input (exact products, one
// rounding per addition; checked on the device with operands whose sums
// round differently in each order), so the head products' partial sums keep
// one FP32 rounding per term, and the error stays of the order of plain
// FP32's.
__device__ inline void two_sum(float& s, float& e, float x) {
  const float t = s + x;
  const float bp = t - s;
  e += (s - (t - bp)) + (x - bp);
  s = t;
}

template <typename TB, typename TC, int BN>
__device__ __attribute__((always_inline)) inline void bst_comp_body(const GemmJob* __restrict__ jp, int t,
                                                                    double* smem) {
  constexpr int CB = BN / 16, PB = bst_pitch<float, BN>();
  const int col0 = (t - jp->tile0) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int M = jp->m, N = jp->n, K = jp->k, KF = jp->kf, lda = jp->lda, ldb = jp->ldb;
  const int K16 = (K + 15) & ~15;
  const bool fold = jp->kind != PAR_SPLIT_UNFOLD;
  const bool zm = (jp->flags & GEMM_ZERO_MEAN) != 0;
  const size_t pan = (size_t)K16 * PB;
  float* Beh = reinterpret_cast<float*>(smem);
  float* Bel = Beh + pan;
  float* Boh = Bel + pan;
  float* Bol = Boh + pan;
  const gptr<const TB> B = gmem(static_cast<const TB*>(jp->B));
  constexpr int U = 4;
  const int tot = K16 * BN;
  for (int e0 = 0; e0 < tot; e0 += U * 256) {
    double x[U], y[U];
    int kk[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256 + tid;
      kk[u] = e / BN;
      c[u] = e - kk[u] * BN;
      const int gc = col0 + c[u];
      x[u] = y[u] = 0.0;
      if (e < tot && kk[u] < K && gc < N && !(zm && gc < 2)) {
        x[u] = (double)B[(size_t)kk[u] * ldb + gc];
        const int kr = fold ? KF - 1 - kk[u] : K + kk[u];
        if (fold ? kr > kk[u] : kr < KF) y[u] = (double)B[(size_t)kr * ldb + gc];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u * 256 + tid >= tot) continue;
      const int o = kk[u] * PB + c[u];
      const double ve = fold ? x[u] + y[u] : x[u], vo = fold ? x[u] - y[u] : y[u];
      const float he = (float)ve, ho = (float)vo;
      Beh[o] = he;
      Bel[o] = (float)(ve - (double)he);
      Boh[o] = ho;
      Bol[o] = (float)(vo - (double)ho);
    }
  }
  __syncthreads();
  const gptr<const float> Ah = gmem(static_cast<const float*>(jp->A));
  const gptr<const float> A2h = gmem(static_cast<const float*>(jp->A2));
  const gptr<const float> Al = gmem(static_cast<const float*>(jp->Alo));
  const gptr<const float> A2l = gmem(static_cast<const float*>(jp->A2lo));
  const int nrb = (M + 15) >> 4, nkb = K16 >> 4;
  const size_t bo = (size_t)(4 * lk) * PB + l16;
  for (int rb = wave; rb < nrb; rb += 4) {
    flt4 Se[CB], Ee[CB], Xe[CB], So[CB], Eo[CB], Xo[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) Se[cb] = Ee[cb] = Xe[cb] = So[cb] = Eo[cb] = Xo[cb] = flt4{0, 0, 0, 0};
    const size_t ar = (size_t)(rb * 16 + l16) * lda + 4 * lk;
    const gptr<const flt4> aeh = reinterpret_cast<gptr<const flt4>>(Ah + ar);
    const gptr<const flt4> ael = reinterpret_cast<gptr<const flt4>>(Al + ar);
    const gptr<const flt4> aoh = reinterpret_cast<gptr<const flt4>>(A2h + ar);
    const gptr<const flt4> aol = reinterpret_cast<gptr<const flt4>>(A2l + ar);
    flt4 neh = aeh[0], nel = ael[0], noh = aoh[0], nol = aol[0];
    for (int b = 0; b < nkb; ++b) {
      const flt4 xeh = neh, xel = nel, xoh = noh, xol = nol;
      if (b + 1 < nkb) {
        neh = aeh[4 * (b + 1)];
        nel = ael[4 * (b + 1)];
        noh = aoh[4 * (b + 1)];
        nol = aol[4 * (b + 1)];
      }
      const size_t rowo = bo + (size_t)(16 * b) * PB;
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const size_t o = rowo + (size_t)s2 * PB + cb * 16;
          const float beh = Beh[o], bel = Bel[o], boh = Boh[o], bol = Bol[o];
          const flt4 pe = mfma(xeh[s2], beh, flt4{0, 0, 0, 0});
          const flt4 po = mfma(xoh[s2], boh, flt4{0, 0, 0, 0});
          Xe[cb] = mfma(xeh[s2], bel, Xe[cb]);
          Xe[cb] = mfma(xel[s2], beh, Xe[cb]);
          Xo[cb] = mfma(xoh[s2], bol, Xo[cb]);
          Xo[cb] = mfma(xol[s2], boh, Xo[cb]);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float se = Se[cb][r], ee = Ee[cb][r], so = So[cb][r], eo = Eo[cb][r];
            two_sum(se, ee, pe[r]);
            two_sum(so, eo, po[r]);
            Se[cb][r] = se;
            Ee[cb][r] = ee;
            So[cb][r] = so;
            Eo[cb][r] = eo;
          }
        }
    }
    dbl4 E[1][CB], O[1][CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        E[0][cb][r] = (double)Se[cb][r] + (double)Ee[cb][r] + (double)Xe[cb][r];
        O[0][cb][r] = (double)So[cb][r] + (double)Eo[cb][r] + (double)Xo[cb][r];
      }
    // FP64 values in the layout of the FP32 instruction's output
    store_par<float, TC, 1, CB>(jp, E, O, rb * 16, col0, lk, l16);
  }
}

template <typename TB, typename TC, int BN>
__global__ __launch_bounds__(256) void gemm_bst_comp_kernel(const GemmJob* __restrict__ jobs,
                                                            const int* __restrict__ tmap, int total) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int t = xcd_tile(blockIdx.x, total);
  const GemmJob* jp = tile_job(jobs, tmap, t);
  if (masked(jp->skip)) return;
  if (jp->type == GEMM_DDD)
    bst_body<double, double, double, BN>(jp, t, smem);
  else
    bst_comp_body<TB, TC, BN>(jp, t, smem);
}

// NW waves per workgroup (configurations 14, 15: four; 16, 17: eight)
template <typename T, typename TB, typename TC, int BN, int NW>
__global__ __launch_bounds__(64 * NW) void gemm_bst_kernel(const GemmJob* __restrict__ jobs,
                                                           const int* __restrict__ tmap, int total) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int t = xcd_tile(blockIdx.x, total);
  const GemmJob* jp = tile_job(jobs, tmap, t);
  if (masked(jp->skip)) return;
  if (dual_type<T, TB, TC>() && jp->type == GEMM_DDD)
    bst_body<double, double, double, BN, NW>(jp, t, smem);
  else
    bst_body<T, TB, TC, BN, NW>(jp, t, smem);
}

// PAR: the table holds parity products only (else plain ones only): one
// body per kernel, so neither pays for the other's registers.
template <typename T, typename TB, typename TC, int CFG, bool PAR>
__global__ __launch_bounds__(256) void gemm_lds_kernel(const GemmJob* __restrict__ jobs, const int* __restrict__ tmap,
                                                       int total) {
  // gemm_lds_bytes of the table: the panels of its largest form and precision
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int t = xcd_tile(blockIdx.x, total);
  const GemmJob* jp = tile_job(jobs, tmap, t);
  if (masked(jp->skip)) return;
  const bool ddd = dual_type<T, TB, TC>() && jp->type == GEMM_DDD;
  if constexpr (PAR) {
    if (ddd)
      lds_par_body<double, double, double, CFG, ddd_half<CFG>() ? 2 : 1>(jp, t, smem);
    else
      lds_par_body<T, TB, TC, CFG>(jp, t, smem);
  } else {
    if (ddd)
      lds_body<double, double, double, CFG>(jp, t, smem);
    else
      lds_body<T, TB, TC, CFG>(jp, t, smem);
  }
}

namespace {

template <typename T, typename TB, typename TC>
void launch_cfg(const GemmJob* dev_jobs, const int* tmap, int total, int cfg, bool parity, size_t lds,
                hipStream_t s) {
#define PCS_GEMM_REG(C)                                                                                   \
  case C:                                                                                                 \
    hipLaunchKernelGGL((gemm_reg_kernel<T, TB, TC, C>), dim3(total), dim3(256), 0, s, dev_jobs, tmap, total); \
    break;
#define PCS_GEMM_LDS(C)                                                                                       \
  case C:                                                                                                     \
    if (parity)                                                                                               \
      hipLaunchKernelGGL((gemm_lds_kernel<T, TB, TC, C, true>), dim3(total), dim3(256), lds, s, dev_jobs, tmap, \
                         total);                                                                              \
    else                                                                                                      \
      hipLaunchKernelGGL((gemm_lds_kernel<T, TB, TC, C, false>), dim3(total), dim3(256), lds, s, dev_jobs,     \
                         tmap, total);                                                                        \
    break;
  switch (cfg) {
    PCS_GEMM_REG(0)
    PCS_GEMM_REG(1)
    PCS_GEMM_REG(2)
    PCS_GEMM_REG(3)
    PCS_GEMM_LDS(4)
    PCS_GEMM_LDS(5)
    PCS_GEMM_LDS(6)
    PCS_GEMM_LDS(7)
    PCS_GEMM_LDS(8)
    PCS_GEMM_LDS(9)
    PCS_GEMM_LDS(10)
    PCS_GEMM_LDS(11)
    PCS_GEMM_LDS(12)
    PCS_GEMM_LDS(13)
    case 14:
      if (parity)
        hipLaunchKernelGGL((gemm_bst_kernel<T, TB, TC, 32, 4>), dim3(total), dim3(256), lds, s, dev_jobs, tmap, total);
      break;
    case 15:
      if (parity)
        hipLaunchKernelGGL((gemm_bst_kernel<T, TB, TC, 64, 4>), dim3(total), dim3(256), lds, s, dev_jobs, tmap, total);
      break;
    case 16:
      if (parity)
        hipLaunchKernelGGL((gemm_bst_kernel<T, TB, TC, 16, 8>), dim3(total), dim3(512), lds, s, dev_jobs, tmap, total);
      break;
    case 17:
      if (parity)
        hipLaunchKernelGGL((gemm_bst_kernel<T, TB, TC, 32, 8>), dim3(total), dim3(512), lds, s, dev_jobs, tmap, total);
      break;
    default: break;
  }
#undef PCS_GEMM_REG
#undef PCS_GEMM_LDS
}

}  // namespace

bool gemm_cfg_parity(int cfg) { return cfg >= 4 && cfg < GEMM_NCFG; }
bool gemm_cfg_bst(int cfg) { return cfg >= 14 && cfg < GEMM_NCFG; }
bool gemm_type_comp(GemmType t) { return t == GEMM_CDF || t == GEMM_CFD; }

namespace {
template <int CFG>
size_t lds_form(bool parity, size_t esize, bool half) {
  // + 8: the B panel starts on a double boundary
  const int e = parity ? (half && ddd_half<CFG>() ? lds_par<CFG, 2>() : lds_par<CFG>()) : lds_plain<CFG>();
  return esize * (size_t)e + 8;
}
}  // namespace

size_t gemm_lds_bytes(GemmType t, const GemmJob* jobs, int njobs, int cfg) {
  // compute precision of the table's own type (its GEMM_DDD jobs compute in FP64)
  const size_t own = (t == GEMM_FDF || t == GEMM_FFD || gemm_type_comp(t)) ? 4 : 8;
  size_t b = 0;
  for (int j = 0; j < njobs; ++j) {
    if (gemm_type_comp(t) && jobs[j].type != GEMM_DDD) {
      // head and tail panels of both halves, B-stationary only; the compensated kernel has one wave count per
      // panel width, so configuration 17 would repeat 14
      if (!gemm_cfg_bst(cfg) || cfg == 17 || jobs[j].kind == PAR_NONE) return ~(size_t)0 >> 1;
      const size_t pitch = CFG_BN[cfg] + 4;  // bst_pitch
      const size_t x = 4 * (size_t)((jobs[j].k + 15) & ~15) * pitch * 4 + 16;
      b = x > b ? x : b;
      continue;
    }
    const bool par = jobs[j].kind != PAR_NONE;
    const size_t es = jobs[j].type == GEMM_DDD ? 8 : own;
    const bool half = t != GEMM_DDD && jobs[j].type == GEMM_DDD;  // FP64 products of a mixed table
    size_t x = 0;
    switch (cfg) {
      case 4: x = lds_form<4>(par, es, half); break;
      case 5: x = lds_form<5>(par, es, half); break;
      case 6: x = lds_form<6>(par, es, half); break;
      case 7: x = lds_form<7>(par, es, half); break;
      case 8: x = lds_form<8>(par, es, half); break;
      case 9: x = lds_form<9>(par, es, half); break;
      case 10: x = lds_form<10>(par, es, half); break;
      case 11: x = lds_form<11>(par, es, half); break;
      case 12: x = lds_form<12>(par, es, half); break;
      case 13: x = lds_form<13>(par, es, half); break;
      case 14:
      case 15:
      case 16:
      case 17: {
        // the whole K range of the folded panel: two halves of K16 rows
        const size_t pitch = CFG_BN[cfg] + (es == 8 ? 2 : 4);  // bst_pitch
        x = par ? 2 * (size_t)((jobs[j].k + 15) & ~15) * pitch * es + 16 : ~(size_t)0 >> 1;
        break;
      }
      default: break;
    }
    b = x > b ? x : b;
  }
  return b;
}

hipError_t gemm_set_attributes() {
  // the B-stationary kernels stage a whole K range: up to the CU's 160 KB
  const void* k[] = {
      (const void*)gemm_bst_kernel<double, double, double, 32, 4>, (const void*)gemm_bst_kernel<double, double, double, 64, 4>,
      (const void*)gemm_bst_kernel<float, double, float, 32, 4>,   (const void*)gemm_bst_kernel<float, double, float, 64, 4>,
      (const void*)gemm_bst_kernel<float, float, double, 32, 4>,   (const void*)gemm_bst_kernel<float, float, double, 64, 4>,
      (const void*)gemm_bst_kernel<double, double, float, 32, 4>,  (const void*)gemm_bst_kernel<double, double, float, 64, 4>,
      (const void*)gemm_bst_kernel<double, float, double, 32, 4>,  (const void*)gemm_bst_kernel<double, float, double, 64, 4>,
      (const void*)gemm_bst_comp_kernel<double, float, 32>,     (const void*)gemm_bst_comp_kernel<double, float, 64>,
      (const void*)gemm_bst_comp_kernel<float, double, 32>,     (const void*)gemm_bst_comp_kernel<float, double, 64>,
      (const void*)gemm_bst_kernel<double, double, double, 16, 8>, (const void*)gemm_bst_kernel<float, double, float, 16, 8>,
      (const void*)gemm_bst_kernel<float, float, double, 16, 8>,   (const void*)gemm_bst_kernel<double, double, float, 16, 8>,
      (const void*)gemm_bst_kernel<double, float, double, 16, 8>,  (const void*)gemm_bst_comp_kernel<double, float, 16>,
      (const void*)gemm_bst_comp_kernel<float, double, 16>,
      (const void*)gemm_bst_kernel<double, double, double, 32, 8>, (const void*)gemm_bst_kernel<float, double, float, 32, 8>,
      (const void*)gemm_bst_kernel<float, float, double, 32, 8>,   (const void*)gemm_bst_kernel<double, double, float, 32, 8>,
      (const void*)gemm_bst_kernel<double, float, double, 32, 8>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_LDS_MAX);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void gemm_run(GemmType t, const GemmJob* dev_jobs, const int* tmap, int total_tiles, int cfg, bool parity,
              size_t lds, hipStream_t s) {
  if (total_tiles <= 0 || cfg < 0 || cfg >= GEMM_NCFG || (parity && !gemm_cfg_parity(cfg))) return;
  if (gemm_type_comp(t)) {
    // compensated tables: parity products, B-stationary configurations only
    if (!parity || !gemm_cfg_bst(cfg)) return;
    const int bn = CFG_BN[cfg];
    if (t == GEMM_CDF) {
      if (bn == 64)
        hipLaunchKernelGGL((gemm_bst_comp_kernel<double, float, 64>), dim3(total_tiles), dim3(256), lds, s, dev_jobs,
                           tmap, total_tiles);
      else if (bn == 32)
        hipLaunchKernelGGL((gemm_bst_comp_kernel<double, float, 32>), dim3(total_tiles), dim3(256), lds, s, dev_jobs,
                           tmap, total_tiles);
      else
        hipLaunchKernelGGL((gemm_bst_comp_kernel<double, float, 16>), dim3(total_tiles), dim3(256), lds, s, dev_jobs,
                           tmap, total_tiles);
    } else {
      if (bn == 64)
        hipLaunchKernelGGL((gemm_bst_comp_kernel<float, double, 64>), dim3(total_tiles), dim3(256), lds, s, dev_jobs,
                           tmap, total_tiles);
      else if (bn == 32)
        hipLaunchKernelGGL((gemm_bst_comp_kernel<float, double, 32>), dim3(total_tiles), dim3(256), lds, s, dev_jobs,
                           tmap, total_tiles);
      else
        hipLaunchKernelGGL((gemm_bst_comp_kernel<float, double, 16>), dim3(total_tiles), dim3(256), lds, s, dev_jobs,
                           tmap, total_tiles);
    }
    return;
  }
  switch (t) {
    case GEMM_DDD: launch_cfg<double, double, double>(dev_jobs, tmap, total_tiles, cfg, parity, lds, s); break;
    case GEMM_FDF: launch_cfg<float, double, float>(dev_jobs, tmap, total_tiles, cfg, parity, lds, s); break;
    case GEMM_FFD: launch_cfg<float, float, double>(dev_jobs, tmap, total_tiles, cfg, parity, lds, s); break;
    case GEMM_DDF: launch_cfg<double, double, float>(dev_jobs, tmap, total_tiles, cfg, parity, lds, s); break;
    case GEMM_DFD: launch_cfg<double, float, double>(dev_jobs, tmap, total_tiles, cfg, parity, lds, s); break;
    default: break;
  }
}

}  // namespace pcs
