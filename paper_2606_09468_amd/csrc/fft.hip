// Periodic-direction transforms, the fused physical-space products and the
// per-step diagnostics (FP64 path).
//
// Fourier in x and z with full 3/2-rule dealiasing (paper, Section 2): every
// retained mode is placed at its own frequency in a transform of 3/2 the base
// size, products are formed pointwise, and the forward transform is
// truncated back to the retained modes.  Transforms are mixed-radix (8, 4, 2,
// 3) Stockham FFTs done in place in LDS: each pass reads its butterfly inputs
// into registers, synchronises, and writes the outputs to their sorted
// positions, so one buffer suffices.  The lengths of the workloads run plans
// fixed at compile time (constant strides and twiddle indices); where the
// sequences of a pass belong to one wave (x pencils, row diagnostics) the
// synchronisation is that of the wave alone.  Two real fields share one
// complex transform (z = a + i b).  The x lines of those lengths (L = 3 nkx)
// put the radix-3 pass first in the inverse and last in the forward
// transform, so that the spectra enter and leave through registers and the
// zero band of the 3/2 rule is never stored; their power-of-two passes take
// radices up to 16.
//
// x pencil: one workgroup per padded (y', z') line.  It reads the needed
// spectral fields of that line (kx modes), generates the d/dx variants by
// multiplying with i kx, runs the inverse transforms, evaluates
//   N_a  = - u_k d_k u_a                                       (eq. 2)
//   F_ab = - u_k d_k c_ab + (d_k u_a) c_kb + c_ak (d_k u_b)
//          - (eps/Wi) Tr(c - I)(c_ab - delta_ab)                (eq. 1)
// at every point, and writes the forward transforms of the outputs,
// truncated to the retained modes.  d_y v comes from continuity (eq. 3).
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "kernels.hpp"

namespace pcs {

bool make_plan(int L, FftPlan* p) {
  *p = FftPlan{};
  p->L = L;
  int r = L;
  auto take = [&](int R) {
    while (r % R == 0 && p->npass < 12) {
      p->radix[p->npass++] = R;
      r /= R;
    }
  };
  take(8);
  take(4);
  take(2);
  take(3);
  if (r != 1 || L < 2) return false;
  int ns = 1;
  for (int i = 0; i < p->npass; ++i) {
    const int R = p->radix[i];
    p->lr[i] = L / R;
    p->ns[i] = ns;
    p->ts[i] = L / (ns * R);
    p->mlr[i] = fast_div_magic((unsigned)p->lr[i]);
    p->mns[i] = fast_div_magic((unsigned)ns);
    ns *= R;
  }
  return true;
}

namespace {

constexpr int NT = 256;  // threads per workgroup of the transform kernels

// complex values a thread holds in one pass, and the largest multiple of
// every radix that fits (the elements per thread any pass can cover)
template <typename T>
__host__ __device__ constexpr int maxv() {
  return sizeof(T) == 4 ? 24 : 16;
}
__host__ __device__ constexpr int cover(int mv) {
  const int c8 = (mv / 8) * 8, c4 = (mv / 4) * 4, c2 = (mv / 2) * 2, c3 = (mv / 3) * 3;
  const int a = c8 < c4 ? c8 : c4, b = c2 < c3 ? c2 : c3;
  return a < b ? a : b;
}

// floor(n / d) from a multiply-high reciprocal (m = 0 encodes d = 1)
__device__ inline int fdiv(int n, unsigned m) { return m ? (int)__umulhi((unsigned)n, m) : n; }

template <typename T>
struct cx {
  T x, y;
};
template <typename T>
struct V2 {
  typedef T type __attribute__((ext_vector_type(2)));
};

// LDS view of the transform buffers.  FP64: logical element p lives at
// p + p / 16 (one spare slot every 16 complex values), so the strided writes
// of a Stockham pass (lanes R or R Ns elements apart) and the column-wise
// accesses of the z transforms spread over all banks.  FP32 keeps the plain
// layout: there the extra address arithmetic costs more registers (and
// occupancy) than the conflicts it removes (measured on the 3D x pencils).
template <bool PAD>
__host__ __device__ constexpr size_t lds_span(size_t n) {
  return PAD ? n + (n >> 4) + 1 : n;
}
template <typename T>
__host__ __device__ constexpr size_t lds_padded(size_t n) {
  return lds_span<sizeof(T) == 8>(n);
}
// dynamic LDS of the transform kernels (indexed through the symbol, so
// every access stays an LDS instruction)
// An access at a constant offset that is a multiple of 16 adds a constant
// to the padded base, so the strided accesses of a pass share one address
// computation (immediate offsets).
extern __shared__ double fft_lds[];
template <typename T, bool PAD = (sizeof(T) == 8)>
struct LV {
  int off;
  __device__ cx<T>& operator[](int i) const {
    cx<T>* b = reinterpret_cast<cx<T>*>(fft_lds);
    if constexpr (PAD) {
      if (__builtin_constant_p(i) && i >= 0 && (i & 15) == 0) return b[off + (off >> 4) + i + (i >> 4)];
      const int q = off + i;
      return b[q + (q >> 4)];
    } else {
      return b[off + i];
    }
  }
  __device__ LV at(int d) const { return LV{off + d}; }
};
template <typename T>
__device__ inline cx<T> operator+(cx<T> a, cx<T> b) {
  return cx<T>{a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ inline cx<T> operator-(cx<T> a, cx<T> b) {
  return cx<T>{a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ inline cx<T> scal(T s, cx<T> a) {
  return cx<T>{s * a.x, s * a.y};
}

// R-point DFT in registers; sign -1 forward, +1 inverse.
template <typename T, int R>
__device__ inline void butterfly(cx<T>* v, int sign) {
  if constexpr (R == 2) {
    cx<T> t = v[0];
    v[0] = t + v[1];
    v[1] = t - v[1];
  } else if constexpr (R == 4) {
    cx<T> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = v[1] - v[3];
    cx<T> sid = sign > 0 ? cx<T>{-d.y, d.x} : cx<T>{d.y, -d.x};  // (sign i) d
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + sid;
    v[3] = b - sid;
  } else if constexpr (R == 8) {
    // split into even and odd halves: a_q = v_q + v_(q+4) and
    // b_q = w^q (v_q - v_(q+4)), w = exp(sign 2 pi i / 8); X_2m = DFT4(a)_m,
    // X_2m+1 = DFT4(b)_m
    const T h = T(0.70710678118654752440);
    cx<T> a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = v[q] + v[q + 4];
      b[q] = v[q] - v[q + 4];
    }
    // w^1 = h (1 + sign i), w^2 = sign i, w^3 = h (-1 + sign i)
    b[1] = sign > 0 ? cx<T>{h * (b[1].x - b[1].y), h * (b[1].x + b[1].y)}
                    : cx<T>{h * (b[1].x + b[1].y), h * (b[1].y - b[1].x)};
    b[2] = sign > 0 ? cx<T>{-b[2].y, b[2].x} : cx<T>{b[2].y, -b[2].x};
    b[3] = sign > 0 ? cx<T>{-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y)}
                    : cx<T>{h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y)};
    butterfly<T, 4>(a, sign);
    butterfly<T, 4>(b, sign);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v[2 * m] = a[m];
      v[2 * m + 1] = b[m];
    }
  } else if constexpr (R == 16) {
    // 4 x 4: inputs n = 4 n1 + n2, outputs k = k1 + 4 k2; DFT4 over n1,
    // twiddle w16^(n2 k1) (w16 = exp(sign 2 pi i / 16)), DFT4 over n2
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173), h = T(0.70710678118654752440);
    const T sg = T(sign);
    // w16^m for m = 0 .. 9 (cos, sign * sin)
    const cx<T> w[10] = {{1, 0},   {c1, sg * s1},      {h, sg * h},         {s1, sg * c1},  {0, sg},
                         {-s1, sg * c1}, {-h, sg * h}, {-c1, sg * s1},      {-1, 0},        {-c1, -sg * s1}};
    cx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      butterfly<T, 4>(t, sign);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = (n2 && k1) ? cmul(t[k1], w[n2 * k1]) : t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      butterfly<T, 4>(t, sign);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  } else {
    const T h = T(0.86602540378443864676) * T(sign);  // sign * sqrt(3)/2
    cx<T> t1 = v[1] + v[2];
    cx<T> t2 = v[0] - scal(T(0.5), t1);
    cx<T> t3 = scal(h, v[1] - v[2]);
    cx<T> it3 = cx<T>{-t3.y, t3.x};
    v[0] = v[0] + t1;
    v[1] = t2 + it3;
    v[2] = t2 - it3;
  }
}

// Synchronisation around the writes of a pass: the workgroup's barrier, or,
// when the sequences of the pass belong to one wave (WAVE), only a fence that
// keeps the compiler from moving LDS accesses across it (a wave's LDS
// instructions execute in order, so its reads of a pass complete before its
// writes, and its writes before the next pass's reads).
template <bool WAVE>
__device__ __attribute__((always_inline)) inline void pass_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One in-place Stockham pass (pass p of the plan, radix R) over nseq
// sequences of length L: every thread reads its butterfly inputs into
// registers, the threads synchronise, and the outputs go to their sorted
// positions.  twl[m] = exp(-2 pi i m / L).  NTH threads (thread tid: the
// workgroup's, or one wave's lanes for WAVE), at most MV complex values per
// thread: requires nseq L <= NTH cover(MV).
template <typename T, int R, int NTH, int MV, bool WAVE, typename V>
__device__ __attribute__((always_inline)) inline void pass_ip(V buf, int sl, const FftPlan& pl, int p, int nseq,
                                                              const cx<T>* __restrict__ tw, int sign, int tid) {
  constexpr int NB = MV / R;
  const int L = pl.L, LR = pl.lr[p], Ns = pl.ns[p], stride = pl.ts[p];
  const unsigned mLR = pl.mlr[p], mNs = pl.mns[p];
  const int tot = nseq * LR;
  cx<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int idx = tid + q * NTH;
    if (idx < tot) {
      const int s = fdiv(idx, mLR), j = idx - s * LR;
      const V src = buf.at(s * sl + j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * LR];
    }
  }
  pass_sync<WAVE>();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int idx = tid + q * NTH;
    if (idx < tot) {
      const int s = fdiv(idx, mLR), j = idx - s * LR;
      const int k = j - fdiv(j, mNs) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * stride];
          if (sign > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      butterfly<T, R>(v[q], sign);
      const V dst = buf.at(s * sl + (j - k) * R + k);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[q][r];
    }
  }
  pass_sync<WAVE>();
}

// nseq sequences of length pl.L, sequence s at buf + s * sl (sl >= L),
// transformed by the workgroup, or for WAVE by the calling wave alone
// (tid: its lane).  Inlined at every call: as a called function its register
// needs add to the caller's (measured: 211-228 VGPRs in the x-pencil and
// diagnostics kernels).
template <typename T, int NTH = NT, int MV = maxv<T>(), bool WAVE = false, typename V = LV<T>>
__device__ __attribute__((always_inline)) inline void lds_fft(V buf, int sl, const FftPlan& pl, int nseq,
                                                              const cx<T>* __restrict__ tw, int sign,
                                                              int tid = threadIdx.x) {
  for (int p = 0; p < pl.npass; ++p) {
    const int R = pl.radix[p];
    if (R == 8)
      pass_ip<T, 8, NTH, MV, WAVE>(buf, sl, pl, p, nseq, tw, sign, tid);
    else if (R == 4)
      pass_ip<T, 4, NTH, MV, WAVE>(buf, sl, pl, p, nseq, tw, sign, tid);
    else if (R == 2)
      pass_ip<T, 2, NTH, MV, WAVE>(buf, sl, pl, p, nseq, tw, sign, tid);
    else
      pass_ip<T, 3, NTH, MV, WAVE>(buf, sl, pl, p, nseq, tw, sign, tid);
  }
}

// ------------------------------------------------ transforms of a length fixed at compile time
// The plan of make_plan (radix 8 passes, then 4, 2, 3) for a length L known at
// compile time, so that a pass's divisions, strides and twiddle indices fold
// into constants (the runtime plan spends more instructions on index
// arithmetic and plan loads than on the butterflies).
__host__ __device__ constexpr int crad_try(int i) { return i == 0 ? 8 : (i == 1 ? 4 : (i == 2 ? 2 : 3)); }
__host__ __device__ constexpr int cpass_count(int L) {
  int n = 0;
  for (int i = 0; i < 4; ++i)
    while (L > 1 && L % crad_try(i) == 0) {
      L /= crad_try(i);
      ++n;
    }
  return n;
}
__host__ __device__ constexpr int cradix(int L, int p) {
  for (int i = 0; i < 4; ++i)
    while (L > 1 && L % crad_try(i) == 0) {
      if (p == 0) return crad_try(i);
      L /= crad_try(i);
      --p;
    }
  return 1;
}
__host__ __device__ constexpr int cns(int L, int p) {
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= cradix(L, i);
  return ns;
}

// One Stockham pass of radix R over sequences of a length L fixed at compile
// time, NS the product of the radices before it (SIGN: +1 inverse, -1
// forward); as pass_ip otherwise.
template <typename T, int L, int R, int NS, int NTH, int MV, bool WAVE, int SIGN, typename V>
__device__ __attribute__((always_inline)) inline void pass_rn(V buf, int sl, int nseq, const cx<T>* __restrict__ tw,
                                                              int tid) {
  constexpr int LR = L / R, stride = L / (NS * R);
  constexpr int NB = MV / R;
  static_assert(R > 1 && NB >= 1 && L % (NS * R) == 0, "plan");
  const int tot = nseq * LR;
  cx<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int idx = tid + q * NTH;
    if (idx < tot) {
      const int s = idx / LR, j = idx - s * LR;
      const V src = buf.at(s * sl + j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * LR];
    }
  }
  pass_sync<WAVE>();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int idx = tid + q * NTH;
    if (idx < tot) {
      const int s = idx / LR, j = idx - s * LR;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * stride];
          if constexpr (SIGN > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      butterfly<T, R>(v[q], SIGN);
      const V dst = buf.at(s * sl + (j - k) * R + k);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * NS] = v[q][r];
    }
  }
  pass_sync<WAVE>();
}

// pass_ip with the plan of length L fixed
template <typename T, int L, int P, int NTH, int MV, bool WAVE, int SIGN, typename V>
__device__ __attribute__((always_inline)) inline void pass_c(V buf, int sl, int nseq, const cx<T>* __restrict__ tw,
                                                             int tid) {
  static_assert(cpass_count(L) > 0, "plan");
  pass_rn<T, L, cradix(L, P), cns(L, P), NTH, MV, WAVE, SIGN>(buf, sl, nseq, tw, tid);
}

template <typename T, int L, int NTH, int MV, bool WAVE, int SIGN, int P = 0, typename V = LV<T>>
__device__ __attribute__((always_inline)) inline void lds_fft_c(V buf, int sl, int nseq,
                                                                const cx<T>* __restrict__ tw, int tid) {
  if constexpr (P < cpass_count(L)) {
    pass_c<T, L, P, NTH, MV, WAVE, SIGN>(buf, sl, nseq, tw, tid);
    lds_fft_c<T, L, NTH, MV, WAVE, SIGN, P + 1, V>(buf, sl, nseq, tw, tid);
  }
}

// Transform with the compiled plan of length LC, or with the runtime plan
// (LC = 0).
template <typename T, int LC, int NTH, int MV, bool WAVE, int SIGN, typename V>
__device__ __attribute__((always_inline)) inline void fft_any(V buf, int sl, const FftPlan& pl, int nseq,
                                                              const cx<T>* __restrict__ tw, int tid) {
  if constexpr (LC > 0)
    lds_fft_c<T, LC, NTH, MV, WAVE, SIGN, 0, V>(buf, sl, nseq, tw, tid);
  else
    lds_fft<T, NTH, MV, WAVE, V>(buf, sl, pl, nseq, tw, SIGN, tid);
}

// Complex values per lane of the x pencils' wave-local transforms: 16, or 8
// for FP64 lines of a compiled length up to 384 (whose registers would
// otherwise cost a workgroup per CU).
constexpr int XMVW = 16;
template <typename T, int LC>
__host__ __device__ constexpr int xmvw() {
  return (sizeof(T) == 8 && LC > 0 && LC <= 384) ? 8 : XMVW;
}

// ------------------------------------------------ x lines of a compiled length L = 3 nkx
// The 3/2-rule line of an x pencil carries nonzero spectrum at k < nkx and
// k > 2 nkx only (nkx = L / 3 retained modes).  Its inverse transform takes
// the radix-3 pass first, over the stride nkx: butterfly j then reads X_j and
// X_(j + 2 nkx) and nothing of the zero band, and is formed straight from the
// spectra in registers (no packing into LDS, no clearing of the band).  The
// forward transform takes the radix-3 pass last and computes only the
// outputs k < nkx and k > 2 nkx, which the unpacking of the two real fields
// reads, straight from registers.  In both, one lane takes butterflies j and
// nkx - j (j = 0 with nkx / 2), which read and write the same modes.  The
// power-of-two part L / 3 goes in as few passes as radices of at most RM allow,
// bits spread evenly (128: 16 x 8; 64: 8 x 8; 256: 16 x 16).
__host__ __device__ constexpr int clog2(int n) {
  int a = 0;
  while ((1 << a) < n) ++a;
  return a;
}
__host__ __device__ constexpr int xp_count(int L, int RM) { return (clog2(L / 3) + clog2(RM) - 1) / clog2(RM); }
// radix of power-of-two pass i, in the inverse transform's order
__host__ __device__ constexpr int xp_radix(int L, int RM, int i) {
  return 1 << (clog2(L / 3) / xp_count(L, RM) + (i < clog2(L / 3) % xp_count(L, RM) ? 1 : 0));
}
// sequences of length L a wave's passes hold at MV complex values per lane
template <int L, int MV>
__host__ __device__ constexpr int xp_batch() {
  return 64 * MV / L;
}
// the passes after the radix-3 one (inverse) and before it (forward), by NTH
// threads (one wave's lanes for WAVE)
template <typename T, int L, int RM, int MV, int NTH = 64, bool WAVE = true, int I = 0, int NS = 3, typename V>
__device__ __attribute__((always_inline)) inline void xfft_inv_tail(V buf, int sl, int nseq,
                                                                    const cx<T>* __restrict__ tw, int tid) {
  if constexpr (I < xp_count(L, RM)) {
    constexpr int R = xp_radix(L, RM, I);
    pass_rn<T, L, R, NS, NTH, MV, WAVE, +1>(buf, sl, nseq, tw, tid);
    xfft_inv_tail<T, L, RM, MV, NTH, WAVE, I + 1, NS * R, V>(buf, sl, nseq, tw, tid);
  }
}
template <typename T, int L, int RM, int MV, int NTH = 64, bool WAVE = true, int I = 0, int NS = 1, typename V>
__device__ __attribute__((always_inline)) inline void xfft_fwd_head(V buf, int sl, int nseq,
                                                                    const cx<T>* __restrict__ tw, int tid) {
  if constexpr (I < xp_count(L, RM)) {
    constexpr int R = xp_radix(L, RM, xp_count(L, RM) - 1 - I);
    pass_rn<T, L, R, NS, NTH, MV, WAVE, -1>(buf, sl, nseq, tw, tid);
    xfft_fwd_head<T, L, RM, MV, NTH, WAVE, I + 1, NS * R, V>(buf, sl, nseq, tw, tid);
  }
}
// Radix-3 inverse butterfly with a zero middle input: outputs of (x, 0, c).
template <typename T, typename V>
__device__ __attribute__((always_inline)) inline void xp_first3(V dst, cx<T> x, cx<T> c) {
  const T h = T(0.86602540378443864676);
  const cx<T> t2{x.x - T(0.5) * c.x, x.y - T(0.5) * c.y};
  // i * (sqrt(3)/2) * (0 - c)
  const cx<T> it3{h * c.y, -h * c.x};
  dst[0] = x + c;
  dst[1] = t2 + it3;
  dst[2] = t2 - it3;
}
// First inverse pass of unit u of a line Xq (the butterflies j1 = u and
// j2 = nkx - u, or 0 and nkx / 2 for u = 0) from the modes (A1, B1) at j1 and
// (A2, B2) at j2 of the two real fields a, b of the pair: X_k = A_k + i B_k,
// X_(L-k) = conj(A_k) + i conj(B_k), X_0 = Re A_0 + i Re B_0.
template <typename T, typename V>
__device__ __attribute__((always_inline)) inline void xp_first(V Xq, int nkx, int u, cx<T> A1, cx<T> B1, cx<T> A2,
                                                               cx<T> B2) {
  const int j2 = u ? nkx - u : nkx >> 1;
  const cx<T> p1 = u ? cx<T>{A1.x - B1.y, A1.y + B1.x} : cx<T>{A1.x, B1.x};
  const cx<T> p2{A2.x - B2.y, A2.y + B2.x};
  const cx<T> q1{A1.x + B1.y, B1.x - A1.y}, q2{A2.x + B2.y, B2.x - A2.y};
  // X_(j + 2 nkx) = X_(L - (nkx - j)): of mode j2 for j1, of mode j1 for j2
  // (u = 0: zero for j1 = 0, mode nkx / 2 itself for j2)
  xp_first3<T>(Xq.at(3 * u), p1, u ? q2 : cx<T>{0, 0});
  xp_first3<T>(Xq.at(3 * j2), p2, u ? q1 : q2);
}
// Last forward pass (radix 3, stride nkx) at butterfly j of a line Zq:
// outputs Z_j (y0) and Z_(j + 2 nkx) (y2).
template <typename T, typename V>
__device__ __attribute__((always_inline)) inline void xp_last(V Zq, int nkx, int j, const cx<T>* __restrict__ tw,
                                                              cx<T>& y0, cx<T>& y2) {
  const T h = T(0.86602540378443864676);
  const cx<T> v0 = Zq[j], v1 = cmul(Zq[j + nkx], tw[j]), v2 = cmul(Zq[j + 2 * nkx], tw[2 * j]);
  const cx<T> t1 = v1 + v2, d = v1 - v2;
  y0 = v0 + t1;
  // v0 - t1 / 2 + i (sqrt(3)/2) (v1 - v2)
  y2 = cx<T>{v0.x - T(0.5) * t1.x - h * d.y, v0.y - T(0.5) * t1.y + h * d.x};
}
// Spectra of the two real fields at mode k from Z_k and Z_(L-k) (k > 0).
template <typename T>
__device__ __attribute__((always_inline)) inline void xp_unpack(cx<T> Zk, cx<T> Zc, cx<T>& A, cx<T>& B) {
  A = cx<T>{T(0.5) * (Zk.x + Zc.x), T(0.5) * (Zk.y - Zc.y)};
  B = cx<T>{T(0.5) * (Zk.y + Zc.y), T(-0.5) * (Zk.x - Zc.x)};
}

// Largest batch of sequences a pass can hold in registers.
template <typename T, int NTH = NT, int MV = maxv<T>()>
__host__ __device__ inline int fft_batch(int L) {
  return (NTH * cover(MV)) / L;
}

// Hermitian packing of two real-field spectra A_k, B_k into the complex
// sequence whose inverse transform is a + i b.
template <typename T, typename V>
__device__ inline void pack_pair(V X, int L, int k, cx<T> A, cx<T> B) {
  if (k == 0) {
    X[0] = cx<T>{A.x, B.x};
  } else {
    X[k] = cx<T>{A.x - B.y, A.y + B.x};
    X[L - k] = cx<T>{A.x + B.y, B.x - A.y};
  }
}

// Spectra of the two real fields packed in a forward transform Z, at k.
template <typename T, typename V>
__device__ inline void unpack_pair(V Z, int L, int k, cx<T>& A, cx<T>& B) {
  const cx<T> Zk = Z[k];
  if (k == 0) {
    A = cx<T>{Zk.x, 0};
    B = cx<T>{Zk.y, 0};
  } else {
    const cx<T> Zc = Z[L - k];
    A = cx<T>{T(0.5) * (Zk.x + Zc.x), T(0.5) * (Zk.y - Zc.y)};
    B = cx<T>{T(0.5) * (Zk.y + Zc.y), T(-0.5) * (Zk.x - Zc.x)};
  }
}

typedef cx<double> c2;

// index of c_ab in the stored list (2D: xx xy yy; 3D: xx xy xz yy yz zz)
__host__ __device__ constexpr int cidx(int dim, int a, int b) {
  return a > b ? cidx(dim, b, a) : (dim == 2 ? (a == 0 ? b : 2) : (a == 0 ? b : (a == 1 ? 2 + b : 5)));
}

// Real fields fed to the x transforms: source field in the [field][row][kx]
// input and whether d/dx is applied.
//  2D (input: I u, I v, I c3, D u, D c3):
//    u v ux uy vx | cxx cxy cyy | dx c (3) | dy c (3)
//  3D (input: I u v w, I c6, D u, D w, D c6, dz u v w, dz c6):
//    u v w | c (6) | dx u v w | dx c (6) | dy u, dy w | dy c (6) | dz u v w | dz c (6)
__device__ const short XSRC[2][36] = {
    {0, 1, 0, 5, 1, 2, 3, 4, 2, 3, 4, 6, 7, 8},
    {0, 1, 2, 3, 4, 5, 6, 7, 8, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23,
     24, 25}};
__device__ const short XDX[2][36] = {{0, 0, 1, 0, 1, 0, 0, 0, 1, 1, 1, 0, 0, 0},
                                     {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1}};

template <int DIM>
struct XShape {
  static constexpr int NREAL = DIM == 2 ? 14 : 35;
  static constexpr int NP = (NREAL + 1) / 2;
  static constexpr int NOUT = DIM == 2 ? 5 : 9;
  static constexpr int NOP = (NOUT + 1) / 2;
};

// Products of eqs. (1)-(2) at one point (field order as in the tables above);
// r(f) returns real field f at the point.  Outputs: N_x N_y (N_z) then F_ab
// (stored components).
template <int DIM, typename Rd>
__device__ inline void pointwise(const Rd& r, double* o, double eps_wi) {
  // velocity gradient du(k, a) = d_k u_a, with d_y v from continuity
  auto u = [&](int a) -> double { return r(a); };
  auto du = [&](int k, int a) -> double {
    if constexpr (DIM == 2) {
      if (k == 0) return a == 0 ? r(2) : r(4);
      return a == 0 ? r(3) : -r(2);
    } else {
      if (k == 0) return r(9 + a);
      if (k == 2) return r(26 + a);
      return a == 0 ? r(18) : (a == 2 ? r(19) : -(r(9) + r(28)));
    }
  };
  constexpr int C0 = DIM == 2 ? 5 : 3;                  // c components
  constexpr int DX = DIM == 2 ? 8 : 12, DY = DIM == 2 ? 11 : 20, DZ = 29;
  auto c = [&](int a, int b) -> double { return r(C0 + cidx(DIM, a, b)); };
  auto dc = [&](int k, int q) -> double { return r((k == 0 ? DX : (k == 1 ? DY : DZ)) + q); };
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    double s = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) s += u(k) * du(k, a);
    o[a] = -s;
  }
  double tr = 0;
  if (eps_wi != 0.0) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) tr += c(a, a) - 1.0;
  }
  int q = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = a; b < DIM; ++b) {
      double f = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) f += -u(k) * dc(k, q) + du(k, a) * c(k, b) + c(a, k) * du(k, b);
      if (eps_wi != 0.0) f -= eps_wi * tr * (c(a, b) - (a == b ? 1.0 : 0.0));
      o[DIM + q] = f;
      ++q;
    }
}

// Mixed precision split: every padded-grid field is mean(y') + fluctuation,
// the mean being the kx = kz = 0 profile.  Mean profile index of each real
// field (-1: the field has no mean part):
//  2D means: U U' cxx cxy cyy cxx' cxy' cyy'
//  3D means: U W U' W' c (6) c' (6)
__host__ __device__ constexpr int mean_of(int dim, int f) {
  return dim == 2 ? (f == 0 ? 0 : f == 3 ? 1 : (f >= 5 && f <= 7) ? f - 3 : (f >= 11 && f <= 13) ? f - 6 : -1)
                  : (f == 0 ? 0 : f == 2 ? 1 : f == 18 ? 2 : f == 19 ? 3 : (f >= 3 && f <= 8) ? f + 1
                                                                         : (f >= 20 && f <= 25) ? f - 10 : -1);
}
__host__ __device__ constexpr int n_means(int dim) { return dim == 2 ? 8 : 16; }

// Product of the mean profiles in explicit term o at padded row i, FP64.  For
// profiles only the y-derivatives of the mean velocity (U', W') survive
// (v = 0, d/dx = d/dz = 0), so N = 0 and F_ab = U'_a c_yb + c_ay U'_b with
// U'_x = U', U'_z = W', less the sPTT term (eps/Wi) Tr(c - I)(c_ab - delta_ab)
// of the mean profiles.
__device__ inline double mean_product(int dim, int o, gptr<const double> mean, int m1, int i, double eps_wi) {
  auto M = [&](int k) { return mean[(size_t)k * m1 + i]; };
  if (dim == 2) {
    // means: U U' cxx cxy cyy ...; outputs: Nx Ny Fxx Fxy Fyy (c_zz = 1)
    if (o < 2) return 0.0;
    const double tr = M(2) + M(4) - 2.0, cab = o == 3 ? M(3) : M(o) - 1.0;
    const double s = eps_wi != 0.0 ? eps_wi * tr * cab : 0.0;
    if (o == 2) return 2.0 * M(1) * M(3) - s;
    if (o == 3) return M(1) * M(4) - s;
    return -s;
  }
  // means: U W U' W' cxx cxy cxz cyy cyz czz ...; outputs: Nx Ny Nz Fxx Fxy Fxz Fyy Fyz Fzz
  if (o < 3) return 0.0;
  const double Up = M(2), Wp = M(3);
  const double tr = M(4) + M(7) + M(9) - 3.0;
  const double cab = M(o + 1) - ((o == 3 || o == 6 || o == 8) ? 1.0 : 0.0);
  const double s = eps_wi != 0.0 ? eps_wi * tr * cab : 0.0;
  if (o == 3) return 2.0 * Up * M(5) - s;
  if (o == 4) return Up * M(7) - s;
  if (o == 5) return Up * M(8) + M(5) * Wp - s;
  if (o == 7) return Wp * M(7) - s;
  if (o == 8) return 2.0 * Wp * M(8) - s;
  return -s;
}

template <typename T>
struct MF {
  T m, f;  // mean part and fluctuation
};
// fluctuation-containing part of the product of two split fields:
// a b - abar bbar = (abar + a') b' + a' bbar
template <typename T>
__device__ inline T fprod(MF<T> a, MF<T> b) {
  return (a.m + a.f) * b.f + a.f * b.m;
}

// Fluctuation-containing part of the products of eqs. (1)-(2); r(f), m(f):
// fluctuation and mean of real field f at the point.  The sPTT term is
// bilinear in c - I: with T = Tr(c - I) and C = c_ab - delta_ab split the same
// way, its fluctuation part is (eps/Wi) [(Tbar + T') C' + T' Cbar].
template <int DIM, typename T, typename Rd, typename Md>
__device__ inline void pointwise_mixed(const Rd& r, const Md& m, T* o, T eps_wi) {
  auto F = [&](int f) -> MF<T> { return MF<T>{m(f), r(f)}; };
  auto neg = [](MF<T> a) -> MF<T> { return MF<T>{-a.m, -a.f}; };
  auto du = [&](int k, int a) -> MF<T> {
    if constexpr (DIM == 2) {
      if (k == 0) return a == 0 ? F(2) : F(4);
      return a == 0 ? F(3) : neg(F(2));
    } else {
      if (k == 0) return F(9 + a);
      if (k == 2) return F(26 + a);
      if (a == 0) return F(18);
      if (a == 2) return F(19);
      return MF<T>{-(m(9) + m(28)), -(r(9) + r(28))};
    }
  };
  constexpr int C0 = DIM == 2 ? 5 : 3;
  constexpr int DX = DIM == 2 ? 8 : 12, DY = DIM == 2 ? 11 : 20, DZ = 29;
  auto c = [&](int a, int b) -> MF<T> { return F(C0 + cidx(DIM, a, b)); };
  auto dc = [&](int k, int q) -> MF<T> { return F((k == 0 ? DX : (k == 1 ? DY : DZ)) + q); };
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T s = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) s += fprod(F(k), du(k, a));
    o[a] = -s;
  }
  int q = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = a; b < DIM; ++b) {
      T f = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) f += -fprod(F(k), dc(k, q)) + fprod(du(k, a), c(k, b)) + fprod(c(a, k), du(k, b));
      if (eps_wi != T(0)) {
        T tm = T(DIM == 2 ? -2 : -3), tf = 0;  // Tr(c - I) (2D: c_zz = 1)
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
          tm += c(e, e).m;
          tf += c(e, e).f;
        }
        const MF<T> cab = c(a, b);
        f -= eps_wi * fprod(MF<T>{tm, tf}, MF<T>{cab.m - T(a == b ? 1 : 0), cab.f});
      }
      o[DIM + q] = f;
      ++q;
    }
}

// mean: [n_means][M+1] FP64 profiles (MIXED only); pz: padded z rows per y'.
// LC: the line length when it has a compiled plan, else 0.
template <typename T, int DIM, bool MIXED, int NTH, int LC>
__device__ __attribute__((always_inline)) inline void xpencil_body(const XArgs& XA) {
  constexpr int NW = NTH / 64;  // waves
  using XS = XShape<DIM>;
  const gptr<const T> in = gmem(static_cast<const T*>(XA.in));
  const gptr<T> out = gmem(static_cast<T*>(XA.out));
  const int nrows = XA.nrows, nkx = XA.nkx, m1 = XA.m1, pz = XA.pz;
  const FftPlan& pl = XA.pl;
  const gptr<const double> kx = gmem(XA.kx);
  const double eps_wi = XA.eps_wi;
  const gptr<const double> mean = gmem(XA.mean);
  const gptr<double> mcol = gmem(XA.mcol);
  cx<T>* P = reinterpret_cast<cx<T>*>(fft_lds);
  const int L = LC > 0 ? LC : pl.L;
  const int row = blockIdx.x - XA.blk0, tid = threadIdx.x;
  const size_t fstride = (size_t)nrows * nkx * 2;
  const gptr<const T> base = in + (size_t)row * nkx * 2;
  // each wave transforms its own pairs (wave, wave + NW, ...), SW at a time
  constexpr int MVW = xmvw<T, LC>();
  const int SW = fft_batch<T, 64, MVW>(L);
  // padded layout in both precisions (with compiled plans the FP32 conflicts
  // of the strided pass writes cost more than the address arithmetic; the
  // strides that are multiples of 16 take immediate offsets)
  typedef LV<T, true> XV;
  const XV PV{0};
  // twiddle table in LDS (behind the data), read by every radix pass
  cx<T>* twl = P + lds_span<true>((size_t)XS::NP * L);
  typedef typename V2<T>::type T2;
  const short* src = XSRC[DIM - 2];
  const short* dxf = XDX[DIM - 2];
  // each wave packs whole field pairs, so the field tables are read once per
  // pair (wave-uniform) and the lanes stream one field's kx modes
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // loads in issue order: the twiddles (a few per thread), then the first
  // items, whose latency the twiddle stores then overlap (loads complete in
  // order, so the twiddles come first)
  constexpr int TWN = (64 * cover(XMVW) + NTH - 1) / NTH;  // the longest line xpencil_lds_bytes admits
  if constexpr (LC > 0) {
    // compiled lengths (L = 3 nkx): radix-3 first pass from the spectra
    constexpr int NKX = LC / 3, NU = NKX / 2, NUB = (NU + 63) / 64;
    constexpr int RM = MVW < 16 ? MVW : 16, SWX = xp_batch<LC, MVW>();
    static_assert(SWX >= 1 && NKX * 3 == LC, "x line");
    constexpr int nb = XS::NP;
    const XV X = PV;
    // the wave's items: (pair q = wave + NW i, block of 64 units); the loads
    // of GI items (four modes each) are issued before any is transformed
    const int items = max(0, (nb - wave + NW - 1) / NW) * NUB;
    constexpr int GI = (sizeof(T) == 4 && DIM == 3) ? 4 : 2;
    T2 va1[GI], vb1[GI], va2[GI], vb2[GI];
    auto load_units = [&](int i0) {
#pragma unroll
      for (int g = 0; g < GI; ++g) {
        const int it = i0 + g, qi = it / NUB, u = lane + 64 * (it - qi * NUB);
        const int fa = 2 * (wave + NW * qi), fb = fa + 1;
        va1[g] = vb1[g] = va2[g] = vb2[g] = T2{0, 0};
        if (it < items && u < NU) {
          const int j2 = u ? NKX - u : NKX / 2;
          const gptr<const T> pa = base + src[fa] * fstride;
          va1[g] = *reinterpret_cast<gptr<const T2>>(pa + 2 * u);
          va2[g] = *reinterpret_cast<gptr<const T2>>(pa + 2 * j2);
          if (fb < XS::NREAL) {
            const gptr<const T> pb = base + src[fb] * fstride;
            vb1[g] = *reinterpret_cast<gptr<const T2>>(pb + 2 * u);
            vb2[g] = *reinterpret_cast<gptr<const T2>>(pb + 2 * j2);
          }
        }
      }
    };
    T2 tv[TWN];
    {
      const gptr<const T2> tw = gmem(static_cast<const T2*>(XA.tw));
#pragma unroll
      for (int r = 0; r < TWN; ++r) tv[r] = tid + r * NTH < L ? tw[tid + r * NTH] : T2{0, 0};
    }
    load_units(0);
#pragma unroll
    for (int r = 0; r < TWN; ++r)
      if (tid + r * NTH < L) twl[tid + r * NTH] = cx<T>{tv[r][0], tv[r][1]};
    for (int i0 = 0; i0 < items; i0 += GI) {
      if (i0 > 0) load_units(i0);
#pragma unroll
      for (int g = 0; g < GI; ++g) {
        const int it = i0 + g, qi = it / NUB, u = lane + 64 * (it - qi * NUB);
        const int q = wave + NW * qi, fa = 2 * q, fb = fa + 1;
        if (it < items && u < NU) {
          const int j2 = u ? NKX - u : NKX / 2;
          cx<T> A1{va1[g][0], va1[g][1]}, B1{vb1[g][0], vb1[g][1]};
          cx<T> A2{va2[g][0], va2[g][1]}, B2{vb2[g][0], vb2[g][1]};
          const bool da = dxf[fa] != 0, db = fb < XS::NREAL && dxf[fb] != 0;
          if (da || db) {
            const T k1 = T(kx[u]), k2 = T(kx[j2]);
            if (da) {
              A1 = cx<T>{-k1 * A1.y, k1 * A1.x};
              A2 = cx<T>{-k2 * A2.y, k2 * A2.x};
            }
            if (db) {
              B1 = cx<T>{-k1 * B1.y, k1 * B1.x};
              B2 = cx<T>{-k2 * B2.y, k2 * B2.x};
            }
          }
          xp_first<T>(X.at(q * L), NKX, u, A1, B1, A2, B2);
        }
      }
    }
    // every wave's twiddles (each wave's first pass wrote its own pairs)
    __syncthreads();
    const int own = (nb - wave + NW - 1) / NW;
    for (int i0 = 0; i0 < own; i0 += SWX)
      xfft_inv_tail<T, LC, RM, MVW>(X.at((wave + NW * i0) * L), NW * L, min(SWX, own - i0), twl, lane);
    __syncthreads();
  } else {
    constexpr int b0 = 0, nb = XS::NP;
    const XV X = PV;
    // the wave's items are (pair q = wave + NW i, block of 64 kx); G items'
    // loads are issued before any of them is packed
    const int nkb = (nkx + 63) >> 6;
    const int items = max(0, (nb - wave + NW - 1) / NW) * nkb;
    constexpr int G = (sizeof(T) == 4 && DIM == 3) ? 8 : 4;  // measured: 8 costs FP64 and 2D more registers than it saves
    T2 va[G], vb[G];
    auto load_items = [&](int i0) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int it = i0 + u, qi = it / nkb, k = lane + 64 * (it - qi * nkb);
        const int fa = 2 * (b0 + wave + NW * qi), fb = fa + 1;
        va[u] = vb[u] = T2{0, 0};
        if (it < items && k < nkx) {
          va[u] = *reinterpret_cast<gptr<const T2>>(base + src[fa] * fstride + 2 * k);
          if (fb < XS::NREAL) vb[u] = *reinterpret_cast<gptr<const T2>>(base + src[fb] * fstride + 2 * k);
        }
      }
    };
    T2 tv[TWN];
    {
      const gptr<const T2> tw = gmem(static_cast<const T2*>(XA.tw));
#pragma unroll
      for (int r = 0; r < TWN; ++r) tv[r] = tid + r * NTH < L ? tw[tid + r * NTH] : T2{0, 0};
    }
    load_items(0);
#pragma unroll
    for (int r = 0; r < TWN; ++r)
      if (tid + r * NTH < L) twl[tid + r * NTH] = cx<T>{tv[r][0], tv[r][1]};
    // a wave clears, fills and transforms the pairs it owns, in LDS order,
    // so only the twiddles need a workgroup barrier before the transforms;
    // the packing writes every position but the band between the retained
    // modes, which alone is cleared
    for (int q = wave; q < nb; q += NW)
      for (int e = nkx + lane; e <= L - nkx; e += 64) X[q * L + e] = cx<T>{0, 0};
    pass_sync<true>();
    for (int i0 = 0; i0 < items; i0 += G) {
      if (i0 > 0) load_items(i0);
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int it = i0 + u, qi = it / nkb, k = lane + 64 * (it - qi * nkb);
        const int q = wave + NW * qi, fa = 2 * (b0 + q), fb = fa + 1;
        if (it < items && k < nkx) {
          cx<T> A{va[u][0], va[u][1]}, B{vb[u][0], vb[u][1]};
          const bool da = dxf[fa] != 0, db = fb < XS::NREAL && dxf[fb] != 0;
          if (da || db) {
            const T kk = T(kx[k]);
            if (da) A = cx<T>{-kk * A.y, kk * A.x};
            if (db) B = cx<T>{-kk * B.y, kk * B.x};
          }
          pack_pair(X.at(q * L), L, k, A, B);
        }
      }
    }
    __syncthreads();
    const int own = (nb - wave + NW - 1) / NW;
    for (int i0 = 0; i0 < own; i0 += SW)
      fft_any<T, LC, 64, MVW, true, +1>(X.at((wave + NW * i0) * L), NW * L, pl, min(SW, own - i0), twl, lane);
    __syncthreads();
  }
  // pointwise products; outputs overwrite the first pairs at the same point
  T mrow[16];
  if constexpr (MIXED) {
    const int yrow = row / pz;
#pragma unroll
    for (int i = 0; i < n_means(DIM); ++i) mrow[i] = T(mean[(size_t)i * m1 + yrow]);
  }
  for (int n = tid; n < L; n += NTH) {
    T o[2 * XS::NOP];
    auto rd = [&](int f) -> T {
      const cx<T>& z = PV[(f >> 1) * L + n];
      return (f & 1) ? z.y : z.x;
    };
    if constexpr (MIXED) {
      auto md = [&](int f) -> T { return mean_of(DIM, f) >= 0 ? mrow[mean_of(DIM, f)] : T(0); };
      pointwise_mixed<DIM, T>(rd, md, o, T(eps_wi));
    } else {
      pointwise<DIM>(rd, o, eps_wi);
    }
    if constexpr (XS::NOUT & 1) o[2 * XS::NOP - 1] = 0;
#pragma unroll
    for (int q = 0; q < XS::NOP; ++q) PV[q * L + n] = cx<T>{o[2 * q], o[2 * q + 1]};
  }
  __syncthreads();
  const T inv = T(1.0 / L);
  const gptr<T> obase = out + (size_t)row * nkx * 2;
  if constexpr (LC > 0) {
    // compiled lengths: the radix-3 last pass unpacked and stored from registers
    constexpr int NKX = LC / 3, NU = NKX / 2;
    constexpr int RM = MVW < 16 ? MVW : 16, SWX = xp_batch<LC, MVW>();
    constexpr int nb = XS::NOP;
    const XV Z = PV;
    const int own = (nb - wave + NW - 1) / NW;
    for (int i0 = 0; i0 < own; i0 += SWX)
      xfft_fwd_head<T, LC, RM, MVW>(Z.at((wave + NW * i0) * L), NW * L, min(SWX, own - i0), twl, lane);
    for (int q = wave; q < nb; q += NW)
      for (int u = lane; u < NU; u += 64) {
        const int j2 = u ? NKX - u : NKX / 2;
        cx<T> y0a, y2a, y0b, y2b, A1, B1, A2, B2;
        xp_last<T>(Z.at(q * L), NKX, u, twl, y0a, y2a);
        xp_last<T>(Z.at(q * L), NKX, j2, twl, y0b, y2b);
        // mode u pairs Z_u with Z_(L-u) = Z_(2 nkx + j2); mode j2 with Z_(2 nkx + u)
        // (u = 0: mode 0 alone, mode nkx / 2 with its own butterfly's y2)
        if (u) {
          xp_unpack<T>(y0a, y2b, A1, B1);
        } else {
          A1 = cx<T>{y0a.x, 0};
          B1 = cx<T>{y0a.y, 0};
        }
        xp_unpack<T>(y0b, u ? y2a : y2b, A2, B2);
        const int fa = 2 * q, fb = fa + 1;
        const gptr<T> oa = obase + (size_t)fa * fstride;
        *reinterpret_cast<gptr<T2>>(oa + 2 * u) = T2{A1.x * inv, A1.y * inv};
        *reinterpret_cast<gptr<T2>>(oa + 2 * j2) = T2{A2.x * inv, A2.y * inv};
        if (fb < XS::NOUT) {
          const gptr<T> ob = obase + (size_t)fb * fstride;
          *reinterpret_cast<gptr<T2>>(ob + 2 * u) = T2{B1.x * inv, B1.y * inv};
          *reinterpret_cast<gptr<T2>>(ob + 2 * j2) = T2{B2.x * inv, B2.y * inv};
        }
        if constexpr (MIXED && DIM == 2) {
          // the kx = 0 column is the whole mean (2D has no z): complete it in FP64
          if (u == 0) {
            mcol[(size_t)fa * m1 + row] = double(A1.x * inv) + mean_product(2, fa, mean, m1, row, eps_wi);
            if (fb < XS::NOUT)
              mcol[(size_t)fb * m1 + row] = double(B1.x * inv) + mean_product(2, fb, mean, m1, row, eps_wi);
          }
        }
      }
  } else {
    constexpr int q0 = 0, nb = XS::NOP;
    const XV Z = PV;
    const int own = (nb - wave + NW - 1) / NW;
    for (int i0 = 0; i0 < own; i0 += SW)
      fft_any<T, LC, 64, MVW, true, -1>(Z.at((wave + NW * i0) * L), NW * L, pl, min(SW, own - i0), twl, lane);
    for (int q = wave; q < nb; q += NW)
      for (int k = lane; k < nkx; k += 64) {
        cx<T> A, B;
        unpack_pair(Z.at(q * L), L, k, A, B);
        const int fa = 2 * (q0 + q), fb = fa + 1;
        *reinterpret_cast<gptr<T2>>(obase + (size_t)fa * fstride + 2 * k) = T2{A.x * inv, A.y * inv};
        if (fb < XS::NOUT) *reinterpret_cast<gptr<T2>>(obase + (size_t)fb * fstride + 2 * k) = T2{B.x * inv, B.y * inv};
        if constexpr (MIXED && DIM == 2) {
          // the kx = 0 column is the whole mean (2D has no z): complete it in FP64
          if (k == 0) {
            mcol[(size_t)fa * m1 + row] = double(A.x * inv) + mean_product(2, fa, mean, m1, row, eps_wi);
            if (fb < XS::NOUT)
              mcol[(size_t)fb * m1 + row] = double(B.x * inv) + mean_product(2, fb, mean, m1, row, eps_wi);
          }
        }
      }
  }
}

template <typename T, int DIM>
__host__ __device__ constexpr size_t xpencil_lds(int L) {
  return (lds_span<true>((size_t)XShape<DIM>::NP * L) + L) * sizeof(cx<T>);
}

// Compiled plan of a line length in a kernel of NTH threads: the host takes
// 256-thread workgroups only where four fit a CU's LDS, so a length whose
// LDS does not allow that never runs there and takes the runtime plan (its
// compiled passes would only raise the kernel's registers); FP64 lines of 768
// take the runtime plan too (their compiled passes would need registers for
// fewer waves than the LDS admits).
template <typename T, int DIM, int NTH, int L>
__host__ __device__ constexpr int xpencil_lc() {
  if (sizeof(T) == 8 && L == 768) return 0;
  return (NTH > 256 || 4 * xpencil_lds<T, DIM>(L) <= 160 * 1024) ? L : 0;
}

template <typename T, int DIM, bool MIXED, int NTH>
__global__ __launch_bounds__(NTH) void xpencil_kernel(const XArgs* __restrict__ args, int nmem) {
  const XArgs& XA = args[member_of(args, nmem)];
  if (masked(XA.skip)) return;
  switch (XA.pl.L) {
    case 96: xpencil_body<T, DIM, MIXED, NTH, xpencil_lc<T, DIM, NTH, 96>()>(XA); break;
    case 192: xpencil_body<T, DIM, MIXED, NTH, xpencil_lc<T, DIM, NTH, 192>()>(XA); break;
    case 384: xpencil_body<T, DIM, MIXED, NTH, xpencil_lc<T, DIM, NTH, 384>()>(XA); break;
    case 768: xpencil_body<T, DIM, MIXED, NTH, xpencil_lc<T, DIM, NTH, 768>()>(XA); break;
    default: xpencil_body<T, DIM, MIXED, NTH, 0>(XA); break;
  }
}

// ------------------------------------------------ 3D x pencils in field chunks
// Of the 35 real fields of a 3D line only the nine values u, v, w, c enter
// products with each other (the sPTT term); each of the 26 gradients enters
// the explicit terms of eqs. (1)-(2) linearly, with coefficients made of the
// nine values: -u_k d_k u_a in N_a, -u_k d_k c_ab in F_ab, and d_k u_a in
// F_ab through (d_k u_a) c_kb and c_ak (d_k u_b) (d_y v = -(d_x u + d_z w)
// by eq. (3) adds through both of its terms).  The chunked pencil keeps the
// nine values and the nine explicit terms of its points in registers and
// passes the fields through LDS a chunk of CP pairs at a time (one pair per
// wave): the chunk's spectra are packed and inverse transformed, every point
// adds the chunk's contributions, and the LDS takes the next chunk, whose
// global loads are issued before the current chunk's transforms.  A line
// then needs CP pairs of LDS instead of 18, and several lines share a CU.

// kind of real field f of the 3D line: 0 a value (u v w c), 1 a velocity
// gradient d_k u_a, 2 a conformation gradient d_k c_q, 3 the zero pad
__host__ __device__ constexpr int x3_kind(int f) {
  return f < 9 ? 0 : f < 12 ? 1 : f < 18 ? 2 : f < 20 ? 1 : f < 26 ? 2 : f < 29 ? 1 : f < 35 ? 2 : 3;
}
// derivative direction k of gradient f
__host__ __device__ constexpr int x3_dir(int f) { return f < 18 ? 0 : f < 26 ? 1 : 2; }
// component of gradient f: a of d_k u_a, or the stored index q of d_k c_q
__host__ __device__ constexpr int x3_comp(int f) {
  return f < 12 ? f - 9 : f < 18 ? f - 12 : f == 18 ? 0 : f == 19 ? 2 : f < 26 ? f - 20 : f < 29 ? f - 26 : f - 29;
}

// product of two split factors (mean m, fluctuation f): the part containing
// a fluctuation, (am + af) bf + af bm, as fprod, with the terms of a mean part
// that does not exist (HA, HB false: the factor has no mean) left out; FP64
// path: the plain product of the values
template <bool MIXED, bool HA, bool HB, typename T>
__device__ __attribute__((always_inline)) inline T xprod(T am, T af, T bm, T bf) {
  if constexpr (!MIXED)
    return af * bf;
  else if constexpr (HA && HB)
    return (am + af) * bf + af * bm;
  else if constexpr (HA)
    return (am + af) * bf;
  else if constexpr (HB)
    return af * bf + af * bm;
  else
    return af * bf;
}

// Per point of the chunked pencil: the values v = u v w c (mixed: their
// fluctuations; the means are the line's profile values mr = the mean
// profiles at its y row, in the order of mean_of) and the explicit terms
// o = N_x N_y N_z F (6).
template <bool MIXED, typename T>
__device__ __attribute__((always_inline)) inline T x3_umean(const T (&mr)[16], int k) {
  if constexpr (MIXED) return k == 0 ? mr[0] : (k == 2 ? mr[1] : T(0));
  else return T(0);
}
template <bool MIXED, typename T>
__device__ __attribute__((always_inline)) inline T x3_cmean(const T (&mr)[16], int q) {
  if constexpr (MIXED) return mr[4 + q];
  else return T(0);
}

// contributions of G = d_K u_A = (gm, gf) (HG: G has a mean part)
template <int K, int A, bool HG, bool MIXED, typename T>
__device__ __attribute__((always_inline)) inline void x3_vgrad(T gm, T gf, const T (&mr)[16], const T (&v)[9],
                                                               T (&o)[9]) {
  o[A] -= xprod<MIXED, K != 1, HG>(x3_umean<MIXED>(mr, K), v[K], gm, gf);
  int q = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b, ++q) {
      if (a == A) {
        const int kb = cidx(3, K, b);
        o[3 + q] += xprod<MIXED, HG, true>(gm, gf, x3_cmean<MIXED>(mr, kb), v[3 + kb]);
      }
      if (b == A) {
        const int ak = cidx(3, a, K);
        o[3 + q] += xprod<MIXED, true, HG>(x3_cmean<MIXED>(mr, ak), v[3 + ak], gm, gf);
      }
    }
}

// real field F of the line at the point, value s
template <int F, bool MIXED, typename T>
__device__ __attribute__((always_inline)) inline void x3_field(T s, const T (&mr)[16], T (&v)[9], T (&o)[9]) {
  constexpr int kind = x3_kind(F);
  if constexpr (kind == 0) {
    v[F] = s;
  } else if constexpr (kind == 1 || kind == 2) {
    constexpr int K = x3_dir(F), E = x3_comp(F), MI = mean_of(3, F);
    T sm = T(0);
    if constexpr (MIXED && MI >= 0) sm = mr[MI];
    if constexpr (kind == 2) {
      o[3 + E] -= xprod<MIXED, K != 1, (MI >= 0)>(x3_umean<MIXED>(mr, K), v[K], sm, s);
    } else {
      x3_vgrad<K, E, (MI >= 0), MIXED>(sm, s, mr, v, o);
      // d_y v = -(d_x u + d_z w) (d_x u and d_z w have no mean part)
      if constexpr (F == 9 || F == 28) x3_vgrad<1, 1, false, MIXED>(T(0), -s, mr, v, o);
    }
  }
}

// the sPTT term of eq. (1), from the values alone
template <bool MIXED, typename T>
__device__ __attribute__((always_inline)) inline void x3_sptt(T eps_wi, const T (&mr)[16], const T (&v)[9],
                                                              T (&o)[9]) {
  if (eps_wi == T(0)) return;
  T tm = T(-3), tf = T(0);  // Tr(c - I): mean part and fluctuation
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int q = cidx(3, e, e);
    if constexpr (MIXED) {
      tm += mr[4 + q];
      tf += v[3 + q];
    } else {
      tf += v[3 + q] - T(1);
    }
  }
  int q = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b, ++q) {
      const T d = T(a == b ? 1 : 0);
      if constexpr (MIXED)
        o[3 + q] -= eps_wi * xprod<true, true, true>(tm, tf, mr[4 + q] - d, v[3 + q]);
      else
        o[3 + q] -= eps_wi * tf * (v[3 + q] - d);
    }
}

// fields F .. FE - 1 of a chunk that starts at field F0, read from LDS at
// point n (pair j of the chunk at j L)
template <int F, int FE, int F0, bool MIXED, typename T, typename V>
__device__ __attribute__((always_inline)) inline void x3_chunk_fields(V X, int L, int n, const T (&mr)[16], T (&v)[9],
                                                                      T (&o)[9]) {
  if constexpr (F < FE) {
    const cx<T> z = X[((F - F0) >> 1) * L + n];
    x3_field<F, MIXED>(z.x, mr, v, o);
    if constexpr (F + 1 < FE) x3_field<F + 1, MIXED>(z.y, mr, v, o);
    x3_chunk_fields<F + 2, FE, F0, MIXED>(X, L, n, mr, v, o);
  }
}

// calls f(integral_constant<int, I>) for I = I0 .. I1 - 1 in order
template <int I, int I1, typename Fn>
__device__ __attribute__((always_inline)) inline void static_for(Fn&& f) {
  if constexpr (I < I1) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, I1>(f);
  }
}

// threads of a chunked pencil: six waves, one field pair each per chunk,
// and one point per thread for lines up to 384 (measured: 256 threads, two
// points each, need 180 registers)
constexpr int X3C_NTH = 384;

template <typename T, bool MIXED, int NTH, int LC>
__device__ __attribute__((always_inline)) inline void xpencil3c_body(const XArgs& XA) {
  constexpr int CP = NTH / 64;                // field pairs per chunk
  constexpr int NCH = (18 + CP - 1) / CP;    // chunks over the 18 pairs
  constexpr int PPT = (LC + NTH - 1) / NTH;  // points per thread
  constexpr int NKB = (LC / 3 + 63) / 64;    // blocks of 64 kx (nkx = L / 3)
  // one sequence per wave: L / 64 values per lane in every pass
  constexpr int MVW = LC <= 384 ? 8 : 16;
  static_assert(64 * cover(MVW) >= LC, "a wave's pass must cover its sequence");
  typedef typename V2<T>::type T2;
  typedef LV<T, true> XV;
  const XV PV{0};
  const int nkx = XA.nkx, row = blockIdx.x - XA.blk0, tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const size_t fstride = (size_t)XA.nrows * nkx * 2;
  const gptr<const T> base = gmem(static_cast<const T*>(XA.in)) + (size_t)row * nkx * 2;
  const gptr<const double> kx = gmem(XA.kx);
  cx<T>* twl = reinterpret_cast<cx<T>*>(fft_lds) + lds_span<true>((size_t)CP * LC);
  T2 va[NKB], vb[NKB];
  // global loads of this wave's pair of chunk c (fields 2p, 2p + 1; none from 35)
  auto load = [&](int c) {
    const int fa = 2 * (c * CP + wave), fb = fa + 1;
#pragma unroll
    for (int u = 0; u < NKB; ++u) {
      const int k = lane + 64 * u;
      va[u] = vb[u] = T2{0, 0};
      if (k < nkx && fa < 35) {
        va[u] = *reinterpret_cast<gptr<const T2>>(base + XSRC[1][fa] * fstride + 2 * k);
        if (fb < 35) vb[u] = *reinterpret_cast<gptr<const T2>>(base + XSRC[1][fb] * fstride + 2 * k);
      }
    }
  };
  // packs the loaded pair (d/dx applied where the table says) into this
  // wave's sequence, zero between the retained modes
  auto pack = [&](int c) {
    const XV X = PV.at(wave * LC);
    for (int e = nkx + lane; e <= LC - nkx; e += 64) X[e] = cx<T>{0, 0};
    const int fa = 2 * (c * CP + wave), fb = fa + 1;
    const bool da = fa < 35 && XDX[1][fa] != 0, db = fb < 35 && XDX[1][fb] != 0;
#pragma unroll
    for (int u = 0; u < NKB; ++u) {
      const int k = lane + 64 * u;
      if (k < nkx) {
        cx<T> A{va[u][0], va[u][1]}, B{vb[u][0], vb[u][1]};
        if (da || db) {
          const T kk = T(kx[k]);
          if (da) A = cx<T>{-kk * A.y, kk * A.x};
          if (db) B = cx<T>{-kk * B.y, kk * B.x};
        }
        pack_pair(X, LC, k, A, B);
      }
    }
    pass_sync<true>();  // the wave's transform reads what its lanes wrote
  };
  // twiddles (loads issued first), then chunk 0's loads
  constexpr int TWN = (LC + NTH - 1) / NTH;
  T2 tv[TWN];
  {
    const gptr<const T2> g = gmem(static_cast<const T2*>(XA.tw));
#pragma unroll
    for (int r = 0; r < TWN; ++r) tv[r] = tid + r * NTH < LC ? g[tid + r * NTH] : T2{0, 0};
  }
  load(0);
#pragma unroll
  for (int r = 0; r < TWN; ++r)
    if (tid + r * NTH < LC) twl[tid + r * NTH] = cx<T>{tv[r][0], tv[r][1]};
  T mr[16];
  if constexpr (MIXED) {
    const gptr<const double> mean = gmem(XA.mean);
    const int yrow = row / XA.pz;
    // one value per workgroup: kept in scalar registers
#pragma unroll
    for (int i = 0; i < 16; ++i)
      mr[i] = __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(
                                        __builtin_bit_cast(int, T(mean[(size_t)i * XA.m1 + yrow]))));
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) mr[i] = T(0);
  }
  T pv[PPT][9], po[PPT][9];
#pragma unroll
  for (int i = 0; i < PPT; ++i)
#pragma unroll
    for (int q = 0; q < 9; ++q) pv[i][q] = po[i][q] = T(0);
  __syncthreads();  // the twiddles
  static_for<0, NCH>([&](auto cc) {
    constexpr int C = decltype(cc)::value;
    pack(C);
    if constexpr (C + 1 < NCH) load(C + 1);
    fft_any<T, LC, 64, MVW, true, +1>(PV.at(wave * LC), LC, XA.pl, 1, twl, lane);
    __syncthreads();
    constexpr int F0 = 2 * CP * C, FE = (2 * CP * (C + 1) < 35) ? 2 * CP * (C + 1) : 35;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int n = tid + i * NTH;
      if (n < LC) x3_chunk_fields<F0, FE, F0, MIXED>(PV, LC, n, mr, pv[i], po[i]);
    }
    __syncthreads();
  });
  // the explicit terms to LDS as five pairs (the last half zero), forward
  // transforms (a wave per pair), truncation to the retained modes
  const T eps_wi = T(XA.eps_wi);
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int n = tid + i * NTH;
    if (n < LC) {
      x3_sptt<MIXED>(eps_wi, mr, pv[i], po[i]);
#pragma unroll
      for (int q = 0; q < 5; ++q) PV[q * LC + n] = cx<T>{po[i][2 * q], q < 4 ? po[i][2 * q + 1] : T(0)};
    }
  }
  __syncthreads();
  const T inv = T(1.0 / LC);
  const gptr<T> obase = gmem(static_cast<T*>(XA.out)) + (size_t)row * nkx * 2;
  for (int q = wave; q < 5; q += CP) {
    fft_any<T, LC, 64, MVW, true, -1>(PV.at(q * LC), LC, XA.pl, 1, twl, lane);
    for (int k = lane; k < nkx; k += 64) {
      cx<T> A, B;
      unpack_pair(PV.at(q * LC), LC, k, A, B);
      const int fa = 2 * q, fb = fa + 1;
      *reinterpret_cast<gptr<T2>>(obase + (size_t)fa * fstride + 2 * k) = T2{A.x * inv, A.y * inv};
      if (fb < 9) *reinterpret_cast<gptr<T2>>(obase + (size_t)fb * fstride + 2 * k) = T2{B.x * inv, B.y * inv};
    }
  }
}

// One compiled line length per kernel (its registers are those of that
// length alone); xpencil_chunked admits a launch whose lines all have it.
template <typename T, bool MIXED, int NTH, int LC>
__global__ __launch_bounds__(NTH) void xpencil3c_kernel(const XArgs* __restrict__ args, int nmem) {
  const XArgs& XA = args[member_of(args, nmem)];
  if (masked(XA.skip)) return;
  xpencil3c_body<T, MIXED, NTH, LC>(XA);
}

// ---------------------------------------------------------------- z columns
// Complex transforms along the spanwise index of [field][y][z row][kx] data.
// inverse: kz slots (Nyquist slot skipped, optional i kz factor) are placed at
// their own frequency in a length-Lz transform; forward: length-Lz data is
// transformed, divided by Lz and truncated to the retained slots.
// kx columns per workgroup: G of 32, 16 or 8, the largest whose columns fit
// ZLDS_TARGET bytes of LDS (zfft_group), so that several workgroups share a
// CU.  Measured (inverse transforms, ms per launch): 256 x 257 x 128 FP32
// 1.22 with 32 columns of 192 (49 KB) against 0.84 with 16, FP64 2.42 with 16
// (52 KB) against 2.03 with 8; 128 x 129 x 64 FP32 0.100 with 32 columns of
// 96 (25 KB) against 0.105 with 16, FP64 0.251 with 16 against 0.309 with 8.
constexpr size_t ZLDS_TARGET = 40 * 1024;
// Complex values per thread of the z columns: 24 (one register batch holds
// all 32 columns up to length 192; measured faster than 16 in both precisions,
// the compiler also allocating fewer registers for it).
constexpr int ZMV = 24;

// LC: the column length when it has a compiled plan, else 0; ZG: columns
// per workgroup.
template <typename T, int MV, int LC, int ZG>
__device__ __attribute__((always_inline)) inline void zfft_body(const ZArgs& ZA) {
  typedef cx<T> c2;
  const gptr<const T> in = gmem(static_cast<const T*>(ZA.in));
  const gptr<T> out = gmem(static_cast<T*>(ZA.out));
  const int nkx = ZA.nkx, nzs = ZA.nzs, rows_y = ZA.rows, inverse = ZA.inverse;
  const FftPlan& pl = ZA.pl;
  const int* src_field = ZA.src_field;
  const int* deriv = ZA.deriv;
  const gptr<const double> kz = gmem(ZA.kz);
  const gptr<const double> mean = gmem(ZA.mean);
  const gptr<double> mcol = gmem(ZA.mcol);
  c2* A = reinterpret_cast<c2*>(fft_lds);
  const int L = LC > 0 ? LC : pl.L;
  // sequences (one per kx column) at stride L + 1: the column-wise loads and
  // stores of neighbouring kx then fall on different LDS banks
  const int SL = L + 1;
  const LV<T> AV{0};
  c2* twl = A + lds_padded<T>((size_t)ZG * SL);  // twiddle table behind the data
  typedef typename V2<T>::type T2;
  {
    const gptr<const T2> tw = gmem(static_cast<const T2*>(ZA.tw));
    for (int e = threadIdx.x; e < L; e += NT) {
      const T2 t = tw[e];
      twl[e] = c2{t[0], t[1]};
    }
  }
  // local workgroup -> (kx group, row, field).  Pairs (field k, its d/dz)
  // first, in groups of 16 blocks: 8 units of a source field, then the same
  // 8 units of its derivative (a last group of rem < 8 units likewise with
  // rem), then the unpaired fields one after the other
  const int lb = blockIdx.x - ZA.blk0;
  const int U = ZA.ngx * rows_y, np = ZA.npair;
  int f, w;
  if (np > 0 && lb < 2 * np * U) {
    const int q = lb >> 4, r = lb & 15, rem = min(8, np * U - 8 * q);
    const bool second = r >= rem;
    const int unit = 8 * q + (second ? r - rem : r);
    const int k = unit / U;
    w = unit - k * U;
    f = second ? ZA.nfields - np + k : k;
  } else {
    const int lr = lb - 2 * np * U;
    const int k = lr / U;
    w = lr - k * U;
    f = np + k;
  }
  const int gx = w % ZA.ngx, i = w / ZA.ngx;
  const int k0 = gx * ZG;
  const int ng = min(ZG, nkx - k0);
  const unsigned mng = fast_div_magic((unsigned)ng);
  const int tid = threadIdx.x;
  const int rin = inverse ? nzs : L, rout = inverse ? L : nzs;
  const int sf = src_field ? src_field[f] : f;
  const int dz = deriv ? deriv[f] : 0;
  const gptr<const T> ib = in + ((size_t)sf * rows_y + i) * rin * nkx * 2;
  const gptr<T> ob = out + ((size_t)f * rows_y + i) * rout * nkx * 2;
  // as many columns per batch as one pass holds in registers
  // (compiled plans: 16 values per thread, whose registers keep the
  // occupancy of the runtime plan's 24)
  constexpr int MVC = LC > 0 ? 16 : MV;
  if constexpr (LC > 0 && LC % 3 == 0) {
    // padded columns (L = 3 nzs / 2): radix-3 pass first (inverse) or last
    // (forward) over the 3/2-rule band, fed from and stored to HBM through
    // registers (see the x lines); butterfly j holds the stored modes j and
    // nzs / 2 + j (the Nyquist slot, j = 0, is zero)
    if (2 * L == 3 * nzs) {
      constexpr int NZH = LC / 3, S = NT * MVC / LC;
      // FP32 with an even column count: each thread takes two adjacent kx
      // columns (contiguous in HBM) with 16-byte loads and stores
      typedef T T4 __attribute__((ext_vector_type(4)));
      const bool two = sizeof(T) == 4 && ((ng | nkx | k0) & 1) == 0;
      const int nh = ng >> 1;
      const unsigned mnh = fast_div_magic((unsigned)max(nh, 1));
      if (inverse && two) {
        constexpr int PB = 4;
        const int tot = NZH * nh;
        for (int e0 = 0; e0 < tot; e0 += PB * NT) {
          T4 xa[PB], xc[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int e = e0 + tid + u * NT;
            xa[u] = xc[u] = T4{0, 0, 0, 0};
            if (e < tot) {
              const int j = fdiv(e, mnh), g = 2 * (e - j * nh);
              xa[u] = *reinterpret_cast<gptr<const T4>>(ib + ((size_t)j * nkx + k0 + g) * 2);
              if (j > 0) xc[u] = *reinterpret_cast<gptr<const T4>>(ib + ((size_t)(NZH + j) * nkx + k0 + g) * 2);
            }
          }
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < tot) {
              const int j = fdiv(e, mnh), g = 2 * (e - j * nh);
              c2 a0{xa[u][0], xa[u][1]}, c0{xc[u][0], xc[u][1]}, a1{xa[u][2], xa[u][3]}, c1{xc[u][2], xc[u][3]};
              if (dz) {
                const T ka = T(kz[j]), kc = T(kz[NZH + j]);
                a0 = c2{-ka * a0.y, ka * a0.x};
                c0 = c2{-kc * c0.y, kc * c0.x};
                a1 = c2{-ka * a1.y, ka * a1.x};
                c1 = c2{-kc * c1.y, kc * c1.x};
              }
              xp_first3<T>(AV.at(g * SL + 3 * j), a0, c0);
              xp_first3<T>(AV.at((g + 1) * SL + 3 * j), a1, c1);
            }
          }
        }
        __syncthreads();
        for (int b0 = 0; b0 < ng; b0 += S)
          xfft_inv_tail<T, LC, 16, MVC, NT, false>(AV.at(b0 * SL), SL, min(S, ng - b0), twl, tid);
        for (int e = tid; e < L * nh; e += NT) {
          const int z = fdiv(e, mnh), g = 2 * (e - z * nh);
          const c2 v0 = AV[g * SL + z], v1 = AV[(g + 1) * SL + z];
          *reinterpret_cast<gptr<T4>>(ob + ((size_t)z * nkx + k0 + g) * 2) = T4{v0.x, v0.y, v1.x, v1.y};
        }
      } else if (inverse) {
        constexpr int PB = 4;
        const int tot = NZH * ng;
        for (int e0 = 0; e0 < tot; e0 += PB * NT) {
          T2 xa[PB], xc[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int e = e0 + tid + u * NT;
            xa[u] = xc[u] = T2{0, 0};
            if (e < tot) {
              const int j = fdiv(e, mng), g = e - j * ng;
              xa[u] = *reinterpret_cast<gptr<const T2>>(ib + ((size_t)j * nkx + k0 + g) * 2);
              if (j > 0) xc[u] = *reinterpret_cast<gptr<const T2>>(ib + ((size_t)(NZH + j) * nkx + k0 + g) * 2);
            }
          }
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < tot) {
              const int j = fdiv(e, mng), g = e - j * ng;
              c2 a{xa[u][0], xa[u][1]}, c{xc[u][0], xc[u][1]};
              if (dz) {
                const T ka = T(kz[j]), kc = T(kz[NZH + j]);
                a = c2{-ka * a.y, ka * a.x};
                c = c2{-kc * c.y, kc * c.x};
              }
              xp_first3<T>(AV.at(g * SL + 3 * j), a, c);
            }
          }
        }
        __syncthreads();
        for (int b0 = 0; b0 < ng; b0 += S)
          xfft_inv_tail<T, LC, 16, MVC, NT, false>(AV.at(b0 * SL), SL, min(S, ng - b0), twl, tid);
        for (int e = tid; e < L * ng; e += NT) {
          const int z = fdiv(e, mng), g = e - z * ng;
          const c2 v = AV[g * SL + z];
          *reinterpret_cast<gptr<T2>>(ob + ((size_t)z * nkx + k0 + g) * 2) = T2{v.x, v.y};
        }
      } else if (two) {
        constexpr int PER = 8;
        const int tot = L * nh;
        for (int e0 = 0; e0 < tot; e0 += PER * NT) {
          T4 v[PER];
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < tot) {
              const int z = fdiv(e, mnh), g = 2 * (e - z * nh);
              v[u] = *reinterpret_cast<gptr<const T4>>(ib + ((size_t)z * nkx + k0 + g) * 2);
            }
          }
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < tot) {
              const int z = fdiv(e, mnh), g = 2 * (e - z * nh);
              AV[g * SL + z] = c2{v[u][0], v[u][1]};
              AV[(g + 1) * SL + z] = c2{v[u][2], v[u][3]};
            }
          }
        }
        __syncthreads();
        for (int b0 = 0; b0 < ng; b0 += S)
          xfft_fwd_head<T, LC, 16, MVC, NT, false>(AV.at(b0 * SL), SL, min(S, ng - b0), twl, tid);
        const T inv = T(1.0 / L);
        for (int e = tid; e < NZH * nh; e += NT) {
          const int j = fdiv(e, mnh), g = 2 * (e - j * nh);
          c2 y0, y2, w0, w2;
          xp_last<T>(AV.at(g * SL), NZH, j, twl, y0, y2);
          xp_last<T>(AV.at((g + 1) * SL), NZH, j, twl, w0, w2);
          y0 = scal(inv, y0);
          w0 = scal(inv, w0);
          y2 = j ? scal(inv, y2) : c2{0, 0};
          w2 = j ? scal(inv, w2) : c2{0, 0};
          *reinterpret_cast<gptr<T4>>(ob + ((size_t)j * nkx + k0 + g) * 2) = T4{y0.x, y0.y, w0.x, w0.y};
          *reinterpret_cast<gptr<T4>>(ob + ((size_t)(NZH + j) * nkx + k0 + g) * 2) = T4{y2.x, y2.y, w2.x, w2.y};
          // mixed forward transform: the kx = kz = 0 value completed in FP64
          if (mcol && j == 0 && k0 + g == 0)
            mcol[(size_t)f * rows_y + i] = double(y0.x) + mean_product(3, f, mean, rows_y, i, ZA.eps_wi);
        }
      } else {
        constexpr int PER = 8;
        const int tot = L * ng;
        for (int e0 = 0; e0 < tot; e0 += PER * NT) {
          T2 v[PER];
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < tot) {
              const int z = fdiv(e, mng), g = e - z * ng;
              v[u] = *reinterpret_cast<gptr<const T2>>(ib + ((size_t)z * nkx + k0 + g) * 2);
            }
          }
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < tot) {
              const int z = fdiv(e, mng), g = e - z * ng;
              AV[g * SL + z] = c2{v[u][0], v[u][1]};
            }
          }
        }
        __syncthreads();
        for (int b0 = 0; b0 < ng; b0 += S)
          xfft_fwd_head<T, LC, 16, MVC, NT, false>(AV.at(b0 * SL), SL, min(S, ng - b0), twl, tid);
        const T inv = T(1.0 / L);
        for (int e = tid; e < NZH * ng; e += NT) {
          const int j = fdiv(e, mng), g = e - j * ng;
          c2 y0, y2;
          xp_last<T>(AV.at(g * SL), NZH, j, twl, y0, y2);
          y0 = scal(inv, y0);
          y2 = j ? scal(inv, y2) : c2{0, 0};
          *reinterpret_cast<gptr<T2>>(ob + ((size_t)j * nkx + k0 + g) * 2) = T2{y0.x, y0.y};
          *reinterpret_cast<gptr<T2>>(ob + ((size_t)(NZH + j) * nkx + k0 + g) * 2) = T2{y2.x, y2.y};
          // mixed forward transform: the kx = kz = 0 value completed in FP64
          if (mcol && j == 0 && k0 + g == 0)
            mcol[(size_t)f * rows_y + i] = double(y0.x) + mean_product(3, f, mean, rows_y, i, ZA.eps_wi);
        }
      }
      return;
    }
  }
  // gather PER elements per thread before writing LDS, so that many global
  // loads are in flight at once
  constexpr int PER = 8;
  if (inverse) {
    // zero the band between the retained slots (the Nyquist slot's position
    // included); the scatter below writes every other position of a column,
    // at addresses disjoint from the band
    {
      const int h = nzs / 2, nb = L - nzs + 1;
      for (int e = tid; e < ng * nb; e += NT) {
        const int g = e / nb;
        AV[g * SL + h + (e - g * nb)] = c2{0, 0};
      }
    }
    const int tot = nzs * ng;
    for (int e0 = 0; e0 < tot; e0 += PER * NT) {
      c2 v[PER];
      int pos[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + tid + u * NT;
        pos[u] = -1;
        if (e < tot) {
          const int s = fdiv(e, mng), g = e - s * ng;
          if (!(nzs > 1 && s == nzs / 2)) {
            const T2 x = *reinterpret_cast<gptr<const T2>>(ib + ((size_t)s * nkx + k0 + g) * 2);
            v[u] = c2{x[0], x[1]};
            if (dz) {
              const T kk = T(kz[s]);
              v[u] = c2{-kk * v[u].y, kk * v[u].x};
            }
            const int mz = (s < nzs / 2) ? s : s - nzs;
            pos[u] = g * SL + (mz < 0 ? mz + L : mz);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if (pos[u] >= 0) AV[pos[u]] = v[u];
    }
  } else {
    const int tot = L * ng;
    for (int e0 = 0; e0 < tot; e0 += PER * NT) {
      c2 v[PER];
      int pos[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + tid + u * NT;
        pos[u] = -1;
        if (e < tot) {
          const int z = fdiv(e, mng), g = e - z * ng;
          const T2 x = *reinterpret_cast<gptr<const T2>>(ib + ((size_t)z * nkx + k0 + g) * 2);
          v[u] = c2{x[0], x[1]};
          pos[u] = g * SL + z;
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if (pos[u] >= 0) AV[pos[u]] = v[u];
    }
  }
  __syncthreads();
  const int S = fft_batch<T, NT, MVC>(L);
  for (int b0 = 0; b0 < ng; b0 += S) {
    if (inverse)
      fft_any<T, LC, NT, MVC, false, +1>(AV.at(b0 * SL), SL, pl, min(S, ng - b0), twl, tid);
    else
      fft_any<T, LC, NT, MVC, false, -1>(AV.at(b0 * SL), SL, pl, min(S, ng - b0), twl, tid);
  }
  if (inverse) {
    for (int e = tid; e < L * ng; e += NT) {
      const int z = fdiv(e, mng), g = e - z * ng;
      const c2 v = AV[g * SL + z];
      *reinterpret_cast<gptr<T2>>(ob + ((size_t)z * nkx + k0 + g) * 2) = T2{v.x, v.y};
    }
  } else {
    const T inv = T(1.0 / L);
    for (int e = tid; e < nzs * ng; e += NT) {
      const int s = fdiv(e, mng), g = e - s * ng;
      c2 v{0, 0};
      if (!(nzs > 1 && s == nzs / 2)) {
        const int mz = (s < nzs / 2) ? s : s - nzs;
        v = scal(inv, AV[g * SL + (mz < 0 ? mz + L : mz)]);
      }
      *reinterpret_cast<gptr<T2>>(ob + ((size_t)s * nkx + k0 + g) * 2) = T2{v.x, v.y};
      // mixed forward transform: the kx = kz = 0 value completed in FP64
      if (mcol && s == 0 && k0 + g == 0)
        mcol[(size_t)f * rows_y + i] = double(v.x) + mean_product(3, f, mean, rows_y, i, ZA.eps_wi);
    }
  }
}

template <typename T, int MV, int ZG>
__global__ __launch_bounds__(NT) void zfft_kernel(const ZArgs* __restrict__ args, int nmem) {
  const ZArgs& ZA = args[member_of(args, nmem)];
  if (masked(ZA.skip)) return;
  switch (ZA.pl.L) {
    case 64: zfft_body<T, MV, 64, ZG>(ZA); break;  // the diagnostics' base-grid z transforms
    case 96: zfft_body<T, MV, 96, ZG>(ZA); break;
    case 128: zfft_body<T, MV, 128, ZG>(ZA); break;
    case 192: zfft_body<T, MV, 192, ZG>(ZA); break;
    default: zfft_body<T, MV, 0, ZG>(ZA); break;
  }
}

// ---------------------------------------------------------------- diagnostics
// Base-grid values of Tr c, u, v, w on every (y_j, z) line from their spectral
// values (Tr c = c_xx + c_yy (+ c_zz) is formed by the step's last kernel; 2D
// adds the constant c_zz = 1 after the transform) by the inverse x transform.  Per line: min Tr c, counts of
// Tr c < 3 and < 0 (strict), max CFL contribution |u|/dx + |v|/dy_j + |w|/dz,
// sums of |u|^2/2 and Tr c, and non-finite / |Tr c| > 1e12 flags.  Sums are
// reduced in a fixed order (wave butterflies, then waves in index order), so
// replays are bitwise reproducible.
__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline unsigned long long wave_sumu(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline int wave_or(int v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}

// Two waves per line: one transform pair each (so no wave idles during the
// transforms), and small workgroups pack eight lines per CU.
constexpr int DNT = 128;

// LC: the line length when it has a compiled plan, else 0.
template <int LC>
__device__ __attribute__((always_inline)) inline void diag_rows_body(const DRowArgs& DA, DiagPart* wpart,
                                                                     double* wred) {
  const Dims d = DA.d;
  const gptr<const double> in = gmem(DA.in);
  const int zrows = DA.zrows;
  const FftPlan& pl = DA.pl;
  const gptr<const double> ydy = gmem(DA.ydy);
  DiagPart* __restrict__ parts = DA.parts;
  c2* A = reinterpret_cast<c2*>(fft_lds);
  const int L = LC > 0 ? LC : pl.L, nkx = d.nkx;
  const unsigned mkx = fast_div_magic((unsigned)nkx);
  const LV<double> AV{0};
  c2* twl = A + lds_padded<double>(2 * (size_t)L);  // twiddle table behind the data
  {
    typedef V2<double>::type D2;
    const gptr<const D2> tw = gmem(reinterpret_cast<const D2*>(DA.tw));
    for (int e = threadIdx.x; e < L; e += DNT) {
      const D2 t = tw[e];
      twl[e] = c2{t[0], t[1]};
    }
  }
  const int row = blockIdx.x - DA.blk0, tid = threadIdx.x;
  const int nrows = (d.N + 1) * zrows;
  const int j = row / zrows;
  const size_t fstride = (size_t)nrows * nkx * 2;
  const gptr<const double> base = in + (size_t)row * nkx * 2;
  for (int e = tid; e < 2 * L; e += DNT) AV[e] = c2{0, 0};
  __syncthreads();
  const int nf = d.dim == 2 ? 3 : 4;
  for (int e = tid; e < 2 * nkx; e += DNT) {
    const int q = fdiv(e, mkx), k = e - q * nkx;
    const int fa = 2 * q, fb = fa + 1;
    c2 Av{0, 0}, Bv{0, 0};
    if (fa < nf) Av = c2{base[fa * fstride + 2 * k], base[fa * fstride + 2 * k + 1]};
    if (fb < nf) Bv = c2{base[fb * fstride + 2 * k], base[fb * fstride + 2 * k + 1]};
    pack_pair(AV.at(q * L), L, k, Av, Bv);
  }
  __syncthreads();
  // the two pairs: one wave each (lines longer than a wave's batch: the
  // workgroup's passes)
  if (L <= 64 * cover(16)) {
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wave < 2) fft_any<double, LC, 64, 16, true, +1>(AV.at(wave * L), L, pl, 1, twl, tid & 63);
    __syncthreads();
  } else {
    lds_fft<double, DNT, 16>(AV, L, pl, 2, twl, +1);
  }
  const double dx = d.lx / d.nx, dz = d.dim == 3 ? d.lz / d.nz : 1.0;
  const double dyj = ydy[j];
  double mn = 1.0 / 0.0, cf = 0, es = 0, ts = 0;
  unsigned long long n3 = 0, n0 = 0;
  int flag = 0, big = 0;
  // the midplane row (y = 0 exactly at j = N/2) feeds the histograms
  const bool midrow = (j == d.N / 2);
  const double um = (midrow && DA.hbins[1] > 0) ? gmem(DA.umean)[0] : 0.0;
  const double wm = (midrow && DA.hbins[3] > 0 && DA.wmean) ? gmem(DA.wmean)[0] : 0.0;
  auto bin_sample = [&](int qh, double val) {
    const int hb = DA.hbins[qh];
    if (hb <= 0) return;
    const double x = (val - DA.hlo[qh]) * DA.hscale[qh];
    const int bin = !(x < (double)hb) ? hb + 1 : (x < 0.0 ? 0 : (int)x + 1);
    unsigned long long* h = DA.hist + (size_t)qh * (HIST_MAX + 2);
    // one atomic per distinct bin of the wave (a narrow distribution would
    // otherwise send every sample to the same counter)
    unsigned long long todo = __ballot(1);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int b = __shfl(bin, leader);
      const unsigned long long same = __ballot(bin == b);
      if ((tid & 63) == leader) atomicAdd(&h[b], (unsigned long long)__popcll(same));
      todo &= ~same;
    }
  };
  for (int n = tid; n < L; n += DNT) {
    const c2 z0 = AV[n], z1 = AV[L + n];
    const double trc = z0.x + (d.dim == 2 ? 1.0 : 0.0);
    const double u = z0.y, v = z1.x, w = d.dim == 3 ? z1.y : 0.0;
    if (midrow) {
      bin_sample(0, trc);
      bin_sample(1, u - um);
      bin_sample(2, v);
      bin_sample(3, w - wm);
    }
    mn = fmin(mn, trc);
    n3 += (trc < 3.0);
    n0 += (trc < 0.0);
    double c = fabs(u) / dx + fabs(v) / dyj;
    if (d.dim == 3) c += fabs(w) / dz;
    cf = fmax(cf, c);
    es += 0.5 * (u * u + v * v + w * w);
    ts += trc;
    flag |= !(isfinite(trc) && isfinite(u) && isfinite(v) && isfinite(w));
    big |= (fabs(trc) > 1.0e12);
  }
  mn = wave_min(mn);
  cf = wave_max(cf);
  es = wave_sum(es);
  ts = wave_sum(ts);
  n3 = wave_sumu(n3);
  n0 = wave_sumu(n0);
  flag = wave_or(flag);
  big = wave_or(big);
  const int wv = tid >> 6;
  if ((tid & 63) == 0) {
    DiagPart q;
    q.min_trc = mn;
    q.cfl = cf;
    q.esum = es;
    q.tsum = ts;
    q.n_lt3 = n3;
    q.n_lt0 = n0;
    q.nonfinite = flag;
    q.big = big;
    wpart[wv] = q;
  }
  __syncthreads();
  if (tid == 0) {
    DiagPart q = wpart[0];
    for (int w2 = 1; w2 < DNT / 64; ++w2) {
      const DiagPart& o = wpart[w2];
      q.min_trc = fmin(q.min_trc, o.min_trc);
      q.cfl = fmax(q.cfl, o.cfl);
      q.esum += o.esum;
      q.tsum += o.tsum;
      q.n_lt3 += o.n_lt3;
      q.n_lt0 += o.n_lt0;
      q.nonfinite |= o.nonfinite;
      q.big |= o.big;
    }
    parts[row] = q;
  }
  if (!midrow) return;
  // ---- midplane line z: running moments of every histogrammed quantity (the
  // count, sum and sum of squares of its finite samples, reduced in a fixed
  // order), then the velocity gradients d_x u, d_z u, d_x w, d_z w
  const int z = row - j * zrows;
  double* mp = DA.mparts + (size_t)z * HIST_Q * 3;
  auto moments = [&](int qh, auto value) {
    if (DA.hbins[qh] <= 0) return;
    double c = 0, s1 = 0, s2 = 0;
    for (int n = tid; n < L; n += DNT) {
      const double x = value(n);
      if (isfinite(x)) {
        c += 1.0;
        s1 += x;
        s2 += x * x;
      }
    }
    c = wave_sum(c);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    __syncthreads();
    if ((tid & 63) == 0) {
      wred[3 * wv] = c;
      wred[3 * wv + 1] = s1;
      wred[3 * wv + 2] = s2;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0, b = 0, e2 = 0;
      for (int w2 = 0; w2 < DNT / 64; ++w2) {
        a += wred[3 * w2];
        b += wred[3 * w2 + 1];
        e2 += wred[3 * w2 + 2];
      }
      mp[3 * qh] = a;
      mp[3 * qh + 1] = b;
      mp[3 * qh + 2] = e2;
    }
  };
  const double trc_add = d.dim == 2 ? 1.0 : 0.0;
  moments(0, [&](int n) { return AV[n].x + trc_add; });
  moments(1, [&](int n) { return AV[n].y - um; });
  moments(2, [&](int n) { return AV[L + n].x; });
  if (d.dim == 3) moments(3, [&](int n) { return AV[L + n].y - wm; });
  const bool grads = DA.hbins[4] > 0 || DA.hbins[5] > 0 || DA.hbins[6] > 0 || DA.hbins[7] > 0;
  if (!grads) return;
  // pairs (d_x u, d_z u) and (d_x w, d_z w): d_x by i kx on the line's
  // spectra, d_z from the midplane row's z transform with i kz (3D)
  __syncthreads();
  for (int e = tid; e < 2 * L; e += DNT) AV[e] = c2{0, 0};
  __syncthreads();
  const gptr<const double> kxv = gmem(DA.kx);
  for (int e = tid; e < 2 * nkx; e += DNT) {
    const int q = fdiv(e, mkx), k = e - q * nkx;
    c2 Av{0, 0}, Bv{0, 0};
    if (q == 0 || d.dim == 3) {
      const int fsrc = q == 0 ? 1 : 3;  // u and w among the inputs [Tr c, u, v, w]
      const double fr = base[fsrc * fstride + 2 * k], fi = base[fsrc * fstride + 2 * k + 1];
      const double kk = kxv[k];
      Av = c2{-kk * fi, kk * fr};
      if (d.dim == 3) {
        const gptr<const double> zg = gmem(DA.zgrad) + ((size_t)q * zrows + z) * nkx * 2;
        Bv = c2{zg[2 * k], zg[2 * k + 1]};
      }
    }
    pack_pair(AV.at(q * L), L, k, Av, Bv);
  }
  __syncthreads();
  if (L <= 64 * cover(16)) {
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wave < 2) fft_any<double, LC, 64, 16, true, +1>(AV.at(wave * L), L, pl, 1, twl, tid & 63);
    __syncthreads();
  } else {
    lds_fft<double, DNT, 16>(AV, L, pl, 2, twl, +1);
  }
  for (int n = tid; n < L; n += DNT) {
    const c2 g0 = AV[n], g1 = AV[L + n];
    bin_sample(4, g0.x);
    bin_sample(5, g0.y);
    bin_sample(6, g1.x);
    bin_sample(7, g1.y);
  }
  moments(4, [&](int n) { return AV[n].x; });
  moments(5, [&](int n) { return AV[n].y; });
  moments(6, [&](int n) { return AV[L + n].x; });
  moments(7, [&](int n) { return AV[L + n].y; });
}

__global__ __launch_bounds__(DNT) void diag_rows_kernel(const DRowArgs* __restrict__ args, int nmem) {
  __shared__ DiagPart wpart[DNT / 64];
  __shared__ double wred[3 * (DNT / 64)];
  const DRowArgs& DA = args[member_of(args, nmem)];
  if (masked(DA.skip)) return;
  switch (DA.pl.L) {
    case 64: diag_rows_body<64>(DA, wpart, wred); break;
    case 128: diag_rows_body<128>(DA, wpart, wred); break;
    case 256: diag_rows_body<256>(DA, wpart, wred); break;
    case 512: diag_rows_body<512>(DA, wpart, wred); break;
    default: diag_rows_body<0>(DA, wpart, wred); break;
  }
}

// one workgroup per member
// Step record of one member from its per-line partial records: min / max /
// sums over lines in a fixed order (per thread over its lines, then wave
// butterflies, then waves in index order), so replays are bitwise identical.
// One workgroup per member.  (Folding this into the row kernel's last
// workgroup was measured slower: the device-scope fences it needs write back
// the L2 of every XCD once per row workgroup.)
struct FinPart {
  double mn, mmn, cf, es, ts;
  unsigned long long n3, n0, m3, m0;
  int b;
};
__global__ __launch_bounds__(NT) void diag_final_kernel(const DFinArgs* __restrict__ args) {
  const DFinArgs& FA = args[blockIdx.x];
  const Dims& d = FA.d;
  const Phys& p = FA.p;
  const DiagPart* __restrict__ parts = FA.parts;
  const int zrows = FA.zrows, cap = FA.cap;
  const gptr<const double> w = gmem(FA.w);
  DevScalars* __restrict__ sc = FA.sc;
  // the previous record's scalars, loaded with the partials rather than
  // after the reduction
  const gptr<DevScalars> sg = gmem(sc);
  const long long step0 = sg->step;
  const double t0 = sg->t, pi0 = sg->pi;
  const int blowup0 = sg->blowup;
  if (blowup0) return;  // masked run: no record, the step count stays
  __shared__ FinPart fp[NT / 64];
  const int tid = threadIdx.x;
  const int n1 = d.N + 1, nrows = n1 * zrows, mid = d.N / 2;
  const double norm = 1.0 / ((double)d.nx * (d.dim == 3 ? d.nz : 1));
  double mn = 1.0 / 0.0, mmn = 1.0 / 0.0, cf = 0, es = 0, ts = 0;
  unsigned long long n3 = 0, n0 = 0, m3 = 0, m0 = 0;
  int b = 0;
  for (int r = tid; r < nrows; r += NT) {
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
  FinPart v;
  v.mn = wave_min(mn);
  v.mmn = wave_min(mmn);
  v.cf = wave_max(cf);
  v.es = wave_sum(es);
  v.ts = wave_sum(ts);
  v.n3 = wave_sumu(n3);
  v.n0 = wave_sumu(n0);
  v.m3 = wave_sumu(m3);
  v.m0 = wave_sumu(m0);
  v.b = wave_or(b);
  if ((tid & 63) == 0) fp[tid >> 6] = v;
  __syncthreads();
  // running midplane moments: quantity q summed over the midplane lines in order
  if (tid < HIST_Q && ((FA.mom_mask >> tid) & 1)) {
    const gptr<const double> mp = gmem(FA.mparts);
    double c = 0, s1 = 0, s2 = 0;
    for (int zz = 0; zz < zrows; ++zz) {
      const size_t o = ((size_t)zz * HIST_Q + tid) * 3;
      c += mp[o];
      s1 += mp[o + 1];
      s2 += mp[o + 2];
    }
    const gptr<double> ms = gmem(FA.msum) + (size_t)tid * 3;
    ms[0] += c;
    ms[1] += s1;
    ms[2] += s2;
  }
  if (tid != 0) return;
  FinPart t = fp[0];
  for (int w2 = 1; w2 < NT / 64; ++w2) {
    const FinPart& o = fp[w2];
    t.mn = fmin(t.mn, o.mn);
    t.mmn = fmin(t.mmn, o.mmn);
    t.cf = fmax(t.cf, o.cf);
    t.es += o.es;
    t.ts += o.ts;
    t.n3 += o.n3;
    t.n0 += o.n0;
    t.m3 += o.m3;
    t.m0 += o.m0;
    t.b |= o.b;
  }
  const long long step = step0 + 1;
  const double tt = t0 + p.dt;
  DiagRec r;
  r.step = step;
  r.t = tt;
  r.min_trc = t.mn;
  r.mid_min_trc = t.mmn;
  r.cfl = p.dt * t.cf;
  r.dpdx = pi0;
  r.energy = t.es;
  r.mean_trc = t.ts;
  r.n_lt3 = t.n3;
  r.n_lt0 = t.n0;
  r.mid_n_lt3 = t.m3;
  r.mid_n_lt0 = t.m0;
  r.blowup = t.b ? 1 : 0;
  r.reserved = 0;
  FA.ring[(step - 1) % cap] = r;
  sg->step = step;
  sg->t = tt;
  sg->blowup = blowup0 | r.blowup;
}

}  // namespace

// x pencils: 16 complex values per thread (83 VGPRs in FP32 3D, 108 in FP64:
// five and four waves per SIMD).  A CU runs four or five 256-thread
// workgroups unless their LDS does not fit four times; then 512-thread
// workgroups keep 16 waves per CU in flight on the same LDS.  A launch of
// fewer lines than the CUs can hold at 256 threads (a 2D grid: one line per
// padded y row) also takes 512 threads, which halves each line's passes.
int xpencil_threads(int precision, size_t lds, int lines) {
  (void)precision;
  if (lds == 0) return NT;
  if (lines < 4 * 256) return 2 * NT;
  return (160 * 1024) / lds < 4 ? 2 * NT : NT;
}

// The chunked pencil where it was measured faster than the whole line (in
// LDS-limited FP64 lines of 384: 5.07 against 5.31 ms per launch of
// 256 x 257 x 128; slower in FP32 of that size, 2.11 against 2.11 ms, and in
// lines of 192, 0.38 / 0.61 against 0.24 / 0.48 ms for 128 x 129 x 64 in
// FP32 / FP64, where its barriers lengthen each line's chain).
// PCS_XPENCIL_FORM=chunked or =whole in the environment forces a form for
// every length it supports.
bool xpencil_chunked(int dim, int L, int precision) {
  if (dim != 3 || !(L == 96 || L == 192 || L == 384)) return false;
  if (const char* e = std::getenv("PCS_XPENCIL_FORM")) {
    if (!std::strcmp(e, "whole")) return false;
    if (!std::strcmp(e, "chunked")) return true;
  }
  return precision == 0 && L == 384;
}

int xpencil_chunk_threads() { return X3C_NTH; }

template <typename T, bool MIXED>
void launch_x3c(int L, const XArgs* args, int nmem, int blocks, size_t lds, hipStream_t s) {
  if (L == 96)
    hipLaunchKernelGGL((xpencil3c_kernel<T, MIXED, X3C_NTH, 96>), dim3(blocks), dim3(X3C_NTH), lds, s, args, nmem);
  else if (L == 192)
    hipLaunchKernelGGL((xpencil3c_kernel<T, MIXED, X3C_NTH, 192>), dim3(blocks), dim3(X3C_NTH), lds, s, args, nmem);
  else if (L == 384)
    hipLaunchKernelGGL((xpencil3c_kernel<T, MIXED, X3C_NTH, 384>), dim3(blocks), dim3(X3C_NTH), lds, s, args, nmem);
}

void launch_xpencil(int dim, int precision, int threads, int chunk_len, const XArgs* args, int nmem, int blocks,
                    size_t lds, hipStream_t s) {
  if (blocks <= 0) return;
  if (chunk_len > 0) {
    (void)threads;
    if (precision == 0)
      launch_x3c<double, false>(chunk_len, args, nmem, blocks, lds, s);
    else
      launch_x3c<float, true>(chunk_len, args, nmem, blocks, lds, s);
    return;
  }
  if (precision == 0 && threads == NT) {
    if (dim == 2)
      hipLaunchKernelGGL((xpencil_kernel<double, 2, false, NT>), dim3(blocks), dim3(NT), lds, s, args, nmem);
    else
      hipLaunchKernelGGL((xpencil_kernel<double, 3, false, NT>), dim3(blocks), dim3(NT), lds, s, args, nmem);
  } else if (precision == 0) {
    if (dim == 2)
      hipLaunchKernelGGL((xpencil_kernel<double, 2, false, 2 * NT>), dim3(blocks), dim3(2 * NT), lds, s, args,
                         nmem);
    else
      hipLaunchKernelGGL((xpencil_kernel<double, 3, false, 2 * NT>), dim3(blocks), dim3(2 * NT), lds, s, args,
                         nmem);
  } else if (threads == NT) {
    if (dim == 2)
      hipLaunchKernelGGL((xpencil_kernel<float, 2, true, NT>), dim3(blocks), dim3(NT), lds, s, args, nmem);
    else
      hipLaunchKernelGGL((xpencil_kernel<float, 3, true, NT>), dim3(blocks), dim3(NT), lds, s, args, nmem);
  } else {
    if (dim == 2)
      hipLaunchKernelGGL((xpencil_kernel<float, 2, true, 2 * NT>), dim3(blocks), dim3(2 * NT), lds, s, args,
                         nmem);
    else
      hipLaunchKernelGGL((xpencil_kernel<float, 3, true, 2 * NT>), dim3(blocks), dim3(2 * NT), lds, s, args,
                         nmem);
  }
}

int xpencil_blocks(const Dims& d) { return (d.M + 1) * d.pz; }

template <typename T>
void launch_zfft_t(int group, const ZArgs* args, int nmem, int blocks, size_t lds, hipStream_t s) {
  if (group == 32)
    hipLaunchKernelGGL((zfft_kernel<T, ZMV, 32>), dim3(blocks), dim3(NT), lds, s, args, nmem);
  else if (group == 16)
    hipLaunchKernelGGL((zfft_kernel<T, ZMV, 16>), dim3(blocks), dim3(NT), lds, s, args, nmem);
  else
    hipLaunchKernelGGL((zfft_kernel<T, ZMV, 8>), dim3(blocks), dim3(NT), lds, s, args, nmem);
}

void launch_zfft(int precision, int group, const ZArgs* args, int nmem, int blocks, size_t lds, hipStream_t s) {
  if (blocks <= 0) return;
  if (precision == 0)
    launch_zfft_t<double>(group, args, nmem, blocks, lds, s);
  else
    launch_zfft_t<float>(group, args, nmem, blocks, lds, s);
}

int zfft_group(int L, int precision) {
  for (int g : {32, 16})
    if (zfft_lds_bytes(L, precision, g) <= ZLDS_TARGET) return g;
  return 8;
}

int zfft_blocks(int nkx, int rows, int nfields, int group) { return ((nkx + group - 1) / group) * rows * nfields; }

size_t zfft_lds_bytes(int L, int precision, int group) {
  return precision == 0 ? (lds_padded<double>((size_t)group * (L + 1)) + L) * sizeof(cx<double>)
                        : (lds_padded<float>((size_t)group * (L + 1)) + L) * sizeof(cx<float>);
}

void launch_diag_rows(const DRowArgs* args, int nmem, int blocks, size_t lds, hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(diag_rows_kernel, dim3(blocks), dim3(DNT), lds, s, args, nmem);
}

void launch_diag_final(const DFinArgs* args, int nmem, hipStream_t s) {
  if (nmem <= 0) return;
  hipLaunchKernelGGL(diag_final_kernel, dim3(nmem), dim3(NT), 0, s, args);
}

size_t diag_rows_lds_bytes(int L) { return (lds_padded<double>(2 * (size_t)L) + L) * sizeof(c2); }


hipError_t fft_set_attributes() {
  const int lim = 160 * 1024;
  const void* k160[] = {(const void*)xpencil_kernel<double, 2, false, NT>,
                        (const void*)xpencil_kernel<double, 3, false, NT>,
                        (const void*)xpencil_kernel<double, 2, false, 2 * NT>,
                        (const void*)xpencil_kernel<double, 3, false, 2 * NT>,
                        (const void*)xpencil_kernel<float, 2, true, NT>,
                        (const void*)xpencil_kernel<float, 3, true, NT>,
                        (const void*)xpencil_kernel<float, 2, true, 2 * NT>,
                        (const void*)xpencil_kernel<float, 3, true, 2 * NT>,
                        (const void*)xpencil3c_kernel<double, false, X3C_NTH, 96>,
                        (const void*)xpencil3c_kernel<double, false, X3C_NTH, 192>,
                        (const void*)xpencil3c_kernel<double, false, X3C_NTH, 384>,
                        (const void*)xpencil3c_kernel<float, true, X3C_NTH, 96>,
                        (const void*)xpencil3c_kernel<float, true, X3C_NTH, 192>,
                        (const void*)xpencil3c_kernel<float, true, X3C_NTH, 384>,
                        (const void*)zfft_kernel<double, ZMV, 32>,
                        (const void*)zfft_kernel<double, ZMV, 16>,
                        (const void*)zfft_kernel<double, ZMV, 8>,
                        (const void*)zfft_kernel<float, ZMV, 32>,
                        (const void*)zfft_kernel<float, ZMV, 16>,
                        (const void*)zfft_kernel<float, ZMV, 8>};
  for (const void* k : k160) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
  }
  // the row-diagnostics kernel also holds a little static LDS for its reductions
  return hipFuncSetAttribute((const void*)diag_rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
}

size_t xpencil_lds_bytes(int dim, int L, int precision, bool chunked) {
  // a wave's transform batch must hold one sequence
  if (L > 64 * cover(XMVW)) return ~(size_t)0;
  if (chunked) {
    const size_t cp = X3C_NTH / 64;
    return (lds_span<true>(cp * L) + L) * (precision == 0 ? sizeof(cx<double>) : sizeof(cx<float>));
  }
  if (precision == 0) return dim == 2 ? xpencil_lds<double, 2>(L) : xpencil_lds<double, 3>(L);
  return dim == 2 ? xpencil_lds<float, 2>(L) : xpencil_lds<float, 3>(L);
}

}  // namespace pcs
