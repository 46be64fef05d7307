// C ABI of the polymer channel-flow step (declared in include/pcs.h).
//
// pcs_init builds the wall-normal operators on the host, carves the caller's
// device workspace, uploads operators and the initial state, computes the
// per-mode homogeneous solutions of the influence-matrix method with the
// same device kernels as the step, evaluates the first explicit terms as
// history, and captures the step as HIP graphs (one step, and eight steps
// back to back); pcs_step replays them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pcs.h"
#include "host_ops.hpp"
#include "kernels.hpp"

using namespace pcs;

namespace {

constexpr int RING = 4096;
constexpr size_t ALIGN = 256;
constexpr int ZPAIRS = 9;  // d/dz fields of the 3D inverse z-transform table (u, v, w, c)
constexpr size_t RHS_SPLIT_ELEMS = 256 * 1024;  // (row, mode) elements of a launch for separate wall rows
constexpr int Y_FP32 = PCS_Y_FP32, Y_FP64 = PCS_Y_FP64, Y_COMP = PCS_Y_COMP;

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(char* b) : base(b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + ALIGN - 1) & ~(ALIGN - 1);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// A table of products in two equivalent forms: form 0 evaluates every
// product plainly, form 1 the wall-normal ones as parity products (half-size
// E and O products, see GemmJob).  The autotuner times both and keeps the
// faster form and tile configuration; h is the form in use.
struct JobList {
  std::vector<GemmJob> h, forms[2];
  std::vector<int> hmap;  // job index of every logical tile
  GemmJob* dev = nullptr;
  int* tmap = nullptr;
  GemmType type = GEMM_DDD;
  int tiles = 0, cfg = 0, form = 0;
  size_t lds = 0;
  // a plain product in both forms; addp then makes the form-1 copy a parity product
  void add(const void* A, const void* B, int ldb, void* C, int ldc, int m, int n, int k, int flags = 0,
           int scale = SCALE_NONE, const EigScale* es = nullptr, void* C2 = nullptr, int scale2 = SCALE_NONE) {
    GemmJob j{};
    j.type = type;
    j.A = A;
    j.B = B;
    j.C = C;
    j.m = m;
    j.n = n;
    j.k = k;
    j.C2 = C2;
    j.lda = gemm_lda(k);  // operators are stored row-major, padded
    j.ldb = ldb;
    j.ldc = ldc;
    j.alpha = 1.0;
    j.beta = 0.0;
    j.flags = flags;
    j.scale = scale;
    j.scale2 = scale2;
    j.es = es;
    forms[0].push_back(j);
    forms[1].push_back(j);
  }
  // Parity product (kinds and operator halves as described with GemmJob):
  // E and O have mh rows and ke columns; the full sizes are mf and kf.
  // A is the full operator (the plain form's product), Ae / Ao its halves.
  void addp(int kind, const void* A, const void* Ae, const void* Ao, const void* B, int ldb, void* C, int ldc, int mh,
            int n, int ke, int mf, int kf, int sigma, int flags = 0, int scale = SCALE_NONE,
            const EigScale* es = nullptr, void* C2 = nullptr, int scale2 = SCALE_NONE) {
    add(A, B, ldb, C, ldc, mf, n, kf, flags, scale, es, C2, scale2);
    GemmJob& j = forms[1].back();
    j.A = Ae;
    j.m = mh;
    j.k = ke;
    j.lda = gemm_lda(ke);
    j.kind = kind;
    j.A2 = Ao;
    j.mf = mf;
    j.kf = kf;
    j.sigma = sigma;
  }
  // Marks consecutive parity products that fold the same B panel (see
  // GemmJob::pair) so that the B-stationary tiles stage it once for both;
  // error-compensated products are never paired (their kernel stages four
  // panels and computes one product per tile).
  // PCS_PAIR_PANELS=0 in the environment leaves every product unpaired (for
  // comparison).
  void mark_pairs() {
    if (const char* e = std::getenv("PCS_PAIR_PANELS"))
      if (std::atoi(e) == 0) return;
    std::vector<GemmJob>& f = forms[1];
    auto plain_parity = [](const GemmJob& a) {
      return a.kind == PAR_FOLD_UNFOLD && a.scale == SCALE_NONE && a.C2 == nullptr && !gemm_type_comp((GemmType)a.type);
    };
    for (size_t j = 0; j + 1 < f.size();) {
      const GemmJob &a = f[j], &b = f[j + 1];
      if (plain_parity(a) && plain_parity(b) && a.B == b.B && a.k == b.k && a.kf == b.kf && a.ldb == b.ldb &&
          a.n == b.n && a.flags == b.flags && a.type == b.type) {
        f[j].pair = 1;
        f[j + 1].pair = 2;
        j += 2;
      } else {
        ++j;
      }
    }
  }
  int n() const { return (int)forms[0].size(); }
  void clear() {
    h.clear();
    forms[0].clear();
    forms[1].clear();
  }
  void use(int f) {
    form = f;
    h = forms[f];
  }
  // a configuration the table's form can use (the B-stationary ones: parity
  // products only, and only while the whole K range of a panel fits the LDS)
  bool allowed(int c) const {
    if (gemm_cfg_bst(c)) return form == 1 && gemm_lds_bytes(type, h.data(), n(), c) <= GEMM_LDS_MAX;
    if (gemm_type_comp(type)) return false;  // error-compensated tables: B-stationary parity products only
    return form == 0 || gemm_cfg_parity(c);
  }
  // Tile configuration before tuning: the largest tile that still gives
  // every CU a workgroup.
  void prepare() {
    if (gemm_type_comp(type)) {
      // the compensated products exist in the parity form of the B-stationary kernel only
      use(1);
      set_cfg(allowed(14) ? 14 : 15);
      return;
    }
    h = forms[form];
    int c = 7;  // configurations 0 .. 7 grow with the tile
    while (c > 0 && (!allowed(c) || gemm_prepare(h.data(), n(), c) < 256)) --c;
    if (!allowed(c)) c = 4;
    set_cfg(c);
  }
  void set_cfg(int c) {
    cfg = c;
    tiles = gemm_prepare(h.data(), n(), cfg);
    lds = gemm_lds_bytes(type, h.data(), n(), cfg);
    hmap.assign(tiles, 0);
    for (int j = 0; j < n(); ++j)
      for (int t = h[j].tile0; t < (j + 1 < n() ? h[j + 1].tile0 : tiles); ++t) hmap[t] = j;
  }
  // the largest tile count of any form and configuration (the tile map's size)
  int max_tiles() const {
    int mx = 1;
    for (int f = 0; f < 2; ++f) {
      std::vector<GemmJob> c = forms[f];
      for (int g = 0; g < GEMM_NCFG; ++g) mx = std::max(mx, gemm_prepare(c.data(), (int)c.size(), g));
    }
    return mx;
  }
  // shape signature for the tuning cache
  std::vector<int> key() const {
    std::vector<int> k{(int)type, form};
    for (auto& j : h) {
      k.push_back(j.m);
      k.push_back(j.n);
      k.push_back(j.k);
    }
    return k;
  }
  // every job of forms[1] is a parity product and every job of forms[0] a
  // plain one (add is only called through addp)
  void run(hipStream_t s) const { gemm_run(type, dev, tmap, tiles, cfg, form == 1, lds, s); }
};

// Row-major (rows x cols) operator -> the padded row-major copy (gemm_rows
// rows of gemm_lda(cols), zero padding) used as the A operand of the products.
template <typename T = double>
std::vector<T> padded(const std::vector<double>& a, int rows, int cols) {
  const int ld = gemm_lda(cols);
  std::vector<T> t((size_t)gemm_rows(rows) * ld, T(0));
  for (int i = 0; i < rows; ++i)
    for (int k = 0; k < cols; ++k) t[(size_t)i * ld + k] = (T)a[(size_t)i * cols + k];
  return t;
}
// elements of a padded operator with `rows` rows and `cols` columns
size_t opsz(int rows, int cols) { return (size_t)gemm_rows(rows) * gemm_lda(cols); }

// Parity halves of rows [r0, r0 + rows) of the m x k operator A, as rows x
// ceil(k/2) matrices padded to `out_rows` rows: Ae[i][j] = (A[i][j] +
// A[i][k-1-j]) / 2 and Ao[i][j] = (A[i][j] - A[i][k-1-j]) / 2 for j < k-1-j,
// Ae[i][mid] = A[i][mid] and Ao[i][mid] = 0 for the middle column of odd k.
// Acting on B[j] + B[k-1-j] and B[j] - B[k-1-j] they give A B exactly.
void fold(const std::vector<double>& A, int k, int r0, int rows, int out_rows, std::vector<double>& Ae,
          std::vector<double>& Ao) {
  const int ke = (k + 1) / 2;
  Ae.assign((size_t)out_rows * ke, 0.0);
  Ao.assign((size_t)out_rows * ke, 0.0);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < ke; ++j) {
      const long double a = A[(size_t)(r0 + i) * k + j], b = A[(size_t)(r0 + i) * k + (k - 1 - j)];
      if (k - 1 - j > j) {
        Ae[(size_t)i * ke + j] = (double)((a + b) / 2);
        Ao[(size_t)i * ke + j] = (double)((a - b) / 2);
      } else {
        Ae[(size_t)i * ke + j] = (double)a;
      }
    }
}
// Columns [c0, c0 + cols) of rows [0, rows) of the m x k matrix A, as a
// rows x out_cols matrix (zero beyond cols).
std::vector<double> block(const std::vector<double>& A, int k, int rows, int c0, int cols, int out_cols) {
  std::vector<double> t((size_t)rows * out_cols, 0.0);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) t[(size_t)i * out_cols + j] = A[(size_t)i * k + c0 + j];
  return t;
}

bool valid_fft(int L) {
  FftPlan p;
  return make_plan(L, &p);
}

}  // namespace

// One channel simulation: its grid, parameters, operators and every device
// buffer (all inside the caller's workspace), and its own product tables.
struct Member {
  pcs_grid g{};
  pcs_params prm{};
  Dims d{};
  Phys p{};
  const WallOps* ops = nullptr;
  FftPlan plx, plz, pbx, pbz;
  int nq = 0, nh = 0, nyin = 0, nzin = 0, nout = 0, nsolve = 0, nsv = 0;
  double *IMN, *DMN, *D, *D2, *PNM, *DP, *V, *Vinv, *DV, *wV, *lam, *d2i0, *d2in, *w, *ydy, *U1, *kx, *kz;
  // parity halves [even, odd] of the operators of the wide products:
  // padded-grid values and d/dy, D2, D, projection and D P (fold / unfold);
  // V^-1 (fold / split), V and D V (split / unfold)
  double *IMNp[2], *DMNp[2], *D2p[2], *Dp[2], *PNMp[2], *DPp[2], *V4p[2], *V5p[2], *DVp[2], *wVp[2];
  float *IMN32p[2], *DMN32p[2], *PNM32p[2], *DP32p[2];
  // precision 3: FP32 tails of those halves (operator = FP32 head + tail)
  float *IMN32lp[2], *DMN32lp[2], *PNM32lp[2], *DP32lp[2];
  double *twx, *twz, *twbx, *twbz;
  double *infl, *state, *Yin, *Zin, *Zout, *Yout, *S, *DN, *Dc, *D2buf, *hgn, *hvn;
  // SBDF4 history: state fields and explicit terms of step k in slot k mod 4
  // of their ring (null for CNAB2)
  double *qring, *hring;
  double *R, *Xs, *Zphi, *Zv, *Zg, *ZDv, *flux, *CB, *prep, *zbuf;
  EigScale* es;
  // mixed precision: FP32 operators, twiddles and padded-grid buffers, FP64
  // mean profiles on the padded grid, the FP64 mean column of the explicit
  // terms there (mcol) and its projection (smean)
  float *IMN32, *DMN32, *PNM32, *DP32, *twx32, *twz32, *Yin32, *Zin32, *Zout32, *Yout32;
  double *Ybar, *mcol, *smean;
  int *zsrc, *zder;
  DiagPart* parts;
  unsigned long long* hist;  // midplane histogram counts (HIST_Q x (HIST_MAX + 2))
  // midplane moments: per line z [HIST_Q][3] partials, running [HIST_Q][3];
  // zgrad (3D): d/dz of u and w on the midplane row, [2][nz][nkx] complex;
  // zgsrc / zgder: the field table of that z transform
  double *mparts, *msum, *zgrad;
  int *zgsrc, *zgder;
  DiagRec* ring;
  DevScalars* sc;
  // G1: state -> padded grid; Gbar: FP64 mean profiles there (mixed);
  // G1b: D2 and D of the state; G2: projection and D of it; Gm: FP64 mean
  // column projection (mixed); G4 / G5: into / out of the eigenbasis (host
  // tables, merged across the batch); H4 / H5: the same for the homogeneous
  // solutions at init (own device tables)
  JobList G1, Gbar, G1b, G2, Gm, G4, G5, H4, H5;
  int prec = 0;
  // arithmetic of the mixed-precision wall-normal products: yv1 for the
  // padded-grid values and d/dy of the state (G1), yv2 for the projections
  // of the explicit terms (G2); Y_FP32, Y_FP64 (FP64 operators, FP32 grid
  // values) or Y_COMP (error-compensated FP32); fixed by precision 1-3,
  // chosen at initialisation for precision 4
  int yv1 = 0, yv2 = 0;
  double wU1 = 0;
  long long drained = 0;
  int blowup = 0;
  double hlo[HIST_Q] = {}, hhi[HIST_Q] = {};  // midplane histogram ranges and bins (0: off)
  int hbins[HIST_Q] = {};
  size_t nstate = 0;
  std::vector<JobList*> stage_lists() { return {&G1, &Gbar, &G1b, &G2, &Gm, &G4, &G5}; }
};

// A batch of simulations advanced together: each stage of the step is one
// launch over all members (merged product tables, per-member argument tables
// of the stage kernels), captured once as a HIP graph.  A single run is a
// batch of one.
struct Batch {
  std::vector<Member*> mem;
  int dim = 2, prec = 0;
  hipStream_t s = nullptr;
  // Products of the state: GS the padded-grid values and derivatives, GSm
  // (mixed) their FP64 mean profiles, GSb the FP64 D2 and D of the state.
  // GP: projections of the explicit terms (mixed: and the FP64 mean column);
  // G4 / G5: solves.  Mixed-precision tables hold FP32 and FP64 products in
  // one launch.
  JobList GS, GSm, GSb, GP, G4, G5;
  // side streams and fork / join events of the captured steps (branches run
  // beside the main chain inside the graphs)
  hipStream_t side[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> evs;
  // side branches of the captured steps: 0 none, 1 the state products and
  // the diagnostics (GSm, GSb hold their own products; else all are in GS),
  // 2 the diagnostics only
  int branch = 0;
  // eager batch (the allocation-free initialisation): no autotuner timing,
  // no side streams, no graphs; every step is launched kernel by kernel
  bool eager = false;
  // precision 4: the error budget, and per table (state products,
  // projections) and variant the measured error and time (-1: not measured)
  double ybudget = -1;
  double yerr[2][3] = {{-1, -1, -1}, {-1, -1, -1}};
  double yus[2][3] = {{-1, -1, -1}, {-1, -1, -1}};
  // per-member argument tables (host copies, then device) and launch sizes
  std::vector<XArgs> hx;
  std::vector<ZArgs> hzi, hzf, hzd;
  std::vector<DRowArgs> hdr;
  std::vector<DFinArgs> hdf;
  std::vector<RhsArgs> hrhs, hrhsw;  // interior rows; wall rows (launched first)
  std::vector<FinArgs> hfin;
  XArgs* dx = nullptr;
  ZArgs *dzi = nullptr, *dzf = nullptr, *dzd = nullptr;
  DRowArgs* ddr = nullptr;
  DFinArgs* ddf = nullptr;
  RhsArgs *drhs = nullptr, *drhsw = nullptr;
  FinArgs* dfin = nullptr;
  int bx = 0, bzi = 0, bzf = 0, bzd = 0, bdr = 0, brhs = 0, brhsw = 0, bfin = 0;
  size_t lx = 0, lzi = 0, lzf = 0, lzd = 0, ldr = 0;
  int xnt = 0;          // threads per x-pencil workgroup
  int zgi = 32, zgd = 32;  // kx columns per workgroup of the state's and the diagnostics' z transforms
  int xchunk = 0;       // 3D lines in field chunks: their common length (xpencil_chunked), else 0
  // one step, and GRAPH_STEPS steps back to back (fewer launches between steps)
  hipGraph_t graph = nullptr, graphn = nullptr;
  hipGraphExec_t gexec = nullptr, gexecn = nullptr;
  std::vector<JobList*> lists() { return {&GS, &GSm, &GSb, &GP, &G4, &G5}; }
  ~Batch() {
    for (hipGraphExec_t e : {gexec, gexecn})
      if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : {graph, graphn})
      if (g) (void)hipGraphDestroy(g);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    for (hipStream_t t : side)
      if (t) (void)hipStreamDestroy(t);
    for (Member* m : mem) delete m;
  }
};

namespace {

// With PCS_DEBUG set in the environment, failing HIP calls are reported on stderr.
void report(hipError_t e, const char* what, int line) {
  static const bool dbg = std::getenv("PCS_DEBUG") != nullptr;
  if (dbg) std::fprintf(stderr, "pcs: %s failed at api.cpp:%d: %s\n", what, line, hipGetErrorString(e));
}

#define HIPCHK(x)                        \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) {              \
      report(e_, #x, __LINE__);          \
      (void)hipGetLastError();           \
      return PCS_ERR_DEVICE;             \
    }                                    \
  } while (0)

// Init-time uploads are blocking copies, so host temporaries may die at once.
template <typename T>
hipError_t up(T* dst, const std::vector<T>& src, hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  return hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

// A product table and its tile map.
hipError_t up_list(JobList* jl, hipStream_t s) {
  hipError_t e = up(jl->dev, jl->h, s);
  return e != hipSuccess ? e : up(jl->tmap, jl->hmap, s);
}

// Assigns every device buffer of one member (a null base only measures).
void carve(Member* m, Carve& c) {
  const Dims& d = m->d;
  const size_t n1 = d.N + 1, m1 = d.M + 1, ni = d.N - 1, cw = d.cw;
  m->IMN = c.take<double>(opsz(m1, n1));
  m->DMN = c.take<double>(opsz(m1, n1));
  m->D = c.take<double>(opsz(n1, n1));
  m->D2 = c.take<double>(opsz(n1, n1));
  m->PNM = c.take<double>(opsz(n1, m1));
  m->DP = c.take<double>(opsz(n1, m1));
  m->V = c.take<double>(opsz(ni, ni));
  m->Vinv = c.take<double>(opsz(ni, ni));
  m->DV = c.take<double>(opsz(n1, ni));
  m->wV = c.take<double>(opsz(1, ni));
  {
    const int mh = (m1 + 1) / 2, nh = (n1 + 1) / 2, ne = (ni + 1) / 2;
    for (int q = 0; q < 2; ++q) {
      m->IMNp[q] = c.take<double>(opsz(mh, nh));
      m->DMNp[q] = c.take<double>(opsz(mh, nh));
      m->D2p[q] = c.take<double>(opsz(nh, nh));
      m->Dp[q] = c.take<double>(opsz(nh, nh));
      m->PNMp[q] = c.take<double>(opsz(nh, mh));
      m->DPp[q] = c.take<double>(opsz(nh, mh));
      m->V4p[q] = c.take<double>(opsz(ne, ne));
      m->V5p[q] = c.take<double>(opsz(ne, ne));
      m->DVp[q] = c.take<double>(opsz(nh, ne));
      m->wVp[q] = c.take<double>(opsz(1, ne));
      m->IMN32p[q] = m->prec != 0 ? c.take<float>(opsz(mh, nh)) : nullptr;
      m->DMN32p[q] = m->prec != 0 ? c.take<float>(opsz(mh, nh)) : nullptr;
      m->PNM32p[q] = m->prec != 0 ? c.take<float>(opsz(nh, mh)) : nullptr;
      m->DP32p[q] = m->prec != 0 ? c.take<float>(opsz(nh, mh)) : nullptr;
      const bool comp = m->prec == 3 || m->prec == 4;
      m->IMN32lp[q] = comp ? c.take<float>(opsz(mh, nh)) : nullptr;
      m->DMN32lp[q] = comp ? c.take<float>(opsz(mh, nh)) : nullptr;
      m->PNM32lp[q] = comp ? c.take<float>(opsz(nh, mh)) : nullptr;
      m->DP32lp[q] = comp ? c.take<float>(opsz(nh, mh)) : nullptr;
    }
  }
  m->lam = c.take<double>(ni);
  m->d2i0 = c.take<double>(ni);
  m->d2in = c.take<double>(ni);
  m->w = c.take<double>(n1);
  m->ydy = c.take<double>(n1);
  m->U1 = c.take<double>(n1);
  m->kx = c.take<double>(d.nkx);
  m->kz = c.take<double>(d.nzs);
  m->twx = c.take<double>(2 * (size_t)d.px);
  m->twz = c.take<double>(2 * (size_t)d.pz);
  m->twbx = c.take<double>(2 * (size_t)d.nx);
  m->twbz = c.take<double>(2 * (size_t)d.nz);
  m->infl = c.take<double>(6 * n1 * d.nm + 4 * (size_t)d.nm);
  m->state = c.take<double>((size_t)(m->nq + m->nh) * n1 * cw);
  m->qring = m->p.scheme == 1 ? c.take<double>((size_t)4 * m->nq * n1 * cw) : nullptr;
  m->hring = m->p.scheme == 1 ? c.take<double>((size_t)4 * m->nh * n1 * cw) : nullptr;
  const size_t zrow = (size_t)m1 * d.pz * d.nkx * 2;
  const bool mixed = m->prec != 0;
  m->Yin = !mixed ? c.take<double>((size_t)m->nyin * m1 * cw) : nullptr;
  m->Zin = (!mixed && d.dim == 3) ? c.take<double>((size_t)m->nzin * zrow) : nullptr;
  m->Zout = (!mixed && d.dim == 3) ? c.take<double>((size_t)m->nout * zrow) : nullptr;
  m->Yout = !mixed ? c.take<double>((size_t)m->nout * m1 * cw) : nullptr;
  m->Yin32 = mixed ? c.take<float>((size_t)m->nyin * m1 * cw) : nullptr;
  m->Zin32 = (mixed && d.dim == 3) ? c.take<float>((size_t)m->nzin * zrow) : nullptr;
  m->Zout32 = (mixed && d.dim == 3) ? c.take<float>((size_t)m->nout * zrow) : nullptr;
  m->Yout32 = mixed ? c.take<float>((size_t)m->nout * m1 * cw) : nullptr;
  m->IMN32 = mixed ? c.take<float>(opsz(m1, n1)) : nullptr;
  m->DMN32 = mixed ? c.take<float>(opsz(m1, n1)) : nullptr;
  m->PNM32 = mixed ? c.take<float>(opsz(n1, m1)) : nullptr;
  m->DP32 = mixed ? c.take<float>(opsz(n1, m1)) : nullptr;
  m->twx32 = mixed ? c.take<float>(2 * (size_t)d.px) : nullptr;
  m->twz32 = mixed ? c.take<float>(2 * (size_t)d.pz) : nullptr;
  m->Ybar = mixed ? c.take<double>(16 * m1) : nullptr;
  m->mcol = mixed ? c.take<double>((size_t)m->nout * m1) : nullptr;
  m->smean = mixed ? c.take<double>((size_t)m->nout * n1) : nullptr;
  m->S = c.take<double>((size_t)m->nout * n1 * cw);
  m->DN = c.take<double>((size_t)(d.dim == 2 ? 1 : 2) * n1 * cw);
  m->Dc = c.take<double>((size_t)d.nc * n1 * cw);
  m->D2buf = c.take<double>((size_t)m->nsolve * n1 * cw + 2 * n1);
  m->hgn = c.take<double>(n1 * cw);
  m->hvn = c.take<double>(n1 * cw);
  m->R = c.take<double>((size_t)m->nsolve * ni * cw);
  m->Xs = c.take<double>((size_t)(m->nsolve + 1) * ni * cw);
  m->es = c.take<EigScale>(1);
  m->Zphi = c.take<double>(ni * cw);
  m->Zv = c.take<double>(ni * cw);
  m->Zg = d.dim == 3 ? c.take<double>(ni * cw) : nullptr;
  m->ZDv = c.take<double>(n1 * cw);
  m->flux = c.take<double>(cw);
  m->CB = c.take<double>((size_t)d.nc * 2 * cw);
  m->prep = c.take<double>(4 * n1 * cw);
  m->zbuf = d.dim == 3 ? c.take<double>(4 * n1 * (size_t)d.nz * d.nkx * 2) : nullptr;
  m->zsrc = c.take<int>(32);
  m->zder = c.take<int>(32);
  const size_t zrows = d.dim == 3 ? d.nz : 1;
  m->parts = c.take<DiagPart>(n1 * zrows);
  m->hist = c.take<unsigned long long>((size_t)HIST_Q * (HIST_MAX + 2));
  m->mparts = c.take<double>(zrows * HIST_Q * 3);
  m->msum = c.take<double>(HIST_Q * 3);
  m->zgrad = d.dim == 3 ? c.take<double>(2 * (size_t)d.nz * d.nkx * 2) : nullptr;
  m->zgsrc = c.take<int>(2);
  m->zgder = c.take<int>(2);
  m->ring = c.take<DiagRec>(RING);
  m->sc = c.take<DevScalars>(1);
}

pcs_status setup_dims(Member* m, const pcs_grid* g, const pcs_params* p) {
  if (!g || !p) return PCS_ERR_ARG;
  if (g->dim != 2 && g->dim != 3) return PCS_ERR_ARG;
  if (g->nx < 4 || (g->nx & 1) || g->ny < 9 || !(g->ny & 1)) return PCS_ERR_UNSUPPORTED;
  if (g->dim == 2 && g->nz != 1) return PCS_ERR_ARG;
  if (g->dim == 3 && (g->nz < 4 || (g->nz & 1))) return PCS_ERR_UNSUPPORTED;
  if (!(g->lx > 0) || (g->dim == 3 && !(g->lz > 0))) return PCS_ERR_ARG;
  if (!(p->re > 0) || !(p->wi > 0) || !(p->beta >= 0 && p->beta <= 1) || !(p->kappa >= 0) || !(p->dt > 0))
    return PCS_ERR_ARG;
  if (p->forcing != 0 && p->forcing != 1) return PCS_ERR_ARG;
  if (p->precision < 0 || p->precision > 4) return PCS_ERR_ARG;
  if (p->scheme != 0 && p->scheme != 1) return PCS_ERR_ARG;
  if (!valid_fft(3 * g->nx / 2) || !valid_fft(g->nx)) return PCS_ERR_UNSUPPORTED;
  if (g->dim == 3 && (!valid_fft(3 * g->nz / 2) || !valid_fft(g->nz))) return PCS_ERR_UNSUPPORTED;
  m->g = *g;
  m->prm = *p;
  Dims& d = m->d;
  d.dim = g->dim;
  d.N = g->ny - 1;
  d.M = 3 * d.N / 2;
  d.nkx = g->nx / 2;
  d.nzs = g->dim == 2 ? 1 : g->nz;
  d.nm = d.nzs * d.nkx;
  d.cw = 2 * d.nm;
  d.px = 3 * g->nx / 2;
  d.pz = g->dim == 2 ? 1 : 3 * g->nz / 2;
  d.nx = g->nx;
  d.nz = g->dim == 2 ? 1 : g->nz;
  d.nc = g->dim == 2 ? 3 : 6;
  d.lx = g->lx;
  d.lz = g->dim == 2 ? 1.0 : g->lz;
  m->prec = p->precision;
  m->yv1 = m->yv2 = m->prec == 4 ? Y_FP64 : m->prec;
  // every transform's working set must fit one workgroup's LDS
  const size_t lds_max = 160 * 1024;
  if (xpencil_lds_bytes(d.dim, d.px, m->prec) > lds_max) return PCS_ERR_UNSUPPORTED;
  if (diag_rows_lds_bytes(d.nx) > 128 * 1024) return PCS_ERR_UNSUPPORTED;
  if (d.dim == 3 && (zfft_lds_bytes(d.pz, m->prec, zfft_group(d.pz, m->prec)) > lds_max ||
                     zfft_lds_bytes(d.nz, 0, zfft_group(d.nz, 0)) > lds_max))
    return PCS_ERR_UNSUPPORTED;
  Phys& q = m->p;
  q.re = p->re;
  q.wi = p->wi;
  q.beta = p->beta;
  q.kappa = p->kappa;
  q.eps = p->eps;
  q.dt = p->dt;
  q.forcing = p->forcing;
  q.q_or_dpdx = p->q_or_dpdx;
  q.coef = (1.0 - p->beta) / (p->re * p->wi);
  q.nu = p->beta / p->re;
  q.scheme = p->scheme;
  q.ia = p->scheme == 0 ? 1.0 / p->dt : (25.0 / 12.0) / p->dt;
  q.th = p->scheme == 0 ? 0.5 : 1.0;
  m->nq = d.dim == 2 ? 6 : 11;
  m->nh = d.dim == 2 ? 4 : 8;
  m->nyin = d.dim == 2 ? 9 : 17;
  m->nzin = 26;
  m->nout = d.dim == 2 ? 5 : 9;
  m->nsv = d.dim == 2 ? 1 : 2;
  m->nsolve = m->nsv + d.nc;
  m->nstate = 4 + (size_t)(m->nq + m->nh + (p->scheme == 1 ? 3 * m->nq + 2 * m->nh : 0)) * (d.N + 1) * d.cw;
  make_plan(d.px, &m->plx);
  make_plan(d.nx, &m->pbx);
  if (d.dim == 3) {
    make_plan(d.pz, &m->plz);
    make_plan(d.nz, &m->pbz);
  }
  return PCS_OK;
}

// Initial state: laminar profiles in the mean slot plus the seeded
// streamfunction perturbation (divergence-free, no-slip), history zero.
void initial_state(const Member* m, uint64_t seed, double amp, std::vector<double>& st) {
  const Dims& d = m->d;
  const int n1 = d.N + 1;
  const size_t fs = (size_t)n1 * d.cw;
  st.assign((size_t)(m->nq + m->nh) * fs, 0.0);
  const double* y = m->ops->y.data();
  std::vector<double> U(n1), cxx(n1), cxy(n1), cyy(n1);
  laminar(y, n1, m->p.wi, m->p.kappa, U.data(), cxx.data(), cxy.data(), cyy.data());
  const int FC = d.dim == 2 ? 3 : 5;
  const int iyy = d.dim == 2 ? 2 : 3;
  for (int j = 0; j < n1; ++j) {
    const size_t o = (size_t)j * d.cw;
    st[0 * fs + o] = U[j];
    st[(FC + 0) * fs + o] = cxx[j];
    st[(FC + 1) * fs + o] = cxy[j];
    st[(FC + iyy) * fs + o] = cyy[j];
    if (d.dim == 3) st[(FC + 5) * fs + o] = cyy[j];
  }
  // basis p_n = (1 - y^2)^2 T_n, n = 0..4, and two derivatives
  std::vector<double> P(5 * n1), P1(5 * n1), P2(5 * n1);
  for (int j = 0; j < n1; ++j) {
    const double yy = y[j], q = 1.0 - yy * yy;
    double T[5], T1[5], T2[5];
    T[0] = 1;
    T1[0] = 0;
    T2[0] = 0;
    T[1] = yy;
    T1[1] = 1;
    T2[1] = 0;
    for (int n = 1; n < 4; ++n) {
      T[n + 1] = 2 * yy * T[n] - T[n - 1];
      T1[n + 1] = 2 * T[n] + 2 * yy * T1[n] - T1[n - 1];
      T2[n + 1] = 4 * T1[n] + 2 * yy * T2[n] - T2[n - 1];
    }
    for (int n = 0; n < 5; ++n) {
      P[n * n1 + j] = q * q * T[n];
      P1[n * n1 + j] = -4.0 * yy * q * T[n] + q * q * T1[n];
      P2[n * n1 + j] = (12.0 * yy * yy - 4.0) * T[n] - 8.0 * yy * q * T1[n] + q * q * T2[n];
    }
  }
  typedef std::complex<double> cx;
  struct Pot {
    std::vector<cx> f, f1, f2;
  };
  std::map<std::tuple<int, int, int>, Pot> pots;  // (potential, mx, mz)
  SplitMix64 rng(seed);
  auto draw = [&](int pot, int mx, int mz) {
    double th[5];
    for (int n = 0; n < 5; ++n) th[n] = 2.0 * M_PI * rng.u01();
    const bool fits = mx < d.nkx && (d.dim == 2 || std::abs(mz) < d.nz / 2);
    if (!fits) return;
    Pot p;
    p.f.assign(n1, 0);
    p.f1.assign(n1, 0);
    p.f2.assign(n1, 0);
    for (int j = 0; j < n1; ++j) {
      cx a(0), a1(0), a2(0);
      for (int n = 0; n < 5; ++n) {
        const cx c(amp * std::cos(th[n]), amp * std::sin(th[n]));
        a += c * P[n * n1 + j];
        a1 += c * P1[n * n1 + j];
        a2 += c * P2[n * n1 + j];
      }
      p.f[j] = a;
      p.f1[j] = a1;
      p.f2[j] = a2;
    }
    pots[std::make_tuple(pot, mx, mz)] = p;
    if (d.dim == 3 && mx == 0) {
      Pot q = p;
      for (int j = 0; j < n1; ++j) {
        q.f[j] = std::conj(p.f[j]);
        q.f1[j] = std::conj(p.f1[j]);
        q.f2[j] = std::conj(p.f2[j]);
      }
      pots[std::make_tuple(pot, 0, -mz)] = q;
    }
  };
  if (d.dim == 2) {
    for (int mx = 1; mx <= 4; ++mx) draw(0, mx, 0);
  } else {
    for (int pot = 0; pot < 2; ++pot)
      for (int mx = 0; mx <= 4; ++mx)
        for (int mz = -4; mz <= 4; ++mz) {
          if ((mx == 0 && mz == 0) || (mx == 0 && mz < 0)) continue;
          draw(pot, mx, mz);
        }
  }
  const int FPHI = d.dim == 2 ? 2 : 3;
  for (int iz = 0; iz < d.nzs; ++iz) {
    if (d.dim == 3 && iz == d.nzs / 2) continue;
    const int mz = d.dim == 2 ? 0 : (iz < d.nzs / 2 ? iz : iz - d.nzs);
    const double kz = d.dim == 2 ? 0.0 : 2.0 * M_PI * mz / d.lz;
    for (int ix = 0; ix < d.nkx; ++ix) {
      if (iz == 0 && ix == 0) continue;
      const double kx = 2.0 * M_PI * ix / d.lx;
      const double k2 = kx * kx + kz * kz;
      auto ip = pots.find(std::make_tuple(0, ix, mz));
      auto ic = pots.find(std::make_tuple(1, ix, mz));
      if (ip == pots.end() && ic == pots.end()) continue;
      const size_t mo = 2 * ((size_t)iz * d.nkx + ix);
      for (int j = 0; j < n1; ++j) {
        const cx zero(0);
        const cx ps = ip != pots.end() ? ip->second.f[j] : zero, ps1 = ip != pots.end() ? ip->second.f1[j] : zero,
                 ps2 = ip != pots.end() ? ip->second.f2[j] : zero;
        const cx ch = ic != pots.end() ? ic->second.f[j] : zero, ch1 = ic != pots.end() ? ic->second.f1[j] : zero,
                 ch2 = ic != pots.end() ? ic->second.f2[j] : zero;
        const cx I(0, 1);
        const cx u = ps1, w = ch1;
        const cx v = -I * kx * ps - I * kz * ch;
        const cx v2 = -I * kx * ps2 - I * kz * ch2;
        const cx phi = v2 - k2 * v;
        const size_t o = (size_t)j * d.cw + mo;
        st[0 * fs + o] = u.real();
        st[0 * fs + o + 1] = u.imag();
        st[1 * fs + o] = v.real();
        st[1 * fs + o + 1] = v.imag();
        st[FPHI * fs + o] = phi.real();
        st[FPHI * fs + o + 1] = phi.imag();
        if (d.dim == 3) {
          const cx g = I * kz * u - I * kx * w;
          st[2 * fs + o] = w.real();
          st[2 * fs + o + 1] = w.imag();
          st[4 * fs + o] = g.real();
          st[4 * fs + o + 1] = g.imag();
        }
      }
    }
  }
}

void build_jobs(Member* m) {
  const Dims& d = m->d;
  const int n1 = d.N + 1, m1 = d.M + 1, ni = d.N - 1, cw = d.cw;
  const size_t fs = (size_t)n1 * cw, fsm = (size_t)m1 * cw, fsi = (size_t)ni * cw;
  double* st = m->state;
  const int FC = d.dim == 2 ? 3 : 5, FPHI = d.dim == 2 ? 2 : 3;
  const bool mixed = m->prec != 0;
  for (JobList* jl : m->stage_lists()) jl->clear();
  m->H4.clear();
  m->H5.clear();
  // G1: values and d/dy on the padded grid (mixed: of the fluctuation only,
  // written in FP32; computed in FP32, or in FP64 for precision 2)
  // The wide products are parity products (operator halves of the even and
  // odd parts): half rows mh / nh, half columns nh / mh, ne eigen pairs.
  const int mh = (m1 + 1) / 2, nh = (n1 + 1) / 2, ne = (ni + 1) / 2;  // ne: even eigenvectors
  JobList& g1 = m->G1;
  // variant yv1: FP32, FP64, or error-compensated FP32 (FP32 operator
  // heads and tails, parity form only)
  g1.type = mixed ? (m->yv1 == Y_FP64 ? GEMM_DDF : (m->yv1 == Y_COMP ? GEMM_CDF : GEMM_FDF)) : GEMM_DDD;
  const bool f32ops = mixed && m->yv1 != Y_FP64;
  const void* I = f32ops ? (const void*)m->IMN32 : (const void*)m->IMN;
  const void* DI = f32ops ? (const void*)m->DMN32 : (const void*)m->DMN;
  const void* Ip[2] = {f32ops ? (const void*)m->IMN32p[0] : m->IMNp[0], f32ops ? (const void*)m->IMN32p[1] : m->IMNp[1]};
  const void* DIp[2] = {f32ops ? (const void*)m->DMN32p[0] : m->DMNp[0], f32ops ? (const void*)m->DMN32p[1] : m->DMNp[1]};
  void* Y = mixed ? (void*)m->Yin32 : (void*)m->Yin;
  const size_t ysz = mixed ? sizeof(float) : sizeof(double);
  auto yf = [&](int f) { return (void*)((char*)Y + (size_t)f * fsm * ysz); };
  const int zm = mixed ? GEMM_ZERO_MEAN : 0;
  const int nvel = d.dim;
  // values (centrosymmetric operator) and d/dy (centro-antisymmetric) on the padded grid
  auto tails = [&](JobList& jl, float* const (&lo)[2]) {
    if (gemm_type_comp(jl.type)) {
      jl.forms[1].back().Alo = lo[0];
      jl.forms[1].back().A2lo = lo[1];
    }
  };
  auto val = [&](const double* src, void* dst) {
    g1.addp(PAR_FOLD_UNFOLD, I, Ip[0], Ip[1], src, cw, dst, cw, mh, cw, nh, m1, n1, +1, zm);
    tails(g1, m->IMN32lp);
  };
  auto dy = [&](const double* src, void* dst) {
    g1.addp(PAR_FOLD_UNFOLD, DI, DIp[0], DIp[1], src, cw, dst, cw, mh, cw, nh, m1, n1, -1, zm);
    tails(g1, m->DMN32lp);
  };
  // padded-grid inputs: values of u v (w) c, then d/dy of u (w) c; the
  // products are listed with the values and d/dy of one field adjacent, so
  // that they share a staged panel (mark_pairs)
  const int yd0 = nvel + d.nc;  // first d/dy field in the padded-grid input
  val(st + 0 * fs, yf(0));
  dy(st + 0 * fs, yf(yd0));
  val(st + 1 * fs, yf(1));
  if (d.dim == 3) {
    val(st + 2 * fs, yf(2));
    dy(st + 2 * fs, yf(yd0 + 1));
  }
  const int ydc = yd0 + (d.dim == 3 ? 2 : 1);  // first d/dy of c
  for (int a = 0; a < d.nc; ++a) {
    val(st + (FC + a) * fs, yf(nvel + a));
    dy(st + (FC + a) * fs, yf(ydc + a));
  }
  g1.mark_pairs();
  if (mixed) {
    // FP64 mean profiles on the padded grid (real part of the kx = kz = 0 column)
    // 2D: U U' c (3) c' (3); 3D: U W U' W' c (6) c' (6)
    JobList& gb = m->Gbar;
    gb.type = GEMM_DDD;
    double* Yb = m->Ybar;
    int q = 0;
    auto mval = [&](const double* src) {
      gb.addp(PAR_FOLD_UNFOLD, m->IMN, m->IMNp[0], m->IMNp[1], src, cw, Yb + (q++) * m1, 1, mh, 1, nh, m1, n1, +1);
    };
    auto mdy = [&](const double* src) {
      gb.addp(PAR_FOLD_UNFOLD, m->DMN, m->DMNp[0], m->DMNp[1], src, cw, Yb + (q++) * m1, 1, mh, 1, nh, m1, n1, -1);
    };
    mval(st + 0 * fs);
    if (d.dim == 3) mval(st + 2 * fs);
    mdy(st + 0 * fs);
    if (d.dim == 3) mdy(st + 2 * fs);
    for (int a = 0; a < d.nc; ++a) mval(st + (FC + a) * fs);
    for (int a = 0; a < d.nc; ++a) mdy(st + (FC + a) * fs);
  }
  // G1b (FP64): D2 of phi, (g), c and of the mean U, (W); D of every c
  JobList& g1b = m->G1b;
  g1b.type = GEMM_DDD;
  auto d2 = [&](const double* src, double* dst) {
    g1b.addp(PAR_FOLD_UNFOLD, m->D2, m->D2p[0], m->D2p[1], src, cw, dst, cw, nh, cw, nh, n1, n1, +1);
  };
  // SBDF4 has no explicit half of the linear terms: of these it reads only
  // D2 c_xy (and D2 c_yz in 3D), inside the stress divergence
  const bool cn = m->p.scheme == 0;
  auto stress_d2 = [&](int a) { return a == 1 || (d.dim == 3 && a == 4); };
  if (cn) d2(st + FPHI * fs, m->D2buf + 0 * fs);
  if (cn && d.dim == 3) d2(st + 4 * fs, m->D2buf + 1 * fs);
  // D2 and D of each c adjacent (one staged panel, mark_pairs)
  for (int a = 0; a < d.nc; ++a) {
    if (cn || stress_d2(a)) d2(st + (FC + a) * fs, m->D2buf + (m->nsv + a) * fs);
    g1b.addp(PAR_FOLD_UNFOLD, m->D, m->Dp[0], m->Dp[1], st + (FC + a) * fs, cw, m->Dc + a * fs, cw, nh, cw, nh, n1, n1,
             -1);
  }
  double* D2U = m->D2buf + (size_t)m->nsolve * fs;
  if (cn) g1b.addp(PAR_FOLD_UNFOLD, m->D2, m->D2p[0], m->D2p[1], st + 0 * fs, cw, D2U, 1, nh, 1, nh, n1, n1, +1);
  if (cn && d.dim == 3)
    g1b.addp(PAR_FOLD_UNFOLD, m->D2, m->D2p[0], m->D2p[1], st + 2 * fs, cw, D2U + n1, 1, nh, 1, nh, n1, n1, +1);
  g1b.mark_pairs();
  // G2: projection of the explicit terms, and D of the projected N_x, N_z
  // through (D P) (mixed: FP32 operands, FP64 result)
  m->G2.type = mixed ? (m->yv2 == Y_FP64 ? GEMM_DFD : (m->yv2 == Y_COMP ? GEMM_CFD : GEMM_FFD)) : GEMM_DDD;
  const bool f32ops2 = mixed && m->yv2 != Y_FP64;
  const void* P = f32ops2 ? (const void*)m->PNM32 : (const void*)m->PNM;  // (plain form; not used by Y_COMP)
  const void* DP = f32ops2 ? (const void*)m->DP32 : (const void*)m->DP;
  const void* Pp[2] = {f32ops2 ? (const void*)m->PNM32p[0] : m->PNMp[0],
                       f32ops2 ? (const void*)m->PNM32p[1] : m->PNMp[1]};
  const void* DPp[2] = {f32ops2 ? (const void*)m->DP32p[0] : m->DPp[0], f32ops2 ? (const void*)m->DP32p[1] : m->DPp[1]};
  const char* Yo = mixed ? (const char*)m->Yout32 : (const char*)m->Yout;
  // P N of every explicit term, with D P N_x (and D P N_z) beside the P N
  // of the same term (one staged panel, mark_pairs)
  for (int f = 0; f < m->nout; ++f) {
    m->G2.addp(PAR_FOLD_UNFOLD, P, Pp[0], Pp[1], Yo + (size_t)f * fsm * ysz, cw, m->S + f * fs, cw, nh, cw, mh, n1, m1,
               +1);
    tails(m->G2, m->PNM32lp);
    if (f == 0 || (f == 2 && d.dim == 3)) {
      m->G2.addp(PAR_FOLD_UNFOLD, DP, DPp[0], DPp[1], Yo + (size_t)f * fsm * ysz, cw, m->DN + (f / 2) * fs, cw, nh, cw,
                 mh, n1, m1, -1);
      tails(m->G2, m->DP32lp);
    }
  }
  m->G2.mark_pairs();
  if (mixed) {
    // the mean column again, in FP64, from the FP64-completed padded-grid means
    m->Gm.type = GEMM_DDD;
    for (int f = 0; f < m->nout; ++f)
      m->Gm.addp(PAR_FOLD_UNFOLD, m->PNM, m->PNMp[0], m->PNMp[1], m->mcol + (size_t)f * m1, 1, m->smean + f * n1, 1, nh,
                 1, mh, n1, m1, +1);
  }
  // G4: V^-1 R, written scaled by the inverse Helmholtz symbols into
  // Xs = [phi, v, (g), c...] (phi's coefficients give v's as a second output)
  const EigScale* es = m->es;
  double* Xs = m->Xs;
  // (eigen coefficients of the even part in rows [0, ne), of the odd part after)
  auto vinv = [&](JobList& jl, const double* src, double* dst, int scale, double* dst2, int scale2) {
    jl.addp(PAR_FOLD_SPLIT, m->Vinv, m->V4p[0], m->V4p[1], src, cw, dst, cw, ne, cw, ne, ni, ni, +1, 0, scale, es, dst2,
            scale2);
  };
  for (JobList* jl : {&m->G4, &m->H4}) vinv(*jl, m->R, Xs, SCALE_PHI, Xs + fsi, SCALE_V);
  if (d.dim == 3) vinv(m->G4, m->R + fsi, Xs + 2 * fsi, SCALE_PHI, nullptr, SCALE_NONE);
  const int xo = d.dim == 3 ? 3 : 2;
  for (int a = 0; a < d.nc; ++a)
    vinv(m->G4, m->R + (m->nsv + a) * fsi, Xs + (xo + a) * fsi, SCALE_C, nullptr, SCALE_NONE);
  // G5: back from the eigenbasis
  auto vmul = [&](JobList& jl, const double* src, double* dst) {
    jl.addp(PAR_SPLIT_UNFOLD, m->V, m->V5p[0], m->V5p[1], src, cw, dst, cw, ne, cw, ne, ni, ni, +1);
  };
  for (JobList* jl : {&m->G5, &m->H5}) {
    vmul(*jl, Xs, m->Zphi);
    vmul(*jl, Xs + fsi, m->Zv);
    jl->addp(PAR_SPLIT_UNFOLD, m->DV, m->DVp[0], m->DVp[1], Xs + fsi, cw, m->ZDv, cw, nh, cw, ne, n1, ni, -1);
  }
  if (d.dim == 3) vmul(m->G5, Xs + 2 * fsi, m->Zg);
  for (int a = 0; a < d.nc; ++a) vmul(m->G5, Xs + (xo + a) * fsi, st + (FC + a) * fs + cw);
  // w . U_p for the flux constraint: the mean column only (w V split like V)
  m->G5.addp(PAR_SPLIT_UNFOLD, m->wV, m->wVp[0], m->wVp[1], Xs, cw, m->flux, cw, 1, 2, ne, 1, ni, +1);
  // a run whose blow-up flag is set is masked: its products are skipped
  const int* skip = m->sc ? &m->sc->blowup : nullptr;
  for (JobList* jl : m->stage_lists())
    for (int f = 0; f < 2; ++f)
      for (GemmJob& j : jl->forms[f]) j.skip = skip;
  for (JobList* jl : {&m->H4, &m->H5}) jl->prepare();
}

pcs_status upload_member(Member* m, uint64_t seed, double amp, hipStream_t s) {
  const Dims& d = m->d;
  const WallOps* op = m->ops;
  const int n1 = d.N + 1, ni = d.N - 1;
  // operators
  const int m1 = d.M + 1;
  HIPCHK(up(m->IMN, padded(op->IMN, m1, n1), s));
  HIPCHK(up(m->DMN, padded(op->DMN, m1, n1), s));
  HIPCHK(up(m->D, padded(op->D, n1, n1), s));
  HIPCHK(up(m->D2, padded(op->D2, n1, n1), s));
  HIPCHK(up(m->PNM, padded(op->PNM, n1, m1), s));
  // D P: derivative of a projected field straight from the padded grid
  std::vector<double> DP((size_t)n1 * m1);
  for (int i = 0; i < n1; ++i)
    for (int k = 0; k < m1; ++k) {
      long double acc = 0;
      for (int j = 0; j < n1; ++j) acc += (long double)op->D[(size_t)i * n1 + j] * op->PNM[(size_t)j * m1 + k];
      DP[(size_t)i * m1 + k] = (double)acc;
    }
  HIPCHK(up(m->DP, padded(DP, n1, m1), s));
  HIPCHK(up(m->V, padded(op->V, ni, ni), s));
  HIPCHK(up(m->Vinv, padded(op->Vinv, ni, ni), s));
  HIPCHK(up(m->lam, op->lam, s));
  HIPCHK(up(m->d2i0, op->d2_i0, s));
  HIPCHK(up(m->d2in, op->d2_in, s));
  HIPCHK(up(m->w, op->w, s));
  // D restricted to interior columns times V, and w (interior) times V
  std::vector<double> DV((size_t)n1 * ni, 0.0), wV(ni, 0.0);
  for (int i = 0; i < n1; ++i)
    for (int e = 0; e < ni; ++e) {
      long double acc = 0;
      for (int j = 1; j < d.N; ++j) acc += (long double)op->D[(size_t)i * n1 + j] * op->V[(size_t)(j - 1) * ni + e];
      DV[(size_t)i * ni + e] = (double)acc;
    }
  for (int e = 0; e < ni; ++e) {
    long double acc = 0;
    for (int j = 1; j < d.N; ++j) acc += (long double)op->w[j] * op->V[(size_t)(j - 1) * ni + e];
    wV[e] = (double)acc;
  }
  HIPCHK(up(m->DV, padded(DV, n1, ni), s));
  HIPCHK(up(m->wV, padded(wV, 1, ni), s));
  {
    // parity halves (the eigenvectors are even first, then odd)
    const int mh = (m1 + 1) / 2, nh = (n1 + 1) / 2, ne = op->ne, no = op->no;
    std::vector<double> e, o;
    auto put2 = [&](double* const (&dst)[2], int rows, int cols) -> hipError_t {
      hipError_t r = up(dst[0], padded(e, rows, cols), s);
      return r != hipSuccess ? r : up(dst[1], padded(o, rows, cols), s);
    };
    auto put2f = [&](float* const (&dst)[2], int rows, int cols) -> hipError_t {
      hipError_t r = up(dst[0], padded<float>(e, rows, cols), s);
      return r != hipSuccess ? r : up(dst[1], padded<float>(o, rows, cols), s);
    };
    const bool mixed = m->prec != 0;
    // FP32 tails of the halves (precisions 3 and 4): v - fp32(v), rounded to FP32
    auto put2t = [&](float* const (&dst)[2], int rows, int cols) -> hipError_t {
      if (m->prec != 3 && m->prec != 4) return hipSuccess;
      std::vector<double> te(e.size()), to(o.size());
      for (size_t i = 0; i < e.size(); ++i) te[i] = e[i] - (double)(float)e[i];
      for (size_t i = 0; i < o.size(); ++i) to[i] = o[i] - (double)(float)o[i];
      hipError_t r = up(dst[0], padded<float>(te, rows, cols), s);
      return r != hipSuccess ? r : up(dst[1], padded<float>(to, rows, cols), s);
    };
    fold(op->IMN, n1, 0, mh, mh, e, o);
    HIPCHK(put2(m->IMNp, mh, nh));
    if (mixed) HIPCHK(put2f(m->IMN32p, mh, nh));
    HIPCHK(put2t(m->IMN32lp, mh, nh));
    fold(op->DMN, n1, 0, mh, mh, e, o);
    HIPCHK(put2(m->DMNp, mh, nh));
    if (mixed) HIPCHK(put2f(m->DMN32p, mh, nh));
    HIPCHK(put2t(m->DMN32lp, mh, nh));
    fold(op->D2, n1, 0, nh, nh, e, o);
    HIPCHK(put2(m->D2p, nh, nh));
    fold(op->D, n1, 0, nh, nh, e, o);
    HIPCHK(put2(m->Dp, nh, nh));
    fold(op->PNM, m1, 0, nh, nh, e, o);
    HIPCHK(put2(m->PNMp, nh, mh));
    if (mixed) HIPCHK(put2f(m->PNM32p, nh, mh));
    HIPCHK(put2t(m->PNM32lp, nh, mh));
    fold(DP, m1, 0, nh, nh, e, o);
    HIPCHK(put2(m->DPp, nh, mh));
    if (mixed) HIPCHK(put2f(m->DP32p, nh, mh));
    HIPCHK(put2t(m->DP32lp, nh, mh));
    // V^-1: even rows act on the folded sums, odd rows on the differences
    std::vector<double> e2, o2;
    fold(op->Vinv, ni, 0, ne, ne, e, o2);
    fold(op->Vinv, ni, ne, no, ne, e2, o);
    HIPCHK(put2(m->V4p, ne, ne));
    // V and D V: first half of the rows, even and odd eigenvector columns
    e = block(op->V, ni, ne, 0, ne, ne);
    o = block(op->V, ni, ne, ne, no, ne);
    HIPCHK(put2(m->V5p, ne, ne));
    e = block(DV, ni, nh, 0, ne, ne);
    o = block(DV, ni, nh, ne, no, ne);
    HIPCHK(put2(m->DVp, nh, ne));
    e = block(wV, ni, 1, 0, ne, ne);
    o = block(wV, ni, 1, ne, no, ne);
    HIPCHK(put2(m->wVp, 1, ne));
  }
  std::vector<double> ydy(n1);
  const double* y = op->y.data();
  for (int j = 1; j < d.N; ++j) ydy[j] = 0.5 * (y[j - 1] - y[j + 1]);
  ydy[0] = y[0] - y[1];
  ydy[d.N] = y[d.N - 1] - y[d.N];
  HIPCHK(up(m->ydy, ydy, s));
  std::vector<double> kx(d.nkx), kz(d.nzs, 0.0);
  for (int i = 0; i < d.nkx; ++i) kx[i] = 2.0 * M_PI * i / d.lx;
  if (d.dim == 3)
    for (int i = 0; i < d.nzs; ++i) {
      const int mz = (i < d.nzs / 2) ? i : (i == d.nzs / 2 ? 0 : i - d.nzs);
      kz[i] = 2.0 * M_PI * mz / d.lz;
    }
  HIPCHK(up(m->kx, kx, s));
  HIPCHK(up(m->kz, kz, s));
  EigScale es{};
  es.lam = m->lam;
  es.kx = m->kx;
  es.kz = m->kz;
  es.nkx = d.nkx;
  es.dim = d.dim;
  es.ia = m->p.ia;
  es.th = m->p.th;
  es.nu = m->p.nu;
  es.wi = m->p.wi;
  es.kappa = m->p.kappa;
  HIPCHK(up(m->es, std::vector<EigScale>{es}, s));
  HIPCHK(up(m->twx, twiddles(d.px, -1), s));
  HIPCHK(up(m->twbx, twiddles(d.nx, -1), s));
  if (m->prec != 0) {
    HIPCHK(up(m->IMN32, padded<float>(op->IMN, m1, n1), s));
    HIPCHK(up(m->DMN32, padded<float>(op->DMN, m1, n1), s));
    HIPCHK(up(m->PNM32, padded<float>(op->PNM, n1, m1), s));
    HIPCHK(up(m->DP32, padded<float>(DP, n1, m1), s));
    auto tf = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
    HIPCHK(up(m->twx32, tf(twiddles(d.px, -1)), s));
    if (d.dim == 3) HIPCHK(up(m->twz32, tf(twiddles(d.pz, -1)), s));
  }
  if (d.dim == 3) {
    HIPCHK(up(m->twz, twiddles(d.pz, -1), s));
    HIPCHK(up(m->twbz, twiddles(d.nz, -1), s));
    // z-transform input table: the 17 y-transformed fields, then d/dz of u v w c6
    // (fields 17 + k = d/dz of field k < ZPAIRS, the pairing the kernel's block order takes)
    std::vector<int> src(26), der(26);
    for (int f = 0; f < 17; ++f) {
      src[f] = f;
      der[f] = 0;
    }
    for (int f = 0; f < ZPAIRS; ++f) {
      src[17 + f] = f;
      der[17 + f] = 1;
    }
    HIPCHK(up(m->zsrc, src, s));
    HIPCHK(up(m->zder, der, s));
    // midplane d/dz of u (field 1 of the diagnostics inputs) and w (field 3)
    HIPCHK(up(m->zgsrc, std::vector<int>{1 * (d.N + 1), 3 * (d.N + 1)}, s));
    HIPCHK(up(m->zgder, std::vector<int>{1, 1}, s));
  }
  // initial state
  std::vector<double> st;
  initial_state(m, seed, amp, st);
  HIPCHK(up(m->state, st, s));
  DevScalars sc0{};
  sc0.pi = m->p.forcing == 1 ? m->p.q_or_dpdx : 2.0 / m->p.re;
  HIPCHK(hipMemcpy(m->sc, &sc0, sizeof(sc0), hipMemcpyHostToDevice));
  // the member's own product tables (homogeneous solutions at init)
  HIPCHK(up_list(&m->H4, s));
  HIPCHK(up_list(&m->H5, s));
  return PCS_OK;
}

// Initial state and device scalars (again after tuning, whose timing launches
// write into the state's solve targets).
pcs_status reset_state(Member* m, uint64_t seed, double amp, hipStream_t s) {
  std::vector<double> st;
  initial_state(m, seed, amp, st);
  HIPCHK(up(m->state, st, s));
  DevScalars sc0{};
  sc0.pi = m->p.forcing == 1 ? m->p.q_or_dpdx : 2.0 / m->p.re;
  HIPCHK(hipMemcpy(m->sc, &sc0, sizeof(sc0), hipMemcpyHostToDevice));
  return PCS_OK;
}

// Side branches of the captured steps (0, 1 or 2, as Batch::branch):
// cross-queue edges of a graph cost several microseconds each (measured
// 5-12 us on the main chain), which the overlap repays only for steps of
// enough work; here both branches from about a million padded-grid points
// per step (a 3D or an ensemble step), none below (one 2D channel of
// 256 x 257 measured 9240 steps/s without, 9028 with the diagnostics branch
// alone, 8488 with both).  PCS_GRAPH_BRANCHES=0, 1 or 2 forces the choice.
int use_branches(const Batch* b) {
  if (const char* e = std::getenv("PCS_GRAPH_BRANCHES")) {
    const int v = std::atoi(e);
    return v >= 0 && v <= 2 ? v : 0;
  }
  double pts = 0;
  for (const Member* m : b->mem) pts += (double)(m->d.M + 1) * m->d.px * m->d.pz;
  return pts >= (double)(1 << 20) ? 1 : 0;
}

// Merges the members' tables of the given stages into one batch table (in
// that order; the table's type is the first non-FP64 type among them).
void merge_list(JobList& dst, const std::vector<Member*>& mem, std::initializer_list<JobList Member::*> lps) {
  dst.clear();
  dst.type = GEMM_DDD;
  for (JobList Member::*lp : lps)
    for (Member* m : mem) {
      const JobList& src = m->*lp;
      if (src.n() && src.type != GEMM_DDD && dst.type == GEMM_DDD) dst.type = src.type;
      for (int f = 0; f < 2; ++f) dst.forms[f].insert(dst.forms[f].end(), src.forms[f].begin(), src.forms[f].end());
    }
  dst.use(0);
  if (dst.n()) dst.prepare();
}

// Builds the merged product tables, the per-member argument tables of the
// stage kernels and the launch sizes (workgroups, LDS) of every stage.
void build_batch(Batch* b) {
  const std::vector<Member*>& mem = b->mem;
  // with side branches the mean and D2 / D products get launches of their
  // own; else one launch holds every product of the state (the single-column
  // mean products first: their short tiles start early)
  b->branch = use_branches(b);
  if (b->branch == 1) {
    merge_list(b->GS, mem, {&Member::G1});
    merge_list(b->GSm, mem, {&Member::Gbar});
    merge_list(b->GSb, mem, {&Member::G1b});
  } else {
    merge_list(b->GS, mem, {&Member::Gbar, &Member::G1, &Member::G1b});
    merge_list(b->GSm, mem, {});
    merge_list(b->GSb, mem, {});
  }
  merge_list(b->GP, mem, {&Member::Gm, &Member::G2});
  merge_list(b->G4, mem, {&Member::G4});
  merge_list(b->G5, mem, {&Member::G5});
  b->hx.clear();
  b->hzi.clear();
  b->hzf.clear();
  b->hzd.clear();
  b->hdr.clear();
  b->hdf.clear();
  b->hrhs.clear();
  b->hrhsw.clear();
  b->hfin.clear();
  b->bx = b->bzi = b->bzf = b->bzd = b->bdr = b->brhs = b->brhsw = b->bfin = 0;
  b->lx = b->lzi = b->lzf = b->lzd = b->ldr = 0;
  // one column group per z-transform launch: the smallest any member's length asks for
  b->zgi = b->zgd = 32;
  for (Member* m : mem)
    if (m->d.dim == 3) {
      b->zgi = std::min(b->zgi, zfft_group(m->d.pz, m->prec));
      b->zgd = std::min(b->zgd, zfft_group(m->d.nz, 0));
    }
  b->xchunk = mem[0]->d.px;
  for (Member* m : mem)
    if (!xpencil_chunked(m->d.dim, m->d.px, m->prec) || m->d.px != mem[0]->d.px) b->xchunk = 0;
  // right-hand sides: wall rows first, then the interior rows reading their
  // new wall values, where the launch is large enough for the re-read wall rows
  // to cost more than the second launch's latency (measured: 3D 256 x 257 x 128
  // 0.79 -> 0.72 ms, 128 x 129 x 64 0.117 -> 0.106 ms; 2D 256 x 257, 33K
  // elements, 13 -> 17 us); else one launch whose threads recompute them
  size_t rhs_elems = 0;
  for (Member* m : mem) rhs_elems += (size_t)(m->d.N + 1) * m->d.nm;
  bool rhs_split = rhs_elems >= RHS_SPLIT_ELEMS;
  // PCS_RHS_FORM=split or =fused forces a form (both give the same arithmetic)
  if (const char* e = std::getenv("PCS_RHS_FORM")) {
    if (!std::strcmp(e, "split")) rhs_split = true;
    if (!std::strcmp(e, "fused")) rhs_split = false;
  }
  for (Member* m : mem) {
    const Dims& d = m->d;
    const bool mixed = m->prec != 0;
    const int n1 = d.N + 1, m1 = d.M + 1;
    const void* twx = mixed ? (const void*)m->twx32 : (const void*)m->twx;
    const void* twz = mixed ? (const void*)m->twz32 : (const void*)m->twz;
    void* yin = mixed ? (void*)m->Yin32 : (void*)m->Yin;
    void* yout = mixed ? (void*)m->Yout32 : (void*)m->Yout;
    void* zin = mixed ? (void*)m->Zin32 : (void*)m->Zin;
    void* zout = mixed ? (void*)m->Zout32 : (void*)m->Zout;
    XArgs x{};
    x.in = d.dim == 3 ? zin : yin;
    x.out = d.dim == 3 ? zout : yout;
    x.nrows = xpencil_blocks(d);
    x.nkx = d.nkx;
    x.m1 = m1;
    x.pz = d.pz;
    x.pl = m->plx;
    x.kx = m->kx;
    x.tw = twx;
    x.eps_wi = m->p.eps / m->p.wi;
    x.mean = m->Ybar;
    x.mcol = d.dim == 2 ? m->mcol : nullptr;
    const int* skip = m->sc ? &m->sc->blowup : nullptr;  // the run's blow-up flag masks its work
    x.skip = skip;
    x.blk0 = b->bx;
    b->bx += x.nrows;
    b->lx = std::max(b->lx, xpencil_lds_bytes(d.dim, d.px, m->prec, b->xchunk > 0));
    b->hx.push_back(x);
    if (d.dim == 3) {
      // the state transforms run in the member's precision, the diagnostics' in FP64
      const int ngx = (d.nkx + b->zgi - 1) / b->zgi;
      const int ngd = (d.nkx + b->zgd - 1) / b->zgd;
      ZArgs zi{};
      zi.in = yin;
      zi.out = zin;
      zi.nkx = d.nkx;
      zi.nzs = d.nzs;
      zi.rows = m1;
      zi.nfields = m->nzin;
      zi.ngx = ngx;
      zi.inverse = 1;
      zi.pl = m->plz;
      zi.src_field = m->zsrc;
      zi.deriv = m->zder;
      zi.npair = ZPAIRS;
      zi.kz = m->kz;
      zi.tw = twz;
      zi.skip = skip;
      zi.blk0 = b->bzi;
      b->bzi += zfft_blocks(d.nkx, m1, m->nzin, b->zgi);
      b->lzi = std::max(b->lzi, zfft_lds_bytes(d.pz, m->prec, b->zgi));
      b->hzi.push_back(zi);
      ZArgs zf = zi;
      zf.in = zout;
      zf.out = yout;
      zf.nfields = m->nout;
      zf.inverse = 0;
      zf.src_field = nullptr;
      zf.deriv = nullptr;
      zf.npair = 0;
      zf.mean = m->Ybar;
      zf.mcol = m->mcol;
      zf.eps_wi = m->p.eps / m->p.wi;
      zf.blk0 = b->bzf;
      b->bzf += zfft_blocks(d.nkx, m1, m->nout, b->zgi);
      b->lzf = std::max(b->lzf, zfft_lds_bytes(d.pz, m->prec, b->zgi));
      b->hzf.push_back(zf);
      ZArgs zd{};
      zd.in = m->prep;
      zd.out = m->zbuf;
      zd.nkx = d.nkx;
      zd.nzs = d.nzs;
      zd.rows = n1;
      zd.nfields = 4;
      zd.ngx = ngd;
      zd.inverse = 1;
      zd.pl = m->pbz;
      zd.tw = m->twbz;
      zd.skip = skip;
      zd.blk0 = b->bzd;
      b->bzd += zfft_blocks(d.nkx, n1, 4, b->zgd);
      b->lzd = std::max(b->lzd, zfft_lds_bytes(d.nz, 0, b->zgd));
      b->hzd.push_back(zd);
      // d/dz of u and w on the midplane row (the velocity-gradient PDFs): the
      // same launch, one row, fields picked by whole-field offsets from that row
      ZArgs zg = zd;
      zg.in = m->prep + (size_t)(d.N / 2) * d.cw;
      zg.out = m->zgrad;
      zg.rows = 1;
      zg.nfields = 2;
      zg.src_field = m->zgsrc;
      zg.deriv = m->zgder;
      zg.kz = m->kz;
      zg.blk0 = b->bzd;
      b->bzd += zfft_blocks(d.nkx, 1, 2, b->zgd);
      b->hzd.push_back(zg);
    }
    DRowArgs r{};
    r.d = d;
    r.in = d.dim == 3 ? m->zbuf : m->prep;
    r.zrows = d.dim == 3 ? d.nz : 1;
    r.pl = m->pbx;
    r.tw = m->twbx;
    r.ydy = m->ydy;
    r.kx = m->kx;
    r.parts = m->parts;
    r.hist = m->hist;
    r.zgrad = m->zgrad;
    r.mparts = m->mparts;
    for (int q = 0; q < HIST_Q; ++q) {
      r.hbins[q] = m->hbins[q];
      r.hlo[q] = m->hlo[q];
      r.hscale[q] = m->hbins[q] > 0 ? m->hbins[q] / (m->hhi[q] - m->hlo[q]) : 0.0;
    }
    // mean-mode u and w at the midplane row: the kx = kz = 0 slot of the
    // diagnostics inputs [Tr c, u, v, w] at j = N/2
    r.umean = m->prep + (size_t)1 * n1 * d.cw + (size_t)(d.N / 2) * d.cw;
    r.wmean = d.dim == 3 ? m->prep + (size_t)3 * n1 * d.cw + (size_t)(d.N / 2) * d.cw : nullptr;
    r.skip = skip;
    r.blk0 = b->bdr;
    b->bdr += n1 * r.zrows;
    b->ldr = std::max(b->ldr, diag_rows_lds_bytes(d.nx));
    b->hdr.push_back(r);
    DFinArgs f{};
    f.d = d;
    f.p = m->p;
    f.parts = m->parts;
    f.zrows = r.zrows;
    f.w = m->w;
    f.sc = m->sc;
    f.ring = m->ring;
    f.cap = RING;
    f.mparts = m->mparts;
    f.msum = m->msum;
    f.mom_mask = 0;
    for (int q = 0; q < HIST_Q; ++q)
      if (m->hbins[q] > 0) f.mom_mask |= 1 << q;
    b->hdf.push_back(f);
    const int eblocks = (n1 * d.nm + ELEM_THREADS - 1) / ELEM_THREADS;
    RhsArgs h{};
    h.d = d;
    h.p = m->p;
    h.st = m->state;
    h.D2buf = m->D2buf;
    h.Dc = m->Dc;
    h.S = m->S;
    h.smean = m->smean;
    h.DN = m->DN;
    h.kx = m->kx;
    h.kz = m->kz;
    h.d2i0 = m->d2i0;
    h.d2in = m->d2in;
    h.R = m->R;
    h.hvn = m->hvn;
    h.hgn = m->hgn;
    h.CB = m->CB;
    h.qring = m->qring;
    h.hring = m->hring;
    h.sc = m->sc;
    if (rhs_split) {
      h.blk0 = b->brhsw;
      b->brhsw += (2 * d.nm + ELEM_THREADS - 1) / ELEM_THREADS;
      b->hrhsw.push_back(h);
    }
    h.blk0 = b->brhs;
    b->brhs += ((rhs_split ? n1 - 2 : n1) * d.nm + ELEM_THREADS - 1) / ELEM_THREADS;
    b->hrhs.push_back(h);
    FinArgs q{};
    q.d = d;
    q.p = m->p;
    q.Zphi = m->Zphi;
    q.Zv = m->Zv;
    q.Zg = m->Zg;
    q.ZDv = m->ZDv;
    q.flux = m->flux;
    q.infl = m->infl;
    q.U1 = m->U1;
    q.wU1 = m->wU1;
    q.CB = m->CB;
    q.hvn = m->hvn;
    q.hgn = m->hgn;
    q.S = m->S;
    q.smean = m->smean;
    q.kx = m->kx;
    q.kz = m->kz;
    q.st = m->state;
    q.prep = m->prep;
    q.sc = m->sc;
    q.blk0 = b->bfin;
    b->bfin += eblocks;
    b->hfin.push_back(q);
  }
  b->xnt = b->xchunk > 0 ? xpencil_chunk_threads() : xpencil_threads(b->prec, b->lx, b->bx);
}

// Carves every member, builds all tables, and carves the batch's device
// tables after the members; with base == nullptr only measures.
size_t layout(Batch* b, char* base) {
  Carve c(base);
  for (Member* m : b->mem) carve(m, c);
  for (Member* m : b->mem) build_jobs(m);
  build_batch(b);
  std::vector<JobList*> all = b->lists();
  for (Member* m : b->mem) {
    all.push_back(&m->H4);
    all.push_back(&m->H5);
  }
  for (JobList* jl : all) {
    jl->dev = c.take<GemmJob>(std::max(1, jl->n()));
    jl->tmap = c.take<int>(jl->max_tiles());
  }
  const size_t n = b->mem.size();
  b->dx = c.take<XArgs>(n);
  b->dzi = c.take<ZArgs>(n);
  b->dzf = c.take<ZArgs>(n);
  b->dzd = c.take<ZArgs>(2 * n);
  b->ddr = c.take<DRowArgs>(n);
  b->ddf = c.take<DFinArgs>(n);
  b->drhs = c.take<RhsArgs>(n);
  b->drhsw = c.take<RhsArgs>(n);
  b->dfin = c.take<FinArgs>(n);
  return c.off;
}

// Stage boundaries: mark(i) is called before stage i and once more at the
// end; the eager profiling path records a HIP event there.  Every stage is
// one kernel launch (or none where it does not apply), all on the caller's
// stream.
enum Stage {
  ST_GEMM_MEAN, ST_GEMM_STATE, ST_GEMM_D2, ST_ZFFT_INV, ST_XPENCIL, ST_ZFFT_FWD, ST_GEMM_PROJ, ST_RHS, ST_GEMM_VINV,
  ST_GEMM_V, ST_FINALIZE, ST_DIAG_ZFFT, ST_DIAG_ROWS, ST_DIAG_FINAL, ST_COUNT
};
static_assert(ST_COUNT == PCS_NSTAGE, "stage table");
const char* const STAGE_NAMES[ST_COUNT] = {"gemm_mean", "gemm_state", "gemm_d2",   "zfft_inv",  "xpencil",
                                            "zfft_fwd",  "gemm_proj",  "rhs",       "gemm_vinv", "gemm_v",
                                            "finalize",  "diag_zfft",  "diag_rows", "diag_final"};

// mark(i) returns how many times stage i is launched back to back (1 in a
// normal step; the profiling path repeats every stage whose outputs do not
// feed its own inputs, i.e. all but the final diagnostics record).
struct NoMark {
  int operator()(int) const { return 1; }
};

template <typename Mark>
void explicit_stage(Batch* b, const Mark& mark) {
  hipStream_t s = b->s;
  const int nm = (int)b->mem.size();
  for (int r = mark(ST_GEMM_MEAN); r > 0; --r) b->GSm.run(s);
  for (int r = mark(ST_GEMM_STATE); r > 0; --r) b->GS.run(s);
  for (int r = mark(ST_GEMM_D2); r > 0; --r) b->GSb.run(s);
  for (int r = mark(ST_ZFFT_INV); r > 0; --r)
    if (b->dim == 3) launch_zfft(b->prec, b->zgi, b->dzi, nm, b->bzi, b->lzi, s);
  for (int r = mark(ST_XPENCIL); r > 0; --r)
    launch_xpencil(b->dim, b->prec, b->xnt, b->xchunk, b->dx, nm, b->bx, b->lx, s);
  for (int r = mark(ST_ZFFT_FWD); r > 0; --r)
    if (b->dim == 3) launch_zfft(b->prec, b->zgi, b->dzf, nm, b->bzf, b->lzf, s);
  for (int r = mark(ST_GEMM_PROJ); r > 0; --r) b->GP.run(s);
  for (int r = mark(ST_RHS); r > 0; --r) launch_rhs(b->drhsw, b->brhsw, b->drhs, b->brhs, nm, s);
}

template <typename Mark>
void enqueue_step(Batch* b, const Mark& mark) {
  hipStream_t s = b->s;
  const int nm = (int)b->mem.size();
  explicit_stage(b, mark);
  for (int r = mark(ST_GEMM_VINV); r > 0; --r) b->G4.run(s);
  for (int r = mark(ST_GEMM_V); r > 0; --r) b->G5.run(s);
  for (int r = mark(ST_FINALIZE); r > 0; --r) launch_finalize(b->dfin, nm, b->bfin, s);
  for (int r = mark(ST_DIAG_ZFFT); r > 0; --r)
    if (b->dim == 3) launch_zfft(0, b->zgd, b->dzd, (int)b->hzd.size(), b->bzd, b->lzd, s);
  for (int r = mark(ST_DIAG_ROWS); r > 0; --r) launch_diag_rows(b->ddr, nm, b->bdr, b->ldr, s);
  for (int r = mark(ST_DIAG_FINAL); r > 0; --r) launch_diag_final(b->ddf, nm, s);
  mark(ST_COUNT);
}

// The diagnostics of the state that the last finalize wrote, on stream t.
void enqueue_diagnostics(Batch* b, hipStream_t t) {
  const int nm = (int)b->mem.size();
  if (b->dim == 3) launch_zfft(0, b->zgd, b->dzd, (int)b->hzd.size(), b->bzd, b->lzd, t);
  launch_diag_rows(b->ddr, nm, b->bdr, b->ldr, t);
  launch_diag_final(b->ddf, nm, t);
}

// One step for graph capture, with side branches beside the main chain:
// branch 1 computes the FP64 mean profiles (read by the x pencils) and the
// FP64 D2 / D products of the state (read by the right-hand sides) while the
// FP32 padded-grid products, transforms and projections run; branch 2
// (diag_prev) computes the diagnostics of the previous step's state, which
// only have to finish before this step overwrites the state (the products
// of the solves write c, finalize the rest and the diagnostics inputs).
// ev: four events.  The launches and their order within each chain are those
// of enqueue_step.  The step record (diag_final) advances the device step
// counter, and the SBDF4 right-hand sides index the history rings with it:
// with any SBDF4 run in the batch, the right-hand sides therefore wait for
// the previous step's diagnostics branch (CNAB2 reads no counter there and
// waits only before the state is overwritten).
void enqueue_step_branched(Batch* b, bool diag_prev, hipEvent_t* ev) {
  hipStream_t s = b->s, s1 = b->side[0], s2 = b->side[1];
  const int nm = (int)b->mem.size();
  const bool prod = b->branch == 1;
  bool ring = false;
  for (const Member* m : b->mem) ring |= m->p.scheme == 1;
  (void)hipEventRecord(ev[0], s);  // the previous step's state is complete
  if (prod) {
    (void)hipStreamWaitEvent(s1, ev[0], 0);
    b->GSm.run(s1);
    (void)hipEventRecord(ev[1], s1);
    b->GSb.run(s1);
    (void)hipEventRecord(ev[2], s1);
  }
  if (diag_prev) {
    (void)hipStreamWaitEvent(s2, ev[0], 0);
    enqueue_diagnostics(b, s2);
    (void)hipEventRecord(ev[3], s2);
  }
  b->GS.run(s);
  if (b->dim == 3) launch_zfft(b->prec, b->zgi, b->dzi, nm, b->bzi, b->lzi, s);
  if (prod) (void)hipStreamWaitEvent(s, ev[1], 0);
  launch_xpencil(b->dim, b->prec, b->xnt, b->xchunk, b->dx, nm, b->bx, b->lx, s);
  if (b->dim == 3) launch_zfft(b->prec, b->zgi, b->dzf, nm, b->bzf, b->lzf, s);
  b->GP.run(s);
  if (prod) (void)hipStreamWaitEvent(s, ev[2], 0);
  if (diag_prev && ring) (void)hipStreamWaitEvent(s, ev[3], 0);
  launch_rhs(b->drhsw, b->brhsw, b->drhs, b->brhs, nm, s);
  b->G4.run(s);
  if (diag_prev && !ring) (void)hipStreamWaitEvent(s, ev[3], 0);
  b->G5.run(s);
  launch_finalize(b->dfin, nm, b->bfin, s);
}

// Tile autotuner: times each candidate tile configuration of a product table
// on the device (results of the timing launches are discarded) and keeps the
// fastest.  Choices are cached per table shape for the process lifetime, and
// across processes in the file named by PCS_TUNE_CACHE (if set): one line per
// choice, "<arch> <choice> <key...>" (arch as the device reports it, up to the
// first ':'; key: the table's shape signature); lines of this device's arch are
// loaded before tuning, and every new choice is appended, so a table shape
// keeps its tiles (and its summation order) from one process to the next.
std::map<std::vector<int>, int>& tune_cache() {
  static std::map<std::vector<int>, int> c;
  return c;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a(prop.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

void load_tune_file(const char* path, const std::string& arch) {
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string a;
    int choice = -1;
    if (!(ls >> a >> choice) || a != arch || choice < 0 || choice >= 2 * GEMM_NCFG) continue;
    std::vector<int> key;
    for (int v; ls >> v;) key.push_back(v);
    if (!key.empty()) tune_cache()[key] = choice;
  }
}

void append_tune_file(const char* path, const std::string& arch, const std::vector<int>& key, int choice) {
  std::ofstream out(path, std::ios::app);
  out << arch << ' ' << choice;
  for (int v : key) out << ' ' << v;
  out << '\n';
}

// With PCS_DEBUG set, the autotuner reports every timing on stderr.
bool tune_log() {
  static const bool on = std::getenv("PCS_DEBUG") != nullptr;
  return on;
}

pcs_status autotune(Batch* b) {
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  // PCS_PRODUCT_FORM=plain or =parity restricts the choice to one form of
  // every table (for testing both; default: both forms are timed)
  int forms = 3;
  if (const char* f = std::getenv("PCS_PRODUCT_FORM")) {
    if (!std::strcmp(f, "plain")) forms = 1;
    if (!std::strcmp(f, "parity")) forms = 2;
  }
  // PCS_GEMM_CFG=c forces tile configuration c where the form allows it
  // (for testing every configuration; default: all are timed)
  int only = -1;
  if (const char* c = std::getenv("PCS_GEMM_CFG")) {
    only = std::atoi(c);
    if (only < 0 || only >= GEMM_NCFG) only = -1;
  }
  const char* tune_path = std::getenv("PCS_TUNE_CACHE");
  const std::string arch = tune_path ? device_arch() : std::string();
  if (tune_path) load_tune_file(tune_path, arch);
  hipStream_t s = b->s;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (JobList* jl : b->lists()) {
    if (!jl->n()) continue;
    jl->use(0);
    auto key = jl->key();
    key.push_back(forms);
    key.push_back(only);
    key.push_back(GEMM_NCFG);  // the candidate set: choices made among fewer configurations do not apply
    auto it = tune_cache().find(key);
    int best = -1, bestf = 0;
    if (it != tune_cache().end()) {
      best = it->second % GEMM_NCFG;
      bestf = it->second / GEMM_NCFG;
    } else {
      float tbest = 1e30f;
      for (int f = 0; f < 2; ++f) {
        if (!(forms & (1 << f))) continue;
        jl->use(f);
        for (int cfg = 0; cfg < GEMM_NCFG; ++cfg) {
          if (!jl->allowed(cfg) || (only >= 0 && cfg != only && jl->allowed(only))) continue;
          jl->set_cfg(cfg);
          HIPCHK(up_list(jl, s));
          jl->run(s);  // warm-up
          HIPCHK(hipEventRecord(e0, s));
          for (int r = 0; r < 3; ++r) jl->run(s);
          HIPCHK(hipEventRecord(e1, s));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          if (tune_log())
            std::fprintf(stderr, "pcs: table of %d products (type %d): form %d cfg %2d tiles %6d lds %6zu: %8.2f us\n",
                         jl->n(), (int)jl->type, f, cfg, jl->tiles, jl->lds, ms * 1e3f / 3);
          if (ms < tbest) {
            tbest = ms;
            best = cfg;
            bestf = f;
          }
        }
      }
      if (best >= 0) {
        tune_cache()[key] = bestf * GEMM_NCFG + best;
        if (tune_path) append_tune_file(tune_path, arch, key, bestf * GEMM_NCFG + best);
      }
    }
    if (best < 0) {
      // no candidate under the forced form (the compensated tables have the
      // parity form only): the table's default
      jl->use(0);
      jl->prepare();
    } else {
      jl->use(bestf);
      jl->set_cfg(best);
    }
    HIPCHK(up_list(jl, s));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PCS_OK;
}

// Homogeneous solutions of the influence-matrix method for one member, with
// the same product kernels as the step (own small tables), and w . U_1.
pcs_status homogeneous_solutions(Member* m, hipStream_t s) {
  const Dims& d = m->d;
  const size_t fsi = (size_t)(d.N - 1) * d.cw;
  HIPCHK(hipMemsetAsync(m->R, 0, m->nsolve * fsi * sizeof(double), s));
  launch_homog_rhs(d, m->p, m->d2i0, m->d2in, m->R, s);
  m->H4.run(s);
  m->H5.run(s);
  launch_influence(d, m->Zphi, m->Zv, m->ZDv, m->kz, m->infl, m->U1, s);
  HIPCHK(hipGetLastError());
  std::vector<double> U1(d.N + 1);
  HIPCHK(hipMemcpyAsync(U1.data(), m->U1, U1.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double acc = 0;
  for (int j = 0; j <= d.N; ++j) acc += m->ops->w[j] * U1[j];
  m->wU1 = acc;
  return PCS_OK;
}

// Merged product tables and argument tables to the device (after the
// homogeneous solutions, which fix w . U_1 in the finalize arguments).
pcs_status upload_tables(Batch* b) {
  hipStream_t s = b->s;
  for (size_t i = 0; i < b->mem.size(); ++i) b->hfin[i].wU1 = b->mem[i]->wU1;
  for (JobList* jl : b->lists())
    if (jl->n()) HIPCHK(up_list(jl, s));
  HIPCHK(up(b->dx, b->hx, s));
  if (!b->hzi.empty()) {
    HIPCHK(up(b->dzi, b->hzi, s));
    HIPCHK(up(b->dzf, b->hzf, s));
    HIPCHK(up(b->dzd, b->hzd, s));
  }
  HIPCHK(up(b->ddr, b->hdr, s));
  HIPCHK(up(b->ddf, b->hdf, s));
  HIPCHK(up(b->drhs, b->hrhs, s));
  HIPCHK(up(b->drhsw, b->hrhsw, s));
  HIPCHK(up(b->dfin, b->hfin, s));
  return PCS_OK;
}

// History := explicit terms of the current state (the first step is CNAB1).
pcs_status history_from_state(Batch* b) {
  hipStream_t s = b->s;
  explicit_stage(b, NoMark());
  HIPCHK(hipGetLastError());
  for (Member* m : b->mem) {
    const Dims& d = m->d;
    const size_t fs = (size_t)(d.N + 1) * d.cw;
    double* hist = m->state + (size_t)m->nq * fs;
    HIPCHK(hipMemcpyAsync(hist, m->hvn, fs * sizeof(double), hipMemcpyDeviceToDevice, s));
    int h = 1;
    if (d.dim == 3) HIPCHK(hipMemcpyAsync(hist + (h++) * fs, m->hgn, fs * sizeof(double), hipMemcpyDeviceToDevice, s));
    const int SF = d.dim == 2 ? 2 : 3;
    HIPCHK(hipMemcpyAsync(hist + h * fs, m->S + SF * fs, d.nc * fs * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (m->smean) {
      // mixed precision: the mean column of F comes from the FP64 projection
      const int n1 = d.N + 1;
      for (int a = 0; a < d.nc; ++a)
        HIPCHK(hipMemcpy2DAsync(hist + (h + a) * fs, d.cw * sizeof(double), m->smean + (size_t)(SF + a) * n1,
                                sizeof(double), sizeof(double), n1, hipMemcpyDeviceToDevice, s));
    }
  }
  return PCS_OK;
}

constexpr int GRAPH_STEPS = 8;

// Captures `steps` consecutive steps as one graph (null on failure: the
// caller then launches eagerly).
void capture_steps(Batch* b, int steps, hipGraph_t* graph, hipGraphExec_t* exec) {
  *graph = nullptr;
  *exec = nullptr;
  if (hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (b->side[0] && b->side[1] && (int)b->evs.size() >= 4 * steps) {
    for (int i = 0; i < steps; ++i) enqueue_step_branched(b, i > 0, &b->evs[4 * i]);
    enqueue_diagnostics(b, b->s);  // the last step's
  } else {
    for (int i = 0; i < steps; ++i) enqueue_step(b, NoMark());
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(b->s, &g) != hipSuccess || g == nullptr) {
    (void)hipGetLastError();
    return;
  }
  hipGraphExec_t ge = nullptr;
  if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    return;
  }
  *graph = g;
  *exec = ge;
}

pcs_status capture(Batch* b) {
  if (b->s == nullptr) return PCS_OK;  // the legacy default stream cannot be captured
  // side streams (default priority) and events for the branches; without
  // them the graphs hold the single chain
  bool ok = b->branch != 0;
  for (hipStream_t& t : b->side)
    if (ok && !t && hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) {
      t = nullptr;
      ok = false;
    }
  while (ok && (int)b->evs.size() < 4 * GRAPH_STEPS) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      ok = false;
      break;
    }
    b->evs.push_back(e);
  }
  if (!ok) (void)hipGetLastError();
  capture_steps(b, 1, &b->graph, &b->gexec);
  if (b->gexec) capture_steps(b, GRAPH_STEPS, &b->graphn, &b->gexecn);
  return PCS_OK;
}

// Validates and sizes a batch of n runs (all of one dimension and one
// precision); fills b->mem.
pcs_status setup_batch(Batch* b, int32_t n, const pcs_grid* grids, const pcs_params* params, size_t* bytes) {
  if (n <= 0 || !grids || !params) return PCS_ERR_ARG;
  for (int32_t i = 0; i < n; ++i) {
    Member* m = new (std::nothrow) Member();
    if (!m) return PCS_ERR_ARG;
    b->mem.push_back(m);
    pcs_status st = setup_dims(m, &grids[i], &params[i]);
    if (st != PCS_OK) return st;
    if (m->d.dim != b->mem[0]->d.dim || m->prec != b->mem[0]->prec) return PCS_ERR_UNSUPPORTED;
  }
  b->dim = b->mem[0]->d.dim;
  b->prec = b->mem[0]->prec;
  *bytes = layout(b, nullptr);
  return PCS_OK;
}

pcs_status sbdf4_cold_start(Member* m, hipStream_t s, long long step);
pcs_status member_set_state(Member* m, hipStream_t s, const double* host, size_t n);

// Largest difference of `got` from `ref` relative to the largest magnitude
// of `ref`, per field of rows x cw values (columns 0 and 1, the mean mode,
// excluded: the mixed path carries that mode in FP64 elsewhere), maximised
// over the fields; infinite for a non-finite difference.
template <typename T>
double field_error(const T* got, const T* ref, size_t nf, size_t rows, size_t cw) {
  double worst = 0;
  for (size_t f = 0; f < nf; ++f) {
    double dmax = 0, rmax = 0;
    for (size_t r = 0; r < rows; ++r)
      for (size_t c = 2; c < cw; ++c) {
        const size_t i = (f * rows + r) * cw + c;
        const double d = std::fabs((double)got[i] - (double)ref[i]);
        if (!(d <= dmax)) dmax = d;  // also NaN
        rmax = std::max(rmax, std::fabs((double)ref[i]));
      }
    if (!std::isfinite(dmax)) return INFINITY;
    if (dmax > 0) worst = std::max(worst, rmax > 0 ? dmax / rmax : INFINITY);
  }
  return worst;
}

// Precision 4: the variant of each wall-normal product table, chosen under
// the error budget (see pcs_params.precision).  Every variant runs the
// explicit half of a step on the initial state; the FP64-operator variant
// is the reference.  A variant of the state products is judged by its own
// outputs (the padded-grid values and d/dy), a variant of the projections
// by its outputs under the reference state products, so that each error
// belongs to one table.  Times are those of the table's launch after
// tuning; an eager batch is not timed and prefers FP32, then FP64.  Leaves
// the batch built with the choice, tuned, and the tables of the homogeneous
// solutions uploaded; the state is reset by the caller.
pcs_status choose_y_variants(Batch* b, const uint64_t* seeds, double amp) {
  double budget = 1e-5;
  if (const char* e = std::getenv("PCS_Y_ERROR_BUDGET")) {
    char* end = nullptr;
    const double v = std::strtod(e, &end);
    if (end == e || !(v >= 0) || !std::isfinite(v)) return PCS_ERR_ARG;
    budget = v;
  }
  b->ybudget = budget;
  hipStream_t s = b->s;
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  if (!b->eager) {
    HIPCHK(hipEventCreate(&ev.e[0]));
    HIPCHK(hipEventCreate(&ev.e[1]));
  }
  auto time_us = [&](const JobList& jl, double* out) -> pcs_status {
    jl.run(s);  // warm-up
    HIPCHK(hipEventRecord(ev.e[0], s));
    for (int r = 0; r < 5; ++r) jl.run(s);
    HIPCHK(hipEventRecord(ev.e[1], s));
    HIPCHK(hipEventSynchronize(ev.e[1]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    *out = ms * 1e3 / 5;
    return PCS_OK;
  };
  auto rebuild = [&](int v1, int v2) -> pcs_status {
    for (Member* m : b->mem) {
      m->yv1 = v1;
      m->yv2 = v2;
      build_jobs(m);
    }
    build_batch(b);
    pcs_status st = PCS_OK;
    if (!b->eager && (st = autotune(b)) != PCS_OK) return st;
    return PCS_OK;
  };
  const size_t nm = b->mem.size();
  // per member: reference padded-grid values (FP32) and projections (FP64)
  std::vector<std::vector<float>> yref(nm);
  std::vector<std::vector<double>> sref(nm);
  std::vector<float> ybuf;
  std::vector<double> sbuf;
  // runs the explicit half of a step in variants (v1, v2) and measures the
  // state products (t1, e1) and / or the projections (t2, e2)
  auto trial = [&](int v1, int v2, int t1, int t2) -> pcs_status {
    pcs_status st = rebuild(v1, v2);
    if (st != PCS_OK) return st;
    for (size_t i = 0; i < nm; ++i)
      if ((st = reset_state(b->mem[i], seeds[i], amp, s)) != PCS_OK) return st;
    if ((st = upload_tables(b)) != PCS_OK) return st;
    explicit_stage(b, NoMark());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    const bool ref = v1 == Y_FP64 && v2 == Y_FP64;
    for (size_t i = 0; i < nm; ++i) {
      const Member* m = b->mem[i];
      const size_t cw = m->d.cw, m1 = m->d.M + 1, n1 = m->d.N + 1;
      if (ref || t1 > 0) {
        std::vector<float>& y = ref ? yref[i] : ybuf;
        y.resize((size_t)m->nyin * m1 * cw);
        HIPCHK(hipMemcpy(y.data(), m->Yin32, y.size() * sizeof(float), hipMemcpyDeviceToHost));
        if (!ref)
          b->yerr[0][t1 - 1] = std::max(std::max(b->yerr[0][t1 - 1], 0.0),
                                        field_error(y.data(), yref[i].data(), m->nyin, m1, cw));
      }
      if (ref || t2 > 0) {
        // the projections S (nout fields), then D N (1 or 2 fields)
        std::vector<double>& q = ref ? sref[i] : sbuf;
        const size_t ns = (size_t)m->nout * n1 * cw, nd = (size_t)(m->d.dim == 2 ? 1 : 2) * n1 * cw;
        q.resize(ns + nd);
        HIPCHK(hipMemcpy(q.data(), m->S, ns * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(q.data() + ns, m->DN, nd * sizeof(double), hipMemcpyDeviceToHost));
        if (!ref)
          b->yerr[1][t2 - 1] =
              std::max(std::max(b->yerr[1][t2 - 1], 0.0),
                       field_error(q.data(), sref[i].data(), m->nout + (m->d.dim == 2 ? 1 : 2), n1, cw));
      }
    }
    if (!b->eager) {
      if (t1 > 0 || ref) {
        double us = 0;
        if ((st = time_us(b->GS, &us)) != PCS_OK) return st;
        b->yus[0][(ref ? Y_FP64 : t1) - 1] = us;
      }
      if (t2 > 0 || ref) {
        double us = 0;
        if ((st = time_us(b->GP, &us)) != PCS_OK) return st;
        b->yus[1][(ref ? Y_FP64 : t2) - 1] = us;
      }
    }
    return PCS_OK;
  };
  pcs_status st = trial(Y_FP64, Y_FP64, 0, 0);
  if (st != PCS_OK) return st;
  b->yerr[0][Y_FP64 - 1] = b->yerr[1][Y_FP64 - 1] = 0.0;
  std::vector<int> cand{Y_FP32};
  if (!b->eager) cand.push_back(Y_COMP);
  for (int v : cand) {
    if ((st = trial(v, Y_FP64, v, 0)) != PCS_OK || (st = trial(Y_FP64, v, 0, v)) != PCS_OK) return st;
  }
  // the fastest variant within the budget, FP64 unless another is strictly
  // faster (eager: the first of FP32, FP64)
  int pick[2];
  for (int t = 0; t < 2; ++t) {
    pick[t] = Y_FP64;
    if (b->eager) {
      if (b->yerr[t][Y_FP32 - 1] <= budget) pick[t] = Y_FP32;
      continue;
    }
    for (int v : cand)
      if (b->yerr[t][v - 1] <= budget && b->yus[t][v - 1] < b->yus[t][pick[t] - 1]) pick[t] = v;
  }
  if ((st = rebuild(pick[0], pick[1])) != PCS_OK) return st;
  for (Member* m : b->mem) {
    HIPCHK(up_list(&m->H4, s));
    HIPCHK(up_list(&m->H5, s));
  }
  return PCS_OK;
}

pcs_status init_batch(Batch* b, int32_t n, const pcs_grid* grids, const pcs_params* params, const uint64_t* seeds,
                      double amp, void* workspace, size_t bytes, void* stream) {
  if (!workspace || !seeds || !std::isfinite(amp)) return PCS_ERR_ARG;
  size_t need = 0;
  pcs_status st = setup_batch(b, n, grids, params, &need);
  if (st != PCS_OK) return st;
  if (bytes < need || (reinterpret_cast<uintptr_t>(workspace) % ALIGN) != 0) return PCS_ERR_WORKSPACE;
  for (Member* m : b->mem) {
    m->ops = wall_ops(m->d.N);
    if (!m->ops) return PCS_ERR_UNSUPPORTED;
  }
  layout(b, static_cast<char*>(workspace));
  b->s = static_cast<hipStream_t>(stream);
  if (hipError_t e = gemm_set_attributes(); e != hipSuccess) {
    report(e, "gemm_set_attributes", __LINE__);
    return PCS_ERR_DEVICE;
  }
  if (hipError_t e = fft_set_attributes(); e != hipSuccess) {
    report(e, "fft_set_attributes", __LINE__);
    return PCS_ERR_DEVICE;
  }
  for (int32_t i = 0; i < n; ++i)
    if ((st = upload_member(b->mem[i], seeds[i], amp, b->s)) != PCS_OK) return st;
  if (b->prec == 4) {
    if ((st = choose_y_variants(b, seeds, amp)) != PCS_OK) return st;
  } else if (!b->eager && (st = autotune(b)) != PCS_OK) {
    return st;
  }
  for (int32_t i = 0; i < n; ++i)
    if ((st = reset_state(b->mem[i], seeds[i], amp, b->s)) != PCS_OK ||
        (st = homogeneous_solutions(b->mem[i], b->s)) != PCS_OK)
      return st;
  if ((st = upload_tables(b)) != PCS_OK || (st = history_from_state(b)) != PCS_OK) return st;
  for (Member* m : b->mem)
    if ((st = sbdf4_cold_start(m, b->s, 0)) != PCS_OK) return st;
  hipError_t e1 = hipStreamSynchronize(b->s), e2 = hipGetLastError();
  if (e1 != hipSuccess || e2 != hipSuccess) {
    report(e1 != hipSuccess ? e1 : e2, "init synchronise", __LINE__);
    return PCS_ERR_DEVICE;
  }
  if (!b->eager) capture(b);
  return PCS_OK;
}

pcs_status step_batch(Batch* b, int32_t nsteps) {
  int left = nsteps;
  if (b->gexecn)
    for (; left >= GRAPH_STEPS; left -= GRAPH_STEPS)
      if (hipGraphLaunch(b->gexecn, b->s) != hipSuccess) return PCS_ERR_DEVICE;
  for (; left > 0; --left) {
    if (b->gexec) {
      if (hipGraphLaunch(b->gexec, b->s) != hipSuccess) return PCS_ERR_DEVICE;
    } else {
      enqueue_step(b, NoMark());
    }
  }
  return hipGetLastError() == hipSuccess ? PCS_OK : PCS_ERR_DEVICE;
}

pcs_status member_diagnostics(Member* m, hipStream_t s, pcs_diag* outp, int32_t max, int32_t* n_out) {
  if (!n_out || max < 0 || (max > 0 && !outp)) return PCS_ERR_ARG;
  *n_out = 0;
  DevScalars sc;
  HIPCHK(hipMemcpyAsync(&sc, m->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  long long first = m->drained + 1;
  if (sc.step - first + 1 > RING) first = sc.step - RING + 1;
  long long cnt = sc.step - first + 1;
  if (cnt > max) cnt = max;
  std::vector<DiagRec> recs((size_t)(cnt > 0 ? cnt : 0));
  // records of steps first .. first+cnt-1 sit at ring slots (step-1) % RING:
  // at most two contiguous pieces
  long long done = 0;
  while (done < cnt) {
    const long long slot = (first + done - 1) % RING;
    const long long piece = std::min<long long>(cnt - done, RING - slot);
    HIPCHK(hipMemcpyAsync(&recs[done], m->ring + slot, (size_t)piece * sizeof(DiagRec), hipMemcpyDeviceToHost, s));
    done += piece;
  }
  HIPCHK(hipStreamSynchronize(s));
  static_assert(sizeof(DiagRec) == sizeof(pcs_diag), "diagnostic record layout");
  if (cnt > 0) std::memcpy(outp, recs.data(), (size_t)cnt * sizeof(pcs_diag));
  *n_out = (int32_t)cnt;
  m->drained = first + cnt - 1;
  if (sc.blowup) m->blowup = 1;
  return m->blowup ? PCS_BLOWUP : PCS_OK;
}

// Midplane histograms (Section 3: the PDF of Tr c behind eqs. (4)-(5), and
// those of the velocity fluctuations): sets the range and bins of quantity q
// of run `idx` (nbins = 0: off), clears its counts and updates the argument
// table the captured steps read.
static_assert(HIST_MAX == PCS_HIST_MAX, "histogram capacity");
static_assert(HIST_Q == 8 && PCS_PDF_TRC == 0 && PCS_PDF_U == 1 && PCS_PDF_V == 2 && PCS_PDF_W == 3 &&
                  PCS_PDF_DUDX == 4 && PCS_PDF_DUDZ == 5 && PCS_PDF_DWDX == 6 && PCS_PDF_DWDZ == 7,
              "quantities");
// quantities that need the spanwise direction (w or d/dz)
bool needs_3d(int q) { return q == PCS_PDF_W || q == PCS_PDF_DUDZ || q == PCS_PDF_DWDX || q == PCS_PDF_DWDZ; }
pcs_status member_hist_setup(Batch* b, int idx, int q, double lo, double hi, int32_t nbins) {
  if (q < 0 || q >= HIST_Q || (needs_3d(q) && b->mem[idx]->d.dim != 3)) return PCS_ERR_ARG;
  if (nbins < 0 || nbins > HIST_MAX) return PCS_ERR_ARG;
  if (nbins > 0 && !(std::isfinite(lo) && std::isfinite(hi) && lo < hi && std::isfinite(nbins / (hi - lo))))
    return PCS_ERR_ARG;
  Member* m = b->mem[idx];
  hipStream_t s = b->s;
  HIPCHK(hipStreamSynchronize(s));
  m->hlo[q] = lo;
  m->hhi[q] = hi;
  m->hbins[q] = nbins;
  DRowArgs& r = b->hdr[idx];
  r.hbins[q] = nbins;
  r.hlo[q] = lo;
  r.hscale[q] = nbins > 0 ? nbins / (hi - lo) : 0.0;
  HIPCHK(hipMemcpy(b->ddr + idx, &r, sizeof(r), hipMemcpyHostToDevice));
  DFinArgs& f = b->hdf[idx];
  f.mom_mask = nbins > 0 ? (f.mom_mask | (1 << q)) : (f.mom_mask & ~(1 << q));
  HIPCHK(hipMemcpy(b->ddf + idx, &f, sizeof(f), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(m->hist + (size_t)q * (HIST_MAX + 2), 0, (HIST_MAX + 2) * sizeof(unsigned long long)));
  HIPCHK(hipMemset(m->msum + (size_t)q * 3, 0, 3 * sizeof(double)));
  return PCS_OK;
}

// Running moments of quantity q: [samples, sum, sum of squares].
pcs_status batch_y_choice(const Batch* b, pcs_ychoice* out) {
  if (!out) return PCS_ERR_ARG;
  out->variant[0] = b->mem[0]->yv1;
  out->variant[1] = b->mem[0]->yv2;
  out->budget = b->ybudget;
  for (int t = 0; t < 2; ++t)
    for (int v = 0; v < 3; ++v) {
      out->error[t][v] = b->yerr[t][v];
      out->time_us[t][v] = b->yus[t][v];
    }
  return PCS_OK;
}

pcs_status member_moments(Member* m, hipStream_t s, int q, double* out) {
  if (q < 0 || q >= HIST_Q || !out || m->hbins[q] <= 0) return PCS_ERR_ARG;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(out, m->msum + (size_t)q * 3, 3 * sizeof(double), hipMemcpyDeviceToHost));
  return PCS_OK;
}

pcs_status member_hist_get(Member* m, hipStream_t s, int q, uint64_t* counts, int32_t n) {
  if (q < 0 || q >= HIST_Q) return PCS_ERR_ARG;
  if (!counts || m->hbins[q] <= 0 || n != m->hbins[q] + 2) return PCS_ERR_ARG;
  HIPCHK(hipStreamSynchronize(s));
  static_assert(sizeof(uint64_t) == sizeof(unsigned long long), "count type");
  HIPCHK(hipMemcpy(counts, m->hist + (size_t)q * (HIST_MAX + 2), (size_t)n * sizeof(uint64_t),
                   hipMemcpyDeviceToHost));
  return PCS_OK;
}

// SBDF4 history in the order of the flat state after (q, h): q^{n-1}, q^{n-2},
// q^{n-3}, then X^{n-2}, X^{n-3}, each as its ring slot for state index n.
struct HistBlock {
  double* dev;
  size_t doubles;
};
std::vector<HistBlock> history_blocks(const Member* m, long long n) {
  std::vector<HistBlock> out;
  if (m->p.scheme != 1) return out;
  const size_t fs = (size_t)(m->d.N + 1) * m->d.cw, qs = (size_t)m->nq * fs, hs = (size_t)m->nh * fs;
  for (int k = 1; k <= 3; ++k) out.push_back({m->qring + (size_t)((n - k) & 3) * qs, qs});
  for (int k = 2; k <= 3; ++k) out.push_back({m->hring + (size_t)((n - k) & 3) * hs, hs});
  return out;
}

// SBDF4 start from a single state at step n: a constant past, q^{n-k} := q^n
// and X^{n-k} := X^{n-1} (the explicit terms the state's history holds).
pcs_status sbdf4_cold_start(Member* m, hipStream_t s, long long step = 0) {
  const size_t qs = (size_t)m->nq * (m->d.N + 1) * m->d.cw;
  const std::vector<HistBlock> hb = history_blocks(m, step);
  for (size_t i = 0; i < hb.size(); ++i)  // three state blocks, then two explicit ones
    HIPCHK(hipMemcpyAsync(hb[i].dev, i < 3 ? m->state : m->state + qs, hb[i].doubles * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  return PCS_OK;
}

pcs_status member_get_state(Member* m, hipStream_t s, double* host, size_t n) {
  if (!host || n != m->nstate) return PCS_ERR_ARG;
  DevScalars sc;
  HIPCHK(hipMemcpyAsync(&sc, m->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const size_t base = (size_t)(m->nq + m->nh) * (m->d.N + 1) * m->d.cw;
  HIPCHK(hipMemcpyAsync(host + 4, m->state, base * sizeof(double), hipMemcpyDeviceToHost, s));
  size_t o = 4 + base;
  for (const HistBlock& hb : history_blocks(m, sc.step)) {
    HIPCHK(hipMemcpyAsync(host + o, hb.dev, hb.doubles * sizeof(double), hipMemcpyDeviceToHost, s));
    o += hb.doubles;
  }
  HIPCHK(hipStreamSynchronize(s));
  host[0] = (double)sc.step;
  host[1] = sc.t;
  host[2] = sc.pi;
  host[3] = 0.0;
  return PCS_OK;
}

}  // namespace

struct pcs_sim {
  Batch b;
  int static_dev = -1;  // device whose static workspace this run holds (pcs_init_static), else -1
  Member* m() { return b.mem[0]; }
};

namespace {

// ---- allocation-free initialisation (pcs_init_static)
// The workspace of such runs is this file-scope device array: one copy per
// GPU, resident from the library's load until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: its device
// address on each GPU comes from hipGetSymbolAddress, taken once per device
// with that device current and kept in static_slots; only that address is
// ever passed to kernels, memsets or copies.
constexpr size_t STATIC_BYTES = (size_t)64 << 20;
static_assert(STATIC_BYTES == PCS_STATIC_BYTES, "static workspace size");
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
struct StaticSlot {
  void* ptr = nullptr;  // device address of scratch on this GPU
  bool busy = false;    // held by a live handle
};
std::mutex static_mu;
StaticSlot static_slots[MAX_DEVICES];

}  // namespace

struct pcs_ens {
  Batch b;
};

extern "C" {

pcs_status pcs_workspace_bytes(const pcs_grid* grid, const pcs_params* params, size_t* bytes) {
  if (!bytes || !grid || !params) return PCS_ERR_ARG;
  Batch b;
  return setup_batch(&b, 1, grid, params, bytes);
}

pcs_status pcs_init(const pcs_grid* grid, const pcs_params* params, uint64_t seed, double amp, void* workspace,
                    size_t bytes, void* stream, pcs_sim** out) {
  if (!out) return PCS_ERR_ARG;
  *out = nullptr;
  if (!grid || !params) return PCS_ERR_ARG;
  pcs_sim* sim = new (std::nothrow) pcs_sim();
  if (!sim) return PCS_ERR_ARG;
  const pcs_status st = init_batch(&sim->b, 1, grid, params, &seed, amp, workspace, bytes, stream);
  if (st != PCS_OK) {
    delete sim;
    return st;
  }
  *out = sim;
  return PCS_OK;
}

pcs_status pcs_init_static(const pcs_grid* grid, const pcs_params* params, uint64_t seed, double amp, void* stream,
                           pcs_sim** out) {
  if (!out) return PCS_ERR_ARG;
  *out = nullptr;
  if (!grid || !params) return PCS_ERR_ARG;
  size_t need = 0;
  {
    Batch probe;
    const pcs_status st = setup_batch(&probe, 1, grid, params, &need);
    if (st != PCS_OK) return st;
  }
  if (need > STATIC_BYTES) return PCS_ERR_WORKSPACE;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return PCS_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(static_mu);
  StaticSlot& slot = static_slots[dev];
  if (slot.busy) return PCS_ERR_WORKSPACE;  // another live handle holds this GPU's array
  if (!slot.ptr) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return PCS_ERR_DEVICE;
    slot.ptr = p;
  }
  // the array keeps the previous run's contents: start from zeros
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(hipMemsetAsync(slot.ptr, 0, need, s));
  pcs_sim* sim = new (std::nothrow) pcs_sim();
  if (!sim) return PCS_ERR_ARG;
  sim->b.eager = true;
  const pcs_status st = init_batch(&sim->b, 1, grid, params, &seed, amp, slot.ptr, need, stream);
  if (st != PCS_OK) {
    delete sim;
    return st;
  }
  slot.busy = true;
  sim->static_dev = dev;
  *out = sim;
  return PCS_OK;
}

pcs_status pcs_step(pcs_sim* sim, int32_t nsteps) {
  if (!sim || nsteps < 0) return PCS_ERR_ARG;
  if (sim->m()->blowup) return PCS_ERR_STATE;
  return step_batch(&sim->b, nsteps);
}

pcs_status pcs_diagnostics(pcs_sim* sim, pcs_diag* outp, int32_t max, int32_t* n_out) {
  if (!sim) return PCS_ERR_ARG;
  return member_diagnostics(sim->m(), sim->b.s, outp, max, n_out);
}

pcs_status pcs_state_size(pcs_sim* sim, size_t* n) {
  if (!sim || !n) return PCS_ERR_ARG;
  *n = sim->m()->nstate;
  return PCS_OK;
}

pcs_status pcs_get_state(pcs_sim* sim, double* host, size_t n) {
  if (!sim) return PCS_ERR_ARG;
  return member_get_state(sim->m(), sim->b.s, host, n);
}

pcs_status pcs_set_state(pcs_sim* sim, const double* host, size_t n) {
  if (!sim || !host) return PCS_ERR_ARG;
  return member_set_state(sim->m(), sim->b.s, host, n);
}

}  // extern "C"

namespace {

pcs_status member_set_state(Member* m, hipStream_t s, const double* host, size_t n) {
  if (!host) return PCS_ERR_ARG;
  const size_t base = (size_t)(m->nq + m->nh) * (m->d.N + 1) * m->d.cw;
  // SBDF4 also takes the CNAB2 layout (no earlier states): constant past
  const bool short_form = m->p.scheme == 1 && n == 4 + base;
  if (n != m->nstate && !short_form) return PCS_ERR_ARG;
  for (size_t i = 0; i < 3; ++i)
    if (!std::isfinite(host[i])) return PCS_ERR_ARG;
  // the step index selects ring slots on the device: a whole number in [0, 2^53]
  if (!(host[0] >= 0.0 && host[0] <= 9007199254740992.0) || host[0] != std::floor(host[0])) return PCS_ERR_ARG;
  // the run may still be in use by steps enqueued earlier (an ensemble's other
  // runs, or this run's own steps): finish them first
  HIPCHK(hipStreamSynchronize(s));
  DevScalars sc{};
  sc.step = (long long)host[0];
  sc.t = host[1];
  sc.pi = host[2];
  HIPCHK(hipMemcpyAsync(m->state, host + 4, base * sizeof(double), hipMemcpyHostToDevice, s));
  if (short_form) {
    pcs_status st = sbdf4_cold_start(m, s, sc.step);
    if (st != PCS_OK) return st;
  } else {
    size_t o = 4 + base;
    for (const HistBlock& hb : history_blocks(m, sc.step)) {
      HIPCHK(hipMemcpyAsync(hb.dev, host + o, hb.doubles * sizeof(double), hipMemcpyHostToDevice, s));
      o += hb.doubles;
    }
  }
  HIPCHK(hipMemcpyAsync(m->sc, &sc, sizeof(sc), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  m->drained = sc.step;
  m->blowup = 0;
  return PCS_OK;
}

}  // namespace

extern "C" {

pcs_status pcs_midplane_histogram_setup(pcs_sim* sim, double lo, double hi, int32_t nbins) {
  if (!sim) return PCS_ERR_ARG;
  return member_hist_setup(&sim->b, 0, PCS_PDF_TRC, lo, hi, nbins);
}

pcs_status pcs_midplane_histogram(pcs_sim* sim, uint64_t* counts, int32_t n) {
  if (!sim) return PCS_ERR_ARG;
  return member_hist_get(sim->m(), sim->b.s, PCS_PDF_TRC, counts, n);
}

pcs_status pcs_midplane_pdf_setup(pcs_sim* sim, int32_t quantity, double lo, double hi, int32_t nbins) {
  if (!sim) return PCS_ERR_ARG;
  return member_hist_setup(&sim->b, 0, quantity, lo, hi, nbins);
}

pcs_status pcs_midplane_pdf(pcs_sim* sim, int32_t quantity, uint64_t* counts, int32_t n) {
  if (!sim) return PCS_ERR_ARG;
  return member_hist_get(sim->m(), sim->b.s, quantity, counts, n);
}

pcs_status pcs_midplane_moments(pcs_sim* sim, int32_t quantity, double* out) {
  if (!sim) return PCS_ERR_ARG;
  return member_moments(sim->m(), sim->b.s, quantity, out);
}

pcs_status pcs_y_choice(pcs_sim* sim, pcs_ychoice* out) {
  if (!sim) return PCS_ERR_ARG;
  return batch_y_choice(&sim->b, out);
}

pcs_status batch_stage_times(Batch* b, int32_t nsteps, int32_t reps, double* ms, int32_t nstage) {
  hipEvent_t ev[ST_COUNT + 1];
  for (int i = 0; i <= ST_COUNT; ++i) HIPCHK(hipEventCreate(&ev[i]));
  std::vector<double> acc(ST_COUNT, 0.0);
  pcs_status st = PCS_OK;
  for (int k = 0; k < nsteps && st == PCS_OK; ++k) {
    // the row diagnostics also add the step's midplane samples to the
    // histograms, so they run once per step like the step record
    enqueue_step(b, [&](int i) {
      (void)hipEventRecord(ev[i], b->s);
      return (i == ST_DIAG_FINAL || i == ST_DIAG_ROWS) ? 1 : (int)reps;
    });
    if (hipEventSynchronize(ev[ST_COUNT]) != hipSuccess) {
      st = PCS_ERR_DEVICE;
      break;
    }
    for (int i = 0; i < ST_COUNT; ++i) {
      float t = 0;
      if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) st = PCS_ERR_DEVICE;
      acc[i] += t / ((i == ST_DIAG_FINAL || i == ST_DIAG_ROWS) ? 1 : reps);
    }
  }
  for (int i = 0; i <= ST_COUNT; ++i) (void)hipEventDestroy(ev[i]);
  // stages with no launch in this batch report 0
  bool present[ST_COUNT];
  for (bool& x : present) x = true;
  present[ST_GEMM_MEAN] = b->GSm.n() > 0;
  present[ST_GEMM_STATE] = b->GS.n() > 0;
  present[ST_GEMM_D2] = b->GSb.n() > 0;
  present[ST_ZFFT_INV] = present[ST_ZFFT_FWD] = present[ST_DIAG_ZFFT] = b->dim == 3;
  for (int i = 0; i < ST_COUNT; ++i) ms[i] = present[i] ? acc[i] / nsteps : 0.0;
  for (int i = ST_COUNT; i < nstage; ++i) ms[i] = 0.0;
  return st;
}

pcs_status pcs_stage_times(pcs_sim* sim, int32_t nsteps, int32_t reps, double* ms, int32_t nstage) {
  if (!sim || nsteps <= 0 || reps <= 0 || !ms || nstage < ST_COUNT) return PCS_ERR_ARG;
  if (sim->m()->blowup) return PCS_ERR_STATE;
  return batch_stage_times(&sim->b, nsteps, reps, ms, nstage);
}

const char* pcs_stage_name(int32_t i) { return (i >= 0 && i < ST_COUNT) ? STAGE_NAMES[i] : nullptr; }

pcs_status pcs_destroy(pcs_sim* sim) {
  if (!sim) return PCS_ERR_ARG;
  if (sim->b.s)
    (void)hipStreamSynchronize(sim->b.s);
  else
    (void)hipDeviceSynchronize();
  if (sim->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(static_mu);
    static_slots[sim->static_dev].busy = false;
  }
  delete sim;
  return PCS_OK;
}

pcs_status pcs_ensemble_workspace_bytes(int32_t n, const pcs_grid* grids, const pcs_params* params, size_t* bytes) {
  if (!bytes) return PCS_ERR_ARG;
  Batch b;
  return setup_batch(&b, n, grids, params, bytes);
}

pcs_status pcs_ensemble_init(int32_t n, const pcs_grid* grids, const pcs_params* params, const uint64_t* seeds,
                             double amp, void* workspace, size_t bytes, void* stream, pcs_ens** out) {
  if (!out) return PCS_ERR_ARG;
  *out = nullptr;
  pcs_ens* e = new (std::nothrow) pcs_ens();
  if (!e) return PCS_ERR_ARG;
  const pcs_status st = init_batch(&e->b, n, grids, params, seeds, amp, workspace, bytes, stream);
  if (st != PCS_OK) {
    delete e;
    return st;
  }
  *out = e;
  return PCS_OK;
}

pcs_status pcs_ensemble_step(pcs_ens* e, int32_t nsteps) {
  if (!e || nsteps < 0) return PCS_ERR_ARG;
  return step_batch(&e->b, nsteps);
}

pcs_status pcs_ensemble_diagnostics(pcs_ens* e, int32_t run, pcs_diag* outp, int32_t max, int32_t* n_out) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_diagnostics(e->b.mem[run], e->b.s, outp, max, n_out);
}

pcs_status pcs_ensemble_state_size(pcs_ens* e, int32_t run, size_t* n) {
  if (!e || !n || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  *n = e->b.mem[run]->nstate;
  return PCS_OK;
}

pcs_status pcs_ensemble_get_state(pcs_ens* e, int32_t run, double* host, size_t n) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_get_state(e->b.mem[run], e->b.s, host, n);
}

pcs_status pcs_ensemble_set_state(pcs_ens* e, int32_t run, const double* host, size_t n) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_set_state(e->b.mem[run], e->b.s, host, n);
}

pcs_status pcs_ensemble_run_status(pcs_ens* e, int32_t run) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  Member* m = e->b.mem[run];
  DevScalars sc;
  HIPCHK(hipMemcpyAsync(&sc, m->sc, sizeof(sc), hipMemcpyDeviceToHost, e->b.s));
  HIPCHK(hipStreamSynchronize(e->b.s));
  if (sc.blowup) m->blowup = 1;
  return sc.blowup ? PCS_ERR_STATE : PCS_OK;
}

pcs_status pcs_ensemble_midplane_histogram_setup(pcs_ens* e, int32_t run, double lo, double hi, int32_t nbins) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_hist_setup(&e->b, run, PCS_PDF_TRC, lo, hi, nbins);
}

pcs_status pcs_ensemble_midplane_histogram(pcs_ens* e, int32_t run, uint64_t* counts, int32_t n) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_hist_get(e->b.mem[run], e->b.s, PCS_PDF_TRC, counts, n);
}

pcs_status pcs_ensemble_midplane_pdf_setup(pcs_ens* e, int32_t run, int32_t quantity, double lo, double hi,
                                           int32_t nbins) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_hist_setup(&e->b, run, quantity, lo, hi, nbins);
}

pcs_status pcs_ensemble_midplane_pdf(pcs_ens* e, int32_t run, int32_t quantity, uint64_t* counts, int32_t n) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_hist_get(e->b.mem[run], e->b.s, quantity, counts, n);
}

pcs_status pcs_ensemble_midplane_moments(pcs_ens* e, int32_t run, int32_t quantity, double* out) {
  if (!e || run < 0 || run >= (int32_t)e->b.mem.size()) return PCS_ERR_ARG;
  return member_moments(e->b.mem[run], e->b.s, quantity, out);
}

pcs_status pcs_ensemble_stage_times(pcs_ens* e, int32_t nsteps, int32_t reps, double* ms, int32_t nstage) {
  if (!e || nsteps <= 0 || reps <= 0 || !ms || nstage < ST_COUNT) return PCS_ERR_ARG;
  return batch_stage_times(&e->b, nsteps, reps, ms, nstage);
}

pcs_status pcs_ensemble_y_choice(pcs_ens* e, pcs_ychoice* out) {
  if (!e) return PCS_ERR_ARG;
  return batch_y_choice(&e->b, out);
}

pcs_status pcs_ensemble_destroy(pcs_ens* e) {
  if (!e) return PCS_ERR_ARG;
  if (e->b.s)
    (void)hipStreamSynchronize(e->b.s);
  else
    (void)hipDeviceSynchronize();
  delete e;
  return PCS_OK;
}

const char* pcs_status_string(pcs_status s) {
  switch (s) {
    case PCS_OK: return "ok";
    case PCS_BLOWUP: return "blow-up flagged (non-finite value or |Tr c| > 1e12)";
    case PCS_ERR_ARG: return "invalid argument";
    case PCS_ERR_UNSUPPORTED: return "unsupported size or option";
    case PCS_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
    case PCS_ERR_DEVICE: return "HIP runtime error";
    case PCS_ERR_STATE: return "run has blown up; set a new state first";
    default: return "unknown status";
  }
}

}  // extern "C"
