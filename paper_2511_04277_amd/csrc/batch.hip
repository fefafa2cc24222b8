// Batched radiative pipeline: many open models of uneven size, one or two
// spectral bands each, enforced and solved together.
//
// Enforcement (thesis Sec. 3.5.5) runs all instances in the same grids: the
// tile pairs, row blocks and rows of every instance are concatenated and each
// block finds its instance by a binary search over prefix sums; per-instance
// device flags stop converged instances without host synchronisation.
//
// The Gebhart solves (App. B.2) of all (instance, band) problems advance in
// lockstep through the same two-level block LDU schedule as the single solve;
// at every schedule step one grouped launch carries the diagonal-block
// inverses, or the MFMA GEMM tiles, of every problem that has that step.
// The grouped GEMM is persistent: its grid is capped near the number of
// resident workgroups and each workgroup walks the tile list.
//
// rad_batch_prepare builds the schedule and uploads its descriptor tables
// once; rad_batch_run only launches kernels, so it can be captured in a HIP
// graph and replayed.
#include <cstring>
#include <vector>

#include "emu_split.h"
#include "enforce_kernels.h"
#include "gebhart_kernels.h"

struct rad_batch_plan {
  int count = 0;
  int nprob = 0;
  int precision = RAD_PREC_FP64;
  int kappa = RAD_KAPPA_FRACVAR;
  std::vector<rad_instance> inst;
  size_t work_bytes = 0;
  void* prepared_for = nullptr;
  // filled by layout()
  struct InstOff { size_t ctrl, scale, inv_area, blkmax, finred, partial; int t; long pairs; };
  struct ProbOff { int inst, band, n, np, P2; long ldk, ldy, ldx, ldp, ldw, ldt; size_t kf, dinv, y, x, r, p, sc, w, v, scr;
                   size_t da, db, xa, xb, pa, pb; };
  std::vector<InstOff> io;
  std::vector<ProbOff> po;
  size_t tables_off = 0;
  // launch schedule (table offsets relative to the tables block)
  struct Launch { int kind; int trans; int ts; unsigned grid; size_t off, off2; int count; double flops, bytes; };
  std::vector<Launch> factor, back, fwd, resid;
  size_t off_enf = 0, off_fblk = 0, off_row = 0, off_pd = 0, off_nprow = 0, off_nrow = 0;
  size_t off_pair_map = 0, off_fin_map = 0;
  double sweep_bytes = 0.0;  // algorithmic bytes of one sweep over every instance
  long total_pairs = 0, total_fblk = 0, total_fin = 0, total_rows = 0, total_nprow = 0, total_nrow = 0;
};

namespace rad {
namespace {

enum { L_GJ = 0, L_GEMM = 1, L_COPY = 2, L_TRI_INIT = 3, L_EMU_EXP_KC = 4, L_EMU_EXP_RC = 5, L_EMU_SPLIT_KC = 6,
       L_EMU_SPLIT_RC = 7, L_EMU_GEMM = 8 };

// One operand of the int8-emulated products of a batched launch (the digits
// and exponents of each problem's operands have buffers of their own): the
// operand's rows [0, 64 T), k blocks [0, nkb); part: per-k-block exponents
// of a rows-contiguous operand.
struct EmuJob {
  EmuOperand op;
  int8_t* dig;
  int* ex;
  int* part;
  int T, nkb;
};

// scale exponents, k-contiguous rows: four rows per block
__global__ void __launch_bounds__(256)
b_emu_rowexp_kc(const EmuJob* __restrict__ jobs, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const EmuJob& j = jobs[q];
  emu_rowexp_kc_body(j.op, 0, j.T * EMU_TILE, j.ex, static_cast<int>(blockIdx.x - start[q]));
}

// scale exponents, rows contiguous: one 64-row tile x one k block per block
__global__ void __launch_bounds__(256)
b_emu_rowexp_rc(const EmuJob* __restrict__ jobs, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const EmuJob& j = jobs[q];
  const int b = static_cast<int>(blockIdx.x - start[q]);
  emu_rowexp_rc_body(j.op, b % j.T, b / j.T, j.part, static_cast<long>(j.T) * EMU_TILE);
}

// digits: one 64-row x 64-k block per block
template <bool KC>
__global__ void __launch_bounds__(256)
b_emu_split(const EmuJob* __restrict__ jobs, const long* __restrict__ start, int count) {
  __shared__ double tile[EMU_TILE][EMU_KB + 1];
  const int q = find_segment(start, count, blockIdx.x);
  const EmuJob& j = jobs[q];
  const int b = static_cast<int>(blockIdx.x - start[q]);
  emu_split_body<EMU_S, KC>(j.op, j.T, b % j.T, b / j.T, j.ex, j.part, j.nkb, j.dig, tile);
}

// one row-block copy of a batched launch: rows [0, rows) of src -> dst, cols columns
template <class T>
struct CopyJob {
  const T* src;
  long lds;
  T* dst;
  long ldd;
  int cols;
};

template <class T>
__global__ void __launch_bounds__(256)
b_copy_jobs(const CopyJob<T>* __restrict__ jobs, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const CopyJob<T> j = jobs[q];
  const long i = blockIdx.x - start[q];
  for (int c = threadIdx.x; c < j.cols; c += blockDim.x) j.dst[i * j.ldd + c] = j.src[i * j.lds + c];
}

template <class T>
__global__ void __launch_bounds__(256)
b_tri_init(const TriJob<T>* __restrict__ jobs, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  tri_init_row<T>(jobs[q], static_cast<int>(blockIdx.x - start[q]));
}

struct ProbDesc {
  const double* F;
  long ldf;
  int n, np;
  const double* eps;
  const double* rho;
  double* B;
  long ldb;
  void* kf;
  long ldk;
  void* dinv;
  void* y;
  long ldy;
  double* x;
  double* r;
  long ldx;
  double* p;
  long ldp;
  Scalars* sc;
};

// ------------------------------------------------ row-flat batched kernels ---
template <class T>
__global__ void __launch_bounds__(256)
b_form(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const int i = static_cast<int>(blockIdx.x - start[q]);
  const int n = d.n, np = d.np;
  const double* frow = d.F + static_cast<long>(i) * d.ldf;
  T* krow = static_cast<T*>(d.kf) + static_cast<long>(i) * d.ldk;
  T* yrow = static_cast<T*>(d.y) + static_cast<long>(i) * d.ldy;
  int bad = 0;
  const long jend = d.ldk > d.ldy ? d.ldk : d.ldy;
  for (long j = threadIdx.x; j < jend; j += blockDim.x) {
    double kv = (i == j) ? 1.0 : 0.0;
    double yv = 0.0;
    if (i < n && j <= n) {
      const double f = frow[j];
      bad |= !(f >= 0.0 && f <= 1.0e300);
      if (j < n) {
        kv = kv - f * d.rho[j];
        yv = f * d.eps[j];
      } else {
        yv = f;  // space column: no emissivity factor (eq. B.6)
      }
    }
    if (j < d.ldk) krow[j] = (j < np) ? static_cast<T>(kv) : T(0);
    if (j < d.ldy) yrow[j] = static_cast<T>(yv);
  }
  if (i < n && threadIdx.x == 0) {
    const double e = d.eps[i], r = d.rho[i];
    bad |= !(e >= 0.0 && e <= 1.0 && r >= 0.0 && r <= 1.0);
  }
  if (bad) raise_status(&d.sc->status, RAD_ENONFINITE);
}

__global__ void __launch_bounds__(256)
b_form_p64(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const int i = static_cast<int>(blockIdx.x - start[q]);
  for (long j = threadIdx.x; j < d.ldp; j += blockDim.x)
    d.p[static_cast<long>(i) * d.ldp + j] =
        (i < d.n && j < d.n) ? d.F[static_cast<long>(i) * d.ldf + j] * d.rho[j] : 0.0;
}

// zero the refinement iterate and residual rows (np rows of ldx)
__global__ void __launch_bounds__(256)
b_zero_xr(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const long i = blockIdx.x - start[q];
  for (long j = threadIdx.x; j < d.ldx; j += blockDim.x) {
    d.x[i * d.ldx + j] = 0.0;
    d.r[i * d.ldx + j] = 0.0;
  }
}

// which: 0 = Y(T) -> B, 1 = Y(T) -> X64, 2 = X64 -> B      (rows < n, cols <= n)
template <class T>
__global__ void __launch_bounds__(256)
b_copy(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count, int which) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const long i = blockIdx.x - start[q];
  for (int j = threadIdx.x; j <= d.n; j += blockDim.x) {
    if (which == 2) {
      d.B[i * d.ldb + j] = d.x[i * d.ldx + j];
    } else {
      const double v = static_cast<double>(static_cast<const T*>(d.y)[i * d.ldy + j]);
      if (which == 0) d.B[i * d.ldb + j] = v; else d.x[i * d.ldx + j] = v;
    }
  }
}

__global__ void b_scalars_init(const ProbDesc* __restrict__ pd, int count, int full) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  Scalars* sc = pd[q].sc;
  if (full) sc->status = 0;
  sc->max_r = 0.0;
  sc->max_d = 0.0;
  sc->red[0] = sc->red[1] = 0.0;
}

// R = E - X  (rows < n, cols <= n)
__global__ void __launch_bounds__(256)
b_residual_init(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const long i = blockIdx.x - start[q];
  const double* f = d.F + i * d.ldf;
  for (int j = threadIdx.x; j <= d.n; j += blockDim.x) {
    const double e = (j < d.n) ? f[j] * d.eps[j] : f[d.n];
    d.r[i * d.ldx + j] = e - d.x[i * d.ldx + j];
  }
}

// Y32 <- R, records max |R|
__global__ void __launch_bounds__(256)
b_residual_to_rhs(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const long i = blockIdx.x - start[q];
  float* y = static_cast<float*>(d.y);
  double m = 0.0;
  for (int j = threadIdx.x; j <= d.n; j += blockDim.x) {
    const double v = d.r[i * d.ldx + j];
    m = fmax(m, fabs(v));
    y[i * d.ldy + j] = static_cast<float>(v);
  }
  block_max(m, &d.sc->max_r);
}

// X += Y32, records max |delta|
__global__ void __launch_bounds__(256)
b_apply_correction(const ProbDesc* __restrict__ pd, const long* __restrict__ start, int count) {
  const int q = find_segment(start, count, blockIdx.x);
  const ProbDesc& d = pd[q];
  const long i = blockIdx.x - start[q];
  const float* y = static_cast<const float*>(d.y);
  double m = 0.0;
  for (int j = threadIdx.x; j <= d.n; j += blockDim.x) {
    const double v = static_cast<double>(y[i * d.ldy + j]);
    m = fmax(m, fabs(v));
    d.x[i * d.ldx + j] += v;
  }
  block_max(m, &d.sc->max_d);
}

// persistent grouped GEMM: workgroups walk the concatenated tile list of
// TS x TS tiles
template <class T, bool TRANS_A, int TS>
__global__ void __launch_bounds__(256, TS == GEMM_TILE ? 2 : 4)
gemm_grouped_persistent(const GemmArgs<T>* __restrict__ probs, const int* __restrict__ tile_start, int nprob) {
  // Tiles are taken in list order, so consecutive tiles go to different
  // XCDs: the problems of a launch differ widely in K, and giving each XCD a
  // contiguous range (as for one product) would load some XCDs with all the
  // large problems.
  const int total = tile_start[nprob];
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const int t = b;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const GemmArgs<T>& g = probs[lo];
    int ntx = 0;
    for (int q = 0; q < g.nseg; ++q) ntx += g.N[q] > 0 ? (g.N[q] + TS - 1) / TS : 0;
    int bx, by;
    grouped_tile(t - tile_start[lo], ntx, (g.M + TS - 1) / TS, TILE_GROUP, bx, by);
    gemm_tile<T, TRANS_A, TS, false>(g, bx, by);
  }
}

// The same walk with one 64 x 64 tile per workgroup (grid = all tiles, so the
// hardware hands them out in list order, round robin over the XCDs): without
// the persistent loop the tile keeps its C values in registers across the K
// loop, as the single-product kernel does.
template <class T, bool TRANS_A>
__global__ void __launch_bounds__(256, 4)
gemm_grouped_tiles(const GemmArgs<T>* __restrict__ probs, const int* __restrict__ tile_start, int nprob) {
  const int t = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const GemmArgs<T>& g = probs[lo];
  int ntx = 0;
  for (int q = 0; q < g.nseg; ++q) ntx += g.N[q] > 0 ? (g.N[q] + 63) / 64 : 0;
  int bx, by;
  grouped_tile(t - tile_start[lo], ntx, (g.M + 63) / 64, TILE_GROUP, bx, by);
  gemm_tile<T, TRANS_A, 64, true>(g, bx, by);
}

// resident workgroups of the persistent kernel: two 128-tiles per CU; the
// 64-tile launches take one workgroup per tile
inline unsigned grouped_grid(int ts, int tiles) {
  return ts == GEMM_TILE ? std::min<unsigned>(static_cast<unsigned>(tiles), 2 * 256) : static_cast<unsigned>(tiles);
}

// ------------------------------------------------------------- host side ---
struct TableBuilder {
  std::vector<char> data;
  template <class X>
  size_t add(const X* p, size_t n) {
    size_t off = align_up(data.size(), 256);
    data.resize(off + sizeof(X) * n);
    if (n) std::memcpy(data.data() + off, p, sizeof(X) * n);
    return off;
  }
};

// One grouped GEMM launch over the products a (cleared).  Grouped launches
// take 64 x 64 tiles unless a product is in place: their persistent grids
// hold many problems' tiles at once, where the smaller tile balances better
// (measured on the 64-model batch: 100.5 ms per step vs 107.4 ms with the
// single-product rule).  False if there is no work.
template <class U>
bool gemm_launch(TableBuilder* tb, std::vector<GemmArgs<U>>& a, bool trans, rad_batch_plan::Launch& L) {
  int t128 = 0;
  bool inplace = false;
  double flops = 0.0, bytes = 0.0;
  for (auto& g : a) {
    t128 += gemm_tiles<U>(g);
    inplace = inplace || g.inplace;
    flops += gemm_flops(g);
    bytes += gemm_bytes(g);
  }
  if (t128 == 0) {
    a.clear();
    return false;
  }
  const int ts = inplace ? GEMM_TILE : 64;
  std::vector<int> st(a.size() + 1, 0);
  for (size_t k = 0; k < a.size(); ++k) {
    const GemmArgs<U>& g = a[k];
    const int n = (g.M <= 0 || g.K <= 0) ? 0
                  : (ts == GEMM_TILE ? gemm_tiles<U>(a[k]) : tiles_x<U, 64>(g) * ((g.M + 63) / 64));
    st[k + 1] = st[k] + n;
  }
  L = rad_batch_plan::Launch{};
  L.kind = L_GEMM;
  L.trans = trans ? 1 : 0;
  L.ts = ts;
  L.flops = flops;
  L.bytes = bytes;
  L.count = static_cast<int>(a.size());
  L.off = tb->add(a.data(), a.size());
  L.off2 = tb->add(st.data(), st.size());
  L.grid = grouped_grid(ts, st.back());
  a.clear();
  return true;
}

template <class T>
struct Sched {
  rad_batch_plan* P;
  char* base;
  TableBuilder* tb;
  T* kf(int q) { return reinterpret_cast<T*>(base + P->po[q].kf); }
  T* dinv(int q) { return reinterpret_cast<T*>(base + P->po[q].dinv); }
  T* y(int q) { return reinterpret_cast<T*>(base + P->po[q].y); }
  Scalars* sc(int q) { return reinterpret_cast<Scalars*>(base + P->po[q].sc); }
  T* w(int q) { return reinterpret_cast<T*>(base + P->po[q].w); }
  T* v(int q) { return reinterpret_cast<T*>(base + P->po[q].v); }
  T* scr(int q) { return reinterpret_cast<T*>(base + P->po[q].scr); }
  TriJob<T> tri_job(int q) {
    const auto& o = P->po[q];
    return TriJob<T>{kf(q), o.ldk, dinv(q), o.np, w(q), v(q), o.ldw, scr(q), o.ldt};
  }
  // RAD_PREC_FP64_I8: the K = 1024 products of the outer updates and of the
  // back substitution run as int8 digit products, as in the single solve
  bool emu() const { return P->precision == RAD_PREC_FP64_I8; }
  EmuJob emu_job(const EmuOperand& op, bool is_a, int q) {
    const auto& o = P->po[q];
    return EmuJob{op, reinterpret_cast<int8_t*>(base + (is_a ? o.da : o.db)),
                  reinterpret_cast<int*>(base + (is_a ? o.xa : o.xb)),
                  reinterpret_cast<int*>(base + (is_a ? o.pa : o.pb)), (op.R + EMU_TILE - 1) / EMU_TILE,
                  (op.K + EMU_KB - 1) / EMU_KB};
  }
  // C(i, j) -= op(A) B over all tiles; column j < N0 of C0, then N1 of C1
  static EmuGemmArgs emu_gemm_args(const EmuJob& a, const EmuJob& b, int M, int N0, double* C0, long ldc0, int N1,
                                   double* C1, long ldc1) {
    return EmuGemmArgs{a.dig, a.ex, b.dig, b.ex, a.T, b.T, a.nkb, 0, a.T, 0, b.T, M, -1.0, N1 > 0 ? 2 : 1,
                       {N0, N1}, {C0, C1}, {ldc0, ldc1}};
  }
  void emit_jobs(std::vector<rad_batch_plan::Launch>& out, int kind, size_t off, const std::vector<long>& st,
                 int count, double bytes) {
    rad_batch_plan::Launch L{};
    L.kind = kind;
    L.count = count;
    L.off = off;
    L.off2 = tb->add(st.data(), st.size());
    L.grid = static_cast<unsigned>(st.back());
    L.bytes = bytes;
    out.push_back(L);
  }
  // exponents and digits of every operand, then the products of every problem
  void emit_emu(std::vector<rad_batch_plan::Launch>& out, std::vector<EmuJob>& kc, std::vector<EmuJob>& rc,
                std::vector<EmuGemmArgs>& g, std::vector<double>& flops, std::vector<double>& bytes) {
    for (int kind = 0; kind < 2; ++kind) {
      std::vector<EmuJob>& jobs = kind == 0 ? kc : rc;
      if (jobs.empty()) continue;
      const size_t off = tb->add(jobs.data(), jobs.size());
      const int cnt = static_cast<int>(jobs.size());
      std::vector<long> s_exp(1, 0), s_split(1, 0);
      double elems = 0.0;
      for (const EmuJob& j : jobs) {
        const long rows = static_cast<long>(j.T) * EMU_TILE;
        s_exp.push_back(s_exp.back() + (kind == 0 ? (rows + 3) / 4 : static_cast<long>(j.T) * j.nkb));
        s_split.push_back(s_split.back() + static_cast<long>(j.T) * j.nkb);
        elems += static_cast<double>(j.op.R) * j.op.K;
      }
      // algorithmic bytes of the split as in the single solve: read 8, write 7 per element
      if (kind == 0) {
        emit_jobs(out, L_EMU_EXP_KC, off, s_exp, cnt, 0.0);
        emit_jobs(out, L_EMU_SPLIT_KC, off, s_split, cnt, (8.0 + EMU_S) * elems);
      } else {
        emit_jobs(out, L_EMU_EXP_RC, off, s_exp, cnt, 0.0);
        emit_jobs(out, L_EMU_SPLIT_RC, off, s_split, cnt, (8.0 + EMU_S) * elems);
      }
      jobs.clear();
    }
    if (g.empty()) return;
    std::vector<int> st(g.size() + 1, 0);
    double f = 0.0, b = 0.0;
    for (size_t k = 0; k < g.size(); ++k) {
      st[k + 1] = st[k] + g[k].ntx * g[k].nty;
      f += flops[k];
      b += bytes[k];
    }
    rad_batch_plan::Launch L{};
    L.kind = L_EMU_GEMM;
    L.count = static_cast<int>(g.size());
    L.off = tb->add(g.data(), g.size());
    L.off2 = tb->add(st.data(), st.size());
    L.grid = static_cast<unsigned>(st.back());  // one workgroup per tile
    L.flops = f;
    L.bytes = b;
    if (st.back() > 0) out.push_back(L);
    g.clear();
    flops.clear();
    bytes.clear();
  }
  static double emu_flops(int M, int N, int K) { return 2.0 * M * N * K; }
  static double emu_bytes(int M, int N, int K) { return 16.0 * M * N + EMU_S * (static_cast<double>(M) + N) * K; }
  void emit_rows(std::vector<rad_batch_plan::Launch>& out, int kind, size_t off, std::vector<long>& rs, int count) {
    rad_batch_plan::Launch L{};
    L.kind = kind;
    L.count = count;
    L.off = off;
    L.off2 = tb->add(rs.data(), rs.size());
    L.grid = static_cast<unsigned>(rs.back());
    out.push_back(L);
  }

  void emit_gemm(std::vector<rad_batch_plan::Launch>& out, std::vector<GemmArgs<T>>& a, bool trans) {
    rad_batch_plan::Launch L;
    if (gemm_launch<T>(tb, a, trans, L)) out.push_back(L);
  }
  void emit_gj(std::vector<rad_batch_plan::Launch>& out, std::vector<GjJob<T>>& j) {
    if (j.empty()) return;
    rad_batch_plan::Launch L{};
    L.kind = L_GJ;
    L.count = static_cast<int>(j.size());
    L.grid = static_cast<unsigned>(j.size());
    L.off = tb->add(j.data(), j.size());
    out.push_back(L);
    j.clear();
  }

  int max_panels() {
    int m = 0;
    for (auto& p : P->po) m = std::max(m, static_cast<int>(ceil_div(p.np, NB2)));
    return m;
  }

  // factorization with fused forward elimination (same order as factor_forward)
  void factor() {
    std::vector<GjJob<T>> gj;
    std::vector<GemmArgs<T>> g;
    const int mp = max_panels();
    for (int pan = 0; pan < mp; ++pan) {
      for (int kk = 0; kk < NB2 / NB; ++kk) {
        for (int q = 0; q < P->nprob; ++q) {
          const auto& o = P->po[q];
          const int c0 = pan * NB2;
          if (c0 >= o.np) continue;
          const int c1 = std::min(c0 + NB2, o.np), k0 = c0 + kk * NB;
          if (k0 >= c1) continue;
          gj.push_back(GjJob<T>{kf(q) + static_cast<long>(k0) * o.ldk + k0, o.ldk,
                                dinv(q) + static_cast<long>(k0) * NB, sc(q)});
        }
        emit_gj(P->factor, gj);
        for (int q = 0; q < P->nprob; ++q) {  // X = A21 D^{-1}
          const auto& o = P->po[q];
          const int c0 = pan * NB2;
          if (c0 >= o.np) continue;
          const int c1 = std::min(c0 + NB2, o.np), k0 = c0 + kk * NB, r1 = k0 + NB;
          if (k0 >= c1 || r1 >= o.np) continue;
          T* x = kf(q) + static_cast<long>(r1) * o.ldk + k0;
          GemmArgs<T> a = gemm_args<T>(x, o.ldk, o.np - r1, NB, T(1), T(0));
          gemm_add_segment<T>(a, dinv(q) + static_cast<long>(k0) * NB, NB, x, o.ldk, NB);
          a.inplace = 1;  // X overwrites the A21 it reads
          g.push_back(a);
        }
        emit_gemm(P->factor, g, false);
        for (int q = 0; q < P->nprob; ++q) {  // panel update
          const auto& o = P->po[q];
          const int c0 = pan * NB2;
          if (c0 >= o.np) continue;
          const int c1 = std::min(c0 + NB2, o.np), k0 = c0 + kk * NB, r1 = k0 + NB;
          if (k0 >= c1 || r1 >= c1) continue;
          GemmArgs<T> a = gemm_args<T>(kf(q) + static_cast<long>(r1) * o.ldk + k0, o.ldk, o.np - r1, NB, T(-1),
                                       T(1));
          gemm_add_segment<T>(a, kf(q) + static_cast<long>(k0) * o.ldk + r1, o.ldk,
                              kf(q) + static_cast<long>(r1) * o.ldk + r1, o.ldk, c1 - r1);
          g.push_back(a);
        }
        emit_gemm(P->factor, g, false);
      }
      rows_and_outer(P->factor, pan, true);
    }
  }

  // panel rows right of the panel (block forward substitution) and the
  // K = panel-width update below it; with_k = false updates Y only
  void rows_and_outer(std::vector<rad_batch_plan::Launch>& out, int pan, bool with_k) {
    std::vector<GemmArgs<T>> g;
    for (int kk = 0; kk + 1 < NB2 / NB; ++kk) {
      for (int q = 0; q < P->nprob; ++q) {
        const auto& o = P->po[q];
        const int c0 = pan * NB2;
        if (c0 >= o.np) continue;
        const int c1 = std::min(c0 + NB2, o.np), k0 = c0 + kk * NB, r1 = k0 + NB;
        if (r1 >= c1) continue;
        GemmArgs<T> a =
            gemm_args<T>(kf(q) + static_cast<long>(r1) * o.ldk + k0, o.ldk, c1 - r1, NB, T(-1), T(1));
        if (with_k && c1 < o.np)
          gemm_add_segment<T>(a, kf(q) + static_cast<long>(k0) * o.ldk + c1, o.ldk,
                              kf(q) + static_cast<long>(r1) * o.ldk + c1, o.ldk, o.np - c1);
        gemm_add_segment<T>(a, y(q) + static_cast<long>(k0) * o.ldy, o.ldy, y(q) + static_cast<long>(r1) * o.ldy,
                            o.ldy, o.n + 1);
        g.push_back(a);
      }
      emit_gemm(out, g, false);
    }
    if constexpr (std::is_same<T, double>::value) {
      if (emu() && with_k) {  // L block (k contiguous), then U block and right-hand sides (rows contiguous)
        std::vector<EmuJob> kc, rc;
        std::vector<EmuGemmArgs> eg;
        std::vector<double> ef, eb;
        for (int q = 0; q < P->nprob; ++q) {
          const auto& o = P->po[q];
          const int c0 = pan * NB2;
          if (c0 >= o.np) continue;
          const int c1 = std::min(c0 + NB2, o.np);
          if (c1 >= o.np) continue;
          const int M = o.np - c1, K = c1 - c0;
          const EmuOperand oa{{kf(q) + static_cast<long>(c1) * o.ldk + c0, nullptr}, {o.ldk, 0}, {1, 0}, M, M, K};
          const EmuOperand ob{{kf(q) + static_cast<long>(c0) * o.ldk + c1, y(q) + static_cast<long>(c0) * o.ldy},
                              {1, 1}, {o.ldk, o.ldy}, M, M + o.n + 1, K};
          const EmuJob ja = emu_job(oa, true, q), jb = emu_job(ob, false, q);
          kc.push_back(ja);
          rc.push_back(jb);
          eg.push_back(emu_gemm_args(ja, jb, M, M, kf(q) + static_cast<long>(c1) * o.ldk + c1, o.ldk, o.n + 1,
                                     y(q) + static_cast<long>(c1) * o.ldy, o.ldy));
          ef.push_back(emu_flops(M, M + o.n + 1, K));
          eb.push_back(emu_bytes(M, M + o.n + 1, K));
        }
        emit_emu(out, kc, rc, eg, ef, eb);
        return;
      }
    }
    for (int q = 0; q < P->nprob; ++q) {
      const auto& o = P->po[q];
      const int c0 = pan * NB2;
      if (c0 >= o.np) continue;
      const int c1 = std::min(c0 + NB2, o.np);
      if (c1 >= o.np) continue;
      GemmArgs<T> a = gemm_args<T>(kf(q) + static_cast<long>(c1) * o.ldk + c0, o.ldk, o.np - c1, c1 - c0, T(-1),
                                   T(1));
      if (with_k)
        gemm_add_segment<T>(a, kf(q) + static_cast<long>(c0) * o.ldk + c1, o.ldk,
                            kf(q) + static_cast<long>(c1) * o.ldk + c1, o.ldk, o.np - c1);
      gemm_add_segment<T>(a, y(q) + static_cast<long>(c0) * o.ldy, o.ldy, y(q) + static_cast<long>(c1) * o.ldy,
                          o.ldy, o.n + 1);
      g.push_back(a);
    }
    emit_gemm(out, g, false);
  }

  void forward_only() {
    const int mp = max_panels();
    for (int pan = 0; pan < mp; ++pan) rows_and_outer(P->fwd, pan, false);
  }

  // W_p = U_pp^-1, V_p = L_pp^-1 of every problem's panels (same joins as the
  // single-model tri_level launches)
  void panel_inverses() {
    std::vector<TriJob<T>> jobs;
    std::vector<long> rs(1, 0);
    for (int q = 0; q < P->nprob; ++q) {
      jobs.push_back(tri_job(q));
      rs.push_back(rs.back() + P->po[q].np);
    }
    emit_rows(P->factor, L_TRI_INIT, tb->add(jobs.data(), jobs.size()), rs, P->nprob);
    std::vector<GemmArgs<T>> g;
    for (int b = NB; b < NB2; b *= 2)
      for (int stage = 0; stage < 2; ++stage) {
        for (int q = 0; q < P->nprob; ++q) {
          const TriJob<T> j = tri_job(q);
          for (int p = 0; p < P->po[q].P2; ++p)
            for (int pr = 0; pr < NB2 / (2 * b); ++pr)
              for (int mat = 0; mat < 2; ++mat) {
                GemmArgs<T> a;
                if (tri_level_args<T>(j, b, stage, p, pr, mat, a)) g.push_back(a);
              }
        }
        emit_gemm(P->factor, g, false);
      }
  }

  // back substitution, each problem from its own last panel down:
  // Y_p <- W_p Y_p (through the scratch), then the rows above the panel
  void back() {
    std::vector<GemmArgs<T>> g;
    const int mp = max_panels();
    for (int rp = 0; rp < mp; ++rp) {
      std::vector<CopyJob<T>> cj;
      std::vector<long> rs(1, 0);
      for (int q = 0; q < P->nprob; ++q) {
        const auto& o = P->po[q];
        const int pan = o.P2 - 1 - rp;
        if (pan < 0) continue;
        const int c0 = pan * NB2, L = std::min(c0 + NB2, o.np) - c0;
        GemmArgs<T> a = gemm_args<T>(w(q) + static_cast<long>(pan) * NB2 * o.ldw, o.ldw, L, L, T(1), T(0));
        a.tri = 1;
        gemm_add_segment<T>(a, y(q) + static_cast<long>(c0) * o.ldy, o.ldy, scr(q), o.ldy, o.n + 1);
        g.push_back(a);
        cj.push_back(CopyJob<T>{scr(q), o.ldy, y(q) + static_cast<long>(c0) * o.ldy, o.ldy, o.n + 1});
        rs.push_back(rs.back() + L);
      }
      emit_gemm(P->back, g, false);
      if (!cj.empty()) emit_rows(P->back, L_COPY, tb->add(cj.data(), cj.size()), rs, static_cast<int>(cj.size()));
      if constexpr (std::is_same<T, double>::value) {
        if (emu()) {  // rows above the panel: U's column block (k contiguous) times the panel's rows of Y
          std::vector<EmuJob> kc, rc;
          std::vector<EmuGemmArgs> eg;
          std::vector<double> ef, eb;
          for (int q = 0; q < P->nprob; ++q) {
            const auto& o = P->po[q];
            const int pan = o.P2 - 1 - rp;
            if (pan <= 0) continue;
            const int c0 = pan * NB2, c1 = std::min(c0 + NB2, o.np), K = c1 - c0;
            const EmuOperand oa{{kf(q) + c0, nullptr}, {o.ldk, 0}, {1, 0}, c0, c0, K};
            const EmuOperand ob{{y(q) + static_cast<long>(c0) * o.ldy, nullptr}, {1, 0}, {o.ldy, 0}, o.n + 1,
                                o.n + 1, K};
            const EmuJob ja = emu_job(oa, true, q), jb = emu_job(ob, false, q);
            kc.push_back(ja);
            rc.push_back(jb);
            eg.push_back(emu_gemm_args(ja, jb, c0, o.n + 1, y(q), o.ldy, 0, nullptr, 0));
            ef.push_back(emu_flops(c0, o.n + 1, K));
            eb.push_back(emu_bytes(c0, o.n + 1, K));
          }
          emit_emu(P->back, kc, rc, eg, ef, eb);
          continue;
        }
      }
      for (int q = 0; q < P->nprob; ++q) {  // rows above the panel
        const auto& o = P->po[q];
        const int pan = o.P2 - 1 - rp;
        if (pan <= 0) continue;
        const int c0 = pan * NB2, c1 = std::min(c0 + NB2, o.np);
        GemmArgs<T> a = gemm_args<T>(kf(q) + c0, o.ldk, c0, c1 - c0, T(-1), T(1));
        gemm_add_segment<T>(a, y(q) + static_cast<long>(c0) * o.ldy, o.ldy, y(q), o.ldy, o.n + 1);
        g.push_back(a);
      }
      emit_gemm(P->back, g, false);
    }
  }

  void residual() {
    std::vector<GemmArgs<double>> g;
    for (int q = 0; q < P->nprob; ++q) {
      const auto& o = P->po[q];
      double* p = reinterpret_cast<double*>(base + o.p);
      double* x = reinterpret_cast<double*>(base + o.x);
      double* r = reinterpret_cast<double*>(base + o.r);
      GemmArgs<double> a = gemm_args<double>(p, o.ldp, o.n, static_cast<int>(ceil_div(o.n, 32) * 32), 1.0, 1.0);
      gemm_add_segment<double>(a, x, o.ldx, r, o.ldx, o.n + 1);
      g.push_back(a);
    }
    rad_batch_plan::Launch L;
    if (!gemm_launch<double>(tb, g, false, L)) return;
    P->resid.push_back(L);
  }
};

size_t elem(int prec) { return prec == RAD_PREC_FP32_IR ? 4 : 8; }

// buffer layout of the workspace (tables come last, see build_tables)
void layout(rad_batch_plan* P) {
  size_t used = 0;
  auto take = [&](size_t bytes) {
    const size_t off = align_up(used, 256);
    used = off + align_up(bytes, 256);
    return off;
  };
  P->io.clear();
  P->po.clear();
  for (int i = 0; i < P->count; ++i) {
    const size_t n = static_cast<size_t>(P->inst[i].n);
    rad_batch_plan::InstOff o{};
    o.t = static_cast<int>(ceil_div(static_cast<int64_t>(n), 64));
    o.pairs = static_cast<long>(o.t) * (o.t + 1) / 2;
    o.ctrl = take(sizeof(EnfCtrl));
    o.scale = take(n * sizeof(double));
    o.inv_area = take(n * sizeof(double));
    o.blkmax = take(2 * static_cast<size_t>(o.pairs) * sizeof(double));
    o.finred = take(3 * static_cast<size_t>(fin_blocks(static_cast<int64_t>(n))) * sizeof(double));
    o.partial = take(static_cast<size_t>(o.t + 1) * n * sizeof(double));
    P->io.push_back(o);
  }
  const size_t es = elem(P->precision);
  for (int i = 0; i < P->count; ++i) {
    for (int b = 0; b < P->inst[i].bands; ++b) {
      rad_batch_plan::ProbOff o{};
      o.inst = i;
      o.band = b;
      o.n = static_cast<int>(P->inst[i].n);
      o.np = static_cast<int>(ceil_div(o.n, NB) * NB);
      o.ldk = static_cast<long>(o.np + 128 / es);
      o.ldy = rhs_ld(o.n, static_cast<long>(128 / es));
      o.ldx = rhs_ld(o.n, pad_elems<double>());
      o.ldp = static_cast<long>(o.np + pad_elems<double>());
      o.kf = take(static_cast<size_t>(o.np) * o.ldk * es);
      o.dinv = take(static_cast<size_t>(o.np / NB) * NB * NB * es);
      o.y = take(static_cast<size_t>(o.np) * o.ldy * es);
      o.sc = take(sizeof(Scalars));
      o.P2 = static_cast<int>(ceil_div(o.np, NB2));
      o.ldw = static_cast<long>(NB2 + 128 / es);
      o.ldt = tri_ldt(static_cast<long>(128 / es));
      o.w = take(static_cast<size_t>(o.P2) * NB2 * o.ldw * es);
      o.v = take(static_cast<size_t>(o.P2) * NB2 * o.ldw * es);
      o.scr = take(std::max(static_cast<size_t>(NB2) * o.ldy, tri_tmp_elems(o.P2, static_cast<long>(128 / es))) * es);
      if (P->precision == RAD_PREC_FP64_I8 && o.np > NB2) {  // operands of the emulated K = 1024 products
        const long rb = static_cast<long>(o.np) + o.n + 1;
        o.da = take(emu_digit_bytes(o.np, NB2));
        o.db = take(emu_digit_bytes(rb, NB2));
        o.xa = take(emu_scale_count(o.np) * sizeof(int));
        o.xb = take(emu_scale_count(rb) * sizeof(int));
        o.pa = take(emu_part_count(o.np, NB2) * sizeof(int));
        o.pb = take(emu_part_count(rb, NB2) * sizeof(int));
      }
      if (P->precision == RAD_PREC_FP32_IR) {
        o.x = take(static_cast<size_t>(o.np) * o.ldx * 8);
        o.r = take(static_cast<size_t>(o.np) * o.ldx * 8);
        o.p = take(static_cast<size_t>(o.np) * o.ldp * 8);
      }
      P->po.push_back(o);
    }
  }
  P->nprob = static_cast<int>(P->po.size());
  P->tables_off = align_up(used, 256);
}

// descriptor tables and schedule for a workspace at `base` (may be null to size them)
void build_tables(rad_batch_plan* P, char* base, TableBuilder& tb) {
  P->factor.clear();
  P->sweep_bytes = 0.0;
  P->back.clear();
  P->fwd.clear();
  P->resid.clear();
  // enforcement instances
  std::vector<EnfInst> ei;
  std::vector<long> pair_start(1, 0), fblk_start(1, 0), fin_start(1, 0), row_start(1, 0);
  for (int i = 0; i < P->count; ++i) {
    const rad_instance& s = P->inst[i];
    const auto& o = P->io[i];
    EnfInst e{};
    e.F = s.F;
    e.ldf = static_cast<long>(s.ldf);
    e.n = static_cast<int>(s.n);
    e.t = o.t;
    e.pairs = o.pairs;
    e.area = s.area;
    e.inv_area = reinterpret_cast<double*>(base + o.inv_area);
    e.nrays = s.n_rays;
    e.mode = P->kappa;
    e.scale = reinterpret_cast<double*>(base + o.scale);
    e.partial = reinterpret_cast<double*>(base + o.partial);
    e.blkmax = reinterpret_cast<double*>(base + o.blkmax);
    e.finred = reinterpret_cast<double*>(base + o.finred);
    e.ctrl = reinterpret_cast<EnfCtrl*>(base + o.ctrl);
    ei.push_back(e);
    pair_start.push_back(pair_start.back() + o.pairs);
    fblk_start.push_back(fblk_start.back() + ceil_div(s.n, 256));
    fin_start.push_back(fin_start.back() + fin_blocks(s.n));
    row_start.push_back(row_start.back() + s.n);
    P->sweep_bytes += 16.0 * static_cast<double>(s.n) * (s.n + 1);
  }
  P->total_pairs = pair_start.back();
  P->total_fblk = fblk_start.back();
  P->total_fin = fin_start.back();
  P->total_rows = row_start.back();
  P->off_enf = tb.add(ei.data(), ei.size());
  {
    // block maps of the batched sweep (tile pairs) and finalize (row blocks)
    std::vector<EnfBlk> pm, fm;
    pm.reserve(static_cast<size_t>(P->total_pairs));
    fm.reserve(static_cast<size_t>(P->total_fin));
    for (int i = 0; i < P->count; ++i) {
      for (long b = 0; b < pair_start[i + 1] - pair_start[i]; ++b) pm.push_back(EnfBlk{i, static_cast<int>(b)});
      for (long b = 0; b < fin_start[i + 1] - fin_start[i]; ++b) fm.push_back(EnfBlk{i, static_cast<int>(b)});
    }
    P->off_pair_map = tb.add(pm.data(), pm.size());
    P->off_fin_map = tb.add(fm.data(), fm.size());
  }
  P->off_fblk = tb.add(fblk_start.data(), fblk_start.size());
  P->off_row = tb.add(row_start.data(), row_start.size());
  // solve problems
  std::vector<ProbDesc> pd;
  std::vector<long> nprow(1, 0), nrow(1, 0);
  for (int q = 0; q < P->nprob; ++q) {
    const auto& o = P->po[q];
    const rad_instance& s = P->inst[o.inst];
    ProbDesc d{};
    d.F = s.F;
    d.ldf = static_cast<long>(s.ldf);
    d.n = o.n;
    d.np = o.np;
    d.eps = s.eps[o.band];
    d.rho = s.rho[o.band];
    d.B = s.B[o.band];
    d.ldb = static_cast<long>(s.ldb[o.band]);
    d.kf = base + o.kf;
    d.ldk = o.ldk;
    d.dinv = base + o.dinv;
    d.y = base + o.y;
    d.ldy = o.ldy;
    d.x = reinterpret_cast<double*>(base + o.x);
    d.r = reinterpret_cast<double*>(base + o.r);
    d.ldx = o.ldx;
    d.p = reinterpret_cast<double*>(base + o.p);
    d.ldp = o.ldp;
    d.sc = reinterpret_cast<Scalars*>(base + o.sc);
    pd.push_back(d);
    nprow.push_back(nprow.back() + o.np);
    nrow.push_back(nrow.back() + o.n);
  }
  P->total_nprow = nprow.back();
  P->total_nrow = nrow.back();
  P->off_pd = tb.add(pd.data(), pd.size());
  P->off_nprow = tb.add(nprow.data(), nprow.size());
  P->off_nrow = tb.add(nrow.data(), nrow.size());
  if (P->precision != RAD_PREC_FP32_IR) {
    Sched<double> sch{P, base, &tb};
    sch.factor();
    sch.panel_inverses();
    sch.back();
  } else {
    Sched<float> sch{P, base, &tb};
    sch.factor();
    sch.panel_inverses();
    sch.back();
    sch.forward_only();
    sch.residual();
  }
}

template <class T>
hipError_t run_launches(const std::vector<rad_batch_plan::Launch>& ls, const char* tables, hipStream_t s) {
  for (const auto& L : ls) {
    if (L.kind >= L_EMU_EXP_KC && L.kind <= L_EMU_SPLIT_RC) {
      const EmuJob* jobs = reinterpret_cast<const EmuJob*>(tables + L.off);
      const long* st = reinterpret_cast<const long*>(tables + L.off2);
      ProfScope prof(s, RAD_PROF_I8X_SPLIT, 0.0, L.bytes);
      if (L.kind == L_EMU_EXP_KC)
        hipLaunchKernelGGL(b_emu_rowexp_kc, dim3(L.grid), dim3(256), 0, s, jobs, st, L.count);
      else if (L.kind == L_EMU_EXP_RC)
        hipLaunchKernelGGL(b_emu_rowexp_rc, dim3(L.grid), dim3(256), 0, s, jobs, st, L.count);
      else if (L.kind == L_EMU_SPLIT_KC)
        hipLaunchKernelGGL(b_emu_split<true>, dim3(L.grid), dim3(256), 0, s, jobs, st, L.count);
      else
        hipLaunchKernelGGL(b_emu_split<false>, dim3(L.grid), dim3(256), 0, s, jobs, st, L.count);
    } else if (L.kind == L_EMU_GEMM) {
      ProfScope prof(s, RAD_PROF_GEMM_I8X, L.flops, L.bytes);
      hipLaunchKernelGGL(emu_gemm_grouped_tiles<EMU_S>, dim3(L.grid), dim3(EMU_THREADS), 0, s,
                         reinterpret_cast<const EmuGemmArgs*>(tables + L.off),
                         reinterpret_cast<const int*>(tables + L.off2), L.count);
    } else if (L.kind == L_COPY) {
      hipLaunchKernelGGL(b_copy_jobs<T>, dim3(L.grid), dim3(256), 0, s,
                         reinterpret_cast<const CopyJob<T>*>(tables + L.off),
                         reinterpret_cast<const long*>(tables + L.off2), L.count);
    } else if (L.kind == L_TRI_INIT) {
      hipLaunchKernelGGL(b_tri_init<T>, dim3(L.grid), dim3(256), 0, s,
                         reinterpret_cast<const TriJob<T>*>(tables + L.off),
                         reinterpret_cast<const long*>(tables + L.off2), L.count);
    } else if (L.kind == L_GJ) {
      ProfScope prof(s, RAD_PROF_DIAG_INVERSE, 2.0 * NB * NB * NB * L.count, 0.0);
      hipLaunchKernelGGL(gj_batched<T>, dim3(L.grid), dim3(GJ_THREADS), 0, s,
                         reinterpret_cast<const GjJob<T>*>(tables + L.off));
    } else {
      ProfScope prof(s, gemm_prof_kind<T>(L.trans != 0), L.flops, L.bytes);
      const GemmArgs<T>* a = reinterpret_cast<const GemmArgs<T>*>(tables + L.off);
      const int* ts = reinterpret_cast<const int*>(tables + L.off2);
      if (L.ts == GEMM_TILE) {
        if (L.trans)
          hipLaunchKernelGGL((gemm_grouped_persistent<T, true, GEMM_TILE>), dim3(L.grid), dim3(256), 0, s, a, ts,
                             L.count);
        else
          hipLaunchKernelGGL((gemm_grouped_persistent<T, false, GEMM_TILE>), dim3(L.grid), dim3(256), 0, s, a, ts,
                             L.count);
      } else {
        if (L.trans)
          hipLaunchKernelGGL((gemm_grouped_tiles<T, true>), dim3(L.grid), dim3(256), 0, s, a, ts, L.count);
        else
          hipLaunchKernelGGL((gemm_grouped_tiles<T, false>), dim3(L.grid), dim3(256), 0, s, a, ts, L.count);
      }
    }
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" int32_t rad_batch_plan_create(const rad_instance* inst, int32_t count, int32_t precision,
                                         int32_t kappa_mode, rad_batch_plan** plan, size_t* work_bytes) {
  ApiRange range("rad_batch_plan_create");
  clear_error();
  RAD_REQUIRE(plan && work_bytes, RAD_EINVAL, "rad_batch_plan_create: NULL output");
  *plan = nullptr;
  RAD_REQUIRE(inst && count >= 1 && count <= (1 << 16), RAD_EINVAL, "rad_batch_plan_create: bad instance list");
  RAD_REQUIRE(precision == RAD_PREC_FP64 || precision == RAD_PREC_FP32_IR || precision == RAD_PREC_FP64_I8,
              RAD_EINVAL, "rad_batch_plan_create: unknown precision");
  RAD_REQUIRE(kappa_mode == RAD_KAPPA_FRACVAR || kappa_mode == RAD_KAPPA_HALF, RAD_EINVAL,
              "rad_batch_plan_create: unknown kappa_mode");
  for (int i = 0; i < count; ++i) {
    const rad_instance& s = inst[i];
    RAD_REQUIRE(s.n >= 1 && s.n <= (1 << 20) && s.ldf >= s.n + 1 && s.F && s.area, RAD_EINVAL,
                "rad_batch_plan_create: instance with bad n, ldf, F or area");
    RAD_REQUIRE(kappa_mode == RAD_KAPPA_HALF || s.n_rays, RAD_EINVAL,
                "rad_batch_plan_create: n_rays required for RAD_KAPPA_FRACVAR");
    RAD_REQUIRE(s.bands == 1 || s.bands == 2, RAD_EINVAL, "rad_batch_plan_create: bands must be 1 or 2");
    for (int b = 0; b < s.bands; ++b)
      RAD_REQUIRE(s.eps[b] && s.rho[b] && s.B[b] && s.ldb[b] >= s.n + 1, RAD_EINVAL,
                  "rad_batch_plan_create: band with NULL eps/rho/B or ldb < n+1");
  }
  rad_batch_plan* P = new rad_batch_plan();
  P->count = count;
  P->precision = precision;
  P->kappa = kappa_mode;
  P->inst.assign(inst, inst + count);
  layout(P);
  TableBuilder tb;
  // table sizes do not depend on the workspace address; size them at a dummy one
  build_tables(P, reinterpret_cast<char*>(static_cast<uintptr_t>(1) << 24), tb);
  P->work_bytes = P->tables_off + align_up(tb.data.size(), 256);
  *plan = P;
  *work_bytes = P->work_bytes;
  return RAD_OK;
}

extern "C" void rad_batch_plan_destroy(rad_batch_plan* plan) { delete plan; }

extern "C" int32_t rad_batch_prepare(rad_batch_plan* P, void* work, size_t work_bytes, void* stream) {
  ApiRange range("rad_batch_prepare");
  clear_error();
  RAD_REQUIRE(P, RAD_EINVAL, "rad_batch_prepare: NULL plan");
  RAD_REQUIRE(work && work_bytes >= P->work_bytes && reinterpret_cast<uintptr_t>(work) % 256 == 0,
              RAD_EWORKSPACE, "rad_batch_prepare: workspace too small or not 256-byte aligned");
  TableBuilder tb;
  build_tables(P, static_cast<char*>(work), tb);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RAD_HIP_CHECK(hipMemcpyAsync(static_cast<char*>(work) + P->tables_off, tb.data.data(), tb.data.size(),
                               hipMemcpyHostToDevice, s));
  RAD_HIP_CHECK(hipStreamSynchronize(s));
  P->prepared_for = work;
  return RAD_OK;
}

extern "C" int32_t rad_batch_run(const rad_batch_plan* P, void* work, double enforce_tol, int32_t enforce_iters,
                                 int32_t ir_steps, void* stream) {
  ApiRange range("rad_batch_run");
  clear_error();
  RAD_REQUIRE(P && work, RAD_EINVAL, "rad_batch_run: NULL plan or workspace");
  RAD_REQUIRE(P->prepared_for == work, RAD_EINVAL, "rad_batch_run: workspace was not prepared with this plan");
  RAD_REQUIRE(enforce_iters >= 0 && ir_steps >= 0 && enforce_tol >= 0.0, RAD_EINVAL,
              "rad_batch_run: negative iteration count or tolerance");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const char* tables = static_cast<const char*>(work) + P->tables_off;
  const EnfInst* ei = reinterpret_cast<const EnfInst*>(tables + P->off_enf);
  const long* fblk_start = reinterpret_cast<const long*>(tables + P->off_fblk);
  const EnfBlk* pair_map = reinterpret_cast<const EnfBlk*>(tables + P->off_pair_map);
  const EnfBlk* fin_map = reinterpret_cast<const EnfBlk*>(tables + P->off_fin_map);
  const long* row_start = reinterpret_cast<const long*>(tables + P->off_row);
  const ProbDesc* pd = reinterpret_cast<const ProbDesc*>(tables + P->off_pd);
  const long* nprow = reinterpret_cast<const long*>(tables + P->off_nprow);
  const long* nrow = reinterpret_cast<const long*>(tables + P->off_nrow);
  const int C = P->count, Q = P->nprob;
  const unsigned cb = static_cast<unsigned>(ceil_div(C, 64)), qb = static_cast<unsigned>(ceil_div(Q, 64));
  // ---- enforcement of every instance (fixed launches, device-side stop)
  hipLaunchKernelGGL(enf_init_batched, dim3(cb), dim3(64), 0, s, ei, C);
  if (enforce_iters > 0) {
    hipLaunchKernelGGL(enf_inv_area_batched, dim3(static_cast<unsigned>(P->total_fblk)), dim3(256), 0, s, ei,
                       fblk_start, C);
    for (int it = 0; it < enforce_iters; ++it) {
      {
        ProfScope prof(s, RAD_PROF_ENFORCE_SWEEP, 0.0, P->sweep_bytes);
        hipLaunchKernelGGL(enf_sweep_batched, dim3(static_cast<unsigned>(P->total_pairs)), dim3(ENF_THREADS), 0, s,
                           ei, pair_map, it == 0 ? 1 : 0);
      }
      hipLaunchKernelGGL(enf_finalize_batched, dim3(static_cast<unsigned>(P->total_fin)), dim3(256), 0, s, ei,
                         fin_map, enforce_tol);
    }
    hipLaunchKernelGGL(enf_apply_scale_batched, dim3(static_cast<unsigned>(P->total_rows)), dim3(256), 0, s, ei,
                       row_start, C);
  }
  // ---- Gebhart solves of every (instance, band)
  hipLaunchKernelGGL(b_scalars_init, dim3(qb), dim3(64), 0, s, pd, Q, 1);
  const unsigned npr = static_cast<unsigned>(P->total_nprow), nr = static_cast<unsigned>(P->total_nrow);
  if (P->precision != RAD_PREC_FP32_IR) {
    hipLaunchKernelGGL(b_form<double>, dim3(npr), dim3(256), 0, s, pd, nprow, Q);
    RAD_HIP_CHECK(run_launches<double>(P->factor, tables, s));
    RAD_HIP_CHECK(run_launches<double>(P->back, tables, s));
    hipLaunchKernelGGL(b_copy<double>, dim3(nr), dim3(256), 0, s, pd, nrow, Q, 0);
  } else {
    hipLaunchKernelGGL(b_form<float>, dim3(npr), dim3(256), 0, s, pd, nprow, Q);
    RAD_HIP_CHECK(run_launches<float>(P->factor, tables, s));
    RAD_HIP_CHECK(run_launches<float>(P->back, tables, s));
    if (ir_steps == 0) {
      hipLaunchKernelGGL(b_copy<float>, dim3(nr), dim3(256), 0, s, pd, nrow, Q, 0);
    } else {
      hipLaunchKernelGGL(b_zero_xr, dim3(npr), dim3(256), 0, s, pd, nprow, Q);
      hipLaunchKernelGGL(b_form_p64, dim3(npr), dim3(256), 0, s, pd, nprow, Q);
      hipLaunchKernelGGL(b_copy<float>, dim3(nr), dim3(256), 0, s, pd, nrow, Q, 1);
      for (int st = 0; st < ir_steps; ++st) {
        hipLaunchKernelGGL(b_scalars_init, dim3(qb), dim3(64), 0, s, pd, Q, 0);
        hipLaunchKernelGGL(b_residual_init, dim3(nr), dim3(256), 0, s, pd, nrow, Q);
        RAD_HIP_CHECK(run_launches<double>(P->resid, tables, s));
        hipLaunchKernelGGL(b_residual_to_rhs, dim3(nr), dim3(256), 0, s, pd, nrow, Q);
        RAD_HIP_CHECK(run_launches<float>(P->fwd, tables, s));
        RAD_HIP_CHECK(run_launches<float>(P->back, tables, s));
        hipLaunchKernelGGL(b_apply_correction, dim3(nr), dim3(256), 0, s, pd, nrow, Q);
      }
      hipLaunchKernelGGL(b_copy<float>, dim3(nr), dim3(256), 0, s, pd, nrow, Q, 2);
    }
  }
  RAD_HIP_CHECK(hipGetLastError());
  return RAD_OK;
}

extern "C" int32_t rad_batch_stats(const rad_batch_plan* P, const void* work, rad_stats* out, void* stream) {
  ApiRange range("rad_batch_stats");
  clear_error();
  RAD_REQUIRE(P && work && out, RAD_EINVAL, "rad_batch_stats: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const char* base = static_cast<const char*>(work);
  std::vector<EnfCtrl> ec(P->count);
  std::vector<Scalars> sc(P->nprob);
  for (int i = 0; i < P->count; ++i)
    RAD_HIP_CHECK(hipMemcpyAsync(&ec[i], base + P->io[i].ctrl, sizeof(EnfCtrl), hipMemcpyDeviceToHost, s));
  for (int q = 0; q < P->nprob; ++q)
    RAD_HIP_CHECK(hipMemcpyAsync(&sc[q], base + P->po[q].sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  RAD_HIP_CHECK(hipStreamSynchronize(s));
  int32_t worst = RAD_OK;
  for (int i = 0; i < P->count; ++i) {
    rad_stats& o = out[i];
    o = rad_stats{};
    o.iters = ec[i].iters;
    o.converged = ec[i].converged;
    o.closure_defect = ec[i].last_defect;
    o.recip_err = ec[i].last_recip;
    o.device_status = ec[i].status;
  }
  for (int q = 0; q < P->nprob; ++q) {
    rad_stats& o = out[P->po[q].inst];
    o.device_status = std::min(o.device_status, sc[q].status);
    o.ir_correction = std::max(o.ir_correction, sc[q].max_d);
    o.ir_residual = std::max(o.ir_residual, sc[q].max_r);
  }
  for (int i = 0; i < P->count; ++i) worst = std::min(worst, out[i].device_status);
  if (worst < 0) set_error("rad_batch_stats: an instance reported a device-side error (see device_status)");
  return worst;
}
