// Multi-node aggregation (thesis Sec. 5.2.3, eq. 5.6-5.7; first two rows of
// eq. 5.28 for one-sided faces) as one read of the sub-face matrix.
//
//   csr_rank, csr_offsets, csr_scatter: stable counting sort of the group map
//               into member lists (each group's members in increasing index
//               order), so every later sum runs in a fixed order.
//   agg_reduce: workgroup = (row group G, chunk of 256 column groups H); each
//               thread owns one output Y_GH and sums w_i X_ij over i in G,
//               j in H in member order, then divides by W_G.
#include <algorithm>

#include "common.h"

namespace rad {
namespace {

constexpr int CSR_CHUNK = 1024;   // indices per rank block
constexpr int AGG_THREADS = 256;

// Stable counting sort of the group map in three passes.  (1) One block per
// chunk of CSR_CHUNK indices: each index's rank among equal ids earlier in
// its chunk, and the chunk's count per group.  (2) One block: per group, the
// offset of each chunk's run (chunks in order) and the group offsets (scan
// over groups).  (3) Scatter: index i goes to
// offs[g_i] + chunk_off[chunk][g_i] + rank_i, so members appear in
// increasing index order and every later sum runs in a fixed order.
__global__ void __launch_bounds__(CSR_CHUNK)
csr_rank(const int* __restrict__ group, int n, int g, int* __restrict__ rank, int* __restrict__ cnt,
         int* __restrict__ status) {
  __shared__ __align__(16) int chunk[CSR_CHUNK];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int i = c * CSR_CHUNK + tid;
  int gi = i < n ? group[i] : -1;
  if (i < n && (gi < 0 || gi >= g)) {
    atomicMin(status, RAD_EINVAL);
    gi = -1;
  }
  chunk[tid] = gi;
  __syncthreads();
  if (gi < 0) return;
  // equal ids before tid in the chunk; the loop bound (a multiple of 64) is
  // the same for every lane of a wave (no divergence), four ids per LDS read
  // and four reads in flight
  const int qend = (tid | 63) + 1;
  int r = 0;
  for (int q0 = 0; q0 < qend; q0 += 16) {
    int4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const int4*>(&chunk[q0 + 4 * u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + 4 * u;
      r += (v[u].x == gi && q < tid) + (v[u].y == gi && q + 1 < tid) + (v[u].z == gi && q + 2 < tid) +
           (v[u].w == gi && q + 3 < tid);
    }
  }
  rank[i] = r;
  atomicMax(&cnt[static_cast<long>(c) * g + gi], r + 1);  // the chunk's count of gi (cnt starts at zero)
}

// one block: cnt (nch x g, zero where a group is absent from a chunk) becomes
// the chunk offsets in place; offs[G] = sum of the counts of groups < G.
// Thread t takes the groups G = t, t + 1024, ... (coalesced), eight chunk
// counts in flight at a time; the group totals are scanned by the block in
// rounds of 1024 groups.
__global__ void __launch_bounds__(1024)
csr_offsets(int* __restrict__ cnt, int nch, int g, int* __restrict__ offs, int* __restrict__ status) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int carry = 0;
  for (int G0 = 0; G0 < g; G0 += 1024) {
    const int G = G0 + tid;
    int run = 0;
    if (G < g) {
      for (int c0 = 0; c0 < nch; c0 += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cnt[static_cast<long>(min(c0 + u, nch - 1)) * g + G];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (c0 + u < nch) {
            cnt[static_cast<long>(c0 + u) * g + G] = run;
            run += v[u];
          }
      }
      if (run == 0) atomicMin(status, RAD_EINVAL);  // empty group
    }
    int x = run;  // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (tid < 64) {  // inclusive scan of the 16 wave totals
      int t = tid < 16 ? wsum[tid] : 0;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const int y = __shfl_up(t, off);
        if (lane >= off) t += y;
      }
      if (tid < 16) wsum[tid] = t;
    }
    __syncthreads();
    if (G < g) offs[G] = carry + (wv > 0 ? wsum[wv - 1] : 0) + x - run;
    carry += wsum[15];
    __syncthreads();  // wsum is rewritten in the next round
  }
  if (tid == 0) offs[g] = carry;
}

__global__ void __launch_bounds__(256)
csr_scatter(const int* __restrict__ group, int n, int g, const int* __restrict__ rank,
            const int* __restrict__ cnt, const int* __restrict__ offs, int* __restrict__ members) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int gi = group[i];
  if (gi < 0 || gi >= g) return;
  const int c = i / CSR_CHUNK;
  members[offs[gi] + cnt[static_cast<long>(c) * g + gi] + rank[i]] = i;
}

__global__ void __launch_bounds__(AGG_THREADS)
agg_reduce(const double* __restrict__ X, long ldx, int n, const double* __restrict__ w,
           const int* __restrict__ offs, const int* __restrict__ members, int g,
           double* __restrict__ Y, long ldy, double* __restrict__ gw, int divide) {
  const int G = blockIdx.y;
  const int H = blockIdx.x * AGG_THREADS + threadIdx.x;  // output column (g == space)
  const int rb = offs[G], re = offs[G + 1];
  double wsum = 0.0;
  for (int a = rb; a < re; ++a) wsum += w[members[a]];
  if (H > g) return;
  double acc = 0.0;
  if (H == g) {
    for (int a = rb; a < re; ++a) {
      int i = members[a];
      acc += w[i] * X[static_cast<long>(i) * ldx + n];
    }
  } else {
    const int cb = offs[H], ce = offs[H + 1];
    for (int a = rb; a < re; ++a) {
      int i = members[a];
      const double* row = X + static_cast<long>(i) * ldx;
      double s = 0.0;
      for (int b = cb; b < ce; ++b) s += row[members[b]];
      acc += w[i] * s;
    }
  }
  Y[static_cast<long>(G) * ldy + H] = divide ? acc / wsum : acc;
  if (gw && H == 0) gw[G] = wsum;
}

// The same sums with one workgroup per row group G and each member row of G
// staged whole in LDS: the row is read once with coalesced loads, and the
// column groups' gathers hit LDS instead of scattered HBM lines.  Thread t
// owns the outputs H = t, t + AGGL_THREADS, ... (at most HPT of them) in
// registers; every sum runs in the same member order as agg_reduce, so both
// give the same bits.  Used when a row of X fits in AGGL_MAX_LDS.
constexpr int AGGL_THREADS = 512;
constexpr size_t AGGL_MAX_LDS = 150 * 1024;

// One or two weightings of the same sums (NWT): the column-group sums
// sum_{j in H} X_ij are formed once per member row and enter both outputs,
// each in the same order and with the same rounding as a call of its own.
struct AggOut {
  const double* w[2];  // per-row weights
  double* Y[2];        // g x (g+1) outputs
  double* gw[2];       // group weights (nullable)
};

template <int HPT, int NWT>
__global__ void __launch_bounds__(AGGL_THREADS)
agg_reduce_lds(const double* __restrict__ X, long ldx, int n, const int* __restrict__ offs,
               const int* __restrict__ members, int g, AggOut o, long ldy, int divide) {
  extern __shared__ double xrow[];  // n + 1
  const int G = blockIdx.x;
  const int rb = offs[G], re = offs[G + 1];
  double acc[NWT][HPT];
#pragma unroll
  for (int t = 0; t < NWT; ++t)
#pragma unroll
    for (int k = 0; k < HPT; ++k) acc[t][k] = 0.0;
  double wsum[NWT];
#pragma unroll
  for (int t = 0; t < NWT; ++t) wsum[t] = 0.0;
  for (int a = rb; a < re; ++a) {
    const int i = members[a];
    double wi[NWT];
#pragma unroll
    for (int t = 0; t < NWT; ++t) {
      wi[t] = o.w[t][i];
      wsum[t] += wi[t];
    }
    const double* row = X + static_cast<long>(i) * ldx;
    __syncthreads();  // the previous row's gathers are done
    // eight loads per thread in flight (addresses clamped to the row, so no
    // load waits behind a bounds branch)
    for (int j0 = 0; j0 <= n; j0 += 8 * AGGL_THREADS) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = __builtin_nontemporal_load(row + min(j0 + u * AGGL_THREADS + static_cast<int>(threadIdx.x), n));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u * AGGL_THREADS + static_cast<int>(threadIdx.x);
        if (j <= n) xrow[j] = v[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int H = threadIdx.x + k * AGGL_THREADS;
      if (H < g) {
        const int cb = offs[H], ce = offs[H + 1];
        double sv = 0.0;
        for (int b0 = cb; b0 < ce; b0 += 4) {  // four index loads in flight, sums in member order
          int m[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) m[u] = members[min(b0 + u, ce - 1)];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (b0 + u < ce) sv += xrow[m[u]];
        }
#pragma unroll
        for (int t = 0; t < NWT; ++t) acc[t][k] += wi[t] * sv;
      } else if (H == g) {
#pragma unroll
        for (int t = 0; t < NWT; ++t) acc[t][k] += wi[t] * xrow[n];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NWT; ++t) {
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int H = threadIdx.x + k * AGGL_THREADS;
      if (H <= g) o.Y[t][static_cast<long>(G) * ldy + H] = divide ? acc[t][k] / wsum[t] : acc[t][k];
    }
    if (o.gw[t] && threadIdx.x == 0) o.gw[t][G] = wsum[t];
  }
}

// agg_reduce_lds when the row fits in LDS and the outputs in registers, else
// agg_reduce (once per weighting)
template <int NWT>
void launch_agg_n(const double* X, long ldx, int n, const AggOut& o, const int* offs, const int* members, int g,
                  long ldy, int divide, hipStream_t s) {
  const size_t lds = static_cast<size_t>(n + 1) * sizeof(double);
  const int hpt = (g + AGGL_THREADS) / AGGL_THREADS;  // ceil((g + 1) / AGGL_THREADS)
  if (lds <= AGGL_MAX_LDS && hpt <= 32) {
    // dynamic LDS beyond the default 64 KB has to be allowed per kernel
    auto allow = [](const void* fn) {
      return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(AGGL_MAX_LDS)) ==
             hipSuccess;
    };
    const void* fn = hpt <= 4    ? reinterpret_cast<const void*>(&agg_reduce_lds<4, NWT>)
                     : hpt <= 16 ? reinterpret_cast<const void*>(&agg_reduce_lds<16, NWT>)
                                 : reinterpret_cast<const void*>(&agg_reduce_lds<32, NWT>);
    if (lds <= 64 * 1024 || allow(fn)) {
      if (hpt <= 4)
        hipLaunchKernelGGL((agg_reduce_lds<4, NWT>), dim3(static_cast<unsigned>(g)), dim3(AGGL_THREADS), lds, s, X,
                           ldx, n, offs, members, g, o, ldy, divide);
      else if (hpt <= 16)
        hipLaunchKernelGGL((agg_reduce_lds<16, NWT>), dim3(static_cast<unsigned>(g)), dim3(AGGL_THREADS), lds, s, X,
                           ldx, n, offs, members, g, o, ldy, divide);
      else
        hipLaunchKernelGGL((agg_reduce_lds<32, NWT>), dim3(static_cast<unsigned>(g)), dim3(AGGL_THREADS), lds, s, X,
                           ldx, n, offs, members, g, o, ldy, divide);
      return;
    }
    (void)hipGetLastError();  // the attribute was refused: the gather form below
  }
  dim3 grid(static_cast<unsigned>(ceil_div(g + 1, AGG_THREADS)), static_cast<unsigned>(g));
  for (int t = 0; t < NWT; ++t)
    hipLaunchKernelGGL(agg_reduce, grid, dim3(AGG_THREADS), 0, s, X, ldx, n, o.w[t], offs, members, g, o.Y[t], ldy,
                       o.gw[t], divide);
}

void launch_agg(const double* X, long ldx, int n, const double* w, const int* offs, const int* members, int g,
                double* Y, long ldy, double* gw, int divide, hipStream_t s) {
  launch_agg_n<1>(X, ldx, n, AggOut{{w, nullptr}, {Y, nullptr}, {gw, nullptr}}, offs, members, g, ldy, divide, s);
}

__global__ void __launch_bounds__(256) zero_ints(int* __restrict__ p, long count) {
  for (long q = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; q < count;
       q += static_cast<long>(gridDim.x) * blockDim.x)
    p[q] = 0;
}

struct AggLayout {
  int* status;
  int* offs;
  int* members;
  int* rank;
  int* cnt;     // chunks x g
  int nch;
  size_t bytes;
  bool ok;
};

AggLayout agg_layout(void* work, size_t bytes, int64_t n, int64_t g) {
  Carve cv(work, bytes);
  AggLayout l;
  l.nch = static_cast<int>(ceil_div(n, CSR_CHUNK));
  l.status = cv.take<int>(1);
  l.offs = cv.take<int>(static_cast<size_t>(g + 1));
  l.members = cv.take<int>(static_cast<size_t>(n));
  l.rank = cv.take<int>(static_cast<size_t>(n));
  l.cnt = cv.take<int>(static_cast<size_t>(l.nch) * g);
  l.bytes = cv.used;
  l.ok = cv.ok;
  return l;
}

// Two-sided nodes (eq. 5.29): the share of face pair (a, b) in the sum over
// the face pairs of its node pair, D_GH = sum_{a' in G, b' in H} F_a'b'.
// Group ids outside [0, g) (reported by the CSR build) write 0 and read nothing.
__global__ void __launch_bounds__(256)
vf_fraction(const double* __restrict__ F, long ldf, int nf, const int* __restrict__ group, int g,
            const double* __restrict__ D, long ldd, double* __restrict__ R, long ldr) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b > nf) return;
  const int H = b < nf ? group[b] : g;
  for (int a = blockIdx.y; a < nf; a += gridDim.y) {
    const int G = group[a];
    double out = 0.0;
    if (G >= 0 && G < g && H >= 0 && H <= g) {
      const double den = D[static_cast<long>(G) * ldd + H];
      if (den != 0.0) out = F[static_cast<long>(a) * ldf + b] / den;
    }
    R[static_cast<long>(a) * ldr + b] = out;
  }
}

// The same quotients with one workgroup per node G: its row of D is staged
// in LDS once, then the rows of G's faces stream through (coalesced loads
// and stores; the column-to-node map is read coalesced and stays in cache,
// the gathers hit LDS).  Used when g + 1 doubles fit in VF_LDS_BYTES.
constexpr size_t VF_LDS_BYTES = 64 * 1024;

__global__ void __launch_bounds__(256)
vf_fraction_lds(const double* __restrict__ F, long ldf, int nf, const int* __restrict__ group, int g,
                const int* __restrict__ offs, const int* __restrict__ members, const double* __restrict__ D,
                long ldd, double* __restrict__ R, long ldr) {
  extern __shared__ double drow[];  // g + 1
  const int G = blockIdx.x;
  for (int h = threadIdx.x; h <= g; h += blockDim.x) drow[h] = D[static_cast<long>(G) * ldd + h];
  __syncthreads();
  for (int m = offs[G]; m < offs[G + 1]; ++m) {
    const int a = members[m];
    const double* frow = F + static_cast<long>(a) * ldf;
    double* rrow = R + static_cast<long>(a) * ldr;
    // eight columns per thread with their loads in flight together
    // (addresses clamped into the row; selects on computed values only)
    for (int b0 = 0; b0 <= nf; b0 += 8 * 256) {
      int hv[8];
      double fv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = min(b0 + u * 256 + static_cast<int>(threadIdx.x), nf);
        hv[u] = group[min(b, nf - 1)];
        fv[u] = __builtin_nontemporal_load(frow + b);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + u * 256 + static_cast<int>(threadIdx.x);
        if (b > nf) break;
        const int H = b < nf ? hv[u] : g;
        const double den = (H >= 0 && H <= g) ? drow[H] : 0.0;
        rrow[b] = den != 0.0 ? fv[u] / den : 0.0;
      }
    }
  }
}

// eq. C.4: eps_GH = (sum_{a in G} eps_a S_a sum_{b in H} B_ab) / (sum_{a in G} S_a sum_{b in H} B_ab);
// a pair without exchange gets the node's area-mean emissivity.
__global__ void __launch_bounds__(256)
ne_ratio(const double* __restrict__ num, const double* __restrict__ den, long ldd, const double* __restrict__ we,
         const double* __restrict__ ws, int g, double* __restrict__ E, long lde) {
  const int H = blockIdx.x * 256 + threadIdx.x;
  if (H > g) return;
  for (int G = blockIdx.y; G < g; G += gridDim.y) {
    // both loads in flight together: the select is marked unpredictable, so
    // the quotient (and its load) is not moved behind a branch on d
    const double d = den[static_cast<long>(G) * ldd + H];
    const double q = num[static_cast<long>(G) * ldd + H];
    const double r = q / d, mean = we[G] / ws[G];
    E[static_cast<long>(G) * lde + H] = __builtin_unpredictable(d != 0.0) ? r : mean;
  }
}

// eps_a S_a per face, with the range checks of the optical inputs
__global__ void __launch_bounds__(256)
face_weights(const double* __restrict__ eps, const double* __restrict__ area, int n, double* __restrict__ out,
             int* __restrict__ status) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= n) return;
  const double e = eps[a], s = area[a];
  if (!(e >= 0.0 && e <= 1.0 && s > 0.0 && s <= 1.0e300)) atomicMin(status, RAD_ENONFINITE);
  out[a] = e * s;
}

__global__ void __launch_bounds__(256) fill_ones(double* __restrict__ p, int n) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a < n) p[a] = 1.0;
}

// CSR of the group map (members of each group in face order), shared by the reductions of one call
void agg_build(const int32_t* group, int n, int g, const AggLayout& l, hipStream_t s) {
  const long ncnt = static_cast<long>(l.nch) * g;
  hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, l.status, 1L);
  hipLaunchKernelGGL(zero_ints, dim3(static_cast<unsigned>(std::min<long>(ceil_div(ncnt, 256), 4096))), dim3(256), 0,
                     s, l.cnt, ncnt);
  hipLaunchKernelGGL(csr_rank, dim3(static_cast<unsigned>(l.nch)), dim3(CSR_CHUNK), 0, s, group, n, g, l.rank,
                     l.cnt, l.status);
  hipLaunchKernelGGL(csr_offsets, dim3(1), dim3(1024), 0, s, l.cnt, l.nch, g, l.offs, l.status);
  hipLaunchKernelGGL(csr_scatter, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, group, n, g,
                     l.rank, l.cnt, l.offs, l.members);
}

void agg_sums(const double* X, long ldx, int n, const double* w, const AggLayout& l, int g, double* Y, long ldy,
              double* gw, hipStream_t s) {
  ProfScope prof(s, RAD_PROF_AGGREGATE, 0.0, 8.0 * static_cast<double>(n) * (n + 1));
  launch_agg(X, ldx, n, w, l.offs, l.members, g, Y, ldy, gw, 0, s);
}

// the same sums under two weightings in one pass over X
void agg_sums2(const double* X, long ldx, int n, const double* w0, const double* w1, const AggLayout& l, int g,
               double* Y0, double* Y1, long ldy, double* gw0, double* gw1, hipStream_t s) {
  ProfScope prof(s, RAD_PROF_AGGREGATE, 0.0, 8.0 * static_cast<double>(n) * (n + 1));
  launch_agg_n<2>(X, ldx, n, AggOut{{w0, w1}, {Y0, Y1}, {gw0, gw1}}, l.offs, l.members, g, ldy, 0, s);
}

int read_status(const int* dev, hipStream_t s, int* out) {
  if (hipMemcpyAsync(out, dev, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return RAD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RAD_EHIP;
  return RAD_OK;
}

struct TwoSidedLayout {
  AggLayout agg;
  double* w;     // per-face weights (ones, or eps S)
  double* d0;    // g x (g+1) pair sums
  double* d1;    // g x (g+1) pair sums (emissivity denominator)
  double* gw0;   // g group weights
  double* gw1;
  long ldd;
  size_t bytes;
  bool ok;
};

TwoSidedLayout two_sided_layout(void* work, size_t bytes, int64_t nf, int64_t g, bool emissivity) {
  TwoSidedLayout t{};
  t.agg = agg_layout(work, bytes, nf, g);
  const size_t off = align_up(t.agg.bytes, 256);
  Carve cv(work && bytes > off ? static_cast<char*>(work) + off : nullptr, bytes > off ? bytes - off : 0);
  t.ldd = g + 1;
  t.w = cv.take<double>(static_cast<size_t>(nf));
  t.d0 = cv.take<double>(static_cast<size_t>(g) * t.ldd);
  if (emissivity) {
    t.d1 = cv.take<double>(static_cast<size_t>(g) * t.ldd);
    t.gw0 = cv.take<double>(static_cast<size_t>(g));
    t.gw1 = cv.take<double>(static_cast<size_t>(g));
  }
  t.bytes = off + cv.used;
  t.ok = t.agg.ok && cv.ok;
  return t;
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" size_t rad_aggregate_workspace_bytes(int64_t n, int64_t g) {
  if (n < 1 || g < 1) return 0;
  return agg_layout(nullptr, 0, n, g).bytes;
}

extern "C" int32_t rad_aggregate_nodes(const double* X, int64_t n, int64_t ldx,
                                       const double* weight, const int32_t* group, int64_t g,
                                       double* Y, int64_t ldy, double* group_weight, void* work,
                                       size_t work_bytes, rad_stats* stats, void* stream) {
  ApiRange range("rad_aggregate_nodes");
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 24), RAD_EINVAL, "rad_aggregate_nodes: n out of range");
  RAD_REQUIRE(g >= 1 && g <= n, RAD_EINVAL, "rad_aggregate_nodes: g must be in [1, n]");
  RAD_REQUIRE(ldx >= n + 1 && ldy >= g + 1, RAD_EINVAL, "rad_aggregate_nodes: ld too small");
  RAD_REQUIRE(X && weight && group && Y, RAD_EINVAL, "rad_aggregate_nodes: NULL pointer");
  RAD_REQUIRE(ceil_div(n, CSR_CHUNK) * g <= (int64_t(1) << 31) - 1, RAD_EINVAL,
              "rad_aggregate_nodes: too many groups for this n");
  AggLayout l = agg_layout(work, work_bytes, n, g);
  RAD_REQUIRE(l.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_aggregate_nodes: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n), gi = static_cast<int>(g);
  const long ncnt = static_cast<long>(l.nch) * g;
  hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, l.status, 1L);
  hipLaunchKernelGGL(zero_ints, dim3(static_cast<unsigned>(std::min<long>(ceil_div(ncnt, 256), 4096))), dim3(256), 0,
                     s, l.cnt, ncnt);
  hipLaunchKernelGGL(csr_rank, dim3(static_cast<unsigned>(l.nch)), dim3(CSR_CHUNK), 0, s, group, ni, gi, l.rank,
                     l.cnt, l.status);
  hipLaunchKernelGGL(csr_offsets, dim3(1), dim3(1024), 0, s, l.cnt, l.nch, gi, l.offs, l.status);
  hipLaunchKernelGGL(csr_scatter, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, group, ni, gi,
                     l.rank, l.cnt, l.offs, l.members);
  {
    ProfScope prof(s, RAD_PROF_AGGREGATE, 0.0, 8.0 * static_cast<double>(n) * (n + 1));
    launch_agg(X, static_cast<long>(ldx), ni, weight, l.offs, l.members, gi, Y, static_cast<long>(ldy),
               group_weight, 1, s);
  }
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats) return RAD_OK;
  int st = 0;
  RAD_HIP_CHECK(hipMemcpyAsync(&st, l.status, sizeof(int), hipMemcpyDeviceToHost, s));
  RAD_HIP_CHECK(hipStreamSynchronize(s));
  *stats = rad_stats{};
  stats->device_status = st;
  if (st < 0) {
    set_error("rad_aggregate_nodes: empty group or group id out of [0, g)");
    return st;
  }
  return RAD_OK;
}

extern "C" size_t rad_view_fractions_workspace_bytes(int64_t nf, int64_t g) {
  if (nf < 1 || g < 1) return 0;
  return two_sided_layout(nullptr, 0, nf, g, false).bytes;
}

extern "C" int32_t rad_view_fractions(const double* F, int64_t nf, int64_t ldf, const int32_t* group, int64_t g,
                                      double* R, int64_t ldr, void* work, size_t work_bytes, rad_stats* stats,
                                      void* stream) {
  ApiRange range("rad_view_fractions");
  clear_error();
  RAD_REQUIRE(nf >= 1 && nf <= (1 << 24), RAD_EINVAL, "rad_view_fractions: nf out of range");
  RAD_REQUIRE(g >= 1 && g <= nf, RAD_EINVAL, "rad_view_fractions: g must be in [1, nf]");
  RAD_REQUIRE(ldf >= nf + 1 && ldr >= nf + 1, RAD_EINVAL, "rad_view_fractions: ld too small");
  RAD_REQUIRE(F && group && R, RAD_EINVAL, "rad_view_fractions: NULL pointer");
  RAD_REQUIRE(ceil_div(nf, CSR_CHUNK) * g <= (int64_t(1) << 31) - 1, RAD_EINVAL,
              "rad_view_fractions: too many groups for this nf");
  TwoSidedLayout t = two_sided_layout(work, work_bytes, nf, g, false);
  RAD_REQUIRE(t.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_view_fractions: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(nf), gi = static_cast<int>(g);
  agg_build(group, ni, gi, t.agg, s);
  hipLaunchKernelGGL(fill_ones, dim3(static_cast<unsigned>(ceil_div(nf, 256))), dim3(256), 0, s, t.w, ni);
  agg_sums(F, static_cast<long>(ldf), ni, t.w, t.agg, gi, t.d0, t.ldd, nullptr, s);
  const size_t lds = static_cast<size_t>(g + 1) * sizeof(double);
  if (lds <= VF_LDS_BYTES) {
    // (rows of faces whose node id is out of range are left unwritten; the
    // call reports that error when stats are requested)
    hipLaunchKernelGGL(vf_fraction_lds, dim3(static_cast<unsigned>(g)), dim3(256), lds, s, F, static_cast<long>(ldf),
                       ni, group, gi, t.agg.offs, t.agg.members, t.d0, t.ldd, R, static_cast<long>(ldr));
  } else {
    hipLaunchKernelGGL(vf_fraction, dim3(static_cast<unsigned>(ceil_div(nf + 1, 256)),
                                         static_cast<unsigned>(std::min<int64_t>(nf, 32768))),
                       dim3(256), 0, s, F, static_cast<long>(ldf), ni, group, gi, t.d0, t.ldd, R,
                       static_cast<long>(ldr));
  }
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats) return RAD_OK;
  int st = 0;
  int rc = read_status(t.agg.status, s, &st);
  if (rc != RAD_OK) return rc;
  *stats = rad_stats{};
  stats->device_status = st;
  if (st < 0) {
    set_error("rad_view_fractions: empty group or group id out of [0, g)");
    return st;
  }
  return RAD_OK;
}

extern "C" size_t rad_node_emissivity_workspace_bytes(int64_t nf, int64_t g) {
  if (nf < 1 || g < 1) return 0;
  return two_sided_layout(nullptr, 0, nf, g, true).bytes;
}

extern "C" int32_t rad_node_emissivity(const double* B, int64_t nf, int64_t ldb, const double* eps,
                                       const double* area, const int32_t* group, int64_t g, double* E,
                                       int64_t lde, void* work, size_t work_bytes, rad_stats* stats,
                                       void* stream) {
  ApiRange range("rad_node_emissivity");
  clear_error();
  RAD_REQUIRE(nf >= 1 && nf <= (1 << 24), RAD_EINVAL, "rad_node_emissivity: nf out of range");
  RAD_REQUIRE(g >= 1 && g <= nf, RAD_EINVAL, "rad_node_emissivity: g must be in [1, nf]");
  RAD_REQUIRE(ldb >= nf + 1 && lde >= g + 1, RAD_EINVAL, "rad_node_emissivity: ld too small");
  RAD_REQUIRE(B && eps && area && group && E, RAD_EINVAL, "rad_node_emissivity: NULL pointer");
  RAD_REQUIRE(ceil_div(nf, CSR_CHUNK) * g <= (int64_t(1) << 31) - 1, RAD_EINVAL,
              "rad_node_emissivity: too many groups for this nf");
  TwoSidedLayout t = two_sided_layout(work, work_bytes, nf, g, true);
  RAD_REQUIRE(t.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_node_emissivity: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(nf), gi = static_cast<int>(g);
  agg_build(group, ni, gi, t.agg, s);
  hipLaunchKernelGGL(face_weights, dim3(static_cast<unsigned>(ceil_div(nf, 256))), dim3(256), 0, s, eps, area, ni,
                     t.w, t.agg.status);
  agg_sums2(B, static_cast<long>(ldb), ni, t.w, area, t.agg, gi, t.d0, t.d1, t.ldd, t.gw0, t.gw1, s);
  hipLaunchKernelGGL(ne_ratio, dim3(static_cast<unsigned>(ceil_div(g + 1, 256)), static_cast<unsigned>(std::min<int64_t>(g, 32768))), dim3(256),
                     0, s, t.d0, t.d1, t.ldd, t.gw0, t.gw1, gi, E, static_cast<long>(lde));
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats) return RAD_OK;
  int st = 0;
  int rc = read_status(t.agg.status, s, &st);
  if (rc != RAD_OK) return rc;
  *stats = rad_stats{};
  stats->device_status = st;
  if (st < 0) {
    set_error(st == RAD_ENONFINITE ? "rad_node_emissivity: eps outside [0, 1] or area not > 0"
                                   : "rad_node_emissivity: empty group or group id out of [0, g)");
    return st;
  }
  return RAD_OK;
}
