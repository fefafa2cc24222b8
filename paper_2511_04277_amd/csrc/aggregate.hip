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
  __shared__ int chunk[CSR_CHUNK];
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
  int r = 0;
#pragma unroll 8
  for (int q = 0; q < tid; ++q) r += (chunk[q] == gi);
  bool last = true;
  for (int q = tid + 1; q < CSR_CHUNK; ++q)
    if (chunk[q] == gi) {
      last = false;
      break;
    }
  rank[i] = r;
  if (last) cnt[static_cast<long>(c) * g + gi] = r + 1;
}

// one block: cnt (nch x g, zero where a group is absent from a chunk) becomes
// the chunk offsets in place; offs[G] = sum of the counts of groups < G
__global__ void __launch_bounds__(1024)
csr_offsets(int* __restrict__ cnt, int nch, int g, int* __restrict__ offs, int* __restrict__ status) {
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int per = (g + 1023) / 1024;
  const int g0 = tid * per, g1 = min(g, g0 + per);
  int sum = 0;
  for (int G = g0; G < g1; ++G) {
    int run = 0;
    for (int c = 0; c < nch; ++c) {
      const int v = cnt[static_cast<long>(c) * g + G];
      cnt[static_cast<long>(c) * g + G] = run;
      run += v;
    }
    if (run == 0) atomicMin(status, RAD_EINVAL);  // empty group
    offs[G] = run;  // total for now
    sum += run;
  }
  part[tid] = sum;
  __syncthreads();
  if (tid == 0) {  // exclusive scan over the 1024 thread totals
    int run = 0;
    for (int q = 0; q < 1024; ++q) {
      const int v = part[q];
      part[q] = run;
      run += v;
    }
    offs[g] = run;
  }
  __syncthreads();
  int run = part[tid];
  for (int G = g0; G < g1; ++G) {
    const int v = offs[G];
    offs[G] = run;
    run += v;
  }
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
           double* __restrict__ Y, long ldy, double* __restrict__ gw) {
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
  Y[static_cast<long>(G) * ldy + H] = acc / wsum;
  if (gw && H == 0) gw[G] = wsum;
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
  dim3 grid(static_cast<unsigned>(ceil_div(g + 1, AGG_THREADS)), static_cast<unsigned>(g));
  {
    ProfScope prof(s, RAD_PROF_AGGREGATE, 0.0, 8.0 * static_cast<double>(n) * (n + 1));
    hipLaunchKernelGGL(agg_reduce, grid, dim3(AGG_THREADS), 0, s, X, static_cast<long>(ldx),
                       static_cast<int>(n), weight, l.offs, l.members, static_cast<int>(g), Y,
                       static_cast<long>(ldy), group_weight);
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
