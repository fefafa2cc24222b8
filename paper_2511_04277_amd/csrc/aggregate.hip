// Multi-node aggregation (thesis Sec. 5.2.3, eq. 5.6-5.7; first two rows of
// eq. 5.28 for one-sided faces) as one read of the sub-face matrix.
//
//   csr_build : single workgroup, stable counting sort of the group map into
//               member lists (each group's members in increasing index order),
//               so every later sum runs in a fixed order.
//   agg_reduce: workgroup = (row group G, chunk of 256 column groups H); each
//               thread owns one output Y_GH and sums w_i X_ij over i in G,
//               j in H in member order, then divides by W_G.
#include "common.h"

namespace rad {
namespace {

constexpr int CSR_THREADS = 1024;
constexpr int AGG_THREADS = 256;

__global__ void __launch_bounds__(CSR_THREADS)
csr_build(const int* __restrict__ group, int n, int g, int* __restrict__ offs,
          int* __restrict__ members, int* __restrict__ status) {
  extern __shared__ int sh[];       // g+1 counters, then a chunk of group ids
  int* cnt = sh;
  int* chunk = sh + (g + 1);
  const int tid = threadIdx.x;
  for (int q = tid; q <= g; q += blockDim.x) cnt[q] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) {
    int gi = group[i];
    if (gi < 0 || gi >= g) {
      atomicMin(status, RAD_EINVAL);
    } else {
      atomicAdd(&cnt[gi], 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int q = 0; q < g; ++q) {
      int c = cnt[q];
      if (c == 0) atomicMin(status, RAD_EINVAL);
      offs[q] = run;
      cnt[q] = run;  // becomes the running insert position
      run += c;
    }
    offs[g] = run;
  }
  __syncthreads();
  // stable placement, chunk by chunk in index order
  for (int base = 0; base < n; base += blockDim.x) {
    int i = base + tid;
    int gi = (i < n) ? group[i] : -1;
    if (gi >= g) gi = -1;
    chunk[tid] = gi;
    __syncthreads();
    if (gi >= 0) {
      int rank = 0;
      for (int q = 0; q < tid; ++q) rank += (chunk[q] == gi);
      members[cnt[gi] + rank] = i;
    }
    __syncthreads();
    if (gi >= 0) {
      // the last member of this group inside the chunk advances the cursor
      bool last = true;
      for (int q = tid + 1; q < blockDim.x; ++q)
        if (chunk[q] == gi) { last = false; break; }
      if (last) {
        int rank = 0;
        for (int q = 0; q < tid; ++q) rank += (chunk[q] == gi);
        cnt[gi] += rank + 1;
      }
    }
    __syncthreads();
  }
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

__global__ void zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

struct AggLayout {
  int* status;
  int* offs;
  int* members;
  size_t bytes;
  bool ok;
};

AggLayout agg_layout(void* work, size_t bytes, int64_t n, int64_t g) {
  Carve cv(work, bytes);
  AggLayout l;
  l.status = cv.take<int>(1);
  l.offs = cv.take<int>(static_cast<size_t>(g + 1));
  l.members = cv.take<int>(static_cast<size_t>(n));
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
  // counters for all groups plus one id per thread must fit in LDS
  RAD_REQUIRE((g + 1 + CSR_THREADS) * sizeof(int) <= 150 * 1024, RAD_EINVAL,
              "rad_aggregate_nodes: too many groups for one launch");
  AggLayout l = agg_layout(work, work_bytes, n, g);
  RAD_REQUIRE(l.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_aggregate_nodes: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(64), 0, s, l.status);
  size_t lds = (g + 1 + CSR_THREADS) * sizeof(int);
  hipLaunchKernelGGL(csr_build, dim3(1), dim3(CSR_THREADS), lds, s, group, static_cast<int>(n),
                     static_cast<int>(g), l.offs, l.members, l.status);
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
