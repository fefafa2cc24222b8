// MFMA GEMM building block for the dense solves (FP64 and FP32 on gfx950).
//
//   C[seg] = beta * C[seg] + alpha * op(A) * B[seg]
//
// op(A) is M x K (row-major A, or the transpose of a row-major K x M array);
// B and C are row-major.  The columns of C may span two segments with their
// own base pointers (used to update a factor matrix and its right-hand sides
// in one launch).
//
// Tiling: a 256-thread workgroup computes a 128 x 128 tile; each of its four
// waves owns 64 x 64 = 4 x 4 blocks of v_mfma_{f64,f32}_16x16x4.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace rad {

template <class T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register r of lane l holds row (l/16 + 4r), column l%16
  static __device__ __forceinline__ int orow(int l, int r) { return (l >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register r of lane l holds row (4(l/16) + r), column l%16
  static __device__ __forceinline__ int orow(int l, int r) { return 4 * (l >> 4) + r; }
};

template <class T>
struct GemmArgs {
  const T* A;
  long lda;
  int M, K;
  T alpha, beta;
  int tri;             // shape of op(A): 0 full, 1 upper (row tile m0 reads k >= m0),
                       // 2 lower (k < m0 + 128); the skipped entries must be zero
  int nseg;
  int ntile[2];        // 128-wide column tiles per segment
  int N[2];
  const T* B[2];
  long ldb[2];
  T* C[2];
  long ldc[2];
};

constexpr int GEMM_TILE = 128;

// C tile epilogue: C = beta C + alpha acc, stores masked to M x N.
template <class T>
__device__ __forceinline__ void store_tile(const typename Mfma<T>::v4 (&acc)[4][4], const GemmArgs<T>& g,
                                           T* __restrict__ Cm, long ldc, int M, int N, int wr0, int wc0,
                                           int l) {
  const int li = l & 15;
  const bool full = (wr0 + 64 <= M) && (wc0 + 64 <= N);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr0 + rb * 16 + Mfma<T>::orow(l, r);
        const int j = wc0 + cb * 16 + li;
        if (full || (i < M && j < N)) {
          T v = g.alpha * acc[rb][cb][r];
          T* p = Cm + static_cast<long>(i) * ldc + j;
          if (g.beta != T(0)) v += g.beta * *p;
          *p = v;
        }
      }
}

// The workgroup stages each 128 x KC slab of op(A) and KC x 128 slab of B
// once, with 16-byte global loads, into double-buffered LDS; the four waves
// read their MFMA fragments from LDS.  Within a K chunk, lane group g takes
// k = g KC/4 + s at MFMA step s.  One barrier per chunk.
//
// Operand contract (all operands are the solver's own padded buffers):
// op(A) is readable for rows < roundup(M, 128) and k < roundup(K, 32), B for
// rows < roundup(K, 32) and columns < roundup(N, 128); entries with k >= K
// are zero.  Base pointers and leading dimensions are 16-byte aligned.  Only
// the stores are masked.
// K chunk per LDS stage: FP64 uses 16 (2 x 32 KB stages), FP32 32 (2 x 17 KB),
// so two workgroups share a CU and one's epilogue overlaps the other's MFMAs.
template <class T>
struct GemmCfg {
  static constexpr int KC = sizeof(T) == 8 ? 16 : 32;
  static constexpr int PA = 2;   // row padding of the A slab (elements)
  static constexpr int PB = 2;   // row padding of the B slab (elements)
  static constexpr int EPT = KC / 2;  // slab elements per thread per operand
};

// LDS slab of op(A) for one K chunk: row-major [128][KC] when A is read by
// rows; K-major [KC][128] when op(A) is a transpose (its global rows are k),
// so both cases store 16-byte runs without bank conflicts.
template <class T, bool TRANS_A>
struct ASlab {
  static constexpr int R = GEMM_TILE, C = GemmCfg<T>::KC + GemmCfg<T>::PA;
};
template <class T>
struct ASlab<T, true> {
  static constexpr int R = GemmCfg<T>::KC, C = GEMM_TILE + GemmCfg<T>::PB;
};

template <class T, int NE>
__device__ __forceinline__ void loadv(const T* __restrict__ src, T (&r)[NE]) {
  typedef T v2 __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int per = 16 / sizeof(T);
  const v2* p = reinterpret_cast<const v2*>(src);
#pragma unroll
  for (int q = 0; q < NE / per; ++q) {
    v2 x = p[q];
#pragma unroll
    for (int e = 0; e < per; ++e) r[q * per + e] = x[e];
  }
}

template <class T, bool TRANS_A>
__device__ __forceinline__ void lds_stage_load(const T* __restrict__ A, long lda, const T* __restrict__ Bm,
                                               long ldb, int m0, int n0, int kc, T (&ra)[GemmCfg<T>::EPT],
                                               T (&rb)[GemmCfg<T>::EPT]) {
  constexpr int KC = GemmCfg<T>::KC, E = GemmCfg<T>::EPT;
  constexpr int TPR = GEMM_TILE / E;  // threads per 128-wide slab row
  const int t = threadIdx.x;
  if (!TRANS_A)  // thread -> op(A) row t/2, E consecutive k
    loadv<T, E>(A + static_cast<long>(m0 + (t >> 1)) * lda + kc + (t & 1) * E, ra);
  else           // op(A)[m][k] = At[k][m]: thread -> k row t/TPR, E consecutive m
    loadv<T, E>(A + static_cast<long>(kc + t / TPR) * lda + m0 + (t % TPR) * E, ra);
  loadv<T, E>(Bm + static_cast<long>(kc + t / TPR) * ldb + n0 + (t % TPR) * E, rb);
  (void)KC;
}

template <class T, bool TRANS_A>
__device__ __forceinline__ void lds_stage_store(T (*sA)[(ASlab<T, TRANS_A>::C)],
                                                T (*sB)[GEMM_TILE + GemmCfg<T>::PB],
                                                const T (&ra)[GemmCfg<T>::EPT], const T (&rb)[GemmCfg<T>::EPT]) {
  constexpr int E = GemmCfg<T>::EPT;
  constexpr int TPR = GEMM_TILE / E;
  const int t = threadIdx.x;
  if (!TRANS_A) {
    const int m = t >> 1, k0 = (t & 1) * E;
#pragma unroll
    for (int q = 0; q < E; ++q) sA[m][k0 + q] = ra[q];
  } else {
    const int k = t / TPR, mb = (t % TPR) * E;
#pragma unroll
    for (int q = 0; q < E; ++q) sA[k][mb + q] = ra[q];
  }
  const int k = t / TPR, nb = (t % TPR) * E;
#pragma unroll
  for (int q = 0; q < E; ++q) sB[k][nb + q] = rb[q];
}

// One 128 x 128 output tile: column-tile index bx (over both segments),
// row-tile index by.
template <class T, bool TRANS_A>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T>& g, int bx, int by) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int KC = GemmCfg<T>::KC, E = GemmCfg<T>::EPT;
  __shared__ T sA[2][ASlab<T, TRANS_A>::R][ASlab<T, TRANS_A>::C];
  __shared__ T sB[2][KC][GEMM_TILE + GemmCfg<T>::PB];
  int ct = bx;
  int seg = 0;
  if (ct >= g.ntile[0]) {
    seg = 1;
    ct -= g.ntile[0];
  }
  const T* __restrict__ Bm = g.B[seg];
  T* __restrict__ Cm = g.C[seg];
  const long ldb = g.ldb[seg], ldc = g.ldc[seg];
  const T* __restrict__ A = g.A;
  const long lda = g.lda;
  const int N = g.N[seg], M = g.M, K = g.K;
  const int m0 = by * GEMM_TILE, n0 = ct * GEMM_TILE;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int li = l & 15, lg = l >> 4;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;

  v4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4{0, 0, 0, 0};

  T ra[E], rb[E];
  // K range of this row tile (triangular op(A) skips its zero blocks)
  const int kbeg = g.tri == 1 ? m0 : 0;
  const int kend = g.tri == 2 ? min(K, m0 + GEMM_TILE) : K;
  const int nch = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;
  if (nch > 0) {
    lds_stage_load<T, TRANS_A>(A, lda, Bm, ldb, m0, n0, kbeg, ra, rb);
    lds_stage_store<T, TRANS_A>(sA[0], sB[0], ra, rb);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < nch;
    if (more) lds_stage_load<T, TRANS_A>(A, lda, Bm, ldb, m0, n0, kbeg + (c + 1) * KC, ra, rb);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = lg * (KC / 4) + s;
      T fa[4], fb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        fa[q] = TRANS_A ? sA[buf][k][wr + q * 16 + li] : sA[buf][wr + q * 16 + li][k];
        fb[q] = sB[buf][k][wc + q * 16 + li];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = Mfma<T>::mma(fa[x], fb[y], acc[x][y]);
    }
    if (more) lds_stage_store<T, TRANS_A>(sA[buf ^ 1], sB[buf ^ 1], ra, rb);
    __syncthreads();
  }
  store_tile<T>(acc, g, Cm, ldc, M, N, m0 + wr, n0 + wc, l);
}

// Tile order.  The hardware hands workgroup k of a launch to XCD k % 8, and
// each XCD has its own L2.  The dispatch index is first remapped so that each
// XCD owns a contiguous range of logical tiles, then the logical tiles are
// walked in groups of TILE_GROUP tile rows, column by column, so the tiles
// one XCD runs at the same time share a few A row panels and B column panels
// instead of touching a new B panel per tile.
constexpr int NUM_XCD = 8;
constexpr int TILE_GROUP = 8;

__device__ __forceinline__ int xcd_contiguous(int pid, int total) {
  const int q = total / NUM_XCD, rem = total % NUM_XCD;
  const int x = pid % NUM_XCD, loc = pid / NUM_XCD;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + loc;
}

__device__ __forceinline__ void grouped_tile(int L, int ntx, int nty, int& bx, int& by) {
  const int per = TILE_GROUP * ntx;
  const int grp = L / per, r0 = grp * TILE_GROUP;
  const int gs = min(nty - r0, TILE_GROUP), w = L - grp * per;
  by = r0 + w % gs;
  bx = w / gs;
}

template <class T, bool TRANS_A>
__global__ void __launch_bounds__(256, 2) gemm_lds(GemmArgs<T> g) {
  const int ntx = g.ntile[0] + g.ntile[1];
  const int nty = (g.M + GEMM_TILE - 1) / GEMM_TILE;
  int bx, by;
  grouped_tile(xcd_contiguous(blockIdx.x, ntx * nty), ntx, nty, bx, by);
  gemm_tile<T, TRANS_A>(g, bx, by);
}

// Host: number of 128 x 128 tiles of a product (fills g.ntile).
template <class T>
inline int gemm_tiles(GemmArgs<T>& a) {
  if (a.M <= 0 || a.K <= 0) {
    a.ntile[0] = a.ntile[1] = 0;
    return 0;
  }
  int total = 0;
  for (int q = 0; q < 2; ++q) {
    a.ntile[q] = (q < a.nseg && a.N[q] > 0) ? (a.N[q] + GEMM_TILE - 1) / GEMM_TILE : 0;
    total += a.ntile[q];
  }
  return total * ((a.M + GEMM_TILE - 1) / GEMM_TILE);
}

// Profiling kind and algorithmic work of one product (A read once, B read
// once, C written once and also read when beta != 0).
template <class T>
inline int gemm_prof_kind(bool trans_a) {
  if (sizeof(T) == 8) return trans_a ? RAD_PROF_GEMM_F64_T : RAD_PROF_GEMM_F64;
  return trans_a ? RAD_PROF_GEMM_F32_T : RAD_PROF_GEMM_F32;
}
template <class T>
inline double gemm_flops(const GemmArgs<T>& a) {
  double ncols = 0.0;
  for (int q = 0; q < a.nseg; ++q) ncols += a.N[q];
  double mk = static_cast<double>(a.M) * a.K;  // multiply-adds per column
  if (a.tri != 0) {
    mk = 0.0;
    for (int m0 = 0; m0 < a.M; m0 += GEMM_TILE) {
      const int rows = std::min(GEMM_TILE, a.M - m0);
      const int kb = a.tri == 1 ? m0 : 0, ke = a.tri == 2 ? std::min(a.K, m0 + GEMM_TILE) : a.K;
      mk += static_cast<double>(rows) * std::max(0, ke - kb);
    }
  }
  return 2.0 * mk * ncols;
}
template <class T>
inline double gemm_bytes(const GemmArgs<T>& a) {
  double ncols = 0.0;
  for (int q = 0; q < a.nseg; ++q) ncols += a.N[q];
  const double c = (a.beta != T(0) ? 2.0 : 1.0) * a.M * ncols;
  return sizeof(T) * (static_cast<double>(a.M) * a.K + static_cast<double>(a.K) * ncols + c);
}

// Host-side launcher: one or two column segments.
template <class T>
inline hipError_t launch_gemm(const GemmArgs<T>& a0, bool trans_a, hipStream_t s) {
  GemmArgs<T> a = a0;
  if (a.M <= 0 || a.K <= 0) return hipSuccess;
  int total = 0;
  for (int q = 0; q < 2; ++q) {
    a.ntile[q] = (q < a.nseg && a.N[q] > 0) ? (a.N[q] + GEMM_TILE - 1) / GEMM_TILE : 0;
    total += a.ntile[q];
  }
  if (total == 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>(total) * static_cast<unsigned>((a.M + GEMM_TILE - 1) / GEMM_TILE));
  ProfScope prof(s, gemm_prof_kind<T>(trans_a), gemm_flops(a), gemm_bytes(a));
  if (trans_a)
    hipLaunchKernelGGL((gemm_lds<T, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_lds<T, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <class T>
inline GemmArgs<T> gemm_args(const T* A, long lda, int M, int K, T alpha, T beta) {
  GemmArgs<T> a{};
  a.A = A;
  a.lda = lda;
  a.M = M;
  a.K = K;
  a.alpha = alpha;
  a.beta = beta;
  a.nseg = 0;
  return a;
}

template <class T>
inline void gemm_add_segment(GemmArgs<T>& a, const T* B, long ldb, T* C, long ldc, int N) {
  a.B[a.nseg] = B;
  a.ldb[a.nseg] = ldb;
  a.C[a.nseg] = C;
  a.ldc[a.nseg] = ldc;
  a.N[a.nseg] = N;
  a.nseg += 1;
}

}  // namespace rad
