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
  int tri;             // shape of op(A) by 128-blocks: 0 full, 1 block upper (rows of
                       // block b read k >= 128 b), 2 block lower (k < 128 (b + 1));
                       // the skipped entries must be zero
  int inplace;         // 1: C overwrites the rows of op(A) it reads (N <= 128): one
                       // column tile per row block, so only 128 x 128 tiles are safe
  int nseg;
  int ntile[2];        // 128-wide column tiles per segment
  int N[2];
  const T* B[2];
  long ldb[2];
  T* C[2];
  long ldc[2];
};

constexpr int GEMM_TILE = 128;   // tile of the grouped launches and tile counts (ntile)

// C tile epilogue: C = beta C + alpha acc, stores masked to M x N.  NBR x NBR
// MFMA blocks of 16 x 16 per wave.
template <class T, int NBR>
__device__ __forceinline__ void store_tile(const typename Mfma<T>::v4 (&acc)[NBR][NBR], const GemmArgs<T>& g,
                                           T* __restrict__ Cm, long ldc, int M, int N, int wr0, int wc0,
                                           int l) {
  const int li = l & 15;
  const bool full = (wr0 + 16 * NBR <= M) && (wc0 + 16 * NBR <= N);
  // per row block: the C values are loaded together (addresses clamped into
  // the matrix rather than a bounds branch per element, which would make
  // every load wait for the one before it), then fused and stored
#pragma unroll
  for (int rb = 0; rb < NBR; ++rb) {
    T cv[NBR][4] = {};
    if (g.beta != T(0)) {
#pragma unroll
      for (int cb = 0; cb < NBR; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = min(wr0 + rb * 16 + Mfma<T>::orow(l, r), M - 1);
          const int j = min(wc0 + cb * 16 + li, N - 1);
          cv[cb][r] = Cm[static_cast<long>(i) * ldc + j];
        }
    }
#pragma unroll
    for (int cb = 0; cb < NBR; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr0 + rb * 16 + Mfma<T>::orow(l, r);
        const int j = wc0 + cb * 16 + li;
        if (full || (i < M && j < N)) {
          // one explicit fused form, so every tile shape rounds alike
          const T ax = g.alpha * acc[rb][cb][r];
          Cm[static_cast<long>(i) * ldc + j] = g.beta != T(0) ? fma(g.beta, cv[cb][r], ax) : ax;
        }
      }
  }
}

// The workgroup stages each TS x KC slab of op(A) and KC x TS slab of B
// once, with 16-byte global loads, into double-buffered LDS; the four waves
// (2 x 2, each TS/2 x TS/2) read their MFMA fragments from LDS.  Within a K
// chunk, lane group g takes k = g KC/4 + s at MFMA step s.  One barrier per
// chunk; global loads run two chunks ahead of the MFMAs.  TS = 128 for
// large products; TS = 64 gives four times the workgroups for narrow or
// short ones.
//
// Operand contract (all operands are the solver's own padded buffers):
// op(A) is readable for rows < roundup(M, 128) and k < roundup(K, 32), B for
// rows < roundup(K, 32) and columns < roundup(N, 128); entries with k >= K
// are zero.  Base pointers and leading dimensions are 16-byte aligned.  Only
// the stores are masked.
// K chunk per LDS stage: FP64 uses 16 (2 x 32 KB stages at TS = 128), FP32 32
// (2 x 17 KB), so two workgroups share a CU and one's epilogue overlaps the
// other's MFMAs.
template <class T>
struct GemmCfg {
  static constexpr int KC = sizeof(T) == 8 ? 16 : 32;
  static constexpr int PA = 2;   // row padding of the A slab (elements)
  static constexpr int PB = 2;   // row padding of the B slab (elements)
};

// LDS slab of op(A) for one K chunk: row-major [TS][KC] when A is read by
// rows; K-major [KC][TS] when op(A) is a transpose (its global rows are k),
// so both cases store 16-byte runs.
template <class T, bool TRANS_A, int TS>
struct ASlab {
  static constexpr int R = TS, C = GemmCfg<T>::KC + GemmCfg<T>::PA;
};
template <class T, int TS>
struct ASlab<T, true, TS> {
  static constexpr int R = GemmCfg<T>::KC, C = TS + GemmCfg<T>::PB;
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

// elements of each slab per thread
template <class T, int TS>
constexpr int slab_ept() { return TS * GemmCfg<T>::KC / 256; }

template <class T, bool TRANS_A, int TS>
__device__ __forceinline__ void lds_stage_load(const T* __restrict__ A, long lda, const T* __restrict__ Bm,
                                               long ldb, int m0, int n0, int kc, T (&ra)[slab_ept<T, TS>()],
                                               T (&rb)[slab_ept<T, TS>()]) {
  constexpr int KC = GemmCfg<T>::KC, E = slab_ept<T, TS>();
  constexpr int TPR = TS / E;   // threads per TS-wide slab row
  constexpr int TPA = KC / E;   // threads per row of a row-major A slab
  const int t = threadIdx.x;
  if (!TRANS_A)  // thread -> op(A) row t / TPA, E consecutive k
    loadv<T, E>(A + static_cast<long>(m0 + t / TPA) * lda + kc + (t % TPA) * E, ra);
  else           // op(A)[m][k] = At[k][m]: thread -> k row t / TPR, E consecutive m
    loadv<T, E>(A + static_cast<long>(kc + t / TPR) * lda + m0 + (t % TPR) * E, ra);
  loadv<T, E>(Bm + static_cast<long>(kc + t / TPR) * ldb + n0 + (t % TPR) * E, rb);
}

template <class T, bool TRANS_A, int TS>
__device__ __forceinline__ void lds_stage_store(T (*sA)[(ASlab<T, TRANS_A, TS>::C)],
                                                T (*sB)[TS + GemmCfg<T>::PB],
                                                const T (&ra)[slab_ept<T, TS>()], const T (&rb)[slab_ept<T, TS>()]) {
  constexpr int KC = GemmCfg<T>::KC, E = slab_ept<T, TS>();
  constexpr int TPR = TS / E;
  constexpr int TPA = KC / E;
  const int t = threadIdx.x;
  if (!TRANS_A) {
    const int m = t / TPA, k0 = (t % TPA) * E;
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

// One TS x TS output tile: column-tile index bx (over both segments),
// row-tile index by.  With 64 x 64 tiles each lane loads its C values into
// registers before the K loop (the registers fit four workgroups per CU), so
// the epilogue does not wait on them: 4-12 % faster on the K = 128 panel
// updates, bitwise the same results (CPRE; persistent kernels, whose tile
// loop would spill the extra registers, keep the plain epilogue).
template <class T, bool TRANS_A, int TS = GEMM_TILE, bool CPRE = (TS == 64)>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T>& g, int bx, int by) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int KC = GemmCfg<T>::KC, E = slab_ept<T, TS>();
  constexpr int NBR = TS / 32;   // 16 x 16 blocks per wave side
  __shared__ T sA[2][ASlab<T, TRANS_A, TS>::R][ASlab<T, TRANS_A, TS>::C];
  __shared__ T sB[2][KC][TS + GemmCfg<T>::PB];
  const int nt0 = (g.nseg > 0 && g.N[0] > 0) ? (g.N[0] + TS - 1) / TS : 0;
  int ct = bx;
  int seg = 0;
  if (ct >= nt0) {
    seg = 1;
    ct -= nt0;
  }
  const T* __restrict__ Bm = g.B[seg];
  T* __restrict__ Cm = g.C[seg];
  const long ldb = g.ldb[seg], ldc = g.ldc[seg];
  const T* __restrict__ A = g.A;
  const long lda = g.lda;
  const int N = g.N[seg], M = g.M, K = g.K;
  const int m0 = by * TS, n0 = ct * TS;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int li = l & 15, lg = l >> 4;
  const int wr = (wave >> 1) * (TS / 2), wc = (wave & 1) * (TS / 2);
  const bool full = (m0 + wr + 16 * NBR <= M) && (n0 + wc + 16 * NBR <= N);
  T cv[NBR][NBR][4];
  if (CPRE) {
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int cb = 0; cb < NBR; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = m0 + wr + rb * 16 + Mfma<T>::orow(l, r), j = n0 + wc + cb * 16 + li;
          cv[rb][cb][r] = (g.beta != T(0) && (full || (i < M && j < N))) ? Cm[static_cast<long>(i) * ldc + j] : T(0);
        }
  }

  v4 acc[NBR][NBR];
#pragma unroll
  for (int a = 0; a < NBR; ++a)
#pragma unroll
    for (int b = 0; b < NBR; ++b) acc[a][b] = v4{0, 0, 0, 0};

  // two register stages: chunk c + 2 is loaded from global memory while
  // chunk c is multiplied from LDS and chunk c + 1 (loaded one chunk
  // earlier) is stored to the other LDS buffer, so each load has a whole
  // chunk of MFMAs to arrive
  T ra0[E], rb0[E], ra1[E], rb1[E];
  // K range of this row tile: a triangular op(A) is zero by 128-blocks, so
  // the row tile skips the blocks left (upper) or right (lower) of its block
  const int mb = (m0 / GEMM_TILE) * GEMM_TILE;
  const int kbeg = g.tri == 1 ? mb : 0;
  const int kend = g.tri == 2 ? min(K, mb + GEMM_TILE) : K;
  const int nch = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;
  if (nch > 0) {
    lds_stage_load<T, TRANS_A, TS>(A, lda, Bm, ldb, m0, n0, kbeg, ra0, rb0);
    lds_stage_store<T, TRANS_A, TS>(sA[0], sB[0], ra0, rb0);
  }
  if (nch > 1) lds_stage_load<T, TRANS_A, TS>(A, lda, Bm, ldb, m0, n0, kbeg + KC, ra1, rb1);
  __syncthreads();
  // chunk c from LDS buffer buf; la/lb receive chunk c + 2, sa/sb hold c + 1
  auto step = [&](int c, int buf, T (&la)[E], T (&lb)[E], const T (&sa)[E], const T (&sb)[E]) {
    if (c + 2 < nch) lds_stage_load<T, TRANS_A, TS>(A, lda, Bm, ldb, m0, n0, kbeg + (c + 2) * KC, la, lb);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = lg * (KC / 4) + s;
      T fa[NBR], fb[NBR];
#pragma unroll
      for (int q = 0; q < NBR; ++q) {
        fa[q] = TRANS_A ? sA[buf][k][wr + q * 16 + li] : sA[buf][wr + q * 16 + li][k];
        fb[q] = sB[buf][k][wc + q * 16 + li];
      }
#pragma unroll
      for (int x = 0; x < NBR; ++x)
#pragma unroll
        for (int y = 0; y < NBR; ++y) acc[x][y] = Mfma<T>::mma(fa[x], fb[y], acc[x][y]);
    }
    if (c + 1 < nch) lds_stage_store<T, TRANS_A, TS>(sA[buf ^ 1], sB[buf ^ 1], sa, sb);
    __syncthreads();
  };
  for (int c = 0; c < nch; c += 2) {
    step(c, 0, ra0, rb0, ra1, rb1);
    if (c + 1 < nch) step(c + 1, 1, ra1, rb1, ra0, rb0);
  }
  if (!CPRE) {
    store_tile<T, NBR>(acc, g, Cm, ldc, M, N, m0 + wr, n0 + wc, l);
    return;
  }
  // the same fused form as store_tile, with C from the registers
#pragma unroll
  for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
    for (int cb = 0; cb < NBR; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wr + rb * 16 + Mfma<T>::orow(l, r), j = n0 + wc + cb * 16 + li;
        if (full || (i < M && j < N)) {
          const T ax = g.alpha * acc[rb][cb][r];
          Cm[static_cast<long>(i) * ldc + j] = g.beta != T(0) ? fma(g.beta, cv[rb][cb][r], ax) : ax;
        }
      }
}

// Tile order.  The hardware hands workgroup k of a launch to XCD k % 8, and
// each XCD has its own L2.  The dispatch index is first remapped so that each
// XCD owns a contiguous range of logical tiles, then the logical tiles are
// walked in groups of TILE_GROUP tile rows, column by column, so the tiles
// one XCD runs at the same time share a few A row panels and B column panels
// instead of touching a new B panel per tile.  A block-triangular operand
// makes the work per tile row differ (up to 8x), so those products walk whole
// tile columns instead: each XCD then holds a range of columns with every
// row, and all XCDs get the same work.
constexpr int TILE_GROUP = 8;

__device__ __forceinline__ void grouped_tile(int L, int ntx, int nty, int group, int& bx, int& by) {
  const int per = group * ntx;
  const int grp = L / per, r0 = grp * group;
  const int gs = min(nty - r0, group), w = L - grp * per;
  by = r0 + w % gs;
  bx = w / gs;
}

template <class T, int TS>
inline int tiles_x(const GemmArgs<T>& g) {
  int t = 0;
  for (int q = 0; q < g.nseg; ++q) t += g.N[q] > 0 ? (g.N[q] + TS - 1) / TS : 0;
  return t;
}

template <class T, bool TRANS_A, int TS>
__global__ void __launch_bounds__(256, TS == GEMM_TILE ? 2 : 4) gemm_lds(GemmArgs<T> g) {
  const int nt0 = (g.nseg > 0 && g.N[0] > 0) ? (g.N[0] + TS - 1) / TS : 0;
  const int nt1 = (g.nseg > 1 && g.N[1] > 0) ? (g.N[1] + TS - 1) / TS : 0;
  const int ntx = nt0 + nt1;
  const int nty = (g.M + TS - 1) / TS;
  int bx, by;
  grouped_tile(xcd_contiguous(blockIdx.x, ntx * nty), ntx, nty, g.tri ? nty : TILE_GROUP, bx, by);
  gemm_tile<T, TRANS_A, TS>(g, bx, by);
}

// Runtime choice of the tile: a product with fewer than small_tile_below
// 128 x 128 tiles (precision index 0 = FP64, 1 = FP32) runs with 64 x 64
// tiles.  Set by rad_tuning_set (tuning.cpp), chosen by the autotuner.
struct GemmTuning {
  int small_tile_below[2];
  int side_chunk_tiles;  // row chunks of the side-stream trailing update (0: one launch)
};
GemmTuning& gemm_tuning();

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
  const int big = gemm_tiles<T>(a);
  if (big == 0) return hipSuccess;
  ProfScope prof(s, gemm_prof_kind<T>(trans_a), gemm_flops(a), gemm_bytes(a));
  const bool small = !a.inplace && big < gemm_tuning().small_tile_below[sizeof(T) == 8 ? 0 : 1];
  if (small) {
    const unsigned grid = static_cast<unsigned>(tiles_x<T, 64>(a)) * static_cast<unsigned>((a.M + 63) / 64);
    if (trans_a)
      hipLaunchKernelGGL((gemm_lds<T, true, 64>), dim3(grid), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((gemm_lds<T, false, 64>), dim3(grid), dim3(256), 0, s, a);
  } else {
    const unsigned grid = static_cast<unsigned>(big);
    if (trans_a)
      hipLaunchKernelGGL((gemm_lds<T, true, GEMM_TILE>), dim3(grid), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((gemm_lds<T, false, GEMM_TILE>), dim3(grid), dim3(256), 0, s, a);
  }
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
