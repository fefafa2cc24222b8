// MFMA GEMM building block for the dense solves (FP64 and FP32 on gfx950).
//
//   C[seg] = beta * C[seg] + alpha * rowscale .* (op(A) .* colscale) * B[seg]
//
// op(A) is M x K (row-major A, or the transpose of a row-major K x M array);
// B and C are row-major.  The columns of C may span two segments with their
// own base pointers (used to update a factor matrix and its right-hand sides
// in one launch).  All bounds are checked, so ragged shapes are fine.
//
// Tiling: a 256-thread workgroup computes a 128 x 128 tile; each of its four
// waves owns 64 x 64 = 4 x 4 blocks of v_mfma_{f64,f32}_16x16x4.  Fragments
// are loaded straight from global memory into registers (no LDS): within a
// 16-wide K chunk, lane group g = lane / 16 takes k = 4g + s at MFMA step s,
// so each lane reads 4 consecutive K entries of a row of A and every 16-lane
// group reads 16 consecutive entries of a row of B.  The next chunk is loaded
// while the current one is multiplied.
#pragma once

#include <hip/hip_runtime.h>

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
  const T* colscale;   // length K or null: op(A)[:, k] *= colscale[k]
  const T* rowscale;   // length M or null: product row i *= rowscale[i]
  T alpha, beta;
  int nseg;
  int ntile[2];        // 128-wide column tiles per segment
  int N[2];
  const T* B[2];
  long ldb[2];
  T* C[2];
  long ldc[2];
};

constexpr int GEMM_TILE = 128;
constexpr int GEMM_KC = 16;

template <class T, bool TRANS_A>
__global__ void __launch_bounds__(256, sizeof(T) == 8 ? 1 : 2) gemm_mfma(GemmArgs<T> g) {
  typedef typename Mfma<T>::v4 v4;
  int ct = blockIdx.x;
  int seg = 0;
  if (ct >= g.ntile[0]) {
    seg = 1;
    ct -= g.ntile[0];
  }
  const T* __restrict__ Bm = g.B[seg];
  T* __restrict__ Cm = g.C[seg];
  const long ldb = g.ldb[seg], ldc = g.ldc[seg];
  const int N = g.N[seg], M = g.M, K = g.K;
  const T* __restrict__ A = g.A;
  const long lda = g.lda;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int li = l & 15, lg = l >> 4;
  const int wr0 = blockIdx.y * GEMM_TILE + (wave >> 1) * 64;
  const int wc0 = ct * GEMM_TILE + (wave & 1) * 64;

  v4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4{0, 0, 0, 0};

  T fa[4][4], fb[4][4], na[4][4], nb[4][4];
  auto load = [&](int kc, T (&xa)[4][4], T (&xb)[4][4]) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int i = wr0 + rb * 16 + li;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kc + 4 * lg + s;
        T v = T(0);
        if (i < M && k < K) {
          v = TRANS_A ? A[static_cast<long>(k) * lda + i] : A[static_cast<long>(i) * lda + k];
          if (g.colscale) v *= g.colscale[k];
        }
        xa[rb][s] = v;
      }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int j = wc0 + cb * 16 + li;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kc + 4 * lg + s;
        xb[cb][s] = (j < N && k < K) ? Bm[static_cast<long>(k) * ldb + j] : T(0);
      }
    }
  };

  load(0, fa, fb);
  for (int kc = 0; kc < K; kc += GEMM_KC) {
    const bool more = kc + GEMM_KC < K;
    if (more) load(kc + GEMM_KC, na, nb);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = Mfma<T>::mma(fa[rb][s], fb[cb][s], acc[rb][cb]);
    if (more) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          fa[a][s] = na[a][s];
          fb[a][s] = nb[a][s];
        }
    }
  }
  // C may alias A or B (in-place block products): every wave must finish
  // reading before any wave writes.
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr0 + rb * 16 + Mfma<T>::orow(l, r);
        const int j = wc0 + cb * 16 + li;
        if (i < M && j < N) {
          T v = acc[rb][cb][r];
          if (g.rowscale) v *= g.rowscale[i];
          v *= g.alpha;
          T* p = Cm + static_cast<long>(i) * ldc + j;
          if (g.beta != T(0)) v += g.beta * *p;
          *p = v;
        }
      }
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
  dim3 grid(static_cast<unsigned>(total), static_cast<unsigned>((a.M + GEMM_TILE - 1) / GEMM_TILE));
  double ncols = 0.0;
  for (int q = 0; q < a.nseg; ++q) ncols += a.N[q];
  ProfScope prof(s, sizeof(T) == 8 ? RAD_PROF_GEMM_F64 : RAD_PROF_GEMM_F32,
                 2.0 * a.M * ncols * a.K, 0.0);
  if (trans_a)
    hipLaunchKernelGGL((gemm_mfma<T, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_mfma<T, false>), grid, dim3(256), 0, s, a);
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
