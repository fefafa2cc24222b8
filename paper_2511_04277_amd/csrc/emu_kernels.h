// FP64 matrix products emulated on the int8 matrix cores (gfx950).
//
//   C[seg] += alpha * A * B,   A: M x K,  B: K x N,  C FP64
//
// Error-free splitting (Ozaki's scheme): every row r of an operand (a row of
// A, a column of B) is scaled by the power of two sigma_r = 2^e_r >
// max_k |X_rk| and written as S signed 7-bit digits,
//
//   X_rk = sigma_r * sum_{s<S} d_s(r,k) 2^{-7(s+1)} + t_rk,   |d_s| <= 127,
//   |t_rk| < sigma_r 2^{-7S},
//
// each step (scale by 128, truncate, subtract) exact in FP64.  Products of
// digit matrices D^A_s D^B_t are exact in int32 (v_mfma_i32_16x16x64_i8);
// the pairs with s + t >= S are dropped, and the kept pairs accumulate in
// int32 per class d = s + t over the whole K (|sum| <= S K 127^2 < 2^31 for
// K <= EMU_MAX_K), so the FP64 work is one fold per output element:
// sum_d acc_d 2^{-7(d+2)}, times sigma^A_i sigma^B_j.  Per element the result
// differs from the exact product by less than
//   (S + 3) K sigma^A_i sigma^B_j 2^{-7S}
// (the two tails and the dropped pairs) plus the fold's FP64 rounding; with
// S = 7 that is 2^-49 per unit of K sigma^A sigma^B as a worst case, and in
// practice (errors of random sign) about 2^-49 sqrt(K) of the row and column
// maxima.
//
// Digit layout (written by emu_split in emu_split.h, read by emu_gemm): operand rows padded
// to a multiple of 64 (T tiles) and k to 64 nkb.  The 64 rows x S slices x
// 64 k of k block kb of row tile rt are block kb T + rt, S * 256 chunks of 16
// bytes, laid out exactly as the GEMM keeps them in LDS: chunk c
// (k 16c..16c+15) of row rr of slice s at position emu_lds_idx(s, rr, c), so
// the GEMM stages a block with straight 1 KB global-to-LDS copies.  Padding
// digits are zero.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gemm.h"

namespace rad {

constexpr int EMU_S = 7;          // digits per operand element
constexpr int EMU_TILE = 64;      // C tile of one workgroup (64 x 64)
constexpr int EMU_KB = 64;        // k per stage (one MFMA 16 x 16 x 64)
constexpr int EMU_THREADS = 256;  // four waves, 32 x 32 of C each
constexpr int EMU_MAX_K = 16384;  // S K 127^2 < 2^31 for S = 7
constexpr int EMU_EXP_NONE = -2000;  // scale exponent of an all-zero row

typedef int emu_v4i __attribute__((ext_vector_type(4)));

// LDS position of 16-byte chunk c of row r of slice s in a 64-row block.
// The chunk index is XOR-swizzled with row bits so that the 16 (or 8) lanes
// of one ds_read_b128 phase, which read rows r..r+15 at one chunk, hit
// distinct banks.
__device__ __forceinline__ int emu_lds_idx(int s, int r, int c) {
  return ((s * EMU_TILE + r) << 2) + (c ^ (((r >> 1) ^ (r >> 2)) & 3));
}

// ---- the product --------------------------------------------------------

struct EmuGemmArgs {
  const int8_t* A;   // digits of A: mt 64-row tiles per k block
  const int* xa;     // scale exponents of the rows of A
  const int8_t* B;   // digits of B^T (rows = columns of C): nt tiles per k block
  const int* xb;     // scale exponents of the columns of B
  int mt, nt, nkb;
  int ty0, nty;      // the launch covers A tiles [ty0, ty0 + nty) ...
  int tx0, ntx;      // ... times B tiles [tx0, tx0 + ntx)
  int M;             // rows i < M of C are written
  double alpha;
  int nseg;          // column j < N[0]: C[0][i ldc[0] + j]; else C[1][i ldc[1] + j - N[0]]
  int N[2];
  double* C[2];
  long ldc[2];
};

// One 64 x 64 tile of C per workgroup, two workgroups per CU (56 KB of LDS
// each, at most 256 registers per lane).  Per k block: the block's digits
// arrive in LDS by global-to-LDS copies, every wave reads all its fragments
// (S slices x 2 row blocks of A, S x 2 column blocks of B) into registers, the
// LDS is released and the next block's copies start, and the 28 digit-pair
// MFMAs run from registers meanwhile into S int32 class accumulators that
// persist over the whole K.  During the last block's MFMAs the freed LDS
// receives the tile's C block and its row and column scale exponents (tiles
// that lie whole inside one column segment), so the epilogue does not wait
// on global loads: 14-17 % faster on K = 1024 products than loading C in
// the epilogue, bitwise the same results.
template <int S>
__device__ __forceinline__ void emu_gemm_tile(const EmuGemmArgs& g, int bx, int by,
                                              emu_v4i (*lds)[S * EMU_TILE * 4]) {
  constexpr int CH = S * EMU_TILE * 4;  // 16-byte chunks per operand block
  static_assert(2 * CH * 16 >= EMU_TILE * EMU_TILE * 8 + 2 * EMU_TILE * 4, "C block must fit the LDS");
  // the wave index is uniform: the copies' addresses become a scalar base and
  // one lane offset
  const int t = threadIdx.x, l = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const emu_v4i* ga = reinterpret_cast<const emu_v4i*>(g.A) + static_cast<long>(by) * CH;
  const emu_v4i* gb = reinterpret_cast<const emu_v4i*>(g.B) + static_cast<long>(bx) * CH;
  const long stride_a = static_cast<long>(g.mt) * CH;
  const long stride_b = static_cast<long>(g.nt) * CH;
  // copies of one k block: wave w moves 1 KB pieces w, w + 4, ... of A then
  // B.  The B copies carry the sc0 cache policy: B's column panels stream
  // past the 8 tile rows that an XCD holds at a time; alone on a 7168 x 8193
  // x 1024 product the bit makes the kernel 18-24 % faster (A with it too: no
  // further gain); inside the solve the difference is within noise.
  auto stage = [&](int kb) {
    const emu_v4i* sa = ga + kb * stride_a;
    const emu_v4i* sb = gb + kb * stride_b;
    static_assert(CH % 256 == 0, "whole pieces per wave");
#pragma unroll
    for (int i = 0; i < CH / 256; ++i) {
      const int p = w + 4 * i;
      __builtin_amdgcn_global_load_lds(sa + p * 64 + l, (__attribute__((address_space(3))) void*)(&lds[0][p * 64]), 16, 0, 0);
      __builtin_amdgcn_global_load_lds(sb + p * 64 + l, (__attribute__((address_space(3))) void*)(&lds[1][p * 64]), 16, 0, 1);
    }
  };
  // a tile whole inside one column segment stages C in LDS (row-major 64 x 64
  // doubles, then 64 row and 64 column exponents)
  const int row0t = by * EMU_TILE, col0t = bx * EMU_TILE;
  const int seg0 = (g.nseg > 1 && col0t >= g.N[0]) ? 1 : 0;
  const int cc0 = col0t - (seg0 ? g.N[0] : 0);
  const bool cpre =
      __builtin_amdgcn_readfirstlane(row0t + EMU_TILE <= g.M && seg0 < g.nseg && cc0 + EMU_TILE <= g.N[seg0]);
  double* cl = reinterpret_cast<double*>(&lds[0][0]);
  int* xl = reinterpret_cast<int*>(cl + EMU_TILE * EMU_TILE);
  auto stage_c = [&]() {
    const double* cbase = g.C[seg0] + static_cast<long>(row0t) * g.ldc[seg0] + cc0;
    const long cld = g.ldc[seg0];
    // wave w copies rows 16 w .. 16 w + 15, two 512-byte rows per instruction
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = 16 * w + 2 * q + (l >> 5), c = l & 31;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const emu_v4i*>(cbase + r * cld + 2 * c),
                                       (__attribute__((address_space(3))) void*)(cl + (16 * w + 2 * q) * EMU_TILE),
                                       16, 0, 0);
    }
    if (w == 0)
      __builtin_amdgcn_global_load_lds(g.xa + row0t + l, (__attribute__((address_space(3))) void*)(xl), 4, 0, 0);
    else if (w == 1)
      __builtin_amdgcn_global_load_lds(g.xb + col0t + l, (__attribute__((address_space(3))) void*)(xl + EMU_TILE), 4,
                                       0, 0);
  };
  const int fr = l & 15, fc = l >> 4;
  emu_v4i ci[S][2][2];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) ci[d][i][j] = emu_v4i{0, 0, 0, 0};
  // one k block: wait for its copies, read the fragments, release the LDS,
  // issue the next copies, then the digit-pair MFMAs (pair (s, u) into class
  // s + u; consecutive MFMAs go to different classes)
  auto block = [&](auto next) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
    __syncthreads();                // and everyone else's
    emu_v4i af[S][2], bf[S][2];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[s][i] = lds[0][emu_lds_idx(s, wr + 16 * i + fr, fc)];
        bf[s][i] = lds[1][emu_lds_idx(s, wc + 16 * i + fr, fc)];
      }
    __syncthreads();  // every wave holds its fragments: the LDS is free
    next();
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int u = 0; u < S - s; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            ci[s + u][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[s][i], bf[u][j], ci[s + u][i][j], 0, 0, 0);
  };
  // A tile whose operand rows (or columns) all have zero scale exponents
  // (all-zero rows of A, columns of B: coplanar faces see each other with
  // zero view factor, so whole 64 x 64 blocks of the factors and right-hand
  // sides are zero) adds nothing to C; every wave finds the same answer and
  // leaves before copying anything.
  {
    const int ea = g.xa[row0t + l], eb = g.xb[col0t + l];  // both loads in flight together
    const bool za = __all(ea == EMU_EXP_NONE), zb = __all(eb == EMU_EXP_NONE);
    if (za | zb) return;
  }
  stage(0);
  // the last block is peeled so that the C staging's addresses are not held
  // across the loop
  for (int kb = 0; kb + 1 < g.nkb; ++kb) block([&] { stage(kb + 1); });
  block([&] {
    if (cpre) stage_c();
  });
  // epilogue: lane l holds rows 4 (l / 16) + v, column l % 16 of each block;
  // one FP64 fold of the S class sums per element
  const int row0 = row0t + wr, col0 = col0t + wc;
  if (cpre) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const long ldc = g.ldc[seg0];
    double* Cb = g.C[seg0] + static_cast<long>(row0) * ldc + (cc0 + wc);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int eb = xl[EMU_TILE + wc + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = 16 * i + 4 * fc + v;
          const int ea = xl[wr + rr];
          if (ea == EMU_EXP_NONE || eb == EMU_EXP_NONE) continue;  // a zero row or column adds nothing
          double x = 0.0;
#pragma unroll
          for (int d = S - 1; d >= 0; --d) x = fma(static_cast<double>(ci[d][i][j][v]), ldexp(1.0, -7 * (d + 2)), x);
          const double c0 = cl[(wr + rr) * EMU_TILE + wc + 16 * j + fr];
          Cb[static_cast<long>(rr) * ldc + 16 * j + fr] = fma(g.alpha, ldexp(x, ea + eb), c0);
        }
    }
    return;
  }
  // edge tiles: per column block, C and the exponents with every load issued
  // before the first is used (addresses clamped into the matrix; the padded
  // exponent arrays cover every row and column of a tile)
  int eav[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) eav[i][v] = g.xa[row0 + 16 * i + 4 * fc + v];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = col0 + 16 * j + fr;
    const int seg = (g.nseg > 1 && col >= g.N[0]) ? 1 : 0;
    const int cc = col - (seg ? g.N[0] : 0);
    const int nseg_cols = seg ? g.N[1] : g.N[0];
    double* Cc = (seg ? g.C[1] : g.C[0]) + min(cc, nseg_cols - 1);
    const long ldc = seg ? g.ldc[1] : g.ldc[0];
    const int eb = g.xb[col];
    double cv[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) cv[i][v] = Cc[static_cast<long>(min(row0 + 16 * i + 4 * fc + v, g.M - 1)) * ldc];
    if (seg >= g.nseg || cc >= nseg_cols) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + 16 * i + 4 * fc + v;
        const int ea = eav[i][v];
        if (row >= g.M || ea == EMU_EXP_NONE || eb == EMU_EXP_NONE) continue;  // a zero row or column adds nothing
        double x = 0.0;
#pragma unroll
        for (int d = S - 1; d >= 0; --d) x = fma(static_cast<double>(ci[d][i][j][v]), ldexp(1.0, -7 * (d + 2)), x);
        Cc[static_cast<long>(row) * ldc] = fma(g.alpha, ldexp(x, ea + eb), cv[i][v]);
      }
  }
}

template <int S>
__global__ __launch_bounds__(EMU_THREADS, 2) void emu_gemm(EmuGemmArgs g) {
  __shared__ emu_v4i lds[2][S * EMU_TILE * 4];  // [A, B][chunk]
  int bx, by;
  grouped_tile(xcd_contiguous(blockIdx.x, g.ntx * g.nty), g.ntx, g.nty, TILE_GROUP, bx, by);
  emu_gemm_tile<S>(g, bx + g.tx0, by + g.ty0, lds);
}

// Many products in one launch with one workgroup per tile (grid = the
// concatenated tile list, handed out in list order): each tile stages its C
// block in LDS as emu_gemm does.
template <int S>
__global__ __launch_bounds__(EMU_THREADS, 2) void emu_gemm_grouped_tiles(const EmuGemmArgs* __restrict__ probs,
                                                                         const int* __restrict__ tile_start,
                                                                         int nprob) {
  __shared__ emu_v4i lds[2][S * EMU_TILE * 4];
  const int b = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const EmuGemmArgs& g = probs[lo];
  int bx, by;
  grouped_tile(b - tile_start[lo], g.ntx, g.nty, TILE_GROUP, bx, by);
  emu_gemm_tile<S>(g, bx + g.tx0, by + g.ty0, lds);
}

// ---- host side ------------------------------------------------------------

inline hipError_t emu_launch(const EmuGemmArgs& g, hipStream_t s) {
  if (g.ntx <= 0 || g.nty <= 0 || g.nkb <= 0) return hipSuccess;
  hipLaunchKernelGGL(emu_gemm<EMU_S>, dim3(g.ntx * g.nty), dim3(EMU_THREADS), 0, s, g);
  return hipGetLastError();
}

}  // namespace rad
