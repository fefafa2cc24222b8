// Operand scaling and splitting for the int8-emulated FP64 products of
// emu_kernels.h: the scale exponent of every operand row and the S digit
// slices of every operand element, written in the digit layout that the
// product stages into LDS with straight copies.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "emu_kernels.h"

namespace rad {

// Operand access: row r < R0 is element (r, k) at X[0][r sr[0] + k sk[0]],
// row R0 <= r < R at X[1][(r - R0) sr[1] + k sk[1]]; both segments have the
// same orientation (k contiguous, or rows contiguous).  Rows r >= R and
// k >= K of the padded range read as zero.
struct EmuOperand {
  const double* X[2];
  long sr[2], sk[2];
  int R0, R, K;
};

// Row r of an operand as a base pointer and k stride.  A row r >= R (the
// padding of the last tile) maps to row 0 with ok = false: its loads read a
// valid address and are discarded, so that no load sits behind a branch and
// a thread's loads are all in flight together.
struct EmuRow {
  const double* p;
  long sk;
  bool ok;
};

__device__ __forceinline__ EmuRow emu_row(const EmuOperand& op, int r) {
  const bool ok = r < op.R;
  const int rr = ok ? r : 0;
  const bool q = rr >= op.R0;
  const double* X = q ? op.X[1] : op.X[0];
  const long sr = q ? op.sr[1] : op.sr[0];
  return EmuRow{X + static_cast<long>(rr - (q ? op.R0 : 0)) * sr, q ? op.sk[1] : op.sk[0], ok};
}

// Element (row, k) of the operand, zero outside R x K (k clamped to K - 1 for
// the address; K >= 1 wherever a split is launched).  The select is marked
// unpredictable: otherwise the compiler turns a select on a loaded value
// into a branch around the load, and every load waits for the previous one.
__device__ __forceinline__ double emu_elem(const EmuRow& w, int k, int K) {
  const double v = w.p[static_cast<long>(min(k, K - 1)) * w.sk];
  const bool keep = w.ok & (k < K);
  return __builtin_unpredictable(keep) ? v : 0.0;
}

// Scale exponents e_r (max_k |X_rk| < 2^e_r; EMU_EXP_NONE for a zero row) of
// rows [r0, r1).  k-contiguous rows: one wave per row, sixteen loads per lane
// in flight per 1024 k.
__device__ __forceinline__ void emu_rowexp_kc_body(const EmuOperand& op, int r0, int r1, int* __restrict__ ex,
                                                   int blk) {
  const int r = r0 + blk * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (r >= r1) return;
  const EmuRow w = emu_row(op, r);
  double m = 0.0;
  for (int k0 = 0; k0 < op.K; k0 += 16 * 64) {
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = emu_elem(w, k0 + l + 64 * j, op.K);
#pragma unroll
    for (int j = 0; j < 16; ++j) m = fmax(m, fabs(v[j]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  int e = 0;
  if (m > 0.0) frexp(m, &e);  // m = f 2^e, f in [0.5, 1): m < 2^e
  if (l == 0) ex[r] = m > 0.0 ? e : EMU_EXP_NONE;
}

static __global__ __launch_bounds__(256) void emu_rowexp_kc(EmuOperand op, int r0, int r1, int* __restrict__ ex) {
  emu_rowexp_kc_body(op, r0, r1, ex, blockIdx.x);
}

// Rows contiguous in memory: a workgroup takes one 64-row tile rt x one k
// block kb (lane l of wave w reads row l at k = w, w + 4, ..., every load
// instruction 512 contiguous bytes, sixteen loads per lane in flight) and
// stores the exponent of each row's k block in part[kb Rp + r] (Rp: the
// operand's padded row count); the digit pass takes the maximum over the k
// blocks, so no atomics and no initial fill are needed.
__device__ __forceinline__ void emu_rowexp_rc_body(const EmuOperand& op, int rt, int kb, int* __restrict__ part,
                                                   long Rp) {
  __shared__ double wm[4][EMU_TILE];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = rt * EMU_TILE + l, k0 = kb * EMU_KB + wv;
  const EmuRow w = emu_row(op, r);
  double v[EMU_KB / 4];
#pragma unroll
  for (int j = 0; j < EMU_KB / 4; ++j) v[j] = emu_elem(w, k0 + 4 * j, op.K);
  double m = 0.0;
#pragma unroll
  for (int j = 0; j < EMU_KB / 4; ++j) m = fmax(m, fabs(v[j]));
  wm[wv][l] = m;
  __syncthreads();
  if (wv == 0) {
    m = fmax(fmax(wm[0][l], wm[1][l]), fmax(wm[2][l], wm[3][l]));
    int e = EMU_EXP_NONE;
    if (m > 0.0) frexp(m, &e);
    part[kb * Rp + r] = e;
  }
}

static __global__ __launch_bounds__(256) void emu_rowexp_rc(EmuOperand op, int rt0, int* __restrict__ part, long Rp) {
  emu_rowexp_rc_body(op, rt0 + blockIdx.x, blockIdx.y, part, Rp);
}

// Digits of one 64-row x 64-k block per workgroup (row tile rt of T).  The
// block's doubles are read with 512-byte contiguous loads in whichever
// orientation the operand has (sixteen per thread, all in flight) and
// transposed through LDS; thread t forms the S digits of 16 consecutive k of
// row t / 4 (chunk c = t % 4), and a wave's stores of one slice are one
// contiguous 1 KB piece of the block.  k-contiguous operands read their
// exponents from ex; rows-contiguous ones take the maximum of the nkb
// per-k-block exponents in part (layout of emu_rowexp_rc, Rp = 64 T; the four
// threads of a row read a quarter each), and the workgroups of k block 0
// store it in ex for the product.
template <int S, bool KC>
__device__ __forceinline__ void emu_split_body(const EmuOperand& op, int T, int rt, int kb, int* __restrict__ ex,
                                               const int* __restrict__ part, int nkb, int8_t* __restrict__ out,
                                               double (*tile)[EMU_KB + 1]) {
  const int t = threadIdx.x;
  const int r0 = rt * EMU_TILE, k0 = kb * EMU_KB;
  constexpr int NL = EMU_TILE * EMU_KB / 256;
  double v[NL];
  if (KC) {  // lane: one k; the workgroup's rows t / 64, t / 64 + 4, ...
#pragma unroll
    for (int it = 0; it < NL; ++it) v[it] = emu_elem(emu_row(op, r0 + it * 4 + (t >> 6)), k0 + (t & 63), op.K);
  } else {  // lane: one row; k = t / 64, t / 64 + 4, ...
    const EmuRow w = emu_row(op, r0 + (t & 63));
#pragma unroll
    for (int it = 0; it < NL; ++it) v[it] = emu_elem(w, k0 + it * 4 + (t >> 6), op.K);
  }
  const int row = t >> 2, c = t & 3;
  int e;
  if (KC) {
    e = ex[r0 + row];
  } else {
    const long Rp = static_cast<long>(T) * EMU_TILE;
    e = EMU_EXP_NONE;
    for (int q0 = 0; q0 < nkb; q0 += 16) {
      int pv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) pv[j] = part[min(q0 + c + 4 * j, nkb - 1) * Rp + r0 + row];
#pragma unroll
      for (int j = 0; j < 4; ++j) e = max(e, pv[j]);
    }
    e = max(e, __shfl_xor(e, 1));
    e = max(e, __shfl_xor(e, 2));
    if (kb == 0 && c == 0) ex[r0 + row] = e;
  }
#pragma unroll
  for (int it = 0; it < NL; ++it) {
    if (KC) tile[it * 4 + (t >> 6)][t & 63] = v[it];
    else tile[t & 63][it * 4 + (t >> 6)] = v[it];
  }
  __syncthreads();
  const int es = e == EMU_EXP_NONE ? 0 : e;
  union {
    emu_v4i v;
    int8_t b[16];
  } dg[S];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double a = ldexp(tile[row][c * 16 + i], -es);  // exact
#pragma unroll
    for (int s = 0; s < S; ++s) {
      a *= 128.0;
      const double d = __builtin_trunc(a);
      a -= d;
      dg[s].b[i] = static_cast<int8_t>(static_cast<int>(d));
    }
  }
  emu_v4i* blk = reinterpret_cast<emu_v4i*>(out) + (static_cast<long>(kb) * T + rt) * S * 256;
#pragma unroll
  for (int s = 0; s < S; ++s) blk[emu_lds_idx(s, row, c)] = dg[s].v;
}

template <int S, bool KC>
__global__ __launch_bounds__(256) void emu_split(EmuOperand op, int T, int rt0, int* __restrict__ ex,
                                                 const int* __restrict__ part, int8_t* __restrict__ out) {
  __shared__ double tile[EMU_TILE][EMU_KB + 1];
  emu_split_body<S, KC>(op, T, rt0 + blockIdx.x, blockIdx.y, ex, part, gridDim.y, out, tile);
}

// ---- host side ------------------------------------------------------------

// Bytes of the digits of an operand with R rows and K columns.
inline size_t emu_digit_bytes(long R, long K) {
  return static_cast<size_t>((R + EMU_TILE - 1) / EMU_TILE) * EMU_TILE * ((K + EMU_KB - 1) / EMU_KB) * EMU_KB * EMU_S;
}

// Scale exponents and digits of the row tiles [t0, t1) of one operand (kc: k
// contiguous in memory, else rows; t1 < 0: up to the last tile).  ex receives
// one exponent per padded row; the digits land where the whole operand's
// layout puts them, so disjoint tile ranges may be prepared by separate calls.
// A rows-contiguous operand needs part, emu_part_count(R, K) ints of scratch
// (per-k-block exponents).
inline hipError_t emu_prepare(const EmuOperand& op, bool kc, int8_t* dig, int* ex, int* part, hipStream_t s,
                              int t0 = 0, int t1 = -1) {
  const int T = (op.R + EMU_TILE - 1) / EMU_TILE;
  const int nkb = (op.K + EMU_KB - 1) / EMU_KB;
  if (t1 < 0 || t1 > T) t1 = T;
  if (t0 >= t1 || nkb == 0) return hipSuccess;
  const int r0 = t0 * EMU_TILE, r1 = t1 * EMU_TILE, nr = r1 - r0;
  if (kc) {
    hipLaunchKernelGGL(emu_rowexp_kc, dim3((nr + 3) / 4), dim3(256), 0, s, op, r0, r1, ex);
    hipLaunchKernelGGL((emu_split<EMU_S, true>), dim3(t1 - t0, nkb), dim3(256), 0, s, op, T, t0, ex,
                       static_cast<const int*>(nullptr), dig);
  } else {
    if (!part) return hipErrorInvalidValue;
    const long Rp = static_cast<long>(T) * EMU_TILE;
    hipLaunchKernelGGL(emu_rowexp_rc, dim3(t1 - t0, nkb), dim3(256), 0, s, op, t0, part, Rp);
    hipLaunchKernelGGL((emu_split<EMU_S, false>), dim3(t1 - t0, nkb), dim3(256), 0, s, op, T, t0, ex,
                       static_cast<const int*>(part), dig);
  }
  return hipGetLastError();
}

// Entries of the exponent array of an operand with R rows.
inline size_t emu_scale_count(long R) { return static_cast<size_t>((R + EMU_TILE - 1) / EMU_TILE) * EMU_TILE; }

// Entries of the per-k-block exponent scratch of a rows-contiguous operand.
inline size_t emu_part_count(long R, long K) {
  return emu_scale_count(R) * static_cast<size_t>((K + EMU_KB - 1) / EMU_KB);
}

}  // namespace rad
