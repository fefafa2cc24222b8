// Enforcement kernels (thesis Sec. 3.5.5) shared by the single-instance and
// batched entry points.  See enforce.hip for the algorithm.
#pragma once

#include "common.h"

namespace rad {
namespace {

constexpr int ET = 64;          // tile edge (doubles)
constexpr int ETP = ET + 1;     // padded LDS row (conflict-free transpose)
// 8 waves of 8 tile rows each: at 4 waves per SIMD (two workgroups per
// CU) the sweep keeps twice the loads in flight of a 4-wave shape
constexpr int ENF_THREADS = 512;
constexpr int ENW = ENF_THREADS / 64;  // waves per sweep workgroup

struct EnfCtrl {
  int status;        // device-raised status (0 ok, negative error)
  int converged;     // 1 once the tolerance is met
  int iters;         // iterations executed
  int done;          // finalize blocks of the current iteration that finished
  double last_defect, last_recip;
};


// One enforcement problem as the kernels see it.
struct EnfInst {
  double* F;
  long ldf;
  int n, t;                 // faces, 64-wide tiles per side
  long pairs;               // t (t + 1) / 2 tile pairs
  const double* area;
  const double* inv_area;   // 1 / A_i (workspace)
  const double* nrays;      // null for kappa = 1/2
  int mode;
  double* scale;            // 1 / s_i of the last closure step
  double* partial;          // (t + 1) x n partial row sums
  double* blkmax;           // 2 per tile pair: max |eta_ij - eta_ji|, max eta
  double* finred;           // 3 per finalize block: closure defect, the two maxima
  EnfCtrl* ctrl;
};

constexpr int ERW = ET / ENW;  // tile rows per wave
static_assert(2 + 2 * ENW <= ET, "the row partials and maxima reuse rows of the tile buffer");

// Element col of a row whose base pointer is wave-uniform: the byte offset
// is a 32-bit lane value, so loads and stores take the scalar-base form and
// one offset register serves every row.
// (readfirstlane pins the row pointer to scalar registers, so the compiler
// cannot fold the lane offset into a per-row vector address).
// The pointer is rebuilt in the global address space: a generic (flat)
// pointer would make every access a flat instruction with a 64-bit address
// per lane, which costs two registers per load in flight.
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gchar* uniform_ptr(const double* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v >> 32));
  return reinterpret_cast<gchar*>((static_cast<unsigned long long>(hi) << 32) | lo);
}
// F streams through once per sweep (it is larger than the last-level cache
// at the sizes that matter), so its loads and stores are nontemporal.
__device__ __forceinline__ double row_ld(const double* row, unsigned col) {
  return __builtin_nontemporal_load(reinterpret_cast<const gdouble*>(uniform_ptr(row) + col * 8u));
}
__device__ __forceinline__ void row_st(double* row, unsigned col, double v) {
  __builtin_nontemporal_store(v, reinterpret_cast<gdouble*>(uniform_ptr(row) + col * 8u));
}

// kappa of eq. 3.25 from the pair (f_ij, f_ji) and c = A^2 / N of both faces:
// kappa = b / (a + b), a = c_i (1 - f_ij) f_ji, b = c_j (1 - f_ji) f_ij (the
// variances of eq. 3.23 multiplied by F_ij F_ji); 1/2 when both vanish.
// The quotient uses the hardware reciprocal refined by two Newton steps.
// Every operation rounds as written (no contraction into fused multiply-adds
// beyond the two explicit Newton steps), so the result does not depend on how
// the compiler schedules the surrounding code.
__device__ __forceinline__ double kappa_c(double fij, double fji, double ci, double cj) {
#pragma clang fp contract(off)
  const double a = ci * (1.0 - fij) * fji;
  const double b = cj * (1.0 - fji) * fij;
  const double s = a + b;
  double r = __builtin_amdgcn_rcp(s);
  r = r * __builtin_fma(-s, r, 2.0);
  r = r * __builtin_fma(-s, r, 2.0);
  return s > 0.0 ? b * r : 0.5;
}

// One workgroup per tile pair (I, J), I <= J, of 64 x 64 tiles.  Lane l of
// wave w holds column l of tile rows w, w + ENW, ..., so every load and
// store instruction of a wave moves one contiguous 512-byte tile row.  The
// partner tile (J, I) is staged through LDS (65-double rows), where each
// unordered pair {i, j} meets its mirror; the previous iteration's closure
// scale 1 / s_i is applied on load.  The thread that updates pair (i, j)
// also produces the partner's entry (j, i), and its ERW pairs all lie in one
// partner row, so the partner's row sums are formed in registers; the own
// tile's rows are summed after a transpose through the same LDS buffer.
// All sums run in a fixed order (bitwise reproducible).  DIAG: I == J (each
// unordered pair once, the diagonal kept, the space column carried along);
// EDGE: the tile pair crosses n (clamped loads, masked stores).
template <bool DIAG, bool EDGE, bool HALF>
__device__ __forceinline__ void enf_sweep_tile(const EnfInst& in, long pair, int I, int J, int first,
                                               double (*sB)[ETP], double (*rowc)[ET]) {
#pragma clang fp contract(off)
  double* __restrict__ F = in.F;
  const long ldf = in.ldf;
  const int n = in.n;
  const double* __restrict__ area = in.area;
  const double* __restrict__ inv_area = in.inv_area;
  const double* __restrict__ nrays = in.nrays;
  const bool half = HALF;
  const double* __restrict__ inv_scale = in.scale;
  const int r0 = I * ET, c0 = J * ET;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  int bad = 0;

  // The tiles' loads go out first, so that their latency covers the loads
  // of the per-row constants below.  Own tile (I, J): a[k] = F(r0 + w +
  // ENW k, c0 + l); partner tile (J, I): b[k] = F(c0 + w + ENW k, r0 + l).
  // Row pointers are wave-uniform and the lane adds its column, so loads
  // use a scalar base.
  const int jg = c0 + l;
  const int jgc = (EDGE && jg >= n) ? n - 1 : jg;
  const int ig = r0 + l;
  const int igc = (EDGE && ig >= n) ? n - 1 : ig;
  double a[ERW], b[ERW];
#pragma unroll
  for (int k = 0; k < ERW; ++k) {
    const int i = r0 + w + ENW * k;
    const int ic = (EDGE && i >= n) ? n - 1 : i;
    a[k] = row_ld(F + static_cast<long>(ic) * ldf, jgc);
  }
  if (!DIAG) {
#pragma unroll
    for (int k = 0; k < ERW; ++k) {
      const int jr = c0 + w + ENW * k;
      const int jrc = (EDGE && jr >= n) ? n - 1 : jr;
      b[k] = row_ld(F + static_cast<long>(jrc) * ldf, igc);
    }
  }
  // per-row constants: area, 1 / area, A^2 / N and the previous closure
  // scale 1 / s of the own tile's rows (rowc[0..3]) and of the partner
  // tile's rows (rowc[4..7])
  if (tid < (DIAG ? ET : 2 * ET)) {
    const int q = tid < ET ? 0 : 4;
    const int base = tid < ET ? r0 : c0;
    const int rl = tid & (ET - 1);
    const int i = (EDGE && base + rl >= n) ? n - 1 : base + rl;
    const double ai = area[i];
    rowc[q + 0][rl] = ai;
    rowc[q + 1][rl] = inv_area[i];
    rowc[q + 2][rl] = half ? 0.0 : ai * ai / nrays[i];
    rowc[q + 3][rl] = first ? 1.0 : inv_scale[i];
  }
  __syncthreads();
  // scaled by the positive finite 1 / s (1 on the first sweep); negative or
  // non-finite inputs stay so and are caught where the pair is formed
#pragma unroll
  for (int k = 0; k < ERW; ++k) {
    const int i = r0 + w + ENW * k;
    double v = a[k];
    if (EDGE && !(i < n && jg < n)) v = 0.0;
    a[k] = v * rowc[3][w + ENW * k];
  }
  // partner tile into LDS: sB[jl][il] = F(c0 + jl, r0 + il)
  if (!DIAG) {
#pragma unroll
    for (int k = 0; k < ERW; ++k) {
      const int jr = c0 + w + ENW * k;
      double v = b[k];
      if (EDGE && !(jr < n && ig < n)) v = 0.0;
      sB[w + ENW * k][l] = v * rowc[7][w + ENW * k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < ERW; ++k) sB[w + ENW * k][l] = a[k];
  }
  __syncthreads();

  // reciprocity on each unordered pair {i, j}, i != j, exactly once
  double rmax = 0.0, emax = 0.0, sb = 0.0;
  // constants of row c0 + l (the partner's row; on a diagonal tile the own rows)
  const double aj = rowc[DIAG ? 0 : 4][l], iaj = rowc[DIAG ? 1 : 5][l];
  const double cj = rowc[DIAG ? 2 : 6][l];
#pragma unroll
  for (int k = 0; k < ERW; ++k) {
    const int il = w + ENW * k;
    const double ai = rowc[0][il];
    if (DIAG) {
      if (l == il) {                               // the diagonal keeps its value
        emax = fmax(emax, ai * a[k]);
        bad |= !(a[k] >= 0.0) || !(a[k] <= 1.0e300);
      }
      if (l <= il) continue;                       // handled by the owner of (l, il)
    }
    const double iai = rowc[1][il];
    const double fij = a[k], fji = sB[l][il];
    bad |= !(fij >= 0.0) || !(fij <= 1.0e300) || !(fji >= 0.0) || !(fji <= 1.0e300);
    const double eij = ai * fij, eji = aj * fji;
    rmax = fmax(rmax, fabs(eij - eji));
    emax = fmax(emax, fmax(eij, eji));
    const double kp = half ? 0.5 : kappa_c(fij, fji, rowc[2][il], cj);
    const double eh = kp * eij + (1.0 - kp) * eji;
    const double bji = eh * iaj;
    a[k] = eh * iai;
    sB[l][il] = bji;
    sb += bji;
    // fold this pair into the running maxima and the error flag now: left to
    // itself the compiler keeps every pair's terms live and reduces them as a
    // tree after the loop, which doubles the registers of the kernel
    __asm__ volatile("" : "+v"(rmax), "+v"(emax), "+v"(bad), "+v"(sb));
  }
  __syncthreads();
  if (DIAG) {
#pragma unroll
    for (int k = 0; k < ERW; ++k)
      if (l < w + ENW * k) a[k] = sB[w + ENW * k][l];  // written by the owner of the mirror
  }

  // own tile back to F
#pragma unroll
  for (int k = 0; k < ERW; ++k) {
    const int i = r0 + w + ENW * k;
    if (!EDGE || (i < n && jg < n)) row_st(F + static_cast<long>(i) * ldf, jg, a[k]);
  }
  if (!DIAG) {  // partner tile back to F
    const int ig = r0 + l;
#pragma unroll
    for (int k = 0; k < ERW; ++k) {
      const int jr = c0 + w + ENW * k;
      if (!EDGE || (jr < n && ig < n)) row_st(F + static_cast<long>(jr) * ldf, ig, sB[w + ENW * k][l]);
    }
  }
  __syncthreads();
  // own tile transposed into LDS, then each thread sums ERW entries of row l
#pragma unroll
  for (int k = 0; k < ERW; ++k) sB[l][w + ENW * k] = a[k];
  for (int off = 32; off > 0; off >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, off));
    emax = fmax(emax, __shfl_xor(emax, off));
  }
  __syncthreads();
  double sa = 0.0;
#pragma unroll
  for (int k = 0; k < ERW; ++k) sa += sB[w + ENW * k][l];
  __syncthreads();
  // the transposed tile has been summed: LDS rows 2.. take this wave's
  // partial sums of the partner's row l and of the own row l, rows 0 and 1
  // the wave maxima
  sB[2 + w][l] = sb;
  sB[2 + ENW + w][l] = sa;
  if (l == 0) {
    sB[0][w] = rmax;
    sB[1][w] = emax;
  }
  __syncthreads();
  if (w == 0) {
    double s_own = 0.0, s_par = 0.0;
#pragma unroll
    for (int q = 0; q < ENW; ++q) {
      s_own += sB[2 + ENW + q][l];
      s_par += sB[2 + q][l];
    }
    const int t = in.t;
    double* __restrict__ partial = in.partial;
    if (!EDGE || r0 + l < n) partial[static_cast<long>(J) * n + r0 + l] = s_own;
    if (!DIAG && (!EDGE || c0 + l < n)) partial[static_cast<long>(I) * n + c0 + l] = s_par;
    if (DIAG && (!EDGE || r0 + l < n)) {  // the space column of the tile's rows rides with the diagonal tile
      double* sp = F + static_cast<long>(r0 + l) * ldf + n;
      double v = *sp;
      bad |= !(v >= 0.0) || !(v <= 1.0e300);
      v *= rowc[3][l];
      *sp = v;
      partial[static_cast<long>(t) * n + r0 + l] = v;
    }
    if (l == 0) {
      double x = sB[0][0], y = sB[1][0];
      for (int q = 1; q < ENW; ++q) {
        x = fmax(x, sB[0][q]);
        y = fmax(y, sB[1][q]);
      }
      in.blkmax[2 * pair] = x;
      in.blkmax[2 * pair + 1] = y;
    }
  }
  if (bad) raise_status(&in.ctrl->status, RAD_ENONFINITE);
}

__device__ __forceinline__ void enf_sweep_body(const EnfInst& in, long pair, int first) {
  if (in.ctrl->converged || in.ctrl->status < 0) return;
  __shared__ double sB[ET][ETP];
  __shared__ double rowc[8][ET];  // per-row constants of the own and the partner tile
  int I, J;
  pair_from_index(pair, in.t, I, J);
  I = __builtin_amdgcn_readfirstlane(I);  // workgroup-uniform: keeps tile addressing scalar
  J = __builtin_amdgcn_readfirstlane(J);
  const bool edge = (I + 1) * ET > in.n || (J + 1) * ET > in.n;
  if (in.mode == RAD_KAPPA_HALF) {
    if (I == J) {
      if (edge) enf_sweep_tile<true, true, true>(in, pair, I, J, first, sB, rowc);
      else enf_sweep_tile<true, false, true>(in, pair, I, J, first, sB, rowc);
    } else {
      if (edge) enf_sweep_tile<false, true, true>(in, pair, I, J, first, sB, rowc);
      else enf_sweep_tile<false, false, true>(in, pair, I, J, first, sB, rowc);
    }
  } else {
    if (I == J) {
      if (edge) enf_sweep_tile<true, true, false>(in, pair, I, J, first, sB, rowc);
      else enf_sweep_tile<true, false, false>(in, pair, I, J, first, sB, rowc);
    } else {
      if (edge) enf_sweep_tile<false, true, false>(in, pair, I, J, first, sB, rowc);
      else enf_sweep_tile<false, false, false>(in, pair, I, J, first, sB, rowc);
    }
  }
}

// Tile pairs in row order (I, I), (I, I + 1), ...: consecutive pairs share
// the own tiles' rows, so each XCD takes a contiguous range of them and the
// cache lines two neighbouring tiles share meet in one L2.
__global__ void __launch_bounds__(ENF_THREADS, 6) enf_sweep(EnfInst in, int first) {
  enf_sweep_body(in, xcd_contiguous(blockIdx.x, gridDim.x), first);
}

// index of the last entry of start[0..count) that is <= v
__device__ __forceinline__ int find_segment(const long* __restrict__ start, int count, long v) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Block map of a batched grid: block b works for instance inst on its local
// block local (one load per block instead of a binary search over the
// instance offsets, whose dependent loads delayed every block's start).
struct EnfBlk {
  int inst, local;
};

// all instances of a batch in one grid: map[b] names the instance and its tile pair
__global__ void __launch_bounds__(ENF_THREADS, 6)
enf_sweep_batched(const EnfInst* __restrict__ ins, const EnfBlk* __restrict__ map, int first) {
  const EnfBlk m = map[blockIdx.x];
  enf_sweep_body(ins[m.inst], m.local, first);
}

// finalize blocks (FIN_ROWS rows each), declared ahead of the decide step
constexpr int FIN_LANES = 8;
constexpr int FIN_ROWS = 256 / FIN_LANES;  // rows per 256-thread block

// Iteration count, closure defect, reciprocity error and the stop flag from
// the finalize blocks' maxima, run by the instance's last finalize block.
__device__ __forceinline__ void enf_decide_body(const EnfInst& in, double tol) {
  EnfCtrl* ctrl = in.ctrl;
  if (ctrl->converged || ctrl->status < 0) return;
  const int nf = (in.n + FIN_ROWS - 1) / FIN_ROWS;
  double d = 0.0, rm = 0.0, em = 0.0;
  for (int b = threadIdx.x; b < nf; b += blockDim.x) {
    d = fmax(d, in.finred[3 * b]);
    rm = fmax(rm, in.finred[3 * b + 1]);
    em = fmax(em, in.finred[3 * b + 2]);
  }
  __shared__ double fr[3][4];
  for (int off = 32; off > 0; off >>= 1) {
    d = fmax(d, __shfl_xor(d, off));
    rm = fmax(rm, __shfl_xor(rm, off));
    em = fmax(em, __shfl_xor(em, off));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    fr[0][w] = d;
    fr[1][w] = rm;
    fr[2][w] = em;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q) {
      d = fmax(d, fr[0][q]);
      rm = fmax(rm, fr[1][q]);
      em = fmax(em, fr[2][q]);
    }
    d = fmax(d, fr[0][0]);
    rm = fmax(rm, fr[1][0]);
    em = fmax(em, fr[2][0]);
    ctrl->iters += 1;
    ctrl->last_defect = d;
    ctrl->last_recip = em > 0.0 ? rm / em : 0.0;
    if (tol > 0.0 && d <= tol) ctrl->converged = 1;
  }
}

// Row sums s_i of the (t + 1) partials of each row: part p = 0..7 of a row
// sums every 8th partial (q = p, p + 8, ...) in order, then the eight parts
// combine as ((0 + 1) + (2 + 3)) + ((4 + 5) + (6 + 7)) (fixed order).  Thread
// t takes part t / 32 of row t % 32, so each load instruction of a wave reads
// two 256-byte runs of consecutive rows of one partial.  Each block's maxima
// go to finred; the block that finishes last (a counter in the control
// block, one atomic per block) reduces them and decides.

__device__ __forceinline__ void enf_finalize_body(const EnfInst& in, int blk, int nblocks, double tol) {
  const int n = in.n, t = in.t;
  const double* __restrict__ partial = in.partial;
  double* __restrict__ scale = in.scale;  // receives 1 / s_i
  const double* __restrict__ blkmax = in.blkmax;
  const long nblk = in.pairs;
  EnfCtrl* ctrl = in.ctrl;
  if (ctrl->converged || ctrl->status < 0) return;
  __shared__ double ps[FIN_LANES][FIN_ROWS];
  const int part = threadIdx.x / FIN_ROWS;
  const int r = threadIdx.x % FIN_ROWS;
  const int i = blk * FIN_ROWS + r;
  double s = 0.0;
  if (i < n) {
    const double* __restrict__ col = partial + i;
    int q = part;
    // eight loads in flight; the sum still runs over q in increasing order
    for (; q + 7 * FIN_LANES <= t; q += 8 * FIN_LANES) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[static_cast<long>(q + u * FIN_LANES) * n];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q <= t; q += FIN_LANES) s += col[static_cast<long>(q) * n];
  }
  ps[part][r] = s;
  __syncthreads();
  double d = 0.0;
  if (part == 0 && i < n) {
    s = ((ps[0][r] + ps[1][r]) + (ps[2][r] + ps[3][r])) + ((ps[4][r] + ps[5][r]) + (ps[6][r] + ps[7][r]));
    if (!(s > 0.0)) raise_status(&ctrl->status, RAD_EZEROROW);
    scale[i] = 1.0 / s;
    d = fabs(s - 1.0);
  }
  double rm = 0.0, em = 0.0;
  const long tid = static_cast<long>(blk) * blockDim.x + threadIdx.x;
  for (long b = tid; b < nblk; b += static_cast<long>(nblocks) * blockDim.x) {
    rm = fmax(rm, blkmax[2 * b]);
    em = fmax(em, blkmax[2 * b + 1]);
  }
  // block maxima to finred (the decide kernel reduces the blocks; no atomics)
  __shared__ double fr[3][4];
  for (int off = 32; off > 0; off >>= 1) {
    d = fmax(d, __shfl_xor(d, off));
    rm = fmax(rm, __shfl_xor(rm, off));
    em = fmax(em, __shfl_xor(em, off));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    fr[0][w] = d;
    fr[1][w] = rm;
    fr[2][w] = em;
  }
  __syncthreads();
  __shared__ int last;
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c) {
      double x = fr[c][0];
      for (int q = 1; q < 4; ++q) x = fmax(x, fr[c][q]);
      in.finred[3 * static_cast<long>(blk) + c] = x;
    }
    __threadfence();  // the maxima are visible before the block counts itself done
    last = atomicAdd(&ctrl->done, 1) == nblocks - 1;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) ctrl->done = 0;
    enf_decide_body(in, tol);
  }
}

inline long fin_blocks(int64_t n) { return ceil_div(n, FIN_ROWS); }

__global__ void __launch_bounds__(256) enf_finalize(EnfInst in, double tol) {
  enf_finalize_body(in, blockIdx.x, gridDim.x, tol);
}

// map[b]: the instance and FIN_ROWS-row block of block b
__global__ void __launch_bounds__(256)
enf_finalize_batched(const EnfInst* __restrict__ ins, const EnfBlk* __restrict__ map, double tol) {
  const EnfBlk m = map[blockIdx.x];
  const EnfInst& in = ins[m.inst];
  enf_finalize_body(in, m.local, (in.n + FIN_ROWS - 1) / FIN_ROWS, tol);
}


__device__ __forceinline__ void enf_apply_scale_body(const EnfInst& in, long row) {
  if (in.ctrl->status < 0 || in.ctrl->iters == 0) return;
  const double s = in.scale[row];  // 1 / row sum
  double* p = in.F + row * in.ldf;
  for (int j = threadIdx.x; j <= in.n; j += blockDim.x) p[j] = p[j] * s;
}

__global__ void __launch_bounds__(256) enf_apply_scale(EnfInst in) { enf_apply_scale_body(in, blockIdx.x); }

// blocks [row_start[k], row_start[k+1]) are the rows of instance k
__global__ void __launch_bounds__(256)
enf_apply_scale_batched(const EnfInst* __restrict__ ins, const long* __restrict__ row_start, int count) {
  const int k = find_segment(row_start, count, blockIdx.x);
  enf_apply_scale_body(ins[k], blockIdx.x - row_start[k]);
}

__device__ __forceinline__ void enf_inv_area_body(const EnfInst& in, int i) {
  if (i >= in.n) return;
  const double a = in.area[i];
  if (!(a > 0.0 && a <= 1.0e300)) raise_status(&in.ctrl->status, RAD_EINVAL);
  const_cast<double*>(in.inv_area)[i] = 1.0 / a;
}

__global__ void __launch_bounds__(256) enf_inv_area(EnfInst in) {
  enf_inv_area_body(in, blockIdx.x * blockDim.x + threadIdx.x);
}

// blocks [blk_start[k], blk_start[k+1]) cover the faces of instance k (256 per block)
__global__ void __launch_bounds__(256)
enf_inv_area_batched(const EnfInst* __restrict__ ins, const long* __restrict__ blk_start, int count) {
  const int k = find_segment(blk_start, count, blockIdx.x);
  enf_inv_area_body(ins[k], static_cast<int>(blockIdx.x - blk_start[k]) * blockDim.x + threadIdx.x);
}

__device__ __forceinline__ void enf_init_body(EnfCtrl* ctrl) {
  {
    ctrl->status = 0;
    ctrl->converged = 0;
    ctrl->iters = 0;
    ctrl->done = 0;
    ctrl->last_defect = ctrl->last_recip = 0.0;
  }
}

__global__ void enf_init(EnfCtrl* ctrl) {
  if (threadIdx.x == 0) enf_init_body(ctrl);
}

__global__ void enf_init_batched(const EnfInst* __restrict__ ins, int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) enf_init_body(ins[k].ctrl);
}

}  // namespace
}  // namespace rad
