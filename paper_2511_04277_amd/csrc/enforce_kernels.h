// Enforcement kernels (thesis Sec. 3.5.5) shared by the single-instance and
// batched entry points.  See enforce.hip for the algorithm.
#pragma once

#include "common.h"

namespace rad {
namespace {

constexpr int ET = 64;          // tile edge (doubles)
constexpr int ETP = ET + 1;     // padded LDS row (conflict-free transpose)
constexpr int ENF_THREADS = 256;

struct EnfCtrl {
  int status;        // device-raised status (0 ok, negative error)
  int converged;     // 1 once the tolerance is met
  int iters;         // iterations executed
  int pad;
  double defect[2];  // closure defect per iteration parity (atomic max)
  double recip[2];   // max |eta_ij - eta_ji| per parity (atomic max)
  double etamax[2];  // max eta per parity (atomic max)
  double last_defect, last_recip;
};

__device__ inline double kappa_of(double fij, double fji, double ai, double aj,
                                  double ni, double nj, int mode) {
  if (mode == RAD_KAPPA_HALF) return 0.5;
  // eq. 3.25 with s2_ij = A_i^2 (1-F_ij)/(N_i F_ij); numerator and
  // denominator multiplied by F_ij F_ji so that zeros need no infinities.
  double a = ai * ai * (1.0 - fij) * fji / ni;
  double b = aj * aj * (1.0 - fji) * fij / nj;
  double s = a + b;
  return s > 0.0 ? b / s : 0.5;
}

__device__ inline void pair_from_index(long p, int t, int& I, int& J) {
  // row-wise enumeration of the upper triangle (I <= J) of a t x t tile grid
  double tt = 2.0 * t + 1.0;
  int i = static_cast<int>((tt - sqrt(tt * tt - 8.0 * static_cast<double>(p))) * 0.5);
  if (i < 0) i = 0;
  if (i > t - 1) i = t - 1;
  auto start = [t](long r) { return r * t - r * (r - 1) / 2; };
  while (i > 0 && start(i) > p) --i;
  while (i + 1 < t && start(i + 1) <= p) ++i;
  I = i;
  J = static_cast<int>(i + (p - start(i)));
}

// Thread t owns row r = t / 4 of the 64 x 64 tile (I, J) and its 16
// consecutive columns cq*16 .. cq*16+15 (cq = t % 4) in registers; the partner
// tile (J, I) sits in LDS.  Both tiles are read and written as 128-byte runs.
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
  EnfCtrl* ctrl;
};

__device__ __forceinline__ void enf_sweep_body(const EnfInst& in, long pair, int first) {
  double* __restrict__ F = in.F;
  const long ldf = in.ldf;
  const int n = in.n, t = in.t;
  const double* __restrict__ area = in.area;
  const double* __restrict__ inv_area = in.inv_area;
  const double* __restrict__ nrays = in.nrays;
  const int mode = in.mode;
  const double* __restrict__ inv_scale = in.scale;
  double* __restrict__ partial = in.partial;
  double* __restrict__ blkmax = in.blkmax;
  EnfCtrl* ctrl = in.ctrl;
  if (ctrl->converged || ctrl->status < 0) return;
  __shared__ double sB[ET][ETP];
  __shared__ double red[2][ENF_THREADS / 64];
  int I, J;
  pair_from_index(pair, t, I, J);
  const int r0 = I * ET, c0 = J * ET;
  const int tid = threadIdx.x;
  const int r = tid >> 2, cq = tid & 3, cb = cq * 16;
  const bool diag = (I == J);
  const int i = r0 + r;          // this thread's row of tile (I, J)
  const int ip = c0 + r;         // this thread's row of the partner tile (J, I)
  int bad = 0;

  // Interior tiles (the vast majority) load and store unconditionally; edge
  // tiles clamp their addresses and zero the entries beyond n, which the pair
  // arithmetic below leaves at zero.
  const bool interior = (r0 + ET <= n) && (c0 + ET <= n);
  double a[16];
  {
    const int ic = i < n ? i : n - 1;
    const double si = first ? 1.0 : inv_scale[ic];
    const double* src = F + static_cast<long>(ic) * ldf;
    if (interior) {
#pragma unroll
      for (int e = 0; e < 16; ++e) a[e] = src[c0 + cb + e];
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int j = c0 + cb + e;
        const double v = src[j < n ? j : n - 1];
        a[e] = (i < n && j < n) ? v : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      bad |= !(a[e] >= 0.0) || !(a[e] <= 1.0e300);
      a[e] *= si;
    }
  }
  if (!diag) {
    const int ipc = ip < n ? ip : n - 1;
    const double sj = first ? 1.0 : inv_scale[ipc];
    const double* src = F + static_cast<long>(ipc) * ldf;
    double v[16];
    if (interior) {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = src[r0 + cb + e];
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int j = r0 + cb + e;
        const double x = src[j < n ? j : n - 1];
        v[e] = (ip < n && j < n) ? x : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      bad |= !(v[e] >= 0.0) || !(v[e] <= 1.0e300);
      sB[r][cb + e] = v[e] * sj;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) sB[r][cb + e] = a[e];
  }
  __syncthreads();

  // reciprocity on each unordered pair {i, j}, i != j, exactly once
  double rmax = 0.0, emax = 0.0;
  const int ic = i < n ? i : n - 1;
  const double ai = area[ic];
  const double iai = inv_area[ic];
  const double ni = nrays ? nrays[ic] : 1.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int c = cb + e;
    const int j = c0 + c;
    const int jc = j < n ? j : n - 1;
    if (diag) {
      if (c == r) emax = fmax(emax, ai * a[e]);  // diagonal keeps its value
      if (c <= r) continue;                       // handled by the owner of (c, r)
    }
    const double fij = a[e], fji = sB[c][r];
    const double aj = area[jc];
    const double eij = ai * fij, eji = aj * fji;
    rmax = fmax(rmax, fabs(eij - eji));
    emax = fmax(emax, fmax(eij, eji));
    const double nj = nrays ? nrays[jc] : 1.0;
    const double k = kappa_of(fij, fji, ai, aj, ni, nj, mode);
    const double eh = k * eij + (1.0 - k) * eji;
    a[e] = eh * iai;
    sB[c][r] = eh * inv_area[jc];
  }
  __syncthreads();
  if (diag) {
#pragma unroll
    for (int e = 0; e < 16; ++e)
      if (cb + e < r) a[e] = sB[r][cb + e];  // lower-triangle values written by their pair owner
  }

  // write back and form the partial row sums (4-lane reductions, fixed order)
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) sa += a[e];
  if (interior) {
    double* dst = F + static_cast<long>(i) * ldf + c0 + cb;
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[e] = a[e];
  } else if (i < n) {
    double* dst = F + static_cast<long>(i) * ldf + c0 + cb;
#pragma unroll
    for (int e = 0; e < 16; ++e)
      if (c0 + cb + e < n) dst[e] = a[e];
  }
  if (!diag) {
    double v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      v[e] = sB[r][cb + e];
      sb += v[e];
    }
    double* dst = F + static_cast<long>(ip) * ldf + r0 + cb;
    if (interior) {
#pragma unroll
      for (int e = 0; e < 16; ++e) dst[e] = v[e];
    } else if (ip < n) {
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (r0 + cb + e < n) dst[e] = v[e];
    }
  }
  sa += __shfl_xor(sa, 1);
  sa += __shfl_xor(sa, 2);
  sb += __shfl_xor(sb, 1);
  sb += __shfl_xor(sb, 2);
  if (cq == 0) {
    if (i < n) {
      partial[static_cast<long>(J) * n + i] = sa;
      if (diag) {  // the space column of row i rides with the diagonal tile
        double* sp = F + static_cast<long>(i) * ldf + n;
        double v = *sp;
        bad |= !(v >= 0.0) || !(v <= 1.0e300);
        if (!first) v *= inv_scale[i];
        *sp = v;
        partial[static_cast<long>(t) * n + i] = v;
      }
    }
    if (!diag && ip < n) partial[static_cast<long>(I) * n + ip] = sb;
  }
  if (bad) raise_status(&ctrl->status, RAD_ENONFINITE);
  for (int off = 32; off > 0; off >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, off));
    emax = fmax(emax, __shfl_xor(emax, off));
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = rmax;
    red[1][tid >> 6] = emax;
  }
  __syncthreads();
  if (tid == 0) {
    double x = red[0][0], y = red[1][0];
    for (int w = 1; w < ENF_THREADS / 64; ++w) {
      x = fmax(x, red[0][w]);
      y = fmax(y, red[1][w]);
    }
    blkmax[2 * pair] = x;
    blkmax[2 * pair + 1] = y;
  }
}

__global__ void __launch_bounds__(ENF_THREADS) enf_sweep(EnfInst in, int first) {
  enf_sweep_body(in, blockIdx.x, first);
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

// all instances of a batch in one grid: blocks [pair_start[k], pair_start[k+1]) are instance k
__global__ void __launch_bounds__(ENF_THREADS)
enf_sweep_batched(const EnfInst* __restrict__ ins, const long* __restrict__ pair_start, int count, int first) {
  const int k = find_segment(pair_start, count, blockIdx.x);
  enf_sweep_body(ins[k], blockIdx.x - pair_start[k], first);
}

__device__ __forceinline__ void enf_finalize_body(const EnfInst& in, int blk, int nblocks, int parity) {
  const int n = in.n, t = in.t;
  const double* __restrict__ partial = in.partial;
  double* __restrict__ scale = in.scale;  // receives 1 / s_i
  const double* __restrict__ blkmax = in.blkmax;
  const long nblk = in.pairs;
  EnfCtrl* ctrl = in.ctrl;
  if (ctrl->converged || ctrl->status < 0) return;
  const int i = blk * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int q = 0; q <= t; ++q) s += partial[static_cast<long>(q) * n + i];
    if (!(s > 0.0)) raise_status(&ctrl->status, RAD_EZEROROW);
    scale[i] = 1.0 / s;
    d = fabs(s - 1.0);
  }
  double rm = 0.0, em = 0.0;
  for (long b = i; b < nblk; b += static_cast<long>(nblocks) * blockDim.x) {
    rm = fmax(rm, blkmax[2 * b]);
    em = fmax(em, blkmax[2 * b + 1]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    d = fmax(d, __shfl_xor(d, off));
    rm = fmax(rm, __shfl_xor(rm, off));
    em = fmax(em, __shfl_xor(em, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(&ctrl->defect[parity], d);
    atomic_max_nonneg(&ctrl->recip[parity], rm);
    atomic_max_nonneg(&ctrl->etamax[parity], em);
  }
}

__global__ void __launch_bounds__(256) enf_finalize(EnfInst in, int parity) {
  enf_finalize_body(in, blockIdx.x, gridDim.x, parity);
}

// blocks [blk_start[k], blk_start[k+1]) are the row blocks of instance k
__global__ void __launch_bounds__(256)
enf_finalize_batched(const EnfInst* __restrict__ ins, const long* __restrict__ blk_start, int count, int parity) {
  const int k = find_segment(blk_start, count, blockIdx.x);
  const int nb = static_cast<int>(blk_start[k + 1] - blk_start[k]);
  enf_finalize_body(ins[k], static_cast<int>(blockIdx.x - blk_start[k]), nb, parity);
}

__device__ __forceinline__ void enf_decide_body(EnfCtrl* ctrl, int parity, double tol) {
  if (ctrl->converged || ctrl->status < 0) return;
  ctrl->iters += 1;
  double d = ctrl->defect[parity];
  double e = ctrl->etamax[parity];
  ctrl->last_defect = d;
  ctrl->last_recip = e > 0.0 ? ctrl->recip[parity] / e : 0.0;
  if (tol > 0.0 && d <= tol) ctrl->converged = 1;
  // clear the other parity for the next iteration
  int o = parity ^ 1;
  ctrl->defect[o] = 0.0;
  ctrl->recip[o] = 0.0;
  ctrl->etamax[o] = 0.0;
}

__global__ void enf_decide(EnfCtrl* ctrl, int parity, double tol) {
  if (threadIdx.x == 0) enf_decide_body(ctrl, parity, tol);
}

__global__ void enf_decide_batched(const EnfInst* __restrict__ ins, int count, int parity, double tol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) enf_decide_body(ins[k].ctrl, parity, tol);
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
    ctrl->pad = 0;
    for (int q = 0; q < 2; ++q) ctrl->defect[q] = ctrl->recip[q] = ctrl->etamax[q] = 0.0;
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
