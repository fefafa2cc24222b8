// Iterative closure + reciprocity enforcer for open systems (thesis
// Sec. 3.5.5) as HBM-streaming sweeps on gfx950.
//
// One iteration = one read and one write of F:
//   sweep    : each workgroup owns a tile pair {(I,J), (J,I)}, I <= J, of the
//              square block (64 x 64 doubles each).  On load it applies the
//              closure scale of the previous iteration (F_ij / s_i, eq. 3.39-
//              3.40 with omega = eta, as a product with 1/s_i), then the
//              reciprocity step (eq. 3.18-3.20, kappa from eq. 3.25 or 1/2),
//              reading the partner tile through LDS so both tiles are read and
//              written as coalesced rows; it emits per-(row, column-tile)
//              partial row sums of the new values.  Diagonal-tile workgroups
//              also carry the space column.
//   finalize : s_i = sum of the partials in fixed tile order (reproducible),
//              stores 1/s_i, closure defect max |s_i - 1|.
//   decide   : convergence flag and statistics (device-side, no host sync).
// The last closure scale is applied by a final streaming pass.
#include "common.h"

#include <algorithm>

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
__global__ void __launch_bounds__(ENF_THREADS)
enf_sweep(double* __restrict__ F, long ldf, int n, int t,
          const double* __restrict__ area, const double* __restrict__ inv_area,
          const double* __restrict__ nrays, int mode, const double* __restrict__ inv_scale,
          double* __restrict__ partial, double* __restrict__ blkmax, EnfCtrl* ctrl, int first) {
  if (ctrl->converged || ctrl->status < 0) return;
  __shared__ double sB[ET][ETP];
  __shared__ double red[2][ENF_THREADS / 64];
  int I, J;
  pair_from_index(blockIdx.x, t, I, J);
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
    blkmax[2 * static_cast<long>(blockIdx.x)] = x;
    blkmax[2 * static_cast<long>(blockIdx.x) + 1] = y;
  }
}

__global__ void __launch_bounds__(256)
enf_finalize(int n, int t, const double* __restrict__ partial, double* __restrict__ scale /* 1/s */,
             const double* __restrict__ blkmax, long nblk, EnfCtrl* ctrl, int parity) {
  if (ctrl->converged || ctrl->status < 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int q = 0; q <= t; ++q) s += partial[static_cast<long>(q) * n + i];
    if (!(s > 0.0)) raise_status(&ctrl->status, RAD_EZEROROW);
    scale[i] = 1.0 / s;
    d = fabs(s - 1.0);
  }
  double rm = 0.0, em = 0.0;
  for (long b = i; b < nblk; b += static_cast<long>(gridDim.x) * blockDim.x) {
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

__global__ void enf_decide(EnfCtrl* ctrl, int parity, double tol) {
  if (threadIdx.x != 0 || ctrl->converged || ctrl->status < 0) return;
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

__global__ void __launch_bounds__(256)
enf_apply_scale(double* __restrict__ F, long ldf, int n, const double* __restrict__ scale,
                const EnfCtrl* ctrl) {
  if (ctrl->status < 0 || ctrl->iters == 0) return;
  const long row = blockIdx.x;
  const double s = scale[row];  // 1 / row sum
  double* p = F + row * ldf;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) p[j] = p[j] * s;
}

__global__ void __launch_bounds__(256)
enf_inv_area(const double* __restrict__ area, int n, double* __restrict__ inv_area, EnfCtrl* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = area[i];
  if (!(a > 0.0 && a <= 1.0e300)) raise_status(&ctrl->status, RAD_EINVAL);
  inv_area[i] = 1.0 / a;
}

__global__ void enf_init(EnfCtrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->status = 0;
    ctrl->converged = 0;
    ctrl->iters = 0;
    ctrl->pad = 0;
    for (int q = 0; q < 2; ++q) ctrl->defect[q] = ctrl->recip[q] = ctrl->etamax[q] = 0.0;
    ctrl->last_defect = ctrl->last_recip = 0.0;
  }
}

struct EnfLayout {
  EnfCtrl* ctrl;
  double* scale;
  double* inv_area;
  double* blkmax;
  double* partial;
  size_t bytes;
  bool ok;
};

EnfLayout enf_layout(void* work, size_t work_bytes, int64_t n) {
  Carve cv(work, work_bytes);
  int64_t t = ceil_div(n, ET);
  EnfLayout l;
  l.ctrl = cv.take<EnfCtrl>(1);
  l.scale = cv.take<double>(static_cast<size_t>(n));
  l.inv_area = cv.take<double>(static_cast<size_t>(n));
  l.blkmax = cv.take<double>(static_cast<size_t>(t * (t + 1)));
  l.partial = cv.take<double>(static_cast<size_t>((t + 1) * n));
  l.bytes = cv.used;
  l.ok = cv.ok;
  return l;
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" size_t rad_enforce_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return enf_layout(nullptr, 0, n).bytes;
}

extern "C" int32_t rad_enforce_vf(double* F, int64_t n, int64_t ldf, const double* area,
                                  const double* n_rays, int32_t kappa_mode, double tol,
                                  int32_t max_iter, void* work, size_t work_bytes,
                                  rad_stats* stats, void* stream) {
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_enforce_vf: n out of range");
  RAD_REQUIRE(ldf >= n + 1, RAD_EINVAL, "rad_enforce_vf: ldf < n+1");
  RAD_REQUIRE(F && area, RAD_EINVAL, "rad_enforce_vf: NULL F or area");
  RAD_REQUIRE(kappa_mode == RAD_KAPPA_FRACVAR || kappa_mode == RAD_KAPPA_HALF, RAD_EINVAL,
              "rad_enforce_vf: unknown kappa_mode");
  RAD_REQUIRE(kappa_mode == RAD_KAPPA_HALF || n_rays, RAD_EINVAL,
              "rad_enforce_vf: n_rays required for RAD_KAPPA_FRACVAR");
  RAD_REQUIRE(max_iter >= 1, RAD_EINVAL, "rad_enforce_vf: max_iter < 1");
  RAD_REQUIRE(tol >= 0.0 && tol == tol, RAD_EINVAL, "rad_enforce_vf: tol < 0");
  EnfLayout l = enf_layout(work, work_bytes, n);
  RAD_REQUIRE(l.ok && (reinterpret_cast<uintptr_t>(work) % 256 == 0), RAD_EWORKSPACE,
              "rad_enforce_vf: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int t = static_cast<int>(ceil_div(n, ET));
  const long pairs = static_cast<long>(t) * (t + 1) / 2;
  RAD_REQUIRE(pairs < (1L << 31), RAD_EINVAL, "rad_enforce_vf: too many tiles");
  hipLaunchKernelGGL(enf_init, dim3(1), dim3(64), 0, s, l.ctrl);
  hipLaunchKernelGGL(enf_inv_area, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, area,
                     static_cast<int>(n), l.inv_area, l.ctrl);
  // tol mode: launch iterations in batches; a converged flag makes the rest
  // of a batch exit at once, so the stop is exact without a sync per step.
  const int batch = tol > 0.0 ? 8 : max_iter;
  int launched = 0;
  while (launched < max_iter) {
    int nb = std::min(batch, max_iter - launched);
    for (int k = 0; k < nb; ++k) {
      int it = launched + k;
      int parity = it & 1;
      {
        ProfScope prof(s, RAD_PROF_ENFORCE_SWEEP, 0.0, 16.0 * static_cast<double>(n) * (n + 1));
        hipLaunchKernelGGL(enf_sweep, dim3(static_cast<unsigned>(pairs)), dim3(ENF_THREADS), 0, s,
                           F, static_cast<long>(ldf), static_cast<int>(n), t, area, l.inv_area, n_rays,
                           kappa_mode, l.scale, l.partial, l.blkmax, l.ctrl, it == 0 ? 1 : 0);
      }
      hipLaunchKernelGGL(enf_finalize, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s,
                         static_cast<int>(n), t, l.partial, l.scale, l.blkmax, pairs, l.ctrl, parity);
      hipLaunchKernelGGL(enf_decide, dim3(1), dim3(64), 0, s, l.ctrl, parity, tol);
    }
    RAD_HIP_CHECK(hipGetLastError());
    launched += nb;
    if (tol > 0.0 && launched < max_iter) {
      int conv = 0, st = 0;
      RAD_HIP_CHECK(hipMemcpyAsync(&conv, &l.ctrl->converged, sizeof(int), hipMemcpyDeviceToHost, s));
      RAD_HIP_CHECK(hipMemcpyAsync(&st, &l.ctrl->status, sizeof(int), hipMemcpyDeviceToHost, s));
      RAD_HIP_CHECK(hipStreamSynchronize(s));
      if (conv || st < 0) break;
    }
  }
  hipLaunchKernelGGL(enf_apply_scale, dim3(static_cast<unsigned>(n)), dim3(256), 0, s, F,
                     static_cast<long>(ldf), static_cast<int>(n), l.scale, l.ctrl);
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats) return RAD_OK;
  EnfCtrl h;
  RAD_HIP_CHECK(hipMemcpyAsync(&h, l.ctrl, sizeof(EnfCtrl), hipMemcpyDeviceToHost, s));
  RAD_HIP_CHECK(hipStreamSynchronize(s));
  *stats = rad_stats{};
  stats->iters = h.iters;
  stats->converged = h.converged;
  stats->device_status = h.status;
  stats->closure_defect = h.last_defect;
  stats->recip_err = h.last_recip;
  if (h.status < 0) {
    set_error(h.status == RAD_EZEROROW ? "rad_enforce_vf: a row of F sums to zero"
                                       : "rad_enforce_vf: F has a negative or non-finite entry");
    return h.status;
  }
  if (tol > 0.0 && !h.converged) return RAD_WNOTCONVERGED;
  return RAD_OK;
}
