// Iterative closure + reciprocity enforcer for open systems (thesis
// Sec. 3.5.5) as HBM-streaming sweeps on gfx950.
//
// One iteration = one read and one write of F:
//   sweep    : each workgroup owns a tile pair {(I,J), (J,I)}, I <= J, of the
//              square block (64 x 64 doubles each).  On load it applies the
//              closure scale of the previous iteration (F_ij / s_i, eq. 3.39-
//              3.40 with omega = eta), then the reciprocity step (eq. 3.18-
//              3.20, kappa from eq. 3.25 or 1/2) using an LDS transpose so
//              both tiles are read and written with coalesced rows; it emits
//              per-(row, column-tile) partial row sums of the new values.
//              Diagonal-tile workgroups also carry the space column.
//   finalize : s_i = sum of the partials in fixed tile order (reproducible),
//              closure defect max |s_i - 1|.
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

__global__ void __launch_bounds__(ENF_THREADS)
enf_sweep(double* __restrict__ F, long ldf, int n, int t,
          const double* __restrict__ area, const double* __restrict__ nrays,
          int mode, const double* __restrict__ scale, double* __restrict__ partial,
          EnfCtrl* ctrl, int parity, int first) {
  if (ctrl->converged || ctrl->status < 0) return;
  __shared__ double sA[ET][ETP];
  __shared__ double sB[ET][ETP];
  __shared__ double red[3][ENF_THREADS / 64];
  int I, J;
  pair_from_index(blockIdx.x, t, I, J);
  const int r0 = I * ET, c0 = J * ET;
  const int tid = threadIdx.x;
  const int c = tid & (ET - 1);
  const int rg = tid >> 6;   // 0..3
  const bool diag = (I == J);
  int bad = 0;

  // load tile A = F[r0.., c0..] and B = F[c0.., r0..] (scaled) into LDS
  for (int m = 0; m < ET / 4; ++m) {
    int r = rg + 4 * m;
    int i = r0 + r, j = c0 + c;
    double v = 0.0;
    if (i < n && j < n) {
      v = F[static_cast<long>(i) * ldf + j];
      bad |= !(v >= 0.0) || !(v <= 1.0e300);
      if (!first) v = v / scale[i];
    }
    sA[r][c] = v;
    if (!diag) {
      int i2 = c0 + r, j2 = r0 + c;
      double w = 0.0;
      if (i2 < n && j2 < n) {
        w = F[static_cast<long>(i2) * ldf + j2];
        bad |= !(w >= 0.0) || !(w <= 1.0e300);
        if (!first) w = w / scale[i2];
      }
      sB[r][c] = w;
    }
  }
  __syncthreads();

  // reciprocity on the pair; each unordered pair {i,j}, i != j, once
  double rmax = 0.0, emax = 0.0;
  for (int m = 0; m < ET / 4; ++m) {
    int r = rg + 4 * m;
    int i = r0 + r, j = c0 + c;
    if (i >= n || j >= n) continue;
    if (diag) {
      if (c <= r) continue;  // handled by the (c, r) thread; diagonal unchanged
      double fij = sA[r][c], fji = sA[c][r];
      double ai = area[i], aj = area[j];
      double eij = ai * fij, eji = aj * fji;
      rmax = fmax(rmax, fabs(eij - eji));
      emax = fmax(emax, fmax(eij, eji));
      double ni = nrays ? nrays[i] : 1.0, nj = nrays ? nrays[j] : 1.0;
      double k = kappa_of(fij, fji, ai, aj, ni, nj, mode);
      double eh = k * eij + (1.0 - k) * eji;
      sA[r][c] = eh / ai;
      sA[c][r] = eh / aj;
    } else {
      double fij = sA[r][c], fji = sB[c][r];
      double ai = area[i], aj = area[j];
      double eij = ai * fij, eji = aj * fji;
      rmax = fmax(rmax, fabs(eij - eji));
      emax = fmax(emax, fmax(eij, eji));
      double ni = nrays ? nrays[i] : 1.0, nj = nrays ? nrays[j] : 1.0;
      double k = kappa_of(fij, fji, ai, aj, ni, nj, mode);
      double eh = k * eij + (1.0 - k) * eji;
      sA[r][c] = eh / ai;
      sB[c][r] = eh / aj;
    }
  }
  if (diag) {
    // diagonal entries keep their (scaled) value; include them in eta max
    if (tid < ET && r0 + tid < n) emax = fmax(emax, area[r0 + tid] * sA[tid][tid]);
  }
  __syncthreads();

  // write both tiles back (coalesced rows)
  for (int m = 0; m < ET / 4; ++m) {
    int r = rg + 4 * m;
    int i = r0 + r, j = c0 + c;
    if (i < n && j < n) F[static_cast<long>(i) * ldf + j] = sA[r][c];
    if (!diag) {
      int i2 = c0 + r, j2 = r0 + c;
      if (i2 < n && j2 < n) F[static_cast<long>(i2) * ldf + j2] = sB[r][c];
    }
  }
  // partial row sums in a fixed order: thread r < 64 sums row r of sA,
  // threads 64..127 sum the rows of sB; diagonal tiles add the space column.
  if (tid < ET) {
    int i = r0 + tid;
    if (i < n) {
      double s = 0.0;
      for (int q = 0; q < ET; ++q) s += sA[tid][q];
      if (diag) {
        double* sp = F + static_cast<long>(i) * ldf + n;
        double v = *sp;
        bad |= !(v >= 0.0) || !(v <= 1.0e300);
        if (!first) v = v / scale[i];
        *sp = v;
        partial[static_cast<long>(t) * n + i] = v;
      }
      partial[static_cast<long>(J) * n + i] = s;
    }
  } else if (tid < 2 * ET && !diag) {
    int rr = tid - ET;
    int i = c0 + rr;
    if (i < n) {
      double s = 0.0;
      for (int q = 0; q < ET; ++q) s += sB[rr][q];
      partial[static_cast<long>(I) * n + i] = s;
    }
  }
  if (bad) raise_status(&ctrl->status, RAD_ENONFINITE);
  // block max of the reciprocity error and of eta
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
    double a = red[0][0], b = red[1][0];
    for (int w = 1; w < ENF_THREADS / 64; ++w) {
      a = fmax(a, red[0][w]);
      b = fmax(b, red[1][w]);
    }
    atomic_max_nonneg(&ctrl->recip[parity], a);
    atomic_max_nonneg(&ctrl->etamax[parity], b);
  }
}

__global__ void __launch_bounds__(256)
enf_finalize(int n, int t, const double* __restrict__ partial, double* __restrict__ scale,
             EnfCtrl* ctrl, int parity) {
  if (ctrl->converged || ctrl->status < 0) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int q = 0; q <= t; ++q) s += partial[static_cast<long>(q) * n + i];
    if (!(s > 0.0)) raise_status(&ctrl->status, RAD_EZEROROW);
    scale[i] = s;
    d = fabs(s - 1.0);
  }
  for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(&ctrl->defect[parity], d);
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
  const double s = scale[row];
  double* p = F + row * ldf;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) p[j] = p[j] / s;
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
                           F, static_cast<long>(ldf), static_cast<int>(n), t, area, n_rays,
                           kappa_mode, l.scale, l.partial, l.ctrl, parity, it == 0 ? 1 : 0);
      }
      hipLaunchKernelGGL(enf_finalize, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s,
                         static_cast<int>(n), t, l.partial, l.scale, l.ctrl, parity);
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
