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
//   decide   : convergence flag and statistics (device-side, no host sync),
//              by the finalize block that finishes last.
// The last closure scale is applied by a final streaming pass.
#include "enforce_kernels.h"

#include <algorithm>

namespace rad {
namespace {

struct EnfLayout {
  EnfCtrl* ctrl;
  double* scale;
  double* inv_area;
  double* blkmax;
  double* finred;
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
  l.finred = cv.take<double>(static_cast<size_t>(3 * fin_blocks(n)));
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
  EnfInst in;
  in.F = F;
  in.ldf = static_cast<long>(ldf);
  in.n = static_cast<int>(n);
  in.t = t;
  in.pairs = pairs;
  in.area = area;
  in.inv_area = l.inv_area;
  in.nrays = n_rays;
  in.mode = kappa_mode;
  in.scale = l.scale;
  in.partial = l.partial;
  in.blkmax = l.blkmax;
  in.finred = l.finred;
  in.ctrl = l.ctrl;
  hipLaunchKernelGGL(enf_init, dim3(1), dim3(64), 0, s, l.ctrl);
  hipLaunchKernelGGL(enf_inv_area, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, in);
  // tol mode: launch iterations in batches; a converged flag makes the rest
  // of a batch exit at once, so the stop is exact without a sync per step.
  const int batch = tol > 0.0 ? 8 : max_iter;
  int launched = 0;
  while (launched < max_iter) {
    int nb = std::min(batch, max_iter - launched);
    for (int k = 0; k < nb; ++k) {
      int it = launched + k;
      {
        ProfScope prof(s, RAD_PROF_ENFORCE_SWEEP, 0.0, 16.0 * static_cast<double>(n) * (n + 1));
        hipLaunchKernelGGL(enf_sweep, dim3(static_cast<unsigned>(pairs)), dim3(ENF_THREADS), 0, s, in,
                           it == 0 ? 1 : 0);
      }
      hipLaunchKernelGGL(enf_finalize, dim3(static_cast<unsigned>(fin_blocks(n))), dim3(256), 0, s, in, tol);
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
  hipLaunchKernelGGL(enf_apply_scale, dim3(static_cast<unsigned>(n)), dim3(256), 0, s, in);
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
