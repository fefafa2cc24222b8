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
#include <atomic>
#include <cstdio>
#include <mutex>
#include <string>

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

namespace rad {
namespace {

// Host-side argument checks shared by both entry points.
int32_t enforce_check_args(const char* who, double* F, int64_t n, int64_t ldf, const double* area,
                           const double* n_rays, int32_t kappa_mode, double tol, int32_t max_iter) {
  static thread_local char msg[160];
  auto fail = [&](int32_t code, const char* what) {
    snprintf(msg, sizeof msg, "%s: %s", who, what);
    set_error(msg);
    return code;
  };
  if (!(n >= 1 && n <= (1 << 20))) return fail(RAD_EINVAL, "n out of range");
  if (!(ldf >= n + 1)) return fail(RAD_EINVAL, "ldf < n+1");
  if (!(F && area)) return fail(RAD_EINVAL, "NULL F or area");
  if (!(kappa_mode == RAD_KAPPA_FRACVAR || kappa_mode == RAD_KAPPA_HALF))
    return fail(RAD_EINVAL, "unknown kappa_mode");
  if (!(kappa_mode == RAD_KAPPA_HALF || n_rays)) return fail(RAD_EINVAL, "n_rays required for RAD_KAPPA_FRACVAR");
  if (!(max_iter >= 1)) return fail(RAD_EINVAL, "max_iter < 1");
  if (!(tol >= 0.0 && tol == tol)) return fail(RAD_EINVAL, "tol < 0");
  return RAD_OK;
}

// The iteration itself, on scratch laid out by enf_layout (either the
// caller's workspace or the library's static scratch).
int32_t enforce_run(const char* who, double* F, int64_t n, int64_t ldf, const double* area,
                    const double* n_rays, int32_t kappa_mode, double tol, int32_t max_iter, const EnfLayout& l,
                    rad_stats* stats, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int t = static_cast<int>(ceil_div(n, ET));
  const long pairs = static_cast<long>(t) * (t + 1) / 2;
  RAD_REQUIRE(pairs < (1L << 31), RAD_EINVAL, std::string(who) + ": too many tiles");
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
    set_error(std::string(who) + (h.status == RAD_EZEROROW ? ": a row of F sums to zero"
                                                           : ": F has a negative or non-finite entry"));
    return h.status;
  }
  if (tol > 0.0 && !h.converged) return RAD_WNOTCONVERGED;
  return RAD_OK;
}

// ---- the allocation-free variant ------------------------------------------
// Its scratch is one array in device memory, reserved when the code object is
// loaded and held by each GPU until the process ends; every call on a GPU
// shares that GPU's copy.
constexpr size_t ENF_NOALLOC_BYTES = RAD_ENFORCE_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[ENF_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::atomic<void*> scratch_ptr[MAX_DEVICES];
std::mutex scratch_mutex;

// Device address of the current device's copy of ``scratch``, looked up once
// per device (the array's host-side name is not a device address).
int32_t scratch_for_current_device(void** out) {
  int dev = -1;
  RAD_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("rad_enforce_vf_noalloc: device ordinal beyond the supported range");
    return RAD_EINVAL;
  }
  void* p = scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(scratch_mutex);
    p = scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      RAD_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p) {
        set_error("rad_enforce_vf_noalloc: no device address for the static scratch");
        return RAD_EHIP;
      }
      scratch_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return RAD_OK;
}

}  // namespace
}  // namespace rad

extern "C" int32_t rad_enforce_vf(double* F, int64_t n, int64_t ldf, const double* area,
                                  const double* n_rays, int32_t kappa_mode, double tol,
                                  int32_t max_iter, void* work, size_t work_bytes,
                                  rad_stats* stats, void* stream) {
  ApiRange range("rad_enforce_vf");
  clear_error();
  int32_t rc = enforce_check_args("rad_enforce_vf", F, n, ldf, area, n_rays, kappa_mode, tol, max_iter);
  if (rc != RAD_OK) return rc;
  EnfLayout l = enf_layout(work, work_bytes, n);
  RAD_REQUIRE(l.ok && (reinterpret_cast<uintptr_t>(work) % 256 == 0), RAD_EWORKSPACE,
              "rad_enforce_vf: workspace too small or not 256-byte aligned");
  return enforce_run("rad_enforce_vf", F, n, ldf, area, n_rays, kappa_mode, tol, max_iter, l, stats, stream);
}

extern "C" int32_t rad_enforce_vf_noalloc(double* F, int64_t n, int64_t ldf, const double* area,
                                          const double* n_rays, int32_t kappa_mode, double tol,
                                          int32_t max_iter, rad_stats* stats, void* stream) {
  ApiRange range("rad_enforce_vf_noalloc");
  clear_error();
  int32_t rc = enforce_check_args("rad_enforce_vf_noalloc", F, n, ldf, area, n_rays, kappa_mode, tol, max_iter);
  if (rc != RAD_OK) return rc;
  const size_t need = enf_layout(nullptr, 0, n).bytes;
  if (need > ENF_NOALLOC_BYTES) {
    static thread_local char msg[192];
    snprintf(msg, sizeof msg,
             "rad_enforce_vf_noalloc: n = %lld needs %zu bytes of scratch, more than the built-in %zu "
             "(n <= 16384 fits); use rad_enforce_vf with a workspace",
             static_cast<long long>(n), need, ENF_NOALLOC_BYTES);
    set_error(msg);
    return RAD_EWORKSPACE;
  }
  void* base = nullptr;
  rc = scratch_for_current_device(&base);
  if (rc != RAD_OK) return rc;
  EnfLayout l = enf_layout(base, ENF_NOALLOC_BYTES, n);
  RAD_REQUIRE(l.ok, RAD_EWORKSPACE, "rad_enforce_vf_noalloc: scratch layout failed");
  return enforce_run("rad_enforce_vf_noalloc", F, n, ldf, area, n_rays, kappa_mode, tol, max_iter, l, stats,
                     stream);
}
