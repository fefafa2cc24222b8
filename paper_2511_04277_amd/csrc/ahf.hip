// Absorbed heat fluxes from REFs and direct heat fluxes (thesis Sec. 4.2.3,
// eq. 4.6), for m load cases at once:
//
//   Qa[i][c] = A_i eps_i Qd[i][c] + sum_j B_ji A_j rho_j Qd[j][c]
//
// The sum is a transposed product with the N x N block of B, which is read
// once (HBM-bound).  ahf_weights forms w_jc = A_j rho_j Qd[j][c] (zero-padded
// to MC cases).  ahf_partial: one wave per (64 CI consecutive faces, chunk of
// rows j); a lane owns CI faces i, 64 apart, and sums B_ji w_jc over the
// chunk's rows.  w_jc is the same for every lane, so it comes through scalar
// loads (no LDS, no barriers) and feeds the FMAs as a scalar operand; each row
// of B is CI 512-byte vector loads per wave, U rows in flight.  ahf_final adds
// the direct term and the chunk sums in chunk order (fixed order: bitwise
// reproducible).
#include <algorithm>

#include "common.h"

namespace rad {
namespace {

constexpr int AHF_THREADS = 256;
constexpr int AHF_WAVE = 64;
constexpr int AHF_MAX_CHUNKS = 64;
constexpr int AHF_TARGET_WAVES = 2048;  // 8 per CU

// Per padded case count MC: U rows of B in flight per lane and CI faces per
// lane (measured at N = 8192: MC <= 8 streams B at 6.0-6.3 TB/s with two
// faces per lane; MC = 16 is bound by the scalar weight loads and prefers
// four faces per lane, so each weight feeds four FMAs).  B is streamed once,
// so its loads are nontemporal.
template <int MC>
struct AhfShape {
  static constexpr int U = MC >= 16 ? 2 : MC >= 8 ? 4 : 8;
  static constexpr int CI = MC >= 16 ? 4 : 2;
};

template <int MC>
__global__ void __launch_bounds__(AHF_THREADS)
ahf_weights(int n, const double* __restrict__ rho, const double* __restrict__ area, const double* __restrict__ qd,
            long ldq, int m, double* __restrict__ w) {
  const long t = static_cast<long>(blockIdx.x) * AHF_THREADS + threadIdx.x;
  if (t >= static_cast<long>(n) * MC) return;
  const int j = static_cast<int>(t / MC), c = static_cast<int>(t % MC);
  w[t] = c < m ? area[j] * rho[j] * qd[static_cast<long>(j) * ldq + c] : 0.0;
}

template <int MC, int U = AhfShape<MC>::U, int CI = AhfShape<MC>::CI, bool NT = true>
__global__ void __launch_bounds__(AHF_WAVE)
ahf_partial(const double* __restrict__ B, long ldb, int n, const double* __restrict__ w, int rows,
            double* __restrict__ part) {
  // lane owns faces i0 + 64 q, q < CI (lanes past the last face load a valid
  // column and store nothing)
  const int i0 = blockIdx.x * AHF_WAVE * CI + threadIdx.x;
  const int j0 = blockIdx.y * rows, j1 = min(n, j0 + rows);
  double acc[CI][MC];
  const double* bcol[CI];
#pragma unroll
  for (int q = 0; q < CI; ++q) {
    bcol[q] = B + min(i0 + AHF_WAVE * q, n - 1);
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[q][c] = 0.0;
  }
  auto load = [&](int q, int j) {
    const double* p = bcol[q] + static_cast<long>(j) * ldb;
    return NT ? __builtin_nontemporal_load(p) : *p;
  };
  int j = j0;
  for (; j + U <= j1; j += U) {
    double b[U][CI];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < CI; ++q) b[u][q] = load(q, j + u);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* wj = w + static_cast<long>(j + u) * MC;
#pragma unroll
      for (int c = 0; c < MC; ++c) {
        const double wc = wj[c];
#pragma unroll
        for (int q = 0; q < CI; ++q) acc[q][c] = fma(b[u][q], wc, acc[q][c]);
      }
    }
  }
  for (; j < j1; ++j) {
    double b[CI];
#pragma unroll
    for (int q = 0; q < CI; ++q) b[q] = load(q, j);
    const double* wj = w + static_cast<long>(j) * MC;
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      const double wc = wj[c];
#pragma unroll
      for (int q = 0; q < CI; ++q) acc[q][c] = fma(b[q], wc, acc[q][c]);
    }
  }
#pragma unroll
  for (int q = 0; q < CI; ++q) {
    const int i = i0 + AHF_WAVE * q;
    if (i >= n) break;
    double* p = part + (static_cast<long>(blockIdx.y) * n + i) * MC;
#pragma unroll
    for (int c = 0; c < MC; ++c) p[c] = acc[q][c];
  }
}

template <int MC>
__global__ void __launch_bounds__(AHF_THREADS)
ahf_final(const double* __restrict__ part, int chunks, int n, const double* __restrict__ eps,
          const double* __restrict__ area, const double* __restrict__ qd, long ldq, int m,
          double* __restrict__ qa, long lda) {
  const long t = static_cast<long>(blockIdx.x) * AHF_THREADS + threadIdx.x;
  if (t >= static_cast<long>(n) * m) return;
  const int i = static_cast<int>(t / m), c = static_cast<int>(t % m);
  double s = area[i] * eps[i] * qd[static_cast<long>(i) * ldq + c];
  const double* p = part + static_cast<long>(i) * MC + c;
  const long stride = static_cast<long>(n) * MC;
  int k = 0;
  for (; k + 8 <= chunks; k += 8) {  // eight loads in flight, added in chunk order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(k + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; k < chunks; ++k) s += p[k * stride];
  qa[static_cast<long>(i) * lda + c] = s;
}

int cases_pad(int64_t m) { return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : 16; }

int ahf_chunks(int64_t n, int mc) {
  const int64_t col_waves = ceil_div(n, AHF_WAVE * (mc >= 16 ? AhfShape<16>::CI : AhfShape<1>::CI));
  const int64_t by_waves = std::max<int64_t>(1, AHF_TARGET_WAVES / col_waves);
  const int64_t by_rows = std::max<int64_t>(1, n / AHF_WAVE);  // at least 64 rows per chunk
  return static_cast<int>(std::min<int64_t>({AHF_MAX_CHUNKS, by_waves, by_rows}));
}

// workspace: w (n x MC) then the chunk sums (chunks x n x MC), both 256-byte aligned
size_t ahf_w_bytes(int64_t n, int mc) { return static_cast<size_t>(ceil_div(n * mc * 8, 256) * 256); }

template <int MC>
void ahf_launch(const double* B, long ldb, int n, const double* eps, const double* rho, const double* area,
                const double* qd, long ldq, int m, double* qa, long lda, char* work, hipStream_t s) {
  const int chunks = ahf_chunks(n, MC);
  const int rows = static_cast<int>(ceil_div(n, chunks));
  double* w = reinterpret_cast<double*>(work);
  double* part = reinterpret_cast<double*>(work + ahf_w_bytes(n, MC));
  hipLaunchKernelGGL((ahf_weights<MC>), dim3(static_cast<unsigned>(ceil_div(static_cast<int64_t>(n) * MC, AHF_THREADS))),
                     dim3(AHF_THREADS), 0, s, n, rho, area, qd, ldq, m, w);
  {
    ProfScope prof(s, RAD_PROF_AHF, 2.0 * static_cast<double>(n) * n * m, 8.0 * static_cast<double>(n) * n);
    hipLaunchKernelGGL((ahf_partial<MC>), dim3(static_cast<unsigned>(ceil_div(n, AHF_WAVE * AhfShape<MC>::CI)), chunks),
                       dim3(AHF_WAVE), 0, s, B, ldb, n, w, rows, part);
  }
  hipLaunchKernelGGL((ahf_final<MC>), dim3(static_cast<unsigned>(ceil_div(static_cast<int64_t>(n) * m, AHF_THREADS))),
                     dim3(AHF_THREADS), 0, s, part, chunks, n, eps, area, qd, ldq, m, qa, lda);
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" size_t rad_absorbed_flux_workspace_bytes(int64_t n, int64_t m) {
  if (n < 1 || m < 1 || m > RAD_AHF_MAX_CASES) return 0;
  const int mc = cases_pad(m);
  return ahf_w_bytes(n, mc) + static_cast<size_t>(ahf_chunks(n, mc)) * static_cast<size_t>(n) * mc * sizeof(double);
}

extern "C" int32_t rad_absorbed_flux(const double* B, int64_t n, int64_t ldb, const double* eps,
                                     const double* rho, const double* area, const double* Qd, int64_t m,
                                     int64_t ldq, double* Qa, int64_t lda, void* work, size_t work_bytes,
                                     void* stream) {
  ApiRange range("rad_absorbed_flux");
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_absorbed_flux: n out of range");
  RAD_REQUIRE(m >= 1 && m <= RAD_AHF_MAX_CASES, RAD_EINVAL, "rad_absorbed_flux: m outside [1, RAD_AHF_MAX_CASES]");
  RAD_REQUIRE(ldb >= n + 1 && ldq >= m && lda >= m, RAD_EINVAL, "rad_absorbed_flux: leading dimension too small");
  RAD_REQUIRE(B && eps && rho && area && Qd && Qa, RAD_EINVAL, "rad_absorbed_flux: NULL pointer");
  RAD_REQUIRE(work && work_bytes >= rad_absorbed_flux_workspace_bytes(n, m) &&
                  reinterpret_cast<uintptr_t>(work) % 256 == 0,
              RAD_EWORKSPACE, "rad_absorbed_flux: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n), mi = static_cast<int>(m);
  char* ws = static_cast<char*>(work);
  switch (cases_pad(m)) {
    case 1: ahf_launch<1>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, ws, s); break;
    case 2: ahf_launch<2>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, ws, s); break;
    case 4: ahf_launch<4>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, ws, s); break;
    case 8: ahf_launch<8>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, ws, s); break;
    default: ahf_launch<16>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, ws, s); break;
  }
  RAD_HIP_CHECK(hipGetLastError());
  return RAD_OK;
}
