// Absorbed heat fluxes from REFs and direct heat fluxes (thesis Sec. 4.2.3,
// eq. 4.6), for m load cases at once:
//
//   Qa[i][c] = A_i eps_i Qd[i][c] + sum_j B_ji A_j rho_j Qd[j][c]
//
// The sum is a transposed product with the N x N block of B, which is read
// once (HBM-bound).  ahf_partial: workgroup = (256 consecutive faces i, one
// chunk of rows j); each thread owns face i and sums B_ji w_jc over its
// chunk's rows, with w_jc = A_j rho_j Qd[j][c] staged in LDS, so every load
// instruction reads 2 KB of one row of B.  ahf_final adds the direct term and
// the chunk sums in chunk order (fixed order: bitwise reproducible).
#include <algorithm>

#include "common.h"

namespace rad {
namespace {

constexpr int AHF_THREADS = 256;
constexpr int AHF_MAX_CHUNKS = 64;
constexpr int AHF_ROWS = 128;  // rows of w staged in LDS at a time

template <int MC>
__global__ void __launch_bounds__(AHF_THREADS)
ahf_partial(const double* __restrict__ B, long ldb, int n, const double* __restrict__ rho,
            const double* __restrict__ area, const double* __restrict__ qd, long ldq, int m, int rows,
            double* __restrict__ part) {
  __shared__ double w[AHF_ROWS][MC];
  const int i = blockIdx.x * AHF_THREADS + threadIdx.x;
  const int j0 = blockIdx.y * rows, j1 = min(n, j0 + rows);
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  for (int jb = j0; jb < j1; jb += AHF_ROWS) {
    const int nr = min(AHF_ROWS, j1 - jb);
    __syncthreads();  // the previous block of w is consumed
    for (int e = threadIdx.x; e < nr * MC; e += AHF_THREADS) {
      const int r = e / MC, c = e % MC, j = jb + r;
      w[r][c] = c < m ? area[j] * rho[j] * qd[static_cast<long>(j) * ldq + c] : 0.0;
    }
    __syncthreads();
    if (i < n) {
      const double* bj = B + static_cast<long>(jb) * ldb + i;
#pragma unroll 4
      for (int r = 0; r < nr; ++r) {
        const double b = bj[static_cast<long>(r) * ldb];
#pragma unroll
        for (int c = 0; c < MC; ++c) acc[c] = fma(b, w[r][c], acc[c]);
      }
    }
  }
  if (i >= n) return;
  double* p = part + (static_cast<long>(blockIdx.y) * n + i) * MC;
#pragma unroll
  for (int c = 0; c < MC; ++c) p[c] = acc[c];
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
  for (int k = 0; k < chunks; ++k) s += part[(static_cast<long>(k) * n + i) * MC + c];
  qa[static_cast<long>(i) * lda + c] = s;
}

int cases_pad(int64_t m) { return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : 16; }

int ahf_chunks(int64_t n) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(AHF_MAX_CHUNKS, ceil_div(n, AHF_ROWS))));
}

template <int MC>
void ahf_launch(const double* B, long ldb, int n, const double* eps, const double* rho, const double* area,
                const double* qd, long ldq, int m, double* qa, long lda, double* part, hipStream_t s) {
  const int chunks = ahf_chunks(n);
  const int rows = static_cast<int>(ceil_div(n, chunks));
  {
    ProfScope prof(s, RAD_PROF_AHF, 2.0 * static_cast<double>(n) * n * m, 8.0 * static_cast<double>(n) * n);
    hipLaunchKernelGGL((ahf_partial<MC>), dim3(static_cast<unsigned>(ceil_div(n, AHF_THREADS)), chunks),
                       dim3(AHF_THREADS), 0, s, B, ldb, n, rho, area, qd, ldq, m, rows, part);
  }
  hipLaunchKernelGGL((ahf_final<MC>), dim3(static_cast<unsigned>(ceil_div(static_cast<int64_t>(n) * m, AHF_THREADS))),
                     dim3(AHF_THREADS), 0, s, part, chunks, n, eps, area, qd, ldq, m, qa, lda);
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" size_t rad_absorbed_flux_workspace_bytes(int64_t n, int64_t m) {
  if (n < 1 || m < 1 || m > RAD_AHF_MAX_CASES) return 0;
  return static_cast<size_t>(ahf_chunks(n)) * static_cast<size_t>(n) * cases_pad(m) * sizeof(double);
}

extern "C" int32_t rad_absorbed_flux(const double* B, int64_t n, int64_t ldb, const double* eps,
                                     const double* rho, const double* area, const double* Qd, int64_t m,
                                     int64_t ldq, double* Qa, int64_t lda, void* work, size_t work_bytes,
                                     void* stream) {
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
  double* part = static_cast<double*>(work);
  switch (cases_pad(m)) {
    case 1: ahf_launch<1>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, part, s); break;
    case 2: ahf_launch<2>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, part, s); break;
    case 4: ahf_launch<4>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, part, s); break;
    case 8: ahf_launch<8>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, part, s); break;
    default: ahf_launch<16>(B, ldb, ni, eps, rho, area, Qd, ldq, mi, Qa, lda, part, s); break;
  }
  RAD_HIP_CHECK(hipGetLastError());
  return RAD_OK;
}
