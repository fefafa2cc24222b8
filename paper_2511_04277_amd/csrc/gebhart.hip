// Open-system Gebhart REF solve (thesis App. B.2, eq. B.6-B.11) and its
// adjoint on gfx950.
//
//   K = I - F_sq diag(rho),  E = [F_sq diag(eps) | F_space],  B = K^{-1} E.
//
// K is strictly diagonally dominant by rows (sum_k rho_k F_ik <= max rho < 1),
// so block Gaussian elimination needs no pivoting and every Schur complement
// stays dominant.  The factorization is a block LDU with 128 x 128 blocks that
// never splits a diagonal block:  for panel k,
//   D_k^{-1}       Gauss-Jordan inverse of the diagonal block (one workgroup, LDS)
//   X   = A21 D^{-1}                (MFMA GEMM, in place: block column of L)
//   A22 -= X A12,  Y2 -= X Y1       (MFMA GEMM over the trailing matrix and the
//                                     n+1 right-hand sides in one launch)
// so K = L U with L block-unit-lower (blocks X) and U block-upper (diagonal
// blocks D_k, off-diagonal blocks A12); the forward substitution of E is
// fused into the trailing updates.  Back substitution: B_k = D_k^{-1} Y_k,
// Y_top -= U_top,k B_k.  The matrix K is padded to a multiple of 128 with
// identity blocks, which leaves the solution unchanged.
//
// RAD_PREC_FP32_IR runs the same factorization and solves in FP32 MFMA, then
// refines in FP64: R = E - K B = (E - B) + F_sq diag(rho) B as an FP64 MFMA
// GEMM, delta = K^{-1} R with the FP32 factors, B += delta.
//
// Adjoint: K^T = U^T L^T, so Lambda = K^{-T} G is a block forward solve with
// U^T (diagonal blocks D_k^{-T}) followed by a block backward solve with L^T,
// both reusing the stored factors through transposed-A GEMMs.
#include "common.h"
#include "gemm.h"

#include <algorithm>
#include <cmath>

namespace rad {
namespace {

constexpr int NB = 128;          // factorization block
constexpr int GJ_THREADS = 1024;

template <class T>
constexpr long pad_elems() { return 128 / static_cast<long>(sizeof(T)); }

// ---------------------------------------------------------------- layout ----
struct FactorLayout {
  int64_t n, np, P;
  long ldk;
  size_t kf_off, dinv_off, bytes;
};

template <class T>
FactorLayout factor_layout(int64_t n) {
  FactorLayout f;
  f.n = n;
  f.np = ceil_div(n, NB) * NB;
  f.P = f.np / NB;
  f.ldk = static_cast<long>(f.np + pad_elems<T>());
  f.kf_off = 0;
  f.dinv_off = align_up(static_cast<size_t>(f.np) * f.ldk * sizeof(T), 256);
  f.bytes = f.dinv_off + align_up(static_cast<size_t>(f.P) * NB * NB * sizeof(T), 256);
  return f;
}

inline long rhs_ld(int64_t n, long pad) { return static_cast<long>(ceil_div(n + 1, 64) * 64 + pad); }

struct Scalars {
  int status;
  int pad;
  double max_r;      // max |residual|
  double max_d;      // max |correction|
  double red[2];     // REF check outputs / spare
};

template <class T>
struct Fact {
  T* kf;
  long ldk;
  T* dinv;
  int n, np, P;
};

template <class T>
Fact<T> make_fact(void* base, const FactorLayout& l) {
  Fact<T> f;
  f.kf = reinterpret_cast<T*>(static_cast<char*>(base) + l.kf_off);
  f.ldk = l.ldk;
  f.dinv = reinterpret_cast<T*>(static_cast<char*>(base) + l.dinv_off);
  f.n = static_cast<int>(l.n);
  f.np = static_cast<int>(l.np);
  f.P = static_cast<int>(l.P);
  return f;
}

// ---------------------------------------------------------------- kernels ---
__global__ void scalars_init(Scalars* sc) {
  if (threadIdx.x == 0) {
    sc->status = 0;
    sc->max_r = 0.0;
    sc->max_d = 0.0;
    sc->red[0] = sc->red[1] = 0.0;
  }
}

__global__ void scalars_init_partial(Scalars* sc) {
  if (threadIdx.x == 0) {
    sc->max_r = 0.0;
    sc->max_d = 0.0;
  }
}

// R = G - Lambda (fp64)
__global__ void __launch_bounds__(256)
adj_residual_init(const double* __restrict__ G, long ldg, int n, const double* __restrict__ L, long ldl,
                  double* __restrict__ R, long ldr) {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j <= n; j += blockDim.x)
    R[static_cast<long>(i) * ldr + j] = G[static_cast<long>(i) * ldg + j] - L[static_cast<long>(i) * ldl + j];
}

__global__ void check_optical(const double* __restrict__ eps, const double* __restrict__ rho,
                              int n, Scalars* sc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e = eps ? eps[i] : 0.5, r = rho[i];
  if (!(e >= 0.0 && e <= 1.0 && r >= 0.0 && r <= 1.0)) raise_status(&sc->status, RAD_ENONFINITE);
}

// K (padded with identity) and E (padded with zeros) in precision T.
template <class T>
__global__ void __launch_bounds__(256)
geb_form(const double* __restrict__ F, long ldf, int n, const double* __restrict__ eps,
         const double* __restrict__ rho, T* __restrict__ KF, long ldk, int np,
         T* __restrict__ Y, long ldy, int wy, Scalars* sc) {
  const int i = blockIdx.x;
  const double* frow = F + static_cast<long>(i) * ldf;
  T* krow = KF + static_cast<long>(i) * ldk;
  T* yrow = Y + static_cast<long>(i) * ldy;
  int bad = 0;
  const int jend = np > wy ? np : wy;
  for (int j = threadIdx.x; j < jend; j += blockDim.x) {
    double kv = (i == j) ? 1.0 : 0.0;
    double yv = 0.0;
    if (i < n && j <= n) {
      double f = frow[j];
      bad |= !(f >= 0.0 && f <= 1.0e300);
      if (j < n) {
        kv = kv - f * rho[j];
        yv = f * eps[j];
      } else {
        yv = f;  // space column: no emissivity factor (eq. B.6)
      }
    }
    if (j < np) krow[j] = static_cast<T>(kv);
    if (j < wy) yrow[j] = static_cast<T>(yv);
  }
  if (bad) raise_status(&sc->status, RAD_ENONFINITE);
}

// In-place Gauss-Jordan inverse of one NB x NB diagonal block, no pivoting.
template <class T>
__global__ void __launch_bounds__(GJ_THREADS)
gj_inverse(const T* __restrict__ A, long lda, T* __restrict__ out, Scalars* sc) {
  __shared__ T M[NB][NB + 1];
  const int tid = threadIdx.x;
  const int j = tid & (NB - 1);
  const int i0 = tid >> 7;                 // 0..7
  constexpr int R = NB / (GJ_THREADS / NB); // 16 rows per thread
  for (int q = 0; q < R; ++q) {
    int i = i0 + 8 * q;
    M[i][j] = A[static_cast<long>(i) * lda + j];
  }
  __syncthreads();
  int singular = 0;
  for (int p = 0; p < NB; ++p) {
    T piv = M[p][p];
    T mpj = M[p][j];
    T mip[R];
#pragma unroll
    for (int q = 0; q < R; ++q) mip[q] = M[i0 + 8 * q][p];
    __syncthreads();
    T d = T(1) / piv;
    // K has unit diagonal scale and its pivots stay >= 1 - max rho for valid
    // input; a pivot below this threshold means a (numerically) singular K.
    const double tiny = sizeof(T) == 8 ? 1e-11 : 1e-5;
    if (!(fabs(static_cast<double>(piv)) > tiny) || !(fabs(static_cast<double>(d)) < 1e300)) {
      singular = 1;
      d = T(0);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      int i = i0 + 8 * q;
      T v;
      if (i == p) {
        v = (j == p) ? d : mpj * d;
      } else if (j == p) {
        v = -mip[q] * d;
      } else {
        v = M[i][j] - mip[q] * (mpj * d);
      }
      M[i][j] = v;
    }
    __syncthreads();
  }
  for (int q = 0; q < R; ++q) {
    int i = i0 + 8 * q;
    out[i * NB + j] = M[i][j];
  }
  if (singular && tid == 0) raise_status(&sc->status, RAD_ESINGULAR);
}

// B (fp64, n x (n+1)) <- Y (T)
template <class T>
__global__ void __launch_bounds__(256)
store_solution(const T* __restrict__ Y, long ldy, int n, double* __restrict__ B, long ldb) {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j <= n; j += blockDim.x)
    B[static_cast<long>(i) * ldb + j] = static_cast<double>(Y[static_cast<long>(i) * ldy + j]);
}

__device__ inline void block_max(double v, double* target) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(target, v);
}

// R = E - B  (fp64), E from F and eps on the fly
__global__ void __launch_bounds__(256)
residual_init(const double* __restrict__ F, long ldf, int n, const double* __restrict__ eps,
              const double* __restrict__ B, long ldb, double* __restrict__ R, long ldr) {
  const int i = blockIdx.x;
  const double* f = F + static_cast<long>(i) * ldf;
  const double* b = B + static_cast<long>(i) * ldb;
  double* r = R + static_cast<long>(i) * ldr;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) {
    double e = (j < n) ? f[j] * eps[j] : f[n];
    r[j] = e - b[j];
  }
}

// Y32 <- R (rows < n), records max |R|
__global__ void __launch_bounds__(256)
residual_to_rhs(const double* __restrict__ R, long ldr, int n, float* __restrict__ Y, long ldy,
                Scalars* sc) {
  const int i = blockIdx.x;
  double m = 0.0;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) {
    double v = R[static_cast<long>(i) * ldr + j];
    m = fmax(m, fabs(v));
    Y[static_cast<long>(i) * ldy + j] = static_cast<float>(v);
  }
  block_max(m, &sc->max_r);
}

// X += Y32 (rows < n), records max |delta|
__global__ void __launch_bounds__(256)
apply_correction(const float* __restrict__ Y, long ldy, int n, double* __restrict__ X, long ldx,
                 Scalars* sc) {
  const int i = blockIdx.x;
  double m = 0.0;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) {
    double d = static_cast<double>(Y[static_cast<long>(i) * ldy + j]);
    m = fmax(m, fabs(d));
    X[static_cast<long>(i) * ldx + j] += d;
  }
  block_max(m, &sc->max_d);
}

// Y (T, padded rows zero) <- G (fp64)
template <class T>
__global__ void __launch_bounds__(256)
load_rhs(const double* __restrict__ G, long ldg, int n, T* __restrict__ Y, long ldy, int wy) {
  const int i = blockIdx.x;
  T* y = Y + static_cast<long>(i) * ldy;
  for (int j = threadIdx.x; j < wy; j += blockDim.x)
    y[j] = (j <= n && i < n) ? static_cast<T>(G[static_cast<long>(i) * ldg + j]) : T(0);
}

// REF closure residual: one wave per row, fixed-order reduction.
__global__ void __launch_bounds__(256)
ref_closure(const double* __restrict__ B, long ldb, int n, Scalars* sc) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  double s = 0.0;
  if (row < n)
    for (int j = l; j <= n; j += 64) s += B[static_cast<long>(row) * ldb + j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  double d = (row < n) ? fabs(s - 1.0) : 0.0;
  if (l == 0) atomic_max_nonneg(&sc->red[0], d);
}

// REF reciprocity residual max |eps_i A_i B_ij - eps_j A_j B_ji| over 64x64 tile pairs
__global__ void __launch_bounds__(256)
ref_reciprocity(const double* __restrict__ B, long ldb, int n, const double* __restrict__ eps,
                const double* __restrict__ area, Scalars* sc) {
  __shared__ double sT[64][65];
  const int I = blockIdx.y, J = blockIdx.x;
  if (J < I) return;
  const int tid = threadIdx.x, c = tid & 63, rg = tid >> 6;
  for (int m = 0; m < 16; ++m) {
    int r = rg + 4 * m;
    int i = J * 64 + r, j = I * 64 + c;
    sT[r][c] = (i < n && j < n) ? eps[i] * area[i] * B[static_cast<long>(i) * ldb + j] : 0.0;
  }
  __syncthreads();
  double mx = 0.0;
  for (int m = 0; m < 16; ++m) {
    int r = rg + 4 * m;
    int i = I * 64 + r, j = J * 64 + c;
    if (i < n && j < n) {
      double g = eps[i] * area[i] * B[static_cast<long>(i) * ldb + j];
      mx = fmax(mx, fabs(g - sT[c][r]));
    }
  }
  block_max(mx, &sc->red[1]);
}

__global__ void copy_scalars_out(const Scalars* sc, double* out) {
  if (threadIdx.x == 0) {
    out[0] = sc->red[0];
    out[1] = sc->red[1];
  }
}

// grad_eps[k] = sum_i Lambda_ik F_ik   (column reduction, fixed order)
__global__ void __launch_bounds__(256)
adj_grad_eps(const double* __restrict__ L, long ldl, const double* __restrict__ F, long ldf,
             int n, double* __restrict__ ge) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += L[static_cast<long>(i) * ldl + k] * F[static_cast<long>(i) * ldf + k];
  ge[k] = s;
}

// grad_rho[k] = (1/rho_k) sum_j B_kj (Lambda_kj - G_kj)   (one wave per row)
__global__ void __launch_bounds__(256)
adj_grad_rho(const double* __restrict__ L, long ldl, const double* __restrict__ G, long ldg,
             const double* __restrict__ B, long ldb, const double* __restrict__ rho, int n,
             double* __restrict__ gr) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (k >= n) return;
  double s = 0.0;
  for (int j = l; j <= n; j += 64)
    s += B[static_cast<long>(k) * ldb + j] *
         (L[static_cast<long>(k) * ldl + j] - G[static_cast<long>(k) * ldg + j]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (l == 0 && rho[k] >= 1e-3) gr[k] = s / rho[k];
}

// direct form for small rho_k: sum_j B_kj sum_i F_ik Lambda_ij
__global__ void __launch_bounds__(256)
adj_grad_rho_direct(const double* __restrict__ L, long ldl, const double* __restrict__ F, long ldf,
                    const double* __restrict__ B, long ldb, const double* __restrict__ rho, int n,
                    double* __restrict__ gr) {
  const int k = blockIdx.x;
  if (rho[k] >= 1e-3) return;
  __shared__ double red[4];
  double acc = 0.0;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += F[static_cast<long>(i) * ldf + k] * L[static_cast<long>(i) * ldl + j];
    acc += B[static_cast<long>(k) * ldb + j] * t;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) gr[k] = red[0] + red[1] + red[2] + red[3];
}

// Lambda_out (fp64, n x (n+1)) <- Y (T)
template <class T>
__global__ void __launch_bounds__(256)
copy_out(const T* __restrict__ Y, long ldy, int n, double* __restrict__ X, long ldx) {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j <= n; j += blockDim.x)
    X[static_cast<long>(i) * ldx + j] = static_cast<double>(Y[static_cast<long>(i) * ldy + j]);
}

// ---------------------------------------------------------------- drivers ---
#define RAD_GEMM(args, trans)                                  \
  do {                                                         \
    hipError_t _e = launch_gemm((args), (trans), s);           \
    if (_e != hipSuccess) return _e;                           \
  } while (0)

// LDU factorization of K in place; if Y is given, its rows are eliminated too.
template <class T>
hipError_t factor_forward(const Fact<T>& f, T* Y, long ldy, int wy, Scalars* sc, hipStream_t s) {
  for (int k = 0; k < f.P; ++k) {
    const long r0 = static_cast<long>(k) * NB;
    T* akk = f.kf + r0 * f.ldk + r0;
    T* dk = f.dinv + r0 * NB;
    {
      ProfScope prof(s, RAD_PROF_DIAG_INVERSE, 2.0 * NB * NB * NB, 0.0);
      hipLaunchKernelGGL(gj_inverse<T>, dim3(1), dim3(GJ_THREADS), 0, s, akk, f.ldk, dk, sc);
    }
    if (k + 1 == f.P) break;
    const long r1 = r0 + NB;
    const int m = f.np - static_cast<int>(r1);
    T* a21 = f.kf + r1 * f.ldk + r0;
    GemmArgs<T> x = gemm_args<T>(a21, f.ldk, m, NB, T(1), T(0));
    gemm_add_segment<T>(x, dk, NB, a21, f.ldk, NB);
    RAD_GEMM(x, false);
    GemmArgs<T> t = gemm_args<T>(a21, f.ldk, m, NB, T(-1), T(1));
    gemm_add_segment<T>(t, f.kf + r0 * f.ldk + r1, f.ldk, f.kf + r1 * f.ldk + r1, f.ldk, m);
    if (Y) gemm_add_segment<T>(t, Y + r0 * ldy, ldy, Y + r1 * ldy, ldy, wy);
    RAD_GEMM(t, false);
  }
  return hipGetLastError();
}

// Y <- L^{-1} Y with the stored factors (for refinement right-hand sides).
template <class T>
hipError_t forward_only(const Fact<T>& f, T* Y, long ldy, int wy, hipStream_t s) {
  for (int k = 0; k + 1 < f.P; ++k) {
    const long r0 = static_cast<long>(k) * NB, r1 = r0 + NB;
    GemmArgs<T> t = gemm_args<T>(f.kf + r1 * f.ldk + r0, f.ldk, f.np - static_cast<int>(r1), NB, T(-1), T(1));
    gemm_add_segment<T>(t, Y + r0 * ldy, ldy, Y + r1 * ldy, ldy, wy);
    RAD_GEMM(t, false);
  }
  return hipSuccess;
}

// Out <- U^{-1} Y.  Out may alias Y.  Only the first n rows are formed.
template <class T>
hipError_t back_solve(const Fact<T>& f, T* Y, long ldy, int wy, T* Out, long ldo, hipStream_t s) {
  for (int k = f.P - 1; k >= 0; --k) {
    const long r0 = static_cast<long>(k) * NB;
    const int kk = std::min<int>(NB, f.n - static_cast<int>(r0));
    GemmArgs<T> d = gemm_args<T>(f.dinv + r0 * NB, NB, kk, kk, T(1), T(0));
    gemm_add_segment<T>(d, Y + r0 * ldy, ldy, Out + r0 * ldo, ldo, wy);
    RAD_GEMM(d, false);
    if (k == 0) break;
    GemmArgs<T> u = gemm_args<T>(f.kf + r0, f.ldk, static_cast<int>(r0), kk, T(-1), T(1));
    gemm_add_segment<T>(u, Out + r0 * ldo, ldo, Y, ldy, wy);
    RAD_GEMM(u, false);
  }
  return hipSuccess;
}

// Lambda <- K^{-T} Y in place:  U^T Z = Y  then  L^T Lambda = Z.
template <class T>
hipError_t transposed_solve(const Fact<T>& f, T* Y, long ldy, int wy, hipStream_t s) {
  for (int k = 0; k < f.P; ++k) {
    const long r0 = static_cast<long>(k) * NB;
    // Z_k = D_k^{-T} Y_k
    GemmArgs<T> d = gemm_args<T>(f.dinv + r0 * NB, NB, NB, NB, T(1), T(0));
    gemm_add_segment<T>(d, Y + r0 * ldy, ldy, Y + r0 * ldy, ldy, wy);
    RAD_GEMM(d, true);
    if (k + 1 == f.P) break;
    const long r1 = r0 + NB;
    // Y_below -= (U_{k, below})^T Z_k
    GemmArgs<T> u = gemm_args<T>(f.kf + r0 * f.ldk + r1, f.ldk, f.np - static_cast<int>(r1), NB, T(-1), T(1));
    gemm_add_segment<T>(u, Y + r0 * ldy, ldy, Y + r1 * ldy, ldy, wy);
    RAD_GEMM(u, true);
  }
  for (int k = f.P - 1; k >= 1; --k) {
    const long r0 = static_cast<long>(k) * NB;
    // Y_above -= (X_{k, above})^T Lambda_k
    GemmArgs<T> x = gemm_args<T>(f.kf + r0 * f.ldk, f.ldk, static_cast<int>(r0), NB, T(-1), T(1));
    gemm_add_segment<T>(x, Y + r0 * ldy, ldy, Y, ldy, wy);
    RAD_GEMM(x, true);
  }
  return hipSuccess;
}

struct GebWork {
  Scalars* sc;
  void* y;      // RHS / solution (T), np x ldy
  long ldy;
  double* r;    // FP64 residual (n x ldr), refinement only
  long ldr;
  double* lam;  // FP64 Lambda (adjoint refinement when the caller gives none)
  long ldl;
  size_t bytes;
  bool ok;
};

GebWork geb_work(void* work, size_t bytes, int64_t n, int32_t prec, bool adjoint) {
  Carve cv(work, bytes);
  GebWork w{};
  const int64_t np = ceil_div(n, NB) * NB;
  w.sc = cv.take<Scalars>(1);
  if (prec == RAD_PREC_FP64) {
    w.ldy = rhs_ld(n, pad_elems<double>());
    w.y = cv.take<double>(static_cast<size_t>(np) * w.ldy);
  } else {
    w.ldy = rhs_ld(n, pad_elems<float>());
    w.y = cv.take<float>(static_cast<size_t>(np) * w.ldy);
    w.ldr = static_cast<long>(ceil_div(n + 1, 16) * 16);
    w.r = cv.take<double>(static_cast<size_t>(n) * w.ldr);
    if (adjoint) {
      w.ldl = w.ldr;
      w.lam = cv.take<double>(static_cast<size_t>(n) * w.ldl);
    }
  }
  w.bytes = cv.used;
  w.ok = cv.ok;
  return w;
}

size_t factor_bytes(int64_t n, int32_t prec) {
  return prec == RAD_PREC_FP64 ? factor_layout<double>(n).bytes : factor_layout<float>(n).bytes;
}

int read_scalars(Scalars* dev, Scalars* host, hipStream_t s) {
  RAD_HIP_CHECK(hipMemcpyAsync(host, dev, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  RAD_HIP_CHECK(hipStreamSynchronize(s));
  return RAD_OK;
}

// FP64 residual R = E - K X = (E - X) + F_sq diag(rho) X  (X n x (n+1) fp64)
hipError_t residual64(const double* F, long ldf, int n, const double* eps, const double* rho,
                      const double* X, long ldx, double* R, long ldr, hipStream_t s) {
  hipLaunchKernelGGL(residual_init, dim3(n), dim3(256), 0, s, F, ldf, n, eps, X, ldx, R, ldr);
  GemmArgs<double> a = gemm_args<double>(F, ldf, n, n, 1.0, 1.0);
  a.colscale = rho;
  gemm_add_segment<double>(a, X, ldx, R, ldr, n + 1);
  return launch_gemm(a, false, s);
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" size_t rad_gebhart_factor_bytes(int64_t n, int32_t precision) {
  if (n < 1 || (precision != RAD_PREC_FP64 && precision != RAD_PREC_FP32_IR)) return 0;
  return factor_bytes(n, precision);
}

extern "C" size_t rad_gebhart_workspace_bytes(int64_t n, int32_t precision) {
  if (n < 1 || (precision != RAD_PREC_FP64 && precision != RAD_PREC_FP32_IR)) return 0;
  return geb_work(nullptr, 0, n, precision, false).bytes;
}

extern "C" int32_t rad_gebhart_ref(const double* F, int64_t n, int64_t ldf, const double* eps,
                                   const double* rho, double* B, int64_t ldb, int32_t precision,
                                   double ir_tol, int32_t ir_max, void* factors, size_t fbytes,
                                   void* work, size_t wbytes, rad_stats* stats, void* stream) {
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_gebhart_ref: n out of range");
  RAD_REQUIRE(ldf >= n + 1 && ldb >= n + 1, RAD_EINVAL, "rad_gebhart_ref: ldf or ldb < n+1");
  RAD_REQUIRE(F && eps && rho && B && factors, RAD_EINVAL, "rad_gebhart_ref: NULL pointer");
  RAD_REQUIRE(precision == RAD_PREC_FP64 || precision == RAD_PREC_FP32_IR, RAD_EINVAL,
              "rad_gebhart_ref: unknown precision");
  RAD_REQUIRE(ir_max >= 0 && ir_tol >= 0.0, RAD_EINVAL, "rad_gebhart_ref: ir_max < 0 or ir_tol < 0");
  RAD_REQUIRE(fbytes >= factor_bytes(n, precision) && reinterpret_cast<uintptr_t>(factors) % 256 == 0,
              RAD_EWORKSPACE, "rad_gebhart_ref: factor buffer too small or not 256-byte aligned");
  GebWork w = geb_work(work, wbytes, n, precision, false);
  RAD_REQUIRE(w.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_gebhart_ref: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n);
  hipLaunchKernelGGL(scalars_init, dim3(1), dim3(64), 0, s, w.sc);
  hipLaunchKernelGGL(check_optical, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s,
                     eps, rho, ni, w.sc);
  int ir_steps = 0;
  Scalars h{};
  if (precision == RAD_PREC_FP64) {
    FactorLayout fl = factor_layout<double>(n);
    Fact<double> f = make_fact<double>(factors, fl);
    double* Y = static_cast<double*>(w.y);
    hipLaunchKernelGGL(geb_form<double>, dim3(f.np), dim3(256), 0, s, F, static_cast<long>(ldf), ni, eps,
                       rho, f.kf, f.ldk, f.np, Y, w.ldy, ni + 1, w.sc);
    RAD_HIP_CHECK(factor_forward<double>(f, Y, w.ldy, ni + 1, w.sc, s));
    RAD_HIP_CHECK(back_solve<double>(f, Y, w.ldy, ni + 1, B, static_cast<long>(ldb), s));
  } else {
    FactorLayout fl = factor_layout<float>(n);
    Fact<float> f = make_fact<float>(factors, fl);
    float* Y = static_cast<float*>(w.y);
    hipLaunchKernelGGL(geb_form<float>, dim3(f.np), dim3(256), 0, s, F, static_cast<long>(ldf), ni, eps,
                       rho, f.kf, f.ldk, f.np, Y, w.ldy, ni + 1, w.sc);
    RAD_HIP_CHECK(factor_forward<float>(f, Y, w.ldy, ni + 1, w.sc, s));
    RAD_HIP_CHECK(back_solve<float>(f, Y, w.ldy, ni + 1, Y, w.ldy, s));
    hipLaunchKernelGGL(store_solution<float>, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, B,
                       static_cast<long>(ldb));
    for (int step = 0; step < ir_max; ++step) {
      hipLaunchKernelGGL(scalars_init_partial, dim3(1), dim3(64), 0, s, w.sc);
      RAD_HIP_CHECK(residual64(F, static_cast<long>(ldf), ni, eps, rho, B, static_cast<long>(ldb), w.r,
                               w.ldr, s));
      hipLaunchKernelGGL(residual_to_rhs, dim3(ni), dim3(256), 0, s, w.r, w.ldr, ni, Y, w.ldy, w.sc);
      RAD_HIP_CHECK(forward_only<float>(f, Y, w.ldy, ni + 1, s));
      RAD_HIP_CHECK(back_solve<float>(f, Y, w.ldy, ni + 1, Y, w.ldy, s));
      hipLaunchKernelGGL(apply_correction, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, B,
                         static_cast<long>(ldb), w.sc);
      ++ir_steps;
      int rc = read_scalars(w.sc, &h, s);
      if (rc != RAD_OK) return rc;
      if (h.status < 0 || h.max_d <= ir_tol) break;
    }
  }
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats && precision == RAD_PREC_FP64) return RAD_OK;
  int rc = read_scalars(w.sc, &h, s);
  if (rc != RAD_OK) return rc;
  if (stats) {
    *stats = rad_stats{};
    stats->ir_steps = ir_steps;
    stats->device_status = h.status;
    stats->ir_correction = h.max_d;
    stats->ir_residual = h.max_r;
    stats->converged = (precision == RAD_PREC_FP64) || (ir_steps > 0 && h.max_d <= ir_tol);
  }
  if (h.status < 0) {
    set_error(h.status == RAD_ESINGULAR ? "rad_gebhart_ref: singular diagonal block of K"
                                        : "rad_gebhart_ref: F, eps or rho out of range or non-finite");
    return h.status;
  }
  if (precision == RAD_PREC_FP32_IR && ir_max > 0 && !(h.max_d <= ir_tol)) return RAD_WNOTCONVERGED;
  return RAD_OK;
}

extern "C" size_t rad_ref_check_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return align_up(sizeof(Scalars), 256);
}

extern "C" int32_t rad_ref_check(const double* B, int64_t n, int64_t ldb, const double* eps,
                                 const double* area, double* out, void* work, size_t wbytes,
                                 void* stream) {
  clear_error();
  RAD_REQUIRE(n >= 1 && ldb >= n + 1, RAD_EINVAL, "rad_ref_check: bad n or ldb");
  RAD_REQUIRE(B && eps && area && out, RAD_EINVAL, "rad_ref_check: NULL pointer");
  RAD_REQUIRE(work && wbytes >= sizeof(Scalars) && reinterpret_cast<uintptr_t>(work) % 256 == 0,
              RAD_EWORKSPACE, "rad_ref_check: workspace too small or misaligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scalars* sc = static_cast<Scalars*>(work);
  const int ni = static_cast<int>(n);
  hipLaunchKernelGGL(scalars_init, dim3(1), dim3(64), 0, s, sc);
  hipLaunchKernelGGL(ref_closure, dim3(static_cast<unsigned>(ceil_div(n, 4))), dim3(256), 0, s, B,
                     static_cast<long>(ldb), ni, sc);
  const unsigned t = static_cast<unsigned>(ceil_div(n, 64));
  hipLaunchKernelGGL(ref_reciprocity, dim3(t, t), dim3(256), 0, s, B, static_cast<long>(ldb), ni, eps,
                     area, sc);
  hipLaunchKernelGGL(copy_scalars_out, dim3(1), dim3(64), 0, s, sc, out);
  RAD_HIP_CHECK(hipGetLastError());
  return RAD_OK;
}

extern "C" size_t rad_adjoint_workspace_bytes(int64_t n, int32_t precision) {
  if (n < 1 || (precision != RAD_PREC_FP64 && precision != RAD_PREC_FP32_IR)) return 0;
  return geb_work(nullptr, 0, n, precision, true).bytes;
}

extern "C" int32_t rad_gebhart_ref_adjoint(const void* factors, size_t fbytes, int32_t precision,
                                           const double* F, int64_t n, int64_t ldf, const double* rho,
                                           const double* B, int64_t ldb, const double* G, int64_t ldg,
                                           double* grad_eps, double* grad_rho, double* Lambda,
                                           int64_t ldl, double ir_tol, int32_t ir_max, void* work,
                                           size_t wbytes, rad_stats* stats, void* stream) {
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_gebhart_ref_adjoint: n out of range");
  RAD_REQUIRE(ldf >= n + 1 && ldb >= n + 1 && ldg >= n + 1 && (!Lambda || ldl >= n + 1), RAD_EINVAL,
              "rad_gebhart_ref_adjoint: leading dimension < n+1");
  RAD_REQUIRE(factors && F && rho && B && G && grad_eps && grad_rho, RAD_EINVAL,
              "rad_gebhart_ref_adjoint: NULL pointer");
  RAD_REQUIRE(precision == RAD_PREC_FP64 || precision == RAD_PREC_FP32_IR, RAD_EINVAL,
              "rad_gebhart_ref_adjoint: unknown precision");
  RAD_REQUIRE(ir_max >= 0 && ir_tol >= 0.0, RAD_EINVAL, "rad_gebhart_ref_adjoint: bad ir_max / ir_tol");
  RAD_REQUIRE(fbytes >= factor_bytes(n, precision), RAD_EWORKSPACE,
              "rad_gebhart_ref_adjoint: factor buffer smaller than the factorization of n");
  GebWork w = geb_work(work, wbytes, n, precision, true);
  RAD_REQUIRE(w.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_gebhart_ref_adjoint: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n);
  hipLaunchKernelGGL(scalars_init, dim3(1), dim3(64), 0, s, w.sc);
  const double* lam = nullptr;
  long ldlam = 0;
  int ir_steps = 0;
  Scalars h{};
  if (precision == RAD_PREC_FP64) {
    FactorLayout fl = factor_layout<double>(n);
    Fact<double> f = make_fact<double>(const_cast<void*>(factors), fl);
    double* Y = static_cast<double*>(w.y);
    hipLaunchKernelGGL(load_rhs<double>, dim3(f.np), dim3(256), 0, s, G, static_cast<long>(ldg), ni, Y,
                       w.ldy, ni + 1);
    RAD_HIP_CHECK(transposed_solve<double>(f, Y, w.ldy, ni + 1, s));
    lam = Y;
    ldlam = w.ldy;
    if (Lambda)
      hipLaunchKernelGGL(copy_out<double>, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, Lambda,
                         static_cast<long>(ldl));
  } else {
    FactorLayout fl = factor_layout<float>(n);
    Fact<float> f = make_fact<float>(const_cast<void*>(factors), fl);
    float* Y = static_cast<float*>(w.y);
    double* L64 = Lambda ? Lambda : w.lam;
    const long ld64 = Lambda ? static_cast<long>(ldl) : w.ldl;
    hipLaunchKernelGGL(load_rhs<float>, dim3(f.np), dim3(256), 0, s, G, static_cast<long>(ldg), ni, Y,
                       w.ldy, ni + 1);
    RAD_HIP_CHECK(transposed_solve<float>(f, Y, w.ldy, ni + 1, s));
    hipLaunchKernelGGL(store_solution<float>, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, L64, ld64);
    for (int step = 0; step < ir_max; ++step) {
      hipLaunchKernelGGL(scalars_init_partial, dim3(1), dim3(64), 0, s, w.sc);
      // R = G - K^T Lambda = (G - Lambda) + diag(rho) F_sq^T Lambda
      hipLaunchKernelGGL(adj_residual_init, dim3(ni), dim3(256), 0, s, G, static_cast<long>(ldg), ni, L64,
                         ld64, w.r, w.ldr);
      GemmArgs<double> a = gemm_args<double>(F, static_cast<long>(ldf), ni, ni, 1.0, 1.0);
      a.rowscale = rho;
      gemm_add_segment<double>(a, L64, ld64, w.r, w.ldr, ni + 1);
      RAD_HIP_CHECK(launch_gemm(a, true, s));
      hipLaunchKernelGGL(residual_to_rhs, dim3(ni), dim3(256), 0, s, w.r, w.ldr, ni, Y, w.ldy, w.sc);
      RAD_HIP_CHECK(transposed_solve<float>(f, Y, w.ldy, ni + 1, s));
      hipLaunchKernelGGL(apply_correction, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, L64, ld64, w.sc);
      ++ir_steps;
      int rc = read_scalars(w.sc, &h, s);
      if (rc != RAD_OK) return rc;
      if (h.max_d <= ir_tol) break;
    }
    lam = L64;
    ldlam = ld64;
  }
  hipLaunchKernelGGL(adj_grad_eps, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, lam,
                     ldlam, F, static_cast<long>(ldf), ni, grad_eps);
  hipLaunchKernelGGL(adj_grad_rho, dim3(static_cast<unsigned>(ceil_div(n, 4))), dim3(256), 0, s, lam, ldlam,
                     G, static_cast<long>(ldg), B, static_cast<long>(ldb), rho, ni, grad_rho);
  hipLaunchKernelGGL(adj_grad_rho_direct, dim3(ni), dim3(256), 0, s, lam, ldlam, F, static_cast<long>(ldf),
                     B, static_cast<long>(ldb), rho, ni, grad_rho);
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats) return RAD_OK;
  int rc = read_scalars(w.sc, &h, s);
  if (rc != RAD_OK) return rc;
  *stats = rad_stats{};
  stats->ir_steps = ir_steps;
  stats->device_status = h.status;
  stats->ir_correction = h.max_d;
  stats->ir_residual = h.max_r;
  stats->converged = (precision == RAD_PREC_FP64) || (ir_steps > 0 && h.max_d <= ir_tol);
  if (precision == RAD_PREC_FP32_IR && ir_max > 0 && !(h.max_d <= ir_tol)) return RAD_WNOTCONVERGED;
  return RAD_OK;
}
