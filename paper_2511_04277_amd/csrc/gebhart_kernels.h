// Kernels and layouts of the open-system Gebhart solve, shared by the
// single-instance and batched entry points.  See gebhart.hip.
#pragma once

#include "common.h"
#include "gemm.h"

#include <algorithm>
#include <cmath>

namespace rad {
namespace {

constexpr int NB = 128;          // diagonal block (Gauss-Jordan inverse)
constexpr int NB2 = 1024;        // panel width of the two-level updates

template <class T>
constexpr long pad_elems() { return 128 / static_cast<long>(sizeof(T)); }

// ---------------------------------------------------------------- layout ----
// Factor buffer: K's LDU factors in place (np x ldk), the inverted 128 x 128
// diagonal blocks, and per 1024-wide panel p the inverses of the panel's
// diagonal block of U (W_p, upper) and of L (V_p, unit lower), NB2 x ldw each.
struct FactorLayout {
  int64_t n, np, P;
  long ldk;
  int P2;
  long ldw;
  size_t kf_off, dinv_off, w_off, v_off, bytes;
};

template <class T>
FactorLayout factor_layout(int64_t n) {
  FactorLayout f;
  f.n = n;
  f.np = ceil_div(n, NB) * NB;
  f.P = f.np / NB;
  f.ldk = static_cast<long>(f.np + pad_elems<T>());
  f.P2 = static_cast<int>(ceil_div(f.np, NB2));
  f.ldw = NB2 + pad_elems<T>();
  f.kf_off = 0;
  f.dinv_off = align_up(static_cast<size_t>(f.np) * f.ldk * sizeof(T), 256);
  f.w_off = f.dinv_off + align_up(static_cast<size_t>(f.P) * NB * NB * sizeof(T), 256);
  const size_t wbytes = align_up(static_cast<size_t>(f.P2) * NB2 * f.ldw * sizeof(T), 256);
  f.v_off = f.w_off + wbytes;
  f.bytes = f.v_off + wbytes;
  return f;
}

// scratch of the panel-inverse products: one b x ldt block per (panel, pair,
// matrix) at every level (b <= NB2 / 2)
inline long tri_ldt(long pad) { return NB2 / 2 + pad; }
inline size_t tri_tmp_elems(int P2, long pad) { return static_cast<size_t>(P2) * NB2 * tri_ldt(pad); }

// right-hand-side buffers: columns padded to a multiple of 128 plus 128 bytes
inline long rhs_ld(int64_t n, long pad) { return static_cast<long>(ceil_div(n + 1, 128) * 128 + pad); }

struct Scalars {
  int status;
  int pad;
  double max_r;      // max |residual|
  double max_d;      // max |correction|
  double red[2];     // REF check outputs
};

template <class T>
struct Fact {
  T* kf;
  long ldk;
  T* dinv;
  int n, np, P;
  T* W;       // panel inverses of U (P2 x NB2 x ldw)
  T* V;       // panel inverses of L
  long ldw;
  int P2;
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
  f.W = reinterpret_cast<T*>(static_cast<char*>(base) + l.w_off);
  f.V = reinterpret_cast<T*>(static_cast<char*>(base) + l.v_off);
  f.ldw = l.ldw;
  f.P2 = l.P2;
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

__global__ void check_optical(const double* __restrict__ eps, const double* __restrict__ rho,
                              int n, Scalars* sc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e = eps ? eps[i] : 0.5, r = rho[i];
  if (!(e >= 0.0 && e <= 1.0 && r >= 0.0 && r <= 1.0)) raise_status(&sc->status, RAD_ENONFINITE);
}

// K (padded with identity) and E (padded with zeros) in precision T.
// Row i of both, one workgroup per row of the padded size.
template <class T>
__global__ void __launch_bounds__(256)
geb_form(const double* __restrict__ F, long ldf, int n, const double* __restrict__ eps,
         const double* __restrict__ rho, T* __restrict__ KF, long ldk, int np,
         T* __restrict__ Y, long ldy, Scalars* sc) {
  const int i = blockIdx.x;
  const double* frow = F + static_cast<long>(i) * ldf;
  T* krow = KF + static_cast<long>(i) * ldk;
  T* yrow = Y + static_cast<long>(i) * ldy;
  int bad = 0;
  const long jend = ldk > ldy ? ldk : ldy;
  for (long j = threadIdx.x; j < jend; j += blockDim.x) {
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
    if (j < ldk) krow[j] = (j < np) ? static_cast<T>(kv) : T(0);
    if (j < ldy) yrow[j] = static_cast<T>(yv);
  }
  if (bad) raise_status(&sc->status, RAD_ENONFINITE);
}

// Radiation-only steady balance (eq. 3.12-3.14 with GR_ij = sigma w_i Y_ij,
// eq. 4.2) in x = T^4, each free row divided by sigma w_i:
//   free i:  (s_i - Y_ii) x_i - sum_{j != i} Y_ij x_j = Q_i / (sigma w_i) + Y_i,space x_space,
//            s_i = sum_{j <= n} Y_ij (the row sum, space included);
//   fixed i: x_i = T_i^4.
// One workgroup per row of the padded matrix; rows past n are identity rows.
__global__ void __launch_bounds__(256)
ss_form(const double* __restrict__ Y, long ldy, int n, const double* __restrict__ w,
        const double* __restrict__ Q, long ldq, int m, const double* __restrict__ tfix, double xs, double sigma,
        double* __restrict__ KF, long ldk, int np, double* __restrict__ R, long ldr, Scalars* sc) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const bool real = i < n;
  const double t = (real && tfix) ? tfix[i] : 0.0;
  const bool fixed = t > 0.0;
  const bool row = real && !fixed;
  const double* yrow = Y + static_cast<long>(i) * ldy;
  int bad = 0;
  double s = 0.0;
  if (row)
    for (long j = threadIdx.x; j <= n; j += blockDim.x) {
      const double v = yrow[j];
      bad |= !(v >= 0.0 && v <= 1.0e300);
      s += v;
    }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  s = (red[0] + red[1]) + (red[2] + red[3]);
  const double wi = real ? w[i] : 1.0;
  if (threadIdx.x == 0 && real) {
    bad |= !(wi > 0.0 && wi <= 1.0e300);
    bad |= !(t >= 0.0 && t <= 1.0e300);
  }
  double* krow = KF + static_cast<long>(i) * ldk;
  for (long j = threadIdx.x; j < ldk; j += blockDim.x) {
    double kv = (i == j) ? 1.0 : 0.0;
    if (row && j < n) {
      const double v = yrow[j];
      kv = (i == j) ? s - v : -v;
    }
    krow[j] = j < np ? kv : 0.0;
  }
  double* rrow = R + static_cast<long>(i) * ldr;
  const double ysp = row ? yrow[n] : 0.0;
  for (long c = threadIdx.x; c < ldr; c += blockDim.x) {
    double rv = 0.0;
    if (real && c < m) {
      if (fixed) {
        rv = (t * t) * (t * t);
      } else {
        const double qv = Q[static_cast<long>(i) * ldq + c];
        bad |= !(qv >= -1.0e300 && qv <= 1.0e300);
        rv = qv / (sigma * wi) + ysp * xs;
      }
    }
    rrow[c] = rv;
  }
  if (bad) raise_status(&sc->status, RAD_ENONFINITE);
}

// T = x^(1/4) for free nodes (x <= 0: no real temperature balances the
// given heat input, reported as RAD_ENONFINITE), the prescribed T otherwise.
__global__ void __launch_bounds__(256)
ss_output(const double* __restrict__ X, long ldx, int n, int m, const double* __restrict__ tfix,
          double* __restrict__ T, long ldt, Scalars* sc) {
  const long q = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= static_cast<long>(n) * m) return;
  const int i = static_cast<int>(q / m), c = static_cast<int>(q % m);
  const double tf = tfix ? tfix[i] : 0.0;
  double out = tf;
  if (!(tf > 0.0)) {
    const double x = X[static_cast<long>(i) * ldx + c];
    if (x > 0.0 && x <= 1.0e300) {
      out = sqrt(sqrt(x));
    } else {
      out = __builtin_nan("");
      raise_status(&sc->status, RAD_ENONFINITE);
    }
  }
  T[static_cast<long>(i) * ldt + c] = out;
}

// ---- least-squares optimum enforcer (eq. 3.41-3.52 with NNR / SPVA) ------
// The projection of F onto {closure rows sum to 1, W_i F_ik = W_k F_ki} over
// the active entries (a_ik = 1) is F_hat = F - A^T y with (A A^T) y = A F - b.
// A A^T has a diagonal closure block (n_i = active entries of row i), a
// diagonal reciprocity block (d_ik = W_i^2 a_ik + W_k^2 a_ki per pair) and a
// coupling with two entries per pair, so eliminating the pair multipliers
// leaves an n x n system for the closure multipliers lambda:
//   S_ii = n_i - sum_{k != i} a_ik W_i^2 / d_ik,  S_ik = a_ik a_ki W_i W_k / d_ik,
//   S lambda = (sum_j a_ij F_ij - 1) - sum_{k != i} a_ik W_i rho_ik / d_ik,
//   rho_ik = W_i a_ik F_ik - W_k a_ki F_ki;
// then F_hat_ik = F_ik - lambda_i - W_i nu_ik with the pair multiplier
//   nu_ik = (rho_ik - a_ik W_i lambda_i + a_ki W_k lambda_k) / d_ik
// (k != i, k < n), and F_hat_ik = F_ik - lambda_i on the diagonal and the
// space column.  A row with no active entry gets lambda_i = 0.

// mask (n x (n+1), ld n+1): 1 = active; SPVA drops the zeros of the input
__global__ void __launch_bounds__(256)
lsq_mask_init(const double* __restrict__ F, long ldf, int n, int spva, uint8_t* __restrict__ mask,
              Scalars* sc) {
  const int i = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k > n) return;
  const double v = F[static_cast<long>(i) * ldf + k];
  if (!(v >= -1.0e300 && v <= 1.0e300)) raise_status(&sc->status, RAD_ENONFINITE);
  mask[static_cast<long>(i) * (n + 1) + k] = (spva && v == 0.0) ? 0 : 1;
}

// Both kernels below take 16 rows i per workgroup and walk the columns k in
// chunks of 64: the rows' own entries F_ik and a_ik are read as contiguous
// 512-byte row pieces, and the partner entries F_ki, a_ki of the chunk (64
// rows of 16 contiguous entries each) are staged in LDS, so no access is
// strided.  Thread t works on rows w + 4j (w = t / 64, j = 0..3) of the block
// and column t % 64 of each chunk.
constexpr int LSQ_RB = 16;  // rows per workgroup
constexpr int LSQ_KC = 64;  // columns per chunk

// the chunk's partner entries F_ki, a_ki (k in [k0, k0 + 64), i in the block)
__device__ __forceinline__ void lsq_stage_partner(const double* __restrict__ F, long ldf,
                                                  const uint8_t* __restrict__ mask, long ldm, int n, int i0, int k0,
                                                  double (*pf)[LSQ_RB + 1], uint8_t (*pm)[LSQ_RB + 1]) {
#pragma unroll
  for (int q = 0; q < LSQ_KC * LSQ_RB / 256; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int kk = e / LSQ_RB, ii = e % LSQ_RB;
    const int k = k0 + kk, i = i0 + ii;
    const bool in = k < n && i < n;
    pf[kk][ii] = in ? F[static_cast<long>(k) * ldf + i] : 0.0;
    pm[kk][ii] = in ? mask[static_cast<long>(k) * ldm + i] : 0;
  }
}

__global__ void __launch_bounds__(256)
lsq_schur(const double* __restrict__ F, long ldf, int n, const double* __restrict__ W,
          const uint8_t* __restrict__ mask, double* __restrict__ KF, long ldk, int np,
          double* __restrict__ Y, long ldy) {
  __shared__ double pf[LSQ_KC][LSQ_RB + 1];
  __shared__ uint8_t pm[LSQ_KC][LSQ_RB + 1];
  const int i0 = blockIdx.x * LSQ_RB;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const long ldm = n + 1;
  double cnt[4], rsum[4], sub[4], tt[4], wi[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + w + 4 * j;
    cnt[j] = rsum[j] = sub[j] = tt[j] = 0.0;
    wi[j] = i < n ? W[i] : 0.0;
  }
  if (i0 < n) {
    for (int k0 = 0; k0 <= n; k0 += LSQ_KC) {
      // the rows' own entries of the chunk, loaded before the partner tile
      // so that both sets of loads are in flight together
      const int k = k0 + l;
      int am[4];
      double fv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = i0 + w + 4 * j;
        const bool in = i < n && k <= n;
        am[j] = in ? mask[static_cast<long>(i) * ldm + k] : 0;
        fv[j] = in ? F[static_cast<long>(i) * ldf + k] : 0.0;
      }
      __syncthreads();  // the previous chunk's partner reads are done
      lsq_stage_partner(F, ldf, mask, ldm, n, i0, k0, pf, pm);
      __syncthreads();
      if (k > n) continue;
      const double wk = k < n ? W[k] : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ii = w + 4 * j, i = i0 + ii;
        if (i >= n) continue;
        const int aik = am[j];
        const double fik = fv[j];
        cnt[j] += aik;
        rsum[j] += aik ? fik : 0.0;
        if (k < n && k != i) {
          double sik = 0.0;
          const int aki = pm[l][ii];
          const double d = wi[j] * wi[j] * aik + wk * wk * aki;
          if (d > 0.0) {
            const double rho = (aik ? wi[j] * fik : 0.0) - (aki ? wk * pf[l][ii] : 0.0);
            if (aik) {
              sub[j] += wi[j] * wi[j] / d;
              tt[j] += wi[j] * rho / d;
            }
            if (aik && aki) sik = wi[j] * wk / d;
          }
          KF[static_cast<long>(i) * ldk + k] = sik;
        }
      }
    }
  }
  // row sums over the 64 lanes of the wave (fixed order)
#pragma unroll
  for (int j = 0; j < 4; ++j)
    for (int off = 32; off > 0; off >>= 1) {
      cnt[j] += __shfl_xor(cnt[j], off);
      rsum[j] += __shfl_xor(rsum[j], off);
      sub[j] += __shfl_xor(sub[j], off);
      tt[j] += __shfl_xor(tt[j], off);
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + w + 4 * j;
    if (i >= np) continue;
    double* krow = KF + static_cast<long>(i) * ldk;
    double* yrow = Y + static_cast<long>(i) * ldy;
    if (i < n) {
      // the diagonal, the padding columns, and the right-hand side
      for (long k = n + l; k < ldk; k += 64) krow[k] = 0.0;
      if (l == 0) {
        krow[i] = cnt[j] > 0.0 ? cnt[j] - sub[j] : 1.0;
        yrow[0] = cnt[j] > 0.0 ? (rsum[j] - 1.0) - tt[j] : 0.0;
      }
      for (long c = 1 + l; c < ldy; c += 64) yrow[c] = 0.0;
    } else {
      // padding rows: identity
      for (long k = l; k < ldk; k += 64) krow[k] = k == i ? 1.0 : 0.0;
      for (long c = l; c < ldy; c += 64) yrow[c] = 0.0;
    }
  }
}

// F_hat from lambda (column 0 of Y); NNR: negative active entries leave the
// next round's mask; every entry of the mask is written (ping-pong buffers).
// One workgroup per 16 rows x one 64-column chunk (grid: chunks x row blocks).
__global__ void __launch_bounds__(256)
lsq_update(const double* __restrict__ F, long ldf, int n, const double* __restrict__ W,
           const uint8_t* __restrict__ mask, const double* __restrict__ Y, long ldy, int nnr,
           uint8_t* __restrict__ mask_next, double* __restrict__ Fo, long ldo, int* __restrict__ negatives) {
  __shared__ double pf[LSQ_KC][LSQ_RB + 1];
  __shared__ uint8_t pm[LSQ_KC][LSQ_RB + 1];
  __shared__ double yk[LSQ_KC];
  const int k0 = blockIdx.x * LSQ_KC, i0 = blockIdx.y * LSQ_RB;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const long ldm = n + 1;
  lsq_stage_partner(F, ldf, mask, ldm, n, i0, k0, pf, pm);
  if (t < LSQ_KC) yk[t] = k0 + t < n ? Y[static_cast<long>(k0 + t) * ldy] : 0.0;
  __syncthreads();
  const int k = k0 + l;
  int neg_count = 0;
  if (k <= n) {
    const double wk = k < n ? W[k] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ii = w + 4 * j, i = i0 + ii;
      if (i >= n) continue;
      const int aik = mask[static_cast<long>(i) * ldm + k];
      double v = 0.0;
      if (aik) {
        const double li = Y[static_cast<long>(i) * ldy];
        const double fik = F[static_cast<long>(i) * ldf + k];
        v = fik - li;
        if (k < n && k != i) {
          const int aki = pm[l][ii];
          const double wi = W[i];
          const double d = wi * wi + wk * wk * aki;
          const double fki = aki ? pf[l][ii] : 0.0;
          const double nu = ((wi * fik - wk * fki) - wi * li + (aki ? wk * yk[l] : 0.0)) / d;
          // a partner held at zero makes the pair's row read W_i F_ik = 0: exactly zero
          v = aki ? v - wi * nu : 0.0;
        }
      }
      const int neg = nnr && aik && v < 0.0;
      neg_count += neg;
      mask_next[static_cast<long>(i) * ldm + k] = aik && !neg;
      Fo[static_cast<long>(i) * ldo + k] = v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) neg_count += __shfl_xor(neg_count, off);
  if (l == 0 && neg_count > 0) atomicAdd(negatives, neg_count);
}

// P = F_sq diag(rho) in FP64, zero outside n x n (refinement residuals).
__global__ void __launch_bounds__(256)
form_p64(const double* __restrict__ F, long ldf, int n, const double* __restrict__ rho,
         double* __restrict__ P, long ldp) {
  const int i = blockIdx.x;
  for (long j = threadIdx.x; j < ldp; j += blockDim.x)
    P[static_cast<long>(i) * ldp + j] = (i < n && j < n) ? F[static_cast<long>(i) * ldf + j] * rho[j] : 0.0;
}

template <class T>
__global__ void __launch_bounds__(256) fill_zero(T* __restrict__ p, long count) {
  for (long q = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; q < count;
       q += static_cast<long>(gridDim.x) * blockDim.x)
    p[q] = T(0);
}

// Gauss-Jordan inverse of one NB x NB diagonal block, no pivoting, blocked by
// 16.  The block is held as 8 x 8 tiles of 16 x 16 in MFMA accumulator layout:
// wave w (of 4) owns tile rows 2w and 2w+1.  Step s takes
// the 16 x 16 pivot tile P = M(s,s) and applies
//   M(s,s) <- P^-1,   M(s,j) <- P^-1 M(s,j),   M(i,s) <- -M(i,s) P^-1,
//   M(i,j) <- M(i,j) - M(i,s) P^-1 M(s,j)                 (i, j != s),
// i.e. the scalar in-place Gauss-Jordan update with a 16 x 16 pivot; after
// the 8 steps M = A^-1.  P is inverted inside one wave by 16 scalar
// Gauss-Jordan steps with each lane holding four entries of one row (the
// pivot row's entries and the pivot column's entry are broadcast with lane
// shuffles, no barriers; 2.3x faster than one column per lane with lane
// reads, whose results had to pass through scalar registers); the row products (one tile column
// per wave) and the rank-16 updates run on the matrix cores, each wave
// loading its tile-row operand once per step and each tile-column operand
// once for all its tiles.  Two workgroup barriers per step.
// Diagonal dominance of K makes every pivot order stable, so no pivoting is
// needed; the scalar pivots are the same Schur-complement diagonals as in
// unblocked elimination and are checked against the singularity threshold.
constexpr int GJ_WAVES = 4;    // two tile rows per wave; at 254 VGPRs a wave fits on a SIMD beside one GEMM wave
constexpr int GJ_THREADS = 64 * GJ_WAVES;

// 1/x: hardware reciprocal refined by Newton steps to full precision
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}
__device__ __forceinline__ float recip_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return r * (2.0f - x * r);
}

// value of x in lane `lane` (uniform), broadcast to the wave
__device__ __forceinline__ double lane_read(double x, int lane) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(v), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ float lane_read(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// orders this wave's LDS writes before its later LDS reads
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T, int NW>
__device__ __forceinline__ void gj_body(const T* __restrict__ A, long lda, T* __restrict__ out, Scalars* sc) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int BT = 16;
  constexpr int NT = NB / BT;
  constexpr int RPW = NT / NW;        // tile rows per wave
  static_assert(RPW * NW == NT, "NW must divide 8");
  constexpr int LC = BT + 2;
  constexpr int LR = NB + 2;
  __shared__ T sC[2][NB][LC];
  __shared__ T sRo[BT][LR];
  __shared__ T sR[BT][LR];
  __shared__ T sP[BT][BT + 1];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int li = l & 15, lg = l >> 4;
  v4 m[RPW][NT];
#pragma unroll
  for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
    for (int bj = 0; bj < NT; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        m[rr][bj][r] = A[static_cast<long>((w * RPW + rr) * BT + Mfma<T>::orow(l, r)) * lda + bj * BT + li];
  const double tiny = sizeof(T) == 8 ? 1e-11 : 1e-5;
  int singular = 0;
#pragma unroll 1
  for (int s = 0; s < NT; ++s) {
    const int cb = s & 1;
    const int sw = s / RPW, srr = s % RPW;  // owner wave of tile row s, its local row
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int bi = w * RPW + rr;
#pragma unroll
      for (int bj = 0; bj < NT; ++bj) {
        if (bj == s)
#pragma unroll
          for (int r = 0; r < 4; ++r) sC[cb][bi * BT + Mfma<T>::orow(l, r)][li] = m[rr][bj][r];
        if (bi == s)
#pragma unroll
          for (int r = 0; r < 4; ++r) sRo[Mfma<T>::orow(l, r)][bj * BT + li] = m[rr][bj][r];
      }
    }
    if (w == sw) {
      wave_lds_sync();
      // lane (i, q4) = (l % 16, l / 16) holds P(i, 4 q4 .. 4 q4 + 3); each
      // scalar step broadcasts the pivot row's entries of the lane's four
      // columns and the pivot column's entry of its row with lane shuffles
      const int i = li, q4 = lg;
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = sRo[i][s * BT + 4 * q4 + u];
#pragma unroll
      for (int q = 0; q < BT; ++q) {
        const int qq = q >> 2, qu = q & 3;
        T r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = __shfl(v[u], q + 16 * q4);  // P(q, 4 q4 + u)
        const T pc = __shfl(v[qu], i + 16 * qq);                          // P(i, q)
        const T piv = lane_read(v[qu], q + 16 * qq);                      // P(q, q)
        T d = recip_nr(piv);
        if (!(fabs(static_cast<double>(piv)) > tiny) || !(fabs(static_cast<double>(d)) < 1e300)) {
          singular = 1;
          d = T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = 4 * q4 + u;
          const T rj = (j == q) ? d : r[u] * d;  // the new pivot row
          if (i == q) v[u] = rj;
          else v[u] = fma(-pc, rj, j == q ? T(0) : v[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) sP[i][4 * q4 + u] = v[u];
    }
    __syncthreads();
    // new tile row s, spread over the waves: R(s, j) = P^-1 Ro(s, j), R(s, s) = P^-1
    {
      T pa[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) pa[kk] = sP[li][4 * kk + lg];
#pragma unroll
      for (int jj = 0; jj < RPW; ++jj) {
        const int bj = w * RPW + jj;
        if (bj == s) {
#pragma unroll
          for (int r = 0; r < 4; ++r) sR[Mfma<T>::orow(l, r)][bj * BT + li] = sP[Mfma<T>::orow(l, r)][li];
        } else {
          v4 acc = v4{0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc = Mfma<T>::mma(pa[kk], sRo[4 * kk + lg][bj * BT + li], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) sR[Mfma<T>::orow(l, r)][bj * BT + li] = acc[r];
        }
      }
    }
    __syncthreads();
    // rank-16 update of the other tile rows; tile column s becomes -M(i,s) P^-1;
    // tile row s takes R(s, :)
    T av[RPW][4];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) av[rr][kk] = -sC[cb][(w * RPW + rr) * BT + li][4 * kk + lg];
#pragma unroll
    for (int bj = 0; bj < NT; ++bj) {
      T bv[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) bv[kk] = sR[4 * kk + lg][bj * BT + li];
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        if (w * RPW + rr == s) {
#pragma unroll
          for (int r = 0; r < 4; ++r) m[rr][bj][r] = sR[Mfma<T>::orow(l, r)][bj * BT + li];
          continue;
        }
        if (bj == s) m[rr][bj] = v4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) m[rr][bj] = Mfma<T>::mma(av[rr][kk], bv[kk], m[rr][bj]);
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
    for (int bj = 0; bj < NT; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[((w * RPW + rr) * BT + Mfma<T>::orow(l, r)) * NB + bj * BT + li] = m[rr][bj][r];
  if (singular) raise_status(&sc->status, RAD_ESINGULAR);
}
template <class T>
__global__ void __launch_bounds__(GJ_THREADS)
gj_inverse(const T* __restrict__ A, long lda, T* __restrict__ out, Scalars* sc) {
  gj_body<T, GJ_WAVES>(A, lda, out, sc);
}

// many diagonal blocks (of different problems) in one launch
template <class T>
struct GjJob {
  const T* A;
  long lda;
  T* out;
  Scalars* sc;
};

template <class T>
__global__ void __launch_bounds__(GJ_THREADS) gj_batched(const GjJob<T>* __restrict__ jobs) {
  const GjJob<T> jb = jobs[blockIdx.x];
  gj_body<T, GJ_WAVES>(jb.A, jb.lda, jb.out, jb.sc);
}

// ----------------------------------------------------- panel inverses ---
// W_p = U_pp^-1 and V_p = L_pp^-1 for every 1024-wide panel p by recursive
// doubling over its 128-wide diagonal blocks:
//   [A B; 0 C]^-1 = [A^-1, -A^-1 B C^-1; 0, C^-1],
//   [I 0; E I]^-1 = [I, 0; -E, I] generalised to [X 0; E Y]^-1 = [X^-1, 0; -Y^-1 E X^-1, Y^-1],
// starting from W's diagonal blocks D_k^-1 and V's identity blocks.  Level b
// joins pairs of b-wide inverses; each join is two MFMA products, run for all
// panels and pairs in one launch per stage.
template <class T>
struct TriJob {
  const T* kf;
  long ldk;
  const T* dinv;
  int np;
  T* W;
  T* V;
  long ldw;
  T* tmp;      // tri_tmp_elems scratch
  long ldt;
};

// W_p = blockdiag(D_k^-1), V_p = I (zero elsewhere, padded columns included);
// row r of the padded matrix (all panels stacked)
template <class T>
__device__ __forceinline__ void tri_init_row(const TriJob<T>& j, int r) {
  const int p = r / NB2, rl = r % NB2, kb = rl / NB;
  T* wr = j.W + (static_cast<long>(p) * NB2 + rl) * j.ldw;
  T* vr = j.V + (static_cast<long>(p) * NB2 + rl) * j.ldw;
  const T* drow = j.dinv + (static_cast<long>(r / NB) * NB + rl % NB) * NB;
  for (int c = threadIdx.x; c < j.ldw; c += blockDim.x) {
    wr[c] = (c / NB == kb && c < NB2) ? drow[c % NB] : T(0);
    vr[c] = (c == rl) ? T(1) : T(0);
  }
}

template <class T>
__global__ void __launch_bounds__(256) tri_init(TriJob<T> j) {
  tri_init_row<T>(j, blockIdx.x);
}

// Operands of one join at level b: panel p, pair q, matrix mat (0 W, 1 V),
// stage 0 (T = U12 W_bot, T = L21 V_top) or 1 (W12 = -W_top T,
// V21 = -V_bot T).  False when the pair has no bottom half.  Shared by the
// single-model kernel and the batch planner, so both compute identically.
template <class T>
__host__ __device__ inline bool tri_level_args(const TriJob<T>& j, int b, int stage, int p, int q, int mat,
                                               GemmArgs<T>& g) {
  const int nq = NB2 / (2 * b);
  const int c0 = p * NB2;
  const int L = j.np - c0 < NB2 ? j.np - c0 : NB2;
  const int o = 2 * b * q;
  if (o + b >= L) return false;
  const int bb = L - o - b < b ? L - o - b : b;
  T* Wp = j.W + static_cast<long>(p) * NB2 * j.ldw;
  T* Vp = j.V + static_cast<long>(p) * NB2 * j.ldw;
  T* tq = j.tmp + (static_cast<long>(p * nq + q) * 2 + mat) * b * j.ldt;
  const long ldw = j.ldw, ldk = j.ldk;
  g = GemmArgs<T>{};
  g.nseg = 1;
  g.beta = T(0);
  if (mat == 0) {
    if (stage == 0) {
      g.A = j.kf + static_cast<long>(c0 + o) * ldk + (c0 + o + b);
      g.lda = ldk; g.M = b; g.K = bb; g.alpha = T(1);
      g.B[0] = Wp + static_cast<long>(o + b) * ldw + (o + b); g.ldb[0] = ldw;
      g.C[0] = tq; g.ldc[0] = j.ldt; g.N[0] = bb;
    } else {
      g.A = Wp + static_cast<long>(o) * ldw + o;
      g.lda = ldw; g.M = b; g.K = b; g.alpha = T(-1);
      g.B[0] = tq; g.ldb[0] = j.ldt;
      g.C[0] = Wp + static_cast<long>(o) * ldw + (o + b); g.ldc[0] = ldw; g.N[0] = bb;
    }
  } else {
    if (stage == 0) {
      g.A = j.kf + static_cast<long>(c0 + o + b) * ldk + (c0 + o);
      g.lda = ldk; g.M = bb; g.K = b; g.alpha = T(1);
      g.B[0] = Vp + static_cast<long>(o) * ldw + o; g.ldb[0] = ldw;
      g.C[0] = tq; g.ldc[0] = j.ldt; g.N[0] = b;
    } else {
      g.A = Vp + static_cast<long>(o + b) * ldw + (o + b);
      g.lda = ldw; g.M = bb; g.K = bb; g.alpha = T(-1);
      g.B[0] = tq; g.ldb[0] = j.ldt;
      g.C[0] = Vp + static_cast<long>(o + b) * ldw + o; g.ldc[0] = ldw; g.N[0] = b;
    }
  }
  g.ntile[0] = (g.N[0] + GEMM_TILE - 1) / GEMM_TILE;
  g.ntile[1] = 0;
  return true;
}

// Grid: panels x pairs x 2 matrices x (b/64)^2 tiles of 64 x 64 (the joins
// are short latency-bound products, so the smaller tile spreads them over
// four times the CUs).
constexpr int TRI_TS = 64;
template <class T>
__global__ void __launch_bounds__(256, 4) tri_level(TriJob<T> j, int b, int stage) {
  const int tpg = (b / TRI_TS) * (b / TRI_TS);
  const int nq = NB2 / (2 * b);
  int blk = blockIdx.x;
  const int tile = blk % tpg;
  blk /= tpg;
  const int mat = blk % 2;
  blk /= 2;
  GemmArgs<T> g;
  if (!tri_level_args<T>(j, b, stage, blk / nq, blk % nq, mat, g)) return;
  const int ntx = (g.N[0] + TRI_TS - 1) / TRI_TS, nty = (g.M + TRI_TS - 1) / TRI_TS;
  if (tile >= ntx * nty) return;
  gemm_tile<T, false, TRI_TS>(g, tile % ntx, tile / ntx);
}

inline unsigned tri_level_blocks(int P2, int b) {
  return static_cast<unsigned>(P2) * (NB2 / (2 * b)) * 2 * (b / TRI_TS) * (b / TRI_TS);
}

// dst rows [0, rows) <- src, columns < cols (same precision)
template <class T>
__global__ void __launch_bounds__(256)
copy_rows(const T* __restrict__ src, long lds, T* __restrict__ dst, long ldd, int cols) {
  const long i = blockIdx.x;
  // eight loads per thread in flight (addresses clamped into the row)
  for (int j0 = threadIdx.x; j0 < cols; j0 += 8 * blockDim.x) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[i * lds + min(j0 + u * static_cast<int>(blockDim.x), cols - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * static_cast<int>(blockDim.x);
      if (j < cols) dst[i * ldd + j] = v[u];
    }
  }
}

// dst rows [0, rows) <- src, NB columns; 16 rows per workgroup, each thread
// 8 consecutive entries
template <class T>
__global__ void __launch_bounds__(256)
copy_nb_cols(const T* __restrict__ src, long lds, T* __restrict__ dst, long ldd, int rows) {
  const long r = static_cast<long>(blockIdx.x) * 16 + (threadIdx.x >> 4);
  if (r >= rows) return;
  const int c = (threadIdx.x & 15) * (NB / 16);
#pragma unroll
  for (int j = 0; j < NB / 16; ++j) dst[r * ldd + c + j] = src[r * lds + c + j];
}

// dst (D, rows < n, cols <= n) <- src (S)
template <class S, class D>
__global__ void __launch_bounds__(256)
copy_block(const S* __restrict__ src, long lds, int n, D* __restrict__ dst, long ldd) {
  const int i = blockIdx.x;
  for (int j0 = threadIdx.x; j0 <= n; j0 += 8 * blockDim.x) {  // eight loads per thread in flight
    S v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[static_cast<long>(i) * lds + min(j0 + u * static_cast<int>(blockDim.x), n)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * static_cast<int>(blockDim.x);
      if (j <= n) dst[static_cast<long>(i) * ldd + j] = static_cast<D>(v[u]);
    }
  }
}

// max of v over a 256-thread block, merged into *target with one atomic per
// block (every thread of the block must call it)
__device__ inline void block_max(double v, double* target) {
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomic_max_nonneg(target, fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

// R = E - X  (rows < n, cols <= n), E from F and eps on the fly
__global__ void __launch_bounds__(256)
residual_init(const double* __restrict__ F, long ldf, int n, const double* __restrict__ eps,
              const double* __restrict__ X, long ldx, double* __restrict__ R, long ldr) {
  const int i = blockIdx.x;
  const double* f = F + static_cast<long>(i) * ldf;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) {
    double e = (j < n) ? f[j] * eps[j] : f[n];
    R[static_cast<long>(i) * ldr + j] = e - X[static_cast<long>(i) * ldx + j];
  }
}

// R = G - L  (rows < n, cols <= n)
__global__ void __launch_bounds__(256)
adj_residual_init(const double* __restrict__ G, long ldg, int n, const double* __restrict__ L, long ldl,
                  double* __restrict__ R, long ldr) {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j <= n; j += blockDim.x)
    R[static_cast<long>(i) * ldr + j] = G[static_cast<long>(i) * ldg + j] - L[static_cast<long>(i) * ldl + j];
}

// Y32 <- R (rows < n, cols <= n), records max |R|
__global__ void __launch_bounds__(256)
residual_to_rhs(const double* __restrict__ R, long ldr, int n, float* __restrict__ Y, long ldy,
                Scalars* sc) {
  const int i = blockIdx.x;
  double m = 0.0;
  int bad = 0;
  for (int j = threadIdx.x; j <= n; j += blockDim.x) {
    double v = R[static_cast<long>(i) * ldr + j];
    bad |= !(fabs(v) <= 1.0e300);
    m = fmax(m, fabs(v));
    Y[static_cast<long>(i) * ldy + j] = static_cast<float>(v);
  }
  if (bad) raise_status(&sc->status, RAD_ENONFINITE);
  block_max(m, &sc->max_r);
}

// X += Y32 (rows < n, cols <= n), records max |delta|
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

// Y (T, np rows x ldy, zero outside n x (n+1)) <- G (fp64); a non-finite
// entry of G raises RAD_ENONFINITE
template <class T>
__global__ void __launch_bounds__(256)
load_rhs(const double* __restrict__ G, long ldg, int n, T* __restrict__ Y, long ldy, Scalars* sc) {
  const int i = blockIdx.x;
  T* y = Y + static_cast<long>(i) * ldy;
  int bad = 0;
  // eight loads per thread in flight: addresses clamped into G, entries
  // outside its n x (n + 1) range replaced by zero afterwards
  const long gi = static_cast<long>(min(i, n - 1)) * ldg;
  for (long j0 = threadIdx.x; j0 < ldy; j0 += 8 * blockDim.x) {
    double g[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) g[u] = G[gi + min(j0 + u * static_cast<long>(blockDim.x), static_cast<long>(n))];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long j = j0 + u * static_cast<long>(blockDim.x);
      if (j >= ldy) break;
      const bool in = j <= n && i < n;
      const double v = __builtin_unpredictable(in) ? g[u] : 0.0;
      bad |= in && !(fabs(v) <= 1.0e300);
      y[j] = static_cast<T>(v);
    }
  }
  if (bad) raise_status(&sc->status, RAD_ENONFINITE);
}


// REF closure residual: one wave per row sums the n+1 entries; the block's
// maximum of |s_i - 1| goes to blk[blockIdx.x] (no same-address atomics).
__global__ void __launch_bounds__(256)
ref_closure(const double* __restrict__ B, long ldb, int n, double* __restrict__ blk) {
  __shared__ double red[4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  double s = 0.0;
  if (row < n) {
    const double* __restrict__ b = B + static_cast<long>(row) * ldb;
    for (int j = l; j <= n; j += 64) s += b[j];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (l == 0) red[w] = (row < n) ? fabs(s - 1.0) : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// REF reciprocity residual max |eps_i A_i B_ij - eps_j A_j B_ji| (eq. 4.4):
// one workgroup per 64 x 64 tile pair (I, J), I <= J; the partner tile goes
// through LDS so both are read as rows; the pair's maximum goes to blk[pair].
__global__ void __launch_bounds__(256)
ref_reciprocity(const double* __restrict__ B, long ldb, int n, int t, const double* __restrict__ eps,
                const double* __restrict__ area, double* __restrict__ blk) {
  __shared__ double sT[64][65];
  __shared__ double wI[64], wJ[64];
  __shared__ double red[4];
  int I, J;
  pair_from_index(blockIdx.x, t, I, J);
  const int tid = threadIdx.x, c = tid & 63, rg = tid >> 6;
  if (tid < 64) {
    const int i = I * 64 + tid;
    wI[tid] = i < n ? eps[i] * area[i] : 0.0;
  } else if (tid < 128) {
    const int j = J * 64 + tid - 64;
    wJ[tid - 64] = j < n ? eps[j] * area[j] : 0.0;
  }
  double v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {  // partner tile (J, I)
    const int i = J * 64 + rg + 4 * m, j = I * 64 + c;
    v[m] = (i < n && j < n) ? B[static_cast<long>(i) * ldb + j] : 0.0;
  }
  double u[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {  // own tile (I, J)
    const int i = I * 64 + rg + 4 * m, j = J * 64 + c;
    u[m] = (i < n && j < n) ? B[static_cast<long>(i) * ldb + j] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) sT[rg + 4 * m][c] = wJ[rg + 4 * m] * v[m];
  __syncthreads();
  double mx = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int r = rg + 4 * m;
    mx = fmax(mx, fabs(wI[r] * u[m] - sT[c][r]));
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (c == 0) red[rg] = mx;
  __syncthreads();
  if (tid == 0) blk[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// out[0] = max of the closure block maxima, out[1] = of the reciprocity ones
__global__ void __launch_bounds__(256)
ref_final(const double* __restrict__ bc, int nc, const double* __restrict__ br, long nr, double* __restrict__ out) {
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nc; q += 256) a = fmax(a, bc[q]);
  for (long q = threadIdx.x; q < nr; q += 256) b = fmax(b, br[q]);
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off));
    b = fmax(b, __shfl_xor(b, off));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
    out[1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
  }
}

// grad_eps[k] = sum_i Lambda_ik F_ik: partial sums over row chunks of 128,
// then a fixed-order sum of the partials (reproducible).
constexpr int GE_ROWS = 128;
__global__ void __launch_bounds__(256)
adj_grad_eps_partial(const double* __restrict__ L, long ldl, const double* __restrict__ F, long ldf,
                     int n, double* __restrict__ part) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= n) return;
  const int i0 = c * GE_ROWS, i1 = min(n, i0 + GE_ROWS);
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += L[static_cast<long>(i) * ldl + k] * F[static_cast<long>(i) * ldf + k];
  part[static_cast<long>(c) * n + k] = s;
}

__global__ void __launch_bounds__(256)
adj_grad_eps_final(const double* __restrict__ part, int n, int chunks, double* __restrict__ ge) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[static_cast<long>(c) * n + k];
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

}  // namespace
}  // namespace rad
