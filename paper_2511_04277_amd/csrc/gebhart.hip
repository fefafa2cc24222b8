// Open-system Gebhart REF solve (thesis App. B.2, eq. B.6-B.11) and its
// adjoint on gfx950.
//
//   K = I - F_sq diag(rho),  E = [F_sq diag(eps) | F_space],  B = K^{-1} E.
//
// K is strictly diagonally dominant by rows (sum_k rho_k F_ik <= max rho < 1),
// so block Gaussian elimination needs no pivoting and every Schur complement
// stays dominant.  The factorization is a block LDU with 128 x 128 blocks that
// never splits a diagonal block:  for block k,
//   D_k^{-1}        Gauss-Jordan inverse of the diagonal block (one workgroup)
//   X  = A21 D^{-1} (block column of L, in place)
//   A22 -= X A12,   Y2 -= X Y1    (trailing matrix and the n+1 right-hand sides)
// so K = L U with L block-unit-lower (blocks X) and U block-upper (diagonal
// blocks D_k, off-diagonal blocks A12); the forward substitution of E rides
// along with the elimination.  The updates are organised in two levels: inside
// a 1024-wide panel the 128-wide blocks update only the panel (and the panel's
// own rows to its right), and the rest of the matrix receives one K = 1024 MFMA
// GEMM per panel, which keeps the FP64/FP32 matrix cores busy instead of
// streaming the trailing matrix once per 128 columns.  Back substitution and
// the transposed (adjoint) solves use the same two-level order.
//
// All GEMM operands are the solver's own buffers, padded to multiples of 128
// rows / columns (K with identity blocks, right-hand sides and the refinement
// operands with zeros), so the MFMA kernel reads unpredicated tiles and only
// masks its stores; results are copied to the caller's arrays at the end.
//
// RAD_PREC_FP32_IR runs the factorization and solves in FP32 MFMA, then
// refines in FP64:  R = E - K X = (E - X) + P X with P = F_sq diag(rho) (FP64
// MFMA GEMM), delta = K^{-1} R with the FP32 factors, X += delta.
//
// RAD_PREC_FP64_I8 keeps FP64 factors and the FP64 chain, but the products
// with K = panel width (the trailing update and forward substitution of each
// panel, the back substitution's and the transposed solves' updates) run as
// exact int8 digit products on the int8 matrix cores (emu_kernels.h,
// emu_split.h): each operand is scaled per row and split into 7 digits of 7
// bits, and the digit products are accumulated in FP64.
//
// Adjoint: K^T = U^T L^T, so Lambda = K^{-T} G is a block forward solve with
// U^T (diagonal blocks D_k^{-T}) followed by a block backward solve with L^T,
// both reusing the stored factors through transposed-A GEMMs; in FP32_IR mode
// the residual G - K^T Lambda = (G - Lambda) + P^T Lambda is formed in FP64.
#include <type_traits>

#include "emu_split.h"
#include "gebhart_kernels.h"

namespace rad {
namespace {

// ---------------------------------------------------------------- drivers ---
#define RAD_GEMM(args, trans)                                  \
  do {                                                         \
    hipError_t _e = launch_gemm((args), (trans), s);           \
    if (_e != hipSuccess) return _e;                           \
  } while (0)

// Y[r_dst..) -= op(A) * Y[r_src..] (+ optional second segment), small helper
template <class T>
inline GemmArgs<T> update_args(const T* A, long lda, int M, int K) {
  return gemm_args<T>(A, lda, M, K, T(-1), T(1));
}

// Digit buffers of the int8-emulated products (RAD_PREC_FP64_I8).  One set
// serves every product of a solve.  The products run on the caller's stream
// except the side-stream part of a factorization panel's update, which the
// next panel joins before it prepares its own operands; operand splits that
// do not depend on the chain run on the side stream, ordered by events after
// the last product that read the buffer they overwrite.
struct EmuWork {
  int8_t* da;  // digits of op(A)
  int8_t* db;  // digits of B^T
  int* xa;     // scale exponents of the rows of op(A)
  int* xb;     // scale exponents of the columns of B
  int* pa;     // per-k-block exponents of op(A) when its rows are not k-contiguous
  int* pb;     // per-k-block exponents of B's columns
};

// Scale exponents and digits of op(A) (if oa) and of B's row tiles
// [bt0, bt1) (if ob; bt1 < 0: to the end), on stream s.
inline hipError_t emu_split_ops(const EmuWork& e, const EmuOperand* oa, bool akc, const EmuOperand* ob, int bt0,
                                int bt1, hipStream_t s) {
  double elems = 0.0;
  if (oa) elems += static_cast<double>(oa->R) * oa->K;
  if (ob) {
    const int T = (ob->R + EMU_TILE - 1) / EMU_TILE, t1 = bt1 < 0 ? T : std::min(bt1, T);
    elems += std::max(0.0, std::min(static_cast<double>(ob->R), t1 * static_cast<double>(EMU_TILE)) -
                               bt0 * static_cast<double>(EMU_TILE)) * ob->K;
  }
  ProfScope prof(s, RAD_PROF_I8X_SPLIT, 0.0, (8.0 + EMU_S) * elems);
  // the buffers hold operands of K <= NB2 (one panel)
  if (oa) {
    if (oa->K > NB2) return hipErrorInvalidValue;
    hipError_t err = emu_prepare(*oa, akc, e.da, e.xa, e.pa, s);
    if (err != hipSuccess) return err;
  }
  if (ob) {
    if (ob->K > NB2) return hipErrorInvalidValue;
    return emu_prepare(*ob, false, e.db, e.xb, e.pb, s, bt0, bt1);
  }
  return hipSuccess;
}

// Launch arguments for all tiles of C -= op(A) B (callers narrow them).
// C(i, j) is C0[i ldc0 + j] for j < N0 and C1[i ldc1 + j - N0] after.
inline EmuGemmArgs emu_args(const EmuWork& e, const EmuOperand& oa, const EmuOperand& ob, int M, int N0,
                            double* C0, long ldc0, int N1 = 0, double* C1 = nullptr, long ldc1 = 0) {
  const int mt = (oa.R + EMU_TILE - 1) / EMU_TILE, nt = (ob.R + EMU_TILE - 1) / EMU_TILE;
  return EmuGemmArgs{e.da, e.xa, e.db, e.xb, mt, nt, (oa.K + EMU_KB - 1) / EMU_KB, 0, mt, 0, nt, M, -1.0,
                     N1 > 0 ? 2 : 1, {N0, N1}, {C0, C1}, {ldc0, ldc1}};
}

inline hipError_t emu_run(const EmuGemmArgs& g, int K, hipStream_t s) {
  const double rows = std::max(0, std::min(g.M, (g.ty0 + g.nty) * EMU_TILE) - g.ty0 * EMU_TILE);
  const double cols = std::max(0, std::min(g.N[0] + (g.nseg > 1 ? g.N[1] : 0), (g.tx0 + g.ntx) * EMU_TILE) -
                                      g.tx0 * EMU_TILE);
  // algorithmic bytes: C read and written, the digits of both operands read once
  ProfScope prof(s, RAD_PROF_GEMM_I8X, 2.0 * rows * cols * K, 16.0 * rows * cols + EMU_S * (rows + cols) * K);
  return emu_launch(g, s);
}

inline EmuOperand emu_operand(const double* X, long sr, long sk, int R, int K, const double* X1 = nullptr,
                              long sr1 = 0, long sk1 = 0, int R1 = 0) {
  return EmuOperand{{X, X1}, {sr, sr1}, {sk, sk1}, R, R + R1, K};
}

// Step (3) of a factorization panel with int8-emulated products: the panel's
// L block (rows c1.., columns c0..c1) and its U block together with the
// right-hand-side rows (rows c0..c1, columns c1.. of K then of Y) are split
// once - L and the next panel's columns of U on s, the rest of U and the
// right-hand sides on s2 while s updates the next panel's columns; the rest
// is updated on s2 in row chunks, with the same events as the FP64 path.
hipError_t factor_update_emu(const EmuWork& ew, const Fact<double>& f, int c0, int c1, int c2, double* Y, long ldy,
                             int wy, hipStream_t s, hipStream_t s2, SideStream* ss) {
  const long ldk = f.ldk;
  double* kf = f.kf;
  const int M = f.np - c1, K = c1 - c0, wyy = Y ? wy : 0;
  EmuOperand oa = emu_operand(kf + static_cast<long>(c1) * ldk + c0, ldk, 1, M, K);
  EmuOperand ob = emu_operand(kf + static_cast<long>(c0) * ldk + c1, 1, ldk, M, K,
                              Y ? Y + static_cast<long>(c0) * ldy : nullptr, 1, ldy, wyy);
  const int tx_next = (c2 - c1) / EMU_TILE;  // the next panel's column tiles
  hipError_t e = emu_split_ops(ew, &oa, true, &ob, 0, tx_next, s);
  if (e != hipSuccess) return e;
  if (s2 != s) {  // s2's earlier reads of the buffers were joined into s before this step
    e = stream_wait(s2, s, ss->ev[4]);
    if (e != hipSuccess) return e;
  }
  e = emu_split_ops(ew, nullptr, false, &ob, tx_next, -1, s2);
  if (e != hipSuccess) return e;
  const EmuGemmArgs g = emu_args(ew, oa, ob, M, M, kf + static_cast<long>(c1) * ldk + c1, ldk, wyy,
                                 Y ? Y + static_cast<long>(c1) * ldy : nullptr, ldy);
  EmuGemmArgs u = g;
  u.ntx = tx_next;
  e = emu_run(u, K, s);
  if (e != hipSuccess) return e;
  e = stream_wait(s2, s, ss->ev[2]);
  if (e != hipSuccess) return e;
  EmuGemmArgs v = g;
  v.tx0 = tx_next;
  v.ntx = g.nt - tx_next;
  if (v.ntx <= 0) return hipEventRecord(ss->ev[3], s2);
  // row chunks as in the FP64 path (the tuned count is in 128 x 128 tiles)
  int rows = M;
  const int chunk_tiles = gemm_tuning().side_chunk_tiles;
  if (chunk_tiles > 0 && s2 != s) {
    const int tx = (v.ntx * EMU_TILE + GEMM_TILE - 1) / GEMM_TILE;
    rows = std::max(1, chunk_tiles / std::max(1, tx)) * GEMM_TILE;
  }
  bool marked = false;
  for (int r0 = 0; r0 < M; r0 += rows) {
    EmuGemmArgs vc = v;
    vc.ty0 = r0 / EMU_TILE;
    vc.nty = (std::min(rows, M - r0) + EMU_TILE - 1) / EMU_TILE;
    e = emu_run(vc, K, s2);
    if (e != hipSuccess) return e;
    if (!marked && r0 + rows >= std::min(NB2, M)) {
      e = hipEventRecord(ss->ev[3], s2);
      if (e != hipSuccess) return e;
      marked = true;
    }
  }
  return hipSuccess;
}

// LDU factorization of K in place; Y (if given, n+1 columns) is eliminated too.
//
// Look-ahead: the update of panel p's trailing matrix is split.  Its first
// 1024 columns (panel p+1) are updated on the caller's stream s, so panel
// p+1's chain of diagonal inverses and narrow updates can start at once; the
// rest of the trailing matrix and the right-hand sides are updated on the
// side stream s2 meanwhile.  Panel p+1's row-block forward substitution waits
// for that part (event), and the call joins s2 back into s at the end.  The
// arithmetic and its order per element are the same as without the split.
//
// xs (nullable, np x NB elements): scratch for the L-block products
// X = A21 D^-1.  With it they are written out of place and copied back, so
// they take 64 x 64 tiles (two column tiles per row block, four times the
// workgroups of the in-place 128 x 128 form) on the chain of diagonal blocks;
// both forms round identically.
template <class T>
hipError_t factor_forward(const Fact<T>& f, T* Y, long ldy, int wy, Scalars* sc, hipStream_t s,
                          const EmuWork* ew = nullptr, T* xs = nullptr) {
  const long ldk = f.ldk;
  T* kf = f.kf;
  SideStream* ss = nullptr;
  hipError_t e = side_stream(&ss);
  if (e != hipSuccess) return e;
  // without look-ahead the far updates stay on s (the event waits are then no-ops)
  hipStream_t s2 = lookahead_enabled() ? ss->s2 : s;
  e = stream_wait(s2, s, ss->ev[0]);  // s2 starts after the caller's earlier work
  if (e != hipSuccess) return e;
  for (int c0 = 0; c0 < f.np; c0 += NB2) {
    const int c1 = std::min(c0 + NB2, f.np);
    const int c2 = std::min(c1 + NB2, f.np);
    // (1) panel: 128-wide blocks; updates stay inside the panel's columns
    for (int k0 = c0; k0 < c1; k0 += NB) {
      T* dk = f.dinv + static_cast<long>(k0) * NB;
      {
        ProfScope prof(s, RAD_PROF_DIAG_INVERSE, 2.0 * NB * NB * NB, 0.0);
        hipLaunchKernelGGL(gj_inverse<T>, dim3(1), dim3(GJ_THREADS), 0, s,
                           kf + static_cast<long>(k0) * ldk + k0, ldk, dk, sc);
      }
      const int r1 = k0 + NB;
      if (r1 >= f.np) break;
      T* x = kf + static_cast<long>(r1) * ldk + k0;
      GemmArgs<T> a = gemm_args<T>(x, ldk, f.np - r1, NB, T(1), T(0));
      if (xs) {
        gemm_add_segment<T>(a, dk, NB, xs, NB, NB);
        RAD_GEMM(a, false);
        hipLaunchKernelGGL(copy_nb_cols<T>, dim3(static_cast<unsigned>(ceil_div(f.np - r1, 16))), dim3(256), 0, s,
                           xs, static_cast<long>(NB), x, ldk, f.np - r1);
      } else {
        gemm_add_segment<T>(a, dk, NB, x, ldk, NB);
        a.inplace = 1;  // X overwrites the A21 it reads
        RAD_GEMM(a, false);
      }
      if (r1 < c1) {
        GemmArgs<T> u = update_args<T>(x, ldk, f.np - r1, NB);
        gemm_add_segment<T>(u, kf + static_cast<long>(k0) * ldk + r1, ldk, kf + static_cast<long>(r1) * ldk + r1,
                            ldk, c1 - r1);
        RAD_GEMM(u, false);
      }
    }
    // the previous panel's far update must have reached this panel's rows
    // before they are eliminated (its first row chunks; event ev[3])
    if (c0 > 0) {
      e = hipStreamWaitEvent(s, ss->ev[3], 0);
      if (e != hipSuccess) return e;
    }
    // (2) the panel's rows to the right of the panel: block forward substitution
    for (int k0 = c0; k0 + NB < c1; k0 += NB) {
      const int r1 = k0 + NB;
      GemmArgs<T> u = update_args<T>(kf + static_cast<long>(r1) * ldk + k0, ldk, c1 - r1, NB);
      if (c1 < f.np)
        gemm_add_segment<T>(u, kf + static_cast<long>(k0) * ldk + c1, ldk, kf + static_cast<long>(r1) * ldk + c1,
                            ldk, f.np - c1);
      if (Y) gemm_add_segment<T>(u, Y + static_cast<long>(k0) * ldy, ldy, Y + static_cast<long>(r1) * ldy, ldy, wy);
      if (u.nseg) RAD_GEMM(u, false);
    }
    // the rest of the previous panel's far update must be done before the
    // next panel's columns take this panel's update
    if (c0 > 0) {
      e = stream_wait(s, s2, ss->ev[1]);
      if (e != hipSuccess) return e;
    }
    // (3) everything below and right of the panel: K = panel-width GEMMs,
    // the next panel's columns on s, the rest on s2
    if (c1 < f.np && ew) {
      if constexpr (std::is_same<T, double>::value) {
        e = factor_update_emu(*ew, f, c0, c1, c2, Y, ldy, wy, s, s2, ss);
        if (e != hipSuccess) return e;
      }
    } else if (c1 < f.np) {
      GemmArgs<T> u = update_args<T>(kf + static_cast<long>(c1) * ldk + c0, ldk, f.np - c1, c1 - c0);
      gemm_add_segment<T>(u, kf + static_cast<long>(c0) * ldk + c1, ldk, kf + static_cast<long>(c1) * ldk + c1,
                          ldk, c2 - c1);
      RAD_GEMM(u, false);
      e = stream_wait(s2, s, ss->ev[2]);
      if (e != hipSuccess) return e;
      GemmArgs<T> v = update_args<T>(kf + static_cast<long>(c1) * ldk + c0, ldk, f.np - c1, c1 - c0);
      if (c2 < f.np)
        gemm_add_segment<T>(v, kf + static_cast<long>(c0) * ldk + c2, ldk, kf + static_cast<long>(c1) * ldk + c2,
                            ldk, f.np - c2);
      if (Y) gemm_add_segment<T>(v, Y + static_cast<long>(c0) * ldy, ldy, Y + static_cast<long>(c1) * ldy, ldy, wy);
      if (v.nseg) {
        // optionally in row chunks: a launch of s is dispatched only after
        // the grid ahead of it on the other stream has been dispatched whole
        int rows = f.np - c1;
        const int chunk_tiles = gemm_tuning().side_chunk_tiles;
        if (chunk_tiles > 0 && s2 != s) {
          const int tx = gemm_tiles<T>(v) / ((v.M + GEMM_TILE - 1) / GEMM_TILE);  // column tiles
          rows = std::max(1, chunk_tiles / std::max(1, tx)) * GEMM_TILE;
        }
        bool marked = false;
        for (int r0 = 0; r0 < v.M; r0 += rows) {
          GemmArgs<T> vc = v;
          vc.A = v.A + static_cast<long>(r0) * ldk;
          vc.M = std::min(rows, v.M - r0);
          for (int q = 0; q < vc.nseg; ++q) vc.C[q] = v.C[q] + static_cast<long>(r0) * v.ldc[q];
          hipError_t ge = launch_gemm(vc, false, s2);
          if (ge != hipSuccess) return ge;
          // the next panel's rows (the first NB2 rows) are done: its forward
          // substitution may start while the rest is updated
          if (!marked && r0 + vc.M >= std::min(NB2, v.M)) {
            ge = hipEventRecord(ss->ev[3], s2);
            if (ge != hipSuccess) return ge;
            marked = true;
          }
        }
      }
      if (!v.nseg) {  // nothing beyond the next panel: its rows are ready once s2 is
        e = hipEventRecord(ss->ev[3], s2);
        if (e != hipSuccess) return e;
      }
    }
  }
  e = stream_wait(s, s2, ss->ev[1]);  // join
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// Y <- L^{-1} Y with the stored factors (refinement right-hand sides).
template <class T>
hipError_t forward_only(const Fact<T>& f, T* Y, long ldy, int wy, hipStream_t s) {
  const long ldk = f.ldk;
  for (int c0 = 0; c0 < f.np; c0 += NB2) {
    const int c1 = std::min(c0 + NB2, f.np);
    for (int k0 = c0; k0 + NB < c1; k0 += NB) {
      const int r1 = k0 + NB;
      GemmArgs<T> u = update_args<T>(f.kf + static_cast<long>(r1) * ldk + k0, ldk, c1 - r1, NB);
      gemm_add_segment<T>(u, Y + static_cast<long>(k0) * ldy, ldy, Y + static_cast<long>(r1) * ldy, ldy, wy);
      RAD_GEMM(u, false);
    }
    if (c1 < f.np) {
      GemmArgs<T> u = update_args<T>(f.kf + static_cast<long>(c1) * ldk + c0, ldk, f.np - c1, c1 - c0);
      gemm_add_segment<T>(u, Y + static_cast<long>(c0) * ldy, ldy, Y + static_cast<long>(c1) * ldy, ldy, wy);
      RAD_GEMM(u, false);
    }
  }
  return hipSuccess;
}

// W_p = U_pp^-1 and V_p = L_pp^-1 of every panel (seven launches).
template <class T>
hipError_t panel_inverses(const Fact<T>& f, T* tmp, long ldt, hipStream_t s) {
  TriJob<T> j{f.kf, f.ldk, f.dinv, f.np, f.W, f.V, f.ldw, tmp, ldt};
  hipLaunchKernelGGL(tri_init<T>, dim3(f.np), dim3(256), 0, s, j);
  for (int b = NB; b < NB2; b *= 2)
    for (int stage = 0; stage < 2; ++stage)
      hipLaunchKernelGGL(tri_level<T>, dim3(tri_level_blocks(f.P2, b)), dim3(256), 0, s, j, b, stage);
  return hipGetLastError();
}

// Panel products of the back and transposed solves.  Y_p <- op(M_p) Y_p goes
// through one of two scratch panels S[0], S[1] (alternating); the update of
// the other rows reads the product straight from the scratch, and the copy
// back into Y_p runs on the side stream, off the chain of products and
// updates.  Before a scratch panel is overwritten, s waits for the side
// stream's latest copy (issued a whole update earlier, so long finished).
template <class T>
struct PanelSweep {
  T* S[2];
  long lds;
  hipStream_t s, s2;
  SideStream* ss;
  int idx = 0;
  T* cur = nullptr;

  hipError_t init(T* scr, long ld, hipStream_t st) {
    S[0] = scr;
    S[1] = scr + static_cast<long>(NB2) * ld;
    lds = ld;
    s = st;
    hipError_t e = side_stream(&ss);
    if (e != hipSuccess) return e;
    s2 = lookahead_enabled() ? ss->s2 : s;
    return hipSuccess;
  }
  // product of panel rows c0..c0+L into the next scratch panel; returns it in cur
  hipError_t product(const T* Mp, long ldm, bool trans, int tri, int c0, int L, const T* Y, long ldy, int wy) {
    if (idx >= 2) {
      hipError_t e = hipStreamWaitEvent(s, ss->ev[1], 0);
      if (e != hipSuccess) return e;
    }
    cur = S[idx & 1];
    ++idx;
    GemmArgs<T> a = gemm_args<T>(Mp, ldm, L, L, T(1), T(0));
    a.tri = tri;
    gemm_add_segment<T>(a, Y + static_cast<long>(c0) * ldy, ldy, cur, lds, wy);
    return launch_gemm(a, trans, s);
  }
  // copy of the current product into Y_p, on the side stream
  hipError_t copy_back(int c0, int L, T* Y, long ldy, int wy) {
    hipError_t e = stream_wait(s2, s, ss->ev[0]);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(copy_rows<T>, dim3(L), dim3(256), 0, s2, cur, lds, Y + static_cast<long>(c0) * ldy, ldy, wy);
    return hipEventRecord(ss->ev[1], s2);
  }
  hipError_t join() { return stream_wait(s, s2, ss->ev[2]); }
};

// The factor operand of a panel's emulated update in the back and transposed
// solves does not depend on the sweep: it is split on the side stream once
// the previous update (the last reader of the digit buffer) has run, while
// the caller's stream forms the panel's product.
hipError_t emu_presplit(const EmuWork& ew, const EmuOperand& oa, bool akc, PanelSweep<double>& ps, bool* ready) {
  *ready = false;
  if (ps.s2 == ps.s) return hipSuccess;
  hipError_t e = stream_wait(ps.s2, ps.s, ps.ss->ev[4]);
  if (e != hipSuccess) return e;
  e = emu_split_ops(ew, &oa, akc, nullptr, 0, 0, ps.s2);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ps.ss->ev[5], ps.s2);
  if (e != hipSuccess) return e;
  *ready = true;
  return hipSuccess;
}

// C -= op(A) B for the rows outside the panel, B the panel's product in the
// current scratch panel; op(A) split already on the side stream if a_ready.
hipError_t emu_sweep_update(const EmuWork& ew, const EmuOperand& oa, bool akc, bool a_ready, const EmuOperand& ob,
                            int M, int wy, double* C, long ldc, PanelSweep<double>& ps) {
  hipError_t e = emu_split_ops(ew, a_ready ? nullptr : &oa, akc, &ob, 0, -1, ps.s);
  if (e != hipSuccess) return e;
  if (a_ready) {
    e = hipStreamWaitEvent(ps.s, ps.ss->ev[5], 0);
    if (e != hipSuccess) return e;
  }
  return emu_run(emu_args(ew, oa, ob, M, wy, C, ldc), oa.K, ps.s);
}

// Y <- U^{-1} Y in place (all np rows; padded rows stay zero): per panel from
// the last, Y_p <- W_p Y_p, then the rows above take the panel's contribution
// in one K = panel-width product.
template <class T>
hipError_t back_solve(const Fact<T>& f, T* Y, long ldy, int wy, T* scr, long lds, hipStream_t s,
                      const EmuWork* ew = nullptr) {
  const long ldk = f.ldk;
  PanelSweep<T> ps;
  hipError_t e = ps.init(scr, lds, s);
  if (e != hipSuccess) return e;
  const int last_c0 = ((f.np - 1) / NB2) * NB2;
  for (int c0 = last_c0; c0 >= 0; c0 -= NB2) {
    const int c1 = std::min(c0 + NB2, f.np);
    const T* Wp = f.W + static_cast<long>(c0 / NB2) * NB2 * f.ldw;
    bool a_ready = false;
    if (c0 > 0 && ew) {
      if constexpr (std::is_same<T, double>::value)
        e = emu_presplit(*ew, emu_operand(f.kf + c0, ldk, 1, c0, c1 - c0), true, ps, &a_ready);
      if (e != hipSuccess) return e;
    }
    e = ps.product(Wp, f.ldw, false, 1, c0, c1 - c0, Y, ldy, wy);
    if (e != hipSuccess) return e;
    e = ps.copy_back(c0, c1 - c0, Y, ldy, wy);
    if (e != hipSuccess) return e;
    if (c0 > 0 && ew) {
      if constexpr (std::is_same<T, double>::value) {
        e = emu_sweep_update(*ew, emu_operand(f.kf + c0, ldk, 1, c0, c1 - c0), true, a_ready,
                             emu_operand(ps.cur, 1, lds, wy, c1 - c0), c0, wy, Y, ldy, ps);
        if (e != hipSuccess) return e;
      }
    } else if (c0 > 0) {
      GemmArgs<T> u = update_args<T>(f.kf + c0, ldk, c0, c1 - c0);
      gemm_add_segment<T>(u, ps.cur, lds, Y, ldy, wy);
      RAD_GEMM(u, false);
    }
  }
  return ps.join();
}

// Y <- K^{-T} Y in place:  U^T Z = Y  then  L^T Lambda = Z, panel by panel
// with the transposed panel inverses.
template <class T>
hipError_t transposed_solve(const Fact<T>& f, T* Y, long ldy, int wy, T* scr, long lds, hipStream_t s,
                            const EmuWork* ew = nullptr) {
  const long ldk = f.ldk;
  PanelSweep<T> ps;
  hipError_t e = ps.init(scr, lds, s);
  if (e != hipSuccess) return e;
  // U^T Z = Y: forward over panels (op(W_p) = W_p^T is lower triangular)
  for (int c0 = 0; c0 < f.np; c0 += NB2) {
    const int c1 = std::min(c0 + NB2, f.np);
    const T* Wp = f.W + static_cast<long>(c0 / NB2) * NB2 * f.ldw;
    bool a_ready = false;
    if (c1 < f.np && ew) {
      if constexpr (std::is_same<T, double>::value)
        e = emu_presplit(*ew, emu_operand(f.kf + static_cast<long>(c0) * ldk + c1, 1, ldk, f.np - c1, c1 - c0),
                         false, ps, &a_ready);
      if (e != hipSuccess) return e;
    }
    e = ps.product(Wp, f.ldw, true, 2, c0, c1 - c0, Y, ldy, wy);
    if (e != hipSuccess) return e;
    e = ps.copy_back(c0, c1 - c0, Y, ldy, wy);
    if (e != hipSuccess) return e;
    if (c1 < f.np && ew) {
      if constexpr (std::is_same<T, double>::value) {
        e = emu_sweep_update(*ew, emu_operand(f.kf + static_cast<long>(c0) * ldk + c1, 1, ldk, f.np - c1, c1 - c0),
                             false, a_ready, emu_operand(ps.cur, 1, lds, wy, c1 - c0), f.np - c1, wy,
                             Y + static_cast<long>(c1) * ldy, ldy, ps);
        if (e != hipSuccess) return e;
      }
    } else if (c1 < f.np) {  // rows below the panel: (U_{panel, c1..})^T Z_panel
      GemmArgs<T> u = update_args<T>(f.kf + static_cast<long>(c0) * ldk + c1, ldk, f.np - c1, c1 - c0);
      gemm_add_segment<T>(u, ps.cur, lds, Y + static_cast<long>(c1) * ldy, ldy, wy);
      RAD_GEMM(u, true);
    }
  }
  // the second pass reads every panel of Z, so the copies must have landed
  e = ps.join();
  if (e != hipSuccess) return e;
  // L^T Lambda = Z: backward over panels (op(V_p) = V_p^T is upper triangular)
  const int last_c0 = ((f.np - 1) / NB2) * NB2;
  for (int c0 = last_c0; c0 >= 0; c0 -= NB2) {
    const int c1 = std::min(c0 + NB2, f.np);
    const T* Vp = f.V + static_cast<long>(c0 / NB2) * NB2 * f.ldw;
    bool a_ready = false;
    if (c0 > 0 && ew) {
      if constexpr (std::is_same<T, double>::value)
        e = emu_presplit(*ew, emu_operand(f.kf + static_cast<long>(c0) * ldk, 1, ldk, c0, c1 - c0), false, ps,
                         &a_ready);
      if (e != hipSuccess) return e;
    }
    e = ps.product(Vp, f.ldw, true, 1, c0, c1 - c0, Y, ldy, wy);
    if (e != hipSuccess) return e;
    e = ps.copy_back(c0, c1 - c0, Y, ldy, wy);
    if (e != hipSuccess) return e;
    if (c0 > 0 && ew) {
      if constexpr (std::is_same<T, double>::value) {
        e = emu_sweep_update(*ew, emu_operand(f.kf + static_cast<long>(c0) * ldk, 1, ldk, c0, c1 - c0), false,
                             a_ready, emu_operand(ps.cur, 1, lds, wy, c1 - c0), c0, wy, Y, ldy, ps);
        if (e != hipSuccess) return e;
      }
    } else if (c0 > 0) {  // rows above the panel: (X_{panel, 0..c0})^T Lambda_panel
      GemmArgs<T> u = update_args<T>(f.kf + static_cast<long>(c0) * ldk, ldk, c0, c1 - c0);
      gemm_add_segment<T>(u, ps.cur, lds, Y, ldy, wy);
      RAD_GEMM(u, true);
    }
  }
  return ps.join();
}

struct GebWork {
  Scalars* sc;
  void* y;      // RHS / solution (T), np x ldy
  long ldy;
  double* x;    // FP64 iterate (np x ldx), refinement only
  long ldx;
  double* r;    // FP64 residual (np x ldx)
  double* p;    // FP64 P = F_sq diag(rho) (np x ldp), refinement only
  long ldp;
  double* part; // grad_eps partial sums (adjoint)
  EmuWork emu;  // digit buffers (RAD_PREC_FP64_I8)
  void* scr;    // (T) two panels of right-hand sides (2 NB2 x ldy), shared with
                // the panel-inverse products (tri_tmp_elems, ld ldt) and the
                // factorization's L-block products (np x NB)
  long ldt;
  size_t bytes;
  bool ok;
};

GebWork geb_work(void* work, size_t bytes, int64_t n, int32_t prec, bool adjoint) {
  Carve cv(work, bytes);
  GebWork w{};
  const int64_t np = ceil_div(n, NB) * NB;
  w.sc = cv.take<Scalars>(1);
  if (prec == RAD_PREC_FP64 || prec == RAD_PREC_FP64_I8) {
    w.ldy = rhs_ld(n, pad_elems<double>());
    w.y = cv.take<double>(static_cast<size_t>(np) * w.ldy);
    if (prec == RAD_PREC_FP64_I8) {
      // op(A) has at most np rows, B^T at most np + n + 1 (U block and RHS)
      const long rb = np + n + 1;
      w.emu.da = cv.take<int8_t>(emu_digit_bytes(np, NB2));
      w.emu.db = cv.take<int8_t>(emu_digit_bytes(rb, NB2));
      w.emu.xa = cv.take<int>(emu_scale_count(np));
      w.emu.xb = cv.take<int>(emu_scale_count(rb));
      w.emu.pa = cv.take<int>(emu_part_count(np, NB2));
      w.emu.pb = cv.take<int>(emu_part_count(rb, NB2));
    }
  } else {
    w.ldy = rhs_ld(n, pad_elems<float>());
    w.y = cv.take<float>(static_cast<size_t>(np) * w.ldy);
    w.ldx = rhs_ld(n, pad_elems<double>());
    w.x = cv.take<double>(static_cast<size_t>(np) * w.ldx);
    w.r = cv.take<double>(static_cast<size_t>(np) * w.ldx);
    w.ldp = static_cast<long>(np + pad_elems<double>());
    w.p = cv.take<double>(static_cast<size_t>(np) * w.ldp);
  }
  if (adjoint) w.part = cv.take<double>(static_cast<size_t>(ceil_div(n, GE_ROWS) * n));
  {
    const size_t es = prec == RAD_PREC_FP32_IR ? sizeof(float) : sizeof(double);
    const long pad = static_cast<long>(128 / es);
    const int P2 = static_cast<int>(ceil_div(np, NB2));
    w.ldt = tri_ldt(pad);
    // two panels of right-hand sides for the back and transposed solves
    const size_t elems = std::max(static_cast<size_t>(2 * NB2) * w.ldy, tri_tmp_elems(P2, pad));
    w.scr = cv.take<char>(elems * es);
  }
  w.bytes = cv.used;
  w.ok = cv.ok;
  return w;
}

size_t factor_bytes(int64_t n, int32_t prec) {
  return prec == RAD_PREC_FP32_IR ? factor_layout<float>(n).bytes : factor_layout<double>(n).bytes;
}

bool known_precision(int32_t p) { return p == RAD_PREC_FP64 || p == RAD_PREC_FP32_IR || p == RAD_PREC_FP64_I8; }

int read_scalars(Scalars* dev, Scalars* host, hipStream_t s) {
  RAD_HIP_CHECK(hipMemcpyAsync(host, dev, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  RAD_HIP_CHECK(hipStreamSynchronize(s));
  return RAD_OK;
}

template <class T>
void zero(T* p, long count, hipStream_t s) {
  const long blocks = std::min<long>(ceil_div(count, 256), 8192);
  hipLaunchKernelGGL(fill_zero<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, count);
}

}  // namespace
}  // namespace rad

using namespace rad;

extern "C" size_t rad_gebhart_factor_bytes(int64_t n, int32_t precision) {
  if (n < 1 || !known_precision(precision)) return 0;
  return factor_bytes(n, precision);
}

extern "C" size_t rad_gebhart_workspace_bytes(int64_t n, int32_t precision) {
  if (n < 1 || !known_precision(precision)) return 0;
  return geb_work(nullptr, 0, n, precision, false).bytes;
}

extern "C" int32_t rad_gebhart_ref(const double* F, int64_t n, int64_t ldf, const double* eps,
                                   const double* rho, double* B, int64_t ldb, int32_t precision,
                                   double ir_tol, int32_t ir_max, void* factors, size_t fbytes,
                                   void* work, size_t wbytes, rad_stats* stats, void* stream) {
  ApiRange range("rad_gebhart_ref");
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_gebhart_ref: n out of range");
  RAD_REQUIRE(ldf >= n + 1 && ldb >= n + 1, RAD_EINVAL, "rad_gebhart_ref: ldf or ldb < n+1");
  RAD_REQUIRE(F && eps && rho && B && factors, RAD_EINVAL, "rad_gebhart_ref: NULL pointer");
  RAD_REQUIRE(known_precision(precision), RAD_EINVAL, "rad_gebhart_ref: unknown precision");
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
  if (precision != RAD_PREC_FP32_IR) {
    const EmuWork* ew = precision == RAD_PREC_FP64_I8 ? &w.emu : nullptr;
    Fact<double> f = make_fact<double>(factors, factor_layout<double>(n));
    double* Y = static_cast<double*>(w.y);
    hipLaunchKernelGGL(geb_form<double>, dim3(f.np), dim3(256), 0, s, F, static_cast<long>(ldf), ni, eps,
                       rho, f.kf, f.ldk, f.np, Y, w.ldy, w.sc);
    RAD_HIP_CHECK(factor_forward<double>(f, Y, w.ldy, ni + 1, w.sc, s, ew, static_cast<double*>(w.scr)));
    RAD_HIP_CHECK(panel_inverses<double>(f, static_cast<double*>(w.scr), w.ldt, s));
    RAD_HIP_CHECK(back_solve<double>(f, Y, w.ldy, ni + 1, static_cast<double*>(w.scr), w.ldy, s, ew));
    hipLaunchKernelGGL((copy_block<double, double>), dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, B,
                       static_cast<long>(ldb));
  } else {
    Fact<float> f = make_fact<float>(factors, factor_layout<float>(n));
    float* Y = static_cast<float*>(w.y);
    hipLaunchKernelGGL(geb_form<float>, dim3(f.np), dim3(256), 0, s, F, static_cast<long>(ldf), ni, eps,
                       rho, f.kf, f.ldk, f.np, Y, w.ldy, w.sc);
    RAD_HIP_CHECK(factor_forward<float>(f, Y, w.ldy, ni + 1, w.sc, s, nullptr, static_cast<float*>(w.scr)));
    RAD_HIP_CHECK(panel_inverses<float>(f, static_cast<float*>(w.scr), w.ldt, s));
    RAD_HIP_CHECK(back_solve<float>(f, Y, w.ldy, ni + 1, static_cast<float*>(w.scr), w.ldy, s));
    if (ir_max > 0) {
      zero<double>(w.x, static_cast<long>(f.np) * w.ldx, s);
      zero<double>(w.r, static_cast<long>(f.np) * w.ldx, s);
      hipLaunchKernelGGL(form_p64, dim3(f.np), dim3(256), 0, s, F, static_cast<long>(ldf), ni, rho, w.p, w.ldp);
      hipLaunchKernelGGL((copy_block<float, double>), dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, w.x, w.ldx);
      for (int step = 0; step < ir_max; ++step) {
        hipLaunchKernelGGL(scalars_init_partial, dim3(1), dim3(64), 0, s, w.sc);
        hipLaunchKernelGGL(residual_init, dim3(ni), dim3(256), 0, s, F, static_cast<long>(ldf), ni, eps, w.x,
                           w.ldx, w.r, w.ldx);
        GemmArgs<double> a = gemm_args<double>(w.p, w.ldp, ni, static_cast<int>(ceil_div(n, 32) * 32), 1.0, 1.0);
        gemm_add_segment<double>(a, w.x, w.ldx, w.r, w.ldx, ni + 1);
        RAD_HIP_CHECK(launch_gemm(a, false, s));
        hipLaunchKernelGGL(residual_to_rhs, dim3(ni), dim3(256), 0, s, w.r, w.ldx, ni, Y, w.ldy, w.sc);
        RAD_HIP_CHECK(forward_only<float>(f, Y, w.ldy, ni + 1, s));
        RAD_HIP_CHECK(back_solve<float>(f, Y, w.ldy, ni + 1, static_cast<float*>(w.scr), w.ldy, s));
        hipLaunchKernelGGL(apply_correction, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, w.x, w.ldx, w.sc);
        ++ir_steps;
        int rc = read_scalars(w.sc, &h, s);
        if (rc != RAD_OK) return rc;
        if (h.status < 0 || h.max_d <= ir_tol) break;
      }
      hipLaunchKernelGGL((copy_block<double, double>), dim3(ni), dim3(256), 0, s, w.x, w.ldx, ni, B,
                         static_cast<long>(ldb));
    } else {
      hipLaunchKernelGGL((copy_block<float, double>), dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, B,
                         static_cast<long>(ldb));
    }
  }
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats && precision != RAD_PREC_FP32_IR) return RAD_OK;
  int rc = read_scalars(w.sc, &h, s);
  if (rc != RAD_OK) return rc;
  if (stats) {
    *stats = rad_stats{};
    stats->ir_steps = ir_steps;
    stats->device_status = h.status;
    stats->ir_correction = h.max_d;
    stats->ir_residual = h.max_r;
    stats->converged = (precision != RAD_PREC_FP32_IR) || (ir_steps > 0 && h.max_d <= ir_tol);
  }
  if (h.status < 0) {
    set_error(h.status == RAD_ESINGULAR ? "rad_gebhart_ref: singular diagonal block of K"
                                        : "rad_gebhart_ref: F, eps or rho out of range or non-finite");
    return h.status;
  }
  if (precision == RAD_PREC_FP32_IR && ir_max > 0 && !(h.max_d <= ir_tol)) return RAD_WNOTCONVERGED;
  return RAD_OK;
}

extern "C" size_t rad_steady_temperature_workspace_bytes(int64_t n, int32_t precision) {
  if (n < 1 || n > (1 << 20) || (precision != RAD_PREC_FP64 && precision != RAD_PREC_FP64_I8)) return 0;
  return rad_gebhart_workspace_bytes(n, precision);
}

extern "C" int32_t rad_steady_temperature(const double* Y, int64_t n, int64_t ldy, const double* weight,
                                          const double* Q, int64_t m, int64_t ldq, const double* t_fixed,
                                          double t_space, double sigma, double* T, int64_t ldt,
                                          int32_t precision, void* factors, size_t fbytes, void* work,
                                          size_t wbytes, rad_stats* stats, void* stream) {
  ApiRange range("rad_steady_temperature");
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_steady_temperature: n out of range");
  RAD_REQUIRE(m >= 1 && m <= RAD_STEADY_MAX_CASES, RAD_EINVAL,
              "rad_steady_temperature: m outside [1, RAD_STEADY_MAX_CASES]");
  RAD_REQUIRE(ldy >= n + 1 && ldq >= m && ldt >= m, RAD_EINVAL, "rad_steady_temperature: leading dimension too small");
  RAD_REQUIRE(Y && weight && Q && T && factors, RAD_EINVAL, "rad_steady_temperature: NULL pointer");
  RAD_REQUIRE(precision == RAD_PREC_FP64 || precision == RAD_PREC_FP64_I8, RAD_EINVAL,
              "rad_steady_temperature: precision must be RAD_PREC_FP64 or RAD_PREC_FP64_I8");
  RAD_REQUIRE(t_space >= 0.0 && t_space <= 1.0e75 && sigma > 0.0 && sigma <= 1.0e300, RAD_EINVAL,
              "rad_steady_temperature: t_space or sigma out of range");
  RAD_REQUIRE(fbytes >= factor_bytes(n, precision) && reinterpret_cast<uintptr_t>(factors) % 256 == 0,
              RAD_EWORKSPACE, "rad_steady_temperature: factor buffer too small or not 256-byte aligned");
  GebWork w = geb_work(work, wbytes, n, precision, false);
  RAD_REQUIRE(w.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_steady_temperature: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n), mi = static_cast<int>(m);
  // the right-hand sides occupy one full 64-column tile (zero past m)
  constexpr int SS_RHS = 64;
  static_assert(SS_RHS >= RAD_STEADY_MAX_CASES, "right-hand side tile narrower than the case limit");
  const EmuWork* ew = precision == RAD_PREC_FP64_I8 ? &w.emu : nullptr;
  Fact<double> f = make_fact<double>(factors, factor_layout<double>(n));
  double* X = static_cast<double*>(w.y);
  const double xs = (t_space * t_space) * (t_space * t_space);
  hipLaunchKernelGGL(scalars_init, dim3(1), dim3(64), 0, s, w.sc);
  hipLaunchKernelGGL(ss_form, dim3(f.np), dim3(256), 0, s, Y, static_cast<long>(ldy), ni, weight, Q,
                     static_cast<long>(ldq), mi, t_fixed, xs, sigma, f.kf, f.ldk, f.np, X, w.ldy, w.sc);
  RAD_HIP_CHECK(factor_forward<double>(f, X, w.ldy, SS_RHS, w.sc, s, ew, static_cast<double*>(w.scr)));
  RAD_HIP_CHECK(panel_inverses<double>(f, static_cast<double*>(w.scr), w.ldt, s));
  RAD_HIP_CHECK(back_solve<double>(f, X, w.ldy, SS_RHS, static_cast<double*>(w.scr), w.ldy, s, ew));
  hipLaunchKernelGGL(ss_output, dim3(static_cast<unsigned>(ceil_div(n * m, 256))), dim3(256), 0, s, X, w.ldy, ni,
                     mi, t_fixed, T, static_cast<long>(ldt), w.sc);
  RAD_HIP_CHECK(hipGetLastError());
  if (!stats) return RAD_OK;
  Scalars h{};
  int rc = read_scalars(w.sc, &h, s);
  if (rc != RAD_OK) return rc;
  *stats = rad_stats{};
  stats->device_status = h.status;
  stats->converged = 1;
  if (h.status < 0) {
    set_error(h.status == RAD_ESINGULAR
                  ? "rad_steady_temperature: singular balance (a free node without a path to space or a fixed node)"
                  : "rad_steady_temperature: input out of range or non-finite, or no real temperature balances "
                    "the heat input");
    return h.status;
  }
  return RAD_OK;
}

namespace {
struct LsqWork {
  GebWork geb;
  uint8_t* mask[2];
  int* negatives;
  size_t bytes;
  bool ok;
};

LsqWork lsq_work(void* work, size_t bytes, int64_t n, int32_t prec) {
  LsqWork l{};
  const size_t gb = align_up(geb_work(nullptr, 0, n, prec, false).bytes, 256);
  l.geb = geb_work(work, std::min(bytes, gb), n, prec, false);
  Carve cv(work && bytes > gb ? static_cast<char*>(work) + gb : nullptr, bytes > gb ? bytes - gb : 0);
  const size_t mb = static_cast<size_t>(n) * static_cast<size_t>(n + 1);
  l.mask[0] = cv.take<uint8_t>(mb);
  l.mask[1] = cv.take<uint8_t>(mb);
  l.negatives = cv.take<int>(64);
  l.bytes = gb + cv.used;
  l.ok = l.geb.ok && cv.ok;
  return l;
}
}  // namespace

extern "C" size_t rad_enforce_lsq_workspace_bytes(int64_t n, int32_t precision) {
  if (n < 1 || n > (1 << 20) || (precision != RAD_PREC_FP64 && precision != RAD_PREC_FP64_I8)) return 0;
  return lsq_work(nullptr, 0, n, precision).bytes;
}

extern "C" int32_t rad_enforce_lsq(const double* F, int64_t n, int64_t ldf, const double* omega, double* Fout,
                                   int64_t ldo, int32_t flags, int32_t max_rounds, int32_t precision,
                                   void* factors, size_t fbytes, void* work, size_t wbytes, rad_stats* stats,
                                   void* stream) {
  ApiRange range("rad_enforce_lsq");
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= 65535, RAD_EINVAL, "rad_enforce_lsq: n out of range (1..65535)");
  RAD_REQUIRE(ldf >= n + 1 && ldo >= n + 1, RAD_EINVAL, "rad_enforce_lsq: ldf or ldo < n+1");
  RAD_REQUIRE(F && omega && Fout && factors, RAD_EINVAL, "rad_enforce_lsq: NULL pointer");
  RAD_REQUIRE(F != Fout, RAD_EINVAL, "rad_enforce_lsq: F and Fout must not be the same buffer");
  RAD_REQUIRE((flags & ~(RAD_LSQ_NNR | RAD_LSQ_SPVA)) == 0 && max_rounds >= 1, RAD_EINVAL,
              "rad_enforce_lsq: unknown flag or max_rounds < 1");
  RAD_REQUIRE(precision == RAD_PREC_FP64 || precision == RAD_PREC_FP64_I8, RAD_EINVAL,
              "rad_enforce_lsq: precision must be RAD_PREC_FP64 or RAD_PREC_FP64_I8");
  RAD_REQUIRE(fbytes >= factor_bytes(n, precision) && reinterpret_cast<uintptr_t>(factors) % 256 == 0,
              RAD_EWORKSPACE, "rad_enforce_lsq: factor buffer too small or not 256-byte aligned");
  LsqWork l = lsq_work(work, wbytes, n, precision);
  RAD_REQUIRE(l.ok && reinterpret_cast<uintptr_t>(work) % 256 == 0, RAD_EWORKSPACE,
              "rad_enforce_lsq: workspace too small or not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n);
  const int nnr = (flags & RAD_LSQ_NNR) != 0;
  constexpr int LSQ_RHS = 64;
  const GebWork& w = l.geb;
  const EmuWork* ew = precision == RAD_PREC_FP64_I8 ? &w.emu : nullptr;
  Fact<double> f = make_fact<double>(factors, factor_layout<double>(n));
  double* Y = static_cast<double*>(w.y);
  const dim3 egrid(static_cast<unsigned>(ceil_div(n + 1, 256)), static_cast<unsigned>(n));
  const dim3 ugrid(static_cast<unsigned>(ceil_div(n + 1, LSQ_KC)), static_cast<unsigned>(ceil_div(n, LSQ_RB)));
  hipLaunchKernelGGL(scalars_init, dim3(1), dim3(64), 0, s, w.sc);
  hipLaunchKernelGGL(lsq_mask_init, egrid, dim3(256), 0, s, F, static_cast<long>(ldf), ni,
                     (flags & RAD_LSQ_SPVA) ? 1 : 0, l.mask[0], w.sc);
  int rounds = 0, negatives = 0, cur = 0;
  Scalars h{};
  for (;;) {
    ++rounds;
    hipLaunchKernelGGL(fill_zero<int>, dim3(1), dim3(64), 0, s, l.negatives, 1L);
    hipLaunchKernelGGL(lsq_schur, dim3(static_cast<unsigned>(ceil_div(f.np, LSQ_RB))), dim3(256), 0, s, F,
                       static_cast<long>(ldf), ni, omega, l.mask[cur], f.kf, f.ldk, f.np, Y, w.ldy);
    RAD_HIP_CHECK(factor_forward<double>(f, Y, w.ldy, LSQ_RHS, w.sc, s, ew, static_cast<double*>(w.scr)));
    RAD_HIP_CHECK(panel_inverses<double>(f, static_cast<double*>(w.scr), w.ldt, s));
    RAD_HIP_CHECK(back_solve<double>(f, Y, w.ldy, LSQ_RHS, static_cast<double*>(w.scr), w.ldy, s, ew));
    hipLaunchKernelGGL(lsq_update, ugrid, dim3(256), 0, s, F, static_cast<long>(ldf), ni, omega, l.mask[cur], Y,
                       w.ldy, nnr, l.mask[1 - cur], Fout, static_cast<long>(ldo), l.negatives);
    RAD_HIP_CHECK(hipGetLastError());
    RAD_HIP_CHECK(hipMemcpyAsync(&negatives, l.negatives, sizeof(int), hipMemcpyDeviceToHost, s));
    int rc = read_scalars(w.sc, &h, s);  // synchronises the stream
    if (rc != RAD_OK) return rc;
    cur = 1 - cur;
    if (h.status < 0 || !nnr || negatives == 0 || rounds >= max_rounds) break;
  }
  if (stats) {
    *stats = rad_stats{};
    stats->iters = rounds;
    stats->device_status = h.status;
    stats->converged = h.status >= 0 && (!nnr || negatives == 0);
  }
  if (h.status < 0) {
    set_error(h.status == RAD_ESINGULAR ? "rad_enforce_lsq: singular closure system"
                                        : "rad_enforce_lsq: non-finite view factor");
    return h.status;
  }
  return (nnr && negatives > 0) ? RAD_WNOTCONVERGED : RAD_OK;
}

namespace {
// REF check workspace: closure maxima per 4-row block, reciprocity maxima per tile pair
size_t ref_check_bytes(int64_t n) {
  const int64_t t = ceil_div(n, 64);
  return align_up(static_cast<size_t>(ceil_div(n, 4)) * sizeof(double), 256) +
         align_up(static_cast<size_t>(t * (t + 1) / 2) * sizeof(double), 256);
}
}  // namespace

extern "C" size_t rad_ref_check_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return ref_check_bytes(n);
}

extern "C" int32_t rad_ref_check(const double* B, int64_t n, int64_t ldb, const double* eps,
                                 const double* area, double* out, void* work, size_t wbytes,
                                 void* stream) {
  ApiRange range("rad_ref_check");
  clear_error();
  RAD_REQUIRE(n >= 1 && ldb >= n + 1, RAD_EINVAL, "rad_ref_check: bad n or ldb");
  RAD_REQUIRE(B && eps && area && out, RAD_EINVAL, "rad_ref_check: NULL pointer");
  RAD_REQUIRE(n <= (1 << 20), RAD_EINVAL, "rad_ref_check: n out of range");
  RAD_REQUIRE(work && wbytes >= ref_check_bytes(n) && reinterpret_cast<uintptr_t>(work) % 256 == 0,
              RAD_EWORKSPACE, "rad_ref_check: workspace too small or misaligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n);
  const int t = static_cast<int>(ceil_div(n, 64));
  const long pairs = static_cast<long>(t) * (t + 1) / 2;
  const int nc = static_cast<int>(ceil_div(n, 4));
  double* bc = static_cast<double*>(work);
  double* br = reinterpret_cast<double*>(static_cast<char*>(work) + align_up(static_cast<size_t>(nc) * sizeof(double), 256));
  hipLaunchKernelGGL(ref_closure, dim3(static_cast<unsigned>(nc)), dim3(256), 0, s, B, static_cast<long>(ldb), ni, bc);
  hipLaunchKernelGGL(ref_reciprocity, dim3(static_cast<unsigned>(pairs)), dim3(256), 0, s, B, static_cast<long>(ldb),
                     ni, t, eps, area, br);
  hipLaunchKernelGGL(ref_final, dim3(1), dim3(256), 0, s, bc, nc, br, pairs, out);
  RAD_HIP_CHECK(hipGetLastError());
  return RAD_OK;
}

extern "C" size_t rad_adjoint_workspace_bytes(int64_t n, int32_t precision) {
  if (n < 1 || !known_precision(precision)) return 0;
  return geb_work(nullptr, 0, n, precision, true).bytes;
}

extern "C" int32_t rad_gebhart_ref_adjoint(const void* factors, size_t fbytes, int32_t precision,
                                           const double* F, int64_t n, int64_t ldf, const double* rho,
                                           const double* B, int64_t ldb, const double* G, int64_t ldg,
                                           double* grad_eps, double* grad_rho, double* Lambda,
                                           int64_t ldl, double ir_tol, int32_t ir_max, void* work,
                                           size_t wbytes, rad_stats* stats, void* stream) {
  ApiRange range("rad_gebhart_ref_adjoint");
  clear_error();
  RAD_REQUIRE(n >= 1 && n <= (1 << 20), RAD_EINVAL, "rad_gebhart_ref_adjoint: n out of range");
  RAD_REQUIRE(ldf >= n + 1 && ldb >= n + 1 && ldg >= n + 1 && (!Lambda || ldl >= n + 1), RAD_EINVAL,
              "rad_gebhart_ref_adjoint: leading dimension < n+1");
  RAD_REQUIRE(factors && F && rho && B && G && grad_eps && grad_rho, RAD_EINVAL,
              "rad_gebhart_ref_adjoint: NULL pointer");
  RAD_REQUIRE(known_precision(precision), RAD_EINVAL, "rad_gebhart_ref_adjoint: unknown precision");
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
  if (precision != RAD_PREC_FP32_IR) {
    const EmuWork* ew = precision == RAD_PREC_FP64_I8 ? &w.emu : nullptr;
    Fact<double> f = make_fact<double>(const_cast<void*>(factors), factor_layout<double>(n));
    double* Y = static_cast<double*>(w.y);
    hipLaunchKernelGGL(load_rhs<double>, dim3(f.np), dim3(256), 0, s, G, static_cast<long>(ldg), ni, Y, w.ldy,
                       w.sc);
    RAD_HIP_CHECK(transposed_solve<double>(f, Y, w.ldy, ni + 1, static_cast<double*>(w.scr), w.ldy, s, ew));
    lam = Y;
    ldlam = w.ldy;
  } else {
    Fact<float> f = make_fact<float>(const_cast<void*>(factors), factor_layout<float>(n));
    float* Y = static_cast<float*>(w.y);
    hipLaunchKernelGGL(load_rhs<float>, dim3(f.np), dim3(256), 0, s, G, static_cast<long>(ldg), ni, Y, w.ldy,
                       w.sc);
    RAD_HIP_CHECK(transposed_solve<float>(f, Y, w.ldy, ni + 1, static_cast<float*>(w.scr), w.ldy, s));
    zero<double>(w.x, static_cast<long>(f.np) * w.ldx, s);
    hipLaunchKernelGGL((copy_block<float, double>), dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, w.x, w.ldx);
    if (ir_max > 0) {
      zero<double>(w.r, static_cast<long>(f.np) * w.ldx, s);
      hipLaunchKernelGGL(form_p64, dim3(f.np), dim3(256), 0, s, F, static_cast<long>(ldf), ni, rho, w.p, w.ldp);
    }
    for (int step = 0; step < ir_max; ++step) {
      hipLaunchKernelGGL(scalars_init_partial, dim3(1), dim3(64), 0, s, w.sc);
      // R = G - K^T Lambda = (G - Lambda) + P^T Lambda
      hipLaunchKernelGGL(adj_residual_init, dim3(ni), dim3(256), 0, s, G, static_cast<long>(ldg), ni, w.x,
                         w.ldx, w.r, w.ldx);
      GemmArgs<double> a = gemm_args<double>(w.p, w.ldp, ni, static_cast<int>(ceil_div(n, 32) * 32), 1.0, 1.0);
      gemm_add_segment<double>(a, w.x, w.ldx, w.r, w.ldx, ni + 1);
      RAD_HIP_CHECK(launch_gemm(a, true, s));
      hipLaunchKernelGGL(residual_to_rhs, dim3(ni), dim3(256), 0, s, w.r, w.ldx, ni, Y, w.ldy, w.sc);
      RAD_HIP_CHECK(transposed_solve<float>(f, Y, w.ldy, ni + 1, static_cast<float*>(w.scr), w.ldy, s));
      hipLaunchKernelGGL(apply_correction, dim3(ni), dim3(256), 0, s, Y, w.ldy, ni, w.x, w.ldx, w.sc);
      ++ir_steps;
      int rc = read_scalars(w.sc, &h, s);
      if (rc != RAD_OK) return rc;
      if (h.status < 0 || h.max_d <= ir_tol) break;
    }
    lam = w.x;
    ldlam = w.ldx;
  }
  if (Lambda)
    hipLaunchKernelGGL((copy_block<double, double>), dim3(ni), dim3(256), 0, s, lam, ldlam, ni, Lambda,
                       static_cast<long>(ldl));
  const int chunks = static_cast<int>(ceil_div(n, GE_ROWS));
  hipLaunchKernelGGL(adj_grad_eps_partial, dim3(static_cast<unsigned>(ceil_div(n, 256)), chunks), dim3(256), 0, s,
                     lam, ldlam, F, static_cast<long>(ldf), ni, w.part);
  hipLaunchKernelGGL(adj_grad_eps_final, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, w.part,
                     ni, chunks, grad_eps);
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
  stats->converged = (precision != RAD_PREC_FP32_IR) || (ir_steps > 0 && h.max_d <= ir_tol);
  if (h.status < 0) {
    set_error("rad_gebhart_ref_adjoint: non-finite entry of G or of the refinement residual");
    return h.status;
  }
  if (precision == RAD_PREC_FP32_IR && ir_max > 0 && !(h.max_d <= ir_tol)) return RAD_WNOTCONVERGED;
  return RAD_OK;
}
