/*
 * rad.h - C ABI of the gfx950 radiative hot path.
 *
 * Data-parallel core of the radiative pipeline of B. Frangi, "Novel Numerical
 * Methods for Accurate Space Thermal Analysis" (arXiv:2511.04277):
 *
 *   noisy MCRT view factors F  --rad_enforce_vf-->  F satisfying closure and
 *   reciprocity  --rad_gebhart_ref-->  REF matrix B  --rad_aggregate_nodes-->
 *   face / node level factors,  plus  rad_gebhart_ref_adjoint  (dJ/d eps, rho).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Open-system matrices are N x (N+1), row-major, float64, leading dimension
 *   ld >= N+1 (in elements); column N is deep space (thesis Sec. 2.4.12, the
 *   N x (N+1) layout of the open-system view-factor matrix).
 * - Every array argument is a DEVICE pointer unless marked "host".  The caller
 *   owns all memory: the library never allocates or frees device memory inside
 *   a call; scratch comes from the caller's ``work`` buffer, whose size is
 *   given by the matching *_workspace_bytes() query (256-byte alignment).
 * - ``stream`` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *   work on it and return.  When ``stats`` (host) is non-NULL the call waits
 *   for its own work and fills it; device-side errors (non-finite or
 *   out-of-range input, zero row, singular pivot) are only reported then.
 * - Return value: RAD_OK (0), a positive warning, or a negative error code;
 *   rad_last_error() gives a message for the calling thread.  No exception
 *   crosses the ABI.  On an error the outputs are unspecified.
 * - Calls on the same stream are ordered; calls that share a workspace on
 *   different streams race.
 */
#ifndef RAD_H
#define RAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RAD_OK 0
#define RAD_WNOTCONVERGED 1   /* tol > 0 not met within max_iter / ir_max   */
#define RAD_EINVAL (-1)       /* bad size, stride, mode or NULL pointer      */
#define RAD_ENONFINITE (-2)   /* NaN/Inf or out-of-range value in an input   */
#define RAD_EZEROROW (-3)     /* a view-factor row sums to zero              */
#define RAD_ESINGULAR (-4)    /* a pivot block of K is singular              */
#define RAD_EHIP (-5)         /* a HIP runtime call failed                   */
#define RAD_EWORKSPACE (-6)   /* work / factor buffer too small or misaligned */

/* ---- options ----------------------------------------------------------- */
#define RAD_KAPPA_FRACVAR 0   /* fractional-variance weight, eq. 3.23-3.25  */
#define RAD_KAPPA_HALF 1      /* equal weights kappa = 1/2 (eq. 3.20)        */

#define RAD_PREC_FP64 0       /* FP64 MFMA factorization and solves          */
#define RAD_PREC_FP32_IR 1    /* FP32 MFMA factorization and solves, FP64
                                 residual iterative refinement               */
#define RAD_PREC_FP64_I8 2    /* FP64 factorization and solves whose panel-
                                 width products run on the int8 matrix cores
                                 as exact digit products (7 digits of 7 bits
                                 per operand, FP64 accumulation)             */

/* Per-call statistics (host struct). */
typedef struct rad_stats {
  int32_t iters;          /* enforcement iterations executed                 */
  int32_t ir_steps;       /* iterative-refinement steps executed             */
  int32_t converged;      /* 1 if the tolerance was met                      */
  int32_t device_status;  /* status raised by device-side checks (0 = ok)    */
  double closure_defect;  /* max_i |s_i - 1| after the last reciprocity step */
  double recip_err;       /* max|eta_ij - eta_ji| / max eta entering the last
                             iteration (eta_ij = A_i F_ij)                   */
  double ir_correction;   /* max |delta B| of the last refinement step       */
  double ir_residual;     /* max |E - K B| before the last refinement step   */
} rad_stats;

const char* rad_status_string(int32_t code);
const char* rad_last_error(void);
int32_t rad_version(void);

/* ---- iterative closure + reciprocity enforcer ------------------------- */
/*
 * Thesis Sec. 3.5.5 ("Iterative closure and reciprocity enforcer"), applied
 * in place to F (n x (n+1), ld ldf).  Each iteration:
 *   1. reciprocity on the square block, i != j (Sec. 3.5.3, eq. 3.18-3.20):
 *      eta_ij = A_i F_ij, eta^ = kappa eta_ij + (1-kappa) eta_ji, used for
 *      both F_ij = eta^/A_i and F_ji = eta^/A_j; kappa by ``kappa_mode``:
 *      RAD_KAPPA_FRACVAR: kappa = s2_ji / (s2_ij + s2_ji),
 *      s2_ij = A_i^2 (1 - F_ij) / (n_rays_i F_ij) (eq. 3.23-3.25; z cancels;
 *      a zero factor gets all weight moved to its partner; both zero -> 1/2);
 *      RAD_KAPPA_HALF: kappa = 1/2 (reproduces the worked example, Sec. 6.2).
 *      The diagonal and the space column are carried over unchanged.
 *   2. closure over all n+1 columns by least-squares smoothing for open
 *      systems with omega = eta (Sec. 3.5.4, eq. 3.36-3.40): F_ij /= s_i,
 *      s_i = sum_j F_ij.
 * Stopping: with tol > 0 the loop ends after the first iteration whose
 * closure defect max_i |s_i - 1| is <= tol (returns RAD_WNOTCONVERGED if
 * max_iter is reached first); tol == 0 runs exactly max_iter iterations and
 * needs no host synchronisation (graph-capturable when stats == NULL).
 *
 * F:      any ldf >= n+1 works; rows that start on 128-byte boundaries
 *         (F 128-byte aligned, ldf a multiple of 16) let every tile row
 *         load touch only its own cache lines, which makes a sweep about
 *         25 % faster at n = 8192 than ldf = n+1.
 * area:   n face areas A_i > 0.
 * n_rays: n rays emitted per face (> 0); may be NULL for RAD_KAPPA_HALF.
 * work:   >= rad_enforce_workspace_bytes(n).
 * Device checks: F entries finite and >= 0 (RAD_ENONFINITE), zero rows
 * (RAD_EZEROROW).
 */
size_t rad_enforce_workspace_bytes(int64_t n);
int32_t rad_enforce_vf(double* F, int64_t n, int64_t ldf, const double* area,
                       const double* n_rays, int32_t kappa_mode, double tol,
                       int32_t max_iter, void* work, size_t work_bytes,
                       rad_stats* stats, void* stream);

/*
 * Allocation-free variant of rad_enforce_vf, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same iteration, kernels and
 * results as rad_enforce_vf, with the scratch taken from a fixed array of
 * RAD_ENFORCE_NOALLOC_BYTES in device memory that the library reserves when
 * it is loaded, one per GPU, held until the process ends.  n up to 16384
 * fits (n for which rad_enforce_workspace_bytes(n) <= RAD_ENFORCE_NOALLOC_BYTES);
 * a larger n returns RAD_EWORKSPACE with a message and enqueues nothing.
 * The call allocates nothing; the caller passes F, area, n_rays as for
 * rad_enforce_vf.  Every call on one GPU uses that GPU's single scratch
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads) race; serialise them.  The device of ``stream`` must
 * be the current HIP device.
 */
#define RAD_ENFORCE_NOALLOC_BYTES ((size_t)36 << 20)
int32_t rad_enforce_vf_noalloc(double* F, int64_t n, int64_t ldf,
                               const double* area, const double* n_rays,
                               int32_t kappa_mode, double tol, int32_t max_iter,
                               rad_stats* stats, void* stream);

/* ---- open-system Gebhart REF solve ------------------------------------- */
/*
 * Gebhart's matrix method extended to open systems (Sec. 4.2.3, eq. 4.5;
 * App. B.2, eq. B.6-B.11):
 *   K = I - F_sq diag(rho)  (n x n),   E = [F_sq diag(eps) | F_space],
 *   B = K^{-1} E            (n x (n+1), written to B with ld ldb).
 * eps, rho: n values in [0, 1] (independent inputs; rho = 1 - eps for gray
 * opaque faces).  K is strictly diagonally dominant by rows when rho < 1 and
 * the rows of F sum to <= 1, so the factorization is a block LU without
 * pivoting.
 * precision: RAD_PREC_FP64, RAD_PREC_FP32_IR (FP32 factorization/solves,
 *   refinement B += K^{-1}(E - K B) with the residual in FP64 until
 *   max|delta| <= ir_tol or ir_max steps; RAD_WNOTCONVERGED otherwise), or
 *   RAD_PREC_FP64_I8 (FP64 factors and solves; the K = 1024 trailing,
 *   substitution and back-substitution products are exact int8 digit
 *   products with FP64 accumulation, rounding about 2^-49 relative to the
 *   operand row maxima; ir_tol / ir_max ignored).  The factors of FP64_I8
 *   are FP64 factors (same size as RAD_PREC_FP64).
 * factors: caller-owned, >= rad_gebhart_factor_bytes(n, precision); receives
 *   the factorization, which rad_gebhart_ref_adjoint reuses.  It stays valid
 *   until the caller frees or overwrites it.
 * work: >= rad_gebhart_workspace_bytes(n, precision).
 * Device checks: eps, rho outside [0, 1] or non-finite, non-finite F
 *   (RAD_ENONFINITE); a pivot below 1e-11 (FP64) / 1e-5 (FP32) in the
 *   elimination, i.e. a numerically singular K (RAD_ESINGULAR).
 */
size_t rad_gebhart_factor_bytes(int64_t n, int32_t precision);
size_t rad_gebhart_workspace_bytes(int64_t n, int32_t precision);
int32_t rad_gebhart_ref(const double* F, int64_t n, int64_t ldf,
                        const double* eps, const double* rho, double* B,
                        int64_t ldb, int32_t precision, double ir_tol,
                        int32_t ir_max, void* factors, size_t factor_bytes,
                        void* work, size_t work_bytes, rad_stats* stats,
                        void* stream);

/*
 * REF relations as residuals (Sec. 4.2.1, eq. 4.3-4.4), computed in FP64:
 *   out[0] = max_i |sum_{j<=n} B_ij + B_i,space - 1|            (closure)
 *   out[1] = max_{i,j} |eps_i A_i B_ij - eps_j A_j B_ji|        (reciprocity)
 * out: 2 doubles (device).  work: >= rad_ref_check_workspace_bytes(n).
 */
size_t rad_ref_check_workspace_bytes(int64_t n);
int32_t rad_ref_check(const double* B, int64_t n, int64_t ldb, const double* eps,
                      const double* area, double* out, void* work,
                      size_t work_bytes, void* stream);

/* ---- adjoint of the REF solve ------------------------------------------ */
/*
 * Given G = dJ/dB (n x (n+1), ld ldg) for the B computed by rad_gebhart_ref
 * with the same F, rho, ``factors`` and ``precision``:
 *   Lambda = K^{-T} G                       (transposed solve, factors reused;
 *                                            FP64 refinement in FP32_IR mode)
 *   grad_eps[k] = sum_i Lambda_ik F_ik
 *   grad_rho[k] = sum_i sum_j F_ik Lambda_ij B_kj
 *               = (1/rho_k) sum_j B_kj (Lambda_kj - G_kj)  (K^T Lambda = G),
 *     the direct column form being used where rho_k < 1e-3.
 * These are the derivatives through B only (B = K^{-1}E, App. B.2); an
 * objective with explicit eps/rho terms adds its own partials.
 * Lambda (nullable, ld ldl) receives K^{-T} G when non-NULL.
 * In RAD_PREC_FP32_IR the transposed solve is refined in FP64 (residual
 * G - K^T Lambda) until max|delta| <= ir_tol or ir_max steps.
 * Device checks: a non-finite entry of G, or of a refinement residual,
 * raises RAD_ENONFINITE (reported when ``stats`` is non-NULL; the
 * refinement stops at once).
 * work: >= rad_adjoint_workspace_bytes(n, precision).
 */
size_t rad_adjoint_workspace_bytes(int64_t n, int32_t precision);
int32_t rad_gebhart_ref_adjoint(const void* factors, size_t factor_bytes,
                                int32_t precision, const double* F, int64_t n,
                                int64_t ldf, const double* rho, const double* B,
                                int64_t ldb, const double* G, int64_t ldg,
                                double* grad_eps, double* grad_rho, double* Lambda,
                                int64_t ldl, double ir_tol, int32_t ir_max,
                                void* work, size_t work_bytes, rad_stats* stats,
                                void* stream);

/* ---- multi-node aggregation -------------------------------------------- */
/*
 * Surface / node factors from sub-surface factors (Sec. 5.2.3, eq. 5.6-5.7;
 * first two rows of eq. 5.28, one-sided faces):
 *   Y_GH = sum_{i in G} sum_{j in H} w_i X_ij / W_G,
 *   Y_G,space = sum_{i in G} w_i X_i,space / W_G,   W_G = sum_{i in G} w_i.
 * X: n x (n+1) (ld ldx); weight: n values > 0 (w_i = S_i for view factors,
 * eps_i S_i for REFs); group: n int32 in [0, g) (device); Y: g x (g+1)
 * (ld ldy); group_weight: g doubles receiving W_G (nullable).  Every group
 * must be non-empty and every id in range; these are checked on the device
 * and reported (RAD_EINVAL) when ``stats`` is non-NULL.  Sums run in a fixed
 * order (bitwise reproducible).
 * work: >= rad_aggregate_workspace_bytes(n, g).
 */
size_t rad_aggregate_workspace_bytes(int64_t n, int64_t g);
int32_t rad_aggregate_nodes(const double* X, int64_t n, int64_t ldx,
                            const double* weight, const int32_t* group,
                            int64_t g, double* Y, int64_t ldy,
                            double* group_weight, void* work, size_t work_bytes,
                            rad_stats* stats, void* stream);

/* ---- least-squares optimum enforcer ------------------------------------- */
/*
 * Closure + reciprocity enforcement by the least-squares optimum for open
 * systems (Sec. 3.5.5, eq. 3.41-3.52): the view factors closest to F (in the
 * Euclidean norm over all n (n+1) entries) whose rows sum to one and with
 * omega_i F_ik = omega_k F_ki.  Flags: RAD_LSQ_NNR repeats the projection
 * with the negative entries held at zero until none is negative (App. A.1);
 * RAD_LSQ_SPVA holds the zero entries of F at zero from the start
 * (App. A.2).  The projection is solved through the n x n system of the
 * closure multipliers (the reciprocity multipliers eliminated in closed
 * form), factored by the Gebhart solve's block LDU, one solve per round.
 * F: n x (n+1) input, 1 <= n <= 65535 (ld ldf, not modified); omega: n
 * weights (the areas);
 * Fout: n x (n+1) result (ld ldo), a different buffer; max_rounds >= 1.
 * precision: RAD_PREC_FP64 or RAD_PREC_FP64_I8.  factors: >=
 * rad_gebhart_factor_bytes(n, precision); work: >=
 * rad_enforce_lsq_workspace_bytes(n, precision); both 256-byte aligned.
 * Synchronises the stream once per round (the NNR test).  stats (nullable):
 * iters = rounds run.  Returns RAD_WNOTCONVERGED if negative entries remain
 * after max_rounds; RAD_ENONFINITE for a non-finite input.
 */
#define RAD_LSQ_NNR 1
#define RAD_LSQ_SPVA 2
size_t rad_enforce_lsq_workspace_bytes(int64_t n, int32_t precision);
int32_t rad_enforce_lsq(const double* F, int64_t n, int64_t ldf,
                        const double* omega, double* Fout, int64_t ldo,
                        int32_t flags, int32_t max_rounds, int32_t precision,
                        void* factors, size_t factor_bytes, void* work,
                        size_t work_bytes, rad_stats* stats, void* stream);

/* ---- two-sided nodes ---------------------------------------------------- */
/*
 * A node is a sub-surface with C_n faces (one, A, or two, A and B); the
 * face-level matrices below have one row per face, group[a] in [0, g) names
 * the node of face a (device int32), column nf is deep space.  Node view
 * factors and REFs of two-sided nodes (eq. 5.17 / 5.28) are
 * rad_aggregate_nodes with the face areas as weights (W_G = C_n S_n, the
 * node area of eq. 5.36) for view factors and eps_a S_a for REFs.
 *
 * rad_view_fractions: view fractions (Sec. 5.2.5, eq. 5.27 / 5.29), the
 *   share of each face pair in its node pair's total,
 *   R[a][b] = F[a][b] / sum_{a' in G(a), b' in G(b)} F[a'][b'] (b = nf:
 *   deep space, summed over the faces of G(a)); 0 where that total is 0.
 *   F, R: nf x (nf+1) (ld ldf, ldr >= nf+1).
 * rad_node_emissivity: the emissivity of node G towards node H (App. C,
 *   eq. C.4) that makes GR_GH = eps_GH C_G S_G B_GH with the node REF of
 *   eq. 5.17: eps_GH = sum_{a in G} eps_a S_a sum_{b in H} B_ab /
 *   sum_{a in G} S_a sum_{b in H} B_ab; where the denominator is 0, the
 *   node's area-mean emissivity.  B: nf x (nf+1) face REFs (ld ldb); eps,
 *   area: nf face values (eps in [0, 1], area > 0); E: g x (g+1) (ld lde).
 * Every group must be non-empty and every id in range, eps and area in
 * range; these are checked on the device and reported (RAD_EINVAL,
 * RAD_ENONFINITE) when ``stats`` is non-NULL (which synchronises the stream);
 * after such an error the output is unspecified.
 * work: >= the matching *_workspace_bytes(nf, g), 256-byte aligned.
 */
size_t rad_view_fractions_workspace_bytes(int64_t nf, int64_t g);
int32_t rad_view_fractions(const double* F, int64_t nf, int64_t ldf,
                           const int32_t* group, int64_t g, double* R,
                           int64_t ldr, void* work, size_t work_bytes,
                           rad_stats* stats, void* stream);
size_t rad_node_emissivity_workspace_bytes(int64_t nf, int64_t g);
int32_t rad_node_emissivity(const double* B, int64_t nf, int64_t ldb,
                            const double* eps, const double* area,
                            const int32_t* group, int64_t g, double* E,
                            int64_t lde, void* work, size_t work_bytes,
                            rad_stats* stats, void* stream);

/* ---- steady-state node temperatures ------------------------------------ */
/*
 * Radiation-only steady state of the node heat equation (Sec. 3.4.4,
 * eq. 3.14 with dT/dt = 0 and no conductive couplings), with radiative
 * couplings from REFs, GR_ij = sigma w_i Y_ij (eq. 4.2, w_i = eps_i A_i):
 * every free node i balances its heat input against the power it radiates
 * (eq. 3.12-3.13),
 *   sum_{j<n} GR_ij (T_i^4 - T_j^4) + GR_i,space (T_i^4 - t_space^4) = Q_i,
 * for m load cases at once.  Linear in x = T^4: one LU solve (block LDU
 * without pivoting, the Gebhart solve's kernels) of the balance rows scaled
 * by 1 / (sigma w_i); nodes with a prescribed temperature keep it.
 * Y: n x (n+1) REF matrix, face or node level (ld ldy; column n = space),
 *   entries >= 0; weight: n values w_i > 0 (eps_i A_i, or W_G after
 *   aggregation); Q: n x m heat input per node in W (ld ldq >= m);
 *   t_fixed: n values (nullable = all free): > 0 holds node i at that
 *   temperature, 0 leaves it free; t_space >= 0 (K); sigma > 0 (the
 *   Stefan-Boltzmann constant in the caller's units); T: n x m output (K,
 *   ld ldt >= m); 1 <= m <= RAD_STEADY_MAX_CASES.  All device pointers.
 * precision: RAD_PREC_FP64 or RAD_PREC_FP64_I8 (as in rad_gebhart_ref).
 * factors: >= rad_gebhart_factor_bytes(n, precision), receives the
 *   factorization of the balance matrix; work: >=
 *   rad_steady_temperature_workspace_bytes(n, precision); both 256-byte
 *   aligned.
 * Device checks (reported when ``stats`` is non-NULL, which synchronises
 * the stream): negative or non-finite Y, w, Q or t_fixed, or a free node
 * whose T^4 comes out <= 0 (the heat input is a sink no temperature can
 * balance): RAD_ENONFINITE, with T = NaN there; a free node with no path to
 * space or to a fixed node (singular balance): RAD_ESINGULAR.
 */
#define RAD_STEADY_MAX_CASES 64
size_t rad_steady_temperature_workspace_bytes(int64_t n, int32_t precision);
int32_t rad_steady_temperature(const double* Y, int64_t n, int64_t ldy,
                               const double* weight, const double* Q,
                               int64_t m, int64_t ldq, const double* t_fixed,
                               double t_space, double sigma, double* T,
                               int64_t ldt, int32_t precision, void* factors,
                               size_t factor_bytes, void* work,
                               size_t work_bytes, rad_stats* stats,
                               void* stream);

/* ---- absorbed heat fluxes ----------------------------------------------- */
/*
 * Absorbed heat fluxes from REFs and direct heat fluxes (Sec. 4.2.3,
 * eq. 4.6), for m load cases at once:
 *   Qa[i][c] = A_i eps_i Qd[i][c] + sum_{j<n} B_ji A_j rho_j Qd[j][c].
 * B: n x (n+1) REF matrix (ld ldb; the space column is not read); eps, rho,
 * area: n values; Qd: n x m direct heat flux per unit area (ld ldq >= m);
 * Qa: n x m absorbed power (ld lda >= m); 1 <= m <= RAD_AHF_MAX_CASES.  All
 * device pointers.  B is read once; each sum over j runs in a fixed order
 * (bitwise reproducible).
 * work: >= rad_absorbed_flux_workspace_bytes(n, m), 256-byte aligned.
 */
#define RAD_AHF_MAX_CASES 16
size_t rad_absorbed_flux_workspace_bytes(int64_t n, int64_t m);
int32_t rad_absorbed_flux(const double* B, int64_t n, int64_t ldb,
                          const double* eps, const double* rho,
                          const double* area, const double* Qd, int64_t m,
                          int64_t ldq, double* Qa, int64_t lda, void* work,
                          size_t work_bytes, void* stream);

/* ---- batches of models ------------------------------------------------ */
/*
 * Many independent open models of uneven size, each with one or two spectral
 * bands (e.g. solar and infrared optical properties), enforced and solved
 * together: the same enforcement iteration as rad_enforce_vf (Sec. 3.5.5) on
 * every instance, then the Gebhart REF solve of App. B.2 (eq. B.6-B.11) for
 * every (instance, band), with one kernel launch per step of the shared
 * elimination schedule instead of one per instance.
 *
 * rad_instance (host struct) describes one model; its pointers are device
 * pointers and must stay valid while the plan is used:
 *   F      n x (n+1) view factors (ld ldf >= n+1), enforced in place;
 *   area   n face areas > 0;  n_rays  n ray counts (required for FRACVAR);
 *   bands  1 or 2;  eps[b], rho[b]  n optical properties of band b;
 *   B[b]   n x (n+1) output REF matrix of band b (ld ldb[b] >= n+1).
 *
 * rad_batch_plan_create (host only, no device work) copies the instance list,
 * lays out the workspace and builds the launch schedule; *work_bytes receives
 * the workspace size.  rad_batch_prepare uploads the schedule's descriptor
 * tables into ``work`` (256-byte aligned, >= work_bytes) and waits for the
 * copy.  rad_batch_run then only enqueues kernels on ``stream`` and never
 * synchronizes or copies, so a capture of it in a HIP graph replays the whole
 * batch: enforce_iters enforcement iterations (an instance whose closure
 * defect max_i |s_i - 1| falls to enforce_tol > 0 stops early, decided on the
 * device; enforce_iters = 0 skips enforcement and solves F as given), then
 * the solves, with ir_steps FP64 refinement steps in RAD_PREC_FP32_IR mode
 * (ignored for RAD_PREC_FP64 and RAD_PREC_FP64_I8; in RAD_PREC_FP64_I8 the
 * K = 1024 products of problems larger than one 1024-wide panel run as int8
 * digit products, as in rad_gebhart_ref, and give the same bits as it).  rad_batch_stats (host) waits for ``stream``
 * and fills out[0..count) per instance: iters, converged, closure_defect,
 * recip_err of the enforcement, the largest ir_residual / ir_correction over
 * the bands, device_status; it returns the most negative device status.
 * The workspace holds the plan's state: one run at a time per workspace.
 * rad_batch_plan_destroy frees the host plan (not the workspace).
 */
typedef struct rad_instance {
  double* F;
  int64_t n;
  int64_t ldf;
  const double* area;
  const double* n_rays;
  int32_t bands;
  int32_t reserved;
  const double* eps[2];
  const double* rho[2];
  double* B[2];
  int64_t ldb[2];
} rad_instance;

typedef struct rad_batch_plan rad_batch_plan;

int32_t rad_batch_plan_create(const rad_instance* inst, int32_t count,
                              int32_t precision, int32_t kappa_mode,
                              rad_batch_plan** plan, size_t* work_bytes);
int32_t rad_batch_prepare(rad_batch_plan* plan, void* work, size_t work_bytes,
                          void* stream);
int32_t rad_batch_run(const rad_batch_plan* plan, void* work,
                      double enforce_tol, int32_t enforce_iters,
                      int32_t ir_steps, void* stream);
int32_t rad_batch_stats(const rad_batch_plan* plan, const void* work,
                        rad_stats* out, void* stream);
void rad_batch_plan_destroy(rad_batch_plan* plan);

/* ---- tuning ------------------------------------------------------------ */
/*
 * Process-wide knobs of the kernels (defaults: 0, 0, 1, 0), normally applied
 * by the binding from the autotuner's table (paper_2511_04277_amd/tuning.json):
 *   small_tile_below_f64 / _f32: a GEMM with fewer 128 x 128 output tiles
 *     than this runs with 64 x 64 tiles (more workgroups for narrow or short
 *     products); 0 keeps 128 x 128 everywhere;
 *   lookahead: 1 updates the next panel's columns on the caller's stream and
 *     the rest of the trailing matrix on a second stream during the
 *     factorization; 0 keeps every update on the caller's stream;
 *   side_chunk_tiles: with look-ahead, the second stream's update is issued
 *     as row chunks of at most this many 128 x 128 tiles, so launches of the
 *     caller's stream get dispatched between them; 0 issues one launch.
 * Results do not depend on the knobs beyond rounding of the same operations
 * in the same order per element (they are bitwise identical).  Not
 * synchronised: set them while no call is running.
 */
typedef struct rad_tuning {
  int32_t small_tile_below_f64;
  int32_t small_tile_below_f32;
  int32_t lookahead;
  int32_t side_chunk_tiles;
} rad_tuning;

int32_t rad_tuning_get(rad_tuning* out);
int32_t rad_tuning_set(const rad_tuning* in);

/* ---- kernel profiling --------------------------------------------------- */
/*
 * Optional per-launch timing with HIP events, for measuring the hot kernels
 * against their rooflines.  rad_profile_enable(1) makes the calling host
 * thread bracket every launch of the kernels below with two events on the
 * launch's stream; rad_profile_read waits for the recorded events, writes
 * per-kind totals into out[0..count) and resets them.  flops / bytes are the
 * algorithmic work of the launches (2 M N K flops and one pass over A, B and C
 * for a GEMM, C read too when accumulated; one read and one write
 * of the n x (n+1) matrix for an enforcement sweep; one read of it for an
 * aggregation).  Profiling adds two event records per launch (several
 * microseconds each on gfx950), so rad_profile_kinds restricts the timing to
 * the kinds whose bit (1 << RAD_PROF_*) is set in mask (default: all); the
 * other kinds then run without events.  Both settings are per host thread.
 */
#define RAD_PROF_GEMM_F64 0      /* FP64 MFMA GEMM (factorization, solves, residual) */
#define RAD_PROF_GEMM_F32 1      /* FP32 MFMA GEMM                                   */
#define RAD_PROF_ENFORCE_SWEEP 2 /* enforcement sweep                                */
#define RAD_PROF_DIAG_INVERSE 3  /* Gauss-Jordan inverse of a diagonal block         */
#define RAD_PROF_AGGREGATE 4     /* aggregation reduction                            */
#define RAD_PROF_GEMM_F64_T 5    /* FP64 MFMA GEMM with transposed A (adjoint)       */
#define RAD_PROF_GEMM_F32_T 6    /* FP32 MFMA GEMM with transposed A (adjoint)       */
#define RAD_PROF_GEMM_I8X 7      /* FP64 product emulated with int8 MFMA digit products */
#define RAD_PROF_I8X_SPLIT 8     /* operand scaling and digit split for those products */
#define RAD_PROF_AHF 9           /* absorbed heat fluxes (transposed product with B)    */
#define RAD_PROF_KINDS 10

typedef struct rad_kernel_profile {
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
} rad_kernel_profile;

int32_t rad_profile_enable(int32_t on);
int32_t rad_profile_kinds(uint32_t mask);
int32_t rad_profile_read(rad_kernel_profile* out, int32_t count);

#ifdef __cplusplus
}
#endif
#endif /* RAD_H */
