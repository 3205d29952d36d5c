/*
 * cavmg.h - C ABI of the MI355X (gfx950) CAV-multigrid FGMRES solver for the
 * reduced Eulerian velocity-pressure immersed-boundary system.
 *
 * The system (Gruninger & Griffith, Section 2, Eq. intro_saddle / Eq. Eul_schur):
 *     K_E [u; p] = [b_u; b_p],   K_E = [[A, G], [-D, 0]],
 *     A = A0 - dt E_E,  A0 = (rho/dt) I - mu L,  E_E = S E J,
 * on a periodic N x N MAC grid with h = 1/N.
 *
 * Vector layout (every device vector argument): 3 N^2 doubles, [u | v | p],
 * each block an N x N array indexed [i][j] (i = x index, slowest; j = y index,
 * fastest). u_ij sits at (i h, (j+1/2) h), v_ij at ((i+1/2) h, j h), p_ij at
 * the cell centre. Indices are periodic.
 *
 * Execution model: every call enqueues its work on the context's HIP stream.
 * Calls that return statistics or a solve summary synchronise that stream.
 * A context is not thread safe; separate contexts are independent.
 * Ownership: the caller owns every pointer argument; host descriptors are
 * copied during the call; device vectors must stay valid until the work on
 * the stream has finished. The context owns all hierarchy, patch and factor
 * memory (from the caller's allocator when cav_create was given one) and
 * releases it in cav_destroy.
 * Errors: functions return a cav_status; nothing throws across the ABI.
 * cav_last_error(ctx) gives a message for the most recent failure.
 */
#ifndef CAVMG_H
#define CAVMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cav_ctx_s* cav_ctx;

typedef enum {
  CAV_OK = 0,
  CAV_ERR_INVALID_ARG = 1,     /* malformed descriptor, size or non-finite input */
  CAV_ERR_OUT_OF_MEMORY = 2,
  CAV_ERR_HIP = 3,             /* a HIP runtime call failed */
  CAV_ERR_SINGULAR_PATCH = 4,  /* zero pivot or non-finite value in a patch factorisation */
  CAV_ERR_SINGULAR_COARSE = 5, /* zero pivot in the coarsest direct factorisation */
  CAV_ERR_NOT_BUILT = 6,       /* a stage was called before the stages it depends on */
  CAV_WARN_NOT_CONVERGED = 100,/* FGMRES reached max_it without meeting rtol */
  CAV_WARN_FLOOR_LIMITED = 101 /* estimate met rtol, true residual did not (rounding floor) */
} cav_status;

/* Force laws (per Cartesian component, no coupling between components):
 *  TARGET       E = -kappa_t I                              (Section 5.2)
 *  MEMBRANE     F_k = kappa_s/ds^2 (X_{k+1}+X_{k-1}-2X_k), closed curves (Eq. disc_force_law)
 *  BEAM_CLOSED  F = -kappa_b d^4X/ds^4, centred 5-point stencil, closed curves (Section 5.2)
 *  BEAM_OPEN    E = -(kappa_b/ds^4) D2^T D2 - (kappa_s/ds^2) D1^T D1, open curves
 *               (bending by second differences plus stretching springs, free ends)
 *  CSR          caller supplies E (2M x 2M, component-interleaved: row 2k+c is
 *               marker k, component c); E must be structurally symmetric and
 *               W E symmetric negative semidefinite for the method's guarantees.
 *  FIBRE        the clamped flexible fibre of Section 5.3, linearised at X: with
 *               links D_k = X_{k+1} - X_k and ds = seg_ds[0], the energies
 *               bending    kappa_b/(2 ds^5) sum_k (D_k x D_{k+1})^2,
 *               stretching kappa_s/(2 ds) sum_k (|D_k| - ds)^2,
 *               position   K_p/2 |X_m - (clamp_x, clamp_y)|^2,
 *               tangent    K_t/2 |(X_{m+1} - X_{m-1})/(2 ds) - (1, 0)|^2
 *               (m = clamp_marker) give the force F = -(1/ds) grad(sum), and
 *               E = DF = -(1/ds) Hess(sum) couples the two components.
 *               One open segment, M >= 3, 1 <= m <= M-2; X is taken as given
 *               (unwrapped) in the energies. Every 2 x 2 block of markers at
 *               most two apart is stored, zero or not. */
enum { CAV_LAW_TARGET = 0, CAV_LAW_MEMBRANE = 1, CAV_LAW_BEAM_CLOSED = 2, CAV_LAW_BEAM_OPEN = 3,
       CAV_LAW_CSR = 4, CAV_LAW_FIBRE = 5 };

enum { CAV_FAMILY_CAV = 0, CAV_FAMILY_VANKA = 1, CAV_FAMILY_BOX = 2 };  /* patch families (Section 3) */
/* Smoothers: ADDITIVE is the weighted additive sweep of Appendix A
 * (Eq. additive_cav_saddle, Theta = 1/cnt); MULTIPLICATIVE is the
 * multiplicative Schwarz sweep of Section 3.3 in a coloured order (the
 * shared standard patches in 8 phases by (i + 3j) mod 8, then the patches
 * with E_E entries in greedy colour phases; cav_set_phase_order swaps the two
 * groups); patches in one phase are independent, so the sweep equals the
 * sequential sweep in that order. */
enum { CAV_SMOOTHER_ADDITIVE = 0, CAV_SMOOTHER_MULTIPLICATIVE = 1 };
/* Order of the two groups of phases in every multiplicative sweep. */
enum { CAV_ORDER_EXPLICIT_FIRST = 0, CAV_ORDER_STANDARD_FIRST = 1 };  /* default: STANDARD_FIRST */
enum { CAV_PREC_FP64 = 0, CAV_PREC_MIXED = 1 };            /* factor storage policy */
/* Storage of the explicit patch inverses (cav_set_factor_layout). */
enum { CAV_LAYOUT_FULL = 0, CAV_LAYOUT_SYMMETRIC = 1 };    /* default: FULL */

typedef struct {
  int32_t N;         /* finest cells per side; power of two, N >> (n_levels-1) >= 4 */
  int32_t n_levels;  /* hierarchy depth, >= 1; level 0 is the coarsest */
  double rho, mu, dt;
} cav_grid_desc;

typedef struct {
  int32_t M;               /* number of Lagrangian markers (>= 0) */
  const double* X;         /* host, 2M, interleaved (x_k, y_k); any real values (wrapped periodically) */
  const double* omega;     /* host, M quadrature weights (omega_k = ds for uniform spacing) */
  int32_t law;             /* CAV_LAW_* */
  double kappa_t, kappa_s, kappa_b;
  int32_t n_segments;      /* curves for the built-in laws */
  const int32_t* seg_start;/* host, n_segments+1 marker offsets (first = 0, last = M) */
  const int32_t* seg_closed;/* host, n_segments flags */
  const double* seg_ds;    /* host, n_segments uniform spacings */
  int32_t E_nnz;           /* CAV_LAW_CSR only */
  const int32_t* E_rowptr; /* host, 2M+1 */
  const int32_t* E_col;    /* host, E_nnz */
  const double* E_val;     /* host, E_nnz */
  double K_p, K_t;         /* CAV_LAW_FIBRE only: clamp position and tangent penalties */
  int32_t clamp_marker;    /* CAV_LAW_FIBRE only: the clamped marker m */
  double clamp_x, clamp_y; /* CAV_LAW_FIBRE only: the clamp point */
  const double* X_force;   /* CAV_LAW_FIBRE only, optional host 2M: positions at which the energies
                              (force and tangent) are evaluated, links taken as their differences;
                              NULL = X. Ignored when X_disp is set. Interpolation and spreading
                              always use X (Section 2: S and J at the start of the time step) */
  const double* X_disp;    /* CAV_LAW_FIBRE only, optional host 2M: displacement from X; the energies
                              are evaluated at X + X_disp with the links updated incrementally
                              (Section 5.3), D_k = D_k^0 + (X_disp_{k+1} - X_disp_k), so the bending
                              term of a nearly straight fibre keeps the digits that differences of
                              absolute positions would cancel. The Newton step passes dt J^n u here */
  const double* links;     /* CAV_LAW_FIBRE only, optional host 2(M-1): the link vectors D^0 at X
                              carried by a caller that updates them incrementally between steps;
                              NULL = X_{k+1} - X_k. Not used with X_force (without X_disp) */
} cav_structure_desc;

typedef struct {           /* per smoothed level (index = level, 0 unused) */
  int32_t N;
  int32_t n_patches;       /* one per cell */
  int32_t n_explicit;      /* patches with their own factor (enlarged or touching E_E) */
  int32_t max_np;
  double avg_np;           /* over all patches of the level */
  int64_t sum_np2;         /* over explicit patches */
  int64_t n_touched;       /* unknowns inside at least one explicit patch */
  int64_t ee_nnz;          /* nonzeros of the level's E_E */
} cav_level_stats;

typedef struct {
  int32_t n_fp64;          /* explicit patches stored in FP64 */
  int32_t n_fp32;          /* explicit patches stored in FP32 (mixed policy, kappa_1 <= threshold) */
  double max_cond;         /* largest kappa_1 of an equilibrated patch matrix */
  int64_t factor_bytes;    /* bytes the smoother streams per sweep over all levels */
  double coarse_cond_est;  /* not estimated: always -1 */
} cav_factor_stats;

typedef struct {
  double rtol;             /* relative residual target, e.g. 1e-10 */
  int32_t max_it;          /* iteration cap (no restarts) */
  int32_t use_learned;     /* nonzero: apply the attached learned stage after each V-cycle */
  double* history;         /* optional host array of max_it doubles: estimate after each iteration */
} cav_fgmres_opts;

typedef struct {
  int32_t iterations;      /* preconditioner applications */
  int32_t converged;
  double est_rel_residual; /* Givens estimate at exit */
  double true_rel_residual;/* ||b - K x|| / ||b|| evaluated in FP64 after the solve */
  double pressure_mean_removed; /* mean of the pressure RHS that was projected out */
  int32_t learned_accepted, learned_rejected;
} cav_solve_info;

/* ---- lifecycle ---- */
/* Device memory source of a context or net. alloc(bytes, stream, user) returns
 * a device block of at least `bytes` bytes on the object's device, usable by
 * work enqueued on `stream` (the object's current stream) from then on, or
 * NULL (the call that needed it then fails with CAV_ERR_OUT_OF_MEMORY).
 * free(ptr, stream, user) returns a block the object no longer needs: work
 * already enqueued on `stream` may still use it (the library first orders its
 * own side streams before `stream`), so the allocator may hand it out again
 * only to work ordered after that work, as a stream-ordered caching allocator
 * (PyTorch's, for one) does. Both are called from the thread that called into
 * the library, never from a device callback. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} cav_allocator;
/* Creates a context on `device` that enqueues its work on `hip_stream`. With
 * `allocator` (copied; its functions must stay valid until cav_destroy) all of
 * the context's device memory (operator, hierarchy, patch tables, factors,
 * Krylov and smoother workspaces) comes from it and is returned to it; NULL
 * makes the context call hipMalloc itself. CAV_ERR_INVALID_ARG for a bad device or an
 * allocator without both functions. Either way, blocks the context releases
 * stay with it (up to 8 GiB) for later requests of the same size and go back
 * to their source in cav_destroy or when an allocation fails. */
cav_status cav_create(cav_ctx* out, int device, void* hip_stream, const cav_allocator* allocator);
cav_status cav_destroy(cav_ctx ctx);
cav_status cav_set_stream(cav_ctx ctx, void* hip_stream);
const char* cav_status_string(cav_status s);
const char* cav_last_error(cav_ctx ctx);
/* Device memory held by a context: blocks handed out and not yet released
 * (live), released blocks kept for reuse (cached), and the numbers of
 * hipMalloc calls the context made itself and
 * of calls to the caller's allocator (0 and 0 respectively when there is
 * none). Host only; does not synchronise. */
typedef struct {
  int64_t live_bytes, live_blocks, cached_bytes;
  int64_t hip_malloc_calls, allocator_allocs, allocator_frees;
} cav_memory_info;
cav_status cav_memory_stats(cav_ctx ctx, cav_memory_info* out);

/* ---- setup (Section 2, Section 3, Section 4) ----
 * cav_build_operator: assembles J (4-point kernel, fixed 4x4 face box per
 *   marker and component), E for the chosen law, E_E = S E J on the finest
 *   level, the Galerkin coarse E_E^(l-1) = R E_E^(l) P on every coarser level
 *   (R = P^T/4, RT0 velocity prolongation), and the rediscretised Stokes
 *   stencils. Validates the grid (power of two, levels), finite X and E.
 * cav_build_cav_patches: one patch per cell on every level except the
 *   coarsest (Eq. cav_patch_set for CAV_FAMILY_CAV; the standard Vanka patch
 *   for CAV_FAMILY_VANKA), read from the structural pattern of the level's
 *   E_E. `out` (optional) receives n_levels entries.
 * cav_factor_patches: assembles every explicit patch matrix K_p = R_p K_E R_p^T,
 *   applies one row then column max-norm equilibration (powers of two), inverts
 *   it by Gauss-Jordan elimination with partial pivoting, folds the scalings
 *   into the stored inverse and records kappa_1 (Section 3.3). Patches with no
 *   E_E entry share one 5x5 inverse per level. Under CAV_PREC_MIXED a patch
 *   whose kappa_1 <= cond_threshold is stored in FP32. Also forms the
 *   coarsest level's solution operator: the solution of the bordered system
 *   [[K_0, e], [e^T, 0]] (e = constant pressure) on (u, p), computed as the
 *   inverse of the quasi-definite [[A, G], [G^T, -gamma e e^T]] with the
 *   pressure mean removed from its columns (same u, p up to a multiple of e). */
cav_status cav_build_operator(cav_ctx ctx, const cav_grid_desc* grid, const cav_structure_desc* st);
cav_status cav_build_cav_patches(cav_ctx ctx, int family, cav_level_stats* out);
/* B(b,o) box family (Section 3.1): one patch per b x b block of cells (block
 * lower-left cells (i, j) with i, j multiples of b), the union of the Vanka
 * patches of the block expanded by o cells in every direction; smoothing
 * injects each box's correction only into the unknowns of its unexpanded
 * block (restricted injection, Section 3.3), so adjacent blocks both write
 * their shared faces. Both smoothers apply (additive: sum of injected
 * corrections; multiplicative: boxes in greedy colour phases on the K_E
 * conflict graph, block order). Every smoothed grid must be a multiple of b.
 * Patch exports list the box dofs at its block's lower-left cell and nothing
 * elsewhere; out[l].n_patches is the number of boxes. */
cav_status cav_build_box_patches(cav_ctx ctx, int b, int o, cav_level_stats* out);
cav_status cav_factor_patches(cav_ctx ctx, int precision, double cond_threshold, cav_factor_stats* out);
/* Layout of the stored patch inverses, used from the next cav_factor_patches
 * on (layout = CAV_LAYOUT_*). K_E is symmetric (Eq. intro_saddle with the
 * divergence -D = G^T; A and E_E = S E J symmetric), so every K_p = R_p K_E
 * R_p^T and its inverse are symmetric. CAV_LAYOUT_FULL stores all n_p^2
 * entries, column-major. CAV_LAYOUT_SYMMETRIC stores n_p^2 / 2 + 8 n_p of
 * them: for panel k = 0 .. ceil(n_p/16) - 1, columns 16k .. 16k + w - 1
 * (w = min(16, n_p - 16k)) on rows 16k .. n_p - 1, column-major inside the
 * panel with column stride n16 - 16k (n16 = n_p rounded up to a multiple of
 * 16, so columns start on 16-entry boundaries; the padding is never read),
 * panels consecutive (panel k starts at 16 k n16 - 128 k (k - 1));
 * entries above the panels' diagonal 16 x 16 blocks are taken from their
 * mirror images (the computed inverse is symmetric up to rounding). Only the
 * additive smoother reads the symmetric layout: with it, a V-cycle, sweep or
 * solve on a level whose smoother is multiplicative, and cav_autotune,
 * return CAV_ERR_INVALID_ARG. factor_bytes counts the stored entries. */
cav_status cav_set_factor_layout(cav_ctx ctx, int layout);
/* Smoother choice (kind = CAV_SMOOTHER_*). Additive (Appendix A,
 * Eq. additive_cav_saddle): w <- w + alpha sum_p R_p^T Theta_p K_p^{-1} R_p (b - K w),
 * Theta_p = diag(1/cnt). Multiplicative (Section 3.3): for each patch in the
 * coloured order, w <- w + alpha R_p^T K_p^{-1} R_p (b - K w). A stand-alone
 * sweep (cav_level_apply) removes the mean pressure after it; inside a
 * V-cycle the mean is removed once, after the top level's last sweep (K_E
 * does not see a constant pressure, so the cycle's output is the same up to
 * rounding). pre/post = sweeps per V-cycle leg, each starting from the iterate
 * the previous one left (the paper's cycle is (1, 1)). */
cav_status cav_set_smoother(cav_ctx ctx, int kind, double alpha, int pre, int post);
/* Multiplicative phase order (reading: the paper visits patches
 * lexicographically, Section 3.3): CAV_ORDER_STANDARD_FIRST (default) runs
 * the 8 colours of shared standard patches, then the colour phases of patches
 * with E_E entries; CAV_ORDER_EXPLICIT_FIRST the reverse. Both are valid
 * multiplicative orders; they differ in robustness at high stiffness (the
 * standard-first two-grid cycle stays contracting on Table 1's stiffest
 * membrane where the other diverges, and it needs fewer FGMRES iterations on
 * stiff open fibres). Cleared only by another call. */
cav_status cav_set_phase_order(cav_ctx ctx, int order);
/* Bound of every workgroup-barrier wait of the cooperative phase forms and
 * the one-launch sweep, in polls (default 2^21, about a second). A wait that
 * reaches it gives up: its workgroup leaves x unwritten, the kernel finishes,
 * and the next FGMRES solve returns CAV_ERR_HIP (the flag is then cleared).
 * A tiny bound forces that path, for tests of the failure handling. */
cav_status cav_set_wait_limit(cav_ctx ctx, uint32_t polls);
/* Per-level override (kind -1 restores the context's choice): level in
 * 1 .. n_levels-1 uses `kind` with damping `alpha`, e.g. the multiplicative
 * sweep on the finest level and the additive one below it. Cleared by
 * cav_build_operator. */
cav_status cav_set_level_smoother(cav_ctx ctx, int level, int kind, double alpha);

/* ---- application ---- */
/* y = K_E x on the finest level (x, y device, 3N^2, must not alias). */
cav_status cav_apply_operator(cav_ctx ctx, const double* x, double* y);
/* z = V(r): one V(pre,post)-cycle on the finest level (Section 4). */
cav_status cav_vcycle(cav_ctx ctx, const double* r, double* z);
/* Z_q = V(R_q) for k right-hand sides (R, Z device, column-major, k columns
 * of 3N^2, must not alias; k = 0 does nothing): the cycle of cav_vcycle on
 * blocks of 16 columns. Each explicit-patch phase of the multiplicative
 * smoother applies every stored inverse to all columns of a block in one
 * launch as FP64 MFMA products (the inverse is read once per block, not once
 * per column); the other steps run per column. Results agree with cav_vcycle
 * column by column up to summation order (FP64 rounding). Allocates three
 * 16-column buffers per level on first use. */
cav_status cav_vcycle_multi(cav_ctx ctx, int32_t k, const double* R, double* Z);
/* Right-preconditioned FGMRES from x0 = 0 (Section 5): one V-cycle per
 * iteration, CGS2 orthogonalisation with fixed-order reductions, Givens
 * rotations; stops when the estimate <= rtol or on exact breakdown. b is
 * not modified; a nonzero pressure mean in b is projected out and reported.
 * Returns CAV_WARN_NOT_CONVERGED at max_it and CAV_WARN_FLOOR_LIMITED when the
 * estimate met rtol but the true FP64 residual exceeds 10 * rtol. */
cav_status cav_fgmres_solve(cav_ctx ctx, const double* b, double* x, const cav_fgmres_opts* opts,
                            cav_solve_info* info);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * cav_fgmres_solve with the same arguments, kernels and results, whose Krylov
 * workspace lives in a fixed device scratch of 512 MiB that the library holds
 * per device until the process ends (looked up by cav_create), so the call
 * makes no hipMalloc, hipFree or other device allocation. The workspace needs
 * (2 max_it + 3) 3N^2 doubles plus O(max_it) partials (e.g. max_it <= 40 at
 * 512^2, <= 166 at 256^2); larger requests return CAV_ERR_INVALID_ARG with the
 * sizes in cav_last_error. use_learned must be 0 (CAV_ERR_INVALID_ARG
 * otherwise) and no live-timing events are recorded. The context must be
 * built and factored as for cav_fgmres_solve. Every context on one device
 * shares that device's scratch: calls that overlap on one device (other host
 * threads, other streams) race and must be serialised by the caller; each call
 * initialises every part of the scratch it reads. */
cav_status cav_fgmres_solve_noalloc(cav_ctx ctx, const double* b, double* x, const cav_fgmres_opts* opts,
                                    cav_solve_info* info);

/* ---- implicit IB step with a nonlinear force (Section 2 scheme, Section 5.3) ----
 * Interpolation U = J u (Section 2, Eq. intro_saddle) at the positions X of the
 * last cav_build_operator: x device 3N^2 (u, v, p), U device 2M (interleaved).
 * Spreading y_u += S F = h^-2 J^T W F: F device 2M, y device 3N^2 (velocity
 * blocks updated, pressure untouched; each face sums its markers in a fixed
 * order). Both need cav_build_operator; M = 0 is a no-op. */
cav_status cav_ib_interpolate(cav_ctx ctx, const double* x, double* U);
cav_status cav_ib_spread_add(cav_ctx ctx, const double* F, double* y);
/* Host: the fibre law's force density F = -(1/ds) grad(energies) at X_force
 * (else X), F host 2M interleaved (Section 5.3). CAV_ERR_INVALID_ARG for other
 * laws or an invalid descriptor. */
cav_status cav_structure_force(const cav_structure_desc* st, double* F);

typedef struct {
  double rtol, atol;       /* stop when ||R|| <= rtol ||R_0|| or ||R|| <= atol (2-norms) */
  int32_t max_newton;      /* Newton corrections at most */
  double lin_rtol;         /* FGMRES tolerance of every Newton system */
  int32_t lin_max_it;
  int32_t family;          /* CAV_FAMILY_*, rebuilt for every Newton system */
  int32_t precision;       /* CAV_PREC_* */
  double cond_threshold;
  int32_t smoother;        /* CAV_SMOOTHER_* */
  double alpha;
} cav_newton_opts;

typedef struct {
  int32_t newton_its;      /* corrections taken */
  int32_t converged;
  int32_t fgmres_its_total, fgmres_its_max;
  double res0, res;        /* ||R|| at the initial and the final iterate */
  int32_t lin_unconverged; /* Newton systems whose FGMRES stopped at lin_max_it (their
                              corrections are still applied: inexact Newton) */
  int32_t failed_stage;    /* 0: none; on an error status, the stage that failed:
                              1 operator build, 2 patches, 3 factorisation, 4 FGMRES,
                              5 residual or force evaluation */
} cav_newton_info;

/* One backward-Euler step of the IB scheme of Section 2 with the fibre law
 * (Section 5.3), solved by Newton's method: unknowns x = (u, p) (device 3N^2,
 * in: initial guess, out: solution), X^{n+1} = X^n + dt J^n u with J^n, S^n at
 * st->X = X^n, and the residual
 *   R(x) = K_0 x - S^n F(X^n + dt J^n u) - rhs,
 * K_0 the Stokes part of Eq. intro_saddle (A_0 = rho/dt I - mu L, G, -D) and
 * rhs device 3N^2 (rho/dt u^n plus any explicit terms; pressure part, whose
 * mean must be zero: constant pressure is outside the range of K_0, so a
 * nonzero mean would leave a residual no correction removes). Each
 * correction rebuilds the whole hierarchy with E = DF at the current
 * iterate, the energies evaluated at X^n + dt J^n u with the links updated
 * incrementally from st->links (else from X^n) by dt J^n u (st->X_force and
 * st->X_disp ignored; the operator is kept when the iterate's displacement is
 * the one it was built at) and solves K_E dx = -R with
 * CAV-preconditioned FGMRES (lin_rtol) from zero. X_new: optional host 2M, X^{n+1} at the
 * solution. The context keeps the hierarchy of the last Newton system.
 * A Newton system whose FGMRES reaches lin_max_it without meeting lin_rtol
 * still yields its correction (the best of its Krylov space: inexact Newton)
 * and is counted in info->lin_unconverged. CAV_WARN_NOT_CONVERGED only if
 * max_newton corrections do not meet the Newton tolerance; an error status of
 * a stage (build, patches, factorisation, FGMRES, residual) is returned as is
 * with info->failed_stage naming the stage. After any status x holds the last
 * iterate, info the counts and residuals reached so far, and X_new (when the
 * step got as far as a residual evaluation) the configuration of that iterate. */
cav_status cav_newton_solve(cav_ctx ctx, const cav_grid_desc* g, const cav_structure_desc* st, const double* rhs,
                            double* x, double* X_new, const cav_newton_opts* opts, cav_newton_info* info);

/* ---- graph execution and batches of independent systems ----
 * cav_fgmres_solve_graph: the same solve as cav_fgmres_solve (same kernels,
 * reductions and results), with the whole iteration body (V-cycle, K_E apply,
 * CGS2, Givens rotations, next basis vector) captured once into a hipGraph
 * and replayed; the iteration index, rotations and done flag live in device
 * memory, and the host reads one flag per iteration. The graph is captured on
 * a stream the context owns, ordered after the caller's stream, and is
 * re-captured after any setup call. use_learned must be 0.
 * cav_batch_solve: solves n_sys independent systems (ctxs[i], b[i] -> x[i],
 * device vectors of each context's finest size) by rounds: each round runs one
 * iteration of every unfinished system. mode 0 captures the active systems'
 * bodies as parallel branches of ONE graph (one launch per round), recaptured
 * when a quarter of its systems have finished (finished systems replay their
 * last iteration without changing their state); mode 1 launches each system's
 * own graph on its own stream. infos (optional) receives n_sys summaries;
 * returns the first non-OK status of any system. Contexts must be distinct,
 * factored and on one device; synchronises. */
typedef struct {
  int32_t rounds;          /* rounds (iterations of the slowest system) */
  int32_t graph_launches;  /* hipGraphLaunch calls */
  int32_t captures;        /* graph captures */
  int64_t iterations;      /* FGMRES iterations summed over systems */
} cav_batch_stats;
cav_status cav_fgmres_solve_graph(cav_ctx ctx, const double* b, double* x, const cav_fgmres_opts* opts,
                                  cav_solve_info* info);
cav_status cav_batch_solve(cav_ctx* ctxs, int32_t n_sys, const double* const* b, double* const* x,
                           const cav_fgmres_opts* opts, cav_solve_info* infos, int32_t mode,
                           cav_batch_stats* stats);

/* ---- autotuning ----
 * The multiplicative sweep launches one kernel per colour phase; each patch
 * of a phase gets one workgroup of 256, 512 or 1024 threads, or (entry 0) the
 * split form: its residual rows and GEMV row blocks spread over several
 * workgroups in two launches, or (entries 1 and 2) the cooperative form: one
 * launch in which a patch of n rows gets ceil(n / 64) or ceil(n / 128)
 * workgroups that each form all residual rows, meet at a bounded barrier on a
 * per-patch counter, and apply 64 or 128 rows of the inverse, or (entry 3,
 * the default for every bucket) the cooperative form with a shared residual:
 * each of the ceil(n / 64) workgroups forms only its own 64 residual rows,
 * exchanged through device-coherent stores and loads after the barrier
 * (inside a captured graph the one-workgroup form runs instead of any
 * cooperative form). Alternatively the whole sweep of a level runs in one
 * cooperative launch with a bounded grid barrier after each phase, or every
 * explicit phase of a sweep runs in one dataflow launch:
 * workgroups claim the 64-row items of the shared-residual form in phase
 * order from a ticket counter, and an item of patch p starts once every
 * patch of an earlier colour that conflicts with p (shares an unknown or a
 * K_E coupling) has finished the sweep, signalled through per-patch done
 * counters with device-scope release and acquire; non-conflicting patches
 * commute, so the sweep equals the per-phase form bit for bit (inside a
 * captured graph the per-phase forms run instead).
 * cav_autotune times the choices on the context's own phases, per smoothed
 * level and per size bucket of a phase's largest patch (<= 64, <= 128,
 * <= 256, larger), `reps` repetitions each, keeps the fastest, and writes the
 * table (5 ints per level, levels 0 .. n_levels-1, level 0 unused: 4 bucket
 * entries, then the sweep entry: 0 a launch per phase with the bucket
 * entries, 1 the one-launch sweep, 2 the dataflow sweep; the autotuner times
 * 0 against 2 per level and never picks 1: a process's first cooperative
 * launch slows later concurrent graph launches, and that sweep never won) to
 * `table` (optional). Results do
 * not depend on the choice (every patch's and cell's arithmetic is the same).
 * Uses the levels' scratch vectors; synchronises. A barrier wait that times
 * out (cooperative phase form or one-launch sweep) leaves x unwritten from
 * that point and makes the next FGMRES solve return CAV_ERR_HIP. cav_set_tuning applies a stored table, e.g. one cached in a
 * file by the caller. */
cav_status cav_autotune(cav_ctx ctx, int32_t reps, int32_t* table);
cav_status cav_set_tuning(cav_ctx ctx, const int32_t* table);

/* ---- error propagation (Section 5.1, Table 1 diagnostic) ----
 * T_q = X_q - V(K_E X_q) for the k columns X_q (device, column-major, each a
 * finest-level vector): the V-cycle's iteration matrix applied to X. With a
 * two-level hierarchy and X = I this assembles the two-grid iteration matrix
 * whose spectrum Table 1 reports. The cycles run as in cav_vcycle_multi.
 * Enqueued on the context's stream. */
cav_status cav_error_propagation(cav_ctx ctx, int32_t k, const double* X, double* T);

/* ---- per-level access for parity checks ----
 * op: 0 y = K_l x; 1 y = R_l x (level l -> l-1, y on level l-1);
 *     2 y = P_l x (level l-1 -> l, x on level l-1, y on level l);
 *     3 y = S_l(b = x, w = 0) one smoother sweep from zero;
 *     4 y = coarse direct solve (level 0 only);
 *     5 y = V-cycle starting at level l. Device vectors of the level's size. */
cav_status cav_level_apply(cav_ctx ctx, int level, int op, const double* x, double* y);
/* Size of level l's grid (cells per side), or 0. */
int32_t cav_level_N(cav_ctx ctx, int level);
/* Patch sets of level l copied to host: offsets (n_patches+1, int64) and
 * unknown indices (sorted ascending inside each patch). Pass NULL dofs to
 * query the total length through *total. */
cav_status cav_export_patches(cav_ctx ctx, int level, int64_t* offsets, int32_t* dofs, int64_t* total);
/* Multiplicative phases of level l: phases of explicit patches as seed-cell
 * indices (ptr has n_phases+1 offsets into cells). NULL arrays query the sizes.
 * The 8 phases of shared standard patches follow them in every sweep
 * (precede them under CAV_ORDER_STANDARD_FIRST). */
cav_status cav_export_phases(cav_ctx ctx, int level, int32_t* ptr, int32_t* cells, int32_t* n_phases,
                             int32_t* n_cells);

/* ---- host-only analysis (no device needed) ----
 * cav_analyze runs the host part of the setup (force law, E_E = S E J,
 * Galerkin coarsening, patch families, multiplicative phases) exactly as
 * cav_build_operator + cav_build_cav_patches do, and keeps the result in a
 * host handle whose levels can be exported like a context's. */
typedef struct cav_analysis_s* cav_analysis;
cav_status cav_analyze(const cav_grid_desc* grid, const cav_structure_desc* st, int family, cav_analysis* out);
cav_status cav_analyze_box(const cav_grid_desc* grid, const cav_structure_desc* st, int b, int o, cav_analysis* out);
cav_status cav_analysis_destroy(cav_analysis a);
cav_status cav_analysis_export_ee(cav_analysis a, int level, int64_t* rowptr, int32_t* col, double* val,
                                  int64_t* nnz);
cav_status cav_analysis_export_patches(cav_analysis a, int level, int64_t* offsets, int32_t* dofs, int64_t* total);
cav_status cav_analysis_export_phases(cav_analysis a, int level, int32_t* ptr, int32_t* cells, int32_t* n_phases,
                                      int32_t* n_cells);
/* per-unknown touched list of level l: unknowns inside explicit patches and 1/cnt */
cav_status cav_analysis_export_weights(cav_analysis a, int level, int32_t* dofs, double* inv_cnt, int32_t* n_touched);

/* ---- live timing ----
 * Between cav_kernel_timing(ctx, 1, NULL) and a later call, the library
 * records HIP events on its stream around the explicit-patch kernels (the
 * smoother's dominant kernels): one pair around each additive GEMV launch and
 * one pair around each run of consecutive multiplicative phase launches of
 * one kernel form (per sweep and level), plus one pair around every top-level
 * V-cycle. A bracket's duration includes the dispatch gaps between the
 * launches it holds; the coop_* fields repeat the totals of the brackets of
 * cooperative-form launches.
 * A call with out != NULL synchronises the stream and returns the totals
 * since recording started; every call clears the records; enable = 0 stops. */
typedef struct {
  int64_t launches;        /* explicit-patch kernel launches inside the brackets */
  double ms;               /* summed bracket durations */
  double bytes;            /* their summed algorithmic bytes: sum_p n_p^2 s + 20 n_p */
  int64_t vcycles;         /* top-level V-cycles */
  double vcycle_ms;        /* their summed durations */
  int64_t coop_launches;   /* of the above: cooperative-form phase launches */
  double coop_ms;
  double coop_bytes;
  int64_t shared_launches; /* of those: the shared-residual form (entry 3) */
  double shared_ms;
  double shared_bytes;
  int64_t flow_launches;   /* dataflow sweeps (one launch per level sweep); not in coop_* */
  double flow_ms;
  double flow_bytes;       /* the algorithmic bytes of every phase of those sweeps */
} cav_kernel_timing_info;
cav_status cav_kernel_timing(cav_ctx ctx, int enable, cav_kernel_timing_info* out);

/* ---- learned correction stage ----
 * The paper has no learned component; this stage is an extra, optional part
 * of the variable preconditioner that flexible GMRES (Section 5) admits.
 * Net N: R^{3 x N x N} -> R^{3 x N x N}, three periodic 3x3 cross-correlations
 *   y1 = W1 * x, a1 = relu(y1); y2 = W2 * a1, a2 = relu(y2); y3 = W3 * a2,
 *   out[co,i,j] = sum_{ci,a,c} W[co,ci,a,c] x[ci, i+a-1, j+c-1] (mod N),
 * channels 3 -> 32 -> 32 -> 3, no biases. Channels 0, 1, 2 of a sample are the
 * u, v, p blocks of a grid vector (each [i][j]), so a sample is laid out
 * exactly like a solver vector. Master weights are FP32, flat, in the order
 * W1 (32,3,3,3), W2 (32,32,3,3), W3 (3,32,3,3), C-ordered: CAV_NET_WEIGHTS
 * numbers. Kernels round weights, the input and both hidden activations to
 * bfloat16 (nearest even, from FP32) and accumulate in FP32.
 * The net handle owns its weights, Adam state and activation buffers; it is
 * not thread safe; it may be attached to several contexts on its device. */
#define CAV_NET_WEIGHTS 10944
typedef struct cav_net_s* cav_net;
/* weights zero; `allocator` as for cav_create (NULL: hipMalloc) */
cav_status cav_net_create(cav_net* out, int device, void* hip_stream, const cav_allocator* allocator);
cav_status cav_net_destroy(cav_net net);
cav_status cav_net_set_stream(cav_net net, void* hip_stream);
const char* cav_net_last_error(cav_net net);
/* w: host, CAV_NET_WEIGHTS finite floats (copied). Resets the Adam state. */
cav_status cav_net_set_weights(cav_net net, const float* w);
/* Copies the master weights and/or the gradient of the last training step to
 * host arrays of CAV_NET_WEIGHTS floats (either may be NULL); synchronises. */
cav_status cav_net_get_weights(cav_net net, float* w, float* grad);
/* out_b = N(in_b), b < batch. in, out: device FP32, batch x 3 x N x N, N a
 * power of two in [8, 32768]. */
cav_status cav_net_forward(cav_net net, int32_t N, int32_t batch, const float* in, float* out);
/* FP64 correction of one residual: c = ||r|| N(r / ||r||), then the mean of c's
 * pressure block is removed (c = 0 when r = 0). r, c: device, 3N^2 doubles. */
cav_status cav_net_correct(cav_net net, int32_t N, const double* r, double* c);
/* One Adam step (beta 0.9/0.999, eps 1e-8, bias-corrected) on the loss
 *   L = (1/B) sum_b ||N(rhat_s) - ehat_s||^2 / ||ehat_s||^2,  s = index[b]
 * (s = b when index is NULL). rhat, ehat: device FP32, n_samples x 3 x N x N;
 * index: host, batch sample numbers in [0, n_samples). loss (host, optional)
 * receives L before the update; the call synchronises. */
cav_status cav_net_train_step(cav_net net, int32_t N, int32_t batch, const float* rhat, const float* ehat,
                              const int32_t* index, int64_t n_samples, double lr, double* loss);
/* Same Adam step on a loss through K = the finest-level K_E of ctx (N = the
 * context's finest grid; K_E is symmetric, so K^T = K in the gradients),
 * with c_s = N(rhat_s), s = index[b]:
 *   kind 0 (residual):          L = (1/B) sum_b ||K c_s - rhat_s||^2 / ||rhat_s||^2
 *   kind 1 (minimal residual):  L = (1/B) sum_b (1 - <K c_s, rhat_s>^2 / (||K c_s||^2 ||rhat_s||^2)),
 * i.e. the squared residual left by the best multiple of c_s, which is what
 * the FGMRES stage's minimal-residual step achieves; it is invariant to the
 * scale of c_s. Since K ehat = rhat both measure the pair's error through K.
 * The work runs on the context's stream; the call synchronises. */
cav_status cav_net_train_step_residual(cav_net net, cav_ctx ctx, int32_t kind, int32_t batch, const float* rhat,
                                       const int32_t* index, int64_t n_samples, double lr, double* loss);
/* Training pairs from the context's V-cycle: for each exact solution x*_q
 * (device, count x 3N^2), b = K x*, x_0 = 0, x_k = x_{k-1} + V(b - K x_{k-1});
 * after iteration k (1..iters) writes rhat = r_k/||r_k||, ehat = (x* - x_k)/||r_k||
 * with r_k = b - K x_k, as FP32 at sample q*iters + k-1 of rhat/ehat (device,
 * count*iters x 3N^2). The solutions run in blocks of 16 through the cycle
 * of cav_vcycle_multi. Synchronises. */
cav_status cav_learned_pairs(cav_ctx ctx, int32_t count, const double* xstar, int32_t iters, float* rhat,
                             float* ehat);
/* Attach (or detach with NULL) a net for cav_fgmres_solve with use_learned.
 * Each iteration then computes z0 = V(v), r' = v - K z0, c = cav_net_correct(r'),
 * gamma = <r', Kc>/||Kc||^2 and takes z = z0 + gamma c when
 * <r', Kc>^2/||Kc||^2 >= margin ||r'||^2 (the V-cycle judges the correction),
 * otherwise z = z0. The net must match the finest grid. margin in [0, 1). */
cav_status cav_attach_net(cav_ctx ctx, cav_net net, double margin);

/* E_E of level l (unscaled, symmetric) as host CSR over the 2N_l^2 velocity
 * unknowns: rowptr (2N_l^2+1), col, val; NULL col/val queries *nnz. */
cav_status cav_export_ee(cav_ctx ctx, int level, int64_t* rowptr, int32_t* col, double* val, int64_t* nnz);

#ifdef __cplusplus
}
#endif
#endif /* CAVMG_H */
