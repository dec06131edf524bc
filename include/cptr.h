/*
 * cptr.h -- C ABI of the MI355X (gfx950) CPTR-FGMRES library (libcptr.so).
 *
 * The library solves the linearised fully implicit thermal multiphase system
 * A dx = b of one Newton iterate (Section 3, eq:AXR), where A is stored cell by
 * cell as nv x nv blocks (nv = 3: p, S_w, T; nv = 4: p, S_w, S_g, T), with
 * right-preconditioned flexible GMRES and the two-stage constrained
 * pressure-temperature residual (CPTR) preconditioner of Section 3.2:
 *   first stage  M1^{-1} = [A00~^{-1} 0; 0 0], A00 the pressure-temperature
 *                submatrix (eq:A00), A00~^{-1} the block preconditioner of
 *                eq:Aschur with its Schur-complement approximation S~_T (eq:Se),
 *                each inverse one algebraic-multigrid V-cycle;
 *   second stage block ILU(0) of the full matrix (or ILU(1), or the learned
 *                stage of cptr_learn.h);
 *   combination  x1 = M1^{-1} v, b1 = v - A x1, z = M2^{-1} b1 + x1
 *                ("Two-stage preconditioners", Section 3).
 * Other first stages: CPR (Section 3.1, pressure only, optionally with a
 * Quasi-/True-IMPES decoupling operator), the block lower-triangular and
 * block-diagonal (Section 4.4) variants of the block preconditioner, and the
 * unknown-based AMG of the pressure-temperature block (Section 3.4).
 *
 * Conventions shared by every entry point
 *   - All matrix and vector pointers are DEVICE pointers (HIP memory on the
 *     current device) unless stated otherwise.  Host arrays are named *_host.
 *   - BSR: int32 row_ptr[n+1], int32 col_idx[nnzb] (ascending within a row,
 *     diagonal block present), double vals[nnzb*nv*nv] with each block
 *     row-major: vals[k*nv*nv + r*nv + c] = d(equation r of the row cell) /
 *     d(unknown c of the column cell).  The pattern must be structurally
 *     symmetric (cell graph).  Vectors are interleaved: x[i*nv + u].
 *   - Row/column slot ip (default 0) is the weighted, scaled pressure equation
 *     and pressure unknown (eq:weighted, eq:scaling); slot iT (default nv-1)
 *     is the energy equation and temperature unknown.
 *   - S~_T is a scalar CSR matrix on the cell graph (int32/int32/double),
 *     assembled by the caller from eq:Se; it cannot be recovered from A alone.
 *     The options also offer two algebraic approximations formed from A
 *     (cptr_options.schur), for which no S~_T is passed.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *   - Return values: 0 = CPTR_OK, > 0 informational, < 0 error.  No C++
 *     exception crosses this interface.  cptr_last_error() gives the message
 *     of the last failure on the calling thread.
 *   - A handle is not thread safe; distinct handles may be used concurrently
 *     on distinct streams.
 */
#ifndef CPTR_H
#define CPTR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPTR_OK 0
#define CPTR_NOT_CONVERGED 1
#define CPTR_ERR_INVALID_ARG (-1)
#define CPTR_ERR_UNSUPPORTED (-2)
#define CPTR_ERR_NONFINITE (-3)
#define CPTR_ERR_SINGULAR_BLOCK (-4)
#define CPTR_ERR_OOM (-5)
#define CPTR_ERR_HIP (-6)
#define CPTR_ERR_SETUP (-7)

/* first stage */
#define CPTR_FIRST_NONE 0        /* x1 = 0 */
#define CPTR_FIRST_BLOCK 1       /* CPTR-Block: the five steps of eq:Aschur */
#define CPTR_FIRST_BLOCK_LOWER 2 /* left factor of eq:Aschur dropped: the inverse of the block
                                    lower-triangular [A_pp 0; A_Tp S~_T] (steps 1-3 of the five,
                                    d_p = x_p) */
#define CPTR_FIRST_CPR 3         /* CPR: x1 = R_p^T V(A_pp) R_p v */
#define CPTR_FIRST_BD 4          /* CPTR-BD(AMG) (Section 4.4): block-diagonal first stage,
                                    d_p = V(A_pp) b_p, d_T = V(A_TT) b_T (couplings left out) */
#define CPTR_FIRST_UAMG 5        /* CPTR-uAMG (Section 3.4): (d_p; d_T) = V(A_00) (b_p; b_T), one
                                    V-cycle of an unknown-based hierarchy of the coupled
                                    pressure-temperature block in unknown-wise order (each unknown
                                    coarsened on its own diagonal block, couplings kept in the
                                    Galerkin coarse operators) */
#define CPTR_FIRST_BLOCK_UPPER 6 /* right factor of eq:Aschur dropped: the inverse of the block
                                    upper-triangular [A_pp A_pT; 0 S~_T]: d_T = V(S~_T) b_T,
                                    d_p = V(A_pp) (b_p - A_pT d_T) */

/* Decoupling operators G = [I, -D; 0, I] (Section 3.1).  CPR: p = pressure,
 * s = every other unknown in slot order, D one 1 x (nv-1) block per cell; the
 * first stage solves S_p = A_pp - D A_sp with b_p = v_p - D v_s.  CPTR-uAMG
 * (the pressure-temperature extension of Section 3.2): 0 = (p, T), s = the
 * saturations, D one 2 x (nv-2) block per cell; the first stage solves
 * S_0 = A_00 - D A_s0 with b_0 = v_0 - D v_s. */
#define CPTR_DECOUPLE_NONE 0
#define CPTR_DECOUPLE_QI 1       /* Quasi-IMPES: D = diag(A_0s) diag(A_ss)^-1 */
#define CPTR_DECOUPLE_TI 2       /* True-IMPES:  D = colsum(A_0s) colsum(A_ss)^-1 */

/* AMG smoother (amg_sweeps passes before and after the coarse correction) */
#define CPTR_SMOOTHER_L1JACOBI 0 /* x += D_l1^-1 (b - A x), D_l1 = diag(sum_j |a_ij|) */
#define CPTR_SMOOTHER_GS 1       /* symmetric multicolour Gauss-Seidel: greedy colouring of each level
                                    in natural order, colours ascending before the coarse correction
                                    (from x = 0) and descending after it */

/* The Schur complement approximation S~_T of the block first stages */
#define CPTR_SCHUR_ASSEMBLED 0   /* the caller's S~_T of eq:Se (needs the PDE; passed to cptr_setup) */
#define CPTR_SCHUR_ATT 1         /* A_TT (Section 3.3.1) */
#define CPTR_SCHUR_DIAG 2        /* A_TT - A_Tp diag(A_pp)^-1 A_pT (Section 3.3.1), on the cells
                                    within two steps of the cell graph; entry (i, l) starts from
                                    A_TT(i, l) and loses (A_Tp(i,j) / A_pp(j,j)) A_pT(j,l) for the
                                    blocks (i, j) of row i, then (j, l) of row j, both ascending */

/* second stage */
#define CPTR_SECOND_NONE 0       /* z = x1 */
#define CPTR_SECOND_BILU0 1      /* block ILU(0), natural order, level-scheduled solves */
#define CPTR_SECOND_BILU0_MC 2   /* block ILU(0) in greedy multicolour order */
#define CPTR_SECOND_IDENTITY 3   /* z = b1 + x1 */
#define CPTR_SECOND_LEARNED 4    /* learned message-passing stage (cptr_learn.h), BILU(0) natural-order fallback */

/* precision of the preconditioner (FGMRES itself is always FP64) */
#define CPTR_FP64 0
#define CPTR_FP32 1

typedef struct {
  int n;                 /* block rows = cells */
  int nv;                /* unknowns per cell: 3 or 4 */
  int nnzb;              /* stored blocks */
  const int *row_ptr;    /* device, n+1 */
  const int *col_idx;    /* device, nnzb */
  const double *vals;    /* device, nnzb*nv*nv, borrowed (see cptr_setup) */
} cptr_bsr;

typedef struct {
  int n;
  int nnz;
  const int *row_ptr;    /* device, n+1 */
  const int *col_idx;    /* device, nnz */
  const double *vals;    /* device, nnz */
} cptr_csr;

typedef struct {
  int first_stage;       /* CPTR_FIRST_* (default CPTR_FIRST_BLOCK) */
  int second_stage;      /* CPTR_SECOND_* (default CPTR_SECOND_BILU0_MC) */
  int precision;         /* CPTR_FP64 / CPTR_FP32 (default CPTR_FP32) */
  int ip, iT;            /* slots of p and T (defaults 0 and nv-1; iT < 0 means nv-1) */
  double amg_theta;      /* strength threshold of the finest AMG level (0.08), halved per level */
  int amg_max_levels;    /* <= 16 (10) */
  int amg_coarse_size;   /* coarsest level solved directly once n <= this (512) */
  unsigned amg_seed;     /* aggregation priority seed (0) */
  int amg_sweeps;        /* smoother sweeps (amg_smoother) before and after the coarse
                            correction (2) */
  int amg_smooth_p;      /* 1 smoothed aggregation, 0 plain aggregation (1) */
  int amg_smooth_p_T;    /* the same for the second hierarchy alone (S~_T; A_TT for
                            CPTR_FIRST_BD; the temperature block of the CPTR_FIRST_UAMG
                            hierarchy); -1: as amg_smooth_p (0).
                            Plain aggregation keeps the S~_T V-cycle convergent where the
                            smoothed prolongator does not (rows that are not diagonally
                            dominant, three-phase systems) and needs fewer FGMRES iterations
                            on the two-phase systems too */
  int use_graph;         /* 1: replay the preconditioner and the Arnoldi step as HIP graphs (1) */
  int resid_fp64;        /* FP32 mode: form the two-stage residual b1 = v - A x1 from the FP64
                            values of A with FP64 accumulation, then round b1 to FP32 (0).
                            Avoids the FP32 cancellation of b1 on badly scaled systems. */
  int scalar_dia;        /* 1: scalar operators of at least 4096 rows whose entries lie on at
                            most 8 diagonals (the 7-point blocks of a structured grid) are
                            stored by diagonals, without column indices; 0: SELL-64 for all
                            short-row operators (1).  Both give the same sums in the same
                            order. */
  int lrn_columns;       /* 1: the learned stage's inference layers after the first walk
                            columns of tiles along the slowest axis when the cells form a grid
                            numbered with the fastest axis first and a plane is a multiple of
                            16 cells (rows of the -z/+z neighbours kept in registers, -x/+x by
                            lane shuffles); 0: tiles in cell order with every neighbour row
                            gathered (1).  Both give the same result bit for bit. */
  int decoupling;        /* CPTR_DECOUPLE_* for CPTR_FIRST_CPR and CPTR_FIRST_UAMG (NONE);
                            other first stages reject QI / TI with CPTR_ERR_UNSUPPORTED, a
                            singular block of D gives CPTR_ERR_SINGULAR_BLOCK */
  int ilu_level;         /* level of fill of the BILU second stages: 0 (BILU(0)) or 1 (BILU(1):
                            the blocks of A and the level-1 fill, Section 4's ILU(1)) (0);
                            the learned stage's fallback stays BILU(0) */
  int schur;             /* S~_T of CPTR_FIRST_BLOCK(_LOWER, _UPPER): CPTR_SCHUR_* (ASSEMBLED) */
  int lrn_fallback;      /* CPTR_SECOND_LEARNED in fgmres_solve: 1 switch to the BILU(0)
                            fallback on a non-finite Arnoldi step or a restart cycle whose true
                            residual did not halve; 0 never (a non-finite step is then
                            CPTR_ERR_NONFINITE) (1) */
  int amg_smoother;      /* CPTR_SMOOTHER_* of every AMG hierarchy (L1JACOBI) */
  int ilu_part_x, ilu_part_y, ilu_part_z;
                         /* block-Jacobi parts of the BILU second stages (1, 1, 1: none):
                            when A is the 7-point graph of an nx x ny x nz grid numbered x
                            fastest, cell (x, y, z) belongs to part (x px / nx, y py / ny,
                            z pz / nz) and the blocks coupling different parts are left out
                            of the factor -- the block-Jacobi ILU of the paper's parallel
                            runs (Section 4), here to shorten the chains of dependent steps
                            of the triangular solves (natural order: nx + ny + nz - 2 levels
                            become about nx/px + ny/py + nz/pz).  Other patterns with parts
                            give CPTR_ERR_UNSUPPORTED.  The learned stage's fallback keeps the
                            whole natural-order BILU(0) */
  int ilu_accum_fp64;    /* FP32 mode: the BILU triangular solves sum each row in FP64 (the
                            factors and vectors stay FP32 in memory; 0: FP32 sums) (0) */
  int resetup_device;    /* cptr_update_values recomputes the AMG values on the GPU (1) or on
                            the host (0); both give the same values bit for bit.  The GPU
                            form keeps FP64 CSR copies of every level and of its P, R and
                            A P on the device from cptr_setup on (some hundreds of MB per
                            hierarchy at 10^6 cells).  CPTR_FIRST_UAMG and the decoupling
                            operators are re-set up on the host either way (1) */
  int amg_sweeps_T;      /* smoother sweeps of the second hierarchy (S~_T, or A_TT with
                            CPTR_FIRST_BD) before and after its coarse corrections; 0: amg_sweeps.
                            Not used by CPR and CPTR-uAMG, which have no second hierarchy (0) */
} cptr_options;

typedef struct {
  int restart;           /* m of FGMRES(m) (30) */
  double rtol;           /* stop when ||b - A x|| <= rtol ||b|| (1e-6) */
  int maxit;             /* total inner iterations (1000) */
  int nonzero_guess;     /* 0: x0 = 0, 1: x holds the initial guess */
} cptr_solve_opts;

typedef struct {
  int iters;             /* preconditioner applications */
  int restarts;
  int converged;
  double relres_est;     /* |g_{j+1}| / ||b|| at exit */
  double relres_true;    /* ||b - A x|| / ||b||, FP64, at exit */
  double solve_ms;       /* wall time inside fgmres_solve */
  int fell_back;         /* 1 if the learned second stage was replaced by BILU(0) */
} cptr_solve_info;

typedef struct {
  int nlevels[2];        /* AMG levels of A_pp [0] and S~_T [1] (A_TT for CPTR_FIRST_BD;
                            [0] the coupled A_00 and [1] none for CPTR_FIRST_UAMG) */
  int level_rows[2][16];
  int level_nnz[2][16];
  int ilu_levels_lower;  /* dependent steps of the forward sweep */
  int ilu_levels_upper;  /* dependent steps of the backward sweep */
  int ilu_colors;        /* colours of the multicolour order (0 for natural) */
  double setup_ms;
  double apply_bytes;    /* algorithmic HBM bytes of one preconditioner application */
  double spmv_bytes;     /* algorithmic bytes of one FP64 BSR product */
  long long applies;     /* preconditioner applications so far */
} cptr_stats;

typedef struct cptr_handle cptr_handle;

/* Fill *opt with the defaults listed above. */
void cptr_default_options(cptr_options *opt);

/* Build the preconditioner for A (first stage: sub-block extraction eq:A00,
 * two AMG hierarchies for A_pp and S~_T -- A_TT for CPTR_FIRST_BD; one on the
 * coupled 2n x 2n A_00 for CPTR_FIRST_UAMG; second
 * stage: BILU(0) factors).
 *   out   receives the handle (NULL on failure).
 *   A     must stay alive and unchanged until cptr_destroy: A->vals (FP64) is
 *         BORROWED for the FP64 Arnoldi products; everything derived is owned.
 *   S_T   the assembled S~_T of eq:Se; required for CPTR_FIRST_BLOCK(_LOWER, _UPPER)
 *         with CPTR_SCHUR_ASSEMBLED, ignored (may be NULL) otherwise; with
 *         CPTR_SCHUR_ATT / _DIAG the library forms S~_T from A (a zero A_pp
 *         diagonal entry gives CPTR_ERR_SINGULAR_BLOCK).
 *   opt   NULL for defaults.
 * Blocks until setup is complete.  Errors: CPTR_ERR_INVALID_ARG (sizes,
 * unsorted or out-of-range columns, missing diagonal, nv not 3/4, ip == iT,
 * structurally unsymmetric pattern), CPTR_ERR_NONFINITE, CPTR_ERR_SINGULAR_BLOCK
 * (zero pivot in a diagonal block of the ILU factorisation),
 * CPTR_ERR_SETUP (AMG coarsening stalled above 4096 rows), CPTR_ERR_OOM,
 * CPTR_ERR_HIP. */
int cptr_setup(cptr_handle **out, const cptr_bsr *A, const cptr_csr *S_T,
               const cptr_options *opt, void *stream);

/* z = M^{-1} v (one two-stage application).  v, z: device FP64 [n*nv], must
 * not alias.  Asynchronous on `stream`. */
int cptr_apply(cptr_handle *h, const double *v, double *z, void *stream);

/* Only the first stage: x1 = M1^{-1} v prolonged to the full vector (zeros in
 * the saturation slots).  Device FP64 [n*nv].  Asynchronous. */
int cptr_first_stage(cptr_handle *h, const double *v, double *x1, void *stream);

/* The input of the second stage for v: b1 = v - A x1 with x1 = M1^{-1} v the
 * first-stage result ("Two-stage preconditioners", Section 3), formed by the
 * same kernels and in the handle's precision as inside cptr_apply (x1 = 0
 * without a first stage), then widened to FP64.  v, b1: device FP64 [n*nv],
 * must not alias.  Training inputs of a learned second stage.  Asynchronous. */
int cptr_stage_residual(cptr_handle *h, const double *v, double *b1, void *stream);

/* One AMG V-cycle from a zero initial guess on A_pp (which = 0) or the
 * second hierarchy (which = 1: S~_T, or A_TT with CPTR_FIRST_BD), in the
 * handle's precision: x = V(b).  Device FP64 [n]; with CPTR_FIRST_UAMG,
 * which = 0 is the coupled A_00 hierarchy and b, x are [2n] (p rows, then T).
 * Asynchronous. */
int cptr_vcycle(cptr_handle *h, int which, const double *b, double *x, void *stream);

/* Right-preconditioned flexible GMRES(m) (Saad 1993) with the handle's
 * preconditioner; Arnoldi by classical Gram-Schmidt with one
 * re-orthogonalisation in FP64 (two passes over the basis per step: the
 * second projection and normalisation of each new basis vector are applied
 * in the next step, after the preconditioner has been applied to the vector
 * before them, which flexible GMRES permits); stops when the Givens estimate reaches
 * rtol ||b|| and the FP64 true residual confirms it, otherwise restarts.
 * b, x: device FP64 [n*nv]; x is the initial guess if so->nonzero_guess, and
 * is overwritten with the solution.  `so` NULL for defaults; `info` may be
 * NULL.  Blocking (reads one FP64 scalar per iteration).  Returns CPTR_OK or
 * CPTR_NOT_CONVERGED (info filled in both cases). */
int fgmres_solve(cptr_handle *h, const double *b, double *x, const cptr_solve_opts *so,
                 cptr_solve_info *info, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fgmres_solve with its Krylov workspace -- basis, preconditioned vectors,
 * Hessenberg and Givens data, reduction partials, step state -- taken from a
 * device array of the library instead of memory the handle allocates on its
 * first solve.  The array holds CPTR_STATIC_WORKSPACE_BYTES (256 MiB) on every
 * GPU the library runs on and is kept until the process ends.  The call
 * allocates nothing: no hipMalloc, hipFree or hipHostMalloc, no graph capture
 * (every Arnoldi step is launched directly, the per-step results are copied
 * to the calling thread's stack); the preconditioner's memory is the
 * handle's, allocated by cptr_setup.  The workspace needs about
 * (m+1) N 8 + m N zb + 2 N 8 bytes plus 70 KB for restart m, N = n nv
 * unknowns, zb = 4 (FP32 preconditioner) or 8 (FP64); a larger need returns
 * CPTR_ERR_INVALID_ARG before anything is launched.  Every call on one GPU
 * uses the same array and leaves its contents there: calls that overlap on
 * one GPU (other threads, other streams, other handles) race and must be
 * serialised by the caller.  Arguments, results, blocking and the solve
 * itself as fgmres_solve; cptr_krylov_vector does not see its basis. */
#define CPTR_STATIC_WORKSPACE_BYTES (256u << 20)
int fgmres_solve_static(cptr_handle *h, const double *b, double *x, const cptr_solve_opts *so,
                        cptr_solve_info *info, void *stream);

/* y = A x with the matrix of h (Section 3, the linearised system), using the
 * handle's sliced device copy of A (the product of every FGMRES step).
 * x, y: device FP64 [n*nv], must not alias.  Asynchronous on `stream`. */
int cptr_matvec(const cptr_handle *h, const double *x, double *y, void *stream);

/* Copy the Arnoldi basis vector v_j of the most recent FGMRES cycle (device
 * FP64 [n*nv], orthonormal in the 2-norm; Section 3, right-preconditioned
 * GMRES) into `out` (device FP64 [n*nv], caller-owned), ordered on `stream`.
 * The preconditioner of step j was applied to v_j before its second
 * Gram-Schmidt projection and normalisation (a multiple of v_j up to a
 * rounding-level correction), so these stand for its inputs, e.g. training
 * inputs for a learned second stage.  Valid for 0 <= j <= restart after a
 * fgmres_solve with that restart length; only j < (iterations of the last
 * cycle) hold basis vectors of that solve.  CPTR_ERR_INVALID_ARG for a
 * handle without a solve or j out of range. */
int cptr_krylov_vector(const cptr_handle *h, int j, double *out, void *stream);

/* Numeric re-setup for a new Jacobian with the pattern of the one given to
 * cptr_setup (the next Newton iterate or time step; Section 4 solves one such
 * system per nonlinear iteration).  A_vals: device FP64 BSR values in the
 * layout of cptr_bsr.vals (the handle borrows this pointer from now on, as it
 * did the original); S_vals: device FP64 values of S~_T in the pattern given
 * to cptr_setup (required for CPTR_FIRST_BLOCK / _BLOCK_LOWER / _BLOCK_UPPER with
 * CPTR_SCHUR_ASSEMBLED, else ignored: the algebraic S~_T is formed anew from
 * A_vals).
 * The aggregates of both AMG hierarchies and the block ILU's order, pattern
 * and level schedules are kept.  With resetup_device = 1 everything else is
 * recomputed on the GPU: the prolongator values, the Galerkin products R (A P),
 * the l1-Jacobi diagonals, the explicit inverse of the coarsest operator, the
 * algebraic S~_T, the block ILU factors, the sliced copy of A and the learned
 * stage's diagonal-block inverses and edge features, each entry with the
 * operations and summation order of the host setup (results equal to the
 * host re-setup bit for bit); with 0 (and for CPTR_FIRST_UAMG or a decoupling
 * operator) the AMG values are recomputed on the host.  Blocking.  CPTR_ERR_INVALID_ARG for a missing argument,
 * CPTR_ERR_NONFINITE for a non-finite value, CPTR_ERR_SINGULAR_BLOCK as in
 * cptr_setup; on error the handle must be destroyed. */
int cptr_update_values(cptr_handle *h, const double *A_vals, const double *S_vals,
                       void *stream);

/* Kernel timing for roofline figures.  With enable = 1 (totals reset) the
 * handle's later solves skip graph replay and record HIP events on the
 * solve's stream around every launch of the Krylov product w = A z (id 0)
 * and of the learned stage's three inference layers (ids 1, 2, 3; also in
 * cptr_apply); enable = 0 stops and keeps the totals.  The events add no
 * work to the kernels; the launch gaps of a solve without graphs are a few
 * microseconds longer.  cptr_get_kernel_times: average microseconds per
 * launch and launch counts of the four ids (host arrays of 4, NULL to skip;
 * blocks until the timed launches have finished). */
int cptr_kernel_timing(cptr_handle *h, int enable);
int cptr_get_kernel_times(cptr_handle *h, double *avg_us, long long *launches);

/* Introspection.  Integer setup results, copied to host arrays (NULL to skip):
 * the aggregate of every row of AMG level `level` (size = rows of that level),
 * and the level / colour of every cell in the BILU(0) solves (size n). */
int cptr_get_stats(const cptr_handle *h, cptr_stats *st);
int cptr_get_aggregates(const cptr_handle *h, int which, int level, int *agg_host);
int cptr_get_ilu_schedule(const cptr_handle *h, int *lev_lower_host, int *lev_upper_host,
                          int *color_host);

/* y = A x for an FP64 BSR matrix (nv = 3 or 4); device pointers.  The kernel
 * used for the Arnoldi products, exposed for testing.  Asynchronous. */
int cptr_bsr_spmv(int n, int nv, const int *row_ptr, const int *col_idx, const double *vals,
                  const double *x, double *y, void *stream);

const char *cptr_status_string(int status);
const char *cptr_last_error(void);
void cptr_destroy(cptr_handle *h);

#ifdef __cplusplus
}
#endif
#endif
