/*
 * Oracle for the CPTR-FGMRES path: plain, slow, FP64 CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  It is the independent reference that the GPU
 * library is checked against; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * GPU library (no headers, helpers or tables).
 *
 * Contents (each function cites the passage it follows):
 *   - BSR / CSR products;
 *   - smoothed-aggregation AMG (strength, distance-2 maximal independent set,
 *     aggregation, Jacobi-smoothed prolongation, Galerkin product, dense LU
 *     on the coarsest level) and its V-cycle with l1-Jacobi or symmetric
 *     multicolour Gauss-Seidel smoothing; the same built per unknown on the
 *     coupled pressure-temperature block (unknown-based AMG, Section 3.4);
 *   - block ILU(0) and ILU(1) in natural and in multicolour order, level sets;
 *   - the two-stage CPR / CPTR preconditioners of Section 3 with the first
 *     stages CPTR-Block, its lower-triangular and block-diagonal variants,
 *     CPR and CPTR-uAMG, the Quasi-/True-IMPES decoupling operators (Sections
 *     3.1, 3.2) and the algebraic S~_T approximations of Section 3.3.1;
 *   - right-preconditioned flexible GMRES(m) with modified Gram-Schmidt.
 */
#ifndef CPTR_ORACLE_H
#define CPTR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FIRST_NONE = 0, ORC_FIRST_CPTR_BLOCK = 1, ORC_FIRST_CPTR_LOWER = 2,
       ORC_FIRST_CPR = 3, ORC_FIRST_CPTR_BD = 4, ORC_FIRST_CPTR_UAMG = 5, ORC_FIRST_CPTR_UPPER = 6 };
enum { ORC_SECOND_NONE = 0, ORC_SECOND_BILU0 = 1, ORC_SECOND_BILU0_MC = 2,
       ORC_SECOND_IDENTITY = 3, ORC_SECOND_EXACT = 4 };

typedef struct {
  int first_stage;
  int second_stage;
  int ip, iT;          /* slots of pressure and temperature in a block */
  double theta;        /* strength threshold of the finest level */
  int max_levels;
  int coarse_size;
  unsigned seed;       /* priority hash seed of the aggregation */
  int sweeps;          /* l1-Jacobi sweeps before and after the coarse correction */
  int smooth_p;        /* 1: smoothed aggregation, 0: tentative (plain) aggregation */
  int smoother;        /* 0: l1-Jacobi, 1: multicolour Gauss-Seidel (symmetric) */
  const int *ilu_order;/* BILU0 factor order (position -> cell) or NULL */
  const int *ilu_part; /* BILU0 partition (cell -> part, couplings across parts dropped) or NULL */
  int smooth_p_T;      /* prolongator of the S~_T (or A_TT) hierarchy, and of the temperature block of
                          the unknown-based hierarchy: 1 smoothed, 0 plain, -1 as smooth_p */
  int decoupling;      /* CPR and CPTR-uAMG first stages: 0 none, 1 Quasi-IMPES, 2 True-IMPES
                          (Section 3.1; its extension to p-T in Section 3.2) */
  int ilu_level;       /* level of fill of the block ILU second stage: 0 (BILU(0)) or 1 (BILU(1)) */
  int schur;           /* S~_T of the block first stages: 0 the assembled one passed in (eq:Se),
                          1 A_TT, 2 A_TT - A_Tp diag(A_pp)^{-1} A_pT (Section 3.3.1) */
  int sweeps_T;        /* sweeps of the second hierarchy (S~_T or A_TT); 0: sweeps */
} orc_opts;

typedef struct {
  int iters;           /* preconditioner applications (inner iterations) */
  int restarts;
  int converged;
  double relres_est;   /* |g_{j+1}| / ||b|| at exit */
  double relres_true;  /* ||b - A x|| / ||b|| at exit */
} orc_info;

void *orc_create(int n, int nv, const int *rp, const int *ci, const double *vals,
                 const int *srp, const int *sci, const double *svals,
                 const orc_opts *o, int *status);
void orc_destroy(void *h);
int orc_apply(void *h, const double *v, double *z);
int orc_first_stage(void *h, const double *v, double *x1);
/* block ILU factor pattern in factor order: returns the number of blocks;
 * rp [n+1] and ci [nnz] are filled when non-NULL */
int orc_ilu_pattern(void *h, int *rp, int *ci);
int orc_fgmres(void *h, const double *b, double *x, int m, double rtol, int maxit,
               orc_info *info, double *V, double *Z, double *H);

int orc_amg_nlevels(void *h, int which);
int orc_amg_level_info(void *h, int which, int lev, int *n, int *nnz, int *pnnz);
int orc_amg_get_level(void *h, int which, int lev, int *agg, int *arp, int *aci,
                      double *av, int *prp, int *pci, double *pv, double *omega);
int orc_amg_vcycle(void *h, int which, const double *b, double *x);

int orc_ilu_get(void *h, int *perm, int *color, int *lev_lower, int *lev_upper,
                double *lu_vals, double *dinv);

void orc_bsr_spmv(int n, int nv, const int *rp, const int *ci, const double *v,
                  const double *x, double *y);
int orc_strength(int n, const int *rp, const int *ci, const double *v, double theta,
                 int *srp, int *sci);
int orc_mis2_greedy(int n, const int *srp, const int *sci, unsigned seed, int *is_root);
unsigned orc_fmix32(unsigned h);

#ifdef __cplusplus
}
#endif
#endif
