/* The discrete thermal model on the GPU and a Newton loop around the
 * CPTR-FGMRES solver: the steps on either side of the linear solve, so that
 * whole implicit time steps run on the device.
 *
 * Model (Section 2.2): fully implicit DG(0) / two-point flux approximation on
 * an nx x ny x nz grid of cubes of edge dx, cell (i, j, k) = i + nx (j + ny k);
 * water and oil (nv = 3: p, S_w, T) or water, gas and oil (nv = 4: p, S_w,
 * S_g, T), oil eliminated through the saturation constraint; facet mass flux
 * {{K}} (rho k_r / mu)^up ((p_R - p_L) / h - {rho} g.n) with the harmonic
 * permeability {{K}}, the arithmetic density average {rho}, k_r = S and
 * upwinding on the sign of the potential (a tie takes the lower-numbered
 * cell); conductive flux {{k_T}} [T] / h with k_T = (1 - phi) k_rock +
 * phi sum_a S_a k_a; implicit Euler; gravity along -z.  Water viscosity and
 * density follow the Grabowski and Kell-Trangenstein correlations of
 * Appendix A, the heat constants the parameter table of Section 4; the oil
 * (Arrhenius viscosity, exponential density) and gas (ideal gas) data are
 * synthetic choices.  Sources per cell: hot-water injection of a fixed volume
 * rate at 373.15 K, a Peaceman producer at a bottom-hole pressure of
 * 2.7579e7 Pa (open while p exceeds it), a heater of 1e3 W/K towards
 * 373.15 K.
 * Residual rows (the weighted pressure equation and the scaling of
 * Section 4): row 0 = T_ref sum_a c_va F_a, rows 1 .. nv-2 = c_ref T_ref F_a
 * (water, gas), row nv-1 = F_e, T_ref = 288.706 K and c_ref = sum_a S_a c_va
 * of the initial saturations (S_w = 0.1, and S_g = 0.05 three-phase).
 * S~_T (Section 3.3.1, the assembled Schur approximation): the temperature
 * operator with every coefficient frozen at the state, its advection term
 * c_va (dT)^up times the frozen facet mass flux.
 *
 * All arrays are device memory unless stated; vectors of unknowns are
 * cell-major (x[i nv + u]).  Functions return CPTR_OK or a negative
 * CPTR_ERR_* code (cptr.h), with cptr_last_error() describing it. */
#ifndef CPTR_MODEL_H
#define CPTR_MODEL_H

#include "cptr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny, nz;          /* grid, each >= 1 */
  double dx;               /* cube edge (m), > 0 */
  int three_phase;         /* 0: water / oil (nv = 3), 1: water / gas / oil (nv = 4) */
  double dt;               /* implicit Euler step (s), > 0 */
  const double *perm;      /* device, n: permeability (m^2), > 0 */
  const double *poro;      /* device, n: porosity, in (0, 1) */
  const int *inj;          /* host, n_inj cell indices of the injector */
  int n_inj;
  const int *prod;         /* host, n_prod cell indices of the producer */
  int n_prod;
  const int *heat;         /* host, n_heat cell indices of heated cells */
  int n_heat;
} cptr_model_desc;

typedef struct cptr_model cptr_model;

/* Copies perm and poro (the caller's arrays may be freed afterwards).
 * CPTR_ERR_INVALID_ARG for sizes or cell indices out of range. */
int cptr_model_create(cptr_model **out, const cptr_model_desc *d);
void cptr_model_destroy(cptr_model *m);

/* The model's unknowns per cell (3 or 4), cell count and its 7-point BSR
 * pattern (ascending columns per row; device arrays owned by the model, valid
 * until cptr_model_destroy).  S~_T has the same pattern as a scalar CSR. */
int cptr_model_info(const cptr_model *m, int *nv, int *n, int *nnzb, const int **row_ptr,
                    const int **col_idx);

/* The same pattern copied to host arrays of n + 1 and nnzb ints (NULL to skip). */
int cptr_model_pattern(const cptr_model *m, int *row_ptr_host, int *col_idx_host);

/* At state x (n nv) after the previous time step's state xn (n nv): the
 * residual F*(x) (n nv), the Jacobian values (nnzb nv^2, row-major blocks in
 * the model's pattern) and the S~_T values (nnzb); a NULL output is skipped.
 * Derivatives are exact to rounding (forward mode).  Asynchronous on `stream`. */
int cptr_model_assemble(cptr_model *m, const double *x, const double *xn, double *F, double *A_vals,
                        double *S_vals, void *stream);

typedef struct {
  int max_it;            /* Newton iterations (50) */
  double rtol;           /* stop when ||F*(x)|| <= rtol ||F*(x0)|| (1e-8) */
  double stol;           /* or when the step ||lambda dx|| <= stol ||x|| (1e-8) */
  int max_backtrack;     /* halvings of the step in the line search (10) */
  cptr_solve_opts lin;   /* the linear solves (FGMRES(30), rtol 1e-6, 1000 iterations) */
} cptr_newton_opts;

typedef struct {
  int iters;             /* Newton iterations taken */
  int lin_iters;         /* FGMRES iterations, summed */
  int backtracks;        /* step halvings, summed */
  int converged;         /* 1 by rtol or stol, 0 otherwise (iteration limit or line search failure) */
  double fnorm0, fnorm;  /* ||F*|| at the initial and the final state */
  double solve_ms;       /* wall time */
} cptr_newton_info;

void cptr_newton_default_options(cptr_newton_opts *o);

/* One implicit time step by Newton's method with a backtracking line search
 * (Section 3: one linearised solve per iterate; relative function and step
 * tolerances 1e-8).  Per iterate: assemble the Jacobian and S~_T at x,
 * cptr_update_values(h, ...) on them (the handle must come from cptr_setup
 * on this model's pattern, and from then on borrows the model's value
 * arrays), solve J dx = -F*(x) with fgmres_solve from dx = 0, then try
 * x + lambda dx for lambda = 1, 1/2, ... until ||F*(x + lambda dx)|| <=
 * (1 - 1e-4 lambda) ||F*(x)||.  A linear solve that stops at its iteration
 * limit still gives the step (inexact Newton).  x (n nv): the initial guess
 * on entry, the last accepted iterate on return; xn: the previous step's
 * state.  Blocking.  Errors of the re-setup or of the linear solver are
 * returned as theirs; a non-finite initial residual is CPTR_ERR_NONFINITE. */
int cptr_newton_solve(cptr_model *m, cptr_handle *h, double *x, const double *xn, const cptr_newton_opts *o,
                      cptr_newton_info *info, void *stream);

#ifdef __cplusplus
}
#endif

#endif
