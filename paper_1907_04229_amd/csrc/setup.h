// Host-side setup structures and algorithms of libcptr (no HIP dependency,
// so that the setup can also be built and checked on a machine without a GPU).
#pragma once

#include <string>
#include <vector>

#include "../../include/cptr.h"

namespace cptr {

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};


// ---------------------------------------------------------------- host sparse
struct HostCSR {
  int nr = 0, nc = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  int nnz() const { return (int)ci.size(); }
};

// Smoothed-aggregation hierarchy built on the host in FP64.
struct AmgParams {
  double theta = 0.08;
  int max_levels = 10;
  int coarse_size = 512;
  unsigned seed = 0;
  int smooth_p = 1;
};

struct AmgLevelHost {
  HostCSR A;            // level operator
  HostCSR P;            // prolongation to this level from the next (n_l x n_{l+1})
  HostCSR R;            // restriction = P^T
  HostCSR AP;           // pattern of the product A P (no values), kept by amg_build
  std::vector<int> agg; // aggregate of each row (empty on the coarsest level)
  double omega = 0.0;
  bool smooth = false;  // P smoothed (else the tentative prolongator)
};

struct AmgHost {
  std::vector<AmgLevelHost> lev;
  std::vector<double> coarse_inv;  // explicit FP64 inverse of the coarsest operator, row-major
};

// Throws Error on failure.  With `fixed` (aggregates of every non-coarsest
// level of an earlier hierarchy on the same pattern), strength and aggregation
// are skipped and those aggregates reused: only the numerical values of the
// prolongators, the Galerkin products and the coarsest inverse are recomputed.
void amg_build(const HostCSR &fine, const AmgParams &prm, AmgHost &out,
               const std::vector<std::vector<int>> *fixed = nullptr);

// Unknown-based hierarchy (Section 3.4) of the pressure-temperature operator
// in unknown-wise order: rows 0 .. np-1 pressure, np .. n-1 temperature.  Each
// unknown is coarsened on its own diagonal block exactly as amg_build does
// (prm_p for pressure, prm_T's smooth_p for temperature), P = diag(P_p, P_T),
// and the Galerkin coarse operator keeps the couplings; coarse unknowns stay in
// unknown-wise order, temperature aggregates numbered after the pressure ones.
// `fixed` as for amg_build (aggregates in that numbering).
void uamg_build(const HostCSR &fine, int np, const AmgParams &prm_p, const AmgParams &prm_T, AmgHost &out,
                const std::vector<std::vector<int>> *fixed = nullptr);

// Algebraic S~_T from the blocks of A (Section 3.3.1): diag = false: A_TT on
// the cell graph; diag = true: A_TT - A_Tp diag(A_pp)^{-1} A_pT on the cells
// within two steps, entry (i, l) from A_TT(i, l), then minus
// (A_Tp(i,j) / A_pp(j,j)) * A_pT(j,l) for (i, j) in row i, (j, l) in row j, both
// ascending.  Throws CPTR_ERR_SINGULAR_BLOCK on a zero A_pp(j,j).
HostCSR schur_algebraic(int n, int nv, int ip, int iT, const int *rp, const int *ci, const double *vals,
                        bool diag);

// Block ILU(0) in a given row order, FP64 on the host.
struct IluHost {
  int n = 0, nv = 0, ncolor = 0;
  std::vector<int> order;        // factor position -> cell
  std::vector<int> color;        // colour of every cell (0 for natural order)
  std::vector<int> lev_lower;    // level of every cell in the forward sweep
  std::vector<int> lev_upper;    // level of every cell in the backward sweep
  // forward sweep, rows in level order
  std::vector<int> f_rows, f_lev_ptr, f_ptr, f_col;
  std::vector<double> f_val;     // nv*nv per block, L (unit diagonal implied)
  // backward sweep, rows in level order
  std::vector<int> b_rows, b_lev_ptr, b_ptr, b_col;
  std::vector<double> b_val;     // nv*nv per block, strictly upper U
  std::vector<double> dinv;      // nv*nv per cell (natural cell index), inverse of U_ii
  // the factor pattern in factor order, kept for a numeric refactorisation of
  // new values on the same pattern: row p (cell order[p]) holds entries
  // frp[p] .. frp[p+1]-1, columns fci (factor positions, ascending), each the
  // block src of A (-1: fill, starts at zero); dpos[p] is its diagonal entry;
  // dst[k] places entry k in the sweeps: >= 0 block index in f_val, <= -2
  // block index -dst[k]-2 in b_val, -1 the diagonal; fwd: factor positions in
  // forward-sweep order (f_lev_ptr delimits its levels)
  std::vector<int> frp, fci, src, dpos, dst, fwd;
};

// Throws Error (CPTR_ERR_SINGULAR_BLOCK on a zero pivot).
// level: 0 for BILU(0), 1 for BILU(1) (level-1 fill of the block pattern).
// part (optional, one entry per cell): the blocks coupling cells of different
// parts are left out of the factor (block Jacobi over the parts, the parallel
// ILU of Section 4's multi-process runs); the order is chosen on the whole
// pattern first.
void ilu_build(int n, int nv, const int *rp, const int *ci, const double *vals,
               bool multicolor, IluHost &out, int level = 0, const int *part = nullptr);

// Cells of a structured grid in the block-Jacobi parts of the ILU: if the
// pattern is the 7-point graph of an nx x ny x nz grid numbered x fastest
// (offsets 1, nx, nx ny; nx, ny, nz >= 2), returns the part of every cell,
// (x px / nx) + px ((y py / ny) + py (z pz / nz)); otherwise throws
// CPTR_ERR_UNSUPPORTED.
std::vector<int> grid_parts(int n, const int *rp, const int *ci, int px, int py, int pz);

}  // namespace cptr
