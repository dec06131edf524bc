// Block ILU(0) / ILU(1) factorisation (host, FP64) and the level schedule of
// its triangular solves.  ILU(0) is the second stage of CPR and CPTR (Section
// 3; the implementation notes of Section 4 use ILU(0) by default, ILU(1) in
// CPR-AMG-ILU(1)).  ILU(1) factors on the blocks of A plus the level-1 fill.
//
// Factor order: natural cell order, or a greedy multicolour order (colour of
// a cell = smallest colour not used by its lower-numbered neighbours; cells
// renumbered colour by colour, ascending inside a colour).  Optionally the
// cells are split into parts and the couplings between parts are left out
// (block Jacobi, as the parallel ILU(0) of the paper's multi-process runs).  The factor is the
// IKJ form of ILU(0) on nv x nv blocks: for each row i and each lower block
// k < i in order, L_ik = A_ik U_kk^{-1}, then A_ij -= L_ik U_kj for every j > k
// present in both rows.  Diagonal blocks are inverted by Gauss-Jordan
// elimination with partial pivoting.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "setup.h"

namespace cptr {
namespace {

void blk_mul(int nv, const double *a, const double *b, double *c) {
  for (int r = 0; r < nv; r++)
    for (int q = 0; q < nv; q++) {
      double s = 0.0;
      for (int k = 0; k < nv; k++) s += a[r * nv + k] * b[k * nv + q];
      c[r * nv + q] = s;
    }
}

bool blk_inv(int nv, const double *a, double *inv) {
  double m[4][8];
  for (int r = 0; r < nv; r++)
    for (int q = 0; q < 2 * nv; q++) m[r][q] = q < nv ? a[r * nv + q] : (q - nv == r ? 1.0 : 0.0);
  for (int k = 0; k < nv; k++) {
    int p = k;
    for (int r = k + 1; r < nv; r++)
      if (std::fabs(m[r][k]) > std::fabs(m[p][k])) p = r;
    if (m[p][k] == 0.0 || !std::isfinite(m[p][k])) return false;
    if (p != k)
      for (int q = 0; q < 2 * nv; q++) std::swap(m[k][q], m[p][q]);
    double d = m[k][k];
    for (int q = 0; q < 2 * nv; q++) m[k][q] /= d;
    for (int r = 0; r < nv; r++) {
      if (r == k) continue;
      double f = m[r][k];
      for (int q = 0; q < 2 * nv; q++) m[r][q] -= f * m[k][q];
    }
  }
  for (int r = 0; r < nv; r++)
    for (int q = 0; q < nv; q++) inv[r * nv + q] = m[r][nv + q];
  return true;
}

}  // namespace

void ilu_build(int n, int nv, const int *rp, const int *ci, const double *vals,
               bool multicolor, IluHost &out, int level, const int *part) {
  const int b2 = nv * nv;
  out.n = n;
  out.nv = nv;
  out.color.assign(n, 0);
  out.order.resize(n);
  std::vector<int> pos(n);
  if (multicolor) {
    int ncol = 0;
    std::vector<int> mark;
    for (int i = 0; i < n; i++) {
      mark.assign(ncol + 2, 0);
      for (int k = rp[i]; k < rp[i + 1]; k++)
        if (ci[k] < i) mark[out.color[ci[k]]] = 1;
      int c = 0;
      while (mark[c]) c++;
      out.color[i] = c;
      ncol = std::max(ncol, c + 1);
    }
    out.ncolor = ncol;
    int p = 0;
    for (int c = 0; c < ncol; c++)
      for (int i = 0; i < n; i++)
        if (out.color[i] == c) out.order[p++] = i;
  } else {
    out.ncolor = 0;
    for (int i = 0; i < n; i++) out.order[i] = i;
  }
  for (int p = 0; p < n; p++) pos[out.order[p]] = p;

  // renumbered pattern: row p holds the blocks of cell order[p], columns as
  // factor positions, ascending (with a partition, only the blocks inside
  // the cell's part)
  std::vector<int> frp(n + 1, 0), fci, src;
  fci.reserve(rp[n]);
  src.reserve(rp[n]);
  std::vector<std::pair<int, int>> row;
  for (int p = 0; p < n; p++) {
    int i = out.order[p];
    row.clear();
    for (int k = rp[i]; k < rp[i + 1]; k++)
      if (!part || part[ci[k]] == part[i]) row.push_back({pos[ci[k]], k});
    std::sort(row.begin(), row.end());
    for (const auto &e : row) {
      fci.push_back(e.first);
      src.push_back(e.second);
    }
    frp[p + 1] = int(fci.size());
  }
  if (level == 1) {
    // ILU(1): the blocks of A (level 0) and the level-1 fill (p, j) for every
    // lower block (p, q) of A and upper block (q, j) of A, j > q; fill blocks
    // start at zero (src = -1)
    std::vector<int> nrp(n + 1, 0), nci, nsrc;
    std::vector<int> seen(n, -1);
    std::vector<std::pair<int, int>> row;
    for (int p = 0; p < n; p++) {
      row.clear();
      for (int k = frp[p]; k < frp[p + 1]; k++) {
        seen[fci[k]] = p;
        row.push_back({fci[k], src[k]});
      }
      for (int k = frp[p]; k < frp[p + 1]; k++) {
        const int q = fci[k];
        if (q >= p) continue;
        for (int t = frp[q]; t < frp[q + 1]; t++) {
          const int j = fci[t];
          if (j > q && seen[j] != p) {
            seen[j] = p;
            row.push_back({j, -1});
          }
        }
      }
      std::sort(row.begin(), row.end());
      for (const auto &e : row) {
        nci.push_back(e.first);
        nsrc.push_back(e.second);
      }
      nrp[p + 1] = int(nci.size());
    }
    frp.swap(nrp);
    fci.swap(nci);
    src.swap(nsrc);
  }
  const int nnzf = frp[n];
  std::vector<double> lu((size_t)nnzf * b2, 0.0);
  for (int k = 0; k < nnzf; k++)
    if (src[k] >= 0)
      std::copy(vals + (size_t)src[k] * b2, vals + (size_t)src[k] * b2 + b2, lu.begin() + (size_t)k * b2);
  std::vector<int> dpos(n, -1);
  for (int p = 0; p < n; p++)
    for (int k = frp[p]; k < frp[p + 1]; k++)
      if (fci[k] == p) dpos[p] = k;
  std::vector<double> dinv_pos((size_t)n * b2);

  // IKJ factorisation with a column-position map of the current row
  std::vector<int> where(n, -1);
  double tmp[16], prod[16];
  for (int p = 0; p < n; p++) {
    for (int k = frp[p]; k < frp[p + 1]; k++) where[fci[k]] = k;
    for (int k = frp[p]; k < dpos[p]; k++) {
      int q = fci[k];
      blk_mul(nv, &lu[(size_t)k * b2], &dinv_pos[(size_t)q * b2], tmp);
      std::copy(tmp, tmp + b2, &lu[(size_t)k * b2]);
      for (int t = dpos[q] + 1; t < frp[q + 1]; t++) {
        int s = where[fci[t]];
        if (s < 0) continue;
        blk_mul(nv, &lu[(size_t)k * b2], &lu[(size_t)t * b2], prod);
        for (int e = 0; e < b2; e++) lu[(size_t)s * b2 + e] -= prod[e];
      }
    }
    if (!blk_inv(nv, &lu[(size_t)dpos[p] * b2], &dinv_pos[(size_t)p * b2]))
      throw Error{CPTR_ERR_SINGULAR_BLOCK,
                  "zero pivot in the ILU(0) diagonal block of cell " + std::to_string(out.order[p])};
    for (int k = frp[p]; k < frp[p + 1]; k++) where[fci[k]] = -1;
  }

  // level sets in factor order
  std::vector<int> ll(n, 0), lu_(n, 0);
  int nll = 0, nlu = 0;
  for (int p = 0; p < n; p++) {
    int lv = 0;
    for (int k = frp[p]; k < dpos[p]; k++) lv = std::max(lv, ll[fci[k]] + 1);
    ll[p] = lv;
    nll = std::max(nll, lv + 1);
  }
  for (int p = n - 1; p >= 0; p--) {
    int lv = 0;
    for (int k = dpos[p] + 1; k < frp[p + 1]; k++) lv = std::max(lv, lu_[fci[k]] + 1);
    lu_[p] = lv;
    nlu = std::max(nlu, lv + 1);
  }
  out.lev_lower.assign(n, 0);
  out.lev_upper.assign(n, 0);
  for (int p = 0; p < n; p++) {
    out.lev_lower[out.order[p]] = ll[p];
    out.lev_upper[out.order[p]] = lu_[p];
  }
  out.dinv.assign((size_t)n * b2, 0.0);
  for (int p = 0; p < n; p++)
    std::copy(&dinv_pos[(size_t)p * b2], &dinv_pos[(size_t)p * b2] + b2,
              &out.dinv[(size_t)out.order[p] * b2]);

  // sweep schedules: positions sorted by (level, position)
  out.dst.assign(nnzf, -1);
  auto schedule = [&](const std::vector<int> &lev, int nlev, bool lower, std::vector<int> &rows,
                      std::vector<int> &lev_ptr, std::vector<int> &ptr, std::vector<int> &col,
                      std::vector<double> &val, std::vector<int> *order_out) {
    lev_ptr.assign(nlev + 1, 0);
    for (int p = 0; p < n; p++) lev_ptr[lev[p] + 1]++;
    for (int l = 0; l < nlev; l++) lev_ptr[l + 1] += lev_ptr[l];
    std::vector<int> fill(lev_ptr.begin(), lev_ptr.end() - 1), byp(n);
    for (int p = 0; p < n; p++) byp[fill[lev[p]]++] = p;
    if (order_out) *order_out = byp;
    rows.resize(n);
    ptr.assign(n + 1, 0);
    col.clear();
    val.clear();
    for (int t = 0; t < n; t++) {
      int p = byp[t];
      rows[t] = out.order[p];
      int b = lower ? frp[p] : dpos[p] + 1;
      int e = lower ? dpos[p] : frp[p + 1];
      for (int k = b; k < e; k++) {
        out.dst[k] = lower ? int(col.size()) : -int(col.size()) - 2;
        col.push_back(out.order[fci[k]]);
        val.insert(val.end(), &lu[(size_t)k * b2], &lu[(size_t)k * b2] + b2);
      }
      ptr[t + 1] = int(col.size());
    }
  };
  schedule(ll, nll, true, out.f_rows, out.f_lev_ptr, out.f_ptr, out.f_col, out.f_val, &out.fwd);
  schedule(lu_, nlu, false, out.b_rows, out.b_lev_ptr, out.b_ptr, out.b_col, out.b_val, nullptr);
  out.frp.swap(frp);
  out.fci.swap(fci);
  out.src.swap(src);
  out.dpos.swap(dpos);
}

std::vector<int> grid_parts(int n, const int *rp, const int *ci, int px, int py, int pz) {
  // the three axis strides from the off-diagonal offsets of the pattern
  std::vector<int> mags;
  for (int i = 0; i < n; i++)
    for (int k = rp[i]; k < rp[i + 1]; k++)
      if (ci[k] != i) mags.push_back(std::abs(ci[k] - i));
  std::sort(mags.begin(), mags.end());
  mags.erase(std::unique(mags.begin(), mags.end()), mags.end());
  const auto fail = [] { throw Error{CPTR_ERR_UNSUPPORTED, "ILU parts need the 7-point graph of a 3D grid"}; };
  if (mags.size() != 3 || mags[0] != 1 || mags[2] % mags[1] != 0) fail();
  const int nx = mags[1], ny = mags[2] / mags[1];
  if (nx < 2 || ny < 2 || n % (nx * ny) != 0 || n / (nx * ny) < 2) fail();
  const int nz = n / (nx * ny);
  if (px < 1 || py < 1 || pz < 1 || px > nx || py > ny || pz > nz)
    throw Error{CPTR_ERR_INVALID_ARG, "ILU parts per axis must be between 1 and the grid size"};
  // every coupling must be a grid neighbour (x neighbours in the same row)
  for (int i = 0; i < n; i++)
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      const int j = ci[k], d = std::abs(j - i);
      if (d == 1 && j / nx != i / nx) fail();
      if (d == nx && j / (nx * ny) != i / (nx * ny)) fail();
    }
  std::vector<int> part(n);
  for (int i = 0; i < n; i++) {
    const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    part[i] = (int)((long long)x * px / nx) + px * ((int)((long long)y * py / ny) + py * (int)((long long)z * pz / nz));
  }
  return part;
}

}  // namespace cptr
