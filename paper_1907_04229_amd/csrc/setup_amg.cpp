// Smoothed-aggregation AMG setup (host, FP64).
//
// The hierarchy approximates A_pp^{-1} and S~_T^{-1} in the block
// preconditioner of Section 3.3 (the paper uses one AMG V-cycle per inverse),
// and, built per unknown, the coupled A_00^{-1} of the unknown-based first
// stage (Section 3.4).
// Aggregation follows Vanek, Mandel and Brezina (1996) with a distance-2
// maximal independent set computed in parallel rounds (each undecided node
// whose priority is the largest among the undecided nodes within distance 2
// becomes a root); with fixed priorities this yields the same roots as the
// greedy visit in descending priority.
//
// Every floating-point decision and every Galerkin entry is evaluated in a
// fixed order (stated at each step) so that the integer results and the
// coarse operators are reproducible bit for bit.  This file must be compiled
// without floating-point contraction.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "setup.h"

namespace cptr {
namespace {

inline uint32_t fmix32(uint32_t h) {  // MurmurHash3 finalizer (public domain)
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// priority key + 1 (so that 0 means "no candidate"), ordered as (hash, index)
inline uint64_t key1(int i, uint32_t seed) {
  return ((uint64_t(fmix32(uint32_t(i) ^ seed)) << 32) | uint64_t(uint32_t(i))) + 1u;
}

struct Graph {
  std::vector<int> rp, ci;
};

// position of the diagonal and of the transposed entry of every stored entry
void locate(const HostCSR &a, std::vector<int> &diag, std::vector<int> &tpos) {
  int n = a.nr;
  diag.assign(n, -1);
  tpos.assign(a.nnz(), -1);
  for (int i = 0; i < n; i++)
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) {
      int j = a.ci[k];
      if (j == i) diag[i] = k;
      const int *b = a.ci.data() + a.rp[j], *e = a.ci.data() + a.rp[j + 1];
      const int *f = std::lower_bound(b, e, i);
      if (f != e && *f == i) tpos[k] = int(f - a.ci.data());
    }
  for (int i = 0; i < n; i++)
    if (diag[i] < 0) throw Error{CPTR_ERR_INVALID_ARG, "AMG operator row without diagonal"};
  for (size_t k = 0; k < tpos.size(); k++)
    if (tpos[k] < 0) throw Error{CPTR_ERR_INVALID_ARG, "AMG operator pattern is not symmetric"};
}

// i ~ j iff ((a_ij + a_ji) * 0.5)^2 >= theta^2 * |a_ii * a_jj|, FP64, in this order.
Graph strength(const HostCSR &a, double theta) {
  std::vector<int> diag, tpos;
  locate(a, diag, tpos);
  const double t2 = theta * theta;
  Graph g;
  g.rp.assign(a.nr + 1, 0);
  g.ci.reserve(a.nnz());
  for (int i = 0; i < a.nr; i++) {
    const double aii = a.v[diag[i]];
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) {
      int j = a.ci[k];
      if (j == i) continue;
      const double s = (a.v[k] + a.v[tpos[k]]) * 0.5;
      const double lhs = s * s;
      const double rhs = t2 * std::fabs(aii * a.v[diag[j]]);
      if (lhs >= rhs) g.ci.push_back(j);
    }
    g.rp[i + 1] = int(g.ci.size());
  }
  return g;
}

// Distance-2 MIS by synchronous rounds.
std::vector<char> mis2_rounds(const Graph &g, int n, uint32_t seed) {
  std::vector<signed char> state(n, 0);  // 0 undecided, 1 root, -1 excluded
  std::vector<uint64_t> m1(n), key(n);
  std::vector<char> newroot(n), near1(n);
  for (int i = 0; i < n; i++) key[i] = key1(i, seed);
  int undecided = n;
  while (undecided > 0) {
    // largest undecided key in the closed neighbourhood of every node
    for (int j = 0; j < n; j++) {
      uint64_t m = state[j] == 0 ? key[j] : 0;
      for (int k = g.rp[j]; k < g.rp[j + 1]; k++) {
        int q = g.ci[k];
        if (state[q] == 0 && key[q] > m) m = key[q];
      }
      m1[j] = m;
    }
    // a node holding the largest key within distance 2 becomes a root
    for (int i = 0; i < n; i++) {
      newroot[i] = 0;
      if (state[i] != 0) continue;
      uint64_t m = m1[i];
      for (int k = g.rp[i]; k < g.rp[i + 1]; k++) m = std::max(m, m1[g.ci[k]]);
      newroot[i] = (m == key[i]);
    }
    for (int i = 0; i < n; i++)
      if (newroot[i]) { state[i] = 1; undecided--; }
    // exclude every undecided node within distance 2 of a new root
    for (int j = 0; j < n; j++) {
      char f = newroot[j];
      for (int k = g.rp[j]; k < g.rp[j + 1] && !f; k++) f = newroot[g.ci[k]];
      near1[j] = f;
    }
    for (int i = 0; i < n; i++) {
      if (state[i] != 0) continue;
      char f = near1[i];
      for (int k = g.rp[i]; k < g.rp[i + 1] && !f; k++) f = near1[g.ci[k]];
      if (f) { state[i] = -1; undecided--; }
    }
  }
  std::vector<char> root(n);
  for (int i = 0; i < n; i++) root[i] = state[i] == 1;
  return root;
}

// aggregates: root + strong neighbours; remaining nodes join the aggregate of
// the strong neighbour whose root has the largest priority; numbering by
// ascending root index.  Returns the number of aggregates.
int aggregate(const Graph &g, int n, uint32_t seed, std::vector<int> &agg) {
  std::vector<char> root = mis2_rounds(g, n, seed);
  std::vector<int> id(n, -1), rootof(n, -1);
  int na = 0;
  // a root without strong neighbours is an isolated node: it joins no aggregate
  for (int i = 0; i < n; i++)
    if (root[i] && g.rp[i + 1] == g.rp[i]) root[i] = 0;
  for (int i = 0; i < n; i++)
    if (root[i]) id[i] = na++;
  agg.assign(n, -1);
  for (int r = 0; r < n; r++) {
    if (!root[r]) continue;
    agg[r] = id[r];
    rootof[r] = r;
    for (int k = g.rp[r]; k < g.rp[r + 1]; k++) {
      agg[g.ci[k]] = id[r];
      rootof[g.ci[k]] = r;
    }
  }
  std::vector<int> joined(n, -1);
  for (int i = 0; i < n; i++) {
    if (agg[i] >= 0 || g.rp[i + 1] == g.rp[i]) continue;
    int best = -1;
    uint64_t bk = 0;
    for (int k = g.rp[i]; k < g.rp[i + 1]; k++) {
      int r = rootof[g.ci[k]];
      if (r < 0) continue;
      uint64_t kk = key1(r, seed);
      if (kk > bk) { bk = kk; best = r; }
    }
    if (best < 0) throw Error{CPTR_ERR_SETUP, "aggregation left an unassigned node"};
    joined[i] = id[best];
  }
  for (int i = 0; i < n; i++)
    if (agg[i] < 0) agg[i] = joined[i];  // stays -1 for isolated nodes
  return na;
}

HostCSR transpose(const HostCSR &a) {
  HostCSR t;
  t.nr = a.nc;
  t.nc = a.nr;
  t.rp.assign(t.nr + 1, 0);
  t.ci.resize(a.nnz());
  t.v.resize(a.nnz());
  for (int k = 0; k < a.nnz(); k++) t.rp[a.ci[k] + 1]++;
  for (int i = 0; i < t.nr; i++) t.rp[i + 1] += t.rp[i];
  std::vector<int> fill(t.rp.begin(), t.rp.end() - 1);
  for (int i = 0; i < a.nr; i++)
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) {
      int p = fill[a.ci[k]]++;
      t.ci[p] = i;
      t.v[p] = a.v[k];
    }
  return t;
}

// P(i, J) = [agg(i) = J] - (omega / a_ii) * s_iJ, s_iJ = sum of a_ij over row i
// with agg(j) = J in ascending j; omega = 4 / (3 rho), rho = max_i (sum_j |a_ij|
// in ascending j) / |a_ii|.  With smooth = false, P is the tentative prolongator.
HostCSR prolongator(const HostCSR &a, const std::vector<int> &agg, int na, bool smooth,
                    double &omega) {
  int n = a.nr;
  HostCSR p;
  p.nr = n;
  p.nc = na;
  p.rp.assign(n + 1, 0);
  if (!smooth) {
    omega = 0.0;
    for (int i = 0; i < n; i++) {
      if (agg[i] >= 0) {
        p.ci.push_back(agg[i]);
        p.v.push_back(1.0);
      }
      p.rp[i + 1] = int(p.ci.size());
    }
    return p;
  }
  std::vector<double> diag(n);
  double rho = 0.0;
  for (int i = 0; i < n; i++) {
    double s = 0.0, d = 0.0;
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) {
      s += std::fabs(a.v[k]);
      if (a.ci[k] == i) d = a.v[k];
    }
    if (d == 0.0) throw Error{CPTR_ERR_SINGULAR_BLOCK, "zero diagonal in an AMG operator"};
    diag[i] = d;
    double q = s / std::fabs(d);
    if (q > rho) rho = q;
  }
  omega = 4.0 / (3.0 * rho);
  std::vector<int> slot(na, -1);
  std::vector<std::pair<int, double>> row;
  for (int i = 0; i < n; i++) {
    row.clear();
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) {
      int J = agg[a.ci[k]];
      if (J < 0) continue;
      if (slot[J] < 0) {
        slot[J] = int(row.size());
        row.push_back({J, 0.0});
      }
      row[slot[J]].second += a.v[k];
    }
    if (agg[i] >= 0 && slot[agg[i]] < 0) {
      slot[agg[i]] = int(row.size());
      row.push_back({agg[i], 0.0});
    }
    for (auto &e : row) slot[e.first] = -1;
    std::sort(row.begin(), row.end(),
              [](const std::pair<int, double> &x, const std::pair<int, double> &y) {
                return x.first < y.first;
              });
    const double w = omega / diag[i];
    for (auto &e : row) {
      const double d = e.first == agg[i] ? 1.0 : 0.0;
      p.ci.push_back(e.first);
      p.v.push_back(d - w * e.second);
    }
    p.rp[i + 1] = int(p.ci.size());
  }
  return p;
}

// C = A B, each entry accumulated from 0.0 over ascending inner index.
HostCSR multiply(const HostCSR &a, const HostCSR &b) {
  HostCSR c;
  c.nr = a.nr;
  c.nc = b.nc;
  c.rp.assign(a.nr + 1, 0);
  std::vector<int> slot(b.nc, -1);
  std::vector<int> cols;
  std::vector<double> acc;
  for (int i = 0; i < a.nr; i++) {
    cols.clear();
    acc.clear();
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) {
      const double av = a.v[k];
      int m = a.ci[k];
      for (int q = b.rp[m]; q < b.rp[m + 1]; q++) {
        int j = b.ci[q];
        if (slot[j] < 0) {
          slot[j] = int(cols.size());
          cols.push_back(j);
          acc.push_back(0.0);
        }
        acc[slot[j]] += av * b.v[q];
      }
    }
    std::vector<int> order(cols.size());
    for (size_t t = 0; t < order.size(); t++) order[t] = int(t);
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cols[x] < cols[y]; });
    for (int t : order) {
      c.ci.push_back(cols[t]);
      c.v.push_back(acc[t]);
    }
    for (int j : cols) slot[j] = -1;
    c.rp[i + 1] = int(c.ci.size());
  }
  return c;
}

// explicit inverse by Gauss-Jordan elimination with partial pivoting
std::vector<double> dense_inverse(const HostCSR &a) {
  int n = a.nr;
  std::vector<double> m((size_t)n * 2 * n, 0.0);
  for (int i = 0; i < n; i++) {
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++) m[(size_t)i * 2 * n + a.ci[k]] = a.v[k];
    m[(size_t)i * 2 * n + n + i] = 1.0;
  }
  for (int c = 0; c < n; c++) {
    int p = c;
    for (int r = c + 1; r < n; r++)
      if (std::fabs(m[(size_t)r * 2 * n + c]) > std::fabs(m[(size_t)p * 2 * n + c])) p = r;
    double piv = m[(size_t)p * 2 * n + c];
    if (piv == 0.0) throw Error{CPTR_ERR_SETUP, "singular coarsest AMG operator"};
    if (p != c)
      for (int q = 0; q < 2 * n; q++) std::swap(m[(size_t)p * 2 * n + q], m[(size_t)c * 2 * n + q]);
    for (int q = 0; q < 2 * n; q++) m[(size_t)c * 2 * n + q] /= piv;
    for (int r = 0; r < n; r++) {
      if (r == c) continue;
      double f = m[(size_t)r * 2 * n + c];
      if (f == 0.0) continue;
      for (int q = 0; q < 2 * n; q++) m[(size_t)r * 2 * n + q] -= f * m[(size_t)c * 2 * n + q];
    }
  }
  std::vector<double> inv((size_t)n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) inv[(size_t)i * n + j] = m[(size_t)i * 2 * n + n + j];
  return inv;
}

// the square diagonal block of rows and columns r0 .. r1-1, renumbered from 0
HostCSR diag_block(const HostCSR &a, int r0, int r1) {
  HostCSR b;
  b.nr = b.nc = r1 - r0;
  b.rp.assign(b.nr + 1, 0);
  for (int i = r0; i < r1; i++) {
    for (int k = a.rp[i]; k < a.rp[i + 1]; k++)
      if (a.ci[k] >= r0 && a.ci[k] < r1) {
        b.ci.push_back(a.ci[k] - r0);
        b.v.push_back(a.v[k]);
      }
    b.rp[i - r0 + 1] = int(b.ci.size());
  }
  return b;
}

void finish(AmgHost &out) {
  const HostCSR &c = out.lev.back().A;
  if (c.nr > 4096) throw Error{CPTR_ERR_SETUP, "AMG coarsening stalled above 4096 rows"};
  out.coarse_inv = dense_inverse(c);
}

}  // namespace

HostCSR schur_algebraic(int n, int nv, int ip, int iT, const int *rp, const int *ci, const double *vals,
                        bool diag) {
  auto blk = [&](int k, int r, int c) { return vals[((size_t)k * nv + r) * nv + c]; };
  HostCSR s;
  s.nr = s.nc = n;
  s.rp.assign(rp, rp + n + 1);
  if (!diag) {
    s.ci.assign(ci, ci + rp[n]);
    s.v.resize(rp[n]);
    for (int k = 0; k < rp[n]; k++) s.v[k] = blk(k, iT, iT);
    return s;
  }
  std::vector<double> app(n, 0.0), acc(n, 0.0);
  for (int i = 0; i < n; i++)
    for (int k = rp[i]; k < rp[i + 1]; k++)
      if (ci[k] == i) app[i] = blk(k, ip, ip);
  for (int i = 0; i < n; i++)
    if (app[i] == 0.0)
      throw Error{CPTR_ERR_SINGULAR_BLOCK, "zero pressure diagonal entry in cell " + std::to_string(i)};
  std::vector<int> mark(n, -1), cols;
  s.rp.assign(n + 1, 0);
  for (int i = 0; i < n; i++) {
    cols.clear();
    for (int k = rp[i]; k < rp[i + 1]; k++)
      for (int m = rp[ci[k]]; m < rp[ci[k] + 1]; m++)
        if (mark[ci[m]] != i) {
          mark[ci[m]] = i;
          cols.push_back(ci[m]);
        }
    std::sort(cols.begin(), cols.end());
    for (int l : cols) acc[l] = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; k++) acc[ci[k]] = blk(k, iT, iT);
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      const int j = ci[k];
      const double a = blk(k, iT, ip) / app[j];
      for (int m = rp[j]; m < rp[j + 1]; m++) acc[ci[m]] -= a * blk(m, ip, iT);
    }
    for (int l : cols) {
      s.ci.push_back(l);
      s.v.push_back(acc[l]);
    }
    s.rp[i + 1] = int(s.ci.size());
  }
  return s;
}

void uamg_build(const HostCSR &fine, int np, const AmgParams &prm_p, const AmgParams &prm_T, AmgHost &out,
                const std::vector<std::vector<int>> *fixed) {
  if (np < 0 || np > fine.nr) throw Error{CPTR_ERR_INVALID_ARG, "unknown-based AMG: bad pressure block size"};
  out.lev.clear();
  out.lev.emplace_back();
  out.lev[0].A = fine;
  double theta = prm_p.theta;
  const int max_levels = std::min(prm_p.max_levels, 16);
  int npl = np;  // pressure rows of the current level
  for (;;) {
    const size_t l = out.lev.size() - 1;
    if (fixed ? l >= fixed->size()
              : (out.lev.back().A.nr <= prm_p.coarse_size || (int)out.lev.size() >= max_levels))
      break;
    AmgLevelHost &L = out.lev.back();
    const int n = L.A.nr;
    const int lo[2] = {0, npl}, hi[2] = {npl, n};
    HostCSR blk[2];
    std::vector<int> ab[2];
    int na[2] = {0, 0};
    for (int u = 0; u < 2; u++) blk[u] = diag_block(L.A, lo[u], hi[u]);
    if (fixed) {
      const std::vector<int> &f = (*fixed)[l];
      if ((int)f.size() != n) throw Error{CPTR_ERR_SETUP, "aggregates do not match the level size"};
      int top[2] = {0, 0};
      for (int i = 0; i < n; i++) top[i >= npl] = std::max(top[i >= npl], f[i] + 1);
      na[0] = top[0];
      na[1] = std::max(0, top[1] - na[0]);
      for (int u = 0; u < 2; u++) {
        ab[u].resize(hi[u] - lo[u]);
        for (int i = lo[u]; i < hi[u]; i++) {
          const int a = f[i] < 0 ? -1 : f[i] - (u ? na[0] : 0);
          if (a < -1 || a >= na[u]) throw Error{CPTR_ERR_SETUP, "aggregates mix the unknowns"};
          ab[u][i - lo[u]] = a;
        }
      }
    } else {
      for (int u = 0; u < 2; u++) {
        Graph g = strength(blk[u], theta);
        na[u] = aggregate(g, hi[u] - lo[u], prm_p.seed, ab[u]);
      }
      if (na[0] + na[1] >= n) break;  // no coarsening possible
    }
    HostCSR pb[2];
    double om[2] = {0.0, 0.0};
    for (int u = 0; u < 2; u++) {
      const bool smooth = (u == 0 ? prm_p.smooth_p : prm_T.smooth_p) && hi[u] > lo[u];
      pb[u] = prolongator(blk[u], ab[u], na[u], smooth, om[u]);
    }
    // P = diag(P_p, P_T): temperature columns and aggregates shifted by na_p
    L.agg.assign(n, -1);
    L.P = HostCSR();
    L.P.nr = n;
    L.P.nc = na[0] + na[1];
    L.P.rp.assign(n + 1, 0);
    for (int u = 0; u < 2; u++) {
      const int off = u == 0 ? 0 : na[0];
      for (int i = 0; i < hi[u] - lo[u]; i++) {
        if (ab[u][i] >= 0) L.agg[lo[u] + i] = ab[u][i] + off;
        for (int k = pb[u].rp[i]; k < pb[u].rp[i + 1]; k++) {
          L.P.ci.push_back(pb[u].ci[k] + off);
          L.P.v.push_back(pb[u].v[k]);
        }
        L.P.rp[lo[u] + i + 1] = L.P.nnz();
      }
    }
    L.omega = om[0];
    L.R = transpose(L.P);
    HostCSR t = multiply(L.A, L.P);
    HostCSR ac = multiply(L.R, t);
    out.lev.emplace_back();
    out.lev.back().A = std::move(ac);
    npl = na[0];
    theta *= 0.5;
  }
  finish(out);
}

void amg_build(const HostCSR &fine, const AmgParams &prm, AmgHost &out,
               const std::vector<std::vector<int>> *fixed) {
  out.lev.clear();
  out.lev.emplace_back();
  out.lev[0].A = fine;
  double theta = prm.theta;
  int max_levels = std::min(prm.max_levels, 16);
  for (;;) {
    const size_t l = out.lev.size() - 1;
    if (fixed ? l >= fixed->size() : (out.lev.back().A.nr <= prm.coarse_size || (int)out.lev.size() >= max_levels))
      break;
    AmgLevelHost &L = out.lev.back();
    int n = L.A.nr;
    std::vector<int> agg;
    int na = 0;
    if (fixed) {
      agg = (*fixed)[l];
      if ((int)agg.size() != n) throw Error{CPTR_ERR_SETUP, "aggregates do not match the level size"};
      for (int a : agg) na = std::max(na, a + 1);
    } else {
      Graph g = strength(L.A, theta);
      na = aggregate(g, n, prm.seed, agg);
      if (na >= n) break;  // no coarsening possible
    }
    L.agg = agg;
    L.smooth = prm.smooth_p != 0;
    if (prm.smooth_p)
      L.P = prolongator(L.A, agg, na, true, L.omega);
    else
      L.P = prolongator(L.A, agg, na, false, L.omega);
    L.R = transpose(L.P);
    HostCSR t = multiply(L.A, L.P);
    HostCSR ac = multiply(L.R, t);
    t.v.clear();
    t.v.shrink_to_fit();
    L.AP = std::move(t);
    out.lev.emplace_back();
    out.lev.back().A = std::move(ac);
    theta *= 0.5;
  }
  finish(out);
}

}  // namespace cptr
