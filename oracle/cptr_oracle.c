/*
 * Oracle for the CPTR-FGMRES path: plain FP64 CPU code, written for reading,
 * not for speed.  TEST INFRASTRUCTURE ONLY (see cptr_oracle.h).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liborc.so cptr_oracle.c -lm
 * Floating-point contraction is off so that the aggregation decisions taken in
 * FP64 are reproducible bit for bit.
 */
#include "cptr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV 16

/* ------------------------------------------------------------------------ */
/* small sparse containers                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nr, nc, nnz;
  int *rp, *ci;
  double *v;
} csr;

static void csr_alloc(csr *a, int nr, int nc, int nnz) {
  a->nr = nr;
  a->nc = nc;
  a->nnz = nnz;
  a->rp = (int *)calloc((size_t)nr + 1, sizeof(int));
  a->ci = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
  a->v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
}

static void csr_free(csr *a) {
  free(a->rp);
  free(a->ci);
  free(a->v);
  memset(a, 0, sizeof(*a));
}

/* y = A x */
static void csr_mv(const csr *a, const double *x, double *y) {
  for (int i = 0; i < a->nr; i++) {
    double s = 0.0;
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) s += a->v[k] * x[a->ci[k]];
    y[i] = s;
  }
}

/* value of entry (i, j), 0 if not in the pattern (columns ascending) */
static double csr_get(const csr *a, int i, int j) {
  int lo = a->rp[i], hi = a->rp[i + 1] - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (a->ci[mid] == j) return a->v[mid];
    if (a->ci[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return 0.0;
}

static csr csr_transpose(const csr *a) {
  csr t;
  csr_alloc(&t, a->nc, a->nr, a->nnz);
  for (int k = 0; k < a->nnz; k++) t.rp[a->ci[k] + 1]++;
  for (int i = 0; i < a->nc; i++) t.rp[i + 1] += t.rp[i];
  int *pos = (int *)malloc(sizeof(int) * ((size_t)a->nc + 1));
  memcpy(pos, t.rp, sizeof(int) * ((size_t)a->nc + 1));
  for (int i = 0; i < a->nr; i++)
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
      int p = pos[a->ci[k]]++;
      t.ci[p] = i;      /* rows visited ascending => columns of t ascending */
      t.v[p] = a->v[k];
    }
  free(pos);
  return t;
}

void orc_bsr_spmv(int n, int nv, const int *rp, const int *ci, const double *v,
                  const double *x, double *y) {
  for (int i = 0; i < n; i++)
    for (int r = 0; r < nv; r++) {
      double s = 0.0;
      for (int k = rp[i]; k < rp[i + 1]; k++)
        for (int c = 0; c < nv; c++)
          s += v[(size_t)k * nv * nv + r * nv + c] * x[(size_t)ci[k] * nv + c];
      y[(size_t)i * nv + r] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* dense LU with partial pivoting (coarsest AMG level, exact second stage)    */
/* ------------------------------------------------------------------------ */
static int lu_factor(double *a, int *piv, int n) {
  for (int k = 0; k < n; k++) {
    int p = k;
    double best = fabs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; i++)
      if (fabs(a[(size_t)i * n + k]) > best) { best = fabs(a[(size_t)i * n + k]); p = i; }
    piv[k] = p;
    if (best == 0.0) return -1;
    if (p != k)
      for (int j = 0; j < n; j++) {
        double t = a[(size_t)k * n + j];
        a[(size_t)k * n + j] = a[(size_t)p * n + j];
        a[(size_t)p * n + j] = t;
      }
    for (int i = k + 1; i < n; i++) {
      double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
      a[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; j++) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
    }
  }
  return 0;
}

/* Solve with the factor of lu_factor: rows were swapped whole (multipliers
 * included), so the row interchanges are applied to x first, then the unit
 * lower and the upper triangular solves. */
static void lu_solve(const double *a, const int *piv, int n, double *x) {
  for (int k = 0; k < n; k++) {
    double t = x[k];
    x[k] = x[piv[k]];
    x[piv[k]] = t;
  }
  for (int k = 0; k < n; k++)
    for (int i = k + 1; i < n; i++) x[i] -= a[(size_t)i * n + k] * x[k];
  for (int i = n - 1; i >= 0; i--) {
    double s = x[i];
    for (int j = i + 1; j < n; j++) s -= a[(size_t)i * n + j] * x[j];
    x[i] = s / a[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* smoothed aggregation AMG                                                   */
/* (Vanek, Mandel, Brezina 1996; aggregation by a distance-2 maximal         */
/*  independent set).  It stands in for the AMG V-cycles that approximate   */
/*  A_pp^{-1} and S~_T^{-1} in the block preconditioner (Section 3.3).       */
/* ------------------------------------------------------------------------ */

/* MurmurHash3 32-bit finalizer (public domain). */
unsigned orc_fmix32(unsigned h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* priority order: (fmix32(i ^ seed), i) compared lexicographically */
static int prio_greater(int a, int b, unsigned seed) {
  unsigned ha = orc_fmix32((unsigned)a ^ seed), hb = orc_fmix32((unsigned)b ^ seed);
  if (ha != hb) return ha > hb;
  return a > b;
}

/* Strength of connection on the symmetric part:
 *   i ~ j  (j != i)  iff  s*s >= theta^2 |a_ii a_jj|,  s = (a_ij + a_ji) * 0.5
 * evaluated in FP64 exactly in this order of operations.  The pattern must be
 * structurally symmetric.  Output: strength graph as CSR without diagonal. */
int orc_strength(int n, const int *rp, const int *ci, const double *v, double theta,
                 int *srp, int *sci) {
  csr a = {n, n, rp[n], (int *)rp, (int *)ci, (double *)v};
  double t2 = theta * theta;
  int cnt = 0;
  srp[0] = 0;
  for (int i = 0; i < n; i++) {
    double aii = csr_get(&a, i, i);
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      int j = ci[k];
      if (j == i) continue;
      double aji = csr_get(&a, j, i);
      double ajj = csr_get(&a, j, j);
      double s = (v[k] + aji) * 0.5;
      double lhs = s * s;
      double rhs = t2 * fabs(aii * ajj);
      if (lhs >= rhs) {
        if (sci) sci[cnt] = j;
        cnt++;
      }
    }
    srp[i + 1] = cnt;
  }
  return cnt;
}

static int g_seed_for_sort;
static int cmp_prio_desc(const void *pa, const void *pb) {
  int a = *(const int *)pa, b = *(const int *)pb;
  if (a == b) return 0;
  return prio_greater(a, b, (unsigned)g_seed_for_sort) ? -1 : 1;
}

/* Lexicographically-first distance-2 maximal independent set, sequential
 * greedy form: visit nodes by descending priority; a node not yet excluded
 * becomes a root and excludes every node within strength distance 2. */
int orc_mis2_greedy(int n, const int *srp, const int *sci, unsigned seed, int *is_root) {
  int *order = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  char *excl = (char *)calloc((size_t)n + 1, 1);
  for (int i = 0; i < n; i++) order[i] = i;
  g_seed_for_sort = (int)seed;
  qsort(order, (size_t)n, sizeof(int), cmp_prio_desc);
  int nroots = 0;
  for (int i = 0; i < n; i++) is_root[i] = 0;
  for (int t = 0; t < n; t++) {
    int r = order[t];
    if (excl[r]) continue;
    is_root[r] = 1;
    nroots++;
    excl[r] = 1;
    for (int k = srp[r]; k < srp[r + 1]; k++) {
      int j = sci[k];
      excl[j] = 1;
      for (int q = srp[j]; q < srp[j + 1]; q++) excl[sci[q]] = 1;
    }
  }
  free(order);
  free(excl);
  return nroots;
}

typedef struct {
  int nlev;
  csr A[MAXLEV];      /* level operators, A[0] = fine */
  csr P[MAXLEV];      /* prolongation level l+1 -> l   (n_l x n_{l+1}) */
  csr R[MAXLEV];      /* restriction = P^T */
  int *agg[MAXLEV];   /* aggregate of each node of level l */
  double *dl1[MAXLEV];/* l1 row sums */
  double omega[MAXLEV];
  int sweeps;
  int smoother;       /* 0: l1-Jacobi, 1: multicolour Gauss-Seidel */
  int *color[MAXLEV]; /* greedy colouring of each level (Gauss-Seidel) */
  int ncolor[MAXLEV];
  double *lu;         /* coarsest dense LU */
  int *piv;
} amg;

/* Aggregation (ordered steps, all deterministic):
 *  1. strength graph;  2./3. MIS-2 roots (greedy, descending priority);
 *  4. aggregate = root + its strong neighbours;
 *  5. each remaining node joins the step-4 aggregate of a strong neighbour
 *     whose root has the largest priority;
 *  6. strength-isolated nodes belong to no aggregate (zero tentative row);
 *  7. aggregates numbered by ascending root index. */
static int aggregate(int n, const int *srp, const int *sci, unsigned seed, int *agg,
                     int *nagg) {
  int *root = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  orc_mis2_greedy(n, srp, sci, seed, root);
  int *id = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *rootof = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int na = 0;
  /* step 6: a node without strong neighbours (always a root of the MIS-2)
   * belongs to no aggregate: its row of the tentative prolongator is zero */
  for (int i = 0; i < n; i++)
    if (srp[i + 1] == srp[i]) root[i] = 0;
  for (int i = 0; i < n; i++) id[i] = root[i] ? na++ : -1;
  for (int i = 0; i < n; i++) { agg[i] = -1; rootof[i] = -1; }
  for (int r = 0; r < n; r++) {
    if (!root[r]) continue;
    agg[r] = id[r];
    rootof[r] = r;
    for (int k = srp[r]; k < srp[r + 1]; k++) {
      agg[sci[k]] = id[r];
      rootof[sci[k]] = r;
    }
  }
  int *agg4 = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *root4 = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  memcpy(agg4, agg, sizeof(int) * (size_t)n);
  memcpy(root4, rootof, sizeof(int) * (size_t)n);
  int bad = 0;
  for (int i = 0; i < n; i++) {
    if (agg4[i] >= 0 || srp[i + 1] == srp[i]) continue;
    int best = -1;
    for (int k = srp[i]; k < srp[i + 1]; k++) {
      int j = sci[k];
      if (agg4[j] < 0) continue;
      if (best < 0 || prio_greater(root4[j], best, seed)) best = root4[j];
    }
    if (best < 0) { bad = 1; continue; }   /* cannot happen: see step 6 */
    agg[i] = id[best];
  }
  free(agg4); free(root4); free(rootof); free(id); free(root);
  *nagg = na;
  return bad ? -1 : 0;
}

/* P = (I - omega D^{-1} A) P_tent, omega = 4 / (3 rho),
 * rho = max_i sum_j |a_ij| / |a_ii|.
 * Entry (i, J) = [agg(i) = J] - (omega / a_ii) * (sum over j in row i with agg(j) = J
 * of a_ij, summed in ascending j).  Columns of each row ascending. */
static csr smooth_prolongator(const csr *a, const int *agg, int nagg, double *omega_out,
                              int smooth) {
  int n = a->nr;
  double rho = 0.0;
  for (int i = 0; i < n; i++) {
    double s = 0.0;
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) s += fabs(a->v[k]);
    double q = s / fabs(csr_get(a, i, i));
    if (q > rho) rho = q;
  }
  double omega = smooth ? 4.0 / (3.0 * rho) : 0.0;
  *omega_out = omega;
  /* count distinct aggregates per row */
  int *mark = (int *)malloc(sizeof(int) * (size_t)(nagg > 0 ? nagg : 1));
  double *acc = (double *)calloc((size_t)(nagg > 0 ? nagg : 1), sizeof(double));
  for (int J = 0; J < nagg; J++) mark[J] = -1;
  int nnz = 0;
  for (int i = 0; i < n; i++) {
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
      int J = agg[a->ci[k]];
      if (J >= 0 && mark[J] != i) { mark[J] = i; nnz++; }
    }
    if (agg[i] >= 0 && mark[agg[i]] != i) { mark[agg[i]] = i; nnz++; }
  }
  csr p;
  csr_alloc(&p, n, nagg, nnz);
  for (int J = 0; J < nagg; J++) mark[J] = -1;
  int *cols = (int *)malloc(sizeof(int) * 64);
  int cap = 64;
  int pos = 0;
  for (int i = 0; i < n; i++) {
    int nc = 0;
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
      int J = agg[a->ci[k]];
      if (J < 0) continue;
      if (mark[J] != i) {
        mark[J] = i;
        acc[J] = 0.0;
        if (nc == cap) { cap *= 2; cols = (int *)realloc(cols, sizeof(int) * (size_t)cap); }
        cols[nc++] = J;
      }
      acc[J] += a->v[k];
    }
    if (agg[i] >= 0 && mark[agg[i]] != i) {
      mark[agg[i]] = i;
      acc[agg[i]] = 0.0;
      if (nc == cap) { cap *= 2; cols = (int *)realloc(cols, sizeof(int) * (size_t)cap); }
      cols[nc++] = agg[i];
    }
    /* ascending column order (insertion sort: rows are short) */
    for (int x = 1; x < nc; x++) {
      int t = cols[x], y = x - 1;
      while (y >= 0 && cols[y] > t) { cols[y + 1] = cols[y]; y--; }
      cols[y + 1] = t;
    }
    double w = omega / csr_get(a, i, i);
    for (int x = 0; x < nc; x++) {
      int J = cols[x];
      double d = (J == agg[i]) ? 1.0 : 0.0;
      p.ci[pos] = J;
      p.v[pos] = d - w * acc[J];
      pos++;
    }
    p.rp[i + 1] = pos;
  }
  free(cols); free(acc); free(mark);
  return p;
}

/* C = A B with entries accumulated over ascending inner index. */
static csr spgemm(const csr *a, const csr *b) {
  int *mark = (int *)malloc(sizeof(int) * (size_t)(b->nc > 0 ? b->nc : 1));
  double *acc = (double *)calloc((size_t)(b->nc > 0 ? b->nc : 1), sizeof(double));
  for (int j = 0; j < b->nc; j++) mark[j] = -1;
  int nnz = 0;
  for (int i = 0; i < a->nr; i++)
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
      int m = a->ci[k];
      for (int q = b->rp[m]; q < b->rp[m + 1]; q++)
        if (mark[b->ci[q]] != i) { mark[b->ci[q]] = i; nnz++; }
    }
  csr c;
  csr_alloc(&c, a->nr, b->nc, nnz);
  for (int j = 0; j < b->nc; j++) mark[j] = -1;
  int *cols = (int *)malloc(sizeof(int) * (size_t)(b->nc > 0 ? b->nc : 1));
  int pos = 0;
  for (int i = 0; i < a->nr; i++) {
    int nc = 0;
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
      int m = a->ci[k];
      for (int q = b->rp[m]; q < b->rp[m + 1]; q++) {
        int j = b->ci[q];
        if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[nc++] = j; }
        acc[j] += a->v[k] * b->v[q];
      }
    }
    for (int x = 1; x < nc; x++) {
      int t = cols[x], y = x - 1;
      while (y >= 0 && cols[y] > t) { cols[y + 1] = cols[y]; y--; }
      cols[y + 1] = t;
    }
    for (int x = 0; x < nc; x++) { c.ci[pos] = cols[x]; c.v[pos] = acc[cols[x]]; pos++; }
    c.rp[i + 1] = pos;
  }
  free(cols); free(acc); free(mark);
  return c;
}

static csr csr_copy(int n, const int *rp, const int *ci, const double *v) {
  csr a;
  csr_alloc(&a, n, n, rp[n]);
  memcpy(a.rp, rp, sizeof(int) * ((size_t)n + 1));
  memcpy(a.ci, ci, sizeof(int) * (size_t)rp[n]);
  memcpy(a.v, v, sizeof(double) * (size_t)rp[n]);
  return a;
}

static void amg_free(amg *m) {
  for (int l = 0; l < m->nlev; l++) {
    csr_free(&m->A[l]);
    if (l + 1 < m->nlev) { csr_free(&m->P[l]); csr_free(&m->R[l]); }
    free(m->agg[l]); free(m->dl1[l]); free(m->color[l]);
  }
  free(m->lu); free(m->piv);
  memset(m, 0, sizeof(*m));
}

/* Hierarchy: coarsen while n > coarse_size and fewer than max_levels levels;
 * theta is halved from one level to the next; coarsest level: dense LU. */
static csr tentative(int n, const int *agg, int nagg) {
  csr p;
  csr_alloc(&p, n, nagg, n);
  int pos = 0;
  for (int i = 0; i < n; i++) {
    if (agg[i] >= 0) { p.ci[pos] = agg[i]; p.v[pos] = 1.0; pos++; }
    p.rp[i + 1] = pos;
  }
  p.nnz = pos;
  return p;
}

static int amg_finish(amg *m);

static int amg_setup(amg *m, csr fine, double theta, int max_levels, int coarse_size,
                     unsigned seed, int sweeps, int smooth_p, int smoother) {
  memset(m, 0, sizeof(*m));
  m->sweeps = sweeps;
  m->smoother = smoother;
  if (max_levels > MAXLEV) max_levels = MAXLEV;
  m->A[0] = fine;
  int l = 0;
  double th = theta;
  while (m->A[l].nr > coarse_size && l + 1 < max_levels) {
    int n = m->A[l].nr, nagg = 0;
    int *agg = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *srp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int ns = orc_strength(n, m->A[l].rp, m->A[l].ci, m->A[l].v, th, srp, NULL);
    int *sci = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
    orc_strength(n, m->A[l].rp, m->A[l].ci, m->A[l].v, th, srp, sci);
    if (aggregate(n, srp, sci, seed, agg, &nagg) != 0) {
      free(agg); free(srp); free(sci);
      return -2;
    }
    if (nagg >= n) { free(agg); free(srp); free(sci); break; }  /* no coarsening possible */
    m->agg[l] = agg;
    if (smooth_p)
      m->P[l] = smooth_prolongator(&m->A[l], agg, nagg, &m->omega[l], 1);
    else
      m->P[l] = tentative(n, agg, nagg);
    free(srp);
    free(sci);
    m->R[l] = csr_transpose(&m->P[l]);
    csr t = spgemm(&m->A[l], &m->P[l]);
    m->A[l + 1] = spgemm(&m->R[l], &t);
    csr_free(&t);
    l++;
    th *= 0.5;
  }
  m->nlev = l + 1;
  return amg_finish(m);
}

/* Per-level smoother data (l1 row sums, colouring) and the coarsest dense LU of
 * a hierarchy whose operators and transfers are built. */
static int amg_finish(amg *m) {
  for (int k = 0; k < m->nlev; k++) {
    int n = m->A[k].nr;
    m->dl1[k] = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++) {
      double s = 0.0;
      for (int q = m->A[k].rp[i]; q < m->A[k].rp[i + 1]; q++) s += fabs(m->A[k].v[q]);
      m->dl1[k][i] = s;
    }
    /* greedy colouring in natural order: smallest colour unused by lower neighbours */
    m->color[k] = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    m->ncolor[k] = 0;
    for (int i = 0; i < n; i++) {
      int c = 0;
      for (;;) {
        int used = 0;
        for (int q = m->A[k].rp[i]; q < m->A[k].rp[i + 1]; q++)
          if (m->A[k].ci[q] < i && m->color[k][m->A[k].ci[q]] == c) { used = 1; break; }
        if (!used) break;
        c++;
      }
      m->color[k][i] = c;
      if (c + 1 > m->ncolor[k]) m->ncolor[k] = c + 1;
    }
  }
  int nc = m->A[m->nlev - 1].nr;
  if (nc > 4096) return -3;   /* coarsening stalled: refuse a huge dense LU */
  m->lu = (double *)calloc((size_t)nc * nc + 1, sizeof(double));
  m->piv = (int *)malloc(sizeof(int) * ((size_t)nc + 1));
  const csr *c = &m->A[m->nlev - 1];
  for (int i = 0; i < nc; i++)
    for (int q = c->rp[i]; q < c->rp[i + 1]; q++) m->lu[(size_t)i * nc + c->ci[q]] = c->v[q];
  if (lu_factor(m->lu, m->piv, nc) != 0) return -4;
  return 0;
}

/* Rows and columns r0 .. r1-1 of a square CSR, renumbered from 0. */
static csr sub_block(const csr *a, int r0, int r1) {
  int n = r1 - r0, cnt = 0;
  for (int i = r0; i < r1; i++)
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++) cnt += a->ci[k] >= r0 && a->ci[k] < r1;
  csr b;
  csr_alloc(&b, n, n, cnt);
  int pos = 0;
  for (int i = r0; i < r1; i++) {
    for (int k = a->rp[i]; k < a->rp[i + 1]; k++)
      if (a->ci[k] >= r0 && a->ci[k] < r1) { b.ci[pos] = a->ci[k] - r0; b.v[pos] = a->v[k]; pos++; }
    b.rp[i - r0 + 1] = pos;
  }
  return b;
}

/* Unknown-based AMG (Section 3.4) for the pressure-temperature operator A_00
 * in unknown-wise order: the np pressure rows, then the temperature rows.  At
 * every level each unknown is coarsened on its own: strength, aggregation and
 * prolongator are those of the scalar hierarchy above, applied to the diagonal
 * block of that unknown (pressure: smooth_p, temperature: smooth_pT).  So
 * P = diag(P_p, P_T), the Galerkin coarse operator P^T A P keeps the
 * pressure-temperature couplings, and the coarse unknowns are again in
 * unknown-wise order (pressure aggregates first, temperature aggregates
 * numbered after them).  Smoothing acts on the whole coupled rows.  The
 * hierarchy stops on the total size, as the scalar one does, and when neither
 * block coarsens.  omega[l] records the pressure block's weight. */
static int uamg_setup(amg *m, csr fine, int np, double theta, int max_levels, int coarse_size,
                      unsigned seed, int sweeps, int smooth_p, int smooth_pT, int smoother) {
  memset(m, 0, sizeof(*m));
  m->sweeps = sweeps;
  m->smoother = smoother;
  if (max_levels > MAXLEV) max_levels = MAXLEV;
  m->A[0] = fine;
  int l = 0, npl = np;
  double th = theta;
  while (m->A[l].nr > coarse_size && l + 1 < max_levels) {
    int n = m->A[l].nr;
    int r0[2] = {0, npl}, r1[2] = {npl, n}, na[2] = {0, 0};
    int *ab[2];
    csr d[2];
    int bad = 0;
    for (int u = 0; u < 2; u++) {
      int nb = r1[u] - r0[u];
      d[u] = sub_block(&m->A[l], r0[u], r1[u]);
      ab[u] = (int *)malloc(sizeof(int) * (size_t)(nb > 0 ? nb : 1));
      int *srp = (int *)malloc(sizeof(int) * ((size_t)nb + 1));
      int ns = orc_strength(nb, d[u].rp, d[u].ci, d[u].v, th, srp, NULL);
      int *sci = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
      orc_strength(nb, d[u].rp, d[u].ci, d[u].v, th, srp, sci);
      if (aggregate(nb, srp, sci, seed, ab[u], &na[u]) != 0) bad = 1;
      free(srp);
      free(sci);
    }
    if (bad || na[0] + na[1] >= n) {
      for (int u = 0; u < 2; u++) { csr_free(&d[u]); free(ab[u]); }
      if (bad) return -2;
      break;  /* no coarsening possible */
    }
    csr pb[2];
    double om[2] = {0.0, 0.0};
    for (int u = 0; u < 2; u++) {
      int nb = r1[u] - r0[u];
      if ((u == 0 ? smooth_p : smooth_pT) && nb > 0)
        pb[u] = smooth_prolongator(&d[u], ab[u], na[u], &om[u], 1);
      else
        pb[u] = tentative(nb, ab[u], na[u]);
    }
    /* P = diag(P_p, P_T), aggregates of the temperature block shifted by na_p */
    int *agg = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    csr P;
    csr_alloc(&P, n, na[0] + na[1], pb[0].nnz + pb[1].nnz);
    int pos = 0;
    for (int u = 0; u < 2; u++) {
      int off = u == 0 ? 0 : na[0];
      for (int i = 0; i < r1[u] - r0[u]; i++) {
        agg[r0[u] + i] = ab[u][i] < 0 ? -1 : ab[u][i] + off;
        for (int k = pb[u].rp[i]; k < pb[u].rp[i + 1]; k++) {
          P.ci[pos] = pb[u].ci[k] + off;
          P.v[pos] = pb[u].v[k];
          pos++;
        }
        P.rp[r0[u] + i + 1] = pos;
      }
    }
    for (int u = 0; u < 2; u++) { csr_free(&d[u]); csr_free(&pb[u]); free(ab[u]); }
    m->agg[l] = agg;
    m->P[l] = P;
    m->omega[l] = om[0];
    m->R[l] = csr_transpose(&m->P[l]);
    csr t = spgemm(&m->A[l], &m->P[l]);
    m->A[l + 1] = spgemm(&m->R[l], &t);
    csr_free(&t);
    npl = na[0];
    l++;
    th *= 0.5;
  }
  m->nlev = l + 1;
  return amg_finish(m);
}

/* one multicolour Gauss-Seidel sweep: colours in ascending (or descending)
 * order; rows of one colour are not coupled, so each colour is one Jacobi
 * update with the latest values of the other colours */
static void gs_sweep(const amg *m, int l, const double *b, double *x, int reverse) {
  const csr *a = &m->A[l];
  for (int cc = 0; cc < m->ncolor[l]; cc++) {
    int c = reverse ? m->ncolor[l] - 1 - cc : cc;
    for (int i = 0; i < a->nr; i++) {
      if (m->color[l][i] != c) continue;
      double s = b[i], d = 0.0;
      for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
        if (a->ci[k] == i) d = a->v[k];
        else s -= a->v[k] * x[a->ci[k]];
      }
      x[i] = s / d;
    }
  }
}

/* One V-cycle from a zero initial guess on level l: `sweeps` pre-smoothing
 * sweeps (l1-Jacobi, x += D_l1^{-1}(b - A x), or forward multicolour
 * Gauss-Seidel), the residual, restriction by R = P^T, the cycle on the next
 * level, prolongation, then `sweeps` post-smoothing sweeps (l1-Jacobi, or
 * Gauss-Seidel with the colours in descending order); the coarsest level is
 * solved exactly by its LU factors. */
static void vcycle(const amg *m, int l, const double *b, double *x) {
  const csr *a = &m->A[l];
  int n = a->nr;
  if (l == m->nlev - 1) {
    memcpy(x, b, sizeof(double) * (size_t)n);
    lu_solve(m->lu, m->piv, n, x);
    return;
  }
  int nc = m->A[l + 1].nr;
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *bc = (double *)malloc(sizeof(double) * (size_t)nc);
  double *xc = (double *)malloc(sizeof(double) * (size_t)nc);
  if (m->smoother == 1) {
    for (int i = 0; i < n; i++) x[i] = 0.0;
    for (int s = 0; s < m->sweeps; s++) gs_sweep(m, l, b, x, 0);
  } else {
    for (int i = 0; i < n; i++) x[i] = b[i] / m->dl1[l][i];     /* x = 0 + D^{-1}(b - A 0) */
    for (int s = 1; s < m->sweeps; s++) {
      csr_mv(a, x, t);
      for (int i = 0; i < n; i++) x[i] += (b[i] - t[i]) / m->dl1[l][i];
    }
  }
  csr_mv(a, x, t);
  for (int i = 0; i < n; i++) r[i] = b[i] - t[i];
  csr_mv(&m->R[l], r, bc);
  vcycle(m, l + 1, bc, xc);
  csr_mv(&m->P[l], xc, t);
  for (int i = 0; i < n; i++) x[i] += t[i];
  for (int s = 0; s < m->sweeps; s++) {
    if (m->smoother == 1) {
      gs_sweep(m, l, b, x, 1);
      continue;
    }
    csr_mv(a, x, t);
    for (int i = 0; i < n; i++) x[i] += (b[i] - t[i]) / m->dl1[l][i];
  }
  free(t); free(r); free(bc); free(xc);
}

/* ------------------------------------------------------------------------ */
/* block ILU(0)                                                               */
/* Saad, Iterative Methods for Sparse Linear Systems, the IKJ form of ILU(0) */
/* (Algorithm 10.4), applied to nv x nv blocks on the BSR pattern.  The     */
/* second stage of CPR/CPTR uses ILU(0) (Section 4 implementation notes).  */
/* ------------------------------------------------------------------------ */
static void blk_mul(int nv, const double *a, const double *b, double *c) {
  for (int r = 0; r < nv; r++)
    for (int q = 0; q < nv; q++) {
      double s = 0.0;
      for (int k = 0; k < nv; k++) s += a[r * nv + k] * b[k * nv + q];
      c[r * nv + q] = s;
    }
}

/* Gauss-Jordan inverse with partial pivoting */
static int blk_inv(int nv, const double *a, double *inv) {
  double m[8][16];
  for (int r = 0; r < nv; r++)
    for (int q = 0; q < 2 * nv; q++)
      m[r][q] = q < nv ? a[r * nv + q] : (q - nv == r ? 1.0 : 0.0);
  for (int k = 0; k < nv; k++) {
    int p = k;
    for (int r = k + 1; r < nv; r++) if (fabs(m[r][k]) > fabs(m[p][k])) p = r;
    if (m[p][k] == 0.0) return -1;
    if (p != k)
      for (int q = 0; q < 2 * nv; q++) { double t = m[k][q]; m[k][q] = m[p][q]; m[p][q] = t; }
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
  return 0;
}

typedef struct {
  int n, nv;
  int *rp, *ci;      /* pattern (in factor order) */
  int *diag;         /* slot of the diagonal block of each row */
  double *lu;        /* L (strictly lower, unit diag implied) and U (strictly upper) */
  double *dinv;      /* inverses of the U diagonal blocks */
  int *perm;         /* factor row r <- original row perm[r] (NULL: identity) */
  int *color;
  int ncolor;
  int *lev_lower, *lev_upper;
  double *y;
} bilu;

static int bilu_factor(bilu *f) {
  int n = f->n, nv = f->nv, b2 = nv * nv;
  double tmp[64];
  for (int i = 0; i < n; i++) {
    for (int k = f->rp[i]; k < f->rp[i + 1]; k++) {
      int kc = f->ci[k];
      if (kc >= i) break;
      /* a_ik <- a_ik * U_kk^{-1} */
      blk_mul(nv, f->lu + (size_t)k * b2, f->dinv + (size_t)kc * b2, tmp);
      memcpy(f->lu + (size_t)k * b2, tmp, sizeof(double) * b2);
      /* a_ij -= a_ik * u_kj for j > k present in both rows */
      for (int q = f->diag[kc] + 1; q < f->rp[kc + 1]; q++) {
        int j = f->ci[q];
        for (int s = k + 1; s < f->rp[i + 1]; s++) {
          if (f->ci[s] != j) continue;
          double prod[64];
          blk_mul(nv, f->lu + (size_t)k * b2, f->lu + (size_t)q * b2, prod);
          for (int e = 0; e < b2; e++) f->lu[(size_t)s * b2 + e] -= prod[e];
        }
      }
    }
    if (blk_inv(nv, f->lu + (size_t)f->diag[i] * b2, f->dinv + (size_t)i * b2) != 0)
      return -1;
  }
  return 0;
}

/* x = (LU)^{-1} b in factor order */
static void bilu_solve_perm(const bilu *f, const double *b, double *x) {
  int n = f->n, nv = f->nv, b2 = nv * nv;
  double *y = f->y;
  for (int i = 0; i < n; i++) {
    double s[8];
    for (int r = 0; r < nv; r++) s[r] = b[(size_t)i * nv + r];
    for (int k = f->rp[i]; k < f->diag[i]; k++) {
      const double *l = f->lu + (size_t)k * b2;
      const double *yk = y + (size_t)f->ci[k] * nv;
      for (int r = 0; r < nv; r++)
        for (int c = 0; c < nv; c++) s[r] -= l[r * nv + c] * yk[c];
    }
    for (int r = 0; r < nv; r++) y[(size_t)i * nv + r] = s[r];
  }
  for (int i = n - 1; i >= 0; i--) {
    double s[8];
    for (int r = 0; r < nv; r++) s[r] = y[(size_t)i * nv + r];
    for (int k = f->diag[i] + 1; k < f->rp[i + 1]; k++) {
      const double *u = f->lu + (size_t)k * b2;
      const double *xk = x + (size_t)f->ci[k] * nv;
      for (int r = 0; r < nv; r++)
        for (int c = 0; c < nv; c++) s[r] -= u[r * nv + c] * xk[c];
    }
    const double *d = f->dinv + (size_t)i * b2;
    for (int r = 0; r < nv; r++) {
      double t = 0.0;
      for (int c = 0; c < nv; c++) t += d[r * nv + c] * s[c];
      x[(size_t)i * nv + r] = t;
    }
  }
}

static void bilu_free(bilu *f) {
  free(f->rp); free(f->ci); free(f->diag); free(f->lu); free(f->dinv); free(f->perm);
  free(f->color); free(f->lev_lower); free(f->lev_upper); free(f->y);
  memset(f, 0, sizeof(*f));
}

/* Setup.  multicolor = 0: natural order.  multicolor = 1: greedy colouring in
 * natural order (smallest colour unused by earlier neighbours), rows
 * renumbered colour by colour (ascending index inside a colour), then ILU(0)
 * of the renumbered matrix. */
/* Level-1 fill of block ILU(1) (Section 4: ILU(1) as the second stage of
 * CPR-AMG-ILU(1)): with lev = 0 on the blocks of A, a block (i, j) has level
 * 1 when some k < i has (i, k) and (k, j) of level 0 with j > k; the pattern
 * keeps the blocks of level <= 1.  Replaces the (factor-order) pattern of f,
 * fill blocks zero. */
static void bilu_add_fill1(bilu *f) {
  int n = f->n, b2 = f->nv * f->nv;
  int *mark = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *slot = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int c = 0; c < n; c++) mark[c] = -1;
  int *nrp = (int *)calloc((size_t)n + 1, sizeof(int));
  for (int r = 0; r < n; r++) {
    int cnt = 0;
    for (int t = f->rp[r]; t < f->rp[r + 1]; t++) { mark[f->ci[t]] = r; cnt++; }
    for (int t = f->rp[r]; t < f->rp[r + 1]; t++) {
      int k = f->ci[t];
      if (k >= r) continue;
      for (int u = f->rp[k]; u < f->rp[k + 1]; u++) {
        int j = f->ci[u];
        if (j > k && mark[j] != r) { mark[j] = r; cnt++; }
      }
    }
    nrp[r + 1] = nrp[r] + cnt;
  }
  int nnz = nrp[n];
  int *nci = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
  double *nlu = (double *)calloc((size_t)nnz * b2 + 1, sizeof(double));
  for (int c = 0; c < n; c++) mark[c] = -1;
  for (int r = 0; r < n; r++) {
    int pos = nrp[r];
    for (int t = f->rp[r]; t < f->rp[r + 1]; t++) {
      mark[f->ci[t]] = r;
      slot[f->ci[t]] = t;
      nci[pos++] = f->ci[t];
    }
    for (int t = f->rp[r]; t < f->rp[r + 1]; t++) {
      int k = f->ci[t];
      if (k >= r) continue;
      for (int u = f->rp[k]; u < f->rp[k + 1]; u++) {
        int j = f->ci[u];
        if (j > k && mark[j] != r) { mark[j] = r; slot[j] = -1; nci[pos++] = j; }
      }
    }
    /* ascending columns (insertion sort), values of the original blocks */
    for (int a = nrp[r] + 1; a < nrp[r + 1]; a++) {
      int c = nci[a], b = a - 1;
      while (b >= nrp[r] && nci[b] > c) { nci[b + 1] = nci[b]; b--; }
      nci[b + 1] = c;
    }
    for (int a = nrp[r]; a < nrp[r + 1]; a++)
      if (slot[nci[a]] >= 0)
        memcpy(nlu + (size_t)a * b2, f->lu + (size_t)slot[nci[a]] * b2, sizeof(double) * b2);
  }
  free(f->rp); free(f->ci); free(f->lu);
  f->rp = nrp;
  f->ci = nci;
  f->lu = nlu;
  for (int r = 0; r < n; r++) {
    f->diag[r] = -1;
    for (int k = f->rp[r]; k < f->rp[r + 1]; k++) if (f->ci[k] == r) f->diag[r] = k;
  }
  free(mark);
  free(slot);
}

static int bilu_setup(bilu *f, int n, int nv, const int *rp, const int *ci,
                      const double *v, int multicolor, const int *order, const int *part,
                      int level) {
  memset(f, 0, sizeof(*f));
  int b2 = nv * nv, nnzb = rp[n];
  f->n = n;
  f->nv = nv;
  f->rp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
  f->ci = (int *)malloc(sizeof(int) * (size_t)(nnzb > 0 ? nnzb : 1));
  f->diag = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  f->lu = (double *)malloc(sizeof(double) * (size_t)nnzb * b2 + 1);
  f->dinv = (double *)malloc(sizeof(double) * (size_t)n * b2 + 1);
  f->y = (double *)malloc(sizeof(double) * (size_t)n * nv + 1);
  f->color = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *newof = NULL;
  if (multicolor) {
    int ncol = 0;
    for (int i = 0; i < n; i++) {
      int c = 0;
      for (;;) {
        int used = 0;
        for (int k = rp[i]; k < rp[i + 1]; k++)
          if (ci[k] < i && f->color[ci[k]] == c) { used = 1; break; }
        if (!used) break;
        c++;
      }
      f->color[i] = c;
      if (c + 1 > ncol) ncol = c + 1;
    }
    f->ncolor = ncol;
    f->perm = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    newof = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int pos = 0;
    for (int c = 0; c < ncol; c++)
      for (int i = 0; i < n; i++)
        if (f->color[i] == c) { f->perm[pos] = i; newof[i] = pos; pos++; }
  } else if (order) {
    /* caller-given factor order: row r of the factor is cell order[r] */
    for (int i = 0; i < n; i++) f->color[i] = 0;
    f->ncolor = 1;
    f->perm = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    newof = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int r = 0; r < n; r++) { f->perm[r] = order[r]; newof[order[r]] = r; }
  } else {
    for (int i = 0; i < n; i++) f->color[i] = 0;
    f->ncolor = 1;
  }
  /* renumbered pattern with ascending columns; with a partition, couplings
   * between different parts are dropped (block Jacobi) */
  int pos = 0;
  f->rp[0] = 0;
  for (int r = 0; r < n; r++) {
    int i = f->perm ? f->perm[r] : r;
    int len = rp[i + 1] - rp[i];
    int base = pos;
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      if (part && part[ci[k]] != part[i]) continue;
      int c = newof ? newof[ci[k]] : ci[k];
      /* insertion into ascending position */
      int y = pos - 1;
      while (y >= base && f->ci[y] > c) {
        f->ci[y + 1] = f->ci[y];
        memcpy(f->lu + (size_t)(y + 1) * b2, f->lu + (size_t)y * b2, sizeof(double) * b2);
        y--;
      }
      f->ci[y + 1] = c;
      memcpy(f->lu + (size_t)(y + 1) * b2, v + (size_t)k * b2, sizeof(double) * b2);
      pos++;
    }
    (void)len;
    f->rp[r + 1] = pos;
    f->diag[r] = -1;
    for (int k = f->rp[r]; k < f->rp[r + 1]; k++) if (f->ci[k] == r) f->diag[r] = k;
    if (f->diag[r] < 0) { free(newof); return -1; }
  }
  free(newof);
  if (level == 1) bilu_add_fill1(f);
  /* level sets of the triangular solves in factor order */
  f->lev_lower = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  f->lev_upper = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; i++) {
    int lv = 0;
    for (int k = f->rp[i]; k < f->diag[i]; k++) {
      int c = f->lev_lower[f->ci[k]] + 1;
      if (c > lv) lv = c;
    }
    f->lev_lower[i] = lv;
  }
  for (int i = n - 1; i >= 0; i--) {
    int lv = 0;
    for (int k = f->diag[i] + 1; k < f->rp[i + 1]; k++) {
      int c = f->lev_upper[f->ci[k]] + 1;
      if (c > lv) lv = c;
    }
    f->lev_upper[i] = lv;
  }
  return bilu_factor(f);
}

static void bilu_apply(const bilu *f, const double *b, double *x, double *wb, double *wx) {
  int n = f->n, nv = f->nv;
  if (!f->perm) { bilu_solve_perm(f, b, x); return; }
  for (int r = 0; r < n; r++)
    for (int u = 0; u < nv; u++) wb[(size_t)r * nv + u] = b[(size_t)f->perm[r] * nv + u];
  bilu_solve_perm(f, wb, wx);
  for (int r = 0; r < n; r++)
    for (int u = 0; u < nv; u++) x[(size_t)f->perm[r] * nv + u] = wx[(size_t)r * nv + u];
}

/* ------------------------------------------------------------------------ */
/* two-stage CPR / CPTR preconditioner                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
  orc_opts o;
  int n, nv;
  const int *rp, *ci;      /* borrowed */
  const double *v;
  csr App, ApT, ATp;       /* sub-blocks of A (eq:A00), scalar CSR on the cell graph */
  amg amg_p, amg_s;
  int have_p, have_s;
  bilu ilu;
  int have_ilu;
  double *dense_lu;        /* exact second stage */
  int *dense_piv;
  double *bp, *bt, *xp, *dt, *dp, *tmp, *x1, *b1, *wb, *wx;
  double *dcp;             /* decoupling weights D, [n][nv-1] (CPR with QI / TI) */
} orc;

static csr extract(const orc *h, int r, int c) {
  int n = h->n, nv = h->nv;
  csr a;
  csr_alloc(&a, n, n, h->rp[n]);
  memcpy(a.rp, h->rp, sizeof(int) * ((size_t)n + 1));
  memcpy(a.ci, h->ci, sizeof(int) * (size_t)h->rp[n]);
  for (int k = 0; k < h->rp[n]; k++) a.v[k] = h->v[(size_t)k * nv * nv + r * nv + c];
  return a;
}


/* The simple algebraic Schur complement approximation of Section 3.3.1:
 * S = A_TT - A_Tp diag(A_pp)^{-1} A_pT.  Row i holds every cell l reached
 * from i in at most two steps of the cell graph, columns ascending.  Entry
 * (i, l) is A_TT(i, l) (zero where A has no block), then for every block
 * (i, j) of row i in ascending j and every block (j, l) of row j in ascending l
 * it loses (A_Tp(i, j) / A_pp(j, j)) * A_pT(j, l).  Returns 0 and leaves *out
 * empty if some A_pp(j, j) is zero. */
static int schur_diag(const orc *h, csr *out) {
  int n = h->n, nv = h->nv, ip = h->o.ip, iT = h->o.iT;
  const int *rp = h->rp, *ci = h->ci;
  const double *v = h->v;
  int *mark = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  double *acc = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *app = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; i++) {
    mark[i] = -1;
    app[i] = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; k++)
      if (ci[k] == i) app[i] = v[(size_t)k * nv * nv + ip * nv + ip];
  }
  int ok = 1;
  for (int i = 0; i < n; i++) ok &= app[i] != 0.0;
  /* pattern: count, then fill and sort each row */
  int total = 0;
  for (int i = 0; i < n; i++)
    for (int k = rp[i]; k < rp[i + 1]; k++)
      for (int m = rp[ci[k]]; m < rp[ci[k] + 1]; m++)
        if (mark[ci[m]] != i) { mark[ci[m]] = i; total++; }
  csr s;
  csr_alloc(&s, n, n, total);
  for (int i = 0; i < n; i++) mark[i] = -1;
  int pos = 0;
  for (int i = 0; i < n && ok; i++) {
    int b = pos;
    for (int k = rp[i]; k < rp[i + 1]; k++)
      for (int m = rp[ci[k]]; m < rp[ci[k] + 1]; m++)
        if (mark[ci[m]] != i) { mark[ci[m]] = i; s.ci[pos++] = ci[m]; }
    for (int x = b + 1; x < pos; x++) {  /* insertion sort of the row's columns */
      int c = s.ci[x], y = x - 1;
      while (y >= b && s.ci[y] > c) { s.ci[y + 1] = s.ci[y]; y--; }
      s.ci[y + 1] = c;
    }
    for (int x = b; x < pos; x++) acc[s.ci[x]] = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; k++) acc[ci[k]] = v[(size_t)k * nv * nv + iT * nv + iT];
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      int j = ci[k];
      double a = v[(size_t)k * nv * nv + iT * nv + ip] / app[j];
      for (int m = rp[j]; m < rp[j + 1]; m++) acc[ci[m]] -= a * v[(size_t)m * nv * nv + ip * nv + iT];
    }
    for (int x = b; x < pos; x++) s.v[x] = acc[s.ci[x]];
    s.rp[i + 1] = pos;
  }
  free(mark); free(acc); free(app);
  if (!ok) { csr_free(&s); return 0; }
  *out = s;
  return 1;
}

/* Decoupling operator G = [I, -D; 0, I] of Section 3.1 for a split of the
 * unknowns into primary ones (pressure for CPR; pressure and temperature for
 * the CPTR extension of Section 3.2, S_0 = A_00 - D A_s0) and the secondary
 * unknowns s (all the others, in slot order).  D is block diagonal with one
 * npri x ns block per cell:
 *   Quasi-IMPES  D_i = A_0s[i,i] A_ss[i,i]^{-1}            (diagonal blocks)
 *   True-IMPES   D_i = colsum(A_0s)_i colsum(A_ss)_i^{-1}  (sums over the rows
 *                of block column i).
 * Each row d of D_i solves d C = a for the matching row a of the 0-s part and
 * the ns x ns s-s part C, i.e. C^T d^T = a^T.  Layout D[i][row][ns].  Returns
 * -1 if a C is singular. */
static int decoupling_weights(const orc *h, int kind, const int *pri, int npri, double *D) {
  int n = h->n, nv = h->nv, ns = nv - npri;
  int sl[4], q = 0;
  for (int k = 0; k < nv; k++) {
    int prim = 0;
    for (int a = 0; a < npri; a++) prim |= k == pri[a];
    if (!prim) sl[q++] = k;
  }
  double *blk = (double *)calloc((size_t)n * nv * nv, sizeof(double));
  for (int j = 0; j < n; j++)
    for (int k = h->rp[j]; k < h->rp[j + 1]; k++) {
      int i = h->ci[k];
      if (kind == 1 && i != j) continue;  /* QI: the diagonal block only */
      for (int e = 0; e < nv * nv; e++) blk[(size_t)i * nv * nv + e] += h->v[(size_t)k * nv * nv + e];
    }
  int st = 0;
  for (int i = 0; i < n && st == 0; i++) {
    const double *B = blk + (size_t)i * nv * nv;
    double CT[9], d[3];
    int piv[3];
    for (int a = 0; a < ns; a++)
      for (int b = 0; b < ns; b++) CT[a * ns + b] = B[sl[b] * nv + sl[a]];
    if (lu_factor(CT, piv, ns) != 0) { st = -1; break; }
    for (int r = 0; r < npri; r++) {
      for (int a = 0; a < ns; a++) d[a] = B[pri[r] * nv + sl[a]];
      lu_solve(CT, piv, ns, d);
      for (int a = 0; a < ns; a++) D[((size_t)i * npri + r) * ns + a] = d[a];
    }
  }
  free(blk);
  return st;
}

/* The pressure-temperature operator A_00 of eq:A00 in unknown-wise order:
 * [A_pp A_pT; A_Tp A_TT], pressure rows (and columns) 0..n-1, temperature
 * rows n..2n-1, each block on the cell pattern of A.  With decoupling weights
 * D ([n][2][nv-2]) it is S_0 = A_00 - D A_s0 instead (Section 3.2). */
static csr coupled_pT(const orc *h, const double *D) {
  int n = h->n, nv = h->nv, nnz = h->rp[n], ns = nv - 2;
  int sl[2] = {h->o.ip, h->o.iT}, ss[4], q = 0;
  for (int k = 0; k < nv; k++)
    if (k != h->o.ip && k != h->o.iT) ss[q++] = k;
  csr a;
  csr_alloc(&a, 2 * n, 2 * n, 4 * nnz);
  int pos = 0;
  for (int u = 0; u < 2; u++)
    for (int i = 0; i < n; i++) {
      for (int w = 0; w < 2; w++)
        for (int k = h->rp[i]; k < h->rp[i + 1]; k++) {
          const double *B = h->v + (size_t)k * nv * nv;
          double x = B[sl[u] * nv + sl[w]];
          if (D)
            for (int b = 0; b < ns; b++) x -= D[((size_t)i * 2 + u) * ns + b] * B[ss[b] * nv + sl[w]];
          a.ci[pos] = w * n + h->ci[k];
          a.v[pos] = x;
          pos++;
        }
      a.rp[u * n + i + 1] = pos;
    }
  return a;
}

void *orc_create(int n, int nv, const int *rp, const int *ci, const double *vals,
                 const int *srp, const int *sci, const double *svals,
                 const orc_opts *o, int *status) {
  orc *h = (orc *)calloc(1, sizeof(orc));
  h->o = *o;
  h->n = n;
  h->nv = nv;
  h->rp = rp;
  h->ci = ci;
  h->v = vals;
  int st = 0;
  size_t N = (size_t)n;
  h->bp = (double *)calloc(2 * N + 1, sizeof(double));  /* [b_p; b_T] for the unknown-based stage */
  h->bt = (double *)calloc(N + 1, sizeof(double));
  h->xp = (double *)calloc(2 * N + 1, sizeof(double));
  h->dt = (double *)calloc(N + 1, sizeof(double));
  h->dp = (double *)calloc(N + 1, sizeof(double));
  h->tmp = (double *)calloc(N + 1, sizeof(double));
  h->x1 = (double *)calloc(N * nv + 1, sizeof(double));
  h->b1 = (double *)calloc(N * nv + 1, sizeof(double));
  h->wb = (double *)calloc(N * nv + 1, sizeof(double));
  h->wx = (double *)calloc(N * nv + 1, sizeof(double));
  if (o->first_stage != ORC_FIRST_NONE) {
    h->App = extract(h, o->ip, o->ip);
    h->ApT = extract(h, o->ip, o->iT);
    h->ATp = extract(h, o->iT, o->ip);
    csr fine = extract(h, o->ip, o->ip);
    if (o->decoupling != 0 && o->first_stage != ORC_FIRST_CPR && o->first_stage != ORC_FIRST_CPTR_UAMG)
      st = -12;
    if (st == 0 && o->decoupling != 0 && o->first_stage == ORC_FIRST_CPTR_UAMG) {
      /* the CPTR extension (Section 3.2): weights of the p and T rows */
      int pri[2] = {o->ip, o->iT};
      if (nv < 3) st = -12;
      h->dcp = (double *)calloc((size_t)n * 2 * (nv - 2) + 1, sizeof(double));
      if (st == 0 && decoupling_weights(h, o->decoupling, pri, 2, h->dcp) != 0) st = -13;
    } else if (st == 0 && o->decoupling != 0) {
      /* S_p = A_pp - D A_sp on the pattern of A_pp */
      int ns = nv - 1, sl[4], q = 0;
      for (int k = 0; k < nv; k++)
        if (k != o->ip) sl[q++] = k;
      h->dcp = (double *)calloc((size_t)n * ns + 1, sizeof(double));
      if (decoupling_weights(h, o->decoupling, &o->ip, 1, h->dcp) != 0) st = -13;
      for (int i = 0; st == 0 && i < n; i++)
        for (int k = rp[i]; k < rp[i + 1]; k++)
          for (int a = 0; a < ns; a++)
            fine.v[k] -= h->dcp[(size_t)i * ns + a] * vals[(size_t)k * nv * nv + sl[a] * nv + o->ip];
    }
    if (st == 0 && o->first_stage == ORC_FIRST_CPTR_UAMG) {
      /* one unknown-based hierarchy on the coupled A_00 (Section 3.4) */
      csr_free(&fine);
      st = uamg_setup(&h->amg_p, coupled_pT(h, h->dcp), n, o->theta, o->max_levels, o->coarse_size,
                      o->seed, o->sweeps, o->smooth_p, o->smooth_p_T < 0 ? o->smooth_p : o->smooth_p_T,
                      o->smoother);
    } else if (st == 0) {
      st = amg_setup(&h->amg_p, fine, o->theta, o->max_levels, o->coarse_size, o->seed,
                     o->sweeps, o->smooth_p, o->smoother);
    } else {
      csr_free(&fine);
    }
    h->have_p = 1;
    if (st == 0 && (o->first_stage == ORC_FIRST_CPTR_BLOCK || o->first_stage == ORC_FIRST_CPTR_LOWER ||
                    o->first_stage == ORC_FIRST_CPTR_UPPER || o->first_stage == ORC_FIRST_CPTR_BD)) {
      /* the second hierarchy: S~_T (eq:Se, or one of the algebraic
       * approximations of Section 3.3.1), or A_TT for the block-diagonal stage */
      csr s;
      if (o->first_stage == ORC_FIRST_CPTR_BD || o->schur == 1)
        s = extract(h, o->iT, o->iT);
      else if (o->schur == 2) {
        if (!schur_diag(h, &s)) st = -14;
      } else
        s = csr_copy(n, srp, sci, svals);
      if (st == 0) {
        st = amg_setup(&h->amg_s, s, o->theta, o->max_levels, o->coarse_size, o->seed,
                       o->sweeps_T > 0 ? o->sweeps_T : o->sweeps,
                       o->smooth_p_T < 0 ? o->smooth_p : o->smooth_p_T, o->smoother);
        h->have_s = 1;
      }
    }
  }
  if (st == 0 && (o->second_stage == ORC_SECOND_BILU0 || o->second_stage == ORC_SECOND_BILU0_MC)) {
    st = bilu_setup(&h->ilu, n, nv, rp, ci, vals, o->second_stage == ORC_SECOND_BILU0_MC,
                    o->ilu_order, o->ilu_part,
                    o->ilu_level);
    if (st != 0) st = -10;
    h->have_ilu = 1;
  }
  if (st == 0 && o->second_stage == ORC_SECOND_EXACT) {
    size_t d = N * nv;
    h->dense_lu = (double *)calloc(d * d + 1, sizeof(double));
    h->dense_piv = (int *)malloc(sizeof(int) * (d + 1));
    for (int i = 0; i < n; i++)
      for (int k = rp[i]; k < rp[i + 1]; k++)
        for (int r = 0; r < nv; r++)
          for (int c = 0; c < nv; c++)
            h->dense_lu[((size_t)i * nv + r) * d + (size_t)ci[k] * nv + c] =
                vals[(size_t)k * nv * nv + r * nv + c];
    if (lu_factor(h->dense_lu, h->dense_piv, (int)d) != 0) st = -11;
  }
  if (status) *status = st;
  return h;
}

void orc_destroy(void *hv) {
  orc *h = (orc *)hv;
  if (!h) return;
  if (h->o.first_stage != ORC_FIRST_NONE) {
    csr_free(&h->App); csr_free(&h->ApT); csr_free(&h->ATp);
  }
  if (h->have_p) amg_free(&h->amg_p);
  if (h->have_s) amg_free(&h->amg_s);
  if (h->have_ilu) bilu_free(&h->ilu);
  free(h->dense_lu); free(h->dense_piv);
  free(h->bp); free(h->bt); free(h->xp); free(h->dt); free(h->dp); free(h->tmp);
  free(h->x1); free(h->b1); free(h->wb); free(h->wx); free(h->dcp);
  free(h);
}

/* First stage M1^{-1} v, returned prolonged to the full (interleaved) vector.
 *  CPTR block (eq:Aschur, its five steps):
 *    x_p = A_pp^{-1} b_p;  b~_T = b_T - A_Tp x_p;  d_T = S~_T^{-1} b~_T;
 *    b~_p = b_p - A_pT d_T;  d_p = A_pp^{-1} b~_p
 *  CPTR lower (left factor of eq:Aschur dropped, the inverse of the block
 *    lower-triangular [A_pp 0; A_Tp S~_T]): d_p = x_p.
 *  CPTR upper (right factor of eq:Aschur dropped, the inverse of the block
 *    upper-triangular [A_pp A_pT; 0 S~_T]): d_T = S~_T^{-1} b_T,
 *    d_p = A_pp^{-1} (b_p - A_pT d_T).
 *  CPR (Section 3.1): d_p = A_pp^{-1} b_p, d_T = 0; with a decoupling
 *    operator G: d_p = S_p^{-1} (G v)_p, S_p = A_pp - D A_sp, (G v)_p = v_p - D v_s.
 *  CPTR-BD(AMG) (Section 4.4, block-diagonal first stage): d_p = A_pp^{-1} b_p,
 *    d_T = A_TT^{-1} b_T, the couplings A_pT, A_Tp left out.
 *  CPTR-uAMG (Section 3.4): (d_p; d_T) = A_00^{-1} (b_p; b_T) by one V-cycle of
 *    the unknown-based hierarchy of the coupled A_00.
 *  Each inverse is one AMG V-cycle. */
int orc_first_stage(void *hv, const double *v, double *x1) {
  orc *h = (orc *)hv;
  int n = h->n, nv = h->nv, ip = h->o.ip, iT = h->o.iT;
  memset(x1, 0, sizeof(double) * (size_t)n * nv);
  if (h->o.first_stage == ORC_FIRST_NONE) return 0;
  for (int i = 0; i < n; i++) {
    h->bp[i] = v[(size_t)i * nv + ip];
    h->bt[i] = v[(size_t)i * nv + iT];
  }
  if (h->o.decoupling != 0 && h->o.first_stage == ORC_FIRST_CPTR_UAMG) {
    /* (b_p; b_T) = (v_p; v_T) - D v_s, s the slots other than p and T */
    int q = 0, ns = nv - 2;
    for (int k = 0; k < nv; k++) {
      if (k == ip || k == iT) continue;
      for (int i = 0; i < n; i++) {
        h->bp[i] -= h->dcp[((size_t)i * 2 + 0) * ns + q] * v[(size_t)i * nv + k];
        h->bt[i] -= h->dcp[((size_t)i * 2 + 1) * ns + q] * v[(size_t)i * nv + k];
      }
      q++;
    }
  } else if (h->o.decoupling != 0) {
    int q = 0;
    for (int k = 0; k < nv; k++) {
      if (k == ip) continue;
      for (int i = 0; i < n; i++) h->bp[i] -= h->dcp[(size_t)i * (nv - 1) + q] * v[(size_t)i * nv + k];
      q++;
    }
  }
  if (h->o.first_stage == ORC_FIRST_CPTR_UAMG) {
    memcpy(h->bp + n, h->bt, sizeof(double) * (size_t)n);
    vcycle(&h->amg_p, 0, h->bp, h->xp);
    for (int i = 0; i < n; i++) {
      x1[(size_t)i * nv + ip] = h->xp[i];
      x1[(size_t)i * nv + iT] = h->xp[n + i];
    }
    return 0;
  }
  if (h->o.first_stage == ORC_FIRST_CPTR_UPPER) {
    vcycle(&h->amg_s, 0, h->bt, h->dt);
    csr_mv(&h->ApT, h->dt, h->tmp);
    for (int i = 0; i < n; i++) h->tmp[i] = h->bp[i] - h->tmp[i];
    vcycle(&h->amg_p, 0, h->tmp, h->dp);
    for (int i = 0; i < n; i++) {
      x1[(size_t)i * nv + ip] = h->dp[i];
      x1[(size_t)i * nv + iT] = h->dt[i];
    }
    return 0;
  }
  vcycle(&h->amg_p, 0, h->bp, h->xp);
  if (h->o.first_stage == ORC_FIRST_CPTR_BD) {
    vcycle(&h->amg_s, 0, h->bt, h->dt);
    for (int i = 0; i < n; i++) {
      x1[(size_t)i * nv + ip] = h->xp[i];
      x1[(size_t)i * nv + iT] = h->dt[i];
    }
    return 0;
  }
  if (h->o.first_stage == ORC_FIRST_CPR) {
    for (int i = 0; i < n; i++) x1[(size_t)i * nv + ip] = h->xp[i];
    return 0;
  }
  csr_mv(&h->ATp, h->xp, h->tmp);
  for (int i = 0; i < n; i++) h->tmp[i] = h->bt[i] - h->tmp[i];
  vcycle(&h->amg_s, 0, h->tmp, h->dt);
  if (h->o.first_stage == ORC_FIRST_CPTR_LOWER) {
    memcpy(h->dp, h->xp, sizeof(double) * (size_t)n);
  } else {
    csr_mv(&h->ApT, h->dt, h->tmp);
    for (int i = 0; i < n; i++) h->tmp[i] = h->bp[i] - h->tmp[i];
    vcycle(&h->amg_p, 0, h->tmp, h->dp);
  }
  for (int i = 0; i < n; i++) {
    x1[(size_t)i * nv + ip] = h->dp[i];
    x1[(size_t)i * nv + iT] = h->dt[i];
  }
  return 0;
}

/* Two-stage preconditioner (Section 3, "Two-stage preconditioners"):
 *   x1 = M1^{-1} v;  b1 = v - A x1;  z = M2^{-1} b1 + x1. */
int orc_apply(void *hv, const double *v, double *z) {
  orc *h = (orc *)hv;
  int n = h->n, nv = h->nv;
  size_t N = (size_t)n * nv;
  orc_first_stage(h, v, h->x1);
  orc_bsr_spmv(n, nv, h->rp, h->ci, h->v, h->x1, h->b1);
  for (size_t i = 0; i < N; i++) h->b1[i] = v[i] - h->b1[i];
  switch (h->o.second_stage) {
    case ORC_SECOND_NONE:
      for (size_t i = 0; i < N; i++) z[i] = 0.0;
      break;
    case ORC_SECOND_IDENTITY:
      memcpy(z, h->b1, sizeof(double) * N);
      break;
    case ORC_SECOND_EXACT:
      memcpy(z, h->b1, sizeof(double) * N);
      lu_solve(h->dense_lu, h->dense_piv, (int)N, z);
      break;
    default:
      bilu_apply(&h->ilu, h->b1, z, h->wb, h->wx);
  }
  for (size_t i = 0; i < N; i++) z[i] += h->x1[i];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* flexible GMRES(m), right preconditioned (Saad 1993; Saad, Iterative       */
/* Methods, Algorithm 9.6), modified Gram-Schmidt Arnoldi, Givens rotations. */
/* x0 = 0.  Stops when |g_{j+1}| <= rtol ||b||, confirmed by the true        */
/* residual ||b - A x|| <= rtol ||b|| at the end of the cycle; otherwise     */
/* restarts from the current x.  Iterations = preconditioner applications. */
/* ------------------------------------------------------------------------ */
static double dot(const double *a, const double *b, size_t n) {
  double s = 0.0;
  for (size_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

int orc_fgmres(void *hv, const double *b, double *x, int m, double rtol, int maxit,
               orc_info *info, double *Vout, double *Zout, double *Hout) {
  orc *h = (orc *)hv;
  int n = h->n, nv = h->nv;
  size_t N = (size_t)n * nv;
  double *V = (double *)malloc(sizeof(double) * N * (size_t)(m + 1));
  double *Z = (double *)malloc(sizeof(double) * N * (size_t)m);
  double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
  double *cs = (double *)malloc(sizeof(double) * (size_t)m);
  double *sn = (double *)malloc(sizeof(double) * (size_t)m);
  double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *y = (double *)malloc(sizeof(double) * (size_t)m);
  double *r = (double *)malloc(sizeof(double) * N);
  double *w = (double *)malloc(sizeof(double) * N);
  memset(x, 0, sizeof(double) * N);
  double bnorm = sqrt(dot(b, b, N));
  int iters = 0, restarts = 0, converged = 0, first_cycle = 1;
  double est = 0.0, truer = 0.0;
  if (bnorm == 0.0) {
    converged = 1;
    goto done;
  }
  for (;;) {
    orc_bsr_spmv(n, nv, h->rp, h->ci, h->v, x, r);
    for (size_t i = 0; i < N; i++) r[i] = b[i] - r[i];
    double beta = sqrt(dot(r, r, N));
    truer = beta / bnorm;
    if (truer <= rtol) { converged = 1; est = truer; break; }
    if (iters >= maxit) break;
    for (size_t i = 0; i < N; i++) V[i] = r[i] / beta;
    for (int i = 0; i <= m; i++) g[i] = 0.0;
    g[0] = beta;
    int j, k = 0;
    for (j = 0; j < m && iters < maxit; j++) {
      orc_apply(h, V + (size_t)j * N, Z + (size_t)j * N);
      iters++;
      orc_bsr_spmv(n, nv, h->rp, h->ci, h->v, Z + (size_t)j * N, w);
      for (int i = 0; i <= j; i++) {
        double hij = dot(w, V + (size_t)i * N, N);
        H[(size_t)i * m + j] = hij;
        for (size_t q = 0; q < N; q++) w[q] -= hij * V[(size_t)i * N + q];
      }
      double hn = sqrt(dot(w, w, N));
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn != 0.0)
        for (size_t q = 0; q < N; q++) V[(size_t)(j + 1) * N + q] = w[q] / hn;
      else
        for (size_t q = 0; q < N; q++) V[(size_t)(j + 1) * N + q] = 0.0;
      if (first_cycle && Hout) {
        /* unrotated Hessenberg column for the Arnoldi relation */
        for (int i = 0; i <= j + 1; i++) Hout[(size_t)i * m + j] = H[(size_t)i * m + j];
      }
      /* apply previous rotations, then a new one */
      for (int i = 0; i < j; i++) {
        double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      double den = sqrt(a * a + c * c);
      cs[j] = den == 0.0 ? 1.0 : a / den;
      sn[j] = den == 0.0 ? 0.0 : c / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      est = fabs(g[j + 1]) / bnorm;
      k = j + 1;
      if (est <= rtol || hn == 0.0) break;
    }
    if (first_cycle) {
      if (Vout) memcpy(Vout, V, sizeof(double) * N * (size_t)(k + 1));
      if (Zout) memcpy(Zout, Z, sizeof(double) * N * (size_t)k);
      first_cycle = 0;
    }
    /* y = R^{-1} g, x += Z y */
    for (int i = k - 1; i >= 0; i--) {
      double s = g[i];
      for (int q = i + 1; q < k; q++) s -= H[(size_t)i * m + q] * y[q];
      y[i] = s / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; i++)
      for (size_t q = 0; q < N; q++) x[q] += y[i] * Z[(size_t)i * N + q];
    restarts++;
  }
  restarts = restarts > 0 ? restarts - 1 : 0;
done:
  if (info) {
    info->iters = iters;
    info->restarts = restarts;
    info->converged = converged;
    info->relres_est = est;
    info->relres_true = truer;
  }
  free(V); free(Z); free(H); free(cs); free(sn); free(g); free(y); free(r); free(w);
  return converged ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* introspection for the tests                                                */
/* ------------------------------------------------------------------------ */
static amg *pick(orc *h, int which) { return which == 0 ? &h->amg_p : &h->amg_s; }

int orc_amg_nlevels(void *hv, int which) {
  orc *h = (orc *)hv;
  if (which == 0 ? !h->have_p : !h->have_s) return 0;
  return pick(h, which)->nlev;
}

int orc_amg_level_info(void *hv, int which, int lev, int *n, int *nnz, int *pnnz) {
  amg *m = pick((orc *)hv, which);
  if (lev < 0 || lev >= m->nlev) return -1;
  *n = m->A[lev].nr;
  *nnz = m->A[lev].nnz;
  *pnnz = lev + 1 < m->nlev ? m->P[lev].nnz : 0;
  return 0;
}

int orc_amg_get_level(void *hv, int which, int lev, int *agg, int *arp, int *aci,
                      double *av, int *prp, int *pci, double *pv, double *omega) {
  amg *m = pick((orc *)hv, which);
  if (lev < 0 || lev >= m->nlev) return -1;
  const csr *a = &m->A[lev];
  memcpy(arp, a->rp, sizeof(int) * ((size_t)a->nr + 1));
  memcpy(aci, a->ci, sizeof(int) * (size_t)a->nnz);
  memcpy(av, a->v, sizeof(double) * (size_t)a->nnz);
  if (lev + 1 < m->nlev) {
    memcpy(agg, m->agg[lev], sizeof(int) * (size_t)a->nr);
    memcpy(prp, m->P[lev].rp, sizeof(int) * ((size_t)a->nr + 1));
    memcpy(pci, m->P[lev].ci, sizeof(int) * (size_t)m->P[lev].nnz);
    memcpy(pv, m->P[lev].v, sizeof(double) * (size_t)m->P[lev].nnz);
    *omega = m->omega[lev];
  }
  return 0;
}

int orc_amg_vcycle(void *hv, int which, const double *b, double *x) {
  orc *h = (orc *)hv;
  if (which == 0 ? !h->have_p : !h->have_s) return -1;
  vcycle(pick(h, which), 0, b, x);
  return 0;
}

int orc_ilu_get(void *hv, int *perm, int *color, int *lev_lower, int *lev_upper,
                double *lu_vals, double *dinv) {
  orc *h = (orc *)hv;
  if (!h->have_ilu) return -1;
  bilu *f = &h->ilu;
  int n = f->n, b2 = f->nv * f->nv;
  for (int r = 0; r < n; r++) {
    if (perm) perm[r] = f->perm ? f->perm[r] : r;
    if (color) color[r] = f->color[r];
    if (lev_lower) lev_lower[r] = f->lev_lower[r];
    if (lev_upper) lev_upper[r] = f->lev_upper[r];
  }
  if (lu_vals) memcpy(lu_vals, f->lu, sizeof(double) * (size_t)f->rp[n] * b2);
  if (dinv) memcpy(dinv, f->dinv, sizeof(double) * (size_t)n * b2);
  return f->ncolor;
}

int orc_ilu_pattern(void *hv, int *rp, int *ci) {
  orc *h = (orc *)hv;
  if (!h->have_ilu) return -1;
  bilu *f = &h->ilu;
  if (rp) memcpy(rp, f->rp, sizeof(int) * ((size_t)f->n + 1));
  if (ci) memcpy(ci, f->ci, sizeof(int) * (size_t)f->rp[f->n]);
  return f->rp[f->n];
}
