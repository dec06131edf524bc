// Numeric re-setup on the GPU: new matrix values on a kept pattern (the next
// Newton iterate, Section 3).  With the aggregates of every AMG level fixed,
// these kernels recompute the smoothed-prolongator values, the Galerkin
// products A P and R (A P), the l1-Jacobi diagonals, the explicit inverse of
// the coarsest operator, the algebraic S~_T of Section 3.3.1 and the learned
// stage's diagonal-block inverses and edge features.
//
// Every entry is formed with the operations and in the order the host setup
// states for it (the summation orders are given at each kernel), and every
// product and sum is rounded on its own (no fused multiply-add), so that the
// values equal those of the host setup bit for bit.  One thread owns each row
// it writes; no result depends on the timing of other threads.
#pragma once

#include "kernels.h"

namespace cptr {

// error bits of a numeric re-setup (one int on the device)
constexpr int kRsNonfinite = 1;   // a non-finite matrix value
constexpr int kRsSingular = 2;    // zero diagonal entry of an AMG operator, singular diagonal block
constexpr int kRsCoarse = 4;      // singular coarsest operator

__device__ __forceinline__ int rs_find(const int *__restrict__ ci, int lo, int hi, int col) {
  // position of `col` in the ascending columns ci[lo .. hi)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ci[mid] < col)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kBlock) k_rs_finite(size_t n, const double *__restrict__ v, int *flag) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < n; i += stride) bad |= !isfinite(v[i]);
  if (bad) atomicOr(flag, kRsNonfinite);
}

// dst[k] = src[k stride + off]: a scalar sub-block (r, c) of BSR values, or a copy
__global__ void __launch_bounds__(kBlock) k_rs_strided(size_t n, const double *__restrict__ src, int stride, int off,
                                                       double *__restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i * stride + off];
}

// Per row of a level operator, in ascending entry order: s = sum |a_ij| and
// the diagonal value d.  The l1-Jacobi inverse 1 / s (rounded to T); with a
// smoothed prolongator also ratio = s / |d| (whose maximum is rho), and a zero
// d is an error; the Gauss-Seidel smoother also needs d != 0.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rs_rowabs(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                      const double *__restrict__ v, double *__restrict__ diag,
                                                      double *__restrict__ ratio, T *__restrict__ dinv,
                                                      int need_diag, int *flag) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, d = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) {
    s += fabs(v[k]);
    if (ci[k] == i) d = v[k];
  }
  dinv[i] = T(1.0 / s);
  diag[i] = d;
  if (ratio) ratio[i] = s / fabs(d);
  if (need_diag && d == 0.0) atomicOr(flag, kRsSingular);
}

// block maxima of x[0 .. n) (non-negative), then rho = their maximum and
// omega = 4 / (3 rho) in one block
__global__ void __launch_bounds__(kBlock) k_rs_max_partial(int n, const double *__restrict__ x,
                                                           double *__restrict__ part) {
  __shared__ double sm[kBlock];
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) m = fmax(m, x[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void __launch_bounds__(kBlock) k_rs_omega(int nb, const double *__restrict__ part, double *omega) {
#pragma clang fp contract(off)
  __shared__ double sm[kBlock];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *omega = 4.0 / (3.0 * sm[0]);
}

// Smoothed prolongator on a kept pattern: P(i, J) = [agg(i) = J] - (omega /
// a_ii) s_iJ, s_iJ the sum of a_ij over the entries of row i with agg(j) = J
// in ascending entry order from 0; pslot[k] is the P entry of A entry k (-1
// for a column outside every aggregate).
__global__ void __launch_bounds__(kBlock) k_rs_prolong(int n, const int *__restrict__ a_rp,
                                                       const double *__restrict__ a_v, const int *__restrict__ pslot,
                                                       const int *__restrict__ agg, const double *__restrict__ diag,
                                                       const double *__restrict__ omega, const int *__restrict__ p_rp,
                                                       const int *__restrict__ p_ci, double *__restrict__ p_v) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = p_rp[i]; q < p_rp[i + 1]; q++) p_v[q] = 0.0;
  for (int k = a_rp[i]; k < a_rp[i + 1]; k++) {
    const int s = pslot[k];
    if (s >= 0) p_v[s] += a_v[k];
  }
  const double w = *omega / diag[i];
  const int own = agg[i];
  for (int q = p_rp[i]; q < p_rp[i + 1]; q++) {
    const double d = p_ci[q] == own ? 1.0 : 0.0;
    p_v[q] = d - w * p_v[q];
  }
}

// dst[q] = src[idx[q]] (the restriction's values from the prolongator's)
__global__ void __launch_bounds__(kBlock) k_rs_gather(size_t n, const int *__restrict__ idx,
                                                      const double *__restrict__ src, double *__restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// C = A B on C's kept pattern: entry (i, j) accumulated from 0 over the
// entries k of row i of A in ascending order (each row of B holds column j at
// most once), one product and one sum per step.
__global__ void __launch_bounds__(kBlock) k_rs_spgemm(int nr, const int *__restrict__ a_rp, const int *__restrict__ a_ci,
                                                      const double *__restrict__ a_v, const int *__restrict__ b_rp,
                                                      const int *__restrict__ b_ci, const double *__restrict__ b_v,
                                                      const int *__restrict__ c_rp, const int *__restrict__ c_ci,
                                                      double *__restrict__ c_v) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const int c0 = c_rp[i], c1 = c_rp[i + 1];
  for (int q = c0; q < c1; q++) c_v[q] = 0.0;
  for (int k = a_rp[i]; k < a_rp[i + 1]; k++) {
    const double av = a_v[k];
    const int m = a_ci[k];
    for (int q = b_rp[m]; q < b_rp[m + 1]; q++) {
      const int pos = rs_find(c_ci, c0, c1, b_ci[q]);
      if (pos < c1) c_v[pos] = c_v[pos] + av * b_v[q];  // always found on a consistent pattern
    }
  }
}

// The same product with one wavefront per row of C, for rows of many
// products: the entries k of row i of A are still taken in ascending order
// (a barrier between them), and the products of one k go to distinct columns
// of C (a row of B holds each column once), so the lanes take them in
// parallel without changing any entry's order of summation.  The row of C
// (columns and sums) sits in LDS when it holds at most kSpgLds entries.
constexpr int kSpgLds = 4096;

__global__ void __launch_bounds__(64) k_rs_spgemm_wave(const int *__restrict__ a_rp, const int *__restrict__ a_ci,
                                                       const double *__restrict__ a_v, const int *__restrict__ b_rp,
                                                       const int *__restrict__ b_ci, const double *__restrict__ b_v,
                                                       const int *__restrict__ c_rp, const int *__restrict__ c_ci,
                                                       double *__restrict__ c_v) {
#pragma clang fp contract(off)
  __shared__ double acc[kSpgLds];
  __shared__ int col[kSpgLds];
  const int i = blockIdx.x, lane = threadIdx.x;
  const int c0 = c_rp[i], len = c_rp[i + 1] - c0;
  const bool in_lds = len <= kSpgLds;
  const int *cc = in_lds ? col : c_ci + c0;
  double *out = in_lds ? acc : c_v + c0;
  for (int q = lane; q < len; q += 64) {
    out[q] = 0.0;
    if (in_lds) col[q] = c_ci[c0 + q];
  }
  __syncthreads();
  for (int k = a_rp[i]; k < a_rp[i + 1]; k++) {
    const double av = a_v[k];
    const int m = a_ci[k];
    for (int q = b_rp[m] + lane; q < b_rp[m + 1]; q += 64) {
      const int pos = rs_find(cc, 0, len, b_ci[q]);
      if (pos < len) out[pos] = out[pos] + av * b_v[q];
    }
    __syncthreads();
  }
  if (in_lds)
    for (int q = lane; q < len; q += 64) c_v[c0 + q] = acc[q];
}

// value refresh of the device formats of a scalar operator from CSR values
// src[k stride + off] (k the CSR entry)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rs_csr_vals(size_t nnz, const double *__restrict__ src, int stride, int off,
                                                        T *__restrict__ val) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) val[k] = T(src[k * stride + off]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_rs_sell_vals(int nr, const int *__restrict__ rp, const double *__restrict__ src,
                                                         int stride, int off, const int *__restrict__ sptr,
                                                         T *__restrict__ val) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  const int base = sptr[r / kSlice] + r % kSlice;
  for (int k = rp[r]; k < rp[r + 1]; k++) val[base + (k - rp[r]) * kSlice] = T(src[(size_t)k * stride + off]);
}

// diagonal storage: the host forms each stored value as 0 + a_ij in FP64
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rs_dia_vals(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const double *__restrict__ src, int stride, int off, Dia<T> d,
                                                        T *__restrict__ val) {
#pragma clang fp contract(off)
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  for (int k = rp[r]; k < rp[r + 1]; k++) {
    const int o = ci[k] - r;
    int g = 0;
    while (g + 1 < d.ndiag && d.off[g] != o) g++;
    const double a = 0.0 + src[(size_t)k * stride + off];
    val[(size_t)g * nr + r] = T(a);
  }
}

// Gauss-Jordan inverse of the coarsest operator with partial pivoting, on the
// n x 2n array [A | I]: per column c, the pivot row p is the first row r >= c
// of largest |m(r, c)|; rows p and c are swapped, row c is divided by the
// pivot, and every other row r with f = m(r, c) != 0 takes m(r, q) - f m(c, q)
// for all q.
__global__ void __launch_bounds__(kBlock) k_rs_gj_init(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const double *__restrict__ v, double *__restrict__ m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double *row = m + (size_t)i * 2 * n;
  for (int q = 0; q < 2 * n; q++) row[q] = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) row[ci[k]] = v[k];
  row[n + i] = 1.0;
}

constexpr int kGjBlock = 1024;

__global__ void __launch_bounds__(kGjBlock) k_rs_gj_pivot(int n, int c, double *__restrict__ m,
                                                          double *__restrict__ f, int *flag) {
#pragma clang fp contract(off)
  __shared__ double bv[kGjBlock];
  __shared__ int bi[kGjBlock];
  const int t = threadIdx.x;
  const size_t w = 2 * (size_t)n;
  double best = -1.0;
  int bidx = n;
  for (int r = c + t; r < n; r += kGjBlock) {
    const double a = fabs(m[r * w + c]);
    if (a > best) {
      best = a;
      bidx = r;
    }
  }
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int s = kGjBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double o = bv[t + s];
      const int oi = bi[t + s];
      if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
        bv[t] = o;
        bi[t] = oi;
      }
    }
    __syncthreads();
  }
  const int p = bi[0];
  const double piv = m[p * w + c];
  if (piv == 0.0) {
    if (t == 0) atomicOr(flag, kRsCoarse);
    return;  // the whole block returns: piv is the same value in every thread
  }
  if (p != c)
    for (size_t q = t; q < w; q += kGjBlock) {
      const double x = m[p * w + q];
      m[p * w + q] = m[c * w + q];
      m[c * w + q] = x;
    }
  __syncthreads();
  for (size_t q = t; q < w; q += kGjBlock) m[c * w + q] = m[c * w + q] / piv;
  __syncthreads();
  for (int r = t; r < n; r += kGjBlock) f[r] = r == c ? 0.0 : m[r * w + c];
}

__global__ void __launch_bounds__(kBlock) k_rs_gj_elim(int n, int c, double *__restrict__ m,
                                                       const double *__restrict__ f) {
#pragma clang fp contract(off)
  const size_t w = 2 * (size_t)n;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * w) return;
  const int r = int(e / w);
  const double fr = f[r];
  if (r == c || fr == 0.0) return;
  const size_t q = e - (size_t)r * w;
  m[e] = m[e] - fr * m[c * w + q];
}

__global__ void __launch_bounds__(kBlock) k_rs_gj_out(int n, const double *__restrict__ m, double *__restrict__ inv) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = int(e / n), j = int(e - (size_t)i * n);
  inv[e] = m[(size_t)i * 2 * n + n + j];
}

// Algebraic S~_T = A_TT - A_Tp diag(A_pp)^-1 A_pT on its kept pattern (the
// cells within two steps): entry (i, l) starts from A_TT(i, l) (0 outside the
// pattern of A), then for the entries (i, j) of row i and (j, l) of row j,
// both ascending, takes away (A_Tp(i, j) / A_pp(j, j)) A_pT(j, l).
__global__ void __launch_bounds__(kBlock) k_rs_app(int n, int nv, int ip, const int *__restrict__ rp,
                                                   const int *__restrict__ ci, const double *__restrict__ vals,
                                                   double *__restrict__ app, int *flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++)
    if (ci[k] == i) d = vals[((size_t)k * nv + ip) * nv + ip];
  app[i] = d;
  if (d == 0.0) atomicOr(flag, kRsSingular);
}

__global__ void __launch_bounds__(kBlock) k_rs_schur(int n, int nv, int ip, int iT, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const double *__restrict__ vals,
                                                     const double *__restrict__ app, const int *__restrict__ s_rp,
                                                     const int *__restrict__ s_ci, double *__restrict__ s_v) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto blk = [&](int k, int r, int c) { return vals[((size_t)k * nv + r) * nv + c]; };
  const int c0 = s_rp[i], c1 = s_rp[i + 1];
  for (int q = c0; q < c1; q++) s_v[q] = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) {
    const int pos = rs_find(s_ci, c0, c1, ci[k]);
    if (pos < c1) s_v[pos] = blk(k, iT, iT);
  }
  for (int k = rp[i]; k < rp[i + 1]; k++) {
    const int j = ci[k];
    const double a = blk(k, iT, ip) / app[j];
    for (int q = rp[j]; q < rp[j + 1]; q++) {
      const int pos = rs_find(s_ci, c0, c1, ci[q]);
      if (pos < c1) s_v[pos] = s_v[pos] - a * blk(q, ip, iT);
    }
  }
}

// The sliced FP64 copy of A (slices of 64 rows, each padded to its longest
// row; entry k of row i at ((kptr[slice] + k) nv^2 + e) 64 + lane)
__global__ void __launch_bounds__(kBlock) k_rs_sliced(int n, int b2, const int *__restrict__ rp,
                                                      const int *__restrict__ kptr, const double *__restrict__ vals,
                                                      double *__restrict__ sv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int lane = i % 64;
  const size_t k0 = (size_t)kptr[i / 64];
  for (int k = 0; k < rp[i + 1] - rp[i]; k++)
    for (int e = 0; e < b2; e++) sv[((k0 + k) * b2 + e) * 64 + lane] = vals[(size_t)(rp[i] + k) * b2 + e];
}

// FP32 copies of the p and T columns of A in the same slicing (the two-stage
// residual with FP32 values)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rs_pt_cols(int n, int nv, int ip, int iT, const int *__restrict__ rp,
                                                       const int *__restrict__ kptr, const double *__restrict__ vals,
                                                       T *__restrict__ acol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int lane = i % 64;
  const size_t k0 = (size_t)kptr[i / 64];
  for (int k = 0; k < rp[i + 1] - rp[i]; k++) {
    const size_t kk = k0 + k, blk = (size_t)rp[i] + k;
    for (int r = 0; r < nv; r++) {
      acol[((kk * nv + r) * 2 + 0) * 64 + lane] = T(vals[(blk * nv + r) * nv + ip]);
      acol[((kk * nv + r) * 2 + 1) * 64 + lane] = T(vals[(blk * nv + r) * nv + iT]);
    }
  }
}

// BF16 of an FP32 value, rounding to nearest even on the bit pattern (finite inputs)
__device__ __forceinline__ short rs_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// The learned stage's matrix data of one cell: D_i^-1 by Gauss-Jordan with
// partial pivoting on [D_i | I] (first row of largest |pivot|, row divided by
// the pivot, every other row r takes m(r, q) - f m(c, q)), kept in FP32, and
// the edge features E_{i,d} = D_i^-1 A_{i, nbr(i, d)} with each entry summed
// over q ascending from 0, rounded to FP32 and then BF16, stored per
// direction (E) and in the tiled order of the inference layers (Et, runs of
// `run` entries per tile and direction).
template <int NV>
__global__ void __launch_bounds__(kBlock) k_rs_learned(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const double *__restrict__ vals, const int *__restrict__ nbr,
                                                       float *__restrict__ dinv, short *__restrict__ E,
                                                       short *__restrict__ Et, int run, int *flag) {
#pragma clang fp contract(off)
  constexpr int B2 = NV * NV;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int dk = -1;
  for (int k = rp[i]; k < rp[i + 1]; k++)
    if (ci[k] == i) dk = k;
  if (dk < 0) {
    atomicOr(flag, kRsSingular);
    return;
  }
  double m[NV][2 * NV];
#pragma unroll
  for (int r = 0; r < NV; r++)
#pragma unroll
    for (int q = 0; q < 2 * NV; q++) m[r][q] = q < NV ? vals[(size_t)dk * B2 + r * NV + q] : (q - NV == r ? 1.0 : 0.0);
#pragma unroll
  for (int c = 0; c < NV; c++) {
    int p = c;
#pragma unroll
    for (int r = c + 1; r < NV; r++)
      if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
    double pv = 0.0;
#pragma unroll
    for (int r = 0; r < NV; r++)
      if (r == p) pv = m[r][c];
    if (pv == 0.0) {
      atomicOr(flag, kRsSingular);
      return;
    }
    if (p != c) {
#pragma unroll
      for (int r = c + 1; r < NV; r++)
        if (r == p)
#pragma unroll
          for (int q = 0; q < 2 * NV; q++) {
            const double x = m[c][q];
            m[c][q] = m[r][q];
            m[r][q] = x;
          }
    }
    const double d = m[c][c];
#pragma unroll
    for (int q = 0; q < 2 * NV; q++) m[c][q] = m[c][q] / d;
#pragma unroll
    for (int r = 0; r < NV; r++) {
      if (r == c) continue;
      const double f = m[r][c];
#pragma unroll
      for (int q = 0; q < 2 * NV; q++) m[r][q] = m[r][q] - f * m[c][q];
    }
  }
#pragma unroll
  for (int r = 0; r < NV; r++)
#pragma unroll
    for (int c = 0; c < NV; c++) dinv[(size_t)i * B2 + r * NV + c] = float(m[r][NV + c]);
  for (int d = 0; d < 6; d++) {
    const int j = nbr[(size_t)i * 6 + d];
    if (j < 0) continue;
    const int k = rs_find(ci, rp[i], rp[i + 1], j);
    if (k >= rp[i + 1]) continue;  // always found: the neighbour table comes from this pattern
    short *r0 = Et + ((size_t)(i / 16) * 6 + d) * run;
#pragma unroll
    for (int r = 0; r < NV; r++)
#pragma unroll
      for (int c = 0; c < NV; c++) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NV; q++) acc = acc + m[r][NV + q] * vals[(size_t)k * B2 + q * NV + c];
        const short b = rs_bf16(float(acc));
        const int e = r * NV + c;
        E[((size_t)i * 6 + d) * 16 + e] = b;
        r0[(e / 4) * 64 + (i % 16) * 4 + e % 4] = b;
      }
  }
}

}  // namespace cptr
