// Device kernels of libcptr (gfx950).  Included once by cptr.hip.
#pragma once

#include "kernels.h"

namespace cptr {

constexpr int kBlock = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// One-thread-per-row products over SELL-64 or DIA storage.  row_sum(A, row, f)
// returns sum_j a_{row,j} f(j) in ascending column order, f(j) being the
// column's operand (x_j, or a value formed on the fly from several vectors).
// ---------------------------------------------------------------------------
// Slots 0 .. w-1 of the slice, kSellUnroll at a time: a round's index and
// value loads are all issued before its operands are gathered (slot clamped
// to the slice width, so no load depends on a branch); slots past the width
// add exactly nothing, padding slots (column 0, value 0) add 0 * x_0.
constexpr int kSellUnroll = 4;

template <typename T, typename F>
__device__ __forceinline__ T row_sum(const Sell<T> &A, int row, F f) {
  const int s = row >> 6, lane = row & 63;
  const int b = A.sptr[s], w = (A.sptr[s + 1] - b) >> 6;
  const int *__restrict__ c = A.col + b + lane;
  const T *__restrict__ v = A.val + b + lane;
  T acc = T(0);
  for (int k0 = 0; k0 < w; k0 += kSellUnroll) {
    int cc[kSellUnroll];
    T vv[kSellUnroll];
#pragma unroll
    for (int u = 0; u < kSellUnroll; u++) {
      const int k = min(k0 + u, w - 1);
      cc[u] = c[k * kSlice];
      vv[u] = v[k * kSlice];
    }
#pragma unroll
    for (int u = 0; u < kSellUnroll; u++) {
      const T xc = f(cc[u]);
      acc += vv[u] * (k0 + u < w ? xc : T(0));
    }
  }
  return acc;
}

// Slots off the pattern hold zero; their column is clamped into range so the
// operand load stays in bounds, and the operand is replaced by zero so that
// they add exactly nothing.  Diagonals past ndiag repeat the last one (its
// offset is padded on the host) and are masked the same way: the loop has no
// branch, so all loads of the row are in flight together.
template <typename T, typename F>
__device__ __forceinline__ T row_sum(const Dia<T> &A, int row, F f) {
  T v[kMaxDiag], xc[kMaxDiag];
#pragma unroll
  for (int d = 0; d < kMaxDiag; d++) {
    v[d] = A.val[(size_t)min(d, A.ndiag - 1) * A.nrows + row];
    xc[d] = f(min(max(row + A.off[d], 0), A.nrows - 1));
  }
  T acc = T(0);
#pragma unroll
  for (int d = 0; d < kMaxDiag; d++) acc += v[d] * (d < A.ndiag && v[d] != T(0) ? xc[d] : T(0));
  return acc;
}

// y = A x  (mode 0),  y += A x  (mode 1),  y = b - A x  (mode 2)
template <typename Op, int MODE, typename T = typename Op::value_type>
__global__ void __launch_bounds__(kBlock) k_spmv(Op A, const T *__restrict__ x, const T *__restrict__ b,
                                                 T *__restrict__ y) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row >= A.nrows) return;
  const T ax = row_sum(A, row, [&](int c) { return x[c]; });
  if (MODE == 0) y[row] = ax;
  if (MODE == 1) y[row] += ax;
  if (MODE == 2) y[row] = b[row] - ax;
}

// first l1-Jacobi sweep from a zero guess fused with the residual:
//   x = D^{-1} b,  r = b - A D^{-1} b
template <typename Op, typename T = typename Op::value_type>
__global__ void __launch_bounds__(kBlock) k_smooth0_resid(Op A, const T *__restrict__ dinv,
                                                          const T *__restrict__ b, T *__restrict__ x,
                                                          T *__restrict__ r) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row >= A.nrows) return;
  const T acc = row_sum(A, row, [&](int c) { return dinv[c] * b[c]; });
  const T bi = b[row];
  x[row] = dinv[row] * bi;
  r[row] = bi - acc;
}

// the first two l1-Jacobi sweeps from a zero guess in one pass over A:
//   x1 = D^{-1} b,  r1 = b - A x1,  x = x1 + D^{-1} r1
// (the same roundings as a sweep that stores x1 and r1 and one that reads them)
template <typename Op, typename T = typename Op::value_type>
__global__ void __launch_bounds__(kBlock) k_smooth0_next(Op A, const T *__restrict__ dinv,
                                                         const T *__restrict__ b, T *__restrict__ x) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row >= A.nrows) return;
  const T acc = row_sum(A, row, [&](int c) { return dinv[c] * b[c]; });
  const T bi = b[row], di = dinv[row];
  const T x1 = di * bi, r1 = bi - acc;
  x[row] = x1 + di * r1;
}

// x_out = x_in + D^{-1} (b - A x_in)
template <typename Op, typename T = typename Op::value_type>
__global__ void __launch_bounds__(kBlock) k_jacobi(Op A, const T *__restrict__ dinv, const T *__restrict__ b,
                                                   const T *__restrict__ xin, T *__restrict__ xout) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row >= A.nrows) return;
  const T ax = row_sum(A, row, [&](int c) { return xin[c]; });
  xout[row] = xin[row] + dinv[row] * (b[row] - ax);
}

// ---------------------------------------------------------------------------
// CSR products with G lanes per row, for operators with long rows (coarse
// AMG levels, restriction): lanes stride the row, then an xor-shuffle sum.
// ---------------------------------------------------------------------------
// Each lane takes entries lane, lane + G, ... of the row, kCsrvUnroll at a
// time: the index and value loads of a round are all issued before its
// operands are gathered (column clamped into the row, so no load depends on
// a branch), and slots past the row end add exactly nothing.
constexpr int kCsrvUnroll = 4;

template <typename T, int G, typename F>
__device__ __forceinline__ T csrv_row_sum(const int *__restrict__ rp, const int *__restrict__ ci,
                                          const T *__restrict__ val, int row, int lane, F f) {
  const int e = rp[row + 1];
  T acc = T(0);
  for (int k0 = rp[row] + lane; k0 < e; k0 += kCsrvUnroll * G) {
    int c[kCsrvUnroll];
    T v[kCsrvUnroll];
#pragma unroll
    for (int u = 0; u < kCsrvUnroll; u++) {
      const int k = min(k0 + u * G, e - 1);
      c[u] = ci[k];
      v[u] = val[k];
    }
#pragma unroll
    for (int u = 0; u < kCsrvUnroll; u++) {
      const T xc = f(c[u]);
      acc += v[u] * (k0 + u * G < e ? xc : T(0));
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k_csrv_spmv(int n, const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const T *__restrict__ val,
                                                      const T *__restrict__ x,
                                                      const T *__restrict__ b, T *__restrict__ y) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int row = t / G, lane = t % G;
  if (row >= n) return;  // whole G-lane groups exit together (G divides kBlock)
  const T ax = csrv_row_sum<T, G>(rp, ci, val, row, lane, [&](int c) { return x[c]; });
  if (lane != 0) return;
  if (MODE == 0) y[row] = ax;
  if (MODE == 1) y[row] += ax;
  if (MODE == 2) y[row] = b[row] - ax;
}

template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_csrv_jacobi(int n, const int *__restrict__ rp,
                                                        const int *__restrict__ ci,
                                                        const T *__restrict__ val,
                                                        const T *__restrict__ dinv,
                                                        const T *__restrict__ b,
                                                        const T *__restrict__ xin,
                                                        T *__restrict__ xout) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int row = t / G, lane = t % G;
  if (row >= n) return;
  const T bi = b[row], di = dinv[row], xi = xin[row];  // issued before the row's loads
  const T ax = csrv_row_sum<T, G>(rp, ci, val, row, lane, [&](int c) { return xin[c]; });
  if (lane == 0) xout[row] = xi + di * (bi - ax);
}

// x = D^{-1} b, r = b - A D^{-1} b with G lanes per row
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_csrv_smooth0_resid(int n, const int *__restrict__ rp,
                                                               const int *__restrict__ ci,
                                                               const T *__restrict__ val,
                                                               const T *__restrict__ dinv,
                                                               const T *__restrict__ b,
                                                               T *__restrict__ x,
                                                               T *__restrict__ r) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int row = t / G, lane = t % G;
  if (row >= n) return;
  const T bi = b[row], di = dinv[row];
  const T acc = csrv_row_sum<T, G>(rp, ci, val, row, lane, [&](int c) { return dinv[c] * b[c]; });
  if (lane != 0) return;
  x[row] = di * bi;
  r[row] = bi - acc;
}

// the first two sweeps from a zero guess (k_smooth0_next) with G lanes per row
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_csrv_smooth0_next(int n, const int *__restrict__ rp,
                                                              const int *__restrict__ ci,
                                                              const T *__restrict__ val,
                                                              const T *__restrict__ dinv,
                                                              const T *__restrict__ b, T *__restrict__ x) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int row = t / G, lane = t % G;
  if (row >= n) return;
  const T bi = b[row], di = dinv[row];
  const T acc = csrv_row_sum<T, G>(rp, ci, val, row, lane, [&](int c) { return dinv[c] * b[c]; });
  if (lane != 0) return;
  const T x1 = di * bi, r1 = bi - acc;
  x[row] = x1 + di * r1;
}

// coarsest level: x = A_c^{-1} b with the explicit FP64 inverse; one wave per row
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_gemv(const double *__restrict__ inv, int nc,
                                                        const T *__restrict__ b, T *__restrict__ x) {
  const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= nc) return;
  const double *__restrict__ row = inv + (size_t)wave * nc;
  double acc = 0.0;
  for (int c = lane; c < nc; c += 64) acc += row[c] * double(b[c]);
  acc = wave_sum(acc);
  if (lane == 0) x[wave] = T(acc);
}

// ---------------------------------------------------------------------------
// first stage: restriction, two-stage residual, finishing
// ---------------------------------------------------------------------------
// b_p = v_p, b_T = v_T; with decoupling weights (G v restricted, Section 3.1):
// d_rows = 1, D [n][nv-1]: b_p = v_p - D_i v_s over every slot but p, in order;
// d_rows = 2, D [n][2][nv-2]: (b_p; b_T) = (v_p; v_T) - D_i v_s over every slot
// but p and T (the pressure-temperature extension of Section 3.2)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_pT(int n, int nv, int ip, int iT,
                                                        const ApplySlots *__restrict__ slots,
                                                        const T *__restrict__ D, int d_rows,
                                                        T *__restrict__ bp, T *__restrict__ bt) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const gmem<const double> *__restrict__ v = as_global(slots->v);
  T p = T(v[(size_t)i * nv + ip]);
  T t = T(v[(size_t)i * nv + iT]);
  if (D && d_rows == 1) {  // pressure row over every other slot: D [n][nv-1]
    int q = 0;
    for (int k = 0; k < nv; k++) {
      if (k == ip) continue;
      p -= D[(size_t)i * (nv - 1) + q] * T(v[(size_t)i * nv + k]);
      q++;
    }
  } else if (D) {  // pressure and temperature rows over the remaining slots: D [n][2][nv-2]
    const int ns = nv - 2;
    int q = 0;
    for (int k = 0; k < nv; k++) {
      if (k == ip || k == iT) continue;
      const T vk = T(v[(size_t)i * nv + k]);
      p -= D[((size_t)i * 2 + 0) * ns + q] * vk;
      t -= D[((size_t)i * 2 + 1) * ns + q] * vk;
      q++;
    }
  }
  bp[i] = p;
  if (bt) bt[i] = t;
}

// b1 = v - A R^T (d_p, d_T): only the p and T columns of each block are used.
// On the sliced layout of the FP64 product (slices of 64 block rows;
// for block column k of slice s the entries (r, j) of its 64 rows are stored
// contiguously: acol[((kptr[s] + k) NV + r) 2 + j) 64 + lane], padding blocks
// zero).  Wavefront r forms equation r of the slice's rows.
template <int NV, typename T>
__global__ void __launch_bounds__(64 * NV) k_resid_pT_sliced(int n, const int *__restrict__ kptr,
                                                              const int *__restrict__ cols,
                                                              const T *__restrict__ acol,
                                                              const ApplySlots *__restrict__ slots,
                                                              const T *__restrict__ dp,
                                                              const T *__restrict__ dT,
                                                              T *__restrict__ b1) {
  const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sl = blockIdx.x, i = sl * 64 + lane;
  const int k0 = kptr[sl], k1 = kptr[sl + 1];
  T acc = T(0);
  if (dT) {
#pragma unroll 4
    for (int k = k0; k < k1; k++) {
      const int c = cols[(size_t)k * 64 + lane];
      const T *a = acol + ((size_t)k * NV + r) * 2 * 64 + lane;
      acc += a[0] * dp[c] + a[64] * dT[c];
    }
  } else {
#pragma unroll 4
    for (int k = k0; k < k1; k++)
      acc += acol[((size_t)k * NV + r) * 2 * 64 + lane] * dp[cols[(size_t)k * 64 + lane]];
  }
  if (i >= n) return;
  b1[(size_t)i * NV + r] = T(as_global(slots->v)[(size_t)i * NV + r]) - acc;
}

// The same from the FP64 values of the sliced copy of A (columns ip and iT of
// each block are contiguous runs of 64), accumulated in FP64, b1 rounded to T.
template <int NV, typename T>
__global__ void __launch_bounds__(64 * NV) k_resid_pT_sliced64(int n, const int *__restrict__ kptr,
                                                                const int *__restrict__ cols,
                                                                const double *__restrict__ vals, int ip, int iT,
                                                                const ApplySlots *__restrict__ slots,
                                                                const T *__restrict__ dp,
                                                                const T *__restrict__ dT,
                                                                T *__restrict__ b1) {
  const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sl = blockIdx.x, i = sl * 64 + lane;
  const int k0 = kptr[sl], k1 = kptr[sl + 1];
  double acc = 0.0;
  if (dT) {
#pragma unroll 4
    for (int k = k0; k < k1; k++) {
      const int c = cols[(size_t)k * 64 + lane];
      const double *a = vals + ((size_t)k * NV * NV + r * NV) * 64 + lane;
      acc += a[ip * 64] * double(dp[c]) + a[iT * 64] * double(dT[c]);
    }
  } else {
#pragma unroll 4
    for (int k = k0; k < k1; k++) {
      const int c = cols[(size_t)k * 64 + lane];
      acc += vals[((size_t)k * NV * NV + r * NV + ip) * 64 + lane] * double(dp[c]);
    }
  }
  if (i >= n) return;
  b1[(size_t)i * NV + r] = T(as_global(slots->v)[(size_t)i * NV + r] - acc);
}

template <typename T, typename ZT>
__global__ void __launch_bounds__(kBlock) k_finish(int n, int nv, int ip, int iT,
                                                   const T *__restrict__ b1,
                                                   const T *__restrict__ dp,
                                                   const T *__restrict__ dT,
                                                   const ApplySlots *__restrict__ slots) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * nv) return;
  const int i = t / nv, r = t - i * nv;
  T z = b1 ? b1[t] : T(0);
  if (dp && r == ip) z += dp[i];
  if (dT && r == iT) z += dT[i];
  as_global(reinterpret_cast<ZT *>(slots->z))[t] = ZT(z);
}

// ---------------------------------------------------------------------------
// BILU(0) triangular solves, one launch per level; NV threads per row
// ---------------------------------------------------------------------------
// The sums of a row are accumulated in A: T, or FP64 for FP32 factors and
// vectors (storage in T either way; the factors and y are rounded to T).
// forward: y_i = b_i - sum_k L_ik y_k   (in place in y, which holds b1)
template <int NV, typename T, typename A = T>
__global__ void __launch_bounds__(kBlock) k_ilu_fwd(int p0, int cnt, const int *__restrict__ rows,
                                                    const int *__restrict__ ptr,
                                                    const int *__restrict__ col,
                                                    const T *__restrict__ val, T *__restrict__ y) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int q = t / NV, r = t - q * NV;
  if (q >= cnt) return;
  const int p = p0 + q;
  const int i = rows[p];
  A s = A(y[(size_t)i * NV + r]);
  for (int k = ptr[p]; k < ptr[p + 1]; k++) {
    const T *l = val + ((size_t)k * NV + r) * NV;
    const T *yk = y + (size_t)col[k] * NV;
#pragma unroll
    for (int c = 0; c < NV; c++) s -= A(l[c]) * A(yk[c]);
  }
  y[(size_t)i * NV + r] = T(s);
}

// backward: w_i = U_ii^{-1} (y_i - sum_k U_ik w_k), in place in y; also
// writes z_i = w_i + x1_i.
template <int NV, typename T, typename ZT, typename A = T>
__global__ void __launch_bounds__(kBlock) k_ilu_bwd(int p0, int cnt, const int *__restrict__ rows,
                                                    const int *__restrict__ ptr,
                                                    const int *__restrict__ col,
                                                    const T *__restrict__ val,
                                                    const T *__restrict__ dinv, T *__restrict__ y,
                                                    int ip, int iT, const T *__restrict__ dp,
                                                    const T *__restrict__ dT,
                                                    const ApplySlots *__restrict__ slots) {
  // rows never straddle workgroups: kBlock / NV rows per workgroup
  __shared__ A sh[kBlock];
  constexpr int kRows = kBlock / NV;
  const int r = threadIdx.x % NV;
  const int q = blockIdx.x * kRows + threadIdx.x / NV;
  const bool live = q < cnt && threadIdx.x < kRows * NV;
  int i = 0;
  A s = A(0);
  if (live) {
    const int p = p0 + q;
    i = rows[p];
    s = A(y[(size_t)i * NV + r]);
    for (int k = ptr[p]; k < ptr[p + 1]; k++) {
      const T *u = val + ((size_t)k * NV + r) * NV;
      const T *wk = y + (size_t)col[k] * NV;
#pragma unroll
      for (int c = 0; c < NV; c++) s -= A(u[c]) * A(wk[c]);
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  if (!live) return;
  const T *d = dinv + ((size_t)i * NV + r) * NV;
  const int base = threadIdx.x - r;
  A w = A(0);
#pragma unroll
  for (int c = 0; c < NV; c++) w += A(d[c]) * sh[base + c];
  y[(size_t)i * NV + r] = T(w);
  A z = w;
  if (dp && r == ip) z += A(dp[i]);
  if (dT && r == iT) z += A(dT[i]);
  as_global(reinterpret_cast<ZT *>(slots->z))[(size_t)i * NV + r] = ZT(z);
}

// ---------------------------------------------------------------------------
// multicolour Gauss-Seidel smoothing: the rows of one colour (not coupled to
// each other) take x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii with the current
// x of the other colours; one launch per colour
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_color(int cnt, const int *__restrict__ rows,
                                                     const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const T *__restrict__ v, const T *__restrict__ b, T *x) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= cnt) return;
  const int i = rows[t];
  T s = b[i], d = T(1);  // the diagonal entry is present and nonzero on every row (checked at setup)
  for (int k = rp[i]; k < rp[i + 1]; k++) {
    const int j = ci[k];
    if (j == i)
      d = v[k];
    else
      s -= v[k] * x[j];
  }
  x[i] = s / d;
}

// one wavefront per row, for rows with many entries (coarse Galerkin levels):
// the lanes split the row and sum by shuffles
template <typename T>
__device__ __forceinline__ void gs_row_wave(int i, int lane, const int *__restrict__ rp,
                                            const int *__restrict__ ci, const T *__restrict__ v,
                                            const T *__restrict__ b, T *x) {
  // the diagonal entry is present and nonzero on every row (checked at setup);
  // lanes that do not hold it add zero
  T s = T(0), d = T(0);
  for (int k = rp[i] + lane; k < rp[i + 1]; k += 64) {
    const int j = ci[k];
    if (j == i)
      d = v[k];
    else
      s += v[k] * x[j];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o);
    d += __shfl_xor(d, o);
  }
  if (lane == 0) x[i] = (b[i] - s) / d;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_color_wave(int cnt, const int *__restrict__ rows,
                                                          const int *__restrict__ rp, const int *__restrict__ ci,
                                                          const T *__restrict__ v, const T *__restrict__ b, T *x) {
  const int w = (blockIdx.x * kBlock + threadIdx.x) >> 6;  // the same for the whole wavefront
  if (w >= cnt) return;
  gs_row_wave<T>(rows[w], threadIdx.x & 63, rp, ci, v, b, x);
}

// a whole sweep of a small level in one workgroup of kGsWaves wavefronts, a
// wavefront per row, a barrier between colours
constexpr int kGsWaves = 16;
template <typename T>
__global__ void __launch_bounds__(64 * kGsWaves) k_gs_level_wave(int ncol, int reverse, const int *__restrict__ cptr,
                                                                 const int *__restrict__ rows,
                                                                 const int *__restrict__ rp,
                                                                 const int *__restrict__ ci,
                                                                 const T *__restrict__ v, const T *__restrict__ b,
                                                                 T *x) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int cc = 0; cc < ncol; cc++) {
    const int c = reverse ? ncol - 1 - cc : cc;
    for (int t = cptr[c] + wv; t < cptr[c + 1]; t += kGsWaves) gs_row_wave<T>(rows[t], lane, rp, ci, v, b, x);
    __syncthreads();
  }
}

// a whole sweep of a small level in one workgroup: colours in order (reverse:
// descending), a barrier between colours
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_level(int ncol, int reverse, const int *__restrict__ cptr,
                                                     const int *__restrict__ rows, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const T *__restrict__ v,
                                                     const T *__restrict__ b, T *x) {
  for (int cc = 0; cc < ncol; cc++) {
    const int c = reverse ? ncol - 1 - cc : cc;
    for (int t = cptr[c] + threadIdx.x; t < cptr[c + 1]; t += kBlock) {
      const int i = rows[t];
      T s = b[i], d = T(1);
      for (int k = rp[i]; k < rp[i + 1]; k++) {
        const int j = ci[k];
        if (j == i)
          d = v[k];
        else
          s -= v[k] * x[j];
      }
      x[i] = s / d;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BILU numeric refactorisation on a kept pattern: the IKJ form in FP64, one
// thread per factor row, one launch per level of the forward sweep (a row
// reads only rows of earlier levels).  Every product and sum is rounded on
// its own, in the order of the host factorisation, so the factors are the
// host's bit for bit.
// ---------------------------------------------------------------------------
// lu[k] = the block of A that factor entry k starts from (zero for fill)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_ilu_load(int nnzf, const int *__restrict__ src,
                                                     const double *__restrict__ A, double *__restrict__ lu) {
  constexpr int B2 = NV * NV;
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (size_t)nnzf * B2) return;
  const size_t k = t / B2;
  const int s = src[k];
  lu[t] = s >= 0 ? A[(size_t)s * B2 + (t - k * B2)] : 0.0;
}

// c = a b (nv x nv, row-major), each entry summed from 0 over ascending k
template <int NV>
__device__ __forceinline__ void ilu_blk_mul(const double *a, const double *b, double *c) {
#pragma clang fp contract(off)
  for (int r = 0; r < NV; r++)
    for (int q = 0; q < NV; q++) {
      double s = 0.0;
      for (int k = 0; k < NV; k++) s += a[r * NV + k] * b[k * NV + q];
      c[r * NV + q] = s;
    }
}

// inverse by Gauss-Jordan elimination with partial pivoting; false on a zero
// or non-finite pivot
template <int NV>
__device__ __forceinline__ bool ilu_blk_inv(const double *a, double *inv) {
#pragma clang fp contract(off)
  double m[NV][2 * NV];
  for (int r = 0; r < NV; r++)
    for (int q = 0; q < 2 * NV; q++) m[r][q] = q < NV ? a[r * NV + q] : (q - NV == r ? 1.0 : 0.0);
  for (int k = 0; k < NV; k++) {
    int p = k;
    for (int r = k + 1; r < NV; r++)
      if (fabs(m[r][k]) > fabs(m[p][k])) p = r;
    if (m[p][k] == 0.0 || !isfinite(m[p][k])) return false;
    if (p != k)
      for (int q = 0; q < 2 * NV; q++) {
        const double x = m[k][q];
        m[k][q] = m[p][q];
        m[p][q] = x;
      }
    const double d = m[k][k];
    for (int q = 0; q < 2 * NV; q++) m[k][q] /= d;
    for (int r = 0; r < NV; r++) {
      if (r == k) continue;
      const double f = m[r][k];
      for (int q = 0; q < 2 * NV; q++) m[r][q] -= f * m[k][q];
    }
  }
  for (int r = 0; r < NV; r++)
    for (int q = 0; q < NV; q++) inv[r * NV + q] = m[r][NV + q];
  return true;
}

// rows fwd[p0 .. p0+cnt-1] (factor positions of one forward level):
// L_pq = A_pq U_qq^{-1} for the lower entries in column order, then
// A_pj -= L_pq U_qj for every upper entry (q, j) whose column is in row p;
// finally dinvp[p] = U_pp^{-1} (*bad = 1 on a zero pivot)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_ilu_factor(int p0, int cnt, const int *__restrict__ fwd,
                                                       const int *__restrict__ frp, const int *__restrict__ fci,
                                                       const int *__restrict__ dpos, double *__restrict__ lu,
                                                       double *__restrict__ dinvp, int *__restrict__ bad) {
#pragma clang fp contract(off)
  constexpr int B2 = NV * NV;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= cnt) return;
  const int p = fwd[p0 + t];
  const int e = frp[p + 1], dp = dpos[p];
  double L[B2], prod[B2], inv[B2];
  for (int k = frp[p]; k < dp; k++) {
    const int q = fci[k];
    ilu_blk_mul<NV>(lu + (size_t)k * B2, dinvp + (size_t)q * B2, L);
    for (int x = 0; x < B2; x++) lu[(size_t)k * B2 + x] = L[x];
    for (int u = dpos[q] + 1; u < frp[q + 1]; u++) {
      const int j = fci[u];
      int lo = k + 1, hi = e - 1, at = -1;  // columns of row p ascending; j > q puts it after k
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1, c = fci[mid];
        if (c == j) {
          at = mid;
          break;
        }
        if (c < j)
          lo = mid + 1;
        else
          hi = mid - 1;
      }
      if (at < 0) continue;
      ilu_blk_mul<NV>(L, lu + (size_t)u * B2, prod);
      for (int x = 0; x < B2; x++) lu[(size_t)at * B2 + x] -= prod[x];
    }
  }
  if (!ilu_blk_inv<NV>(lu + (size_t)dp * B2, inv)) {
    *bad = 1;
    for (int x = 0; x < B2; x++) inv[x] = 0.0;
  }
  for (int x = 0; x < B2; x++) dinvp[(size_t)p * B2 + x] = inv[x];
}

// the factor entries into the blocks of the two sweeps (dst >= 0: f_val,
// dst <= -2: b_val at -dst-2, -1: diagonal), U_pp^{-1} into cell order
template <int NV, typename T>
__global__ void __launch_bounds__(kBlock) k_ilu_store(int nnzf, int n, const int *__restrict__ dst,
                                                      const int *__restrict__ order, const double *__restrict__ lu,
                                                      const double *__restrict__ dinvp, T *__restrict__ f_val,
                                                      T *__restrict__ b_val, T *__restrict__ dinv) {
  constexpr int B2 = NV * NV;
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t ne = (size_t)nnzf * B2;
  if (t < ne) {
    const size_t k = t / B2, x = t - k * B2;
    const int d = dst[k];
    if (d >= 0)
      f_val[(size_t)d * B2 + x] = T(lu[t]);
    else if (d <= -2)
      b_val[(size_t)(-d - 2) * B2 + x] = T(lu[t]);
  } else if (t < ne + (size_t)n * B2) {
    const size_t u = t - ne, p = u / B2;
    dinv[(size_t)order[p] * B2 + (u - p * B2)] = T(dinvp[u]);
  }
}

// ---------------------------------------------------------------------------
// FP64 BSR product for the Arnoldi step and the true residual
//   y = A x (RESID = false),  y = b - A x (RESID = true)
// 64 block rows per workgroup, NV threads per block row (one per equation).
// ---------------------------------------------------------------------------
// With `slots` non-null, x is read from slots->z (the current Krylov column).
// Row layout of the caller's arrays; the column indices of up to 8 blocks are
// read first, then all their values and x entries, then the products.
template <int NV>
struct SpmvShape {
  static constexpr int R = 64;      // block rows per workgroup
  static constexpr int T = R * NV;  // threads
};

template <int NV, typename XT, bool RESID>
__global__ void __launch_bounds__(SpmvShape<NV>::T) k_bsr_spmv(int n, const int *__restrict__ rp,
                                                               const int *__restrict__ ci,
                                                               const double *__restrict__ vals,
                                                               const XT *__restrict__ xarg,
                                                               const ApplySlots *__restrict__ slots,
                                                               const double *__restrict__ b,
                                                               double *__restrict__ y) {
  constexpr int R = SpmvShape<NV>::R;
  const gmem<const XT> *__restrict__ x = as_global(slots ? reinterpret_cast<const XT *>(slots->z) : xarg);
  const int i = blockIdx.x * R + threadIdx.x / NV, r = threadIdx.x % NV;
  if (i >= n) return;
  double acc = 0.0;
  const int e = rp[i + 1];
  for (int k = rp[i]; k < e; k += 8) {
    int col[8];
#pragma unroll
    for (int q = 0; q < 8; q++) col[q] = k + q < e ? ci[k + q] : -1;
    double av[8][NV];
    double xv[8][NV];
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const bool ok = col[q] >= 0;
      const double *a = vals + ((size_t)(ok ? k + q : k) * NV + r) * NV;  // in bounds either way
      const gmem<const XT> *xc = x + (size_t)(ok ? col[q] : 0) * NV;
#pragma unroll
      for (int c = 0; c < NV; c++) {
        av[q][c] = ok ? a[c] : 0.0;
        xv[q][c] = ok ? double(xc[c]) : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; q++)
#pragma unroll
      for (int c = 0; c < NV; c++) acc += av[q][c] * xv[q][c];
  }
  const size_t o = (size_t)i * NV + r;
  y[o] = RESID ? b[o] - acc : acc;
}

// Sliced copy of the FP64 BSR matrix for the Krylov products: slices of 64
// block rows; slice s holds K_s = (longest row of the slice) block columns,
// kptr[s] = sum of K over the slices before s.  For block column k of the
// slice, entry (r, c) of the blocks of its 64 rows is stored contiguously:
//   vals[((kptr[s] + k) NV^2 + r NV + c) 64 + lane],  cols[(kptr[s] + k) 64 + lane]
// Rows shorter than K_s are padded with zero blocks in their own column.
// Wavefront r of the workgroup forms equation r of the slice's 64 rows, so
// every value load is 64 consecutive doubles.
template <int NV, typename XT, bool RESID>
__global__ void __launch_bounds__(64 * NV) k_bsr_spmv_sliced(int n, const int *__restrict__ kptr,
                                                              const int *__restrict__ cols,
                                                              const double *__restrict__ vals,
                                                              const XT *__restrict__ xarg,
                                                              const ApplySlots *__restrict__ slots,
                                                              const double *__restrict__ b,
                                                              double *__restrict__ y) {
  const gmem<const XT> *__restrict__ x = as_global(slots ? reinterpret_cast<const XT *>(slots->z) : xarg);
  const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sl = blockIdx.x, i = sl * 64 + lane;
  const int k0 = kptr[sl], k1 = kptr[sl + 1];
  double acc = 0.0;
#pragma unroll 4
  for (int k = k0; k < k1; k++) {
    const int col = cols[(size_t)k * 64 + lane];
    const double *a = vals + ((size_t)k * NV * NV + r * NV) * 64 + lane;
    const gmem<const XT> *xc = x + (size_t)col * NV;
#pragma unroll
    for (int c = 0; c < NV; c++) acc += a[c * 64] * double(xc[c]);
  }
  if (i >= n) return;
  const size_t o = (size_t)i * NV + r;
  y[o] = RESID ? b[o] - acc : acc;
}

// ---------------------------------------------------------------------------
// Krylov kernels (FP64).  Basis V is stored vector after vector: V[k*N + i].
// Deterministic reductions: per-block partials, then one fixed-order pass.
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 1024;

// Krylov state kept on the device
struct KState {
  int j;          // current column
  int m;          // restart length
  double beta;
  double hn;      // ||w|| of the last step
  double absg;    // |g_{j+1}|
  double tol;     // rtol ||b||: the cycle stops once |g_{j+1}| <= tol
  int stop;       // set by the step that ends the cycle (tolerance reached, breakdown
                  // or a non-finite value): later steps of the cycle leave the state alone
};

template <int MAXK>
__device__ __forceinline__ void block_store_partials(double (&acc)[MAXK], int kk, double *part) {
  __shared__ double sh[kBlock / 64][MAXK];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < MAXK; k++) {
    if (k < kk) {
      double v = wave_sum(acc[k]);
      if (lane == 0) sh[wv][k] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < kk) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; w++) s += sh[w][threadIdx.x];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;  // k-major: the reduction reads rows
  }
}

// Classical Gram-Schmidt with reorthogonalisation (CGS2) in two passes over
// the basis per Arnoldi step.  Step j leaves the next basis column as
// u = (w - V h1) / ||w|| (the first projection, scaled by the norm of w so
// that the preconditioner's next input has norm <= 1), with h2 = V^T (w - V
// h1) and hn = ||w - V h1 - V h2|| in the state; step j + 1 first applies
// the second projection and the normalisation to it,
//   v_{j+1} = (||w|| u - V h2) / hn,
// in the pass over the basis it makes anyway.  The preconditioner of step
// j + 1 receives u, not v_{j+1}: flexible GMRES needs only A z_{j+1} = w and
// an orthonormal V in the Arnoldi relation, whatever the preconditioned
// vectors are, and u differs from hn / ||w|| v_{j+1} by the second
// projection alone, a rounding-level correction.

// Pass 1 of step j: for j > 0 the correction of column j in place,
//   V[j] <- (V[j] omega - sum_{k<j} h2p[k] V[k]) / hn   (omega^2 = h1[j] and
//   hn = st->hn, both of step j - 1);
// then partial[blk][k] = sum_i V[k][i] w[i] for k <= j, and w2_part[blk] =
// sum_i w[i]^2.
template <int MAXK>
__global__ void __launch_bounds__(kBlock) k_mdot_fix(double *__restrict__ V, size_t N,
                                                     const KState *__restrict__ st,
                                                     const double *__restrict__ h2p,
                                                     const double *__restrict__ h1p,
                                                     const double *__restrict__ w, double *__restrict__ part,
                                                     double *__restrict__ w2_part) {
  const int J = st->j, kk = J + 1;
  double hk[MAXK], acc[MAXK];
  double accJ = 0.0, ww[1] = {0.0};
  const bool fix = J > 0;
  const double omega = fix ? sqrt(h1p[J]) : 1.0;
  const double hn = st->hn;
  const double inv = hn != 0.0 ? 1.0 / hn : 0.0;
#pragma unroll
  for (int k = 0; k < MAXK; k++) {
    acc[k] = 0.0;
    hk[k] = fix && k < J ? h2p[k] : 0.0;
  }
  double *__restrict__ vJ = V + (size_t)J * N;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    // every load of the row is issued before the first product waits on one
    double vk[MAXK];
    const double wi = w[i];
    double v = vJ[i];
#pragma unroll
    for (int k = 0; k < MAXK; k++) vk[k] = k < J ? V[(size_t)k * N + i] : 0.0;
    if (fix) {
      v = v * omega;
#pragma unroll
      for (int k = 0; k < MAXK; k++) v -= vk[k] * hk[k];
      v = v * inv;
      vJ[i] = v;
    }
#pragma unroll
    for (int k = 0; k < MAXK; k++) acc[k] += vk[k] * wi;
    accJ += v * wi;
    ww[0] += wi * wi;
  }
#pragma unroll
  for (int k = 0; k < MAXK; k++)
    if (k == J) acc[k] = accJ;
  block_store_partials<MAXK>(acc, kk, part);
  block_store_partials<1>(ww, 1, w2_part);
}

// Pass 2 of step j: w' = w - V h1 (columns k <= j); partial[blk][k] =
// sum_i V[k][i] w'[i] (the second projection) and w2_part[blk] = sum_i
// w'[i]^2; the next column V[j+1] = w' / ||w|| (||w||^2 = h1[j+1], from pass
// 1; a zero w leaves a zero column).
template <int MAXK>
__global__ void __launch_bounds__(kBlock) k_cgs_update_mdot(double *__restrict__ V, size_t N,
                                                            const int *__restrict__ jdev,
                                                            const double *__restrict__ h,
                                                            const double *__restrict__ w,
                                                            double *__restrict__ part,
                                                            double *__restrict__ w2_part) {
  const int kk = *jdev + 1;
  double acc[MAXK], hk[MAXK];
  double ww[1] = {0.0};
#pragma unroll
  for (int k = 0; k < MAXK; k++) {
    acc[k] = 0.0;
    hk[k] = k < kk ? h[k] : 0.0;
  }
  const double wn = sqrt(h[kk]);
  const double inv = wn != 0.0 ? 1.0 / wn : 0.0;
  double *__restrict__ vn = V + (size_t)kk * N;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    double vk[MAXK];
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < MAXK; k++) {
      vk[k] = k < kk ? V[(size_t)k * N + i] : 0.0;
      wi -= vk[k] * hk[k];
    }
    vn[i] = wi * inv;
    ww[0] += wi * wi;
#pragma unroll
    for (int k = 0; k < MAXK; k++) acc[k] += vk[k] * wi;
  }
  block_store_partials<MAXK>(acc, kk, part);
  block_store_partials<1>(ww, 1, w2_part);
}

// partial[blk][0] = sum_i x[i]^2
__global__ void __launch_bounds__(kBlock) k_norm2_partial(const double *__restrict__ x, size_t N,
                                                          double *__restrict__ part) {
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    acc[0] += x[i] * x[i];
  block_store_partials<1>(acc, 1, part);
}

// out[k] = sum_blk partial[k][blk] for k < kk (kk = *jdev + 1, or kfix when jdev is
// null), and out[kk] = the sum of the row `extra` when given; one workgroup per k; fixed order: thread t sums blocks t, t+256, ...,
// then a fixed tree, so the result does not depend on scheduling.  The loads of
// a thread (nblk <= kDotBlocks) are all issued before the first add.
__global__ void __launch_bounds__(kBlock) k_reduce(const double *__restrict__ part, int nblk,
                                                   const int *__restrict__ jdev, int kfix,
                                                   double *__restrict__ out, int sqrt_out,
                                                   const double *__restrict__ extra) {
  __shared__ double sh[kBlock / 64];
  const int kk = jdev ? *jdev + 1 : kfix;
  const int k = blockIdx.x;
  // with `extra`, workgroup kk sums that row into out[kk]
  if (k > kk || (k == kk && !extra)) return;
  const double *__restrict__ row = k == kk ? extra : part + (size_t)k * nblk;
  constexpr int kPer = kDotBlocks / kBlock;
  double v[kPer];
#pragma unroll
  for (int q = 0; q < kPer; q++) v[q] = row[min((int)threadIdx.x + q * kBlock, nblk - 1)];
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kPer; q++)
    if ((int)threadIdx.x + q * kBlock < nblk) s += v[q];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; w++) t += sh[w];
    out[k] = sqrt_out ? sqrt(t) : t;
  }
}


// Hessenberg column j = h1 + h2 (0..j), hn (j+1, computed here from h2 and
// ||w'||^2 = h2[j+1], kept in the state for the next step's correction); previous rotations, a new
// rotation, g update; j advances.  R is stored (m+1) x m row-major.  One
// wavefront: the lanes load the column and the rotations into LDS, lane 0
// applies them in order, the lanes store the column.
// A step launched after the one that set `stop` changes nothing here, so
// the cycle's solution uses the columns up to that step.
constexpr int kMaxRestart = 64;
__global__ void __launch_bounds__(64) k_givens(KState *st, const double *__restrict__ h1,
                                               const double *__restrict__ h2, double *__restrict__ R,
                                               double *__restrict__ cs, double *__restrict__ sn,
                                               double *__restrict__ g) {
  __shared__ double col[kMaxRestart + 1], c_[kMaxRestart], s_[kMaxRestart];
  if (blockIdx.x != 0 || st->stop) return;
  const int lane = threadIdx.x;
  const int j = st->j, m = st->m;
  // hn = ||w' - V h2|| = sqrt(||w'||^2 - ||h2||^2) (V orthonormal, h2 = V^T w';
  // ||w'||^2 in h2[j + 1], reduced with h2)
  if (lane == 0) {
    double hh = 0.0;
    for (int k = 0; k <= j; k++) hh += h2[k] * h2[k];
    st->hn = sqrt(fmax(h2[j + 1] - hh, 0.0));
  }
  __syncthreads();
  for (int k = lane; k <= j; k += 64) col[k] = h1[k] + h2[k];
  for (int k = lane; k < j; k += 64) {
    c_[k] = cs[k];
    s_[k] = sn[k];
  }
  if (lane == 0) col[j + 1] = st->hn;
  __syncthreads();
  if (lane == 0) {
    for (int k = 0; k < j; k++) {
      const double a = col[k], c = col[k + 1];
      col[k] = c_[k] * a + s_[k] * c;
      col[k + 1] = -s_[k] * a + c_[k] * c;
    }
    const double a = col[j], c = col[j + 1];
    const double den = hypot(a, c);
    const double cj = den == 0.0 ? 1.0 : a / den, sj = den == 0.0 ? 0.0 : c / den;
    cs[j] = cj;
    sn[j] = sj;
    col[j] = den;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
    const double ag = fabs(-sj * gj);
    st->absg = ag;
    st->j = j + 1;
    if (!(ag > st->tol) || st->hn == 0.0 || j + 1 == m) st->stop = 1;  // !(ag > tol) holds for NaN too
  }
  __syncthreads();
  for (int k = lane; k <= j + 1; k += 64) R[(size_t)k * m + j] = col[k];
}

__global__ void k_cycle_init(KState *st, const double *__restrict__ beta, double *__restrict__ g,
                             int m, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->j = 0;
  st->m = m;
  st->beta = *beta;
  st->hn = 0.0;
  st->tol = tol;
  st->stop = 0;
  st->absg = *beta;
  g[0] = *beta;
  for (int k = 1; k <= m; k++) g[k] = 0.0;
}

// v_0 = r / beta
__global__ void __launch_bounds__(kBlock) k_first_vector(double *__restrict__ V, size_t N,
                                                         const double *__restrict__ r,
                                                         const double *__restrict__ beta) {
  const double inv = 1.0 / *beta;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    V[i] = r[i] * inv;
}

// y = R^{-1} g over the first j columns (back substitution)
__global__ void k_solve_y(const KState *st, const double *__restrict__ R,
                          const double *__restrict__ g, double *__restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int kk = st->j, m = st->m;
  for (int i = kk - 1; i >= 0; i--) {
    double s = g[i];
    for (int q = i + 1; q < kk; q++) s -= R[(size_t)i * m + q] * y[q];
    y[i] = s / R[(size_t)i * m + i];
  }
}

// x += Z y over the first j columns
template <typename ZT>
__global__ void __launch_bounds__(kBlock) k_update_x(double *__restrict__ x, const ZT *__restrict__ Z,
                                                     size_t N, const KState *__restrict__ st,
                                                     const double *__restrict__ y) {
  const int kk = st->j;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    double s = x[i];
    for (int k = 0; k < kk; k++) s += double(Z[(size_t)k * N + i]) * y[k];
    x[i] = s;
  }
}

// slots for Krylov column j: v = V_j, z = Z_j
__global__ void k_set_slots_krylov(ApplySlots *slots, const double *V, void *Z, size_t N,
                                   int zbytes, const KState *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  slots->v = V + (size_t)st->j * N;
  slots->z = reinterpret_cast<char *>(Z) + (size_t)st->j * N * zbytes;
}

__global__ void k_set_slots(ApplySlots *slots, const double *v, void *z) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  slots->v = v;
  slots->z = z;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T *__restrict__ x, size_t n, T val) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    x[i] = val;
}

template <typename A, typename B>
__global__ void __launch_bounds__(kBlock) k_convert(const A *__restrict__ a, B *__restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    b[i] = B(a[i]);
}

}  // namespace cptr
