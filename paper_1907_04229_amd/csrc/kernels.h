// Device kernels of libcptr for gfx950 (64-wide wavefronts).
//
// Sparse formats used on the device:
//   * FP64 BSR of the caller (row-major nv x nv blocks) for the Arnoldi
//     products w = A z and the true residual;
//   * SELL-64 ("sliced ELLPACK", one slice per wavefront of 64 rows, each
//     slice padded to its longest row and stored column-major inside the
//     slice) for every scalar operator: the sub-blocks A_pp, A_pT, A_Tp, S~_T,
//     every AMG level and the transfer operators P, R.  A lane reads element
//     k of its row at slice_base + 64 k + lane, so each load instruction of a
//     wave is one contiguous 256 B (FP32) segment;
//   * the p/T columns of A as nv x 2 blocks in the BSR pattern (two-stage
//     residual);
//   * BILU(0) factors grouped by level of the triangular solves.
#pragma once

#include <hip/hip_runtime.h>

namespace cptr {

constexpr int kSlice = 64;

template <typename T>
struct Sell {
  int nrows = 0;
  int nslices = 0;
  const int *sptr = nullptr;  // element offset of each slice, nslices + 1
  const int *col = nullptr;
  const T *val = nullptr;
};

// pointer slots read by the first and last kernels of a preconditioner
// application, so that one captured graph serves every Krylov column
struct ApplySlots {
  const double *v;
  void *z;
};

}  // namespace cptr
