// Device kernels of libcptr for gfx950 (64-wide wavefronts).
//
// Sparse formats used on the device:
//   * FP64 BSR of the caller (row-major nv x nv blocks) for the Arnoldi
//     products w = A z and the true residual;
//   * SELL-64 ("sliced ELLPACK", one slice per wavefront of 64 rows, each
//     slice padded to its longest row and stored column-major inside the
//     slice) for scalar operators with short rows: the sub-blocks A_pp, A_pT,
//     A_Tp, S~_T on unstructured patterns, the prolongators P.  A lane reads
//     element k of its row at slice_base + 64 k + lane, so each load
//     instruction of a wave is one contiguous 256 B (FP32) segment;
//   * DIA (diagonal storage) for the same sub-blocks when their entries lie
//     on a few diagonals, as on a structured grid;
//   * CSR with several lanes per row for long rows (coarse AMG levels, the
//     restrictions R);
//   * the p/T columns of A as nv x 2 blocks in the BSR pattern (two-stage
//     residual);
//   * BILU(0) factors grouped by level of the triangular solves.
#pragma once

#include <hip/hip_runtime.h>

namespace cptr {

constexpr int kSlice = 64;

template <typename T>
struct Sell {
  using value_type = T;
  int nrows = 0;
  int nslices = 0;
  const int *sptr = nullptr;  // element offset of each slice, nslices + 1
  const int *col = nullptr;
  const T *val = nullptr;
};

// Diagonal storage of a square operator whose entries all lie on at most
// kMaxDiag diagonals (the 7-point couplings of a structured grid): entry
// (row, row + off[d]) is val[d * nrows + row], zero where the pattern has no
// entry.  No column indices are read, so an FP32 entry costs 4 B of traffic
// instead of the 8 B of a value + index pair.
constexpr int kMaxDiag = 8;

template <typename T>
struct Dia {
  using value_type = T;
  int nrows = 0;
  int ndiag = 0;
  int off[kMaxDiag] = {};  // ascending column offsets; entries past ndiag repeat the last
  const T *val = nullptr;
};

// Global-memory view of a pointer that a kernel reads from device memory (the
// slots below): accesses through it compile to global, not flat, loads and
// stores, which keeps them off the LDS counter and lets them be scheduled
// with the other global loads.
template <typename T>
using gmem = T __attribute__((address_space(1)));
template <typename T>
__device__ __forceinline__ gmem<T> *as_global(T *p) {
  return (gmem<T> *)p;
}

// pointer slots read by the first and last kernels of a preconditioner
// application, so that one captured graph serves every Krylov column
struct ApplySlots {
  const double *v;
  void *z;
};

}  // namespace cptr
