// libcptr: C ABI (include/cptr.h) of the MI355X CPTR-FGMRES path.
//
// One application of the preconditioner (Section 3.2, "two-stage"), in the
// handle's precision T (float or double):
//   a3  b_p, b_T  <- restriction of v to the p and T slots
//   a4  x_p  = V(A_pp) b_p                   (block preconditioner step 1)
//   a5  b~_T = b_T - A_Tp x_p                (step 2)
//   a6  d_T  = V(S~_T) b~_T                  (step 3)
//   a7  b~_p = b_p - A_pT d_T                (step 4)
//   a8  d_p  = V(A_pp) b~_p                  (step 5)
//   a9  b1   = v - A R^T (d_p, d_T)          (two-stage residual)
//   a10 z    = BILU0^{-1} b1 + R^T (d_p, d_T)
// V(.) is one smoothed-aggregation V-cycle; its coarsest level is applied in
// FP64.  FGMRES (a12, a13) is FP64 throughout; in FP32 mode the preconditioned
// vectors Z are stored in FP32 (they are produced in FP32, so nothing is lost).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cptr_learn.h"
#include "../../include/cptr_model.h"
#include "common.h"
#include "device_kernels.hip"
#include "learned_kernels.hip"
#include "model_kernels.hip"
#include "setup_kernels.hip"

namespace cptr {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

// ---------------------------------------------------------------- device memory
struct DevMem {
  void *p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  DevMem(DevMem &&o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevMem &operator=(DevMem &&o) noexcept {
    if (this != &o) {
      if (p) (void)hipFree(p);
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t b) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    bytes = b;
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{CPTR_ERR_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    }
  }
};

template <typename X>
static inline X *devp(const DevMem &m) { return reinterpret_cast<X *>(m.p); }

template <typename X>
static void upload(DevMem &m, const std::vector<X> &h) {
  m.alloc(h.size() * sizeof(X));
  if (!h.empty()) CPTR_HIP_TRY(hipMemcpy(m.p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice));
}

static inline int nblk(size_t n, int b = kBlock) { return int((n + b - 1) / b); }
static inline int sgrid(size_t n) { return std::max(1, std::min(kDotBlocks, nblk(n))); }

#define LAUNCH_CHECK() CPTR_HIP_TRY(hipGetLastError())

// ---------------------------------------------------------------- scalar operators
// A scalar sparse operator on the device, stored for the kernel that suits
// its pattern: DIA when every entry lies on one of a few diagonals (the
// 7-point fine-level operators of a structured grid), SELL-64 with one thread
// per row for other short rows, CSR with G lanes per row for long rows
// (coarse AMG levels and the restriction, tens to hundreds of entries).
constexpr int kDiaMinRows = 4096;

template <typename T>
struct SpOp {
  enum Fmt { kSell, kDia, kCsrv };
  DevMem sptr, col, val, rp;
  Sell<T> view;
  Dia<T> dia;
  Fmt fmt = kSell;
  int nrows = 0, ncols = 0, lanes = 1;  // lanes: CSR lanes per row
  size_t nnz = 0;

  // Diagonal storage if the pattern spans at most kMaxDiag diagonals and they
  // are at least half full; false leaves the operator untouched.
  bool build_dia(const HostCSR &a) {
    if (a.nr != a.nc || a.nr < kDiaMinRows) return false;
    int off[kMaxDiag], nd = 0;
    for (int r = 0; r < a.nr; r++)
      for (int q = a.rp[r]; q < a.rp[r + 1]; q++) {
        const int o = a.ci[q] - r;
        int d = 0;
        while (d < nd && off[d] != o) d++;
        if (d == nd) {
          if (nd == kMaxDiag) return false;
          off[nd++] = o;
        }
      }
    if (nd == 0 || 2 * (size_t)a.nnz() < (size_t)nd * a.nr) return false;
    std::sort(off, off + nd);
    std::vector<T> v((size_t)nd * a.nr, T(0));
    std::vector<double> acc((size_t)nd * a.nr, 0.0);
    for (int r = 0; r < a.nr; r++)
      for (int q = a.rp[r]; q < a.rp[r + 1]; q++) {
        const int d = int(std::lower_bound(off, off + nd, a.ci[q] - r) - off);
        acc[(size_t)d * a.nr + r] += a.v[q];
      }
    for (size_t i = 0; i < v.size(); i++) v[i] = T(acc[i]);
    upload(val, v);
    dia.nrows = a.nr;
    dia.ndiag = nd;
    for (int d = 0; d < kMaxDiag; d++) dia.off[d] = off[std::min(d, nd - 1)];  // padded: see row_sum
    dia.val = devp<T>(val);
    fmt = kDia;
    return true;
  }

  void build(const HostCSR &a, bool allow_dia = true) {
    nrows = a.nr;
    ncols = a.nc;
    nnz = a.nnz();
    const double avg = a.nr ? double(nnz) / a.nr : 0.0;
    lanes = 1;
    if (avg > 12.0) {
      lanes = 2;
      while (lanes < 64 && lanes * 4 < avg) lanes *= 2;
    }
    if (lanes > 1) {
      fmt = kCsrv;
      upload(rp, a.rp);
      upload(col, a.ci);
      std::vector<T> v(a.v.begin(), a.v.end());
      upload(val, v);
      return;
    }
    if (allow_dia && build_dia(a)) return;
    fmt = kSell;
    int ns = (a.nr + kSlice - 1) / kSlice;
    std::vector<int> sp(ns + 1, 0);
    for (int s = 0; s < ns; s++) {
      int w = 0;
      for (int r = s * kSlice; r < std::min(a.nr, (s + 1) * kSlice); r++)
        w = std::max(w, a.rp[r + 1] - a.rp[r]);
      sp[s + 1] = sp[s] + w * kSlice;
    }
    std::vector<int> c(std::max(sp[ns], 1), 0);
    std::vector<T> v(std::max(sp[ns], 1), T(0));
    for (int s = 0; s < ns; s++)
      for (int lane = 0; lane < kSlice; lane++) {
        int r = s * kSlice + lane;
        if (r >= a.nr) break;
        int k = 0;
        for (int q = a.rp[r]; q < a.rp[r + 1]; q++, k++) {
          c[sp[s] + k * kSlice + lane] = a.ci[q];
          v[sp[s] + k * kSlice + lane] = T(a.v[q]);
        }
      }
    upload(sptr, sp);
    upload(col, c);
    upload(val, v);
    view.nrows = a.nr;
    view.nslices = ns;
    view.sptr = devp<int>(sptr);
    view.col = devp<int>(col);
    view.val = devp<T>(val);
  }
  // New values on the kept pattern: CSR entry k of the operator (device row
  // pointers rp and columns ci, as given to build) is src[k stride + off],
  // stored as build stores it.
  void refresh(hipStream_t st, const int *rp_d, const int *ci_d, const double *src, int stride, int off) {
    if (fmt == kCsrv)
      hipLaunchKernelGGL((k_rs_csr_vals<T>), dim3(nblk(nnz)), dim3(kBlock), 0, st, nnz, src, stride, off,
                         devp<T>(val));
    else if (fmt == kSell)
      hipLaunchKernelGGL((k_rs_sell_vals<T>), dim3(nblk(nrows)), dim3(kBlock), 0, st, nrows, rp_d, src, stride, off,
                         devp<int>(sptr), devp<T>(val));
    else
      hipLaunchKernelGGL((k_rs_dia_vals<T>), dim3(nblk(nrows)), dim3(kBlock), 0, st, nrows, rp_d, ci_d, src, stride,
                         off, dia, devp<T>(val));
    LAUNCH_CHECK();
  }

  // algorithmic bytes of one product: stored values, indices, row/slice offsets
  double bytes() const {
    if (fmt == kDia) return double(dia.ndiag) * nrows * sizeof(T);
    return double(nnz) * (sizeof(T) + 4) + 4.0 * (fmt == kCsrv ? nrows + 1 : view.nslices + 1);
  }

#define CPTR_CSRV_SWITCH(CALL)                  \
  switch (lanes) {                               \
    case 2: CALL(2); break;                      \
    case 4: CALL(4); break;                      \
    case 8: CALL(8); break;                      \
    case 16: CALL(16); break;                    \
    case 32: CALL(32); break;                    \
    default: CALL(64); break;                    \
  }
// one-thread-per-row kernel K over the SELL or DIA view
#define CPTR_ROW_LAUNCH(K, ...)                                                                    \
  do {                                                                                             \
    if (fmt == kDia)                                                                               \
      hipLaunchKernelGGL((K<Dia<T>, ##__VA_ARGS__>), dim3(nblk(nrows)), dim3(kBlock), 0, st, dia, ROW_ARGS); \
    else                                                                                           \
      hipLaunchKernelGGL((K<Sell<T>, ##__VA_ARGS__>), dim3(nblk(nrows)), dim3(kBlock), 0, st, view, ROW_ARGS); \
  } while (0)

  // y = A x (mode 0), y += A x (mode 1), y = b - A x (mode 2)
  template <int MODE>
  void spmv(hipStream_t st, const T *x, const T *b, T *y) const {
    if (fmt != kCsrv) {
#define ROW_ARGS x, b, y
      CPTR_ROW_LAUNCH(k_spmv, MODE);
#undef ROW_ARGS
    } else {
      const int *r = devp<int>(rp), *c = devp<int>(col);
      const T *v = devp<T>(val);
      const int g = nblk((size_t)nrows * lanes);
#define CALL(G) hipLaunchKernelGGL((k_csrv_spmv<T, G, MODE>), dim3(g), dim3(kBlock), 0, st, nrows, r, c, v, x, b, y)
      CPTR_CSRV_SWITCH(CALL)
#undef CALL
    }
    LAUNCH_CHECK();
  }
  void jacobi(hipStream_t st, const T *dinv, const T *b, const T *xin, T *xout) const {
    if (fmt != kCsrv) {
#define ROW_ARGS dinv, b, xin, xout
      CPTR_ROW_LAUNCH(k_jacobi);
#undef ROW_ARGS
    } else {
      const int *r = devp<int>(rp), *c = devp<int>(col);
      const T *v = devp<T>(val);
      const int g = nblk((size_t)nrows * lanes);
#define CALL(G) hipLaunchKernelGGL((k_csrv_jacobi<T, G>), dim3(g), dim3(kBlock), 0, st, nrows, r, c, v, dinv, b, xin, xout)
      CPTR_CSRV_SWITCH(CALL)
#undef CALL
    }
    LAUNCH_CHECK();
  }
  void smooth0_next(hipStream_t st, const T *dinv, const T *b, T *x) const {
    if (fmt != kCsrv) {
#define ROW_ARGS dinv, b, x
      CPTR_ROW_LAUNCH(k_smooth0_next);
#undef ROW_ARGS
    } else {
      const int *r = devp<int>(rp), *c = devp<int>(col);
      const T *v = devp<T>(val);
      const int g = nblk((size_t)nrows * lanes);
#define CALL(G) hipLaunchKernelGGL((k_csrv_smooth0_next<T, G>), dim3(g), dim3(kBlock), 0, st, nrows, r, c, v, dinv, b, x)
      CPTR_CSRV_SWITCH(CALL)
#undef CALL
    }
    LAUNCH_CHECK();
  }
  void smooth0_resid(hipStream_t st, const T *dinv, const T *b, T *x, T *res) const {
    if (fmt != kCsrv) {
#define ROW_ARGS dinv, b, x, res
      CPTR_ROW_LAUNCH(k_smooth0_resid);
#undef ROW_ARGS
    } else {
      const int *r = devp<int>(rp), *c = devp<int>(col);
      const T *v = devp<T>(val);
      const int g = nblk((size_t)nrows * lanes);
#define CALL(G) hipLaunchKernelGGL((k_csrv_smooth0_resid<T, G>), dim3(g), dim3(kBlock), 0, st, nrows, r, c, v, dinv, b, x, res)
      CPTR_CSRV_SWITCH(CALL)
#undef CALL
    }
    LAUNCH_CHECK();
  }
#undef CPTR_ROW_LAUNCH
};

// ---------------------------------------------------------------- AMG on device
constexpr int kSpgWaveMin = 32;   // products per row above which a Galerkin product takes a wavefront per row
constexpr int kGsOneBlock = 2048;  // Gauss-Seidel levels up to this many rows: one workgroup per sweep

template <typename T>
struct AmgDev {
  struct Level {
    SpOp<T> A, P, R;
    DevMem dinv, b, x, y, r;
    DevMem gs_rp, gs_ci, gs_v, gs_rows, gs_cptr;  // Gauss-Seidel: A as CSR, rows grouped by colour
    std::vector<int> gs_ptr;             // colour c holds gs_rows[gs_ptr[c] .. gs_ptr[c+1])
    bool gs_wide = false;                // rows long enough for a wavefront each
    int n = 0;
  };
  std::vector<std::unique_ptr<Level>> lev;
  DevMem coarse_inv;
  int nc = 0;
  int sweeps = 1;
  int smoother = CPTR_SMOOTHER_L1JACOBI;
  std::vector<std::vector<int>> agg;  // host copy of the aggregates (introspection)
  double bytes_per_cycle = 0.0;

  // Numeric re-setup on the device: every level in FP64 CSR with the kept
  // patterns of its setup products (the prolongator P, R = P^T and A P), so
  // that new level-0 values give the values of the whole hierarchy (renumeric).
  struct Num {
    int n = 0;
    bool smooth = false;
    size_t nnz = 0, pnnz = 0, rnnz = 0;
    DevMem a_rp, a_ci, a_v, diag, ratio;                        // level operator A
    DevMem agg, p_rp, p_ci, p_v, pslot;                         // P; pslot: P entry of each A entry
    DevMem r_rp, r_ci, r_src, r_v;                              // R; r_src: P entry of each R entry
    DevMem t_rp, t_ci, t_v;                                     // A P
    bool ap_wave = false, rt_wave = false;  // A P, R (A P): many products per row, a wavefront each
  };
  std::vector<Num> num;   // empty: the hierarchy is re-set up on the host
  DevMem gj, gj_f, scal;  // coarsest [A | I] of the Gauss-Jordan inverse, its column factors; omega, block maxima

  void build_plan(const AmgHost &h) {
    num.clear();
    num.resize(h.lev.size());
    for (size_t l = 0; l < h.lev.size(); l++) {
      const AmgLevelHost &H = h.lev[l];
      Num &N = num[l];
      N.n = H.A.nr;
      N.nnz = H.A.ci.size();
      upload(N.a_rp, H.A.rp);
      upload(N.a_ci, H.A.ci);
      upload(N.a_v, H.A.v);
      if (l + 1 == h.lev.size()) break;
      N.smooth = H.smooth;
      N.diag.alloc((size_t)N.n * 8);
      if (N.smooth) N.ratio.alloc((size_t)N.n * 8);
      N.pnnz = H.P.ci.size();
      N.rnnz = H.R.ci.size();
      upload(N.agg, H.agg);
      upload(N.p_rp, H.P.rp);
      upload(N.p_ci, H.P.ci);
      upload(N.p_v, H.P.v);
      upload(N.r_rp, H.R.rp);
      upload(N.r_ci, H.R.ci);
      upload(N.r_v, H.R.v);
      upload(N.t_rp, H.AP.rp);
      upload(N.t_ci, H.AP.ci);
      N.t_v.alloc(std::max<size_t>(H.AP.ci.size(), 1) * 8);
      {  // products per row of A P and of R (A P)
        double fa = 0.0, fr = 0.0;
        for (int k = 0; k < (int)N.nnz; k++) fa += H.P.rp[H.A.ci[k] + 1] - H.P.rp[H.A.ci[k]];
        for (size_t k = 0; k < N.rnnz; k++) fr += H.AP.rp[H.R.ci[k] + 1] - H.AP.rp[H.R.ci[k]];
        N.ap_wave = fa > kSpgWaveMin * std::max(1, N.n);
        N.rt_wave = fr > kSpgWaveMin * std::max(1, H.R.nr);
      }
      if (N.smooth) {
        std::vector<int> ps(N.nnz, -1);
        for (int i = 0; i < N.n; i++)
          for (int k = H.A.rp[i]; k < H.A.rp[i + 1]; k++) {
            const int J = H.agg[H.A.ci[k]];
            if (J < 0) continue;
            const auto b = H.P.ci.begin() + H.P.rp[i], e = H.P.ci.begin() + H.P.rp[i + 1];
            const auto it = std::lower_bound(b, e, J);
            if (it == e || *it != J) throw Error{CPTR_ERR_SETUP, "prolongator pattern misses an aggregate"};
            ps[k] = int(it - H.P.ci.begin());
          }
        upload(N.pslot, ps);
        // R = P^T entry by entry, in the order of the transpose
        std::vector<int> fill(H.R.rp.begin(), H.R.rp.end() - 1), src(N.rnnz);
        for (int i = 0; i < N.n; i++)
          for (int k = H.P.rp[i]; k < H.P.rp[i + 1]; k++) {
            const int q = fill[H.P.ci[k]]++;
            if (H.R.ci[q] != i) throw Error{CPTR_ERR_SETUP, "restriction pattern is not the transpose"};
            src[q] = k;
          }
        upload(N.r_src, src);
      }
    }
    const int nc = h.lev.back().A.nr;
    gj.alloc((size_t)nc * 2 * nc * 8);
    gj_f.alloc((size_t)nc * 8);
    scal.alloc((1 + kDotBlocks) * 8);
  }

  // C = A B on C's kept pattern (k_rs_spgemm, or k_rs_spgemm_wave for rows of many products)
  static void spgemm(hipStream_t st, bool wave, int nr, const DevMem &arp, const DevMem &aci, const DevMem &av,
                     const DevMem &brp, const DevMem &bci, const DevMem &bv, const DevMem &crp, const DevMem &cci,
                     DevMem &cv) {
    if (nr <= 0) return;
    if (wave)
      hipLaunchKernelGGL(k_rs_spgemm_wave, dim3(nr), dim3(64), 0, st, devp<int>(arp), devp<int>(aci),
                         devp<double>(av), devp<int>(brp), devp<int>(bci), devp<double>(bv), devp<int>(crp),
                         devp<int>(cci), devp<double>(cv));
    else
      hipLaunchKernelGGL(k_rs_spgemm, dim3(nblk(nr)), dim3(kBlock), 0, st, nr, devp<int>(arp), devp<int>(aci),
                         devp<double>(av), devp<int>(brp), devp<int>(bci), devp<double>(bv), devp<int>(crp),
                         devp<int>(cci), devp<double>(cv));
    LAUNCH_CHECK();
  }

  // New values of every level from those of level 0 (num[0].a_v), on the
  // kept aggregates and patterns, as amg_build computes them (see the kernels
  // of the numeric re-setup); errors are or-ed into *flag.
  void renumeric(hipStream_t st, int *flag) {
    const size_t L = lev.size();
    double *omega = devp<double>(scal), *part = omega + 1;
    for (size_t l = 0; l + 1 < L; l++) {
      Num &N = num[l], &C = num[l + 1];
      Level &Lv = *lev[l];
      const bool gs = smoother == CPTR_SMOOTHER_GS;
      hipLaunchKernelGGL((k_rs_rowabs<T>), dim3(nblk(N.n)), dim3(kBlock), 0, st, N.n, devp<int>(N.a_rp),
                         devp<int>(N.a_ci), devp<double>(N.a_v), devp<double>(N.diag),
                         N.smooth ? devp<double>(N.ratio) : (double *)nullptr, devp<T>(Lv.dinv),
                         (N.smooth || gs) ? 1 : 0, flag);
      LAUNCH_CHECK();
      if (N.smooth) {
        const int nb = sgrid(N.n);
        hipLaunchKernelGGL(k_rs_max_partial, dim3(nb), dim3(kBlock), 0, st, N.n, devp<double>(N.ratio), part);
        hipLaunchKernelGGL(k_rs_omega, dim3(1), dim3(kBlock), 0, st, nb, (const double *)part, omega);
        hipLaunchKernelGGL(k_rs_prolong, dim3(nblk(N.n)), dim3(kBlock), 0, st, N.n, devp<int>(N.a_rp),
                           devp<double>(N.a_v), devp<int>(N.pslot), devp<int>(N.agg), devp<double>(N.diag),
                           (const double *)omega, devp<int>(N.p_rp), devp<int>(N.p_ci), devp<double>(N.p_v));
        hipLaunchKernelGGL(k_rs_gather, dim3(nblk(N.rnnz)), dim3(kBlock), 0, st, N.rnnz, devp<int>(N.r_src),
                           devp<double>(N.p_v), devp<double>(N.r_v));
        LAUNCH_CHECK();
      }
      spgemm(st, N.ap_wave, N.n, N.a_rp, N.a_ci, N.a_v, N.p_rp, N.p_ci, N.p_v, N.t_rp, N.t_ci, N.t_v);
      spgemm(st, N.rt_wave, C.n, N.r_rp, N.r_ci, N.r_v, N.t_rp, N.t_ci, N.t_v, C.a_rp, C.a_ci, C.a_v);
      Lv.A.refresh(st, devp<int>(N.a_rp), devp<int>(N.a_ci), devp<double>(N.a_v), 1, 0);
      if (N.smooth) {
        Lv.P.refresh(st, devp<int>(N.p_rp), devp<int>(N.p_ci), devp<double>(N.p_v), 1, 0);
        Lv.R.refresh(st, devp<int>(N.r_rp), devp<int>(N.r_ci), devp<double>(N.r_v), 1, 0);
      }
      if (gs) {
        hipLaunchKernelGGL((k_rs_csr_vals<T>), dim3(nblk(N.nnz)), dim3(kBlock), 0, st, N.nnz,
                           (const double *)devp<double>(N.a_v), 1, 0, devp<T>(Lv.gs_v));
        LAUNCH_CHECK();
      }
    }
    // the coarsest operator's explicit inverse
    const Num &Q = num[L - 1];
    const int m = Q.n;
    double *g = devp<double>(gj), *f = devp<double>(gj_f);
    hipLaunchKernelGGL(k_rs_gj_init, dim3(nblk(m)), dim3(kBlock), 0, st, m, devp<int>(Q.a_rp), devp<int>(Q.a_ci),
                       devp<double>(Q.a_v), g);
    LAUNCH_CHECK();
    for (int c = 0; c < m; c++) {
      hipLaunchKernelGGL(k_rs_gj_pivot, dim3(1), dim3(kGjBlock), 0, st, m, c, g, f, flag);
      hipLaunchKernelGGL(k_rs_gj_elim, dim3(nblk((size_t)m * 2 * m)), dim3(kBlock), 0, st, m, c, g,
                         (const double *)f);
    }
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rs_gj_out, dim3(nblk((size_t)m * m)), dim3(kBlock), 0, st, m, (const double *)g,
                       devp<double>(coarse_inv));
    LAUNCH_CHECK();
  }

  void build(const AmgHost &h, int nsweeps, bool dia, int smoother_kind = CPTR_SMOOTHER_L1JACOBI,
             bool plan = false) {
    sweeps = std::max(1, nsweeps);
    smoother = smoother_kind;
    lev.clear();
    agg.clear();
    num.clear();
    bytes_per_cycle = 0.0;
    if (plan) build_plan(h);
    const size_t s = sizeof(T);
    for (size_t l = 0; l < h.lev.size(); l++) {
      auto L = std::make_unique<Level>();
      const AmgLevelHost &H = h.lev[l];
      L->n = H.A.nr;
      agg.push_back(H.agg);
      L->b.alloc(L->n * s);
      L->x.alloc(L->n * s);
      L->y.alloc(L->n * s);
      L->r.alloc(L->n * s);
      if (l + 1 < h.lev.size()) {
        L->A.build(H.A, dia);
        L->P.build(H.P, dia);
        L->R.build(H.R, dia);
        std::vector<T> d(L->n);
        for (int i = 0; i < L->n; i++) {
          double sum = 0.0;
          for (int k = H.A.rp[i]; k < H.A.rp[i + 1]; k++) sum += std::fabs(H.A.v[k]);
          d[i] = T(1.0 / sum);
        }
        upload(L->dinv, d);
        if (smoother == CPTR_SMOOTHER_GS) {
          // every row needs a nonzero diagonal entry (the sweeps divide by it)
          for (int i = 0; i < L->n; i++) {
            double dii = 0.0;
            for (int k = H.A.rp[i]; k < H.A.rp[i + 1]; k++)
              if (H.A.ci[k] == i) dii = H.A.v[k];
            if (dii == 0.0)
              throw Error{CPTR_ERR_SINGULAR_BLOCK, "Gauss-Seidel smoother: zero diagonal entry in row " +
                                                       std::to_string(i) + " of AMG level " + std::to_string(l)};
          }
          // greedy colouring in natural order: the smallest colour not taken
          // by a lower-numbered neighbour (a proper colouring: the pattern is
          // symmetric); rows grouped by colour, ascending inside a colour
          std::vector<int> col(L->n, 0), mark;
          int ncol = 0;
          for (int i = 0; i < L->n; i++) {
            mark.assign(ncol + 1, 0);
            for (int k = H.A.rp[i]; k < H.A.rp[i + 1]; k++)
              if (H.A.ci[k] < i) mark[col[H.A.ci[k]]] = 1;
            int c = 0;
            while (mark[c]) c++;
            col[i] = c;
            ncol = std::max(ncol, c + 1);
          }
          L->gs_ptr.assign(ncol + 1, 0);
          for (int i = 0; i < L->n; i++) L->gs_ptr[col[i] + 1]++;
          for (int c = 0; c < ncol; c++) L->gs_ptr[c + 1] += L->gs_ptr[c];
          std::vector<int> fill(L->gs_ptr.begin(), L->gs_ptr.end() - 1), rows(L->n);
          for (int i = 0; i < L->n; i++) rows[fill[col[i]]++] = i;
          upload(L->gs_rows, rows);
          upload(L->gs_cptr, L->gs_ptr);
          L->gs_wide = H.A.nnz() >= 16 * (long long)L->n;
          upload(L->gs_rp, H.A.rp);
          upload(L->gs_ci, H.A.ci);
          std::vector<T> av(H.A.v.begin(), H.A.v.end());
          upload(L->gs_v, av);
        }
        double n = L->n;
        if (smoother == CPTR_SMOOTHER_GS) {
          // x = 0; sweeps forward and sweeps backward Gauss-Seidel sweeps, each
          // reading the CSR values and indices, the row list, b_i and x_i and
          // writing x_i (the x_j of the neighbours from cache); the residual
          // b - A x; restriction; prolongation; the final copy to the output
          const double sweep = double(H.A.nnz()) * (s + 4) + 4.0 * (n + 1) + 4.0 * n + 3 * n * s;
          bytes_per_cycle += n * s + (2.0 * sweeps) * sweep + (L->A.bytes() + 3 * n * s)  // b - A x
                             + L->R.bytes() + n * s + H.R.nr * s                          // R r
                             + L->P.bytes() + 2 * n * s + H.P.nc * s                      // x += P x_c
                             + 2 * n * s;                                                 // out = x
        } else {
          // pre: sweeps passes over A, each leaving the residual of its iterate;
          // post: sweeps Jacobi passes; restriction and prolongation once each
          bytes_per_cycle += (2.0 * sweeps) * (L->A.bytes() + 3 * n * s)  // A x, b, dinv, x
                             + L->R.bytes() + n * s + H.R.nr * s          // R r
                             + L->P.bytes() + 2 * n * s + H.P.nc * s;     // x += P x_c
        }
      }
      lev.push_back(std::move(L));
    }
    nc = h.lev.back().A.nr;
    upload(coarse_inv, h.coarse_inv);
    bytes_per_cycle += double(nc) * nc * 8 + 2.0 * nc * s;
  }

  // x = V(b) from a zero guess; b and x are level-0 sized device vectors (T)
  void cycle(hipStream_t st, const T *b, T *x) const { cycle_level(st, 0, b, x); }

  void cycle_level(hipStream_t st, size_t l, const T *b, T *out) const {
    const Level &L = *lev[l];
    if (l + 1 == lev.size()) {
      const int waves_per_block = kBlock / 64;
      hipLaunchKernelGGL((k_coarse_gemv<T>), dim3(nblk(nc, waves_per_block)), dim3(kBlock), 0, st,
                         devp<double>(coarse_inv), nc, b, out);
      LAUNCH_CHECK();
      return;
    }
    T *x = devp<T>(L.x), *y = devp<T>(L.y), *r = devp<T>(L.r);
    const T *dinv = devp<T>(L.dinv);
    const Level &C = *lev[l + 1];
    if (smoother == CPTR_SMOOTHER_GS) {
      // symmetric multicolour Gauss-Seidel: colours ascending before the
      // coarse correction (from x = 0), descending after it
      auto sweep = [&](bool reverse) {
        const int ncol = int(L.gs_ptr.size()) - 1;
        if (L.n <= kGsOneBlock) {  // coarse levels: many colours, few rows each
          if (L.gs_wide)
            hipLaunchKernelGGL((k_gs_level_wave<T>), dim3(1), dim3(64 * kGsWaves), 0, st, ncol, reverse ? 1 : 0,
                               devp<int>(L.gs_cptr), devp<int>(L.gs_rows), devp<int>(L.gs_rp),
                               devp<int>(L.gs_ci), devp<T>(L.gs_v), b, x);
          else
            hipLaunchKernelGGL((k_gs_level<T>), dim3(1), dim3(kBlock), 0, st, ncol, reverse ? 1 : 0,
                               devp<int>(L.gs_cptr), devp<int>(L.gs_rows), devp<int>(L.gs_rp),
                               devp<int>(L.gs_ci), devp<T>(L.gs_v), b, x);
          LAUNCH_CHECK();
          return;
        }
        for (int cc = 0; cc < ncol; cc++) {
          const int c = reverse ? ncol - 1 - cc : cc;
          const int cnt = L.gs_ptr[c + 1] - L.gs_ptr[c];
          if (cnt <= 0) continue;
          if (L.gs_wide)
            hipLaunchKernelGGL((k_gs_color_wave<T>), dim3(nblk((size_t)cnt * 64)), dim3(kBlock), 0, st, cnt,
                               devp<int>(L.gs_rows) + L.gs_ptr[c], devp<int>(L.gs_rp), devp<int>(L.gs_ci),
                               devp<T>(L.gs_v), b, x);
          else
            hipLaunchKernelGGL((k_gs_color<T>), dim3(nblk(cnt)), dim3(kBlock), 0, st, cnt,
                               devp<int>(L.gs_rows) + L.gs_ptr[c], devp<int>(L.gs_rp), devp<int>(L.gs_ci),
                               devp<T>(L.gs_v), b, x);
          LAUNCH_CHECK();
        }
      };
      hipLaunchKernelGGL((k_fill<T>), dim3(sgrid(L.n)), dim3(kBlock), 0, st, x, (size_t)L.n, T(0));
      LAUNCH_CHECK();
      for (int s = 0; s < sweeps; s++) sweep(false);
      L.A.template spmv<2>(st, x, b, r);
      L.R.template spmv<0>(st, r, nullptr, devp<T>(C.b));
      cycle_level(st, l + 1, devp<T>(C.b), devp<T>(C.r));
      L.P.template spmv<1>(st, devp<T>(C.r), nullptr, x);
      for (int s = 0; s < sweeps; s++) sweep(true);
      hipLaunchKernelGGL((k_convert<T, T>), dim3(sgrid(L.n)), dim3(kBlock), 0, st, (const T *)x, out,
                         (size_t)L.n);
      LAUNCH_CHECK();
      return;
    }
    // pre-smoothing from zero: one pass for the first two sweeps, one per
    // further sweep, the last forming the residual of the smoothed iterate
    if (sweeps == 1) {
      L.A.smooth0_resid(st, dinv, b, x, r);
    } else {
      L.A.smooth0_next(st, dinv, b, x);
      for (int s = 2; s < sweeps; s++) {
        L.A.jacobi(st, dinv, b, x, y);
        std::swap(x, y);
      }
      L.A.template spmv<2>(st, x, b, r);
    }
    // restriction, coarse correction, prolongation
    L.R.template spmv<0>(st, r, nullptr, devp<T>(C.b));
    cycle_level(st, l + 1, devp<T>(C.b), devp<T>(C.r));  // coarse result in C.r
    L.P.template spmv<1>(st, devp<T>(C.r), nullptr, x);
    // post-smoothing; the last sweep writes to out
    T *cur = x;
    for (int s = 0; s < sweeps; s++) {
      T *dst = (s == sweeps - 1) ? out : (cur == x ? y : x);
      L.A.jacobi(st, dinv, b, cur, dst);
      cur = dst;
    }
  }
};

// ---------------------------------------------------------------- BILU(0) on device
template <typename T>
struct IluDev {
  DevMem f_rows, f_ptr, f_col, f_val, b_rows, b_ptr, b_col, b_val, dinv;
  // factor pattern for a numeric refactorisation (IluHost's frp .. fwd, order)
  DevMem r_frp, r_fci, r_src, r_dpos, r_dst, r_fwd, r_order;
  int n = 0, nv = 0, nnzf = 0;
  std::vector<int> f_lev_ptr, b_lev_ptr;
  std::vector<char> f_nonempty;  // forward levels holding at least one L block
  std::vector<int> lev_lower, lev_upper, color;
  int ncolor = 0;
  double bytes = 0.0;

  void build(const IluHost &h) {
    upload(f_rows, h.f_rows);
    upload(f_ptr, h.f_ptr);
    upload(f_col, h.f_col);
    upload(b_rows, h.b_rows);
    upload(b_ptr, h.b_ptr);
    upload(b_col, h.b_col);
    std::vector<T> fv(h.f_val.begin(), h.f_val.end()), bv(h.b_val.begin(), h.b_val.end()),
        dv(h.dinv.begin(), h.dinv.end());
    upload(f_val, fv);
    upload(b_val, bv);
    upload(dinv, dv);
    f_lev_ptr = h.f_lev_ptr;
    b_lev_ptr = h.b_lev_ptr;
    f_nonempty.assign(f_lev_ptr.size() - 1, 0);
    for (size_t l = 0; l + 1 < f_lev_ptr.size(); l++)
      f_nonempty[l] = h.f_ptr[f_lev_ptr[l + 1]] > h.f_ptr[f_lev_ptr[l]];
    lev_lower = h.lev_lower;
    lev_upper = h.lev_upper;
    color = h.color;
    ncolor = h.ncolor;
    n = h.n;
    nv = h.nv;
    nnzf = int(h.fci.size());
    upload(r_frp, h.frp);
    upload(r_fci, h.fci);
    upload(r_src, h.src);
    upload(r_dpos, h.dpos);
    upload(r_dst, h.dst);
    upload(r_fwd, h.fwd);
    upload(r_order, h.order);
    const double s = sizeof(T), b2 = double(h.nv) * h.nv;
    const double n = h.n;
    bytes = (h.f_col.size() + h.b_col.size()) * (b2 * s + 4) + 2 * 4 * (n + 1) + 2 * 4 * n  // factors
            + n * b2 * s                                                                      // D^-1
            + 4 * n * h.nv * s;                                                               // b1, y, w
  }

  // New factors from new device FP64 values A (BSR, the pattern the factor was
  // built on), on the GPU: the same IKJ factorisation in FP64 as the host's,
  // bit for bit, then rounded to T.  Blocking; throws on a zero pivot.
  void refactor(const double *A, hipStream_t st) {
    if (nv == 3)
      refactor_nv<3>(A, st);
    else if (nv == 4)
      refactor_nv<4>(A, st);
    else
      throw Error{CPTR_ERR_UNSUPPORTED, "refactorisation for nv = 3 or 4 only"};
  }

  template <int NV>
  void refactor_nv(const double *A, hipStream_t st) {
    constexpr int B2 = NV * NV;
    DevMem lu, dv, bad;
    lu.alloc((size_t)nnzf * B2 * sizeof(double));
    dv.alloc((size_t)n * B2 * sizeof(double));
    bad.alloc(sizeof(int));
    hipLaunchKernelGGL((k_fill<int>), dim3(1), dim3(kBlock), 0, st, (int *)bad.p, (size_t)1, 0);
    hipLaunchKernelGGL((k_ilu_load<NV>), dim3(nblk((size_t)nnzf * B2)), dim3(kBlock), 0, st, nnzf,
                       devp<int>(r_src), A, (double *)lu.p);
    LAUNCH_CHECK();
    for (size_t l = 0; l + 1 < f_lev_ptr.size(); l++) {
      const int p0 = f_lev_ptr[l], cnt = f_lev_ptr[l + 1] - p0;
      if (cnt <= 0) continue;
      hipLaunchKernelGGL((k_ilu_factor<NV>), dim3(nblk(cnt)), dim3(kBlock), 0, st, p0, cnt, devp<int>(r_fwd),
                         devp<int>(r_frp), devp<int>(r_fci), devp<int>(r_dpos), (double *)lu.p, (double *)dv.p,
                         (int *)bad.p);
      LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_ilu_store<NV, T>), dim3(nblk(((size_t)nnzf + n) * B2)), dim3(kBlock), 0, st, nnzf, n,
                       devp<int>(r_dst), devp<int>(r_order), (const double *)lu.p, (const double *)dv.p,
                       devp<T>(f_val), devp<T>(b_val), devp<T>(dinv));
    LAUNCH_CHECK();
    int hb = 0;
    CPTR_HIP_TRY(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    CPTR_HIP_TRY(hipStreamSynchronize(st));
    if (hb) throw Error{CPTR_ERR_SINGULAR_BLOCK, "zero pivot in a block ILU diagonal block"};
  }
};

// ---------------------------------------------------------------- learned stage
// Parameters of the learned second stage on the device (cptr_learn_model).
struct LearnModelDev {
  int nv = 0, np = 0;
  DevMem theta, packed, am, av, grad;
  int step = 0;
  static int nin(int nv) { return kHid * nv; }
  static int nl(int nv) { return kHid * nv * nv + 2 * kHid * kHid + kHid; }
  static int count(int nv) { return nin(nv) + 3 * nl(nv) + nv * kHid; }
  static constexpr int kPacked = kHid * kEdge + 4 * kHid * kHid;  // per layer
  const float *W_in() const { return devp<float>(theta); }
  const float *bias(int l) const { return devp<float>(theta) + nin(nv) + l * nl(nv) + kHid * nv * nv + 2 * kHid * kHid; }
  const float *W_out() const { return devp<float>(theta) + nin(nv) + 3 * nl(nv); }
  const short *We16(int l) const { return devp<short>(packed) + (size_t)l * kPacked; }
  const float *We32(int l) const { return devp<float>(theta) + nin(nv) + l * nl(nv); }
  const short *Ws(int l) const { return We16(l) + kHid * kEdge; }
  const short *Wm(int l) const { return Ws(l) + kHid * kHid; }
  const short *WsT(int l) const { return Wm(l) + kHid * kHid; }
  const short *WmT(int l) const { return WsT(l) + kHid * kHid; }
  void pack(hipStream_t st) {
    if (nv == 3)
      hipLaunchKernelGGL((k_lrn_pack<3>), dim3(nblk(3 * kPacked)), dim3(kBlock), 0, st, devp<float>(theta), devp<short>(packed));
    else
      hipLaunchKernelGGL((k_lrn_pack<4>), dim3(nblk(3 * kPacked)), dim3(kBlock), 0, st, devp<float>(theta), devp<short>(packed));
    LAUNCH_CHECK();
  }
};

static inline short host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// Per-launch timing of chosen kernels inside solves (roofline figures): HIP
// events recorded around each launch on its stream, their elapsed times
// summed when the solve has finished.  Ids: 0 the Krylov product w = A z,
// 1..3 the learned stage's inference layers.
struct KTimer {
  static constexpr int kIds = 4;
  bool on = false;
  std::vector<hipEvent_t> pool;                   // reused event pairs
  std::vector<std::pair<int, int>> pending;       // (id, pair index) not yet summed
  double ms[kIds] = {0, 0, 0, 0};
  long long count[kIds] = {0, 0, 0, 0};
  ~KTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  void reset() {
    pending.clear();
    for (int i = 0; i < kIds; i++) ms[i] = 0.0, count[i] = 0;
  }
  int begin(int id, hipStream_t st) {
    const int pair = int(pending.size());
    if (2 * pair + 2 > (int)pool.size())
      for (int q = 0; q < 2; q++) {
        hipEvent_t e;
        CPTR_HIP_TRY(hipEventCreate(&e));
        pool.push_back(e);
      }
    pending.push_back({id, pair});
    CPTR_HIP_TRY(hipEventRecord(pool[2 * pair], st));
    return pair;
  }
  void end(int pair, hipStream_t st) { CPTR_HIP_TRY(hipEventRecord(pool[2 * pair + 1], st)); }
  void collect() {  // after the stream has finished the recorded work
    for (const auto &q : pending) {
      float t = 0.f;
      CPTR_HIP_TRY(hipEventSynchronize(pool[2 * q.second + 1]));
      CPTR_HIP_TRY(hipEventElapsedTime(&t, pool[2 * q.second], pool[2 * q.second + 1]));
      ms[q.first] += t;
      count[q.first]++;
    }
    pending.clear();
  }
};

// times the launches made during its lifetime when the timer is on
struct KTimeScope {
  KTimer *t;
  hipStream_t st;
  int pair = -1;
  KTimeScope(KTimer *t_, int id, hipStream_t st_) : t(t_), st(st_) {
    if (t && t->on) pair = t->begin(id, st);
  }
  ~KTimeScope() {
    if (pair >= 0) (void)hipEventRecord(t->pool[2 * pair + 1], st);
  }
};

// Matrix-dependent data of the learned stage: neighbour table, BF16 edge
// features D_i^{-1} A_{i,nbr(i,d)}, FP32 diagonal-block inverses, transpose
// positions (for A^T in training), and work buffers.
struct LearnedDev {
  int n = 0, nv = 0, nnzb = 0;
  DevMem nbr, nmask, E, Et, dinv, tpos, r, s, spart, hA, hB;  // Et: E in tile order (load_edge_tiled)
  int stride[3] = {0, 0, 0};  // |column - row| of the neighbours along each axis
  // z-column schedule of the inference layers (k_lrn_layer_col): planes of
  // colP whole tiles, colNZ planes; colP = 0 when the grid does not allow it
  int colP = 0, colNZ = 0;
  bool use_col = true;
  bool have_pass = false;     // an inference pass has filled r, s, hA, hB
  KTimer *timer = nullptr;    // the handle's kernel timer
  DevMem H[4], M[3], Aa[3], dh0, dh1, dm, dhown, z2, res, dz, part, mid;
  bool train_ready = false;

  // neighbours: direction d = 2 axis + (offset > 0), axes by increasing |offset|
  void build(int n_, int nv_, const std::vector<int> &rp, const std::vector<int> &ci,
             const std::vector<double> &vals) {
    n = n_;
    nv = nv_;
    nnzb = rp[n];
    std::vector<int> mags;
    for (int i = 0; i < n; i++)
      for (int k = rp[i]; k < rp[i + 1]; k++)
        if (ci[k] != i) mags.push_back(std::abs(ci[k] - i));
    std::sort(mags.begin(), mags.end());
    mags.erase(std::unique(mags.begin(), mags.end()), mags.end());
    if (mags.size() > 3) throw Error{CPTR_ERR_UNSUPPORTED, "the learned stage needs a 7-point cell graph"};
    const int b2 = nv * nv;
    std::vector<int> nb((size_t)n * kDir, -1), tp(nnzb, -1);
    std::vector<double> dv((size_t)n * b2);
    std::vector<float> df((size_t)n * b2);
    std::vector<short> eb((size_t)n * kDir * kEdge, 0);
    for (int i = 0; i < n; i++) {
      int dk = -1;
      for (int k = rp[i]; k < rp[i + 1]; k++) {
        const int j = ci[k];
        if (j == i) { dk = k; continue; }
        const int axis = int(std::lower_bound(mags.begin(), mags.end(), std::abs(j - i)) - mags.begin());
        const int d = 2 * axis + (j > i ? 1 : 0);
        if (nb[(size_t)i * kDir + d] >= 0) throw Error{CPTR_ERR_UNSUPPORTED, "not a 7-point cell graph"};
        nb[(size_t)i * kDir + d] = j;
        tp[k] = int(std::lower_bound(ci.begin() + rp[j], ci.begin() + rp[j + 1], i) - ci.begin());
      }
      tp[dk] = dk;
      // D_i^{-1} by Gauss-Jordan with partial pivoting
      double m[4][8];
      for (int r = 0; r < nv; r++)
        for (int q = 0; q < 2 * nv; q++)
          m[r][q] = q < nv ? vals[(size_t)dk * b2 + r * nv + q] : (q - nv == r ? 1.0 : 0.0);
      for (int c = 0; c < nv; c++) {
        int p = c;
        for (int r = c + 1; r < nv; r++) if (std::fabs(m[r][c]) > std::fabs(m[p][c])) p = r;
        if (m[p][c] == 0.0) throw Error{CPTR_ERR_SINGULAR_BLOCK, "singular diagonal block"};
        if (p != c) for (int q = 0; q < 2 * nv; q++) std::swap(m[c][q], m[p][q]);
        const double d = m[c][c];
        for (int q = 0; q < 2 * nv; q++) m[c][q] /= d;
        for (int r = 0; r < nv; r++) {
          if (r == c) continue;
          const double f = m[r][c];
          for (int q = 0; q < 2 * nv; q++) m[r][q] -= f * m[c][q];
        }
      }
      for (int r = 0; r < nv; r++)
        for (int c = 0; c < nv; c++) {
          dv[(size_t)i * b2 + r * nv + c] = m[r][nv + c];
          df[(size_t)i * b2 + r * nv + c] = float(m[r][nv + c]);
        }
    }
    for (int i = 0; i < n; i++)
      for (int d = 0; d < kDir; d++) {
        const int j = nb[(size_t)i * kDir + d];
        if (j < 0) continue;
        const int k = int(std::lower_bound(ci.begin() + rp[i], ci.begin() + rp[i + 1], j) - ci.begin());
        for (int r = 0; r < nv; r++)
          for (int c = 0; c < nv; c++) {
            double acc = 0.0;
            for (int q = 0; q < nv; q++) acc += dv[(size_t)i * b2 + r * nv + q] * vals[(size_t)k * b2 + q * nv + c];
            eb[((size_t)i * kDir + d) * kEdge + r * nv + c] = host_bf16(float(acc));
          }
      }
    // the neighbour in direction d is i -+ stride[d / 2]: a presence bit per direction
    for (size_t a = 0; a < mags.size(); a++) stride[a] = mags[a];
    colP = colNZ = 0;
    if (mags.size() == 3 && stride[0] == 1 && stride[2] % 16 == 0 && n % stride[2] == 0) {
      colP = stride[2] / 16;
      colNZ = n / stride[2];
    }
    std::vector<unsigned char> mk(n, 0);
    for (int i = 0; i < n; i++)
      for (int d = 0; d < kDir; d++) {
        const int j = nb[(size_t)i * kDir + d];
        if (j < 0) continue;
        if (j != i + (d & 1 ? 1 : -1) * stride[d / 2]) throw Error{CPTR_ERR_UNSUPPORTED, "not a 7-point cell graph"};
        mk[i] |= (unsigned char)(1u << d);
      }
    upload(nbr, nb);
    upload(nmask, mk);
    upload(E, eb);
    // the forward layers read the edge blocks in tile order (load_edge_tiled):
    // for tile t and direction d one run of the 16 cells' entries, groups of
    // four entries 4g .. 4g + 3 of the 16 cells (128 contiguous bytes; for
    // nv = 3 the last group holds entry 8 and three zeros)
    {
      const int nt = (n + 15) / 16;
      const int run = nv == 3 ? kEdgeRun<3> : kEdgeRun<4>;
      std::vector<short> et((size_t)nt * kDir * run, 0);
      for (int i = 0; i < n; i++)
        for (int d = 0; d < kDir; d++) {
          short *r0 = et.data() + ((size_t)(i / 16) * kDir + d) * run;
          for (int e = 0; e < nv * nv; e++)
            r0[(e / 4) * 64 + (i % 16) * 4 + e % 4] = eb[((size_t)i * kDir + d) * kEdge + e];
        }
      upload(Et, et);
    }
    upload(dinv, df);
    upload(tpos, tp);
    r.alloc((size_t)n * nv * 4);
    s.alloc(4 * 4);
    spart.alloc((size_t)(nblk(n) + 1) * 4 * 8);
    // BF16 activations of the inference pass, tile order, padded to whole tiles
    hA.alloc((size_t)((n + 15) / 16) * 16 * kHid * 2);
    hB.alloc((size_t)((n + 15) / 16) * 16 * kHid * 2);
  }

  // New matrix values on the pattern given to build (device BSR rp, ci,
  // vals): the diagonal-block inverses and the edge features recomputed on
  // the GPU as build computes them; errors or-ed into *flag.
  void refresh(hipStream_t st, const int *rp_d, const int *ci_d, const double *vals, int *flag) {
    if (nv == 3)
      hipLaunchKernelGGL((k_rs_learned<3>), dim3(nblk(n)), dim3(kBlock), 0, st, n, rp_d, ci_d, vals,
                         devp<int>(nbr), devp<float>(dinv), devp<short>(E), devp<short>(Et), kEdgeRun<3>, flag);
    else
      hipLaunchKernelGGL((k_rs_learned<4>), dim3(nblk(n)), dim3(kBlock), 0, st, n, rp_d, ci_d, vals,
                         devp<int>(nbr), devp<float>(dinv), devp<short>(E), devp<short>(Et), kEdgeRun<4>, flag);
    LAUNCH_CHECK();
    have_pass = false;
  }

  void ensure_train() {
    if (train_ready) return;
    const size_t hb = (size_t)n * kHid * 4;
    for (auto &x : H) x.alloc(hb);
    for (auto &x : M) x.alloc(hb);
    for (auto &x : Aa) x.alloc(hb);
    dh0.alloc(hb);
    dh1.alloc(hb);
    dm.alloc(hb);
    dhown.alloc(hb);
    z2.alloc((size_t)n * nv * 8);
    res.alloc((size_t)n * nv * 8);
    dz.alloc((size_t)n * nv * 8);
    const size_t p1 = (size_t)bwd_blocks() * 4 * (2 * kHid * kHid + kHid * kEdge + kHid);
    const size_t p2 = (size_t)nblk((size_t)n * kHid) * kHid * 4;
    part.alloc(std::max(p1, p2) * 4);
    mid.alloc((size_t)kSumGroups * (2 * kHid * kHid + kHid * kEdge + kHid) * 4);
    train_ready = true;
  }
  int ntiles() const { return (n + 15) / 16; }
  // mid[b][e] = sum over the rows p = b, b + g, ... of part[p][e]; returns g
  int sum_rows(hipStream_t st, const float *part_rows, int np, int len) {
    const int g = std::max(1, std::min(kSumGroups, np));
    hipLaunchKernelGGL(k_sum_partials_rows, dim3(g), dim3(kBlock), 0, st, part_rows, np, len, devp<float>(mid));
    LAUNCH_CHECK();
    return g;
  }
  // out[e] += sum over the np rows of part[p][e] (fixed order)
  void sum_partials(hipStream_t st, const float *part_rows, int np, int len, float *out) {
    const int g = sum_rows(st, part_rows, np, len);
    hipLaunchKernelGGL(k_sum_partials_cols, dim3(nblk(len)), dim3(kBlock), 0, st, (const float *)devp<float>(mid),
                       g, len, out, 1);
    LAUNCH_CHECK();
  }
  int bwd_blocks() const { return std::max(1, std::min(512, (ntiles() + 3) / 4)); }

  // The network on b1 (type BT), finished by the read-out `out`; with `store`,
  // the intermediate values of the backward pass are kept (training).
  template <int NV, typename BT, typename ZT, typename XT>
  void forward(hipStream_t st, const LearnModelDev &mdl, const BT *b1, bool store, LrnOut<ZT, XT> out) {
    const int nb = nblk(n);
    hipLaunchKernelGGL((k_lrn_input<NV, BT>), dim3(nb), dim3(kBlock), 0, st, n, devp<float>(dinv), b1,
                       devp<float>(r), devp<double>(spart));
    hipLaunchKernelGGL((k_lrn_scale<NV>), dim3(NV), dim3(kBlock), 0, st, (const double *)devp<double>(spart),
                       nb, double(n), devp<float>(s));
    LAUNCH_CHECK();
    for (int l = 0; l < 3; l++) layer<NV, ZT, XT>(st, mdl, l, store, out);
    have_pass = !store;
  }

  // Layer l (0..2) of the network on the current r and s.  Training (`store`):
  // FP32 activations H[l] -> H[l+1], messages and pre-activations kept.
  // Inference: BF16 activations r -> hA -> hB -> read-out, nothing else kept.
  template <int NV, typename ZT, typename XT>
  void layer(hipStream_t st, const LearnModelDev &mdl, int l, bool store, LrnOut<ZT, XT> out) {
    // a multiple of the XCD count, one wave per tile up to kLayerMaxBlocks
    const int lb = kXcds * std::max(1, std::min(kLayerMaxBlocks, (ntiles() + 3) / 4) / kXcds);
    const unsigned char *nbp = devp<unsigned char>(nmask);
    const int3 str = make_int3(stride[0], stride[1], stride[2]);
    const short *Ep = devp<short>(Et);  // tile order
    const float *sp = devp<float>(s), *rp_ = devp<float>(r);
    const LrnOut<float, float> none{nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr};
    const float *We = mdl.We32(l);
    const short *Ws = mdl.Ws(l), *Wm = mdl.Wm(l);
    const float *bs = mdl.bias(l);
    if (store) {
      float *Ml = devp<float>(M[l]), *Al = devp<float>(Aa[l]);
      if (l == 0)
        hipLaunchKernelGGL((k_lrn_layer<NV, true, false, float, float, float>), dim3(lb), dim3(kBlock), 0, st, n,
                           nbp, str, Ep, sp, (const float *)nullptr, rp_, mdl.W_in(), We, Ws, Wm, bs,
                           devp<float>(H[1]), devp<float>(H[0]), Ml, Al, none);
      else if (l == 1)
        hipLaunchKernelGGL((k_lrn_layer<NV, false, false, float, float, float>), dim3(lb), dim3(kBlock), 0, st, n,
                           nbp, str, Ep, sp, (const float *)devp<float>(H[1]), rp_, mdl.W_in(), We, Ws, Wm, bs,
                           devp<float>(H[2]), (float *)nullptr, Ml, Al, none);
      else
        hipLaunchKernelGGL((k_lrn_layer<NV, false, true, float, ZT, XT>), dim3(lb), dim3(kBlock), 0, st, n, nbp,
                           str, Ep, sp, (const float *)devp<float>(H[2]), rp_, mdl.W_in(), We, Ws, Wm, bs,
                           devp<float>(H[3]), (float *)nullptr, Ml, Al, out);
    } else if (use_col && colP > 0 && l > 0) {
      // the layers after the first (whose input rows are nv floats, not 64
      // BF16 channels); about four waves per SIMD, each walking zlen planes
      // of one column
      KTimeScope ts(timer, 1 + l, st);
      const int nchunk = std::max(1, std::min(colNZ, kColWaves / colP));
      const int zlen = (colNZ + nchunk - 1) / nchunk;
      const int items = colP * ((colNZ + zlen - 1) / zlen);
      const int cb = kXcds * std::max(1, (items + 4 * kXcds - 1) / (4 * kXcds));
      short *ha = devp<short>(hA), *hb = devp<short>(hB);
      const int sy = stride[1];
      if (l == 1)
        hipLaunchKernelGGL((k_lrn_layer_col<NV, false, false, short, float, float>), dim3(cb), dim3(kBlock), 0, st,
                           n, colP, colNZ, zlen, sy, Ep, sp, (const short *)ha, rp_, mdl.W_in(), We, Ws, Wm, bs, hb,
                           none);
      else
        hipLaunchKernelGGL((k_lrn_layer_col<NV, false, true, short, ZT, XT>), dim3(cb), dim3(kBlock), 0, st, n,
                           colP, colNZ, zlen, sy, Ep, sp, (const short *)hb, rp_, mdl.W_in(), We, Ws, Wm, bs,
                           (short *)nullptr, out);
    } else {
      KTimeScope ts(timer, 1 + l, st);
      short *ha = devp<short>(hA), *hb = devp<short>(hB);
      if (l == 0) {
        if constexpr (NV == 3)  // held to three waves per SIMD (it would spill at NV = 4)
          hipLaunchKernelGGL((k_lrn_layer_first<NV, true, false, short, float, float>), dim3(lb), dim3(kBlock), 0,
                             st, n, nbp, str, Ep, sp, (const short *)nullptr, rp_, mdl.W_in(), We, Ws, Wm, bs, ha,
                             (float *)nullptr, (float *)nullptr, (float *)nullptr, none);
        else
          hipLaunchKernelGGL((k_lrn_layer<NV, true, false, short, float, float>), dim3(lb), dim3(kBlock), 0, st, n,
                             nbp, str, Ep, sp, (const short *)nullptr, rp_, mdl.W_in(), We, Ws, Wm, bs, ha,
                             (float *)nullptr, (float *)nullptr, (float *)nullptr, none);
      } else if (l == 1)
        hipLaunchKernelGGL((k_lrn_layer<NV, false, false, short, float, float>), dim3(lb), dim3(kBlock), 0, st, n,
                           nbp, str, Ep, sp, (const short *)ha, rp_, mdl.W_in(), We, Ws, Wm, bs, hb,
                           (float *)nullptr, (float *)nullptr, (float *)nullptr, none);
      else
        hipLaunchKernelGGL((k_lrn_layer<NV, false, true, short, ZT, XT>), dim3(lb), dim3(kBlock), 0, st, n, nbp,
                           str, Ep, sp, (const short *)hb, rp_, mdl.W_in(), We, Ws, Wm, bs, (short *)nullptr,
                           (float *)nullptr, (float *)nullptr, (float *)nullptr, out);
    }
    LAUNCH_CHECK();
  }
  // algorithmic HBM bytes of one inference launch of layer 1 (BF16 activations
  // in and out, the six BF16 nv x nv edge blocks; the presence mask unless the
  // z-column kernel runs, which reads none)
  double layer_bytes() const {
    return (double)n * (2.0 * kHid * 2 + kDir * nv * nv * 2 + (use_col && colP > 0 ? 0 : 1));
  }
};

// ---------------------------------------------------------------- preconditioner
struct PrecondBase {
  virtual ~PrecondBase() = default;
  virtual void apply(hipStream_t st, const ApplySlots *slots, bool z_double) = 0;
  virtual void first_stage(hipStream_t st, const ApplySlots *slots) = 0;
  virtual void stage_residual(hipStream_t st, const ApplySlots *slots, double *out) = 0;
  virtual void vcycle(hipStream_t st, int which, const double *b, double *x) = 0;
  virtual void set_learned(LearnedDev *l, const LearnModelDev *m) = 0;
  virtual bool &fallback_flag() = 0;
  virtual const AmgDev<float> *amgf(int) const { return nullptr; }
  virtual const AmgDev<double> *amgd(int) const { return nullptr; }
};

struct Options {
  cptr_options o;
  int n, nv, nnzb;
};

template <typename T>
struct Precond : PrecondBase {
  Options op;
  const int *rp = nullptr, *ci = nullptr;  // device pattern (caller's)
  DevMem acol;                             // p/T columns of A (nv x 2 per block), sliced layout
  const int *sl_kptr = nullptr, *sl_cols = nullptr;  // slicing of the handle's copy of A
  const double *sl_vals64 = nullptr;  // its FP64 values, when b1 is formed in FP64
  SpOp<T> ApT, ATp;
  AmgDev<T> amg_p, amg_s;
  IluDev<T> ilu;
  DevMem bp, bt, xp, dT, dp, tmp, b1;
  DevMem dcp;  // decoupling weights: CPR D [n][nv-1], CPTR-uAMG D [n][2][nv-2] (empty without)
  DevMem vtmp, ztmp;  // FP64 staging of cptr_vcycle
  bool have_s = false, have_ilu = false;
  double bytes = 0.0;
  LearnedDev *lrn = nullptr;             // owned by the handle
  const LearnModelDev *model = nullptr;  // attached model
  bool fell_back = false;                // learned stage replaced by BILU(0)

  void apply_first(hipStream_t st, const ApplySlots *slots) {
    const int n = op.n, fs = op.o.first_stage;
    const int ip = op.o.ip, iT = op.o.iT;
    if (fs == CPTR_FIRST_NONE) return;
    T *bpp = devp<T>(bp), *btt = devp<T>(bt), *xpp = devp<T>(xp), *dTT = devp<T>(dT),
      *dpp = devp<T>(dp), *t = devp<T>(tmp);
    if (fs == CPTR_FIRST_UAMG) btt = bpp + n;  // (b_p; b_T) in unknown-wise order
    hipLaunchKernelGGL((k_restrict_pT<T>), dim3(nblk(n)), dim3(kBlock), 0, st, n, op.nv, ip, iT, slots,
                       dcp.p ? (const T *)devp<T>(dcp) : (const T *)nullptr, fs == CPTR_FIRST_UAMG ? 2 : 1, bpp,
                       fs == CPTR_FIRST_CPR ? (T *)nullptr : btt);
    LAUNCH_CHECK();
    if (fs == CPTR_FIRST_UAMG) {  // unknown-based: (d_p; d_T) = V(A_00) (b_p; b_T)
      amg_p.cycle(st, bpp, dpp);
      return;
    }
    if (fs == CPTR_FIRST_CPR) {
      amg_p.cycle(st, bpp, dpp);
      return;
    }
    if (fs == CPTR_FIRST_BD) {  // block-diagonal: d_p = V(A_pp) b_p, d_T = V(A_TT) b_T
      amg_p.cycle(st, bpp, dpp);
      amg_s.cycle(st, btt, dTT);
      return;
    }
    if (fs == CPTR_FIRST_BLOCK_UPPER) {  // d_T = V(S~_T) b_T, d_p = V(A_pp) (b_p - A_pT d_T)
      amg_s.cycle(st, btt, dTT);
      ApT.template spmv<2>(st, dTT, bpp, t);
      amg_p.cycle(st, t, dpp);
      return;
    }
    amg_p.cycle(st, bpp, xpp);
    ATp.template spmv<2>(st, xpp, btt, t);
    amg_s.cycle(st, t, dTT);
    if (fs == CPTR_FIRST_BLOCK_LOWER) {
      hipLaunchKernelGGL((k_convert<T, T>), dim3(sgrid(n)), dim3(kBlock), 0, st, xpp, dpp, (size_t)n);
      LAUNCH_CHECK();
      return;
    }
    ApT.template spmv<2>(st, dTT, bpp, t);
    amg_p.cycle(st, t, dpp);
  }

  const T *x1p() const { return op.o.first_stage == CPTR_FIRST_NONE ? nullptr : devp<T>(dp); }
  const T *x1T() const {
    int fs = op.o.first_stage;
    if (fs == CPTR_FIRST_UAMG) return devp<T>(dp) + op.n;
    return (fs == CPTR_FIRST_NONE || fs == CPTR_FIRST_CPR) ? nullptr : devp<T>(dT);
  }

  // a9: the two-stage residual b1 = v - A x1 into b1 (x1 = 0 without a first stage)
  template <int NV>
  void form_b1(hipStream_t st, const ApplySlots *slots) {
    const int n = op.n;
    T *b1p = devp<T>(b1);
    if (sl_vals64)
      hipLaunchKernelGGL((k_resid_pT_sliced64<NV, T>), dim3((n + 63) / 64), dim3(64 * NV), 0, st, n, sl_kptr,
                         sl_cols, sl_vals64, op.o.ip, op.o.iT, slots, x1p() ? x1p() : (const T *)zero_vec(), x1T(),
                         b1p);
    else
      hipLaunchKernelGGL((k_resid_pT_sliced<NV, T>), dim3((n + 63) / 64), dim3(64 * NV), 0, st, n, sl_kptr,
                         sl_cols, devp<T>(acol), slots, x1p() ? x1p() : (const T *)zero_vec(), x1T(), b1p);
    LAUNCH_CHECK();
  }

  // the second stage's input b1 of v (first stage, a9), widened to FP64 into out
  void stage_residual(hipStream_t st, const ApplySlots *slots, double *out) override {
    apply_first(st, slots);
    if (op.nv == 3) form_b1<3>(st, slots);
    else form_b1<4>(st, slots);
    hipLaunchKernelGGL((k_convert<T, double>), dim3(sgrid((size_t)op.n * op.nv)), dim3(kBlock), 0, st,
                       (const T *)devp<T>(b1), out, (size_t)op.n * op.nv);
    LAUNCH_CHECK();
  }

  template <int NV, typename ZT>
  void apply_nv(hipStream_t st, const ApplySlots *slots) {
    const int n = op.n, ss = op.o.second_stage;
    apply_first(st, slots);
    T *b1p = devp<T>(b1);
    // two-stage residual b1 = v - A x1 (x1 = 0 without a first stage)
    if (ss == CPTR_SECOND_NONE) {
      hipLaunchKernelGGL((k_finish<T, ZT>), dim3(nblk((size_t)n * NV)), dim3(kBlock), 0, st, n, NV,
                         op.o.ip, op.o.iT, (const T *)nullptr, x1p(), x1T(), slots);
      LAUNCH_CHECK();
      return;
    }
    form_b1<NV>(st, slots);
    if (ss == CPTR_SECOND_LEARNED && !fell_back) {
      if (!model || !lrn) throw Error{CPTR_ERR_INVALID_ARG, "no learned model attached to this handle"};
      lrn->forward<NV, T, ZT, T>(st, *model, b1p, false,
                                 LrnOut<ZT, T>{model->W_out(), op.o.ip, op.o.iT, x1p(), x1T(), slots, nullptr});
      LAUNCH_CHECK();
      return;
    }
    if (ss == CPTR_SECOND_IDENTITY) {
      hipLaunchKernelGGL((k_finish<T, ZT>), dim3(nblk((size_t)n * NV)), dim3(kBlock), 0, st, n, NV,
                         op.o.ip, op.o.iT, (const T *)b1p, x1p(), x1T(), slots);
      LAUNCH_CHECK();
      return;
    }
    if (op.o.ilu_accum_fp64 && sizeof(T) == 4) ilu_solve<NV, ZT, double>(st, slots);
    else ilu_solve<NV, ZT, T>(st, slots);
  }

  // the BILU second stage on b1 (sums of a row accumulated in A): forward
  // sweep level by level (levels without L blocks are no-ops), then the
  // backward sweep, which also writes z = w + x1
  template <int NV, typename ZT, typename A>
  void ilu_solve(hipStream_t st, const ApplySlots *slots) {
    T *b1p = devp<T>(b1);
    for (size_t l = 0; l + 1 < ilu.f_lev_ptr.size(); l++) {
      if (!ilu.f_nonempty[l]) continue;
      int p0 = ilu.f_lev_ptr[l], cnt = ilu.f_lev_ptr[l + 1] - p0;
      hipLaunchKernelGGL((k_ilu_fwd<NV, T, A>), dim3(nblk((size_t)cnt * NV)), dim3(kBlock), 0, st, p0, cnt,
                         devp<int>(ilu.f_rows), devp<int>(ilu.f_ptr), devp<int>(ilu.f_col),
                         devp<T>(ilu.f_val), b1p);
      LAUNCH_CHECK();
    }
    constexpr int rows_per_block = kBlock / NV;
    for (size_t l = 0; l + 1 < ilu.b_lev_ptr.size(); l++) {
      int p0 = ilu.b_lev_ptr[l], cnt = ilu.b_lev_ptr[l + 1] - p0;
      hipLaunchKernelGGL((k_ilu_bwd<NV, T, ZT, A>), dim3(nblk(cnt, rows_per_block)), dim3(kBlock), 0, st,
                         p0, cnt, devp<int>(ilu.b_rows), devp<int>(ilu.b_ptr), devp<int>(ilu.b_col),
                         devp<T>(ilu.b_val), devp<T>(ilu.dinv), b1p, op.o.ip, op.o.iT, x1p(), x1T(),
                         slots);
      LAUNCH_CHECK();
    }
  }

  DevMem zeros;
  const T *zero_vec() {
    return devp<T>(zeros);
  }

  void apply(hipStream_t st, const ApplySlots *slots, bool z_double) override {
    if (op.nv == 3) {
      if (z_double) apply_nv<3, double>(st, slots);
      else apply_nv<3, T>(st, slots);
    } else {
      if (z_double) apply_nv<4, double>(st, slots);
      else apply_nv<4, T>(st, slots);
    }
  }

  void set_learned(LearnedDev *l, const LearnModelDev *m) override {
    lrn = l;
    model = m;
    fell_back = false;  // a (re)attached model is tried again
  }
  bool &fallback_flag() override { return fell_back; }

  void first_stage(hipStream_t st, const ApplySlots *slots) override {
    apply_first(st, slots);
    const int n = op.n;
    hipLaunchKernelGGL((k_finish<T, double>), dim3(nblk((size_t)n * op.nv)), dim3(kBlock), 0, st, n,
                       op.nv, op.o.ip, op.o.iT, (const T *)nullptr, x1p(), x1T(), slots);
    LAUNCH_CHECK();
  }

  void vcycle(hipStream_t st, int which, const double *b, double *x) override {
    const AmgDev<T> &a = which == 0 ? amg_p : amg_s;
    if (which == 1 && !have_s) throw Error{CPTR_ERR_INVALID_ARG, "no S~_T hierarchy in this handle"};
    const int n = a.lev[0]->n;  // 2n for the coupled unknown-based hierarchy
    T *bb = devp<T>(tmp), *xx = devp<T>(xp);
    hipLaunchKernelGGL((k_convert<double, T>), dim3(sgrid(n)), dim3(kBlock), 0, st, b, bb, (size_t)n);
    a.cycle(st, bb, xx);
    hipLaunchKernelGGL((k_convert<T, double>), dim3(sgrid(n)), dim3(kBlock), 0, st, (const T *)xx, x,
                       (size_t)n);
    LAUNCH_CHECK();
  }
};

// ---------------------------------------------------------------- handle
}  // namespace cptr

struct cptr_handle {
  cptr::Options op;
  const int *rp = nullptr, *ci = nullptr;
  const double *vals = nullptr;
  std::unique_ptr<cptr::PrecondBase> pc;
  cptr::DevMem slots;                 // ApplySlots
  cptr::DevMem sl_kptr, sl_cols, sl_vals;  // sliced copy of A for the FP64 products
  std::vector<int> sl_kptr_host;          // its slice pointers (setup only)
  std::vector<int> st_rp, st_ci;          // pattern of S~_T (numeric re-setup)
  hipStream_t stream = nullptr;       // internal stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_step[2] = {nullptr, nullptr};  // per-step results of FGMRES copied to the host
  cptr_stats stats{};
  // FGMRES workspace
  int m_alloc = 0;
  cptr::DevMem kws;  // Krylov workspace (Kws) for restarts up to m_alloc
  double *pinned = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_m = -1;
  std::unique_ptr<cptr::LearnedDev> lrn;  // learned-stage data of this matrix
  cptr_learn_model *model = nullptr;      // attached model (not owned)
  cptr::DevMem rs_flag, rs_work;          // numeric re-setup on the device: error bits, diag(A_pp)
  cptr::KTimer ktime;                     // cptr_kernel_timing
};

struct cptr_learn_model {
  cptr::LearnModelDev dev;
};

namespace cptr {

// The first stages whose numeric re-setup runs on the GPU; CPTR-uAMG and the
// decoupling operators keep the host re-setup.
static bool resetup_on_device(const cptr_options &o) {
  return o.resetup_device != 0 && o.first_stage != CPTR_FIRST_UAMG && o.decoupling == 0;
}

template <typename T>
static void build_precond(cptr_handle *h, const std::vector<int> &rp, const std::vector<int> &ci,
                          const std::vector<double> &vals, const HostCSR *S,
                          const std::vector<std::vector<int>> *agg_p = nullptr,
                          const std::vector<std::vector<int>> *agg_s = nullptr,
                          IluDev<T> *keep_ilu = nullptr) {
#pragma clang fp contract(off)  // the FP64 setup arithmetic here rounds every operation, as the oracle does
  auto pc = std::make_unique<Precond<T>>();
  Precond<T> &P = *pc;
  const cptr_options &o = h->op.o;
  const int n = h->op.n, nv = h->op.nv, nnzb = h->op.nnzb;
  P.op = h->op;
  P.rp = h->rp;
  P.ci = h->ci;
  const size_t s = sizeof(T);
  // a0: p/T columns of A (in the slicing of the handle's copy of A) and the
  // scalar sub-blocks on the cell graph
  const std::vector<int> &kp = h->sl_kptr_host;
  const int ns = (n + 63) / 64;
  P.sl_kptr = devp<int>(h->sl_kptr);
  P.sl_cols = devp<int>(h->sl_cols);
  // b1 from the FP64 values of the sliced copy (FP64 mode, or on request), else
  // from FP32 copies of the p and T columns
  const bool b1_fp64 = o.resid_fp64 || sizeof(T) == 8;
  if (b1_fp64) P.sl_vals64 = devp<double>(h->sl_vals);
  std::vector<T> acol(b1_fp64 ? 0 : (size_t)kp[ns] * 64 * nv * 2, T(0));
  for (int sl = 0; sl < (b1_fp64 ? 0 : ns); sl++)
    for (int lane = 0; lane < 64; lane++) {
      const int i = sl * 64 + lane;
      if (i >= n) break;
      for (int k = 0; k < rp[i + 1] - rp[i]; k++) {
        const size_t kk = (size_t)kp[sl] + k, blk = (size_t)rp[i] + k;
        for (int r = 0; r < nv; r++) {
          acol[((kk * nv + r) * 2 + 0) * 64 + lane] = T(vals[(blk * nv + r) * nv + o.ip]);
          acol[((kk * nv + r) * 2 + 1) * 64 + lane] = T(vals[(blk * nv + r) * nv + o.iT]);
        }
      }
    }
  if (!b1_fp64) upload(P.acol, acol);
  auto sub = [&](int r, int c) {
    HostCSR a;
    a.nr = a.nc = n;
    a.rp = rp;
    a.ci = ci;
    a.v.resize(nnzb);
    for (int k = 0; k < nnzb; k++) a.v[k] = vals[((size_t)k * nv + r) * nv + c];
    return a;
  };
  for (DevMem *m : {&P.bt, &P.dT, &P.zeros}) m->alloc(n * s);
  // the unknown-based stage works on (p; T) vectors of 2n
  const size_t nu = o.first_stage == CPTR_FIRST_UAMG ? 2 * (size_t)n : n;
  for (DevMem *m : {&P.bp, &P.xp, &P.dp, &P.tmp}) m->alloc(nu * s);
  P.b1.alloc((size_t)n * nv * s);
  hipLaunchKernelGGL((k_fill<T>), dim3(sgrid(n)), dim3(kBlock), 0, 0, devp<T>(P.zeros), (size_t)n, T(0));
  LAUNCH_CHECK();
  AmgParams prm;
  prm.theta = o.amg_theta;
  prm.max_levels = o.amg_max_levels;
  prm.coarse_size = o.amg_coarse_size;
  prm.seed = o.amg_seed;
  prm.smooth_p = o.amg_smooth_p;
  double bytes = 0.0;
  if (o.first_stage != CPTR_FIRST_NONE) {
    AmgHost hp;
    HostCSR pp = sub(o.ip, o.ip);
    // Decoupling (Section 3.1; extended to pressure-temperature in Section
    // 3.2): D from Quasi-IMPES (diagonal blocks) or True-IMPES (column sums of
    // the block columns); each row d of D_i solves d C_i = a_i for C_i the s-s
    // part and a_i the matching row of the primary-s part.  Primary rows: p
    // (CPR, s = every other slot) or p and T (CPTR-uAMG, s = the rest).
    std::vector<int> pri{o.ip}, sl;
    if (o.first_stage == CPTR_FIRST_UAMG) pri.push_back(o.iT);
    for (int k = 0; k < nv; k++)
      if (std::find(pri.begin(), pri.end(), k) == pri.end()) sl.push_back(k);
    const int npri = int(pri.size()), ns = int(sl.size());
    std::vector<double> D;
    if (o.decoupling != 0) {
      if (ns < 1) throw Error{CPTR_ERR_UNSUPPORTED, "decoupling needs a secondary unknown"};
      std::vector<double> blk((size_t)n * nv * nv, 0.0);
      for (int j = 0; j < n; j++)
        for (int k = rp[j]; k < rp[j + 1]; k++) {
          const int i = ci[k];
          if (o.decoupling == CPTR_DECOUPLE_QI && i != j) continue;
          for (int e = 0; e < nv * nv; e++) blk[(size_t)i * nv * nv + e] += vals[(size_t)k * nv * nv + e];
        }
      D.resize((size_t)n * npri * ns);
      for (int i = 0; i < n; i++) {
        const double *B = &blk[(size_t)i * nv * nv];
        double m[3][5];  // [C_i^T | a_i^T for each primary row], Gauss-Jordan with partial pivoting
        for (int a = 0; a < ns; a++) {
          for (int b = 0; b < ns; b++) m[a][b] = B[sl[b] * nv + sl[a]];
          for (int r = 0; r < npri; r++) m[a][ns + r] = B[pri[r] * nv + sl[a]];
        }
        const int nc = ns + npri;
        for (int c = 0; c < ns; c++) {
          int pr = c;
          for (int r = c + 1; r < ns; r++)
            if (std::fabs(m[r][c]) > std::fabs(m[pr][c])) pr = r;
          if (m[pr][c] == 0.0)
            throw Error{CPTR_ERR_SINGULAR_BLOCK, "singular decoupling block at cell " + std::to_string(i)};
          for (int b = 0; b < nc; b++) std::swap(m[c][b], m[pr][b]);
          for (int r = 0; r < ns; r++) {
            if (r == c) continue;
            const double f = m[r][c] / m[c][c];
            for (int b = c; b < nc; b++) m[r][b] -= f * m[c][b];
          }
        }
        for (int r = 0; r < npri; r++)
          for (int a = 0; a < ns; a++) D[((size_t)i * npri + r) * ns + a] = m[a][ns + r] / m[a][a];
      }
      std::vector<T> Dt(D.begin(), D.end());
      upload(P.dcp, Dt);
      bytes += (double)n * npri * ns * s + 8.0 * n * ns;  // D and v_s in the restriction
    }
    if (o.decoupling != 0 && o.first_stage == CPTR_FIRST_CPR) {
      // S_p = A_pp - D A_sp
      for (int i = 0; i < n; i++)
        for (int k = rp[i]; k < rp[i + 1]; k++)
          for (int a = 0; a < ns; a++)
            pp.v[k] -= D[(size_t)i * ns + a] * vals[((size_t)k * nv + sl[a]) * nv + o.ip];
    }
    AmgParams prm_s = prm;  // the second hierarchy, or the temperature block of the coupled one
    if (o.amg_smooth_p_T >= 0) prm_s.smooth_p = o.amg_smooth_p_T;
    if (o.first_stage == CPTR_FIRST_UAMG) {
      // Section 3.4: A_00 = [A_pp A_pT; A_Tp A_TT] in unknown-wise order, one
      // hierarchy coarsened per unknown
      HostCSR c;
      c.nr = c.nc = 2 * n;
      c.rp.assign(2 * n + 1, 0);
      c.ci.reserve(4 * (size_t)nnzb);
      c.v.reserve(4 * (size_t)nnzb);
      // (with decoupling: S_0 = A_00 - D A_s0, Section 3.2)
      const int pt[2] = {o.ip, o.iT};
      for (int u = 0; u < 2; u++)
        for (int i = 0; i < n; i++) {
          for (int w = 0; w < 2; w++)
            for (int k = rp[i]; k < rp[i + 1]; k++) {
              const double *Bk = &vals[(size_t)k * nv * nv];
              double x = Bk[pt[u] * nv + pt[w]];
              if (!D.empty())
                for (int b = 0; b < ns; b++) x -= D[((size_t)i * 2 + u) * ns + b] * Bk[sl[b] * nv + pt[w]];
              c.ci.push_back(w * n + ci[k]);
              c.v.push_back(x);
            }
          c.rp[u * n + i + 1] = int(c.ci.size());
        }
      uamg_build(c, n, prm, prm_s, hp, agg_p);
    } else {
      amg_build(pp, prm, hp, agg_p);
    }
    const bool plan = resetup_on_device(o);
    P.amg_p.build(hp, o.amg_sweeps, o.scalar_dia != 0, o.amg_smoother, plan);
    if (o.first_stage != CPTR_FIRST_CPR && o.first_stage != CPTR_FIRST_UAMG) {
      // the second hierarchy: S~_T, or A_TT for the block-diagonal stage
      AmgHost hs;
      if (o.first_stage == CPTR_FIRST_BD)
        amg_build(sub(o.iT, o.iT), prm_s, hs, agg_s);
      else
        amg_build(*S, prm_s, hs, agg_s);
      P.amg_s.build(hs, o.amg_sweeps_T > 0 ? o.amg_sweeps_T : o.amg_sweeps, o.scalar_dia != 0, o.amg_smoother,
                    plan);
      P.have_s = true;
      if (o.first_stage != CPTR_FIRST_BD) {
        P.ApT.build(sub(o.ip, o.iT), o.scalar_dia != 0);
        P.ATp.build(sub(o.iT, o.ip), o.scalar_dia != 0);
      }
    }
    int ncyc = o.first_stage == CPTR_FIRST_BLOCK ? 2 : 1;
    bytes += 8.0 * n * 2 + 2.0 * n * s;                         // restriction
    bytes += ncyc * P.amg_p.bytes_per_cycle;
    if (P.have_s) {
      bytes += P.amg_s.bytes_per_cycle;
      if (o.first_stage == CPTR_FIRST_BLOCK || o.first_stage == CPTR_FIRST_BLOCK_LOWER)
        bytes += P.ATp.bytes() + 3.0 * n * s;  // b~_T
      if (o.first_stage == CPTR_FIRST_BLOCK || o.first_stage == CPTR_FIRST_BLOCK_UPPER)
        bytes += P.ApT.bytes() + 3.0 * n * s;  // b~_p
    }
  }
  if (o.second_stage == CPTR_SECOND_LEARNED) {
    h->lrn = std::make_unique<LearnedDev>();
    h->lrn->timer = &h->ktime;
    h->lrn->build(n, nv, rp, ci, vals);
    h->lrn->use_col = o.lrn_columns != 0;
    P.lrn = h->lrn.get();
    // learned stage: r = D^-1 b1 (FP32 diagonal blocks, b1, r), then three
    // layers, each reading the presence mask, the BF16 edge blocks and the
    // BF16 activations of its cells (neighbours' from cache) and writing
    // theirs; the output layer's read-out is counted with z below
    bytes += (double)n * (4.0 * nv * nv + 8.0 * nv) + 3.0 * h->lrn->layer_bytes();
  }
  if (o.second_stage == CPTR_SECOND_BILU0 || o.second_stage == CPTR_SECOND_BILU0_MC ||
      o.second_stage == CPTR_SECOND_LEARNED) {
    if (keep_ilu) {
      // numeric re-setup: the kept order, pattern and schedules, new factors
      // computed on the GPU from the handle's device values
      P.ilu = std::move(*keep_ilu);
      P.ilu.refactor(h->vals, 0);
    } else {
      IluHost ih;
      // the learned stage's fallback is the plain natural-order BILU(0), whole
      const bool lrn = o.second_stage == CPTR_SECOND_LEARNED;
      std::vector<int> part;
      if (!lrn && (o.ilu_part_x > 1 || o.ilu_part_y > 1 || o.ilu_part_z > 1))
        part = grid_parts(n, rp.data(), ci.data(), o.ilu_part_x, o.ilu_part_y, o.ilu_part_z);
      ilu_build(n, nv, rp.data(), ci.data(), vals.data(), o.second_stage == CPTR_SECOND_BILU0_MC, ih,
                lrn ? 0 : o.ilu_level, part.empty() ? nullptr : part.data());
      P.ilu.build(ih);
      h->stats.ilu_levels_lower = int(ih.f_lev_ptr.size()) - 1;
      h->stats.ilu_levels_upper = int(ih.b_lev_ptr.size()) - 1;
      h->stats.ilu_colors = ih.ncolor;
    }
    P.have_ilu = true;
    if (o.second_stage != CPTR_SECOND_LEARNED) bytes += P.ilu.bytes;
  }
  if (o.second_stage != CPTR_SECOND_NONE)  // two-stage residual
    bytes += (double)nnzb * (nv * 2 * s + 4) + 4.0 * (n + 1) + 8.0 * n * nv + 2.0 * n * s + n * nv * s;
  bytes += 8.0 * n * nv;  // z
  P.bytes = bytes;
  h->stats.apply_bytes = bytes;
  for (int w = 0; w < 2; w++) {
    const AmgDev<T> &a = w == 0 ? P.amg_p : P.amg_s;
    h->stats.nlevels[w] = int(a.lev.size());
    for (size_t l = 0; l < a.lev.size() && l < 16; l++) {
      h->stats.level_rows[w][l] = a.lev[l]->n;
      h->stats.level_nnz[w][l] = l + 1 < a.lev.size() ? int(a.lev[l]->A.nnz) : a.nc * a.nc;
    }
  }
  h->pc = std::move(pc);
}

template <typename T>
static const AmgDev<T> *amg_of(const cptr_handle *h, int which);
template <>
const AmgDev<float> *amg_of<float>(const cptr_handle *h, int which) {
  auto *p = dynamic_cast<Precond<float> *>(h->pc.get());
  if (!p) return nullptr;
  return which == 0 ? &p->amg_p : &p->amg_s;
}
template <>
const AmgDev<double> *amg_of<double>(const cptr_handle *h, int which) {
  auto *p = dynamic_cast<Precond<double> *>(h->pc.get());
  if (!p) return nullptr;
  return which == 0 ? &p->amg_p : &p->amg_s;
}

template <typename T>
static const IluDev<T> *ilu_of(const cptr_handle *h) {
  auto *p = dynamic_cast<Precond<T> *>(h->pc.get());
  return (p && p->have_ilu) ? &p->ilu : nullptr;
}

// sliced copy of A (layout at k_bsr_spmv_sliced)
static void build_sliced(cptr_handle *h, const std::vector<int> &rp, const std::vector<int> &ci,
                         const std::vector<double> &vals) {
  const int n = h->op.n, nv = h->op.nv, b2 = nv * nv;
  const int ns = (n + 63) / 64;
  std::vector<int> kptr(ns + 1, 0);
  for (int s = 0; s < ns; s++) {
    int K = 0;
    for (int i = s * 64; i < std::min(n, s * 64 + 64); i++) K = std::max(K, rp[i + 1] - rp[i]);
    kptr[s + 1] = kptr[s] + K;
  }
  const size_t nk = (size_t)kptr[ns];
  std::vector<int> cols(nk * 64);
  std::vector<double> sv(nk * b2 * 64, 0.0);
  for (int s = 0; s < ns; s++)
    for (int lane = 0; lane < 64; lane++) {
      const int i = s * 64 + lane;
      for (int k = 0; k < kptr[s + 1] - kptr[s]; k++) {
        const size_t kk = (size_t)kptr[s] + k;
        const bool real = i < n && k < rp[i + 1] - rp[i];
        cols[kk * 64 + lane] = real ? ci[rp[i] + k] : (i < n ? i : 0);
        if (!real) continue;
        const double *blk = vals.data() + (size_t)(rp[i] + k) * b2;
        for (int q = 0; q < b2; q++) sv[(kk * b2 + q) * 64 + lane] = blk[q];
      }
    }
  upload(h->sl_kptr, kptr);
  upload(h->sl_cols, cols);
  upload(h->sl_vals, sv);
  h->sl_kptr_host = std::move(kptr);
}

static void validate_and_fetch(const cptr_bsr *A, const cptr_csr *S, const cptr_options &o,
                               std::vector<int> &rp, std::vector<int> &ci, std::vector<double> &vals,
                               HostCSR &sh) {
  const int n = A->n, nv = A->nv, nnzb = A->nnzb;
  if (n <= 0 || nnzb <= 0 || !A->row_ptr || !A->col_idx || !A->vals)
    throw Error{CPTR_ERR_INVALID_ARG, "empty or null BSR matrix"};
  if (nv != 3 && nv != 4) throw Error{CPTR_ERR_UNSUPPORTED, "nv must be 3 or 4"};
  if (o.ip < 0 || o.ip >= nv || o.iT < 0 || o.iT >= nv || o.ip == o.iT)
    throw Error{CPTR_ERR_INVALID_ARG, "invalid p/T slots"};
  if (o.amg_max_levels < 1 || o.amg_coarse_size < 1 || o.amg_sweeps < 1 || o.amg_sweeps_T < 0 ||
      !(o.amg_theta >= 0.0))
    throw Error{CPTR_ERR_INVALID_ARG, "invalid AMG options"};
  if (o.first_stage < 0 || o.first_stage > 6) throw Error{CPTR_ERR_INVALID_ARG, "invalid first stage"};
  if (o.decoupling < 0 || o.decoupling > 2) throw Error{CPTR_ERR_INVALID_ARG, "invalid decoupling"};
  if (o.ilu_level != 0 && o.ilu_level != 1) throw Error{CPTR_ERR_UNSUPPORTED, "ilu_level must be 0 or 1"};
  if (o.ilu_part_x < 1 || o.ilu_part_y < 1 || o.ilu_part_z < 1)
    throw Error{CPTR_ERR_INVALID_ARG, "ILU parts per axis must be at least 1"};
  if (o.schur < CPTR_SCHUR_ASSEMBLED || o.schur > CPTR_SCHUR_DIAG) throw Error{CPTR_ERR_INVALID_ARG, "invalid schur"};
  if (o.amg_smoother != CPTR_SMOOTHER_L1JACOBI && o.amg_smoother != CPTR_SMOOTHER_GS)
    throw Error{CPTR_ERR_INVALID_ARG, "invalid amg_smoother"};
  if (o.decoupling != 0 && o.first_stage != CPTR_FIRST_CPR && o.first_stage != CPTR_FIRST_UAMG)
    throw Error{CPTR_ERR_UNSUPPORTED, "decoupling operators apply to the CPR and CPTR-uAMG first stages only"};
  if (o.second_stage < 0 || o.second_stage > 4)
    throw Error{CPTR_ERR_UNSUPPORTED, "unsupported second stage"};
  if (o.precision != CPTR_FP32 && o.precision != CPTR_FP64)
    throw Error{CPTR_ERR_INVALID_ARG, "invalid precision"};
  rp.resize(n + 1);
  ci.resize(nnzb);
  vals.resize((size_t)nnzb * nv * nv);
  CPTR_HIP_TRY(hipMemcpy(rp.data(), A->row_ptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  CPTR_HIP_TRY(hipMemcpy(ci.data(), A->col_idx, sizeof(int) * nnzb, hipMemcpyDeviceToHost));
  CPTR_HIP_TRY(hipMemcpy(vals.data(), A->vals, sizeof(double) * vals.size(), hipMemcpyDeviceToHost));
  if (rp[0] != 0 || rp[n] != nnzb) throw Error{CPTR_ERR_INVALID_ARG, "row_ptr does not span nnzb"};
  std::vector<std::pair<int, int>> edges;
  for (int i = 0; i < n; i++) {
    if (rp[i + 1] < rp[i]) throw Error{CPTR_ERR_INVALID_ARG, "row_ptr not monotone"};
    bool diag = false;
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      if (ci[k] < 0 || ci[k] >= n) throw Error{CPTR_ERR_INVALID_ARG, "column index out of range"};
      if (k > rp[i] && ci[k] <= ci[k - 1])
        throw Error{CPTR_ERR_INVALID_ARG, "columns not strictly ascending"};
      diag |= ci[k] == i;
    }
    if (!diag) throw Error{CPTR_ERR_INVALID_ARG, "missing diagonal block in row " + std::to_string(i)};
  }
  // structural symmetry
  for (int i = 0; i < n; i++)
    for (int k = rp[i]; k < rp[i + 1]; k++) {
      int j = ci[k];
      if (!std::binary_search(ci.begin() + rp[j], ci.begin() + rp[j + 1], i))
        throw Error{CPTR_ERR_INVALID_ARG, "pattern is not structurally symmetric"};
    }
  for (double v : vals)
    if (!std::isfinite(v)) throw Error{CPTR_ERR_NONFINITE, "non-finite value in A"};
  const bool need_s = o.first_stage == CPTR_FIRST_BLOCK || o.first_stage == CPTR_FIRST_BLOCK_LOWER ||
                      o.first_stage == CPTR_FIRST_BLOCK_UPPER;
  if (need_s && o.schur != CPTR_SCHUR_ASSEMBLED) {
    // Section 3.3.1's algebraic approximations, formed from A
    sh = schur_algebraic(n, nv, o.ip, o.iT, rp.data(), ci.data(), vals.data(), o.schur == CPTR_SCHUR_DIAG);
  } else if (need_s) {
    if (!S || S->n != n || S->nnz <= 0 || !S->row_ptr || !S->col_idx || !S->vals)
      throw Error{CPTR_ERR_INVALID_ARG, "the block first stage needs S~_T on the cell graph"};
    sh.nr = sh.nc = n;
    sh.rp.resize(n + 1);
    sh.ci.resize(S->nnz);
    sh.v.resize(S->nnz);
    CPTR_HIP_TRY(hipMemcpy(sh.rp.data(), S->row_ptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    CPTR_HIP_TRY(hipMemcpy(sh.ci.data(), S->col_idx, sizeof(int) * S->nnz, hipMemcpyDeviceToHost));
    CPTR_HIP_TRY(hipMemcpy(sh.v.data(), S->vals, sizeof(double) * S->nnz, hipMemcpyDeviceToHost));
    if (sh.rp[0] != 0 || sh.rp[n] != S->nnz) throw Error{CPTR_ERR_INVALID_ARG, "S~_T row_ptr"};
    for (int i = 0; i < n; i++) {
      if (sh.rp[i + 1] < sh.rp[i]) throw Error{CPTR_ERR_INVALID_ARG, "S~_T row_ptr not monotone"};
      for (int k = sh.rp[i]; k < sh.rp[i + 1]; k++) {
        if (sh.ci[k] < 0 || sh.ci[k] >= n) throw Error{CPTR_ERR_INVALID_ARG, "S~_T column out of range"};
        if (k > sh.rp[i] && sh.ci[k] <= sh.ci[k - 1])
          throw Error{CPTR_ERR_INVALID_ARG, "S~_T columns not strictly ascending"};
      }
    }
    for (double v : sh.v)
      if (!std::isfinite(v)) throw Error{CPTR_ERR_NONFINITE, "non-finite value in S~_T"};
  }
}

static int fail(const Error &e) {
  set_last_error(e.msg);
  return e.code;
}

// ---------------------------------------------------------------- FGMRES
template <int NV, typename ZT>
static void launch_spmv(cptr_handle *h, hipStream_t st, const ZT *x, const ApplySlots *sl,
                        const double *b, double *y) {
  const int n = h->op.n;
  const dim3 grid((n + 63) / 64), block(64 * NV);
  const int *kp = devp<int>(h->sl_kptr), *cl = devp<int>(h->sl_cols);
  const double *va = devp<double>(h->sl_vals);
  if (b)
    hipLaunchKernelGGL((k_bsr_spmv_sliced<NV, ZT, true>), grid, block, 0, st, n, kp, cl, va, x, sl, b, y);
  else
    hipLaunchKernelGGL((k_bsr_spmv_sliced<NV, ZT, false>), grid, block, 0, st, n, kp, cl, va, x, sl,
                       (const double *)nullptr, y);
  LAUNCH_CHECK();
}

// y = A x, or y = b - A x when b is given
template <typename ZT>
static void spmv(cptr_handle *h, hipStream_t st, const ZT *x, const double *b, double *y) {
  if (h->op.nv == 3) launch_spmv<3, ZT>(h, st, x, nullptr, b, y);
  else launch_spmv<4, ZT>(h, st, x, nullptr, b, y);
}

// y = A z with z read from the slots
template <typename ZT>
static void spmv_slot(cptr_handle *h, hipStream_t st, const ApplySlots *sl, double *y) {
  if (h->op.nv == 3) launch_spmv<3, ZT>(h, st, nullptr, sl, nullptr, y);
  else launch_spmv<4, ZT>(h, st, nullptr, sl, nullptr, y);
}

// Krylov workspace of one solve: the handle's own (allocated on first use and
// kept) or carved from the library's static device array (fgmres_solve_static)
struct Kws {
  double *V = nullptr;  // (m+1) x N basis
  void *Z = nullptr;    // m x N preconditioned vectors (FP32 or FP64)
  double *w = nullptr, *r = nullptr, *part = nullptr, *h1 = nullptr, *h2 = nullptr, *R = nullptr, *cs = nullptr,
         *sn = nullptr, *g = nullptr, *y = nullptr, *scal = nullptr;
  KState *ks = nullptr;
  double *host = nullptr;  // 4 doubles of host memory the per-step results are copied to
  bool graphs = false;     // the Arnoldi step may be replayed from the handle's captured graph
};

// bytes of each piece of the workspace for restart m and N unknowns, in the
// order they are laid out; each piece starts on a 256-byte boundary
static size_t kws_layout(size_t N, int m, size_t zb, size_t *sizes) {
  const size_t s[] = {(m + 1) * N * 8,         // V
                      m * N * zb,              // Z
                      N * 8,                   // w
                      N * 8,                   // r
                      (size_t)kDotBlocks * (kMaxRestart + 1) * 8,  // part: rows of partial sums
                      72 * 8,                  // h1
                      72 * 8,                  // h2
                      (size_t)(m + 1) * m * 8,  // R
                      (size_t)m * 8,           // cs
                      (size_t)m * 8,           // sn
                      (size_t)(m + 1) * 8,     // g
                      (size_t)m * 8,           // y
                      8 * 8,                   // scal
                      sizeof(KState)};         // ks
  size_t total = 0;
  for (int i = 0; i < 14; i++) {
    if (sizes) sizes[i] = s[i];
    total += (s[i] + 255) / 256 * 256;
  }
  return total;
}

static Kws kws_carve(char *base, size_t N, int m, size_t zb) {
  size_t sz[14];
  kws_layout(N, m, zb, sz);
  char *p[14];
  size_t off = 0;
  for (int i = 0; i < 14; i++) {
    p[i] = base + off;
    off += (sz[i] + 255) / 256 * 256;
  }
  Kws k;
  k.V = (double *)p[0];
  k.Z = p[1];
  k.w = (double *)p[2];
  k.r = (double *)p[3];
  k.part = (double *)p[4];
  k.h1 = (double *)p[5];
  k.h2 = (double *)p[6];
  k.R = (double *)p[7];
  k.cs = (double *)p[8];
  k.sn = (double *)p[9];
  k.g = (double *)p[10];
  k.y = (double *)p[11];
  k.scal = (double *)p[12];
  k.ks = (KState *)p[13];
  return k;
}

static void ensure_krylov(cptr_handle *h, int m) {
  if (h->m_alloc >= m) return;
  const size_t N = (size_t)h->op.n * h->op.nv;
  const size_t zb = h->op.o.precision == CPTR_FP32 ? 4 : 8;
  h->kws.alloc(kws_layout(N, m, zb, nullptr));
  if (!h->pinned) CPTR_HIP_TRY(hipHostMalloc((void **)&h->pinned, 8 * sizeof(double), hipHostMallocDefault));
  h->m_alloc = m;
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    h->graph_m = -1;
  }
}

// the handle's workspace (ensure_krylov(h, m) first)
static Kws kws_of(cptr_handle *h) {
  const size_t N = (size_t)h->op.n * h->op.nv;
  const size_t zb = h->op.o.precision == CPTR_FP32 ? 4 : 8;
  Kws k = kws_carve((char *)h->kws.p, N, h->m_alloc, zb);
  k.host = h->pinned;
  k.graphs = true;
  return k;
}

// ||x||_2 into scal[slot] (device)
static void norm2(const Kws &k, hipStream_t st, const double *x, size_t N, int slot) {
  const int g = sgrid(N);
  hipLaunchKernelGGL(k_norm2_partial, dim3(g), dim3(kBlock), 0, st, x, N, k.part);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, (const double *)k.part, g, (const int *)nullptr, 1,
                     k.scal + slot, 1, (const double *)nullptr);
  LAUNCH_CHECK();
}

static double fetch(const Kws &k, hipStream_t st, const double *dev) {
  CPTR_HIP_TRY(hipMemcpyAsync(k.host, dev, sizeof(double), hipMemcpyDeviceToHost, st));
  CPTR_HIP_TRY(hipStreamSynchronize(st));
  return k.host[0];
}

// one Arnoldi step for column j (read from the device state)
template <typename ZT, int MAXK>
static void arnoldi_step(cptr_handle *h, const Kws &k, hipStream_t st) {
  const size_t N = (size_t)h->op.n * h->op.nv;
  KState *ks = k.ks;
  ApplySlots *sl = devp<ApplySlots>(h->slots);
  const int g = sgrid(N);
  hipLaunchKernelGGL(k_set_slots_krylov, dim3(1), dim3(64), 0, st, sl, (const double *)k.V, k.Z, N, (int)sizeof(ZT),
                     (const KState *)ks);
  LAUNCH_CHECK();
  h->pc->apply(st, sl, sizeof(ZT) == 8);
  // w = A z_j (the column address is read from the slots)
  {
    KTimeScope ts(&h->ktime, 0, st);
    spmv_slot<ZT>(h, st, sl, k.w);
  }
  // CGS2 in two passes over the basis (k_mdot_fix): pass 1 finishes column j
  // (the second projection and normalisation left by step j - 1) and forms
  // h1 = V^T w and ||w||^2 (h1[j+1]); pass 2 forms w' = w - V h1, h2 = V^T w',
  // ||w'||^2 (h2[j+1]) and leaves w' / ||w|| as column j + 1; the rotation
  // step takes hn = ||w' - V h2|| from the norms
  const int *jd = &ks->j;
  double *w2_part = k.part + (size_t)kMaxRestart * kDotBlocks;  // the row after the longest basis
  hipLaunchKernelGGL((k_mdot_fix<MAXK>), dim3(g), dim3(kBlock), 0, st, k.V, N, (const KState *)ks,
                     (const double *)k.h2, (const double *)k.h1, (const double *)k.w, k.part, w2_part);
  hipLaunchKernelGGL(k_reduce, dim3(MAXK + 1), dim3(kBlock), 0, st, (const double *)k.part, g, jd, 0, k.h1, 0,
                     (const double *)w2_part);
  hipLaunchKernelGGL((k_cgs_update_mdot<MAXK>), dim3(g), dim3(kBlock), 0, st, k.V, N, jd, (const double *)k.h1,
                     (const double *)k.w, k.part, w2_part);
  hipLaunchKernelGGL(k_reduce, dim3(MAXK + 1), dim3(kBlock), 0, st, (const double *)k.part, g, jd, 0, k.h2, 0,
                     (const double *)w2_part);
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, ks, (const double *)k.h1, (const double *)k.h2, k.R, k.cs,
                     k.sn, k.g);
  LAUNCH_CHECK();
}


// switch the learned second stage to its BILU(0) fallback; the captured
// Arnoldi graph holds the learned kernels, so it is rebuilt
static void fall_back(cptr_handle *h, hipStream_t st) {
  CPTR_HIP_TRY(hipStreamSynchronize(st));
  h->pc->fallback_flag() = true;
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
  }
  h->graph_m = -1;
}

// Right-preconditioned FGMRES(m) on the workspace k.  The host reads |g_{j+1}|
// and ||w|| of every step; while the residual estimate is far from the
// tolerance the next step of the cycle is enqueued before that read, so the
// GPU does not wait for the host.  A step enqueued after the one that ends the
// cycle leaves the Krylov state alone (KState::stop) and is not counted.
template <typename ZT>
static int fgmres_impl(cptr_handle *h, const Kws &k, const double *b, double *x, const cptr_solve_opts &so,
                       cptr_solve_info &info, hipStream_t user) {
  auto t0 = std::chrono::steady_clock::now();
  const size_t N = (size_t)h->op.n * h->op.nv;
  const int m = so.restart;
  hipStream_t st = h->stream;
  // order the internal stream after the caller's
  CPTR_HIP_TRY(hipEventRecord(h->ev_in, user));
  CPTR_HIP_TRY(hipStreamWaitEvent(st, h->ev_in, 0));
  KState *ks = k.ks;
  double *scal = k.scal;
  norm2(k, st, b, N, 0);
  const double bnorm = fetch(k, st, scal);
  info = cptr_solve_info{};
  info.fell_back = h->pc->fallback_flag() ? 1 : 0;
  if (!std::isfinite(bnorm)) throw Error{CPTR_ERR_NONFINITE, "non-finite right-hand side"};
  if (!so.nonzero_guess || bnorm == 0.0) {
    hipLaunchKernelGGL((k_fill<double>), dim3(sgrid(N)), dim3(kBlock), 0, st, x, N, 0.0);
    LAUNCH_CHECK();
  }
  if (bnorm == 0.0) {
    info.converged = 1;
    CPTR_HIP_TRY(hipStreamSynchronize(st));
    return CPTR_OK;
  }
  const bool use_graph = k.graphs && h->op.o.use_graph != 0 && !h->ktime.on;  // events are not captured
  auto step = [&]() {
    if (m <= 32) arnoldi_step<ZT, 32>(h, k, st);
    else arnoldi_step<ZT, 64>(h, k, st);
  };
  auto capture = [&]() {
    if (!use_graph || h->graph_m == m) return;
    if (h->graph_exec) {
      (void)hipGraphExecDestroy(h->graph_exec);
      (void)hipGraphDestroy(h->graph);
      h->graph_exec = nullptr;
    }
    CPTR_HIP_TRY(hipStreamSynchronize(st));
    CPTR_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      step();
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(st, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    CPTR_HIP_TRY(hipStreamEndCapture(st, &h->graph));
    CPTR_HIP_TRY(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
    h->graph_m = m;
  };
  // enqueue step q of the cycle and the copy of its (||w||, |g_{q+1}|) into
  // host slot q % 2, marked by event q % 2
  auto launch = [&](int q) {
    if (use_graph) CPTR_HIP_TRY(hipGraphLaunch(h->graph_exec, st));
    else step();
    CPTR_HIP_TRY(hipMemcpyAsync(k.host + 2 * (q & 1), &ks->hn, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    CPTR_HIP_TRY(hipEventRecord(h->ev_step[q & 1], st));
  };
  int iters = 0, cycles = 0, converged = 0;
  double est = 0.0, truer = 0.0;
  for (;;) {
    spmv<double>(h, st, x, b, k.r);
    norm2(k, st, k.r, N, 1);
    const double beta = fetch(k, st, scal + 1);
    truer = beta / bnorm;
    if (!std::isfinite(beta)) throw Error{CPTR_ERR_NONFINITE, "non-finite residual"};
    if (truer <= so.rtol) {
      converged = 1;
      if (cycles == 0) est = truer;
      break;
    }
    if (iters >= so.maxit) break;
    capture();
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, st, ks, (const double *)(scal + 1), k.g, m,
                       so.rtol * bnorm);
    hipLaunchKernelGGL(k_first_vector, dim3(sgrid(N)), dim3(kBlock), 0, st, k.V, N, (const double *)k.r,
                       (const double *)(scal + 1));
    LAUNCH_CHECK();
    int done = 0, next = 0;  // steps of this cycle read back / enqueued
    double prev = truer, rate = 1.0;
    bool discard = false;
    launch(next++);
    while (true) {
      // one step ahead when the step being read is not expected to reach the
      // tolerance (its estimate predicted from the last reduction rate)
      if (next == done + 1 && next < m && iters + (next - done) < so.maxit && prev * rate > 1.5 * so.rtol)
        launch(next++);
      CPTR_HIP_TRY(hipEventSynchronize(h->ev_step[done & 1]));
      const double hn = k.host[2 * (done & 1)], absg = k.host[2 * (done & 1) + 1];
      done++;
      iters++;
      h->stats.applies++;
      est = absg / bnorm;
      if (!std::isfinite(est)) {
        // a non-finite learned-stage output: continue with the BILU(0) fallback
        // from the current iterate (this cycle's basis is discarded)
        if (h->op.o.second_stage == CPTR_SECOND_LEARNED && h->op.o.lrn_fallback && !h->pc->fallback_flag()) {
          fall_back(h, st);
          info.fell_back = 1;
          discard = true;
          break;
        }
        CPTR_HIP_TRY(hipStreamSynchronize(st));
        throw Error{CPTR_ERR_NONFINITE, "non-finite Arnoldi step"};
      }
      if (est <= so.rtol || hn == 0.0 || done == m || iters >= so.maxit) break;
      rate = std::min(1.0, est / prev);
      prev = est;
      if (next == done) launch(next++);
    }
    if (discard) continue;
    hipLaunchKernelGGL(k_solve_y, dim3(1), dim3(64), 0, st, (const KState *)ks, (const double *)k.R,
                       (const double *)k.g, k.y);
    hipLaunchKernelGGL((k_update_x<ZT>), dim3(sgrid(N)), dim3(kBlock), 0, st, x, (const ZT *)k.Z, N,
                       (const KState *)ks, (const double *)k.y);
    LAUNCH_CHECK();
    cycles++;
    // stagnation of the learned stage over a whole cycle: fall back as well
    if (h->op.o.second_stage == CPTR_SECOND_LEARNED && h->op.o.lrn_fallback && !h->pc->fallback_flag() &&
        done == m) {
      spmv<double>(h, st, x, b, k.r);
      norm2(k, st, k.r, N, 1);
      const double after = fetch(k, st, scal + 1) / bnorm;
      if (!(after <= 0.5 * truer)) {
        fall_back(h, st);
        info.fell_back = 1;
      }
    }
  }
  CPTR_HIP_TRY(hipEventRecord(h->ev_out, st));
  CPTR_HIP_TRY(hipStreamWaitEvent(user, h->ev_out, 0));
  CPTR_HIP_TRY(hipStreamSynchronize(st));
  info.iters = iters;
  info.restarts = cycles > 0 ? cycles - 1 : 0;
  info.converged = converged;
  info.relres_est = est;
  info.relres_true = truer;
  info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return converged ? CPTR_OK : CPTR_NOT_CONVERGED;
}

// ---------------------------------------------------------------- learned-stage training
// Mean loss over `count` vectors and the mean gradient accumulated in
// model.grad; every step on the device, the reductions in fixed order.
template <int NV>
static double learn_grad_impl(cptr_handle *h, hipStream_t st, const double *b1_all, int count) {
  LearnedDev &L = *h->lrn;
  LearnModelDev &M = h->model->dev;
  L.ensure_train();
  ensure_krylov(h, 1);
  const Kws kw = kws_of(h);
  const int n = L.n;
  const size_t N = (size_t)n * NV;
  const int np = M.np;
  double *scal = kw.scal;
  float *grad = devp<float>(M.grad);
  float *part = devp<float>(L.part);
  hipLaunchKernelGGL((k_fill<float>), dim3(sgrid(np)), dim3(kBlock), 0, st, grad, (size_t)np, 0.f);
  LAUNCH_CHECK();
  const int nin = LearnModelDev::nin(NV), nl = LearnModelDev::nl(NV);
  double loss = 0.0;
  for (int k = 0; k < count; k++) {
    const double *b1 = b1_all + (size_t)k * N;
    norm2(kw, st, b1, N, 2);
    const double bn = fetch(kw, st, scal + 2);
    if (!(bn > 0.0)) continue;
    const double bb = bn * bn;
    double *z2 = devp<double>(L.z2), *res = devp<double>(L.res), *dz = devp<double>(L.dz);
    L.forward<NV, double, double, double>(st, M, b1, true,
                                          LrnOut<double, double>{M.W_out(), 0, 0, nullptr, nullptr, nullptr, z2});
    spmv<double>(h, st, z2, b1, res);
    norm2(kw, st, res, N, 3);
    const double rn = fetch(kw, st, scal + 3);
    loss += rn * rn / bb;
    hipLaunchKernelGGL((k_bsr_spmv_t<NV>), dim3(nblk(N)), dim3(kBlock), 0, st, n, h->rp, h->ci,
                       (const int *)devp<int>(L.tpos), h->vals, (const double *)res, dz);
    const double scale = -2.0 / bb / count;
    float *dh = devp<float>(L.dh0), *dh_next = devp<float>(L.dh1);
    const int nb64 = nblk((size_t)n * kHid);
    hipLaunchKernelGGL((k_lrn_out_bwd<NV>), dim3(nb64), dim3(kBlock), 0, st, n, (const double *)dz, scale,
                       (const float *)devp<float>(L.s), M.W_out(), (const float *)devp<float>(L.H[3]), dh, part);
    L.sum_partials(st, part, nb64, NV * kHid, grad + nin + 3 * nl);
    LAUNCH_CHECK();
    const int bb1 = L.bwd_blocks(), lb = (L.ntiles() + 3) / 4;
    for (int l = 2; l >= 0; l--) {
      hipLaunchKernelGGL((k_lrn_layer_bwd1<NV>), dim3(bb1), dim3(kBlock), 0, st, n, L.ntiles(),
                         (const int *)devp<int>(L.nbr), (const short *)devp<short>(L.E),
                         (const float *)devp<float>(L.s),
                         (const float *)devp<float>(L.H[l]), (const float *)devp<float>(L.M[l]),
                         (const float *)devp<float>(L.Aa[l]), (const float *)dh, M.WsT(l), M.WmT(l),
                         devp<float>(L.dm), devp<float>(L.dhown), part);
      constexpr int nlay = kHid * NV * NV + 2 * kHid * kHid + kHid;
      constexpr int P = 2 * kHid * kHid + kHid * kEdge + kHid;  // one partial row of bwd1
      const int g = L.sum_rows(st, part, bb1 * (kBlock / 64), P);
      hipLaunchKernelGGL((k_lrn_reduce_layer<NV>), dim3(nblk(nlay)), dim3(kBlock), 0, st,
                         (const float *)devp<float>(L.mid), g, grad + nin + l * nl);
      hipLaunchKernelGGL((k_lrn_layer_bwd2<NV>), dim3(lb), dim3(kBlock), 0, st, n, (const int *)devp<int>(L.nbr),
                         (const short *)devp<short>(L.E), (const float *)devp<float>(L.s), M.We16(l), (const float *)devp<float>(L.dm),
                         (const float *)devp<float>(L.dhown), dh_next);
      LAUNCH_CHECK();
      std::swap(dh, dh_next);
    }
    hipLaunchKernelGGL((k_lrn_in_bwd<NV>), dim3(nb64), dim3(kBlock), 0, st, n, (const float *)dh,
                       (const float *)devp<float>(L.r), (const float *)devp<float>(L.s), part);
    L.sum_partials(st, part, nb64, kHid * NV, grad);
    LAUNCH_CHECK();
  }
  CPTR_HIP_TRY(hipStreamSynchronize(st));
  return loss / count;
}

static double learn_grad(cptr_handle *h, hipStream_t st, const double *b1, int count) {
  return h->op.nv == 3 ? learn_grad_impl<3>(h, st, b1, count) : learn_grad_impl<4>(h, st, b1, count);
}

static void ensure_learned_data(cptr_handle *h) {
  if (h->lrn) return;
  const int n = h->op.n, nv = h->op.nv, nnzb = h->op.nnzb;
  std::vector<int> rp(n + 1), ci(nnzb);
  std::vector<double> vals((size_t)nnzb * nv * nv);
  CPTR_HIP_TRY(hipMemcpy(rp.data(), h->rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  CPTR_HIP_TRY(hipMemcpy(ci.data(), h->ci, sizeof(int) * nnzb, hipMemcpyDeviceToHost));
  CPTR_HIP_TRY(hipMemcpy(vals.data(), h->vals, sizeof(double) * vals.size(), hipMemcpyDeviceToHost));
  h->lrn = std::make_unique<LearnedDev>();
  h->lrn->timer = &h->ktime;
  h->lrn->build(n, nv, rp, ci, vals);
  h->lrn->use_col = h->op.o.lrn_columns != 0;
}

}  // namespace cptr

// Krylov workspace of fgmres_solve_static: one array per GPU, loaded with the
// library's code object and held until the process ends.  Host code uses only
// the device address returned for the current device by scratch_ptr(), never
// the name of the array.
static __device__ __align__(256) unsigned char scratch[CPTR_STATIC_WORKSPACE_BYTES];

namespace cptr {
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up once per device
static void *scratch_ptr() {
  int dev = -1;
  CPTR_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error{CPTR_ERR_UNSUPPORTED, "device index beyond 63"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{CPTR_ERR_HIP, std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace cptr

using namespace cptr;

namespace cptr {

// New values for every part of a preconditioner on its kept patterns, on the
// GPU (resetup_on_device): the p/T columns, the level-0 operators of the AMG
// hierarchies and then all their levels, the p-T couplings of the block
// stages and the block ILU factors.
template <typename T>
static void refresh_precond(cptr_handle *h, Precond<T> &P, const double *A, const double *S, hipStream_t st,
                            int *flag) {
  const cptr_options &o = h->op.o;
  const int n = h->op.n, nv = h->op.nv, nnzb = h->op.nnzb, b2 = nv * nv, fs = o.first_stage;
  if (P.acol.p) {
    hipLaunchKernelGGL((k_rs_pt_cols<T>), dim3(nblk(n)), dim3(kBlock), 0, st, n, nv, o.ip, o.iT, h->rp,
                       devp<int>(h->sl_kptr), A, devp<T>(P.acol));
    LAUNCH_CHECK();
  }
  if (fs != CPTR_FIRST_NONE) {
    if (P.amg_p.num.empty() || (P.have_s && P.amg_s.num.empty()))
      throw Error{CPTR_ERR_SETUP, "no device re-setup plan in this handle"};
    auto &N0 = P.amg_p.num[0];
    hipLaunchKernelGGL(k_rs_strided, dim3(nblk(nnzb)), dim3(kBlock), 0, st, (size_t)nnzb, A, b2, o.ip * nv + o.ip,
                       devp<double>(N0.a_v));
    LAUNCH_CHECK();
    if (P.have_s) {
      auto &S0 = P.amg_s.num[0];
      if (fs == CPTR_FIRST_BD || o.schur == CPTR_SCHUR_ATT) {
        hipLaunchKernelGGL(k_rs_strided, dim3(nblk(nnzb)), dim3(kBlock), 0, st, (size_t)nnzb, A, b2,
                           o.iT * nv + o.iT, devp<double>(S0.a_v));
      } else if (o.schur == CPTR_SCHUR_ASSEMBLED) {
        CPTR_HIP_TRY(hipMemcpyAsync(S0.a_v.p, S, S0.nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        if (h->rs_work.bytes < (size_t)n * 8) h->rs_work.alloc((size_t)n * 8);
        hipLaunchKernelGGL(k_rs_app, dim3(nblk(n)), dim3(kBlock), 0, st, n, nv, o.ip, h->rp, h->ci, A,
                           devp<double>(h->rs_work), flag);
        hipLaunchKernelGGL(k_rs_schur, dim3(nblk(n)), dim3(kBlock), 0, st, n, nv, o.ip, o.iT, h->rp, h->ci, A,
                           (const double *)devp<double>(h->rs_work), devp<int>(S0.a_rp), devp<int>(S0.a_ci),
                           devp<double>(S0.a_v));
      }
      LAUNCH_CHECK();
    }
    P.amg_p.renumeric(st, flag);
    if (P.have_s) P.amg_s.renumeric(st, flag);
    if (P.ApT.nrows) {
      P.ApT.refresh(st, h->rp, h->ci, A, b2, o.ip * nv + o.iT);
      P.ATp.refresh(st, h->rp, h->ci, A, b2, o.iT * nv + o.ip);
    }
  }
  if (P.have_ilu) P.ilu.refactor(A, st);
}

static void update_on_device(cptr_handle *h, const double *A, const double *S, hipStream_t st) {
  const int n = h->op.n, nv = h->op.nv;
  const size_t nval = (size_t)h->op.nnzb * nv * nv;
  if (!h->rs_flag.p) h->rs_flag.alloc(sizeof(int));
  int *flag = devp<int>(h->rs_flag);
  int hf = 0;
  auto read_flag = [&]() {
    CPTR_HIP_TRY(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    CPTR_HIP_TRY(hipStreamSynchronize(st));
  };
  hipLaunchKernelGGL((k_fill<int>), dim3(1), dim3(kBlock), 0, st, flag, (size_t)1, 0);
  hipLaunchKernelGGL(k_rs_finite, dim3(sgrid(nval)), dim3(kBlock), 0, st, nval, A, flag);
  LAUNCH_CHECK();
  read_flag();
  if (hf & kRsNonfinite) throw Error{CPTR_ERR_NONFINITE, "non-finite matrix value"};
  h->vals = A;
  hipLaunchKernelGGL(k_rs_sliced, dim3(nblk(n)), dim3(kBlock), 0, st, n, nv * nv, h->rp, devp<int>(h->sl_kptr), A,
                     devp<double>(h->sl_vals));
  LAUNCH_CHECK();
  if (auto *Pf = dynamic_cast<Precond<float> *>(h->pc.get()))
    refresh_precond(h, *Pf, A, S, st, flag);
  else
    refresh_precond(h, *dynamic_cast<Precond<double> *>(h->pc.get()), A, S, st, flag);
  if (h->lrn) h->lrn->refresh(st, h->rp, h->ci, A, flag);
  read_flag();
  if (hf & kRsSingular)
    throw Error{CPTR_ERR_SINGULAR_BLOCK, "zero diagonal entry of an AMG operator or singular diagonal block"};
  if (hf & kRsCoarse) throw Error{CPTR_ERR_SETUP, "singular coarsest AMG operator"};
}

}  // namespace cptr

// ---------------------------------------------------------------- thermal model
struct cptr_model {
  cptr::ModelView view{};
  int nv = 0, nnzb = 0;
  cptr::DevMem perm, poro, wi, well, rp, ci;     // model data and its 7-point pattern
  cptr::DevMem F, Ft, A, S, xt, dx, rhs, part;   // Newton work arrays
  std::vector<double> part_host;
};

namespace cptr {

static void model_assemble(cptr_model *m, const double *x, const double *xn, double *F, double *A, double *S,
                           hipStream_t st) {
  const int n = m->view.n;
  if (m->nv == 3)
    hipLaunchKernelGGL((k_model_assemble<3>), dim3(nblk(n, 128)), dim3(128), 0, st, m->view, x, xn,
                       devp<int>(m->rp), devp<int>(m->ci), F, A, S);
  else
    hipLaunchKernelGGL((k_model_assemble<4>), dim3(nblk(n, 128)), dim3(128), 0, st, m->view, x, xn,
                       devp<int>(m->rp), devp<int>(m->ci), F, A, S);
  LAUNCH_CHECK();
}

// ||x||_2 of a device vector: block sums of squares in a fixed order, added on the host in block order
static double model_norm(cptr_model *m, const double *x, size_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_model_sumsq, dim3(kModelNormBlocks), dim3(kBlock), 0, st, len, x, devp<double>(m->part));
  LAUNCH_CHECK();
  CPTR_HIP_TRY(hipMemcpyAsync(m->part_host.data(), m->part.p, kModelNormBlocks * sizeof(double),
                              hipMemcpyDeviceToHost, st));
  CPTR_HIP_TRY(hipStreamSynchronize(st));
  double s = 0.0;
  for (double v : m->part_host) s += v;
  return std::sqrt(s);
}

}  // namespace cptr

extern "C" {

void cptr_default_options(cptr_options *o) {
  if (!o) return;
  o->first_stage = CPTR_FIRST_BLOCK;
  o->second_stage = CPTR_SECOND_BILU0_MC;
  o->precision = CPTR_FP32;
  o->ip = 0;
  o->iT = -1;
  o->amg_theta = 0.08;
  o->amg_max_levels = 10;
  o->amg_coarse_size = 512;
  o->amg_seed = 0;
  o->amg_sweeps = 2;
  o->amg_smooth_p = 1;
  o->amg_smooth_p_T = 0;
  o->use_graph = 1;
  o->resid_fp64 = 0;
  o->scalar_dia = 1;
  o->lrn_columns = 1;
  o->schur = CPTR_SCHUR_ASSEMBLED;
  o->lrn_fallback = 1;
  o->amg_smoother = CPTR_SMOOTHER_L1JACOBI;
  o->decoupling = CPTR_DECOUPLE_NONE;
  o->ilu_level = 0;
  o->ilu_part_x = o->ilu_part_y = o->ilu_part_z = 1;
  o->ilu_accum_fp64 = 0;
  o->resetup_device = 1;
  o->amg_sweeps_T = 0;
}

int cptr_setup(cptr_handle **out, const cptr_bsr *A, const cptr_csr *S_T, const cptr_options *opt,
               void *stream) {
  if (!out || !A) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  *out = nullptr;
  cptr_handle *h = nullptr;
  try {
    auto t0 = std::chrono::steady_clock::now();
    cptr_options o;
    if (opt) o = *opt;
    else cptr_default_options(&o);
    if (o.iT < 0) o.iT = A->nv - 1;
    CPTR_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    std::vector<int> rp, ci;
    std::vector<double> vals;
    HostCSR sh;
    validate_and_fetch(A, S_T, o, rp, ci, vals, sh);
    h = new cptr_handle();
    h->op.o = o;
    h->op.n = A->n;
    h->op.nv = A->nv;
    h->op.nnzb = A->nnzb;
    h->rp = A->row_ptr;
    h->ci = A->col_idx;
    h->vals = A->vals;
    CPTR_HIP_TRY(hipStreamCreate(&h->stream));
    CPTR_HIP_TRY(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    CPTR_HIP_TRY(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
    for (auto &e : h->ev_step) CPTR_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->slots.alloc(sizeof(ApplySlots));
    build_sliced(h, rp, ci, vals);
    if (o.precision == CPTR_FP32) build_precond<float>(h, rp, ci, vals, &sh);
    else build_precond<double>(h, rp, ci, vals, &sh);
    h->st_rp = sh.rp;
    h->st_ci = sh.ci;
    const int nv = A->nv;
    h->stats.spmv_bytes = (double)A->nnzb * (nv * nv * 8.0 + 4) + 4.0 * (A->n + 1) + 2.0 * 8 * A->n * nv;
    CPTR_HIP_TRY(hipDeviceSynchronize());
    h->stats.setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return CPTR_OK;
  } catch (const Error &e) {
    delete h;
    return fail(e);
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(Error{CPTR_ERR_OOM, "host allocation failed"});
  } catch (...) {
    delete h;
    return fail(Error{CPTR_ERR_SETUP, "unexpected failure in setup"});
  }
}

static int apply_common(cptr_handle *h, const double *v, void *z, void *stream, int what, int which) {
  if (!h || !v || !z) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if ((const void *)v == z) return fail(Error{CPTR_ERR_INVALID_ARG, "input and output alias"});
  try {
    hipStream_t st = (hipStream_t)stream;
    if (what == 2) {
      h->pc->vcycle(st, which, v, (double *)z);
      return CPTR_OK;
    }
    ApplySlots *sl = devp<ApplySlots>(h->slots);
    hipLaunchKernelGGL(k_set_slots, dim3(1), dim3(64), 0, st, sl, v, z);
    LAUNCH_CHECK();
    if (what == 0) {
      h->pc->apply(st, sl, true);
      h->stats.applies++;
    } else if (what == 3) {
      h->pc->stage_residual(st, sl, (double *)z);
    } else {
      h->pc->first_stage(st, sl);
    }
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  } catch (...) {
    return fail(Error{CPTR_ERR_HIP, "unexpected failure"});
  }
}

int cptr_apply(cptr_handle *h, const double *v, double *z, void *stream) {
  return apply_common(h, v, z, stream, 0, 0);
}

int cptr_first_stage(cptr_handle *h, const double *v, double *x1, void *stream) {
  if (h && h->op.o.first_stage == CPTR_FIRST_NONE) {
    try {
      const size_t N = (size_t)h->op.n * h->op.nv;
      hipLaunchKernelGGL((k_fill<double>), dim3(sgrid(N)), dim3(kBlock), 0, (hipStream_t)stream, x1, N, 0.0);
      LAUNCH_CHECK();
      return CPTR_OK;
    } catch (const Error &e) {
      return fail(e);
    }
  }
  return apply_common(h, v, x1, stream, 1, 0);
}

int cptr_stage_residual(cptr_handle *h, const double *v, double *b1, void *stream) {
  return apply_common(h, v, b1, stream, 3, 0);
}

int cptr_vcycle(cptr_handle *h, int which, const double *b, double *x, void *stream) {
  if (!h) return fail(Error{CPTR_ERR_INVALID_ARG, "null handle"});
  if (which != 0 && which != 1) return fail(Error{CPTR_ERR_INVALID_ARG, "which must be 0 or 1"});
  if (h->op.o.first_stage == CPTR_FIRST_NONE)
    return fail(Error{CPTR_ERR_INVALID_ARG, "no AMG hierarchy in this handle"});
  return apply_common(h, b, x, stream, 2, which);
}

int fgmres_solve(cptr_handle *h, const double *b, double *x, const cptr_solve_opts *so_in,
                 cptr_solve_info *info_out, void *stream) {
  if (!h || !b || !x) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  cptr_solve_opts so{30, 1e-6, 1000, 0};
  if (so_in) so = *so_in;
  if (so.restart < 1 || so.restart > 64) return fail(Error{CPTR_ERR_INVALID_ARG, "restart must be in [1, 64]"});
  if (!(so.rtol > 0.0) || so.maxit < 0) return fail(Error{CPTR_ERR_INVALID_ARG, "invalid tolerance or maxit"});
  cptr_solve_info info{};
  try {
    ensure_krylov(h, so.restart);
    const Kws k = kws_of(h);
    int rc = h->op.o.precision == CPTR_FP32 ? fgmres_impl<float>(h, k, b, x, so, info, (hipStream_t)stream)
                                            : fgmres_impl<double>(h, k, b, x, so, info, (hipStream_t)stream);
    if (h->ktime.on) h->ktime.collect();
    if (info_out) *info_out = info;
    return rc;
  } catch (const Error &e) {
    if (info_out) *info_out = info;
    return fail(e);
  } catch (...) {
    return fail(Error{CPTR_ERR_HIP, "unexpected failure in fgmres_solve"});
  }
}

int cptr_kernel_timing(cptr_handle *h, int enable) {
  if (!h) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  try {
    if (enable) h->ktime.reset();
    else h->ktime.collect();
    h->ktime.on = enable != 0;
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_get_kernel_times(cptr_handle *h, double *avg_us, long long *launches) {
  if (!h) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  try {
    h->ktime.collect();
    for (int i = 0; i < KTimer::kIds; i++) {
      if (avg_us) avg_us[i] = h->ktime.count[i] ? 1e3 * h->ktime.ms[i] / double(h->ktime.count[i]) : 0.0;
      if (launches) launches[i] = h->ktime.count[i];
    }
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int fgmres_solve_static(cptr_handle *h, const double *b, double *x, const cptr_solve_opts *so_in,
                        cptr_solve_info *info_out, void *stream) {
  if (!h || !b || !x) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  cptr_solve_opts so{30, 1e-6, 1000, 0};
  if (so_in) so = *so_in;
  if (so.restart < 1 || so.restart > 64) return fail(Error{CPTR_ERR_INVALID_ARG, "restart must be in [1, 64]"});
  if (!(so.rtol > 0.0) || so.maxit < 0) return fail(Error{CPTR_ERR_INVALID_ARG, "invalid tolerance or maxit"});
  const size_t N = (size_t)h->op.n * h->op.nv;
  const size_t zb = h->op.o.precision == CPTR_FP32 ? 4 : 8;
  const size_t need = kws_layout(N, so.restart, zb, nullptr);
  if (need > CPTR_STATIC_WORKSPACE_BYTES)
    return fail(Error{CPTR_ERR_INVALID_ARG, "the Krylov workspace of " + std::to_string(N) + " unknowns and restart " +
                                                std::to_string(so.restart) + " needs " + std::to_string(need) +
                                                " bytes, more than the static workspace's " +
                                                std::to_string((size_t)CPTR_STATIC_WORKSPACE_BYTES)});
  cptr_solve_info info{};
  try {
    Kws k = kws_carve((char *)scratch_ptr(), N, so.restart, zb);
    double host[4] = {0.0, 0.0, 0.0, 0.0};  // per-step results, copied from the device
    k.host = host;
    k.graphs = false;
    int rc = h->op.o.precision == CPTR_FP32 ? fgmres_impl<float>(h, k, b, x, so, info, (hipStream_t)stream)
                                            : fgmres_impl<double>(h, k, b, x, so, info, (hipStream_t)stream);
    if (info_out) *info_out = info;
    return rc;
  } catch (const Error &e) {
    if (info_out) *info_out = info;
    return fail(e);
  } catch (...) {
    return fail(Error{CPTR_ERR_HIP, "unexpected failure in fgmres_solve_static"});
  }
}

int cptr_matvec(const cptr_handle *h, const double *x, double *y, void *stream) {
  if (!h || !x || !y) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if (x == y) return fail(Error{CPTR_ERR_INVALID_ARG, "input and output alias"});
  try {
    cptr_handle *hh = const_cast<cptr_handle *>(h);
    spmv<double>(hh, (hipStream_t)stream, x, nullptr, y);
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_krylov_vector(const cptr_handle *h, int j, double *out, void *stream) {
  if (!h || !out) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if (h->m_alloc < 1 || j < 0 || j > h->m_alloc)
    return fail(Error{CPTR_ERR_INVALID_ARG, "no Krylov basis of that index"});
  const size_t N = (size_t)h->op.n * h->op.nv;
  const hipError_t e = hipMemcpyAsync(out, (const double *)h->kws.p + (size_t)j * N, N * sizeof(double),
                                      hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return fail(Error{CPTR_ERR_HIP, hipGetErrorString(e)});
  return CPTR_OK;
}

int cptr_update_values(cptr_handle *h, const double *A_vals, const double *S_vals, void *stream) {
  if (!h || !A_vals) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  const int fs = h->op.o.first_stage;
  const bool need_s = fs == CPTR_FIRST_BLOCK || fs == CPTR_FIRST_BLOCK_LOWER || fs == CPTR_FIRST_BLOCK_UPPER;
  const bool two_hier = need_s || fs == CPTR_FIRST_BD;  // a second AMG hierarchy to keep
  const bool caller_s = need_s && h->op.o.schur == CPTR_SCHUR_ASSEMBLED;
  if (caller_s && !S_vals) return fail(Error{CPTR_ERR_INVALID_ARG, "S~_T values required by this first stage"});
  try {
    auto t0 = std::chrono::steady_clock::now();
    CPTR_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    CPTR_HIP_TRY(hipDeviceSynchronize());
    if (resetup_on_device(h->op.o) && h->pc) {
      update_on_device(h, A_vals, S_vals, (hipStream_t)stream);
      if (h->graph_exec) {
        (void)hipGraphExecDestroy(h->graph_exec);
        (void)hipGraphDestroy(h->graph);
        h->graph_exec = nullptr;
        h->graph = nullptr;
      }
      h->graph_m = -1;
      CPTR_HIP_TRY(hipDeviceSynchronize());
      h->stats.setup_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      return CPTR_OK;
    }
    const int n = h->op.n, nv = h->op.nv, nnzb = h->op.nnzb;
    std::vector<int> rp(n + 1), ci(nnzb);
    std::vector<double> vals((size_t)nnzb * nv * nv);
    CPTR_HIP_TRY(hipMemcpy(rp.data(), h->rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    CPTR_HIP_TRY(hipMemcpy(ci.data(), h->ci, sizeof(int) * nnzb, hipMemcpyDeviceToHost));
    CPTR_HIP_TRY(hipMemcpy(vals.data(), A_vals, sizeof(double) * vals.size(), hipMemcpyDeviceToHost));
    for (double v : vals)
      if (!std::isfinite(v)) throw Error{CPTR_ERR_NONFINITE, "non-finite matrix value"};
    HostCSR sh;
    if (need_s && !caller_s) {
      sh = schur_algebraic(n, nv, h->op.o.ip, h->op.o.iT, rp.data(), ci.data(), vals.data(),
                           h->op.o.schur == CPTR_SCHUR_DIAG);
    } else if (need_s) {
      sh.nr = sh.nc = n;
      sh.rp = h->st_rp;
      sh.ci = h->st_ci;
      sh.v.resize(sh.ci.size());
      CPTR_HIP_TRY(hipMemcpy(sh.v.data(), S_vals, sizeof(double) * sh.v.size(), hipMemcpyDeviceToHost));
    }
    // the aggregates of the current hierarchies are kept
    std::vector<std::vector<int>> agg_p, agg_s;
    if (fs != CPTR_FIRST_NONE) {
      const auto *Pf = dynamic_cast<const Precond<float> *>(h->pc.get());
      const auto *Pd = dynamic_cast<const Precond<double> *>(h->pc.get());
      auto strip = [](std::vector<std::vector<int>> a) {
        if (!a.empty()) a.pop_back();  // the coarsest level has no aggregates
        return a;
      };
      agg_p = strip(Pf ? Pf->amg_p.agg : Pd->amg_p.agg);
      if (two_hier) agg_s = strip(Pf ? Pf->amg_s.agg : Pd->amg_s.agg);
    }
    // the block ILU's order, pattern and schedules are kept too: its factors
    // are recomputed on the GPU
    std::unique_ptr<IluDev<float>> ilu_f;
    std::unique_ptr<IluDev<double>> ilu_d;
    if (auto *Pf = dynamic_cast<Precond<float> *>(h->pc.get()); Pf && Pf->have_ilu) {
      ilu_f = std::make_unique<IluDev<float>>(std::move(Pf->ilu));
      Pf->have_ilu = false;
    }
    if (auto *Pd = dynamic_cast<Precond<double> *>(h->pc.get()); Pd && Pd->have_ilu) {
      ilu_d = std::make_unique<IluDev<double>>(std::move(Pd->ilu));
      Pd->have_ilu = false;
    }
    h->vals = A_vals;
    build_sliced(h, rp, ci, vals);
    if (h->op.o.precision == CPTR_FP32)
      build_precond<float>(h, rp, ci, vals, need_s ? &sh : nullptr, &agg_p, two_hier ? &agg_s : nullptr,
                           ilu_f.get());
    else
      build_precond<double>(h, rp, ci, vals, need_s ? &sh : nullptr, &agg_p, two_hier ? &agg_s : nullptr,
                            ilu_d.get());
    // the learned stage's matrix data: build_precond made it anew for a
    // learned second stage; a handle of another second stage that was
    // attached for training keeps its own, rebuilt here from the new values
    if (h->lrn && h->op.o.second_stage != CPTR_SECOND_LEARNED) {
      const bool col = h->lrn->use_col;
      h->lrn->build(n, nv, rp, ci, vals);
      h->lrn->use_col = col;
      h->lrn->have_pass = false;
    }
    if (h->lrn && h->model) h->pc->set_learned(h->lrn.get(), &h->model->dev);
    if (h->graph_exec) {
      (void)hipGraphExecDestroy(h->graph_exec);
      (void)hipGraphDestroy(h->graph);
      h->graph_exec = nullptr;
      h->graph = nullptr;
    }
    h->graph_m = -1;
    CPTR_HIP_TRY(hipDeviceSynchronize());
    h->stats.setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  } catch (const std::bad_alloc &) {
    return fail(Error{CPTR_ERR_OOM, "host allocation failed"});
  } catch (...) {
    return fail(Error{CPTR_ERR_HIP, "unexpected failure"});
  }
}

int cptr_get_stats(const cptr_handle *h, cptr_stats *st) {
  if (!h || !st) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  *st = h->stats;
  return CPTR_OK;
}

int cptr_get_aggregates(const cptr_handle *h, int which, int level, int *agg_host) {
  if (!h || (which != 0 && which != 1)) return fail(Error{CPTR_ERR_INVALID_ARG, "bad argument"});
  const std::vector<std::vector<int>> *agg = nullptr;
  if (auto a = amg_of<float>(h, which)) agg = &a->agg;
  if (auto a = amg_of<double>(h, which)) agg = &a->agg;
  if (!agg || level < 0 || level + 1 >= (int)agg->size())
    return fail(Error{CPTR_ERR_INVALID_ARG, "no such aggregation level"});
  const std::vector<int> &v = (*agg)[level];
  if (agg_host) std::copy(v.begin(), v.end(), agg_host);
  return (int)v.size();
}

int cptr_get_ilu_schedule(const cptr_handle *h, int *ll, int *lu, int *color) {
  if (!h) return fail(Error{CPTR_ERR_INVALID_ARG, "null handle"});
  const std::vector<int> *a = nullptr, *b = nullptr, *c = nullptr;
  if (auto f = ilu_of<float>(h)) { a = &f->lev_lower; b = &f->lev_upper; c = &f->color; }
  if (auto f = ilu_of<double>(h)) { a = &f->lev_lower; b = &f->lev_upper; c = &f->color; }
  if (!a) return fail(Error{CPTR_ERR_INVALID_ARG, "no ILU(0) second stage in this handle"});
  if (ll) std::copy(a->begin(), a->end(), ll);
  if (lu) std::copy(b->begin(), b->end(), lu);
  if (color) std::copy(c->begin(), c->end(), color);
  return CPTR_OK;
}

int cptr_bsr_spmv(int n, int nv, const int *rp, const int *ci, const double *vals, const double *x,
                  double *y, void *stream) {
  if (n < 0 || (nv != 3 && nv != 4) || !rp || !ci || !vals || !x || !y)
    return fail(Error{CPTR_ERR_INVALID_ARG, "bad argument"});
  if (n == 0) return CPTR_OK;
  hipStream_t st = (hipStream_t)stream;
  if (nv == 3)
    hipLaunchKernelGGL((k_bsr_spmv<3, double, false>), dim3(nblk(n, SpmvShape<3>::R)), dim3(SpmvShape<3>::T), 0,
                       st, n, rp, ci, vals, x, (const ApplySlots *)nullptr, (const double *)nullptr, y);
  else
    hipLaunchKernelGGL((k_bsr_spmv<4, double, false>), dim3(nblk(n, SpmvShape<4>::R)), dim3(SpmvShape<4>::T), 0,
                       st, n, rp, ci, vals, x, (const ApplySlots *)nullptr, (const double *)nullptr, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(Error{CPTR_ERR_HIP, hipGetErrorString(e)});
  return CPTR_OK;
}

const char *cptr_status_string(int s) {
  switch (s) {
    case CPTR_OK: return "CPTR_OK";
    case CPTR_NOT_CONVERGED: return "CPTR_NOT_CONVERGED";
    case CPTR_ERR_INVALID_ARG: return "CPTR_ERR_INVALID_ARG";
    case CPTR_ERR_UNSUPPORTED: return "CPTR_ERR_UNSUPPORTED";
    case CPTR_ERR_NONFINITE: return "CPTR_ERR_NONFINITE";
    case CPTR_ERR_SINGULAR_BLOCK: return "CPTR_ERR_SINGULAR_BLOCK";
    case CPTR_ERR_OOM: return "CPTR_ERR_OOM";
    case CPTR_ERR_HIP: return "CPTR_ERR_HIP";
    case CPTR_ERR_SETUP: return "CPTR_ERR_SETUP";
    default: return "unknown status";
  }
}

const char *cptr_last_error(void) { return g_last_error.c_str(); }

void cptr_destroy(cptr_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_out) (void)hipEventDestroy(h->ev_out);
  for (auto e : h->ev_step)
    if (e) (void)hipEventDestroy(e);
  h->pc.reset();
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}


size_t cptr_learn_param_count(int nv) {
  return (nv == 3 || nv == 4) ? (size_t)LearnModelDev::count(nv) : 0;
}

int cptr_learn_create(cptr_learn_model **out, int nv, const float *theta_host) {
  if (!out || !theta_host || (nv != 3 && nv != 4)) return fail(Error{CPTR_ERR_INVALID_ARG, "bad argument"});
  *out = nullptr;
  auto *m = new cptr_learn_model();
  try {
    LearnModelDev &d = m->dev;
    d.nv = nv;
    d.np = LearnModelDev::count(nv);
    d.theta.alloc((size_t)d.np * 4);
    d.grad.alloc((size_t)d.np * 4);
    d.am.alloc((size_t)d.np * 4);
    d.av.alloc((size_t)d.np * 4);
    d.packed.alloc((size_t)3 * LearnModelDev::kPacked * 2);
    CPTR_HIP_TRY(hipMemcpy(d.theta.p, theta_host, (size_t)d.np * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL((k_fill<float>), dim3(sgrid(d.np)), dim3(kBlock), 0, 0, devp<float>(d.am), (size_t)d.np, 0.f);
    hipLaunchKernelGGL((k_fill<float>), dim3(sgrid(d.np)), dim3(kBlock), 0, 0, devp<float>(d.av), (size_t)d.np, 0.f);
    d.pack(0);
    CPTR_HIP_TRY(hipDeviceSynchronize());
    *out = m;
    return CPTR_OK;
  } catch (const Error &e) {
    delete m;
    return fail(e);
  }
}

int cptr_learn_set_params(cptr_learn_model *m, const float *theta_host) {
  if (!m || !theta_host) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  try {
    CPTR_HIP_TRY(hipDeviceSynchronize());
    CPTR_HIP_TRY(hipMemcpy(m->dev.theta.p, theta_host, (size_t)m->dev.np * 4, hipMemcpyHostToDevice));
    // new parameters start a new optimisation: Adam moments and step count reset
    CPTR_HIP_TRY(hipMemset(m->dev.am.p, 0, (size_t)m->dev.np * 4));
    CPTR_HIP_TRY(hipMemset(m->dev.av.p, 0, (size_t)m->dev.np * 4));
    m->dev.step = 0;
    m->dev.pack(0);
    CPTR_HIP_TRY(hipDeviceSynchronize());
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_learn_get_params(const cptr_learn_model *m, float *theta_host) {
  if (!m || !theta_host) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  try {
    CPTR_HIP_TRY(hipDeviceSynchronize());
    CPTR_HIP_TRY(hipMemcpy(theta_host, m->dev.theta.p, (size_t)m->dev.np * 4, hipMemcpyDeviceToHost));
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

void cptr_learn_destroy(cptr_learn_model *m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  delete m;
}

int cptr_learn_attach(cptr_handle *h, cptr_learn_model *m) {
  if (!h || !m) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if (m->dev.nv != h->op.nv) return fail(Error{CPTR_ERR_INVALID_ARG, "model and matrix nv differ"});
  try {
    ensure_learned_data(h);
    h->model = m;
    h->pc->set_learned(h->lrn.get(), &m->dev);
    if (h->graph_exec) {  // a graph captured after a fallback holds the BILU(0) stage
      CPTR_HIP_TRY(hipDeviceSynchronize());
      (void)hipGraphExecDestroy(h->graph_exec);
      (void)hipGraphDestroy(h->graph);
      h->graph_exec = nullptr;
      h->graph = nullptr;
    }
    h->graph_m = -1;
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_learn_forward(cptr_handle *h, const double *b1, double *z2, void *stream) {
  if (!h || !b1 || !z2) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if (!h->model || !h->lrn) return fail(Error{CPTR_ERR_INVALID_ARG, "no learned model attached"});
  try {
    hipStream_t st = (hipStream_t)stream;
    LearnedDev &L = *h->lrn;
    const LearnModelDev &M = h->model->dev;
    const LrnOut<double, double> out{M.W_out(), 0, 0, nullptr, nullptr, nullptr, z2};
    if (L.nv == 3) L.forward<3, double, double, double>(st, M, b1, false, out);
    else L.forward<4, double, double, double>(st, M, b1, false, out);
    LAUNCH_CHECK();
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_learn_rerun_layer(cptr_handle *h, int layer, double *z2, void *stream) {
  if (!h || layer < 0 || layer > 2 || (layer == 2 && !z2))
    return fail(Error{CPTR_ERR_INVALID_ARG, "bad argument"});
  if (!h->model || !h->lrn || !h->lrn->have_pass)
    return fail(Error{CPTR_ERR_INVALID_ARG, "no inference pass of the learned stage to repeat"});
  try {
    hipStream_t st = (hipStream_t)stream;
    LearnedDev &L = *h->lrn;
    const LearnModelDev &M = h->model->dev;
    const LrnOut<double, double> out{M.W_out(), 0, 0, nullptr, nullptr, nullptr, z2};
    if (L.nv == 3) L.layer<3, double, double>(st, M, layer, false, out);
    else L.layer<4, double, double>(st, M, layer, false, out);
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_learn_grad(cptr_handle *h, const double *b1, int count, float *loss_host, float *grad_host,
                    void *stream) {
  if (!h || !b1 || count < 1) return fail(Error{CPTR_ERR_INVALID_ARG, "bad argument"});
  if (!h->model || !h->lrn) return fail(Error{CPTR_ERR_INVALID_ARG, "no learned model attached"});
  try {
    hipStream_t st = (hipStream_t)stream;
    const double loss = learn_grad(h, st, b1, count);
    if (loss_host) *loss_host = float(loss);
    if (grad_host)
      CPTR_HIP_TRY(hipMemcpy(grad_host, h->model->dev.grad.p, (size_t)h->model->dev.np * 4, hipMemcpyDeviceToHost));
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_learn_train_step(cptr_handle *h, const double *b1, int count, float lr, float *loss_host,
                          void *stream) {
  if (!h || !b1 || count < 1 || !(lr > 0.f)) return fail(Error{CPTR_ERR_INVALID_ARG, "bad argument"});
  if (!h->model || !h->lrn) return fail(Error{CPTR_ERR_INVALID_ARG, "no learned model attached"});
  try {
    hipStream_t st = (hipStream_t)stream;
    const double loss = learn_grad(h, st, b1, count);
    LearnModelDev &M = h->model->dev;
    M.step++;
    const float b1c = 0.9f, b2c = 0.999f;
    const float c1 = 1.f - std::pow(b1c, (float)M.step), c2 = 1.f - std::pow(b2c, (float)M.step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(M.np)), dim3(kBlock), 0, st, M.np, devp<float>(M.theta),
                       (const float *)devp<float>(M.grad), devp<float>(M.am), devp<float>(M.av), lr, b1c, b2c,
                       1e-8f, c1, c2);
    LAUNCH_CHECK();
    M.pack(st);
    CPTR_HIP_TRY(hipStreamSynchronize(st));
    if (loss_host) *loss_host = float(loss);
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_model_create(cptr_model **out, const cptr_model_desc *d) {
  if (!out || !d || !d->perm || !d->poro) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  *out = nullptr;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || !(d->dx > 0.0) || !(d->dt > 0.0) ||
      (long long)d->nx * d->ny * d->nz > (1LL << 28))
    return fail(Error{CPTR_ERR_INVALID_ARG, "invalid grid or time step"});
  try {
    auto m = std::make_unique<cptr_model>();
    const int nx = d->nx, ny = d->ny, nz = d->nz, n = nx * ny * nz;
    ModelView &v = m->view;
    v.nx = nx;
    v.ny = ny;
    v.nz = nz;
    v.n = n;
    v.dx = d->dx;
    v.vol = d->dx * d->dx * d->dx;
    v.area = d->dx * d->dx;
    v.dt = d->dt;
    m->nv = d->three_phase ? 4 : 3;
    // c_ref: sum_a S_a c_va of the initial saturations (the oil one eliminated)
    {
      using namespace phys;
      const double sw = 0.1, sg = 0.05;
      v.c_ref = d->three_phase ? 0.0 + sw * CV_WATER + sg * CV_GAS + (1.0 - (sw + sg)) * CV_OIL
                               : 0.0 + sw * CV_WATER + (1.0 - sw) * CV_OIL;
    }
    m->perm.alloc((size_t)n * 8);
    m->poro.alloc((size_t)n * 8);
    CPTR_HIP_TRY(hipMemcpy(m->perm.p, d->perm, (size_t)n * 8, hipMemcpyDeviceToDevice));
    CPTR_HIP_TRY(hipMemcpy(m->poro.p, d->poro, (size_t)n * 8, hipMemcpyDeviceToDevice));
    // Peaceman well index 2 pi K dx / ln(r_o / r_w), r_o = 0.198 dx, r_w = 0.01 m
    std::vector<double> perm_h(n);
    CPTR_HIP_TRY(hipMemcpy(perm_h.data(), d->perm, (size_t)n * 8, hipMemcpyDeviceToHost));
    std::vector<double> wi(n);
    const double lr = std::log(0.198 * d->dx / 0.01);
    for (int i = 0; i < n; i++) wi[i] = 2.0 * M_PI * perm_h[i] * d->dx / lr;
    upload(m->wi, wi);
    std::vector<unsigned char> well(n, 0);
    auto mark = [&](const int *c, int cnt, unsigned bit) {
      if (cnt > 0 && !c) throw Error{CPTR_ERR_INVALID_ARG, "null cell list"};
      for (int q = 0; q < cnt; q++) {
        if (c[q] < 0 || c[q] >= n) throw Error{CPTR_ERR_INVALID_ARG, "well cell out of range"};
        well[c[q]] |= (unsigned char)bit;
      }
    };
    mark(d->inj, d->n_inj, 1u);
    mark(d->prod, d->n_prod, 2u);
    mark(d->heat, d->n_heat, 4u);
    upload(m->well, well);
    // the 7-point pattern, ascending columns
    std::vector<int> rp(n + 1, 0), ci;
    ci.reserve((size_t)7 * n);
    const int nxy = nx * ny;
    for (int i = 0; i < n; i++) {
      const int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
      if (iz > 0) ci.push_back(i - nxy);
      if (iy > 0) ci.push_back(i - nx);
      if (ix > 0) ci.push_back(i - 1);
      ci.push_back(i);
      if (ix < nx - 1) ci.push_back(i + 1);
      if (iy < ny - 1) ci.push_back(i + nx);
      if (iz < nz - 1) ci.push_back(i + nxy);
      rp[i + 1] = int(ci.size());
    }
    m->nnzb = int(ci.size());
    upload(m->rp, rp);
    upload(m->ci, ci);
    v.perm = devp<double>(m->perm);
    v.poro = devp<double>(m->poro);
    v.wi = devp<double>(m->wi);
    v.well = devp<unsigned char>(m->well);
    const size_t N = (size_t)n * m->nv;
    for (DevMem *a : {&m->F, &m->Ft, &m->xt, &m->dx, &m->rhs}) a->alloc(N * 8);
    m->A.alloc((size_t)m->nnzb * m->nv * m->nv * 8);
    m->S.alloc((size_t)m->nnzb * 8);
    m->part.alloc(kModelNormBlocks * 8);
    m->part_host.assign(kModelNormBlocks, 0.0);
    *out = m.release();
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  } catch (const std::bad_alloc &) {
    return fail(Error{CPTR_ERR_OOM, "host allocation failed"});
  } catch (...) {
    return fail(Error{CPTR_ERR_HIP, "unexpected failure"});
  }
}

void cptr_model_destroy(cptr_model *m) { delete m; }

int cptr_model_info(const cptr_model *m, int *nv, int *n, int *nnzb, const int **row_ptr, const int **col_idx) {
  if (!m) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if (nv) *nv = m->nv;
  if (n) *n = m->view.n;
  if (nnzb) *nnzb = m->nnzb;
  if (row_ptr) *row_ptr = devp<int>(m->rp);
  if (col_idx) *col_idx = devp<int>(m->ci);
  return CPTR_OK;
}

int cptr_model_pattern(const cptr_model *m, int *row_ptr_host, int *col_idx_host) {
  if (!m) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  try {
    if (row_ptr_host)
      CPTR_HIP_TRY(hipMemcpy(row_ptr_host, m->rp.p, sizeof(int) * (m->view.n + 1), hipMemcpyDeviceToHost));
    if (col_idx_host) CPTR_HIP_TRY(hipMemcpy(col_idx_host, m->ci.p, sizeof(int) * m->nnzb, hipMemcpyDeviceToHost));
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

int cptr_model_assemble(cptr_model *m, const double *x, const double *xn, double *F, double *A_vals,
                        double *S_vals, void *stream) {
  if (!m || !x || !xn) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  try {
    model_assemble(m, x, xn, F, A_vals, S_vals, (hipStream_t)stream);
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  }
}

void cptr_newton_default_options(cptr_newton_opts *o) {
  if (!o) return;
  o->max_it = 50;
  o->rtol = 1e-8;
  o->stol = 1e-8;
  o->max_backtrack = 10;
  o->lin.restart = 30;
  o->lin.rtol = 1e-6;
  o->lin.maxit = 1000;
  o->lin.nonzero_guess = 0;
}

int cptr_newton_solve(cptr_model *m, cptr_handle *h, double *x, const double *xn, const cptr_newton_opts *o_in,
                      cptr_newton_info *info_out, void *stream) {
  if (!m || !h || !x || !xn) return fail(Error{CPTR_ERR_INVALID_ARG, "null argument"});
  if (h->op.n != m->view.n || h->op.nv != m->nv || h->op.nnzb != m->nnzb)
    return fail(Error{CPTR_ERR_INVALID_ARG, "the handle was not set up on this model's pattern"});
  cptr_newton_opts o;
  cptr_newton_default_options(&o);
  if (o_in) o = *o_in;
  if (o.max_it < 0 || o.max_backtrack < 0 || !(o.rtol >= 0.0) || !(o.stol >= 0.0))
    return fail(Error{CPTR_ERR_INVALID_ARG, "invalid Newton options"});
  o.lin.nonzero_guess = 0;
  cptr_newton_info info{};
  const auto t0 = std::chrono::steady_clock::now();
  try {
    hipStream_t st = (hipStream_t)stream;
    const size_t N = (size_t)m->view.n * m->nv;
    double *F = devp<double>(m->F), *Ft = devp<double>(m->Ft), *xt = devp<double>(m->xt);
    double *dx = devp<double>(m->dx), *rhs = devp<double>(m->rhs);
    model_assemble(m, x, xn, F, nullptr, nullptr, st);
    double f = model_norm(m, F, N, st);
    info.fnorm0 = f;
    if (!std::isfinite(f)) throw Error{CPTR_ERR_NONFINITE, "non-finite residual at the initial state"};
    bool done = f == 0.0;
    while (!done && info.iters < o.max_it) {
      model_assemble(m, x, xn, nullptr, devp<double>(m->A), devp<double>(m->S), st);
      int rc = cptr_update_values(h, devp<double>(m->A), devp<double>(m->S), stream);
      if (rc != CPTR_OK) return rc;
      hipLaunchKernelGGL(k_model_neg, dim3(nblk(N)), dim3(kBlock), 0, st, N, (const double *)F, rhs);
      LAUNCH_CHECK();
      cptr_solve_info li{};
      rc = fgmres_solve(h, rhs, dx, &o.lin, &li, stream);
      if (rc != CPTR_OK) return rc;
      info.lin_iters += li.iters;
      // backtracking line search on ||F*||
      double lambda = 1.0, ft = 0.0;
      bool ok = false;
      for (int bt = 0; bt <= o.max_backtrack; bt++) {
        hipLaunchKernelGGL(k_model_axpy, dim3(nblk(N)), dim3(kBlock), 0, st, N, (const double *)x, lambda,
                           (const double *)dx, xt);
        LAUNCH_CHECK();
        model_assemble(m, xt, xn, Ft, nullptr, nullptr, st);
        ft = model_norm(m, Ft, N, st);
        if (std::isfinite(ft) && ft <= (1.0 - 1e-4 * lambda) * f) {
          ok = true;
          break;
        }
        lambda *= 0.5;
        info.backtracks++;
      }
      info.iters++;
      if (!ok) break;  // line search failure: x stays at the last accepted iterate
      const double step = lambda * model_norm(m, dx, N, st);
      CPTR_HIP_TRY(hipMemcpyAsync(x, xt, N * 8, hipMemcpyDeviceToDevice, st));
      std::swap(m->F, m->Ft);
      F = devp<double>(m->F);
      Ft = devp<double>(m->Ft);
      f = ft;
      const double xnorm = model_norm(m, x, N, st);
      done = f <= o.rtol * info.fnorm0 || step <= o.stol * xnorm;
    }
    info.converged = done ? 1 : 0;
    info.fnorm = f;
    CPTR_HIP_TRY(hipStreamSynchronize(st));
    info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    return CPTR_OK;
  } catch (const Error &e) {
    return fail(e);
  } catch (const std::bad_alloc &) {
    return fail(Error{CPTR_ERR_OOM, "host allocation failed"});
  } catch (...) {
    return fail(Error{CPTR_ERR_HIP, "unexpected failure"});
  }
}

}  // extern "C"
