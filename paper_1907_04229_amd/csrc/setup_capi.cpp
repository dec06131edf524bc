// Host-only C entry points of the setup algorithms (libcptr_host.so), so that
// the integer results of the setup (aggregates, ILU levels and colours) and
// the FP64 coarse operators can be inspected on a machine without a GPU.
// The GPU library runs exactly these functions inside cptr_setup.
#include <cstring>

#include "setup.h"

using namespace cptr;

namespace {
struct AmgBox {
  AmgHost h;
  std::string err;
};
struct IluBox {
  IluHost h;
};
thread_local std::string g_err;
}  // namespace

extern "C" {

const char *cptrh_last_error(void) { return g_err.c_str(); }

void *cptrh_amg_build(int n, const int *rp, const int *ci, const double *v, double theta,
                      int max_levels, int coarse_size, unsigned seed, int smooth_p, int *status) {
  auto *b = new AmgBox();
  try {
    HostCSR a;
    a.nr = a.nc = n;
    a.rp.assign(rp, rp + n + 1);
    a.ci.assign(ci, ci + rp[n]);
    a.v.assign(v, v + rp[n]);
    AmgParams p;
    p.theta = theta;
    p.max_levels = max_levels;
    p.coarse_size = coarse_size;
    p.seed = seed;
    p.smooth_p = smooth_p;
    amg_build(a, p, b->h);
    *status = 0;
  } catch (const Error &e) {
    g_err = e.msg;
    *status = e.code;
  }
  return b;
}

// The unknown-based hierarchy of a coupled operator in unknown-wise order
// (rows 0 .. np-1 pressure, the rest temperature).
void *cptrh_uamg_build(int n, int np, const int *rp, const int *ci, const double *v, double theta,
                       int max_levels, int coarse_size, unsigned seed, int smooth_p, int smooth_p_T,
                       int *status) {
  auto *b = new AmgBox();
  try {
    HostCSR a;
    a.nr = a.nc = n;
    a.rp.assign(rp, rp + n + 1);
    a.ci.assign(ci, ci + rp[n]);
    a.v.assign(v, v + rp[n]);
    AmgParams p;
    p.theta = theta;
    p.max_levels = max_levels;
    p.coarse_size = coarse_size;
    p.seed = seed;
    p.smooth_p = smooth_p;
    AmgParams pT = p;
    pT.smooth_p = smooth_p_T;
    uamg_build(a, np, p, pT, b->h);
    *status = 0;
  } catch (const Error &e) {
    g_err = e.msg;
    *status = e.code;
  }
  return b;
}

int cptrh_amg_nlevels(void *h) { return (int)static_cast<AmgBox *>(h)->h.lev.size(); }

int cptrh_amg_level_info(void *h, int l, int *n, int *nnz, int *pnnz) {
  auto &L = static_cast<AmgBox *>(h)->h.lev.at(l);
  *n = L.A.nr;
  *nnz = L.A.nnz();
  *pnnz = L.P.nnz();
  return 0;
}

int cptrh_amg_get(void *h, int l, int *agg, int *arp, int *aci, double *av, int *prp, int *pci,
                  double *pv, double *omega) {
  auto &L = static_cast<AmgBox *>(h)->h.lev.at(l);
  std::memcpy(arp, L.A.rp.data(), sizeof(int) * L.A.rp.size());
  std::memcpy(aci, L.A.ci.data(), sizeof(int) * L.A.ci.size());
  std::memcpy(av, L.A.v.data(), sizeof(double) * L.A.v.size());
  if (!L.agg.empty()) {
    std::memcpy(agg, L.agg.data(), sizeof(int) * L.agg.size());
    std::memcpy(prp, L.P.rp.data(), sizeof(int) * L.P.rp.size());
    std::memcpy(pci, L.P.ci.data(), sizeof(int) * L.P.ci.size());
    std::memcpy(pv, L.P.v.data(), sizeof(double) * L.P.v.size());
    *omega = L.omega;
  }
  return 0;
}

void cptrh_amg_free(void *h) { delete static_cast<AmgBox *>(h); }

// parts: NULL, or three ints (parts along x, y, z of the grid the pattern is on)
void *cptrh_ilu_build(int n, int nv, const int *rp, const int *ci, const double *v, int mc,
                      int level, const int *parts, int *status) {
  auto *b = new IluBox();
  try {
    std::vector<int> part;
    if (parts) part = grid_parts(n, rp, ci, parts[0], parts[1], parts[2]);
    ilu_build(n, nv, rp, ci, v, mc != 0, b->h, level, parts ? part.data() : nullptr);
    *status = 0;
  } catch (const Error &e) {
    g_err = e.msg;
    *status = e.code;
  }
  return b;
}

int cptrh_ilu_get(void *h, int *order, int *lev_lower, int *lev_upper, int *color, double *dinv) {
  auto &I = static_cast<IluBox *>(h)->h;
  size_t n = I.order.size();
  if (order) std::memcpy(order, I.order.data(), sizeof(int) * n);
  if (lev_lower) std::memcpy(lev_lower, I.lev_lower.data(), sizeof(int) * n);
  if (lev_upper) std::memcpy(lev_upper, I.lev_upper.data(), sizeof(int) * n);
  if (color) std::memcpy(color, I.color.data(), sizeof(int) * n);
  if (dinv) std::memcpy(dinv, I.dinv.data(), sizeof(double) * I.dinv.size());
  return I.ncolor;
}

// The factor pattern kept for the GPU refactorisation: sizes (entries, forward
// and backward sweep blocks, forward levels) with null arrays, else the arrays
// frp [n+1], fci / src / dst [nnzf], dpos / fwd [n], f_lev_ptr [levels+1].
int cptrh_ilu_pattern(void *h, int *sizes, int *frp, int *fci, int *src, int *dpos, int *dst, int *fwd,
                      int *f_lev_ptr) {
  auto &I = static_cast<IluBox *>(h)->h;
  if (sizes) {
    sizes[0] = int(I.fci.size());
    sizes[1] = int(I.f_col.size());
    sizes[2] = int(I.b_col.size());
    sizes[3] = int(I.f_lev_ptr.size()) - 1;
  }
  auto cp = [](int *dst_, const std::vector<int> &v) {
    if (dst_) std::memcpy(dst_, v.data(), sizeof(int) * v.size());
  };
  cp(frp, I.frp);
  cp(fci, I.fci);
  cp(src, I.src);
  cp(dpos, I.dpos);
  cp(dst, I.dst);
  cp(fwd, I.fwd);
  cp(f_lev_ptr, I.f_lev_ptr);
  return 0;
}

// Algebraic S~_T of a BSR matrix (schur_algebraic): nnz with null arrays,
// else rp [n+1], ci / v [nnz].  Negative status code on failure.
int cptrh_schur(int n, int nv, int ip, int iT, const int *rp, const int *ci, const double *v, int diag,
                int *srp, int *sci, double *sv) {
  try {
    HostCSR s = schur_algebraic(n, nv, ip, iT, rp, ci, v, diag != 0);
    if (srp) std::memcpy(srp, s.rp.data(), sizeof(int) * s.rp.size());
    if (sci) std::memcpy(sci, s.ci.data(), sizeof(int) * s.ci.size());
    if (sv) std::memcpy(sv, s.v.data(), sizeof(double) * s.v.size());
    return s.nnz();
  } catch (const Error &e) {
    g_err = e.msg;
    return e.code;
  }
}

void cptrh_ilu_free(void *h) { delete static_cast<IluBox *>(h); }

}  // extern "C"
