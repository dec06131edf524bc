// The discrete thermal model on the GPU: the fully implicit DG(0)/TPFA
// residual F*(x) (Section 2.2: cell-wise constant unknowns, two-point facet
// fluxes with harmonic permeability, arithmetic density average and upwind
// mobility, the conductive flux {{k_T}} [T] / h, implicit Euler, wells and
// heaters as cell sources), its Jacobian in the 7-point BSR pattern and the
// assembled S~_T of the temperature Schur approximation (Section 3.3.1).
//
// Rows of a cell's block (the weighted pressure equation and the scaling of
// Section 4): row 0 = T_ref sum_a c_va F_a, rows 1 .. np-1 = c_ref T_ref F_a
// for water (and gas), row nv-1 = F_e.  Columns: p, S_w (, S_g), T; oil is
// the eliminated phase, S_o = 1 - sum of the others.
//
// Derivatives are taken in forward mode (dual numbers carrying the
// derivatives with respect to one cell's unknowns, or to both cells of a
// face), exact up to rounding for these analytic property functions; an
// upwind or producer switch is decided on the value.  One thread owns each
// cell's row: the two cells of a face each evaluate its flux, and a row sums
// its contributions in a fixed order (accumulation and sources, then the
// faces along x, y, z, each with the cell first as left and then as right
// cell), so the result does not depend on thread timing.
#pragma once

#include "kernels.h"

// every product and sum of the model rounded on its own, as the host
// generator's arithmetic is
#pragma float_control(push)
#pragma clang fp contract(off)

namespace cptr {
namespace phys {
// rock and fluid heat constants and the initial pressure (the parameter table
// of Section 4)
constexpr double P_INIT = 4.1369e7, K_T_OIL = 0.15, K_T_WATER = 0.6005638, K_T_ROCK = 1.7295772056;
constexpr double CV_OIL = 2093.4, CV_WATER = 4181.3, CV_ROCK = 920.0, RHO_ROCK = 2650.0;
constexpr double T_INIT = 288.706, T_INJ = 373.15, T_HEATER = 373.15, G = 9.80665, P_BHP = 2.7579e7;
// oil and gas constants, heater and well data: synthetic choices (the paper
// defers its oil and gas data to a companion paper)
constexpr double MU_O_REF = 10.0, MU_O_B = 7400.0, RHO_O_SURF = 999.0, C_OIL = 1.0e-9, BETA_OIL = 4.0e-4;
constexpr double P_SURF = 1.01325e5, GAS_M = 0.016, GAS_R = 8.314462618, MU_GAS = 1.5e-5, CV_GAS = 1700.0;
constexpr double K_T_GAS = 0.03, HEATER_U = 1.0e3, Q_INJ = 1.0e-7;
// water viscosity (Grabowski) and density (Kell, as modified by Trangenstein)
// from the tables of Appendix A
constexpr double GRAB_A = 2.1850, GRAB_B = 0.04012, GRAB_C = 5.1547e-6;
constexpr double KELL_E0 = 999.83952, KELL_E1 = 16.955176, KELL_E2 = -7.987e-3, KELL_E3 = -46.170461e-6,
                 KELL_E4 = 105.56302e-9, KELL_E5 = -280.54353e-12, KELL_E6 = 16.87985e-3, KELL_E7 = 10.2,
                 KELL_CW = 3.98854e-4;
}  // namespace phys

// value and derivatives with respect to N independent unknowns
template <int N>
struct Dn {
  double v;
  double d[N];
};

template <int N>
__device__ __forceinline__ Dn<N> dconst(double c) {
  Dn<N> r;
  r.v = c;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = 0.0;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> dvar(double x, int q0) {
  Dn<N> r = dconst<N>(x);
  r.d[q0] = 1.0;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(const Dn<N> &a, const Dn<N> &b) {
  Dn<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = a.d[q] + b.d[q];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N> &a, const Dn<N> &b) {
  Dn<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = a.d[q] - b.d[q];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N> &a) {
  Dn<N> r;
  r.v = -a.v;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = -a.d[q];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(const Dn<N> &a, const Dn<N> &b) {
  Dn<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = a.d[q] * b.v + a.v * b.d[q];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator/(const Dn<N> &a, const Dn<N> &b) {
  Dn<N> r;
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = (a.d[q] - r.v * b.d[q]) * ib;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(const Dn<N> &a, double c) {
  Dn<N> r = a;
  r.v = a.v + c;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(double c, const Dn<N> &a) {
  return a + c;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N> &a, double c) {
  Dn<N> r = a;
  r.v = a.v - c;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(double c, const Dn<N> &a) {
  Dn<N> r;
  r.v = c - a.v;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = -a.d[q];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(const Dn<N> &a, double c) {
  Dn<N> r;
  r.v = a.v * c;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = a.d[q] * c;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(double c, const Dn<N> &a) {
  return a * c;
}
template <int N>
__device__ __forceinline__ Dn<N> operator/(const Dn<N> &a, double c) {
  Dn<N> r;
  r.v = a.v / c;
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = a.d[q] / c;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator/(double c, const Dn<N> &b) {
  return dconst<N>(c) / b;
}
template <int N>
__device__ __forceinline__ Dn<N> dexp(const Dn<N> &a) {
  Dn<N> r;
  r.v = exp(a.v);
#pragma unroll
  for (int q = 0; q < N; q++) r.d[q] = r.v * a.d[q];
  return r;
}

// ---- phase properties (temperature in K, pressure in Pa) ----------------
// phase index: 0 water, 1 gas (three-phase only), last oil
template <int N>
__device__ __forceinline__ Dn<N> mu_water(const Dn<N> &T) {
  using namespace phys;
  const Dn<N> tf = (T - 273.15) * 1.8 + 32.0;
  return 1.0e-3 * GRAB_A / (-1.0 + GRAB_B * tf + GRAB_C * tf * tf);
}
template <int N>
__device__ __forceinline__ Dn<N> rho_water(const Dn<N> &p, const Dn<N> &T) {
  using namespace phys;
  const Dn<N> tc = T - 273.15;
  const Dn<N> num = KELL_E0 + tc * (KELL_E1 + tc * (KELL_E2 + tc * (KELL_E3 + tc * (KELL_E4 + tc * KELL_E5))));
  return num / (1.0 + KELL_E6 * tc) * dexp(KELL_CW * (p * 1.0e-6 - KELL_E7));
}
template <int N>
__device__ __forceinline__ Dn<N> mu_oil(const Dn<N> &T) {
  using namespace phys;
  return MU_O_REF * dexp(MU_O_B * (1.0 / T - 1.0 / T_INIT));
}
template <int N>
__device__ __forceinline__ Dn<N> rho_oil(const Dn<N> &p, const Dn<N> &T) {
  using namespace phys;
  return RHO_O_SURF * dexp(C_OIL * (p - P_SURF) - BETA_OIL * (T - T_INIT));
}
template <int N>
__device__ __forceinline__ Dn<N> rho_gas(const Dn<N> &p, const Dn<N> &T) {
  using namespace phys;
  return p * GAS_M / (GAS_R * T);
}

template <int NP>
struct Phases;
template <>
struct Phases<2> {  // water, oil
  static __device__ __forceinline__ double cv(int a) { return a == 0 ? phys::CV_WATER : phys::CV_OIL; }
  static __device__ __forceinline__ double kt(int a) { return a == 0 ? phys::K_T_WATER : phys::K_T_OIL; }
  template <int N>
  static __device__ __forceinline__ Dn<N> rho(int a, const Dn<N> &p, const Dn<N> &T) {
    return a == 0 ? rho_water(p, T) : rho_oil(p, T);
  }
  template <int N>
  static __device__ __forceinline__ Dn<N> mu(int a, const Dn<N> &T) {
    return a == 0 ? mu_water(T) : mu_oil(T);
  }
};
template <>
struct Phases<3> {  // water, gas, oil
  static __device__ __forceinline__ double cv(int a) {
    return a == 0 ? phys::CV_WATER : (a == 1 ? phys::CV_GAS : phys::CV_OIL);
  }
  static __device__ __forceinline__ double kt(int a) {
    return a == 0 ? phys::K_T_WATER : (a == 1 ? phys::K_T_GAS : phys::K_T_OIL);
  }
  template <int N>
  static __device__ __forceinline__ Dn<N> rho(int a, const Dn<N> &p, const Dn<N> &T) {
    return a == 0 ? rho_water(p, T) : (a == 1 ? rho_gas(p, T) : rho_oil(p, T));
  }
  template <int N>
  static __device__ __forceinline__ Dn<N> mu(int a, const Dn<N> &T) {
    return a == 0 ? mu_water(T) : (a == 1 ? dconst<N>(phys::MU_GAS) : mu_oil(T));
  }
};

// the model data the kernels read
struct ModelView {
  int nx, ny, nz, n;
  double dx, vol, area, dt;
  double c_ref;          // sum_a S_a c_va of the initial saturations
  const double *perm, *poro, *wi;
  const unsigned char *well;  // bit 0 injector, bit 1 producer, bit 2 heater
};

// rows of F* from the unscaled [F_a ..., F_e] of one cell or one face
template <int NV, int N>
__device__ __forceinline__ void scale_rows(const ModelView &m, const Dn<N> (&c)[NV], Dn<N> (&r)[NV]) {
  using Ph = Phases<NV - 1>;
  constexpr int NP = NV - 1;
  Dn<N> s = Ph::cv(0) * c[0];
#pragma unroll
  for (int a = 1; a < NP; a++) s = s + Ph::cv(a) * c[a];
  r[0] = phys::T_INIT * s;
#pragma unroll
  for (int a = 0; a < NP - 1; a++) r[1 + a] = (m.c_ref * phys::T_INIT) * c[a];
  r[NV - 1] = c[NP];
}

// saturations of all phases from the unknowns (the last one eliminated)
template <int NV, int N>
__device__ __forceinline__ void sats(const Dn<N> (&x)[NV], Dn<N> (&S)[NV - 1]) {
  Dn<N> sum = x[1];
#pragma unroll
  for (int a = 1; a < NV - 2; a++) sum = sum + x[1 + a];
#pragma unroll
  for (int a = 0; a < NV - 2; a++) S[a] = x[1 + a];
  S[NV - 2] = 1.0 - sum;
}

// accumulation (implicit Euler) and well / heater sources of cell i
template <int NV, int N>
__device__ __forceinline__ void cell_terms(const ModelView &m, int i, const Dn<N> (&x)[NV],
                                           const double *__restrict__ xn, Dn<N> (&out)[NV]) {
  using namespace phys;
  using Ph = Phases<NV - 1>;
  constexpr int NP = NV - 1;
  const double phi = m.poro[i];
  Dn<N> S[NP], Sn[NP];
  sats<NV, N>(x, S);
  {
    Dn<N> xnd[NV];
#pragma unroll
    for (int u = 0; u < NV; u++) xnd[u] = dconst<N>(xn[u]);
    sats<NV, N>(xnd, Sn);
  }
  const Dn<N> &p = x[0], &T = x[NV - 1];
  const Dn<N> pn = dconst<N>(xn[0]), Tn = dconst<N>(xn[NV - 1]);
  Dn<N> energy = ((1.0 - phi) * RHO_ROCK * CV_ROCK) * (T - Tn);
#pragma unroll
  for (int a = 0; a < NP; a++) {
    const Dn<N> rho = Ph::rho(a, p, T), rhon = Ph::rho(a, pn, Tn);
    out[a] = (m.vol * phi) * (S[a] * rho - Sn[a] * rhon) / m.dt;
    energy = energy + (phi * Ph::cv(a)) * (S[a] * rho * T - Sn[a] * rhon * Tn);
  }
  out[NP] = m.vol * energy / m.dt;
  const unsigned w = m.well[i];
  if (w & 1u) {  // hot-water injector: a fixed volume rate at T_INJ
    const Dn<N> qw = Q_INJ * rho_water(p, dconst<N>(T_INJ));
    out[0] = out[0] - qw;
    out[NP] = out[NP] - (CV_WATER * T_INJ) * qw;
  }
  if (w & 2u) {  // Peaceman producer at the bottom-hole pressure, open while p > P_BHP
    const Dn<N> dp = p - P_BHP;
    if (dp.v > 0.0) {
#pragma unroll
      for (int a = 0; a < NP; a++) {
        const Dn<N> q = m.wi[i] * S[a] / Ph::mu(a, T) * dp * Ph::rho(a, p, T);
        out[a] = out[a] + q;
        out[NP] = out[NP] + Ph::cv(a) * T * q;
      }
    }
  }
  if (w & 4u) out[NP] = out[NP] - HEATER_U * (T_HEATER - T);  // heater
}

// outflow L -> R of [mass_a ..., energy] through the face between cells L < R
// (axis 0 x, 1 y, 2 z; gravity along -z)
template <int NV, int N>
__device__ __forceinline__ void face_flux(const ModelView &m, int L, int R, int axis, const Dn<N> (&xl)[NV],
                                          const Dn<N> (&xr)[NV], Dn<N> (&out)[NV]) {
  using namespace phys;
  using Ph = Phases<NV - 1>;
  constexpr int NP = NV - 1;
  const double kl = m.perm[L], kr = m.perm[R];
  const double kface = 2.0 * kl * kr / (kl + kr);
  const double gdotn = axis == 2 ? -G : 0.0;
  Dn<N> sl[NP], sr[NP];
  sats<NV, N>(xl, sl);
  sats<NV, N>(xr, sr);
  const Dn<N> &pl = xl[0], &pr = xr[0], &tl = xl[NV - 1], &tr = xr[NV - 1];
  const double phil = m.poro[L], phir = m.poro[R];
  Dn<N> energy = dconst<N>(0.0);
  Dn<N> ktl = dconst<N>((1.0 - phil) * K_T_ROCK), ktr = dconst<N>((1.0 - phir) * K_T_ROCK);
#pragma unroll
  for (int a = 0; a < NP; a++) {
    const Dn<N> rl = Ph::rho(a, pl, tl), rr = Ph::rho(a, pr, tr);
    const Dn<N> pot = (pr - pl) / m.dx - 0.5 * (rl + rr) * gdotn;
    const bool up_r = pot.v > 0.0;  // a tie takes the left (lower-numbered) cell
    const Dn<N> mob = up_r ? rr * sr[a] / Ph::mu(a, tr) : rl * sl[a] / Ph::mu(a, tl);
    const Dn<N> mf = -kface * mob * pot * m.area;
    out[a] = mf;
    energy = energy + Ph::cv(a) * (up_r ? tr : tl) * mf;
    ktl = ktl + phil * sl[a] * Ph::kt(a);
    ktr = ktr + phir * sr[a] * Ph::kt(a);
  }
  const Dn<N> kt = 2.0 * ktl * ktr / (ktl + ktr);
  out[NP] = energy - kt * (tr - tl) / m.dx * m.area;
}

// neighbour of cell (ix, iy, iz) in direction d = 2 axis + (0: +, 1: -), -1 if none
__device__ __forceinline__ int model_nbr(const ModelView &m, int i, int d) {
  const int ix = i % m.nx, iy = (i / m.nx) % m.ny, iz = i / (m.nx * m.ny);
  const int axis = d >> 1, plus = (d & 1) == 0;
  const int c = axis == 0 ? ix : (axis == 1 ? iy : iz);
  const int len = axis == 0 ? m.nx : (axis == 1 ? m.ny : m.nz);
  const int off = axis == 0 ? 1 : (axis == 1 ? m.nx : m.nx * m.ny);
  if (plus) return c + 1 < len ? i + off : -1;
  return c > 0 ? i - off : -1;
}

// BSR position of block (i, j) in row i of the ascending 7-point pattern
__device__ __forceinline__ int model_slot(const int *__restrict__ rp, const int *__restrict__ ci, int i, int j) {
  int lo = rp[i], hi = rp[i + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ci[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// F*(x) (n x nv, cell-major), the Jacobian values (BSR, rp / ci the 7-point
// pattern) and S~_T (CSR on the same cell graph); null outputs are skipped.
template <int NV>
__global__ void __launch_bounds__(128) k_model_assemble(ModelView m, const double *__restrict__ x,
                                                        const double *__restrict__ xn, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, double *__restrict__ F,
                                                        double *__restrict__ A, double *__restrict__ S) {
  constexpr int NP = NV - 1, B2 = NV * NV;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  const double *xi = x + (size_t)i * NV;
  const int kd = model_slot(rp, ci, i, i);
  double f[NV], jd[NV][NV];
  {  // the cell's own terms, with derivatives by its unknowns
    Dn<NV> X[NV], c[NV], r[NV];
#pragma unroll
    for (int u = 0; u < NV; u++) X[u] = dvar<NV>(xi[u], u);
    cell_terms<NV, NV>(m, i, X, xn + (size_t)i * NV, c);
    scale_rows<NV, NV>(m, c, r);
#pragma unroll
    for (int q = 0; q < NV; q++) {
      f[q] = r[q].v;
#pragma unroll
      for (int u = 0; u < NV; u++) jd[q][u] = 0.0 + r[q].d[u];
    }
  }
  for (int d = 0; d < 6; d++) {
    const int j = model_nbr(m, i, d);
    if (j < 0) continue;
    const bool left = (d & 1) == 0;  // this cell is the face's left (lower) cell
    const int L = left ? i : j, R = left ? j : i;
    const double *xL = x + (size_t)L * NV, *xR = x + (size_t)R * NV;
    Dn<2 * NV> XL[NV], XR[NV], c[NV], r[NV];
#pragma unroll
    for (int u = 0; u < NV; u++) {
      XL[u] = dvar<2 * NV>(xL[u], u);
      XR[u] = dvar<2 * NV>(xR[u], NV + u);
    }
    face_flux<NV, 2 * NV>(m, L, R, d >> 1, XL, XR, c);
    scale_rows<NV, 2 * NV>(m, c, r);
    double *off = A ? A + (size_t)model_slot(rp, ci, i, j) * B2 : nullptr;
#pragma unroll
    for (int q = 0; q < NV; q++) {
      if (left) {
        f[q] = f[q] + r[q].v;
#pragma unroll
        for (int u = 0; u < NV; u++) {
          jd[q][u] = jd[q][u] + r[q].d[u];
          if (off) off[q * NV + u] = 0.0 + r[q].d[NV + u];
        }
      } else {
        f[q] = f[q] + (-r[q].v);
#pragma unroll
        for (int u = 0; u < NV; u++) {
          jd[q][u] = jd[q][u] + (-r[q].d[NV + u]);
          if (off) off[q * NV + u] = 0.0 + (-r[q].d[u]);
        }
      }
    }
  }
  if (F)
#pragma unroll
    for (int q = 0; q < NV; q++) F[(size_t)i * NV + q] = f[q];
  if (A)
#pragma unroll
    for (int q = 0; q < NV; q++)
#pragma unroll
      for (int u = 0; u < NV; u++) A[(size_t)kd * B2 + q * NV + u] = jd[q][u];
  if (!S) return;
  // S~_T (eq:Se): coefficients frozen at x, only the temperature increment
  // varies; diagonal from accumulation, producer and heater, and per face the
  // upwinded advection c_va (dT)^up times the frozen mass flux and the conduction
  using namespace phys;
  using Ph = Phases<NP>;
  Dn<1> X[NV];
#pragma unroll
  for (int u = 0; u < NV; u++) X[u] = dconst<1>(xi[u]);
  Dn<1> Sa[NP];
  sats<NV, 1>(X, Sa);
  const double phi = m.poro[i];
  double acc = (1.0 - phi) * RHO_ROCK * CV_ROCK;
#pragma unroll
  for (int a = 0; a < NP; a++) acc = acc + phi * Ph::cv(a) * Sa[a].v * Ph::rho(a, X[0], X[NV - 1]).v;
  double sd = 0.0 + m.vol * acc / m.dt;
  const unsigned w = m.well[i];
  if (w & 2u) {
    const double dp = X[0].v - P_BHP;
    const double on = dp > 0.0 ? 1.0 : 0.0;
#pragma unroll
    for (int a = 0; a < NP; a++) {
      const double q = on * m.wi[i] * Sa[a].v / Ph::mu(a, X[NV - 1]).v * dp * Ph::rho(a, X[0], X[NV - 1]).v;
      sd = sd + Ph::cv(a) * q;
    }
  }
  if (w & 4u) sd = sd + HEATER_U;
  for (int d = 0; d < 6; d++) {
    const int j = model_nbr(m, i, d);
    if (j < 0) continue;
    const bool left = (d & 1) == 0;
    const int L = left ? i : j, R = left ? j : i;
    Dn<1> XL[NV], XR[NV];
#pragma unroll
    for (int u = 0; u < NV; u++) {
      XL[u] = dconst<1>(x[(size_t)L * NV + u]);
      XR[u] = dconst<1>(x[(size_t)R * NV + u]);
    }
    Dn<1> sl[NP], sr[NP];
    sats<NV, 1>(XL, sl);
    sats<NV, 1>(XR, sr);
    const double pl = XL[0].v, pr = XR[0].v;
    const double kl = m.perm[L], kr = m.perm[R];
    const double kface = 2.0 * kl * kr / (kl + kr);
    const double gdotn = (d >> 1) == 2 ? -G : 0.0;
    double dl = 0.0, dr = 0.0;
    double ktl = (1 - m.poro[L]) * K_T_ROCK, ktr = (1 - m.poro[R]) * K_T_ROCK;
#pragma unroll
    for (int a = 0; a < NP; a++) {
      const double rl = Ph::rho(a, XL[0], XL[NV - 1]).v, rr = Ph::rho(a, XR[0], XR[NV - 1]).v;
      const double pot = (pr - pl) / m.dx - 0.5 * (rl + rr) * gdotn;
      const bool up_r = pot > 0.0;
      const double mob = up_r ? rr * sr[a].v / Ph::mu(a, XR[NV - 1]).v : rl * sl[a].v / Ph::mu(a, XL[NV - 1]).v;
      const double mf = -kface * mob * pot * m.area;
      dl = dl + (up_r ? 0.0 : Ph::cv(a) * mf);
      dr = dr + (up_r ? Ph::cv(a) * mf : 0.0);
      ktl = ktl + m.poro[L] * sl[a].v * Ph::kt(a);
      ktr = ktr + m.poro[R] * sr[a].v * Ph::kt(a);
    }
    const double kt = 2.0 * ktl * ktr / (ktl + ktr) * m.area / m.dx;
    dl = dl + kt;
    dr = dr - kt;
    const int so = model_slot(rp, ci, i, j);
    if (left) {
      sd = sd + dl;
      S[so] = 0.0 + dr;
    } else {
      sd = sd + (-dr);
      S[so] = 0.0 + (-dl);
    }
  }
  S[kd] = sd;
}

// partial sums of squares of x[0 .. n): one per block, in a fixed order
// (kModelNormBlocks blocks, the host adds them in block order)
constexpr int kModelNormBlocks = 1024;

__global__ void __launch_bounds__(kBlock) k_model_sumsq(size_t n, const double *__restrict__ x,
                                                        double *__restrict__ part) {
  __shared__ double sm[kBlock];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s = s + x[i] * x[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = sm[threadIdx.x] + sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void __launch_bounds__(kBlock) k_model_neg(size_t n, const double *__restrict__ x, double *__restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = -x[i];
}

// y = x + lambda dx (the Newton trial state)
__global__ void __launch_bounds__(kBlock) k_model_axpy(size_t n, const double *__restrict__ x, double lambda,
                                                       const double *__restrict__ dx, double *__restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] + lambda * dx[i];
}

}  // namespace cptr

#pragma float_control(pop)
