"""Fully implicit DG(0)/TPFA thermal multiphase model on a Cartesian grid.

This module produces the *inputs* of the solver library: the cell-block
Jacobian A (BSR, nv x nv row-major blocks), the right-hand side b = -F*(x),
and the assembled Schur-complement approximation S~_T (scalar CSR).  It holds
none of the preconditioner or Krylov arithmetic.

Discretisation (Section 2.2):
  * cell-wise constant unknowns; the facet flux of phase a between cells L<R is
    the two-point flux  {{K}} (rho k_r / mu)^up ( (p_R-p_L)/h - {rho_a} g.n )
    with the harmonic average {{.}}, arithmetic average {.} and upwinding
    (eq:conswater, eq:consenergy, eq:consoil and the upwind definition that
    follows them);
  * implicit Euler in time (Section 2.2.2);
  * conductive facet flux {{k_T}} [T]/h (eq:consenergy);
  * delta-function sources integrated over one cell (Section 2.2.1).
Equations (rows of each block), following the weighted pressure equation
eq:weighted and the scaling eq:scaling, with the oil saturation eliminated
through the saturation constraint (eq:Sbeta):
  row 0      : T_ref * sum_a c_va F_a          (pressure equation)
  row 1..np-1: c_ref T_ref F_a, a = water(, gas)
  row nv-1   : F_e                             (energy)
Unknowns (columns): p, S_w(, S_g), T.

The Jacobian is formed by complex-step differentiation of the residual, which
is exact to rounding for the analytic property functions used here; the
upwind branch is chosen on the real part, i.e. the derivative of the selected
branch is taken.
"""
import os

import numpy as np

from . import props as P

DAY = 86400.0


class Grid:
    """Cartesian nx x ny x nz grid of cubes of edge dx; index i + nx(j + ny k)."""

    def __init__(self, nx, ny, nz, dx=0.5):
        self.nx, self.ny, self.nz, self.dx = nx, ny, nz, dx
        self.n = nx * ny * nz
        self.vol = dx ** 3
        self.area = dx * dx
        idx = np.arange(self.n).reshape(nz, ny, nx)
        Ls, Rs, gn = [], [], []
        self.segments = []   # (stencil offset, first face, end face) per axis
        nf = 0
        for axis, shape_ok in ((2, nx > 1), (1, ny > 1), (0, nz > 1)):
            if not shape_ok:
                continue
            sl_l = [slice(None)] * 3
            sl_r = [slice(None)] * 3
            sl_l[axis] = slice(0, -1)
            sl_r[axis] = slice(1, None)
            l = idx[tuple(sl_l)].reshape(-1)
            r = idx[tuple(sl_r)].reshape(-1)
            Ls.append(l)
            Rs.append(r)
            off = {2: 1, 1: nx, 0: nx * ny}[axis]
            self.segments.append((off, nf, nf + l.size))
            nf += l.size
            # gravity acts along -z; n points from L to R (+z for z-faces)
            gn.append(np.full(l.size, -P.G if axis == 0 else 0.0))
        if Ls:
            self.fL = np.concatenate(Ls)
            self.fR = np.concatenate(Rs)
            self.gdotn = np.concatenate(gn)
        else:
            self.fL = np.zeros(0, np.int64)
            self.fR = np.zeros(0, np.int64)
            self.gdotn = np.zeros(0)
        self.nf = self.fL.size
        self._pattern = None

    def cell(self, i, j, k):
        return i + self.nx * (j + self.ny * k)

    def bsr_pattern(self):
        """7-point BSR pattern with ascending columns; returns (row_ptr, col_idx,
        slot) where slot[off][i] is the position of block (i, i+off) or -1."""
        if self._pattern is None:
            self._pattern = self._make_pattern()
        return self._pattern

    def scatter_faces(self, arr, idx_of, f_l, f_r):
        """arr[idx_of(L)] += f_l and arr[idx_of(R)] += f_r face by face; within one
        axis every cell is the L (or R) cell of at most one face, so plain
        fancy-index updates are exact."""
        for off, a, b in self.segments:
            arr[idx_of(off, "L", self.fL[a:b])] += f_l[a:b]
            arr[idx_of(off, "R", self.fR[a:b])] += f_r[a:b]

    def _make_pattern(self):
        n, nx, nxy = self.n, self.nx, self.nx * self.ny
        i = np.arange(n)
        ii = i % nx
        jj = (i // nx) % self.ny
        kk = i // nxy
        offs = [(-nxy, kk > 0), (-nx, jj > 0), (-1, ii > 0), (0, np.ones(n, bool)),
                (1, ii < nx - 1), (nx, jj < self.ny - 1), (nxy, kk < self.nz - 1)]
        cnt = np.zeros(n, np.int64)
        for _, m in offs:
            cnt += m
        row_ptr = np.zeros(n + 1, np.int64)
        np.cumsum(cnt, out=row_ptr[1:])
        col = np.empty(row_ptr[-1], np.int64)
        pos = row_ptr[:-1].copy()
        slot = {}
        for off, m in offs:
            col[pos[m]] = i[m] + off
            # offsets of different axes coincide when nx or ny is 1 (-nx = -1,
            # nx ny = nx); such a pair never has both neighbours, so the
            # positions are merged
            slot[off] = np.where(m, pos, slot.get(off, -1))
            pos = pos + m
        return row_ptr, col, slot


class Wells:
    """Injector/producer/heater cell sets (cell indices)."""

    def __init__(self, inj=(), prod=(), heat=()):
        self.inj = np.asarray(inj, np.int64)
        self.prod = np.asarray(prod, np.int64)
        self.heat = np.asarray(heat, np.int64)


class ThermalModel:
    """Two-phase (water/oil) or three-phase (water/gas/oil) thermal model."""

    def __init__(self, grid, perm, poro, three_phase=False, wells=None,
                 dt=10 * DAY, phases=None):
        self.g = grid
        self.perm = np.asarray(perm, float)
        self.poro = np.asarray(poro, float)
        self.three_phase = three_phase
        if phases is None:
            phases = [P.WATER, P.GAS, P.OIL] if three_phase else [P.WATER, P.OIL]
        # the last phase (oil) is the eliminated one
        self.phases = phases
        self.np_ = len(phases)
        self.nv = self.np_ + 1
        self.dt = dt
        self.wells = wells if wells is not None else Wells()
        # initial saturations of the non-eliminated phases (water, gas)
        self.s_init = [0.1, 0.05] if three_phase else [0.1]
        so = 1.0 - sum(self.s_init)
        sats = self.s_init + [so]
        self.t_ref = P.T_INIT
        self.c_ref = sum(s * ph.cv for s, ph in zip(sats, phases))
        # harmonic permeability per face
        kl, kr = self.perm[grid.fL], self.perm[grid.fR]
        self.kface = 2.0 * kl * kr / (kl + kr)
        rw = P.WELL_RW
        ro = 0.198 * grid.dx
        self.wi = 2 * np.pi * self.perm * grid.dx / np.log(ro / rw)

    # ---- state helpers ----------------------------------------------------
    def initial_state(self):
        """Initial state of the first implicit step: uniform S and T, pressure in
        hydrostatic equilibrium with the oil (eliminated) phase, equal to the
        tabulated initial pressure at mid-depth."""
        g = self.g
        n = g.n
        x = np.empty((n, self.nv))
        z = (np.arange(n) // (g.nx * g.ny) + 0.5) * g.dx
        rho_ref = self.phases[-1].rho(P.P_INIT, P.T_INIT)
        x[:, 0] = P.P_INIT + rho_ref * P.G * (0.5 * g.nz * g.dx - z)
        for a, s in enumerate(self.s_init):
            x[:, 1 + a] = s
        x[:, -1] = P.T_INIT
        return x

    def _sats(self, x):
        s = [x[..., 1 + a] for a in range(self.np_ - 1)]
        so = 1.0 - sum(s)
        return s + [so]

    # ---- residual pieces --------------------------------------------------
    def _cell_terms(self, x, xn, cells=None):
        """Accumulation + sources; returns (..., nv) unscaled [F_a..., F_e]."""
        g = self.g
        phi = self.poro if cells is None else self.poro[cells]
        p, T = x[..., 0], x[..., -1]
        pn, Tn = xn[..., 0], xn[..., -1]
        S, Sn = self._sats(x), self._sats(xn)
        out = []
        energy = (1.0 - phi) * P.RHO_ROCK * P.CV_ROCK * (T - Tn)
        for a, ph in enumerate(self.phases):
            rho, rhon = ph.rho(p, T), ph.rho(pn, Tn)
            out.append(g.vol * phi * (S[a] * rho - Sn[a] * rhon) / self.dt)
            energy = energy + phi * ph.cv * (S[a] * rho * T - Sn[a] * rhon * Tn)
        out.append(g.vol * energy / self.dt)
        return out

    def _source_terms(self, x, out):
        """Subtract well/heater sources (mass rates in kg/s, energy in W)."""
        w = self.wells
        p, T = x[..., 0], x[..., -1]
        S = self._sats(x)
        nph = self.np_
        res = [o.copy() if isinstance(o, np.ndarray) else o for o in out]
        if w.inj.size:
            c = w.inj
            qw = P.Q_INJ * P.WATER.rho(p[c], P.T_INJ + 0.0 * T[c])
            res[0][c] = res[0][c] - qw
            res[nph][c] = res[nph][c] - P.CV_WATER * P.T_INJ * qw
        if w.prod.size:
            c = w.prod
            dp = p[c] - P.P_BHP
            on = (dp.real > 0).astype(float)
            for a, ph in enumerate(self.phases):
                q = on * self.wi[c] * S[a][c] / ph.mu(T[c]) * dp * ph.rho(p[c], T[c])
                res[a][c] = res[a][c] + q
                res[nph][c] = res[nph][c] + ph.cv * T[c] * q
        if w.heat.size:
            c = w.heat
            res[nph][c] = res[nph][c] - P.HEATER_U * (P.T_HEATER - T[c])
        return res

    def _face_flux(self, xl, xr):
        """Outflow (L->R) of [mass_a..., energy] through every face."""
        g = self.g
        pl, pr = xl[:, 0], xr[:, 0]
        tl, tr = xl[:, -1], xr[:, -1]
        sl, sr = self._sats(xl), self._sats(xr)
        out = []
        energy = 0.0
        ktl = (1 - self.poro[g.fL]) * P.K_T_ROCK
        ktr = (1 - self.poro[g.fR]) * P.K_T_ROCK
        for a, ph in enumerate(self.phases):
            rl, rr = ph.rho(pl, tl), ph.rho(pr, tr)
            pot = (pr - pl) / g.dx - 0.5 * (rl + rr) * g.gdotn
            up_r = pot.real > 0.0  # tie -> L (lower index) upwind
            mob = np.where(up_r, rr * sr[a] / ph.mu(tr), rl * sl[a] / ph.mu(tl))
            m = -self.kface * mob * pot * g.area
            out.append(m)
            energy = energy + ph.cv * np.where(up_r, tr, tl) * m
            ktl = ktl + self.poro[g.fL] * sl[a] * ph.k_t
            ktr = ktr + self.poro[g.fR] * sr[a] * ph.k_t
        kt = 2.0 * ktl * ktr / (ktl + ktr)
        energy = energy - kt * (tr - tl) / g.dx * g.area
        out.append(energy)
        return out

    def _scale(self, comps):
        """Unscaled [F_a..., F_e] -> rows of F* (eq:weighted, eq:scaling)."""
        nph = self.np_
        rows = [self.t_ref * sum(ph.cv * comps[a] for a, ph in enumerate(self.phases))]
        for a in range(nph - 1):
            rows.append(self.c_ref * self.t_ref * comps[a])
        rows.append(comps[nph])
        return np.stack(rows, axis=-1)

    def residual(self, x, xn):
        """F*(x) as an (n, nv) array."""
        g = self.g
        F = self._scale(self._source_terms(x, self._cell_terms(x, xn)))
        if g.nf:
            f = self._scale(self._face_flux(x[g.fL], x[g.fR]))
            F = F.astype(np.result_type(F, f))
            g.scatter_faces(F, lambda off, side, cells: cells, f, -f)
        return F

    # ---- Jacobian ------------------------------------------------------------
    def jacobian(self, x, xn, h=1e-30):
        """Analytic (complex-step) Jacobian as BSR (row_ptr, col_idx, vals[nnzb, nv, nv])."""
        g, nv = self.g, self.nv
        row_ptr, col, slot = g.bsr_pattern()
        vals = np.zeros((col.size, nv, nv))
        diag = slot[0]
        # cell-local part: derivative of every cell's residual w.r.t. its own unknowns
        for u in range(nv):
            xc = x.astype(complex)
            xc[:, u] += 1j * h
            cell = self._scale(self._source_terms(xc, self._cell_terms(xc, xn)))
            vals[diag, :, u] += cell.imag / h
        if g.nf:
            xl, xr = x[g.fL], x[g.fR]
            dfl = np.empty((g.nf, nv, nv))
            dfr = np.empty((g.nf, nv, nv))

            def column(task):
                side, u = task
                if side == 0:
                    a = xl.astype(complex)
                    a[:, u] += 1j * h
                    d = self._scale(self._face_flux(a, xr)).imag / h
                    dfl[:, :, u] = d
                else:
                    a = xr.astype(complex)
                    a[:, u] += 1j * h
                    d = self._scale(self._face_flux(xl, a)).imag / h
                    dfr[:, :, u] = d

            tasks = [(side, u) for u in range(nv) for side in (0, 1)]
            if g.nf >= 200_000:
                # numpy releases the GIL inside large array operations
                from concurrent.futures import ThreadPoolExecutor
                with ThreadPoolExecutor(max_workers=min(len(tasks), os.cpu_count() or 1)) as ex:
                    list(ex.map(column, tasks))
            else:
                for t in tasks:
                    column(t)
            # d F_L/d x_L += dfl, d F_R/d x_R -= dfr, d F_L/d x_R += dfr, d F_R/d x_L -= dfl
            g.scatter_faces(vals, lambda off, side, cells: diag[cells], dfl, -dfr)
            g.scatter_faces(vals, lambda off, side, cells: slot[off if side == "L" else -off][cells],
                            dfr, -dfl)
        return row_ptr, col, vals

    # ---- Schur complement approximation (eq:Se) -------------------------------
    def schur_approx(self, x):
        """Assemble S~_T of eq:Se at state x as scalar CSR on the cell graph.

        Terms (all coefficients frozen at x, only the temperature increment
        varies): accumulation phi sum_a c_va S_a rho_a / dt + (1-phi) rho_r c_r /dt;
        upwinded advection c_va (dT)^up times the frozen facet mass flux;
        conduction {{k_T}} [dT]/h; production term -sum_a c_va f_a,prod and the
        heater term U D_heaters on the diagonal."""
        g = self.g
        row_ptr, col, slot = g.bsr_pattern()
        vals = np.zeros(col.size)
        diag = slot[0]
        p, T = x[:, 0], x[:, -1]
        S = self._sats(x)
        acc = (1.0 - self.poro) * P.RHO_ROCK * P.CV_ROCK
        for a, ph in enumerate(self.phases):
            acc = acc + self.poro * ph.cv * S[a] * ph.rho(p, T)
        vals[diag] += g.vol * acc / self.dt
        w = self.wells
        if w.prod.size:
            c = w.prod
            dp = p[c] - P.P_BHP
            on = (dp > 0).astype(float)
            for a, ph in enumerate(self.phases):
                q = on * self.wi[c] * S[a][c] / ph.mu(T[c]) * dp * ph.rho(p[c], T[c])
                vals[diag[c]] += ph.cv * q
        if w.heat.size:
            vals[diag[w.heat]] += P.HEATER_U
        if g.nf:
            xl, xr = x[g.fL], x[g.fR]
            pl, pr = xl[:, 0], xr[:, 0]
            tl, tr = xl[:, -1], xr[:, -1]
            sl, sr = self._sats(xl), self._sats(xr)
            dl = np.zeros(g.nf)
            dr = np.zeros(g.nf)
            ktl = (1 - self.poro[g.fL]) * P.K_T_ROCK
            ktr = (1 - self.poro[g.fR]) * P.K_T_ROCK
            for a, ph in enumerate(self.phases):
                rl, rr = ph.rho(pl, tl), ph.rho(pr, tr)
                pot = (pr - pl) / g.dx - 0.5 * (rl + rr) * g.gdotn
                up_r = pot > 0.0
                mob = np.where(up_r, rr * sr[a] / ph.mu(tr), rl * sl[a] / ph.mu(tl))
                m = -self.kface * mob * pot * g.area
                dl += np.where(up_r, 0.0, ph.cv * m)
                dr += np.where(up_r, ph.cv * m, 0.0)
                ktl = ktl + self.poro[g.fL] * sl[a] * ph.k_t
                ktr = ktr + self.poro[g.fR] * sr[a] * ph.k_t
            kt = 2.0 * ktl * ktr / (ktl + ktr) * g.area / g.dx
            dl += kt
            dr -= kt
            g.scatter_faces(vals, lambda off, side, cells: diag[cells], dl, -dr)
            g.scatter_faces(vals, lambda off, side, cells: slot[off if side == "L" else -off][cells],
                            dr, -dl)
        return row_ptr, col, vals
