"""ctypes front end of the FP64 CPU oracle (cptr_oracle.c).

TEST INFRASTRUCTURE ONLY: the independent reference of the CPTR-FGMRES path.
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the GPU library.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "cptr_oracle.c")

FIRST = {"none": 0, "cptr": 1, "cptr_lower": 2, "cpr": 3, "cptr_bd": 4, "cptr_uamg": 5, "cptr_upper": 6}
DECOUPLING = {"none": 0, "qi": 1, "ti": 2}
SCHUR = {"assembled": 0, "att": 1, "diag": 2}
SECOND = {"none": 0, "bilu0": 1, "bilu0_mc": 2, "identity": 3, "exact": 4}


def build(force=True):
    """Compile liborc.so with gcc (no FP contraction, so FP64 decisions are reproducible)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _SO, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
    return _SO


class _Opts(C.Structure):
    _fields_ = [("first_stage", C.c_int), ("second_stage", C.c_int), ("ip", C.c_int),
                ("iT", C.c_int), ("theta", C.c_double), ("max_levels", C.c_int),
                ("coarse_size", C.c_int), ("seed", C.c_uint), ("sweeps", C.c_int),
                ("smooth_p", C.c_int), ("smoother", C.c_int), ("ilu_order", C.c_void_p),
                ("ilu_part", C.c_void_p), ("smooth_p_T", C.c_int), ("decoupling", C.c_int),
                ("ilu_level", C.c_int), ("schur", C.c_int), ("sweeps_T", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("relres_est", C.c_double), ("relres_true", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        vp, ip_, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.c_int, C.c_int, ip_, ip_, dp, ip_, ip_, dp,
                                 C.POINTER(_Opts), ip_]
        L.orc_destroy.argtypes = [vp]
        L.orc_apply.argtypes = [vp, dp, dp]
        L.orc_first_stage.argtypes = [vp, dp, dp]
        L.orc_fgmres.argtypes = [vp, dp, dp, C.c_int, C.c_double, C.c_int,
                                 C.POINTER(_Info), dp, dp, dp]
        L.orc_amg_nlevels.argtypes = [vp, C.c_int]
        L.orc_amg_level_info.argtypes = [vp, C.c_int, C.c_int, ip_, ip_, ip_]
        L.orc_amg_get_level.argtypes = [vp, C.c_int, C.c_int, ip_, ip_, ip_, dp, ip_,
                                        ip_, dp, dp]
        L.orc_amg_vcycle.argtypes = [vp, C.c_int, dp, dp]
        L.orc_ilu_get.argtypes = [vp, ip_, ip_, ip_, ip_, dp, dp]
        L.orc_ilu_pattern.argtypes = [vp, ip_, ip_]
        L.orc_bsr_spmv.argtypes = [C.c_int, C.c_int, ip_, ip_, dp, dp, dp]
        L.orc_strength.argtypes = [C.c_int, ip_, ip_, dp, C.c_double, ip_, ip_]
        L.orc_mis2_greedy.argtypes = [C.c_int, ip_, ip_, C.c_uint, ip_]
        L.orc_fmix32.argtypes = [C.c_uint]
        L.orc_fmix32.restype = C.c_uint
        _lib = L
    return _lib


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ci(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _cd(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def bsr_spmv(row_ptr, col, vals, nv, x):
    rp, ci, v, x = _ci(row_ptr), _ci(col), _cd(vals), _cd(x)
    n = rp.size - 1
    y = np.empty(n * nv)
    lib().orc_bsr_spmv(n, nv, _i(rp), _i(ci), _d(v), _d(x), _d(y))
    return y


def strength(row_ptr, col, vals, theta):
    rp, ci, v = _ci(row_ptr), _ci(col), _cd(vals)
    n = rp.size - 1
    srp = np.empty(n + 1, np.int32)
    cnt = lib().orc_strength(n, _i(rp), _i(ci), _d(v), theta, _i(srp), None)
    sci = np.empty(max(cnt, 1), np.int32)
    lib().orc_strength(n, _i(rp), _i(ci), _d(v), theta, _i(srp), _i(sci))
    return srp, sci[:cnt]


def mis2_greedy(srp, sci, seed=0):
    srp, sci = _ci(srp), _ci(sci)
    n = srp.size - 1
    out = np.empty(max(n, 1), np.int32)
    lib().orc_mis2_greedy(n, _i(srp), _i(sci if sci.size else np.zeros(1, np.int32)),
                          seed, _i(out))
    return out[:n].astype(bool)


def fmix32(h):
    return int(lib().orc_fmix32(h & 0xFFFFFFFF))


class Oracle:
    """The FP64 two-stage CPR/CPTR preconditioner and FGMRES on one system."""

    h = None

    def __init__(self, n, nv, row_ptr, col, vals, st_row_ptr=None, st_col=None,
                 st_vals=None, first="cptr", second="bilu0", ip=0, iT=None,
                 theta=0.08, max_levels=10, coarse_size=512, seed=0, sweeps=2,
                 smooth_p=True, smoother="jacobi", ilu_order=None, ilu_part=None, smooth_p_T=False,
                 decoupling="none", ilu_level=0, schur="assembled", sweeps_T=0):
        self.n, self.nv = n, nv
        self._keep = [_ci(row_ptr), _ci(col), _cd(vals)]
        if st_row_ptr is None:
            st = [np.zeros(n + 1, np.int32), np.zeros(1, np.int32), np.zeros(1)]
        else:
            st = [_ci(st_row_ptr), _ci(st_col), _cd(st_vals)]
        self._keep += st
        extra = [None, None]
        for q, arr in enumerate((ilu_order, ilu_part)):
            if arr is not None:
                a = _ci(arr)
                assert a.size == n
                self._keep.append(a)
                extra[q] = a.ctypes.data
        o = _Opts(FIRST[first], SECOND[second], ip, nv - 1 if iT is None else iT,
                  theta, max_levels, coarse_size, seed, sweeps, int(bool(smooth_p)),
                  {"jacobi": 0, "gs": 1}[smoother], extra[0], extra[1],
                  -1 if smooth_p_T is None else int(bool(smooth_p_T)),
                  DECOUPLING[decoupling], int(ilu_level), SCHUR[schur], int(sweeps_T))
        status = C.c_int(0)
        rp, ci, v, srp, sci, sv = self._keep[:6]
        self.h = lib().orc_create(n, nv, _i(rp), _i(ci), _d(v), _i(srp), _i(sci), _d(sv),
                                  C.byref(o), C.byref(status))
        if status.value != 0:
            lib().orc_destroy(self.h)
            self.h = None
            raise RuntimeError(f"oracle setup failed with status {status.value}")

    @classmethod
    def from_problem(cls, pr, **kw):
        return cls(pr.n, pr.nv, pr.row_ptr, pr.col_idx, pr.vals, pr.st_row_ptr,
                   pr.st_col_idx, pr.st_vals, **kw)

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def apply(self, v):
        v = _cd(v)
        z = np.empty(self.n * self.nv)
        lib().orc_apply(self.h, _d(v), _d(z))
        return z

    def first_stage(self, v):
        v = _cd(v)
        z = np.empty(self.n * self.nv)
        lib().orc_first_stage(self.h, _d(v), _d(z))
        return z

    def fgmres(self, b, m=30, rtol=1e-6, maxit=1000, capture=False):
        b = _cd(b)
        N = self.n * self.nv
        x = np.empty(N)
        info = _Info()
        V = Z = H = None
        if capture:
            V = np.zeros((m + 1, N))
            Z = np.zeros((m, N))
            H = np.zeros((m + 1, m))
        lib().orc_fgmres(self.h, _d(b), _d(x), m, rtol, maxit, C.byref(info),
                         _d(V) if capture else None, _d(Z) if capture else None,
                         _d(H) if capture else None)
        res = dict(iters=info.iters, restarts=info.restarts, converged=bool(info.converged),
                   relres_est=info.relres_est, relres_true=info.relres_true)
        if capture:
            return x, res, V, Z, H
        return x, res

    def amg_levels(self, which):
        """List of dicts per level: A (rp, ci, v), and agg, P (rp, ci, v), omega above the coarsest."""
        L = lib()
        nl = L.orc_amg_nlevels(self.h, which)
        out = []
        for lev in range(nl):
            n, nnz, pnnz = C.c_int(), C.c_int(), C.c_int()
            L.orc_amg_level_info(self.h, which, lev, C.byref(n), C.byref(nnz), C.byref(pnnz))
            n, nnz, pnnz = n.value, nnz.value, pnnz.value
            agg = np.zeros(max(n, 1), np.int32)
            arp = np.zeros(n + 1, np.int32)
            aci = np.zeros(max(nnz, 1), np.int32)
            av = np.zeros(max(nnz, 1))
            prp = np.zeros(n + 1, np.int32)
            pci = np.zeros(max(pnnz, 1), np.int32)
            pv = np.zeros(max(pnnz, 1))
            om = C.c_double(0.0)
            L.orc_amg_get_level(self.h, which, lev, _i(agg), _i(arp), _i(aci), _d(av),
                                _i(prp), _i(pci), _d(pv), C.byref(om))
            d = dict(n=n, A=(arp, aci[:nnz], av[:nnz]))
            if lev + 1 < nl:
                d.update(agg=agg[:n], P=(prp, pci[:pnnz], pv[:pnnz]), omega=om.value)
            out.append(d)
        return out

    def vcycle(self, which, b):
        b = _cd(b)
        x = np.empty_like(b)
        if lib().orc_amg_vcycle(self.h, which, _d(b), _d(x)) != 0:
            raise RuntimeError("no hierarchy")
        return x

    def ilu(self):
        n, nv = self.n, self.nv
        nnzb = lib().orc_ilu_pattern(self.h, None, None)
        if nnzb < 0:
            raise RuntimeError("no ILU")
        frp = np.zeros(n + 1, np.int32)
        fci = np.zeros(max(nnzb, 1), np.int32)
        lib().orc_ilu_pattern(self.h, _i(frp), _i(fci))
        perm = np.zeros(n, np.int32)
        color = np.zeros(n, np.int32)
        ll = np.zeros(n, np.int32)
        lu_ = np.zeros(n, np.int32)
        luv = np.zeros(nnzb * nv * nv)
        dinv = np.zeros(n * nv * nv)
        nc = lib().orc_ilu_get(self.h, _i(perm), _i(color), _i(ll), _i(lu_), _d(luv), _d(dinv))
        if nc < 0:
            raise RuntimeError("no ILU")
        return dict(perm=perm, color=color, lev_lower=ll, lev_upper=lu_, lu=luv,
                    dinv=dinv, ncolor=nc, rp=frp, ci=fci[:nnzb])
