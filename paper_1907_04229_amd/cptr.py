"""Python binding of libcptr (include/cptr.h): argument marshalling only.

Device memory comes from torch tensors on a ROCm device (their data_ptr()),
streams from torch.cuda streams.  Every computation runs in libcptr's HIP
kernels; there is no fallback.  If the library has not been built, loading it
raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcptr.so")

CPTR_OK = 0
CPTR_NOT_CONVERGED = 1
FIRST = {"none": 0, "cptr": 1, "cptr_lower": 2, "cpr": 3, "cptr_bd": 4, "cptr_uamg": 5, "cptr_upper": 6}
SECOND = {"none": 0, "bilu0": 1, "bilu0_mc": 2, "identity": 3, "learned": 4}
PRECISION = {"fp64": 0, "fp32": 1}
DECOUPLING = {"none": 0, "qi": 1, "ti": 2}
SCHUR = {"assembled": 0, "att": 1, "diag": 2}
SMOOTHER = {"l1jacobi": 0, "gs": 1}


class Options(C.Structure):
    _fields_ = [("first_stage", C.c_int), ("second_stage", C.c_int), ("precision", C.c_int),
                ("ip", C.c_int), ("iT", C.c_int), ("amg_theta", C.c_double),
                ("amg_max_levels", C.c_int), ("amg_coarse_size", C.c_int),
                ("amg_seed", C.c_uint), ("amg_sweeps", C.c_int), ("amg_smooth_p", C.c_int),
                ("amg_smooth_p_T", C.c_int),
                ("use_graph", C.c_int), ("resid_fp64", C.c_int),
                ("scalar_dia", C.c_int), ("lrn_columns", C.c_int), ("decoupling", C.c_int),
                ("ilu_level", C.c_int), ("schur", C.c_int), ("lrn_fallback", C.c_int),
                ("amg_smoother", C.c_int), ("ilu_part_x", C.c_int), ("ilu_part_y", C.c_int),
                ("ilu_part_z", C.c_int), ("ilu_accum_fp64", C.c_int), ("resetup_device", C.c_int),
                ("amg_sweeps_T", C.c_int)]


class Bsr(C.Structure):
    _fields_ = [("n", C.c_int), ("nv", C.c_int), ("nnzb", C.c_int), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("vals", C.c_void_p)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int), ("nnz", C.c_int), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("vals", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("rtol", C.c_double), ("maxit", C.c_int),
                ("nonzero_guess", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("relres_est", C.c_double), ("relres_true", C.c_double),
                ("solve_ms", C.c_double), ("fell_back", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("nlevels", C.c_int * 2), ("level_rows", (C.c_int * 16) * 2),
                ("level_nnz", (C.c_int * 16) * 2), ("ilu_levels_lower", C.c_int),
                ("ilu_levels_upper", C.c_int), ("ilu_colors", C.c_int),
                ("setup_ms", C.c_double), ("apply_bytes", C.c_double),
                ("spmv_bytes", C.c_double), ("applies", C.c_longlong)]


class ModelDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("three_phase", C.c_int), ("dt", C.c_double), ("perm", C.c_void_p), ("poro", C.c_void_p),
                ("inj", C.POINTER(C.c_int)), ("n_inj", C.c_int), ("prod", C.POINTER(C.c_int)),
                ("n_prod", C.c_int), ("heat", C.POINTER(C.c_int)), ("n_heat", C.c_int)]


class NewtonOpts(C.Structure):
    _fields_ = [("max_it", C.c_int), ("rtol", C.c_double), ("stol", C.c_double),
                ("max_backtrack", C.c_int), ("lin", SolveOpts)]


class NewtonInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("lin_iters", C.c_int), ("backtracks", C.c_int),
                ("converged", C.c_int), ("fnorm0", C.c_double), ("fnorm", C.c_double),
                ("solve_ms", C.c_double)]


class CptrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load():
    """Load libcptr.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1907_04229_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, ip = C.c_void_p, C.c_int
        L.cptr_default_options.argtypes = [C.POINTER(Options)]
        L.cptr_setup.argtypes = [C.POINTER(vp), C.POINTER(Bsr), C.POINTER(Csr), C.POINTER(Options), vp]
        L.cptr_apply.argtypes = [vp, vp, vp, vp]
        L.cptr_first_stage.argtypes = [vp, vp, vp, vp]
        L.cptr_stage_residual.argtypes = [vp, vp, vp, vp]
        L.cptr_vcycle.argtypes = [vp, ip, vp, vp, vp]
        L.fgmres_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.fgmres_solve_static.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.cptr_krylov_vector.argtypes = [vp, ip, vp, vp]
        L.cptr_matvec.argtypes = [vp, vp, vp, vp]
        L.cptr_update_values.argtypes = [vp, vp, vp, vp]
        L.cptr_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.cptr_get_aggregates.argtypes = [vp, ip, ip, C.POINTER(C.c_int)]
        L.cptr_get_ilu_schedule.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                            C.POINTER(C.c_int)]
        L.cptr_bsr_spmv.argtypes = [ip, ip, vp, vp, vp, vp, vp, vp]
        L.cptr_status_string.restype = C.c_char_p
        L.cptr_status_string.argtypes = [ip]
        L.cptr_last_error.restype = C.c_char_p
        L.cptr_destroy.argtypes = [vp]
        fp = C.POINTER(C.c_float)
        L.cptr_learn_param_count.restype = C.c_size_t
        L.cptr_learn_param_count.argtypes = [ip]
        L.cptr_learn_create.argtypes = [C.POINTER(vp), ip, fp]
        L.cptr_learn_set_params.argtypes = [vp, fp]
        L.cptr_learn_get_params.argtypes = [vp, fp]
        L.cptr_learn_destroy.argtypes = [vp]
        L.cptr_learn_attach.argtypes = [vp, vp]
        L.cptr_learn_forward.argtypes = [vp, vp, vp, vp]
        L.cptr_learn_grad.argtypes = [vp, vp, ip, fp, fp, vp]
        L.cptr_learn_rerun_layer.argtypes = [vp, ip, vp, vp]
        L.cptr_learn_train_step.argtypes = [vp, vp, ip, C.c_float, fp, vp]
        L.cptr_kernel_timing.argtypes = [vp, ip]
        L.cptr_get_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
        ipp = C.POINTER(C.c_int)
        L.cptr_model_create.argtypes = [C.POINTER(vp), C.POINTER(ModelDesc)]
        L.cptr_model_destroy.argtypes = [vp]
        L.cptr_model_info.argtypes = [vp, ipp, ipp, ipp, C.POINTER(vp), C.POINTER(vp)]
        L.cptr_model_pattern.argtypes = [vp, ipp, ipp]
        L.cptr_model_assemble.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.cptr_newton_default_options.argtypes = [C.POINTER(NewtonOpts)]
        L.cptr_newton_solve.argtypes = [vp, vp, vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonInfo), vp]
        _lib = L
    return _lib


def _check(rc, allow=(CPTR_OK,)):
    if rc in allow:
        return rc
    L = load()
    raise CptrError(rc, f"{L.cptr_status_string(rc).decode()}: {L.cptr_last_error().decode()}")


def _ptr(t, dtype=None):
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous ROCm tensors"
    if dtype is not None:
        assert t.dtype == dtype, f"expected {dtype}, got {t.dtype}"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def cptr_default_options(**kw):
    o = Options()
    load().cptr_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "first_stage" and isinstance(v, str):
            v = FIRST[v]
        if k == "second_stage" and isinstance(v, str):
            v = SECOND[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "decoupling" and isinstance(v, str):
            v = DECOUPLING[v]
        if k == "schur" and isinstance(v, str):
            v = SCHUR[v]
        if k == "amg_smoother" and isinstance(v, str):
            v = SMOOTHER[v]
        if k == "ilu_parts":  # (px, py, pz)
            o.ilu_part_x, o.ilu_part_y, o.ilu_part_z = (int(q) for q in v)
            continue
        setattr(o, k, v)
    return o


def cptr_setup(n, nv, row_ptr, col_idx, vals, st_row_ptr=None, st_col_idx=None, st_vals=None,
               options=None, stream=None):
    """Returns an opaque handle.  The tensors must outlive the handle (vals is borrowed)."""
    import torch
    A = Bsr(n, nv, col_idx.numel(), _ptr(row_ptr, torch.int32), _ptr(col_idx, torch.int32),
            _ptr(vals, torch.float64))
    S = None
    if st_row_ptr is not None:
        S = Csr(n, st_col_idx.numel(), _ptr(st_row_ptr, torch.int32), _ptr(st_col_idx, torch.int32),
                _ptr(st_vals, torch.float64))
    h = C.c_void_p()
    _check(load().cptr_setup(C.byref(h), C.byref(A), C.byref(S) if S is not None else None,
                             C.byref(options) if options is not None else None, _stream(stream)))
    return h


def cptr_apply(h, v, z, stream=None):
    import torch
    _check(load().cptr_apply(h, _ptr(v, torch.float64), _ptr(z, torch.float64), _stream(stream)))


def cptr_first_stage(h, v, x1, stream=None):
    import torch
    _check(load().cptr_first_stage(h, _ptr(v, torch.float64), _ptr(x1, torch.float64),
                                   _stream(stream)))


def cptr_stage_residual(h, v, b1, stream=None):
    import torch
    _check(load().cptr_stage_residual(h, _ptr(v, torch.float64), _ptr(b1, torch.float64),
                                      _stream(stream)))


def cptr_vcycle(h, which, b, x, stream=None):
    import torch
    _check(load().cptr_vcycle(h, which, _ptr(b, torch.float64), _ptr(x, torch.float64),
                              _stream(stream)))


def cptr_matvec(h, x, y, stream=None):
    import torch
    _check(load().cptr_matvec(h, _ptr(x, torch.float64), _ptr(y, torch.float64), _stream(stream)))


def cptr_krylov_vector(h, j, out, stream=None):
    import torch
    _check(load().cptr_krylov_vector(h, j, _ptr(out, torch.float64), _stream(stream)))


def fgmres_solve(h, b, x, restart=30, rtol=1e-6, maxit=1000, nonzero_guess=False, stream=None):
    import torch
    so = SolveOpts(restart, rtol, maxit, int(bool(nonzero_guess)))
    info = SolveInfo()
    rc = load().fgmres_solve(h, _ptr(b, torch.float64), _ptr(x, torch.float64), C.byref(so),
                             C.byref(info), _stream(stream))
    _check(rc, allow=(CPTR_OK, CPTR_NOT_CONVERGED))
    return dict(iters=info.iters, restarts=info.restarts, converged=bool(info.converged),
                relres_est=info.relres_est, relres_true=info.relres_true, solve_ms=info.solve_ms,
                fell_back=bool(info.fell_back))


def fgmres_solve_static(h, b, x, restart=30, rtol=1e-6, maxit=1000, nonzero_guess=False, stream=None):
    """fgmres_solve with the library's static Krylov workspace (allocates nothing)."""
    import torch
    so = SolveOpts(restart, rtol, maxit, int(bool(nonzero_guess)))
    info = SolveInfo()
    rc = load().fgmres_solve_static(h, _ptr(b, torch.float64), _ptr(x, torch.float64), C.byref(so),
                                    C.byref(info), _stream(stream))
    _check(rc, allow=(CPTR_OK, CPTR_NOT_CONVERGED))
    return dict(iters=info.iters, restarts=info.restarts, converged=bool(info.converged),
                relres_est=info.relres_est, relres_true=info.relres_true, solve_ms=info.solve_ms,
                fell_back=bool(info.fell_back))


def cptr_update_values(h, A_vals, S_vals=None, stream=None):
    import torch
    _check(load().cptr_update_values(h, _ptr(A_vals, torch.float64), _ptr(S_vals, torch.float64),
                                     _stream(stream)))


def cptr_get_stats(h):
    st = Stats()
    _check(load().cptr_get_stats(h, C.byref(st)))
    d = dict(nlevels=list(st.nlevels), ilu_levels_lower=st.ilu_levels_lower,
             ilu_levels_upper=st.ilu_levels_upper, ilu_colors=st.ilu_colors,
             setup_ms=st.setup_ms, apply_bytes=st.apply_bytes, spmv_bytes=st.spmv_bytes,
             applies=st.applies)
    d["level_rows"] = [list(st.level_rows[w])[:st.nlevels[w]] for w in range(2)]
    d["level_nnz"] = [list(st.level_nnz[w])[:st.nlevels[w]] for w in range(2)]
    return d


def cptr_get_aggregates(h, which, level, nrows):
    out = np.empty(max(nrows, 1), np.int32)
    rc = load().cptr_get_aggregates(h, which, level, out.ctypes.data_as(C.POINTER(C.c_int)))
    if rc < 0:
        _check(rc)
    return out[:rc]


def cptr_get_ilu_schedule(h, n):
    a, b, c = (np.empty(n, np.int32) for _ in range(3))
    p = lambda x: x.ctypes.data_as(C.POINTER(C.c_int))  # noqa: E731
    _check(load().cptr_get_ilu_schedule(h, p(a), p(b), p(c)))
    return a, b, c


def cptr_bsr_spmv(n, nv, row_ptr, col_idx, vals, x, y, stream=None):
    import torch
    _check(load().cptr_bsr_spmv(n, nv, _ptr(row_ptr, torch.int32), _ptr(col_idx, torch.int32),
                                _ptr(vals, torch.float64), _ptr(x, torch.float64),
                                _ptr(y, torch.float64), _stream(stream)))


def cptr_kernel_timing(h, enable):
    _check(load().cptr_kernel_timing(h, int(bool(enable))))


def cptr_get_kernel_times(h):
    """(average us per launch, launches) of ids 0 (Krylov product), 1-3 (learned layers)."""
    us = (C.c_double * 4)()
    cnt = (C.c_longlong * 4)()
    _check(load().cptr_get_kernel_times(h, us, cnt))
    return list(us), list(cnt)


def cptr_destroy(h):
    if h:
        load().cptr_destroy(h)


class Solver:
    """Keeps the device copies of one system alive together with its handle."""

    def __init__(self, problem, device="cuda", **opts):
        import torch
        self.problem = problem
        dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)  # noqa: E731
        self.rp = t(problem.row_ptr, torch.int32)
        self.ci = t(problem.col_idx, torch.int32)
        self.vals = t(problem.vals, torch.float64)
        self.srp = t(problem.st_row_ptr, torch.int32)
        self.sci = t(problem.st_col_idx, torch.int32)
        self.svals = t(problem.st_vals, torch.float64)
        self.n, self.nv = problem.n, problem.nv
        self.options = cptr_default_options(**opts)
        self.h = cptr_setup(self.n, self.nv, self.rp, self.ci, self.vals, self.srp, self.sci,
                            self.svals, self.options)

    @classmethod
    def from_tensors(cls, n, nv, rp, ci, vals, srp, sci, svals, **opts):
        """A solver on device tensors (int32 patterns, float64 values) that
        the object keeps alive; no host problem attached."""
        self = cls.__new__(cls)
        self.problem = None
        self.rp, self.ci, self.vals, self.srp, self.sci, self.svals = rp, ci, vals, srp, sci, svals
        self.n, self.nv = n, nv
        self.options = cptr_default_options(**opts)
        self.h = cptr_setup(n, nv, rp, ci, vals, srp, sci, svals, self.options)
        return self

    def update_values(self, problem):
        """Numeric re-setup for a system with the same pattern (cptr_update_values)."""
        import torch
        assert problem.n == self.n and problem.nv == self.nv
        assert np.array_equal(problem.row_ptr, self.problem.row_ptr)
        assert np.array_equal(problem.col_idx, self.problem.col_idx)
        dev = self.vals.device
        vals = torch.as_tensor(np.ascontiguousarray(problem.vals), dtype=torch.float64, device=dev)
        svals = torch.as_tensor(np.ascontiguousarray(problem.st_vals), dtype=torch.float64, device=dev)
        cptr_update_values(self.h, vals, svals)
        self.vals, self.svals, self.problem = vals, svals, problem  # the handle borrows them now

    def solve(self, b, x=None, **kw):
        import torch
        if not torch.is_tensor(b):
            b = torch.as_tensor(np.ascontiguousarray(b), dtype=torch.float64, device=self.vals.device)
        if x is None:
            x = torch.zeros_like(b)
        info = fgmres_solve(self.h, b, x, **kw)
        return x, info

    def apply(self, v):
        import torch
        z = torch.empty_like(v)
        cptr_apply(self.h, v, z)
        return z

    def stats(self):
        return cptr_get_stats(self.h)

    def close(self):
        if self.h:
            cptr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned second stage (cptr_learn.h)
def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def cptr_learn_param_count(nv):
    return int(load().cptr_learn_param_count(nv))


class LearnModel:
    """Parameters (FP32 master copy, BF16 operands, Adam state) on the device."""

    def __init__(self, nv, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        assert theta.size == cptr_learn_param_count(nv)
        self.nv = nv
        self.h = C.c_void_p()
        _check(load().cptr_learn_create(C.byref(self.h), nv, _fptr(theta)))

    def params(self):
        out = np.empty(cptr_learn_param_count(self.nv), np.float32)
        _check(load().cptr_learn_get_params(self.h, _fptr(out)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        _check(load().cptr_learn_set_params(self.h, _fptr(theta)))

    def attach(self, solver):
        _check(load().cptr_learn_attach(solver.h, self.h))
        solver.model = self

    def close(self):
        if self.h:
            load().cptr_learn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cptr_learn_forward(solver, b1, stream=None):
    import torch
    z = torch.empty_like(b1)
    _check(load().cptr_learn_forward(solver.h, _ptr(b1, torch.float64), _ptr(z, torch.float64),
                                     _stream(stream)))
    return z


def cptr_learn_rerun_layer(solver, layer, z2=None, stream=None):
    import torch
    _check(load().cptr_learn_rerun_layer(solver.h, layer, _ptr(z2, torch.float64) if z2 is not None else None,
                                         _stream(stream)))


def cptr_learn_grad(solver, b1_batch, want_grad=True, stream=None):
    import torch
    count = b1_batch.shape[0]
    loss = C.c_float(0.0)
    g = np.empty(cptr_learn_param_count(solver.nv), np.float32) if want_grad else None
    _check(load().cptr_learn_grad(solver.h, _ptr(b1_batch.contiguous(), torch.float64), count,
                                  C.byref(loss), _fptr(g) if want_grad else None, _stream(stream)))
    return float(loss.value), g


def cptr_learn_train_step(solver, b1_batch, lr, stream=None):
    import torch
    loss = C.c_float(0.0)
    _check(load().cptr_learn_train_step(solver.h, _ptr(b1_batch.contiguous(), torch.float64),
                                        b1_batch.shape[0], float(lr), C.byref(loss),
                                        _stream(stream)))
    return float(loss.value)


# ---------------------------------------------------------------- thermal model (cptr_model.h)
def _host_ints(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


class Model:
    """The DG(0)/TPFA thermal model on the device (cptr_model_*): residual,
    Jacobian and S~_T assembly, and Newton steps with cptr_newton_solve."""

    def __init__(self, shape, perm, poro, three_phase=False, dt=10 * 86400.0, inj=(), prod=(), heat=(),
                 dx=0.5, device="cuda"):
        import torch
        nx, ny, nz = shape
        self.shape = tuple(shape)
        dev = torch.device(device)
        pt = torch.as_tensor(np.ascontiguousarray(perm, dtype=np.float64), device=dev)
        po = torch.as_tensor(np.ascontiguousarray(poro, dtype=np.float64), device=dev)
        lists = [_host_ints(c) for c in (inj, prod, heat)]
        d = ModelDesc(nx, ny, nz, dx, int(bool(three_phase)), dt, _ptr(pt, torch.float64), _ptr(po, torch.float64),
                      lists[0][1], lists[0][0].size, lists[1][1], lists[1][0].size, lists[2][1], lists[2][0].size)
        self.m = C.c_void_p()
        _check(load().cptr_model_create(C.byref(self.m), C.byref(d)))
        nv, n, nnzb = C.c_int(), C.c_int(), C.c_int()
        _check(load().cptr_model_info(self.m, C.byref(nv), C.byref(n), C.byref(nnzb), None, None))
        self.nv, self.n, self.nnzb = nv.value, n.value, nnzb.value
        rp = np.empty(self.n + 1, np.int32)
        ci = np.empty(self.nnzb, np.int32)
        _check(load().cptr_model_pattern(self.m, rp.ctypes.data_as(C.POINTER(C.c_int)),
                                         ci.ctypes.data_as(C.POINTER(C.c_int))))
        self.row_ptr, self.col_idx = rp, ci
        self.rp = torch.as_tensor(rp, device=dev)
        self.ci = torch.as_tensor(ci, device=dev)
        self.device = dev

    def assemble(self, x, xn, F=True, A=True, S=True, stream=None):
        """(F*(x), Jacobian values, S~_T values) as float64 device tensors (None where not asked)."""
        import torch
        N = self.n * self.nv
        Ft = torch.empty(N, dtype=torch.float64, device=self.device) if F else None
        At = torch.empty(self.nnzb * self.nv * self.nv, dtype=torch.float64, device=self.device) if A else None
        St = torch.empty(self.nnzb, dtype=torch.float64, device=self.device) if S else None
        _check(load().cptr_model_assemble(self.m, _ptr(x, torch.float64), _ptr(xn, torch.float64), _ptr(Ft),
                                          _ptr(At), _ptr(St), _stream(stream)))
        return Ft, At, St

    def solver(self, x, xn, **opts):
        """A Solver set up on the Jacobian and S~_T at state x (host setup of the hierarchies)."""
        _, A, S = self.assemble(x, xn, F=False)
        return Solver.from_tensors(self.n, self.nv, self.rp, self.ci, A, self.rp, self.ci, S, **opts)

    def newton(self, solver, x, xn, max_it=50, rtol=1e-8, stol=1e-8, max_backtrack=10, restart=30,
               lin_rtol=1e-6, lin_maxit=1000, stream=None):
        """One implicit time step (cptr_newton_solve); x is updated in place."""
        import torch
        o = NewtonOpts()
        load().cptr_newton_default_options(C.byref(o))
        o.max_it, o.rtol, o.stol, o.max_backtrack = max_it, rtol, stol, max_backtrack
        o.lin = SolveOpts(restart, lin_rtol, lin_maxit, 0)
        info = NewtonInfo()
        _check(load().cptr_newton_solve(self.m, solver.h, _ptr(x, torch.float64), _ptr(xn, torch.float64),
                                        C.byref(o), C.byref(info), _stream(stream)))
        return dict(iters=info.iters, lin_iters=info.lin_iters, backtracks=info.backtracks,
                    converged=bool(info.converged), fnorm0=info.fnorm0, fnorm=info.fnorm,
                    solve_ms=info.solve_ms)

    def close(self):
        if getattr(self, "m", None):
            load().cptr_model_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
