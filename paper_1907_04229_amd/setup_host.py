"""ctypes access to libcptr_host.so: the setup algorithms of libcptr (AMG
hierarchy, BILU(0) factor and schedule) built for the host alone, so that their
integer results can be checked on a machine without a GPU."""
import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcptr_host.so")
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1907_04229_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.cptrh_amg_build.restype = vp
        L.cptrh_amg_build.argtypes = [C.c_int, ip, ip, dp, C.c_double, C.c_int, C.c_int, C.c_uint,
                                      C.c_int, ip]
        L.cptrh_uamg_build.restype = vp
        L.cptrh_uamg_build.argtypes = [C.c_int, C.c_int, ip, ip, dp, C.c_double, C.c_int, C.c_int,
                                       C.c_uint, C.c_int, C.c_int, ip]
        L.cptrh_ilu_pattern.argtypes = [vp] + [ip] * 8
        L.cptrh_schur.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, dp, C.c_int, ip, ip, dp]
        L.cptrh_amg_nlevels.argtypes = [vp]
        L.cptrh_amg_level_info.argtypes = [vp, C.c_int, ip, ip, ip]
        L.cptrh_amg_get.argtypes = [vp, C.c_int, ip, ip, ip, dp, ip, ip, dp, dp]
        L.cptrh_amg_free.argtypes = [vp]
        L.cptrh_ilu_build.restype = vp
        L.cptrh_ilu_build.argtypes = [C.c_int, C.c_int, ip, ip, dp, C.c_int, C.c_int, ip, ip]
        L.cptrh_ilu_get.argtypes = [vp, ip, ip, ip, ip, dp]
        L.cptrh_ilu_free.argtypes = [vp]
        L.cptrh_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def amg_levels(row_ptr, col, vals, theta=0.08, max_levels=10, coarse_size=512, seed=0,
               smooth_p=True):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(vals, np.float64)
    L = load()
    st = C.c_int(0)
    h = L.cptrh_amg_build(rp.size - 1, _i(rp), _i(ci), _d(v), theta, max_levels, coarse_size,
                          seed, int(bool(smooth_p)), C.byref(st))
    return _levels(L, h, st)


def uamg_levels(row_ptr, col, vals, np_, theta=0.08, max_levels=10, coarse_size=512, seed=0,
                smooth_p=True, smooth_p_T=True):
    """The unknown-based hierarchy of a coupled operator whose first np_ rows are pressure."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(vals, np.float64)
    L = load()
    st = C.c_int(0)
    h = L.cptrh_uamg_build(rp.size - 1, np_, _i(rp), _i(ci), _d(v), theta, max_levels, coarse_size,
                           seed, int(bool(smooth_p)), int(bool(smooth_p_T)), C.byref(st))
    return _levels(L, h, st)


def _levels(L, h, st):
    try:
        if st.value != 0:
            raise RuntimeError(f"setup failed ({st.value}): {L.cptrh_last_error().decode()}")
        out = []
        nl = L.cptrh_amg_nlevels(h)
        for l in range(nl):
            n, nnz, pnnz = C.c_int(), C.c_int(), C.c_int()
            L.cptrh_amg_level_info(h, l, C.byref(n), C.byref(nnz), C.byref(pnnz))
            n, nnz, pnnz = n.value, nnz.value, pnnz.value
            agg = np.zeros(max(n, 1), np.int32)
            arp = np.zeros(n + 1, np.int32)
            aci = np.zeros(max(nnz, 1), np.int32)
            av = np.zeros(max(nnz, 1))
            prp = np.zeros(n + 1, np.int32)
            pci = np.zeros(max(pnnz, 1), np.int32)
            pv = np.zeros(max(pnnz, 1))
            om = C.c_double(0.0)
            L.cptrh_amg_get(h, l, _i(agg), _i(arp), _i(aci), _d(av), _i(prp), _i(pci), _d(pv),
                            C.byref(om))
            d = dict(n=n, A=(arp, aci[:nnz], av[:nnz]))
            if l + 1 < nl:
                d.update(agg=agg[:n], P=(prp, pci[:pnnz], pv[:pnnz]), omega=om.value)
            out.append(d)
        return out
    finally:
        L.cptrh_amg_free(h)


def ilu_schedule(row_ptr, col, vals, nv, multicolor, level=0, parts=None):
    """parts: None, or (px, py, pz) block-Jacobi parts of the grid."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(vals, np.float64)
    n = rp.size - 1
    L = load()
    st = C.c_int(0)
    pa = None if parts is None else np.ascontiguousarray(parts, np.int32)
    h = L.cptrh_ilu_build(n, nv, _i(rp), _i(ci), _d(v), int(bool(multicolor)), int(level),
                          None if pa is None else _i(pa), C.byref(st))
    try:
        if st.value != 0:
            raise RuntimeError(f"ILU setup failed ({st.value}): {L.cptrh_last_error().decode()}")
        order, ll, lu, color = (np.zeros(n, np.int32) for _ in range(4))
        dinv = np.zeros(n * nv * nv)
        nc = L.cptrh_ilu_get(h, _i(order), _i(ll), _i(lu), _i(color), _d(dinv))
        sz = np.zeros(4, np.int32)
        L.cptrh_ilu_pattern(h, _i(sz), None, None, None, None, None, None, None)
        nnzf, nfb, nbb, nlev = (int(x) for x in sz)
        frp, dpos, fwd = np.zeros(n + 1, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32)
        fci, src, dst = (np.zeros(max(nnzf, 1), np.int32) for _ in range(3))
        flp = np.zeros(nlev + 1, np.int32)
        L.cptrh_ilu_pattern(h, None, _i(frp), _i(fci), _i(src), _i(dpos), _i(dst), _i(fwd), _i(flp))
        return dict(order=order, lev_lower=ll, lev_upper=lu, color=color, dinv=dinv, ncolor=nc,
                    frp=frp, fci=fci[:nnzf], src=src[:nnzf], dpos=dpos, dst=dst[:nnzf], fwd=fwd,
                    f_lev_ptr=flp, n_fwd_blocks=nfb, n_bwd_blocks=nbb)
    finally:
        L.cptrh_ilu_free(h)


def schur_algebraic(row_ptr, col, vals, nv, ip=0, iT=None, diag=True):
    """The library's algebraic S~_T (A_TT, or A_TT - A_Tp diag(A_pp)^-1 A_pT)."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(vals, np.float64)
    n = rp.size - 1
    iT = nv - 1 if iT is None else iT
    L = load()
    nnz = L.cptrh_schur(n, nv, ip, iT, _i(rp), _i(ci), _d(v), int(bool(diag)), None, None, None)
    if nnz < 0:
        raise RuntimeError(f"S~_T failed ({nnz}): {L.cptrh_last_error().decode()}")
    srp, sci, sv = np.zeros(n + 1, np.int32), np.zeros(max(nnz, 1), np.int32), np.zeros(max(nnz, 1))
    L.cptrh_schur(n, nv, ip, iT, _i(rp), _i(ci), _d(v), int(bool(diag)), _i(srp), _i(sci), _d(sv))
    return srp, sci[:nnz], sv[:nnz]
