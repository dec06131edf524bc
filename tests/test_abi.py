"""The C-ABI library loads and exports every function declared in include/*.h
(no GPU needed: nothing is called)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1907_04229_amd", "libcptr.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "sizeof", "defined"):
                names.add(name)
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1907_04229_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("cptr_setup", "cptr_apply", "fgmres_solve", "cptr_destroy"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(lib, name):
    assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def _options_size_from_header():
    """sizeof(cptr_options) by a C compiler from include/cptr.h."""
    import subprocess
    import tempfile
    src = '#include "cptr.h"\n#include <stdio.h>\nint main(void){printf("%zu", sizeof(cptr_options));return 0;}\n'
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "s.c"), os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        return int(subprocess.check_output([exe]).decode())


def test_status_strings_and_defaults(lib):
    from paper_1907_04229_amd import cptr
    L = cptr.load()
    assert L.cptr_status_string(0) == b"CPTR_OK"
    assert L.cptr_status_string(-4) == b"CPTR_ERR_SINGULAR_BLOCK"
    o = cptr.cptr_default_options()
    assert (o.first_stage, o.second_stage, o.precision, o.amg_sweeps) == (1, 2, 1, 2)
    assert abs(o.amg_theta - 0.08) < 1e-15 and o.amg_coarse_size == 512
    # the fields appended to cptr_options, in the header's order and defaults
    assert (o.amg_smooth_p_T, o.use_graph, o.resid_fp64, o.scalar_dia, o.lrn_columns, o.decoupling,
            o.ilu_level, o.schur, o.lrn_fallback, o.amg_smoother) == (0, 1, 0, 1, 1, 0, 0, 0, 1, 0)
    assert ctypes.sizeof(cptr.Options) == _options_size_from_header()
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert L.cptr_setup(ctypes.byref(h), None, None, None, None) == -1
    assert b"null" in L.cptr_last_error()


def test_binding_stage_codes_match_the_header():
    """The binding's names for the first and second stages and the decoupling
    operators carry the values the header defines."""
    from paper_1907_04229_amd import cptr
    text = open(os.path.join(ROOT, "include", "cptr.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(CPTR_\w+)\s+(-?\d+)", text)}
    first = {"none": "NONE", "cptr": "BLOCK", "cptr_lower": "BLOCK_LOWER", "cpr": "CPR",
             "cptr_bd": "BD", "cptr_uamg": "UAMG", "cptr_upper": "BLOCK_UPPER"}
    assert set(first) == set(cptr.FIRST)
    for k, v in first.items():
        assert cptr.FIRST[k] == defs["CPTR_FIRST_" + v], k
    for k, v in cptr.DECOUPLING.items():
        assert v == defs["CPTR_DECOUPLE_" + k.upper()], k
    for k, v in cptr.SECOND.items():
        assert v == defs["CPTR_SECOND_" + k.upper()], k
    for k, v in cptr.SCHUR.items():
        assert v == defs["CPTR_SCHUR_" + k.upper()], k
    for k, v in cptr.SMOOTHER.items():
        assert v == defs["CPTR_SMOOTHER_" + k.upper()], k
