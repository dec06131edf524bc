"""The library's setup (built for the host) against the oracle, on the CPU.

Aggregation, numbering, the Galerkin coarse operators and the ILU(0) level /
colour schedules must be bit-identical: both sides take every floating-point
decision in FP64 in the same stated order, without contraction."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_04229_amd import setup_host as H
from paper_1907_04229_amd.synth import make_problem


@pytest.fixture(scope="module", autouse=True)
def _built():
    try:
        H.load()
    except ImportError:
        from paper_1907_04229_amd import build
        build.build_host()


CASES = [
    dict(shape=(8, 7, 5), kind="gaussian", sigma=1.5, corr_len=3.0, seed=12),
    dict(shape=(16, 12, 6), kind="iid", sigma=1.0, seed=3, heater=True),
    dict(shape=(12, 10, 8), kind="gaussian", sigma=2.5, corr_len=4.0, seed=4, three_phase=True),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("which", [0, 1])
def test_amg_hierarchy_bit_exact(case, which, oracle_lib):
    pr = make_problem(**CASES[case])
    nv = pr.nv
    if which == 0:
        v = np.ascontiguousarray(pr.vals.reshape(-1, nv, nv)[:, 0, 0])
        rp, ci = pr.row_ptr, pr.col_idx
    else:
        rp, ci, v = pr.st_row_ptr, pr.st_col_idx, pr.st_vals
    for seed, smooth in ((0, True), (5, True), (0, False)):
        o = O.Oracle.from_problem(pr, first="cptr", second="none", coarse_size=16, seed=seed,
                                  smooth_p=smooth, smooth_p_T=smooth)
        ref = o.amg_levels(which)
        got = H.amg_levels(rp, ci, v, coarse_size=16, seed=seed, smooth_p=smooth)
        assert len(got) == len(ref) >= 2
        for a, b in zip(got, ref):
            assert a["n"] == b["n"]
            for x, y in zip(a["A"], b["A"]):
                assert np.array_equal(x, y)            # bit-identical coarse operators
            if "agg" in b:
                assert np.array_equal(a["agg"], b["agg"])
                assert a["omega"] == b["omega"]
                for x, y in zip(a["P"], b["P"]):
                    assert np.array_equal(x, y)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_unknown_based_hierarchy_bit_exact(case, oracle_lib):
    # the coupled pressure-temperature hierarchy of the unknown-based stage
    pr = make_problem(**CASES[case])
    for seed, smooth, smooth_T in ((0, True, False), (5, True, True), (0, False, False)):
        o = O.Oracle.from_problem(pr, first="cptr_uamg", second="none", coarse_size=16, seed=seed,
                                  smooth_p=smooth, smooth_p_T=smooth_T)
        ref = o.amg_levels(0)
        rp, ci, v = ref[0]["A"]
        got = H.uamg_levels(rp, ci, v, pr.n, coarse_size=16, seed=seed, smooth_p=smooth,
                            smooth_p_T=smooth_T)
        assert len(got) == len(ref) >= 2
        for a, b in zip(got, ref):
            assert a["n"] == b["n"]
            for x, y in zip(a["A"], b["A"]):
                assert np.array_equal(x, y)            # bit-identical coarse operators
            if "agg" in b:
                assert np.array_equal(a["agg"], b["agg"])
                assert a["omega"] == b["omega"]
                for x, y in zip(a["P"], b["P"]):
                    assert np.array_equal(x, y)


@pytest.mark.parametrize("mc", [False, True])
@pytest.mark.parametrize("level", [0, 1])
def test_ilu_schedule_matches_oracle(mc, level, oracle_lib):
    # BILU(0) and BILU(1): factor order, level sets of both sweeps, colours,
    # bit for bit; the factors to rounding
    pr = make_problem(shape=(7, 6, 5), kind="iid", seed=9, three_phase=True)
    o = O.Oracle.from_problem(pr, first="none", second="bilu0_mc" if mc else "bilu0", ilu_level=level)
    ref = o.ilu()
    got = H.ilu_schedule(pr.row_ptr, pr.col_idx, pr.vals, pr.nv, mc, level)
    assert np.array_equal(got["order"], ref["perm"])
    cells = ref["perm"]
    assert np.array_equal(got["lev_lower"][cells], ref["lev_lower"])
    assert np.array_equal(got["lev_upper"][cells], ref["lev_upper"])
    if mc:
        assert got["ncolor"] == ref["ncolor"]
        assert np.array_equal(got["color"], ref["color"])
    # the FP64 factors agree to rounding (same algorithm, same order)
    nv = pr.nv
    d_ref = ref["dinv"].reshape(-1, nv, nv)
    d_got = got["dinv"].reshape(-1, nv, nv)[cells]
    assert np.abs(d_ref - d_got).max() <= 1e-12 * np.abs(d_ref).max()


@pytest.mark.parametrize("mc", [False, True])
@pytest.mark.parametrize("parts", [(2, 2, 1), (3, 2, 2)])
def test_partitioned_ilu_matches_oracle(mc, parts, oracle_lib):
    # block Jacobi over grid parts: the library's grid partition is the one
    # written out here from the cell coordinates, and the factor order, level
    # sets, colours and factors match the oracle's ILU with that partition
    pr = make_problem(shape=(7, 6, 5), kind="iid", seed=9, three_phase=True)
    nx, ny, nz = pr.shape
    i = np.arange(pr.n)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    px, py, pz = parts
    part = (x * px // nx + px * (y * py // ny + py * (z * pz // nz))).astype(np.int32)
    o = O.Oracle.from_problem(pr, first="none", second="bilu0_mc" if mc else "bilu0", ilu_part=part)
    ref = o.ilu()
    got = H.ilu_schedule(pr.row_ptr, pr.col_idx, pr.vals, pr.nv, mc, 0, parts=parts)
    assert np.array_equal(got["order"], ref["perm"])
    cells = ref["perm"]
    assert np.array_equal(got["lev_lower"][cells], ref["lev_lower"])
    assert np.array_equal(got["lev_upper"][cells], ref["lev_upper"])
    if not mc:
        # natural order on a box of a x b x c cells: a + b + c - 2 levels
        assert got["lev_lower"].max() + 1 == max(-(-nx // px) + -(-ny // py) + -(-nz // pz) - 2, 1)
    nv = pr.nv
    d_ref = ref["dinv"].reshape(-1, nv, nv)
    d_got = got["dinv"].reshape(-1, nv, nv)[cells]
    assert np.abs(d_ref - d_got).max() <= 1e-12 * np.abs(d_ref).max()
    # no factor block couples two parts
    frp, fci = got["frp"], got["fci"]
    for p in range(pr.n):
        assert (part[cells[fci[frp[p]:frp[p + 1]]]] == part[cells[p]]).all()


def test_grid_parts_reject_other_patterns():
    pr = make_problem(shape=(7, 6, 5), kind="iid", seed=9)
    with pytest.raises(RuntimeError):
        H.ilu_schedule(pr.row_ptr, pr.col_idx, pr.vals, pr.nv, False, 0, parts=(8, 1, 1))   # more parts than cells
    chain = make_problem(shape=(9, 1, 1), kind="iid", seed=3)
    with pytest.raises(RuntimeError):
        H.ilu_schedule(chain.row_ptr, chain.col_idx, chain.vals, chain.nv, False, 0, parts=(2, 1, 1))


@pytest.mark.parametrize("mc", [False, True])
@pytest.mark.parametrize("level", [0, 1])
def test_ilu_refactorisation_pattern_is_consistent(mc, level):
    # what the GPU refactorisation indexes: the forward levels order every row
    # after the rows it reads, each factor block lands in exactly one block of
    # the two sweeps, and each starts from its own block of A (or from zero)
    pr = make_problem(shape=(7, 6, 5), kind="iid", seed=9, three_phase=True)
    f = H.ilu_schedule(pr.row_ptr, pr.col_idx, pr.vals, pr.nv, mc, level)
    n, order = pr.n, f["order"]
    frp, fci, src, dpos, dst, fwd, flp = (f[k] for k in ("frp", "fci", "src", "dpos", "dst", "fwd", "f_lev_ptr"))
    assert sorted(fwd) == list(range(n)) and flp[0] == 0 and flp[-1] == n
    lev = np.empty(n, int)
    for l in range(flp.size - 1):
        lev[fwd[flp[l]:flp[l + 1]]] = l
    nf = nb = 0
    seen_f, seen_b, seen_a = set(), set(), set()
    for p in range(n):
        row = fci[frp[p]:frp[p + 1]]
        assert (np.diff(row) > 0).all() and fci[dpos[p]] == p
        for k in range(frp[p], frp[p + 1]):
            if k < dpos[p]:
                assert lev[fci[k]] < lev[p]
                assert dst[k] >= 0 and dst[k] not in seen_f
                seen_f.add(dst[k])
            elif k > dpos[p]:
                assert dst[k] <= -2 and -dst[k] - 2 not in seen_b
                seen_b.add(-dst[k] - 2)
            else:
                assert dst[k] == -1
            if src[k] >= 0:
                i = order[p]
                assert pr.row_ptr[i] <= src[k] < pr.row_ptr[i + 1] and pr.col_idx[src[k]] == order[fci[k]]
                seen_a.add(src[k])
    assert seen_f == set(range(f["n_fwd_blocks"])) and seen_b == set(range(f["n_bwd_blocks"]))
    assert seen_a == set(range(pr.row_ptr[-1]))           # every block of A is used once
    assert ((src < 0).sum() > 0) == (level == 1)          # fill blocks only with ILU(1)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("schur", ["att", "diag"])
def test_algebraic_schur_bit_exact(case, schur, oracle_lib):
    # the library's S~_T from A (Section 3.3.1) against the oracle's, bit for bit
    pr = make_problem(**CASES[case])
    o = O.Oracle.from_problem(pr, first="cptr", second="none", coarse_size=10_000, schur=schur)
    ref = o.amg_levels(1)[0]["A"]
    got = H.schur_algebraic(pr.row_ptr, pr.col_idx, pr.vals, pr.nv, diag=schur == "diag")
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
