"""Host analyse of the library (no GPU: host-only handle) and the C ABI surface."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import qdmf as Q
from paper_2508_04370_amd import workloads as W

from test_oracle import lp_from_dense

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(Q.LIB_PATH):
        from paper_2508_04370_amd import build as B
        B.build()
    O.build(force=False)


def host_solver(lp, perm=None, **opts):
    return Q.Solver(lp, device=-1, perm=perm, **opts)


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "qdmf.h")).read()
    declared = set(re.findall(r"\b(qdmf_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    lib = Q.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(Q.EXPORTED)


def test_options_struct_layout_matches_defaults():
    o = Q.qdmf_default_options()
    assert o.nb == 64 and o.presort == 1 and o.max_refine == 2 and o.max_refine_mixed == 3
    assert o.alpha == (1 + np.sqrt(17)) / 8 and o.eps_lift == 2.0 ** -52
    assert o.split_solve_front == 1024 and o.syrk_group_front == 1024 and o.syrk_group == 4
    assert o.target_berr == 1e-12 and o.target_berr_mixed == 1e-10 and o.tau_big == 1e-8
    assert o.f_mix == 1024 and o.small_front == 64 and o.amalgamate == 1 and o.mem_cap_bytes == 0
    assert o.syrk_tile_front == 0 and o.mixed_check == 2


@pytest.mark.parametrize("seed", range(6))
def test_matched_mode_supernodes_equal_oracle(seed):
    """With the oracle's ordering and no amalgamation, the library's postorder is the
    identity and its fundamental supernodes equal the oracle's."""
    mode = W.AS if seed % 2 else W.NE
    g = W.rng(31, seed)
    lp = W.ne_random(m=int(g.integers(20, 80)), n=int(g.integers(80, 160)), density=0.05,
                     seed=100 + seed) if mode == W.NE else \
        W.as_staircase(periods=3, rows=20 + seed, cols=40 + 2 * seed, link_cols=5, seed=100 + seed)
    S = O.Sym(lp)
    s = host_solver(lp, perm=S.perm(), amalgamate=0)
    assert np.array_equal(s.sym["perm"], S.perm())
    assert np.array_equal(s.sym["sn_ptr"], S.snptr())
    assert np.array_equal(s.sym["sn_parent"], S.snparent())
    rp, _ = S.front_rows()
    assert np.array_equal(s.sym["sn_front"], np.diff(rp))
    assert s.sym["nnz_l"] == S.nnzL and s.sym["flops_fact"] == S.flops
    s.close()


def _brute_structure(lp, perm):
    """Dense boolean elimination of the permuted pattern (independent of both analyses)."""
    A = np.zeros((lp["m"], lp["n"]), bool)
    for j in range(lp["n"]):
        A[lp["rowidx"][lp["colptr"][j]:lp["colptr"][j + 1]], j] = True
    if lp["mode"] == W.AS:
        N = lp["n"] + lp["m"]
        P = np.zeros((N, N), bool)
        P[lp["n"]:, :lp["n"]] = A
        P[:lp["n"], lp["n"]:] = A.T
    else:
        P = (A.astype(int) @ A.T.astype(int)) > 0
    np.fill_diagonal(P, True)
    Lp = np.tril(P[np.ix_(perm, perm)])
    N = len(perm)
    for k in range(N):
        rows = np.nonzero(Lp[k + 1:, k])[0] + k + 1
        for a in rows:
            Lp[rows[rows >= a], a] = True
    return Lp


@pytest.mark.parametrize("amalgamate", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_own_ordering_structure_vs_brute_force(seed, amalgamate):
    lp = W.as_staircase(periods=2, rows=15 + seed, cols=30, link_cols=4, seed=200 + seed) if seed % 2 \
        else W.ne_random(m=40, n=80, density=0.06, seed=200 + seed)
    s = host_solver(lp, amalgamate=amalgamate)
    sy = s.sym
    perm = sy["perm"]
    assert sorted(perm.tolist()) == list(range(sy["N"]))
    Lp = _brute_structure(lp, perm)
    assert sy["nnz_l"] == Lp.sum()
    cc = Lp.sum(axis=0) - 1
    assert sy["flops_fact"] == float((cc * (cc + 3)).sum())
    snp = sy["sn_ptr"]
    # every supernode's front holds the exact structure of each of its columns, parents hold
    # the children's contribution rows, and fundamental supernodes are exact
    for s_ in range(sy["nsuper"]):
        c0, c1 = snp[s_], snp[s_ + 1]
        f = sy["sn_front"][s_]
        rows_needed = set(range(c0, c1))
        for c in range(c0, c1):
            rows_needed |= set((np.nonzero(Lp[c:, c])[0] + c).tolist())
        assert len(rows_needed) <= f
        if not amalgamate:
            assert len(rows_needed) == f
        par = sy["sn_parent"][s_]
        if par >= 0:
            assert snp[par] >= c1 and sy["sn_level"][par] > sy["sn_level"][s_]
    s.close()


def test_levels_bottom_up():
    lp = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10)
    s = host_solver(lp)
    sy = s.sym
    for t in range(sy["nsuper"]):
        p = sy["sn_parent"][t]
        if p >= 0:
            assert sy["sn_level"][p] >= sy["sn_level"][t] + 1
    assert sy["nlevels"] == sy["sn_level"].max() + 1
    s.close()


def test_grid_nd_ordering_separates():
    lp = W.ne_grid(8, 6, 5, nrhs=1)
    s = host_solver(lp, ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"])
    sy = s.sym
    assert sorted(sy["perm"].tolist()) == list(range(lp["m"]))
    # nested dissection gives a wide tree: many leaves, shallow depth
    assert sy["nlevels"] < 12
    Lp = _brute_structure(lp, sy["perm"])
    assert sy["nnz_l"] == Lp.sum()
    s.close()


# ------------------------------------------------------------------ failure handling

def _expect(code, fn):
    with pytest.raises(Q.QdmfError) as ei:
        fn()
    assert ei.value.code == code


def test_bad_csc_rejected():
    lp = W.ne_random(m=20, n=40, density=0.1)
    h = Q.qdmf_create(-1, None, Q.qdmf_default_options())
    bad = lp["rowidx"].copy()
    bad[1], bad[0] = bad[0], bad[1]  # unsorted within column 0 (it has >= 2 entries?)
    cp = lp["colptr"]
    if cp[1] - cp[0] < 2:
        bad = lp["rowidx"].copy()
        bad[0] = lp["m"] + 5  # out of range
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_analyse(h, lp["m"], lp["n"], cp, bad, lp["mode"]))
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_analyse(h, lp["m"], lp["n"], cp, lp["rowidx"], 7))
    cp2 = cp.copy()
    cp2[3] = cp2[2] - 1
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_analyse(h, lp["m"], lp["n"], cp2, lp["rowidx"], lp["mode"]))
    Q.qdmf_destroy(h)


def test_bad_user_perm_rejected():
    lp = W.ne_random(m=20, n=40, density=0.1)
    o = Q.qdmf_default_options(ordering=Q.QDMF_ORDER_USER)
    h = Q.qdmf_create(-1, None, o)
    perm = np.arange(lp["m"], dtype=np.int32)
    perm[3] = perm[4]
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_analyse(h, lp["m"], lp["n"], lp["colptr"], lp["rowidx"],
                                                           lp["mode"], perm))
    Q.qdmf_destroy(h)


def test_memory_cap_gives_oom():
    lp = W.ne_random()
    o = Q.qdmf_default_options(mem_cap_bytes=1000)
    h = Q.qdmf_create(-1, None, o)
    _expect(Q.QDMF_ERR_OOM, lambda: Q.qdmf_analyse(h, lp["m"], lp["n"], lp["colptr"], lp["rowidx"], lp["mode"]))
    Q.qdmf_destroy(h)


def test_bad_options_rejected():
    for bad in (dict(mixed_check=4), dict(mixed_check=-1), dict(syrk_group=5), dict(small_front=65)):
        _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_create(-1, None, Q.qdmf_default_options(**bad)))


def test_host_only_handle_refuses_numeric_calls():
    lp = W.ne_random(m=20, n=40, density=0.1)
    s = host_solver(lp)
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_set_matrix(s.h, lp["val"]))
    _expect(Q.QDMF_ERR_NO_MATRIX, lambda: Q.qdmf_factorise(s.h, None, 0.0, 1e-8))
    s.close()


def test_order_before_analyse_is_an_error():
    h = Q.qdmf_create(-1, None, Q.qdmf_default_options())
    _expect(Q.QDMF_ERR_NOT_ANALYSED, lambda: Q.qdmf_symbolic(h))
    _expect(Q.QDMF_ERR_NOT_ANALYSED, lambda: Q.qdmf_set_matrix(h, np.zeros(1)))
    Q.qdmf_destroy(h)


def test_invalid_options_rejected():
    o = Q.qdmf_default_options(nb=32)
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_create(-1, None, o))
    o = Q.qdmf_default_options(small_front=65)
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_create(-1, None, o))
    o = Q.qdmf_default_options(split_solve_front=0)
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_create(-1, None, o))
    for bad in (dict(syrk_group=0), dict(syrk_group=5), dict(syrk_group_front=-1)):
        o = Q.qdmf_default_options(**bad)
        _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_create(-1, None, o))


@pytest.mark.parametrize("group", [1, 2, 4])
def test_grouped_windows_leave_the_symbolic_plan_unchanged(group):
    """Grouping the trailing updates changes only the launch plan: the ordering, supernodes,
    factor size and flop count stay those of the ungrouped analysis."""
    lp = W.ne_dense_front(300, seed=3)
    a = host_solver(lp, syrk_group_front=0).sym
    b = host_solver(lp, syrk_group_front=64, syrk_group=group).sym
    for key in ("N", "nnz_l", "nsuper", "max_front", "flops_fact"):
        assert a[key] == b[key], key
    assert np.array_equal(np.asarray(a["perm"]), np.asarray(b["perm"]))


def test_no_float_atomics_in_kernels():
    """Determinism by construction: the only atomics in device code set integer flags (the
    bad-Theta flag and the per-system marks of the mixed-precision FP64 redo), whose final
    value does not depend on the order of the writes."""
    src = open(os.path.join(ROOT, "paper_2508_04370_amd", "csrc", "kernels.hip")).read()
    assert not re.search(r"unsafeAtomic|atomicMax|atomicMin|atomicExch", src)
    for m in re.finditer(r"(atomic[A-Za-z]+|__hip_atomic_[a-z_]+)\s*\(([^,;]*)", src):
        target = m.group(2)
        assert re.search(r"bad_theta|D\.redo", target), m.group(0)


def degenerate(name, seed=0, nrhs=2):
    """Small systems whose K has an empty block, an isolated variable or an isolated row."""
    g = W.rng(71, seed)
    if name == "as_1x1":
        A, mode = np.array([[2.0]]), W.AS
    elif name == "as_empty_col":
        A, mode = np.array([[1.0, 0.0, 2.0], [0.5, 0.0, -1.0]]), W.AS
    elif name == "ne_empty_row":
        A, mode = np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 3.0, 1.0]]), W.NE
    elif name == "as_no_rows":
        A, mode = np.zeros((0, 5)), W.AS
    elif name == "ne_no_cols":
        A, mode = np.zeros((3, 0)), W.NE
    else:
        raise KeyError(name)
    m, n = A.shape
    theta = W.log_uniform(g, 1e-2, 1e2, n)
    if n:
        lp = lp_from_dense(A, mode, theta, 1e-8, 1e-8, name=name)
    else:
        lp = W.LP(m=m, n=0, colptr=np.zeros(1, np.int64), rowidx=np.zeros(0, np.int32), val=np.zeros(0),
                  theta=theta, rho=1e-8, delta=1e-8, mode=mode, name=name)
    lp["r1"] = np.asfortranarray(g.standard_normal((m, nrhs)))
    lp["r7"] = np.asfortranarray(g.standard_normal((n, nrhs)))
    return lp


@pytest.mark.parametrize("name", ["as_1x1", "as_empty_col", "ne_empty_row", "as_no_rows", "ne_no_cols"])
def test_degenerate_patterns_analyse_like_the_oracle(name):
    """An isolated variable, an empty row, no constraints or no variables: the host analysis
    accepts the pattern and its factor has the oracle's size."""
    lp = degenerate(name)
    s = host_solver(lp)
    S = O.Sym(lp)
    assert s.sym["N"] == S.N == (lp["n"] + lp["m"] if lp["mode"] == W.AS else lp["m"])
    assert s.sym["nnz_l"] == S.nnzL


def test_empty_system_analyses_to_nothing():
    lp = W.LP(m=0, n=0, colptr=np.zeros(1, np.int64), rowidx=np.zeros(0, np.int32), val=np.zeros(0),
              theta=np.zeros(0), rho=0.0, delta=0.0, mode=W.AS, name="empty")
    s = host_solver(lp)
    assert (s.sym["N"], s.sym["nnz_l"], s.sym["nsuper"], s.sym["max_front"]) == (0, 0, 0, 0)
