"""Choice between the normal equations and the augmented system (host logic): the count of
the normal-equations pattern against a brute-force product of the boolean pattern, the early
stop of that count, dense columns, and the flops comparison against separate analyses."""
import os

import numpy as np
import pytest

from paper_2508_04370_amd import qdmf as Q
from paper_2508_04370_amd import workloads as W


@pytest.fixture(scope="module")
def h():
    if not os.path.exists(Q.LIB_PATH):
        from paper_2508_04370_amd import build as B
        B.build()
    hh = Q.qdmf_create(-1, None, Q.qdmf_default_options())
    yield hh
    Q.qdmf_destroy(hh)


def ne_pattern_brute(m, n, colptr, rowidx):
    """Lower entries with the diagonal of pattern(A A^T) + I, by a dense boolean product."""
    B = np.zeros((m, n), dtype=np.int64)
    for j in range(n):
        B[rowidx[colptr[j]:colptr[j + 1]], j] = 1
    P = (B @ B.T) > 0
    np.fill_diagonal(P, True)
    return int(np.tril(P).sum())


def csc_from_columns(m, cols):
    colptr = np.zeros(len(cols) + 1, np.int64)
    colptr[1:] = np.cumsum([len(c) for c in cols])
    rowidx = np.concatenate([np.sort(np.asarray(c, np.int32)) for c in cols]).astype(np.int32)
    return colptr, rowidx


@pytest.mark.parametrize("case", ["ne_random", "staircase"])
def test_choice_follows_flops_and_counts_are_exact(h, case):
    lp = W.ne_random() if case == "ne_random" else W.as_staircase(periods=4, rows=50, cols=100, link_cols=10)
    m, n = lp["m"], lp["n"]
    c = Q.qdmf_choose_mode(h, m, n, lp["colptr"], lp["rowidx"])
    assert c["ndense"] == 0 and c["ne_abandoned"] == 0
    assert c["nnz_ne_pattern"] == ne_pattern_brute(m, n, lp["colptr"], lp["rowidx"])
    # the same numbers as the two analyses on their own
    sa = Q.Solver(dict(lp, mode=W.AS), device=-1)
    sn = Q.Solver(dict(lp, mode=W.NE), device=-1)
    assert (c["nnz_l_as"], c["flops_as"]) == (sa.sym["nnz_l"], sa.sym["flops_fact"])
    assert (c["nnz_l_ne"], c["flops_ne"]) == (sn.sym["nnz_l"], sn.sym["flops_fact"])
    sa.close()
    sn.close()
    assert c["mode"] == (W.NE if c["flops_ne"] <= c["flops_as"] else W.AS)


def test_dense_column_rules_out_the_normal_equations(h):
    g = W.rng(91)
    m, n = 300, 600
    cols = [g.choice(m, 3, replace=False) for _ in range(n)]
    cols[17] = np.arange(0, m, 4)  # 75 entries >= max(64, m / 10)
    cp, ri = csc_from_columns(m, cols)
    c = Q.qdmf_choose_mode(h, m, n, cp, ri)
    assert c["ndense"] == 1 and c["ne_abandoned"] == 1 and c["mode"] == W.AS
    assert c["nnz_ne_pattern"] == -1 and c["nnz_l_ne"] == -1 and c["flops_ne"] == -1.0
    # one entry fewer: no longer dense, and the choice goes by the analyses again
    cols[17] = np.arange(0, m, 4)[:63]
    cp, ri = csc_from_columns(m, cols)
    c = Q.qdmf_choose_mode(h, m, n, cp, ri)
    assert c["ndense"] == 0


def test_normal_equations_given_up_when_their_pattern_outgrows_the_as_factor(h):
    """Many medium columns: every column's rows form a clique in A A^T, while the augmented
    system eliminates the rows first.  The count stops at the first entry past nnz(L_AS)."""
    g = W.rng(92)
    m, n = 2000, 200
    cols = [g.choice(m, 50, replace=False) for _ in range(n)]
    cp, ri = csc_from_columns(m, cols)
    c = Q.qdmf_choose_mode(h, m, n, cp, ri)
    full = ne_pattern_brute(m, n, cp, ri)
    assert full > c["nnz_l_as"]
    assert c["ne_abandoned"] == 1 and c["mode"] == W.AS and c["ndense"] == 0
    assert c["nnz_ne_pattern"] == c["nnz_l_as"] + 1
    assert c["nnz_l_ne"] == -1


def test_choice_needs_a_pattern_ordering():
    lp = W.ne_random()
    for o in (Q.QDMF_ORDER_USER, Q.QDMF_ORDER_GRID_ND):
        hh = Q.qdmf_create(-1, None, Q.qdmf_default_options(ordering=o))
        with pytest.raises(Q.QdmfError) as ei:
            Q.qdmf_choose_mode(hh, lp["m"], lp["n"], lp["colptr"], lp["rowidx"])
        assert ei.value.code == Q.QDMF_ERR_INVALID_ARG
        Q.qdmf_destroy(hh)
