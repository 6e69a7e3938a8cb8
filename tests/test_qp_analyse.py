"""Host analyse of quadratic programs (no GPU: host-only handle): Q's couplings in the pattern
against the oracle's fundamental supernodes and against brute-force elimination, and the
argument checks of the Q pattern."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import qdmf as Q
from paper_2508_04370_amd import workloads as W

from test_analyse import _expect
from test_oracle import brute_symbolic, dense_A, random_lp


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(Q.LIB_PATH):
        from paper_2508_04370_amd import build as B
        B.build()
    O.build(force=False)


def qp_cases(seed):
    if seed % 2:
        base = W.as_staircase(periods=3, rows=20 + seed, cols=40 + 2 * seed, link_cols=5, seed=300 + seed)
    else:
        base = random_lp(600 + seed, 25, 60, 0.08, W.AS)
    return W.with_hessian(base, seed=seed, window=6)


def qp_pattern(lp):
    A = dense_A(lp) != 0
    m, n = A.shape
    P = np.zeros((n + m, n + m), bool)
    P[n:, :n] = A
    P[:n, n:] = A.T
    P[:n, :n] = W.q_dense(lp) != 0
    np.fill_diagonal(P, True)
    return P


@pytest.mark.parametrize("seed", range(4))
def test_matched_mode_qp_supernodes_equal_oracle(seed):
    lp = qp_cases(seed)
    S = O.Sym(lp)
    s = Q.Solver(lp, device=-1, perm=S.perm(), amalgamate=0)
    assert np.array_equal(s.sym["perm"], S.perm())
    assert np.array_equal(s.sym["sn_ptr"], S.snptr())
    assert np.array_equal(s.sym["sn_parent"], S.snparent())
    assert s.sym["nnz_l"] == S.nnzL and s.sym["flops_fact"] == S.flops
    s.close()


@pytest.mark.parametrize("seed", range(4))
def test_own_ordering_qp_structure_vs_brute_force(seed):
    lp = qp_cases(seed)
    s = Q.Solver(lp, device=-1, amalgamate=0)
    sy = s.sym
    L, _, cc = brute_symbolic(qp_pattern(lp), sy["perm"])
    assert sy["nnz_l"] == L.sum()
    assert sy["nnz_k"] == np.tril(qp_pattern(lp)).sum()
    s.close()


def test_bad_q_pattern_rejected():
    lp = qp_cases(0)
    h = Q.qdmf_create(-1, None, Q.qdmf_default_options())
    args = (lp["m"], lp["n"], lp["colptr"], lp["rowidx"])
    qcp, qri = lp["q_colptr"], lp["q_rowidx"]
    upper = qri.copy()
    j = int(np.flatnonzero(np.diff(qcp) >= 2)[-1])
    upper[qcp[j]] = j - 1 if j > 0 else lp["n"]  # above the diagonal (or out of range)
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_analyse_qp(h, *args, qcp, upper))
    uns = qri.copy()
    uns[qcp[j]], uns[qcp[j] + 1] = uns[qcp[j] + 1], uns[qcp[j]]
    _expect(Q.QDMF_ERR_INVALID_ARG, lambda: Q.qdmf_analyse_qp(h, *args, qcp, uns))
    Q.qdmf_analyse_qp(h, *args, qcp, qri)  # the good pattern is accepted
    Q.qdmf_destroy(h)
