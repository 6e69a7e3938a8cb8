"""Degenerate and boundary systems on the GPU path against the CPU oracle, through the C ABI
(needs an MI355X): an empty system, systems without constraints or without variables, a
variable in no constraint, a constraint on no variable, and dense fronts whose order sits on
either side of the 64-column pivot window (Section 4.4's blocked factorisation)."""
import numpy as np
import pytest

from paper_2508_04370_amd import workloads as W

from test_analyse import degenerate
from test_gpu_parity import check_against_oracle, gpu_solve, torch_dev  # noqa: F401 (fixture)
from test_oracle import lp_from_dense

pytestmark = pytest.mark.gpu


def dense_as(m, n):
    """Augmented system of a fully dense m x n A: K's largest front is dense with mixed-sign
    pivots (its order is fixed by m and n through the ordering)."""
    g = W.rng(72, m, n)
    A = g.standard_normal((m, n))
    A[A == 0] = 1.0
    lp = lp_from_dense(A, W.AS, W.log_uniform(g, 1e-3, 1e3, n), 1e-8, 1e-8, name=f"dense_as_{m}x{n}")
    lp["r1"] = np.asfortranarray(g.standard_normal((m, 1)))
    lp["r7"] = np.asfortranarray(g.standard_normal((n, 1)))
    return lp


@pytest.mark.parametrize("name", ["as_1x1", "as_empty_col", "ne_empty_row", "as_no_rows", "ne_no_cols"])
def test_degenerate_systems(torch_dev, name):
    lp = degenerate(name)
    g = gpu_solve(torch_dev, lp)
    check_against_oracle(lp, g)


def test_empty_system_is_a_no_op(torch_dev):
    """m = n = 0: factorise and solve launch nothing and report zero pivots and zero error."""
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    lp = W.LP(m=0, n=0, colptr=np.zeros(1, np.int64), rowidx=np.zeros(0, np.int32), val=np.zeros(0),
              theta=np.zeros(0), rho=1e-8, delta=1e-8, mode=W.AS, name="empty")
    print("[gpu case] empty system", flush=True)
    s = Q.Solver(lp, device=0)
    s.factorise(torch.zeros(0, dtype=torch.float64, device=dev), 1e-8, 1e-8)
    fs = s.factor_stats()
    assert (fs["nneg"], fs["npos"], fs["nzero"], fs["n2x2"]) == (0, 0, 0, 0)
    dx, dy = s.solve(None, torch.zeros((0, 3), dtype=torch.float64, device=dev))
    assert dx.shape == (0, 3) and dy.shape == (0, 3)
    ss = s.solve_stats(3)
    assert ss["berr_nw"] == 0.0 and list(ss["steps_per_rhs"]) == [0, 0, 0]
    e = torch.zeros((0, 1), dtype=torch.float64, device=dev)
    with pytest.raises(Q.QdmfError) as err:
        Q.qdmf_graph_capture(s.h, e[:, 0], 1e-8, 1e-8, 0, 1, 1, None, e, e, e)
    assert err.value.code == Q.QDMF_ERR_INVALID_ARG


@pytest.mark.parametrize("f", [63, 64, 65, 127, 128, 129])
def test_dense_ne_front_at_window_boundaries(torch_dev, f):
    """One dense positive definite front of order f (normal equations [I | G]): the last pivot
    window is full, one column short, or one column long."""
    lp = W.ne_dense_front(f, seed=f, nrhs=2)
    g = gpu_solve(torch_dev, lp)
    assert g["solver"].sym["max_front"] == f
    check_against_oracle(lp, g)


# (m, n) -> order of the largest front under the default ordering
AS_BOUNDARY = {(30, 33): 63, (31, 33): 64, (31, 34): 65, (61, 66): 127, (61, 67): 128, (62, 67): 129}


@pytest.mark.parametrize("mn", sorted(AS_BOUNDARY))
def test_dense_as_at_window_boundaries(torch_dev, mn):
    """Dense augmented systems with mixed-sign pivots whose largest front has order 63..65 or
    127..129; inertia (n negative, m positive) and solution against the oracle."""
    lp = dense_as(*mn)
    g = gpu_solve(torch_dev, lp)
    assert g["solver"].sym["max_front"] == AS_BOUNDARY[mn]
    check_against_oracle(lp, g)
