"""Quadratic programs on the GPU (qdmf_analyse_qp / qdmf_set_hessian, then factorise and solve)
against the CPU oracle through the C ABI: backward error against K_static with Q computed by
the oracle, the quasidefinite inertia, ||K||_1, the oracle's pivot sequence in matched mode,
and the diagonal-Q special case."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

from test_gpu_parity import check_against_oracle, gpu_solve, oracle_berr, system_x, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def qp_lp(kind, seed=3):
    if kind == "random":
        base = W.ne_random(m=120, n=260, density=0.03, seed=40 + seed)
        base = W.LP(dict(base, mode=W.AS, rho=1e-8, delta=1e-8,
                         r7=W.rng(41, seed).standard_normal((260, 1))))
        return W.with_hessian(base, seed=seed, window=20)
    if kind == "staircase":
        return W.with_hessian(W.as_staircase(periods=4, rows=50, cols=100, link_cols=10, seed=42 + seed),
                              seed=seed, window=30)
    if kind == "dense_front":  # strong couplings: fronts beyond one 64-column window
        base = W.as_staircase(periods=3, rows=60, cols=150, link_cols=20, seed=43 + seed)
        return W.with_hessian(base, seed=seed, frac=1.0, per_row=6, window=75)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["random", "staircase", "dense_front"])
def test_qp_fp64_against_oracle(torch_dev, kind):
    lp = qp_lp(kind)
    g = gpu_solve(torch_dev, lp)
    print(f"  {kind}: max front {g['solver'].sym['max_front']} nnz(L) {g['solver'].sym['nnz_l']}")
    check_against_oracle(lp, g)


def test_qp_full_staircase_with_hessian(torch_dev):
    """The staircase workload (20000 x 40000) with a Hessian on half of the columns."""
    lp = W.with_hessian(W.as_staircase(), seed=1, frac=0.5, per_row=3, window=50)
    g = gpu_solve(torch_dev, lp)
    fs = g["fstats"]
    assert (fs["nneg"], fs["npos"]) == (lp["n"], lp["m"])
    x = system_x(lp, g["dx"][:, 0], g["dy"][:, 0])
    nw, cw = oracle_berr(lp, lp["theta"], x, lp["r7"][:, 0], lp["r1"][:, 0])
    print(f"  staircase QP: max front {g['solver'].sym['max_front']} berr_nw={nw:.2e} "
          f"gpu={g['sstats']['berr_nw']:.2e}")
    assert nw <= 1e-12
    assert abs(nw - g["sstats"]["berr_nw"]) <= 0.1 * nw + 1e-300


def test_qp_matched_mode_reproduces_oracle_pivots(torch_dev):
    lp = W.with_hessian(W.as_staircase(periods=3, rows=40, cols=80, link_cols=8, seed=9,
                                       theta_range=(1e-1, 1e1), rho=1e-2, delta=1e-2), seed=2, window=15)
    S = O.Sym(lp)
    g = gpu_solve(torch_dev, lp, perm=S.perm(), amalgamate=0)
    s = g["solver"]
    assert np.array_equal(s.sym["sn_ptr"], S.snptr())
    ex = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"]).export()
    gd = s.export_d()
    assert np.array_equal(gd["pivot_order"], ex["fperm"])
    assert np.array_equal(gd["ptype"], ex["ptype"])
    assert np.array_equal(gd["edyn"] != 0, ex["edyn"] != 0)
    rel = np.abs(gd["d"] - ex["d"]) / np.abs(ex["d"])
    print("max relative pivot difference", rel.max())
    assert rel.max() <= 1e-12


def test_qp_mixed_precision_refines_to_target(torch_dev):
    lp = qp_lp("dense_front")
    gmx = gpu_solve(torch_dev, lp, prec=1, f_mix=65)
    assert gmx["solver"].sym["max_front"] >= 65
    x = system_x(lp, gmx["dx"][:, 0], gmx["dy"][:, 0])
    nw, _ = oracle_berr(lp, lp["theta"], x, lp["r7"][:, 0], lp["r1"][:, 0])
    print(f"  mixed QP: berr {nw:.2e} steps {gmx['sstats']['max_steps']}")
    assert nw <= 1e-10


def test_qp_diagonal_q_matches_lp_with_shifted_theta(torch_dev):
    """Q = diag(q) on the GPU against the LP with 1/Theta' = 1/Theta + q on the GPU: the same
    matrix, so the same pivots and the same solution to rounding."""
    base = W.as_staircase(periods=3, rows=40, cols=80, link_cols=8, seed=12, theta_range=(1e-2, 1e2))
    n = base["n"]
    q = W.rng(64).uniform(0.0, 2.0, n)
    lpq = W.LP(dict(base, q_colptr=np.arange(n + 1, dtype=np.int64), q_rowidx=np.arange(n, dtype=np.int32),
                    q_val=q))
    gq = gpu_solve(torch_dev, lpq)
    gl = gpu_solve(torch_dev, base, theta=1.0 / (1.0 / base["theta"] + q))
    for key in ("dx", "dy"):
        assert np.allclose(gq[key], gl[key], rtol=1e-9, atol=1e-9 * np.abs(gl[key]).max())
