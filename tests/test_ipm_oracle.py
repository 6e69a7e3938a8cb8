"""The reference interior point method (oracle/ipm.py) against what fixes it independently:
the optimum of SciPy's HiGHS on feasible LPs, a textbook LP with a known solution, the full
(unreduced) Newton system for the reduced direction, and its own termination test."""
import numpy as np
import pytest

from oracle import ipm as I
from paper_2508_04370_amd import workloads as W

scipy_optimize = pytest.importorskip("scipy.optimize")


@pytest.mark.parametrize("m,n,d,seed", [(50, 100, 0.05, 0), (120, 300, 0.02, 1), (80, 240, 0.03, 2)])
def test_optimum_matches_highs(m, n, d, seed):
    base = W.ne_random(m=m, n=n, density=d, seed=10 + seed)
    lp, b, c = W.feasible_lp(base, seed=seed)
    A = W.lp_dense(lp)
    r = I.ipm(A, b, c, k=2)
    ref = scipy_optimize.linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert r["status"] == "optimal" and ref.status == 0
    assert abs(r["fp"] - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    assert np.all(r["x"] > 0) and np.all(r["z"] > 0)


def test_textbook_lp():
    """max 3 x1 + 5 x2 s.t. x1 <= 4, 2 x2 <= 12, 3 x1 + 2 x2 <= 18 (slacks x3..x5): the
    optimum is x = (2, 6) with value 36."""
    A = np.array([[1.0, 0, 1, 0, 0], [0, 2, 0, 1, 0], [3, 2, 0, 0, 1]])
    b = np.array([4.0, 12, 18])
    c = np.array([-3.0, -5, 0, 0, 0])
    r = I.ipm(A, b, c, k=1)
    assert r["status"] == "optimal"
    assert abs(r["fp"] + 36.0) <= 1e-6
    assert np.allclose(r["x"][:2], [2.0, 6.0], atol=1e-5)


def test_reduced_direction_solves_the_full_newton_system():
    """Without regularisation the direction from the augmented system satisfies
    A dx = r1, A^T dy + dz = r4 and Z dx + X dz = r5."""
    g = W.rng(33)
    base = W.ne_random(m=40, n=90, density=0.08, seed=33)
    lp, b, c = W.feasible_lp(base, seed=3)
    A = W.lp_dense(lp)
    x, z, y = g.uniform(0.1, 2, 90), g.uniform(0.1, 2, 90), g.standard_normal(40)
    r1, r4, r5 = b - A @ x, c - A.T @ y - z, g.standard_normal(90)
    dx, dy, dz = I.newton_direction(A, x, z, z / x, 0.0, r1, r4, r5)
    scale = 1 + np.abs(A).sum() * max(np.abs(dx).max(), np.abs(dy).max())
    assert np.abs(A @ dx - r1).max() <= 1e-10 * scale
    assert np.abs(A.T @ dy + dz - r4).max() <= 1e-10 * scale
    assert np.abs(z * dx + x * dz - r5).max() <= 1e-10 * scale


def test_iterations_reduce_mu_and_end_feasible():
    base = W.ne_random(m=60, n=150, density=0.04, seed=44)
    lp, b, c = W.feasible_lp(base, seed=4)
    A = W.lp_dense(lp)
    r = I.ipm(A, b, c, k=3)
    mus = [h[0] for h in r["history"]]
    assert all(mus[i + 1] < mus[i] for i in range(len(mus) - 1))
    ok, _, _ = I.converged(A, b, c, r["x"], r["y"], r["z"], 1e-8)
    assert ok


def test_corrector_count_bounds():
    assert I.corrector_count(1000, 10.0, 2, 1.0, 6) == 1  # cheap factorisation: the minimum
    assert I.corrector_count(1000, 1e12, 2, 1.0, 6) == 6  # dear factorisation: the maximum
    ks = [I.corrector_count(1000, f, 1, 1.0, 50) for f in (1e4, 1e5, 1e6, 1e7)]
    assert ks == sorted(ks)
