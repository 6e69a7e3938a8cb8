"""The reference interior point method (oracle/ipm.py) against what fixes it independently:
the optimum of SciPy's HiGHS on feasible LPs with and without bounds, textbook LPs with known
solutions, the full (unreduced) Newton system of Section 3 for the reduced direction, and its
own termination test."""
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
    assert np.all(r["x"] > 0) and np.all(r["zl"] > 0)


def highs_bounds(l, u):
    return [(lo, None if np.isinf(hi) else hi) for lo, hi in zip(l, u)]


@pytest.mark.parametrize("m,n,d,seed,upper", [(50, 100, 0.05, 0, 0.5), (120, 300, 0.02, 1, 1.0),
                                              (80, 240, 0.03, 2, 0.2)])
def test_bounded_optimum_matches_highs(m, n, d, seed, upper):
    base = W.ne_random(m=m, n=n, density=d, seed=20 + seed)
    lp, b, c, l, u = W.bounded_lp(base, seed=seed, upper=upper)
    A = W.lp_dense(lp)
    r = I.ipm(A, b, c, l, u, k=2)
    ref = scipy_optimize.linprog(c, A_eq=A, b_eq=b, bounds=highs_bounds(l, u), method="highs")
    assert r["status"] == "optimal" and ref.status == 0
    assert abs(r["fp"] - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    hasu = np.isfinite(u)
    assert np.all(r["x"] > l) and np.all(r["x"][hasu] < u[hasu])
    assert np.all(r["zl"] > 0) and np.all(r["zu"][hasu] > 0) and np.all(r["zu"][~hasu] == 0)


def test_textbook_lp_with_bounds():
    """min -x1 - 2 x2 s.t. x1 + x2 + s = 2, -1 <= x1 <= 1.5, 0 <= x2 <= 1, s >= 0: x2 sits at
    its upper bound, x1 = 1, s = 0, value -3; the dual is y = -1, z^l_s = 1, z^u_2 = 1."""
    A = np.array([[1.0, 1.0, 1.0]])
    b = np.array([2.0])
    c = np.array([-1.0, -2.0, 0.0])
    l = np.array([-1.0, 0.0, 0.0])
    u = np.array([1.5, 1.0, np.inf])
    r = I.ipm(A, b, c, l, u, k=1)
    assert r["status"] == "optimal"
    assert abs(r["fp"] + 3.0) <= 1e-6
    assert np.allclose(r["x"], [1.0, 1.0, 0.0], atol=1e-6)
    assert np.allclose(r["y"], [-1.0], atol=1e-6)
    assert np.allclose(r["zl"], [0.0, 0.0, 1.0], atol=1e-6)
    assert np.allclose(r["zu"], [0.0, 1.0, 0.0], atol=1e-6)


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
    """Without regularisation the direction from the augmented system and the recovery solves
    the unreduced Newton system of Section 3 with bounds, assembled here as one dense matrix in
    the unknowns (dx, dx^l, dx^u, dy, dz^l, dz^u):
    A dx = r1, dx - dx^l = r2, dx + dx^u = r3, A^T dy + dz^l - dz^u = r4,
    Z^l dx^l + X^l dz^l = r5, Z^u dx^u + X^u dz^u = r6."""
    g = W.rng(33)
    m, n = 40, 90
    base = W.ne_random(m=m, n=n, density=0.08, seed=33)
    lp, b, c, l, u = W.bounded_lp(base, seed=3, upper=1.0)  # every upper bound finite
    A = W.lp_dense(lp)
    s = I.State(g.uniform(-1, 1, n), g.uniform(0.1, 2, n), g.uniform(0.1, 2, n), g.standard_normal(m),
                g.uniform(0.1, 2, n), g.uniform(0.1, 2, n))
    hasu = np.ones(n, bool)
    r1, r2, r3, r4, r5, r6 = (g.standard_normal(m),) + tuple(g.standard_normal(n) for _ in range(5))
    tinv = s.zl / s.xl + s.zu / s.xu
    d = I.newton_direction(A, s, hasu, tinv, 0.0, r1, r2, r3, r4, r5, r6)
    Z, E = np.zeros, np.eye(n)
    blocks = [
        [A, Z((m, n)), Z((m, n)), Z((m, m)), Z((m, n)), Z((m, n))],
        [E, -E, Z((n, n)), Z((n, m)), Z((n, n)), Z((n, n))],
        [E, Z((n, n)), E, Z((n, m)), Z((n, n)), Z((n, n))],
        [Z((n, n)), Z((n, n)), Z((n, n)), A.T, E, -E],
        [Z((n, n)), np.diag(s.zl), Z((n, n)), Z((n, m)), np.diag(s.xl), Z((n, n))],
        [Z((n, n)), Z((n, n)), np.diag(s.zu), Z((n, m)), Z((n, n)), np.diag(s.xu)],
    ]
    M = np.block(blocks)
    v = np.concatenate([d.x, d.xl, d.xu, d.y, d.zl, d.zu])
    rhs = np.concatenate([r1, r2, r3, r4, r5, r6])
    scale = 1 + np.abs(M).sum(axis=1).max() * np.abs(v).max()
    assert np.abs(M @ v - rhs).max() <= 1e-10 * scale


def test_standard_form_is_the_special_case_without_bounds():
    """l = 0 and u = +inf reduce the bounded method to min c^T x, A x = b, x >= 0: the same
    iterates whether the bounds are given explicitly or left at their defaults."""
    base = W.ne_random(m=40, n=90, density=0.06, seed=35)
    lp, b, c = W.feasible_lp(base, seed=6)
    A = W.lp_dense(lp)
    r0 = I.ipm(A, b, c, k=2)
    r1 = I.ipm(A, b, c, np.zeros(90), np.full(90, np.inf), k=2)
    assert r0["iters"] == r1["iters"]
    assert np.array_equal(r0["x"], r1["x"]) and np.array_equal(r0["y"], r1["y"])
    assert np.all(r0["zu"] == 0)


def test_iterations_reduce_mu_and_end_feasible():
    base = W.ne_random(m=60, n=150, density=0.04, seed=44)
    lp, b, c = W.feasible_lp(base, seed=4)
    A = W.lp_dense(lp)
    r = I.ipm(A, b, c, k=3)
    mus = [h[0] for h in r["history"]]
    assert all(mus[i + 1] < mus[i] for i in range(len(mus) - 1))
    ok, _, _ = I.converged(A, b, c, np.zeros(150), np.full(150, np.inf), r["state"], 1e-8)
    assert ok


def test_corrector_count_bounds():
    assert I.corrector_count(1000, 10.0, 2, 1.0, 6) == 1  # cheap factorisation: the minimum
    assert I.corrector_count(1000, 1e12, 2, 1.0, 6) == 6  # dear factorisation: the maximum
    ks = [I.corrector_count(1000, f, 1, 1.0, 50) for f in (1e4, 1e5, 1e6, 1e7)]
    assert ks == sorted(ks)


# ---------------------------------------------------------------- quadratic programs

def test_textbook_qp():
    """min (x1^2 + x2^2)/2 - 2 x1 s.t. x1 + x2 + s = 1, x >= 0: the unconstrained minimiser
    x1 = 2 is cut off, so x = (1, 0, 0) with value -1.5; the dual is y = -1, z = (0, 1, 1)."""
    A = np.array([[1.0, 1.0, 1.0]])
    b = np.array([1.0])
    c = np.array([-2.0, 0.0, 0.0])
    Qm = np.diag([1.0, 1.0, 0.0])
    r = I.ipm(A, b, c, k=1, Q=Qm)
    assert r["status"] == "optimal"
    assert abs(r["fp"] + 1.5) <= 1e-6
    assert np.allclose(r["x"], [1.0, 0.0, 0.0], atol=1e-6)
    assert np.allclose(r["y"], [-1.0], atol=1e-6)
    assert np.allclose(r["zl"], [0.0, 1.0, 1.0], atol=1e-6)


def kkt_violation(A, b, c, Qm, l, u, x, y, zl, zu):
    """Largest violation of the optimality conditions of the convex QP, written out here:
    A x = b, l <= x <= u, c + Q x - A^T y - z^l + z^u = 0, z >= 0, (x - l) z^l = (u - x) z^u = 0."""
    hasu = np.isfinite(u)
    v = [np.abs(A @ x - b).max(), np.maximum(l - x, 0).max(), np.maximum(x - u, 0)[hasu].max(initial=0.0),
         np.abs(c + Qm @ x - A.T @ y - zl + zu).max(), np.maximum(-zl, 0).max(), np.maximum(-zu, 0).max(),
         np.abs((x - l) * zl).max(), np.abs(np.where(hasu, (np.where(hasu, u, 0.0) - x) * zu, 0.0)).max()]
    return max(v)


@pytest.mark.parametrize("m,n,d,seed,upper", [(30, 70, 0.08, 0, 0.5), (60, 150, 0.04, 1, 0.0)])
def test_qp_optimum_satisfies_kkt(m, n, d, seed, upper):
    base = W.ne_random(m=m, n=n, density=d, seed=50 + seed)
    lpq = W.with_hessian(W.LP(dict(base, mode=W.AS)), seed=seed, window=8)
    lp, b, c, l, u = W.bounded_lp(lpq, seed=seed, upper=upper)
    A, Qm = W.lp_dense(lp), W.q_dense(lpq)
    r = I.ipm(A, b, c, l, u, k=2, Q=Qm)
    assert r["status"] == "optimal"
    scale = 1 + max(np.abs(b).max(), np.abs(c).max())
    assert kkt_violation(A, b, c, Qm, l, u, r["x"], r["y"], r["zl"], r["zu"]) <= 1e-6 * scale
    # the gap of the termination test is the duality gap of the QP
    assert abs(r["fp"] - r["fd"]) <= 1e-7 * (1 + abs(r["fp"]))


def test_qp_with_far_bounds_is_the_equality_constrained_minimiser():
    """With Q positive definite and every bound far from the optimum, the QP's solution is that
    of the linear KKT system [[Q, -A^T], [A, 0]] [x; y] = [-c; b] (LAPACK)."""
    base = W.ne_random(m=25, n=60, density=0.1, seed=57)
    lpq = W.with_hessian(W.LP(dict(base, mode=W.AS)), seed=4, frac=1.0, window=6, ridge=1.0)
    A, Qm = W.lp_dense(lpq), W.q_dense(lpq)
    g = W.rng(58)
    m, n = A.shape
    b, c = A @ g.uniform(-1, 1, n), g.standard_normal(n)
    K = np.block([[Qm, -A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-c, b]))
    x_star, y_star = sol[:n], sol[n:]
    l = np.full(n, x_star.min() - 1e3)
    r = I.ipm(A, b, c, l, k=2, Q=Qm)
    assert r["status"] == "optimal"
    assert np.allclose(r["x"], x_star, atol=1e-6 * (1 + np.abs(x_star).max()))
    assert np.allclose(r["y"], y_star, atol=1e-6 * (1 + np.abs(y_star).max()))


def test_reduced_qp_direction_solves_the_full_newton_system():
    """The direction of a quadratic program against the unreduced Newton system, whose dual row
    reads -Q dx + A^T dy + dz^l - dz^u = r4."""
    g = W.rng(34)
    m, n = 30, 70
    base = W.ne_random(m=m, n=n, density=0.08, seed=34)
    lpq = W.with_hessian(W.LP(dict(base, mode=W.AS)), seed=5, window=8)
    A, Qm = W.lp_dense(lpq), W.q_dense(lpq)
    s = I.State(g.uniform(-1, 1, n), g.uniform(0.1, 2, n), g.uniform(0.1, 2, n), g.standard_normal(m),
                g.uniform(0.1, 2, n), g.uniform(0.1, 2, n))
    hasu = np.ones(n, bool)
    r1, r2, r3, r4, r5, r6 = (g.standard_normal(m),) + tuple(g.standard_normal(n) for _ in range(5))
    d = I.newton_direction(A, s, hasu, s.zl / s.xl + s.zu / s.xu, 0.0, r1, r2, r3, r4, r5, r6, Qm)
    assert np.abs(A @ d.x - r1).max() <= 1e-9
    assert np.abs(d.x - d.xl - r2).max() <= 1e-9 and np.abs(d.x + d.xu - r3).max() <= 1e-9
    assert np.abs(-Qm @ d.x + A.T @ d.y + d.zl - d.zu - r4).max() <= 1e-9 * (1 + np.abs(d.y).max())
    assert np.abs(s.zl * d.xl + s.xl * d.zl - r5).max() <= 1e-9
    assert np.abs(s.zu * d.xu + s.xu * d.zu - r6).max() <= 1e-9
