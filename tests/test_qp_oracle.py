"""Pins of the CPU oracle for quadratic programs: the (1,1) block of the augmented system becomes
-(Q + Theta^-1 + rho I).  Each test names what fixes the expected value: brute-force
elimination of the pattern, LAPACK on the dense matrix written from its definition, eigenvalue
counts (quasidefiniteness keeps the LP's inertia), and the special case of a diagonal Q, which
is the LP with 1/Theta_j replaced by 1/Theta_j + Q_jj."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

from test_oracle import brute_symbolic, dense_A, random_lp

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def qp(seed, m=30, n=70, density=0.08, frac=0.6, window=10, trange=(1e-3, 1e3)):
    lp = random_lp(500 + seed, m, n, density, W.AS, trange=trange)
    return W.with_hessian(lp, seed=seed, frac=frac, window=window)


def dense_K_qp(lp, theta, rho, delta):
    """K_static = [[-(Q + diag(1/Theta) + rho I), A^T], [A, delta I]] from its definition."""
    A = dense_A(lp)
    m, n = A.shape
    Q = W.q_dense(lp)
    return np.block([[-(Q + np.diag(1.0 / theta + rho)), A.T], [A, delta * np.eye(m)]])


def test_generated_q_is_symmetric_psd_lower_csc():
    lp = qp(0)
    cp, ri = lp["q_colptr"], lp["q_rowidx"]
    for j in range(lp["n"]):
        rows = ri[cp[j]:cp[j + 1]]
        assert np.all(rows >= j) and np.all(np.diff(rows) > 0)
    ev = np.linalg.eigvalsh(W.q_dense(lp))
    assert ev.min() >= -1e-12 * max(1.0, ev.max())
    assert cp[-1] > lp["n"] // 2  # couplings, not just a diagonal


@pytest.mark.parametrize("seed", range(6))
def test_qp_symbolic_matches_brute_force(seed):
    lp = qp(seed, m=12 + seed, n=25 + 2 * seed, density=0.15, window=4)
    S = O.Sym(lp)
    A = dense_A(lp) != 0
    m, n = A.shape
    P = np.zeros((n + m, n + m), bool)
    P[n:, :n] = A
    P[:n, n:] = A.T
    P[:n, :n] = W.q_dense(lp) != 0
    np.fill_diagonal(P, True)
    L, parent, cc = brute_symbolic(P, S.perm())
    assert np.array_equal(S.parent(), parent)
    assert np.array_equal(S.colcount(), cc)
    assert S.nnzL == L.sum()


@pytest.mark.parametrize("seed", range(6))
def test_qp_reconstruction_and_inertia(seed):
    lp = qp(seed, trange=(1e-4, 1e4))
    S = O.Sym(lp)
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"], opts=O.default_opts(nb=4 + seed))
    ex = F.export()
    K = dense_K_qp(lp, lp["theta"], lp["rho"], lp["delta"])
    fp = ex["fperm"]
    Kp = K[np.ix_(fp, fp)] + np.diag(ex["edyn"])
    D = np.diag(ex["d"])
    for k in np.nonzero(ex["ptype"] == 1)[0]:
        D[k + 1, k] = D[k, k + 1] = ex["doff"][k]
    Lm = ex["L"]
    R = Kp - Lm @ D @ Lm.T
    growth = np.abs(Lm) @ np.abs(D) @ np.abs(Lm.T)
    assert np.abs(R).max() <= 50 * S.N * U * max(np.abs(Kp).max(), growth.max())
    st = F.stats()
    ev = np.linalg.eigvalsh(K)
    assert (st["nneg"], st["npos"]) == (lp["n"], lp["m"]) == ((ev < 0).sum(), (ev > 0).sum())
    assert np.isclose(F.knorm(), np.abs(K).sum(axis=0).max(), rtol=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_qp_solution_vs_lapack(seed):
    lp = qp(seed, m=40, n=90, trange=(1e-2, 1e2))
    g = W.rng(61, seed)
    r7, r1 = g.standard_normal(lp["n"]), g.standard_normal(lp["m"])
    S = O.Sym(lp)
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"])
    res = F.solve(r7, r1)
    K = dense_K_qp(lp, lp["theta"], lp["rho"], lp["delta"])
    b = np.concatenate([r7, r1])
    x = np.linalg.solve(K, b)
    xo = np.concatenate([res["dx"][:, 0], res["dy"][:, 0]])
    assert np.abs(xo - x).max() / np.abs(x).max() <= 10 * np.linalg.cond(K) * U
    assert res["berr_nw"][0] <= 1e-12


def test_qp_residual_matches_dense_definition():
    lp = qp(9)
    g = W.rng(62)
    N = lp["n"] + lp["m"]
    x, b = g.standard_normal(N), g.standard_normal(N)
    r, nw, cw, kn = O.residual(lp, lp["theta"], lp["rho"], lp["delta"], x, b)
    K = dense_K_qp(lp, lp["theta"], lp["rho"], lp["delta"])
    assert np.allclose(r, b - K @ x, rtol=1e-12, atol=1e-12 * np.abs(K).max())
    assert np.isclose(kn, np.abs(K).sum(axis=0).max(), rtol=1e-13)
    want_nw = np.abs(b - K @ x).max() / (np.abs(K).sum(1).max() * np.abs(x).max() + np.abs(b).max())
    assert np.isclose(nw, want_nw, rtol=1e-10)
    den = np.abs(K) @ np.abs(x) + np.abs(b)
    assert np.isclose(cw, (np.abs(b - K @ x) / den).max(), rtol=1e-10)


def test_diagonal_q_is_the_lp_with_shifted_theta():
    """Q = diag(q): the (1,1) block -(diag(q) + Theta^-1 + rho I) is the LP's with
    1/Theta'_j = 1/Theta_j + q_j, so both give the same direction (to rounding)."""
    lp = random_lp(77, 30, 70, 0.08, W.AS, trange=(1e-2, 1e2))
    g = W.rng(63)
    q = g.uniform(0.0, 2.0, lp["n"])
    qp_lp = W.LP(dict(lp, q_colptr=np.arange(lp["n"] + 1, dtype=np.int64),
                      q_rowidx=np.arange(lp["n"], dtype=np.int32), q_val=q))
    r7, r1 = g.standard_normal(lp["n"]), g.standard_normal(lp["m"])
    Fq = O.Num(O.Sym(qp_lp), lp["val"], lp["theta"], lp["rho"], lp["delta"]).solve(r7, r1)
    theta2 = 1.0 / (1.0 / lp["theta"] + q)
    Fl = O.Num(O.Sym(lp), lp["val"], theta2, lp["rho"], lp["delta"]).solve(r7, r1)
    for key in ("dx", "dy"):
        assert np.allclose(Fq[key], Fl[key], rtol=1e-9, atol=1e-9 * np.abs(Fl[key]).max())


def test_qp_rejects_bad_q_pattern():
    lp = qp(1)
    bad = W.LP(dict(lp, q_rowidx=lp["q_rowidx"].copy()))
    j = int(np.flatnonzero(np.diff(lp["q_colptr"]) >= 2)[0])
    e = int(lp["q_colptr"][j])
    bad["q_rowidx"][e], bad["q_rowidx"][e + 1] = bad["q_rowidx"][e + 1], bad["q_rowidx"][e]  # unsorted
    with pytest.raises(ValueError):
        O.Sym(bad)
