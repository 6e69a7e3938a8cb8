"""Pins of the CPU oracle against things other than itself (no GPU needed).

Each test names what fixes the expected value: brute-force elimination, LAPACK, eigenvalue
counts, closed forms derived by hand from the paper's formulas, or the paper's own text.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def dense_A(lp):
    A = np.zeros((lp["m"], lp["n"]))
    cp, ri, v = lp["colptr"], lp["rowidx"], lp["val"]
    for j in range(lp["n"]):
        A[ri[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
    return A


def dense_K(lp, theta, rho, delta):
    """K_static straight from equation (regul_matrix)."""
    A = dense_A(lp)
    m, n = A.shape
    if lp["mode"] == W.AS:
        return np.block([[-np.diag(1.0 / theta + rho), A.T], [A, delta * np.eye(m)]])
    tt = 1.0 / (1.0 / theta + rho)
    return (A * tt) @ A.T + delta * np.eye(m)


def lp_from_dense(A, mode, theta, rho, delta, name="dense"):
    m, n = A.shape
    cols = [np.nonzero(A[:, j])[0] for j in range(n)]
    colptr = np.zeros(n + 1, np.int64)
    for j in range(n):
        colptr[j + 1] = colptr[j] + len(cols[j])
    rowidx = np.concatenate(cols).astype(np.int32)
    val = np.concatenate([A[c, j] for j, c in enumerate(cols)])
    return W.LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=np.asarray(theta, float),
                rho=rho, delta=delta, mode=mode, name=name)


def random_lp(seed, m, n, density, mode, trange=(1e-3, 1e3), rho=1e-8, delta=1e-8):
    g = W.rng(99, seed)
    r, c = W.random_lp_pattern(g, m, n, density)
    A = np.zeros((m, n))
    A[r, c] = g.standard_normal(len(r))
    A[A == 0] = 0
    mask = np.zeros((m, n), bool)
    mask[r, c] = True
    A[mask & (A == 0)] = 1.0
    theta = W.log_uniform(g, *trange, n)
    return lp_from_dense(A, mode, theta, rho, delta, name=f"rand{seed}")


def k_pattern(lp):
    """Boolean adjacency of K (with diagonal) in original numbering."""
    A = dense_A(lp) != 0
    m, n = A.shape
    if lp["mode"] == W.AS:
        N = n + m
        P = np.zeros((N, N), bool)
        P[n:, :n] = A
        P[:n, n:] = A.T
    else:
        P = (A.astype(int) @ A.T.astype(int)) > 0
    np.fill_diagonal(P, True)
    return P


def brute_symbolic(P, perm):
    """Dense boolean elimination of the permuted pattern: L pattern, etree, column counts."""
    Q = P[np.ix_(perm, perm)].copy()
    N = len(perm)
    L = np.tril(Q)
    for k in range(N):
        rows = np.nonzero(L[k + 1:, k])[0] + k + 1
        for a in rows:
            L[rows[rows >= a], a] = True
    parent = np.full(N, -1)
    for j in range(N):
        below = np.nonzero(L[j + 1:, j])[0]
        if len(below):
            parent[j] = j + 1 + below[0]
    colcount = L.sum(axis=0)
    return L, parent, colcount


# ---------------------------------------------------------------- symbolic analysis

@pytest.mark.parametrize("seed", range(12))
def test_symbolic_matches_brute_force(seed):
    g = W.rng(7, seed)
    m = int(g.integers(5, 30))
    n = int(g.integers(m, 2 * m + 1))
    mode = W.AS if seed % 2 else W.NE
    lp = random_lp(seed, m, n, 0.15, mode)
    S = O.Sym(lp)
    perm = S.perm()
    assert sorted(perm.tolist()) == list(range(S.N))
    L, parent, cc = brute_symbolic(k_pattern(lp), perm)
    assert np.array_equal(S.parent(), parent)
    assert np.array_equal(S.colcount(), cc)
    assert S.nnzL == L.sum()
    # postorder: every subtree is a contiguous range ending at its root
    size = np.ones(S.N, int)
    for j in range(S.N):
        if parent[j] >= 0:
            assert parent[j] > j
            size[parent[j]] += size[j]
    first = np.arange(S.N) - size + 1
    for j in range(S.N):
        if parent[j] >= 0:
            assert first[parent[j]] <= first[j] and j < parent[j]
    # fundamental supernodes from the definition
    nk = np.bincount(parent[parent >= 0], minlength=S.N)
    starts = [j for j in range(S.N)
              if not (j > 0 and parent[j - 1] == j and nk[j] == 1 and cc[j - 1] == cc[j] + 1)]
    assert S.snptr()[:-1].tolist() == starts
    # front rows = pivot columns + structure of the last column
    rp, rows = S.front_rows()
    snp = S.snptr()
    for s in range(S.nsuper):
        last = snp[s + 1] - 1
        want = list(range(snp[s], snp[s + 1])) + (np.nonzero(L[last + 1:, last])[0] + last + 1).tolist()
        assert rows[rp[s]:rp[s + 1]].tolist() == want


def test_min_degree_fill_matches_dense_minimum_degree():
    """Fill of the oracle's ordering equals that of a dense-matrix minimum degree."""
    for seed in range(6):
        lp = random_lp(100 + seed, 20, 40, 0.1, W.AS if seed % 2 else W.NE)
        P = k_pattern(lp)
        G = P.copy()
        np.fill_diagonal(G, False)
        alive = np.ones(len(G), bool)
        order = []
        for _ in range(len(G)):
            deg = np.where(alive, (G & alive).sum(axis=1), 1 << 30)
            v = int(np.argmin(deg))  # lowest index on ties
            order.append(v)
            nb = np.nonzero(G[v] & alive)[0]
            G[np.ix_(nb, nb)] = True
            np.fill_diagonal(G, False)
            alive[v] = False
        Lb, _, _ = brute_symbolic(P, np.array(order))
        assert O.Sym(lp).nnzL == Lb.sum()


def test_paper_six_node_etree():
    g = json.load(open(os.path.join(GOLD, "etree_6node.json")))
    A = np.zeros((6, 5))
    for j, (a, b) in enumerate([(1, 3), (2, 3), (3, 6), (4, 5), (5, 6)]):
        A[a - 1, j] = 1.0
        A[b - 1, j] = 1.0
    lp = lp_from_dense(A, W.NE, np.ones(5), 0.0, 1.0)
    S = O.Sym(lp, perm=np.arange(6))
    par = S.parent()
    assert S.perm().tolist() == list(range(6))
    for k, v in g["parent_1based"].items():
        assert par[int(k) - 1] == v - 1


# ---------------------------------------------------------------- numeric factorisation

def _factor(lp, theta=None, opts=None, perm=None):
    theta = lp["theta"] if theta is None else theta
    S = O.Sym(lp, perm=perm)
    F = O.Num(S, lp["val"], theta, lp["rho"], lp["delta"], opts=opts)
    return S, F


@pytest.mark.parametrize("seed", range(8))
def test_reconstruction_and_inertia(seed):
    mode = W.AS if seed % 2 else W.NE
    lp = random_lp(200 + seed, 40, 90, 0.06, mode, trange=(1e-4, 1e4))
    S, F = _factor(lp, opts=O.default_opts(nb=4 + seed))  # small windows: several per front
    ex = F.export()
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    fp = ex["fperm"]
    Kp = K[np.ix_(fp, fp)] + np.diag(ex["edyn"])
    N = S.N
    D = np.diag(ex["d"])
    for k in np.nonzero(ex["ptype"] == 1)[0]:
        D[k + 1, k] = D[k, k + 1] = ex["doff"][k]
    Lm = ex["L"]
    assert np.allclose(np.diag(Lm), 1.0)
    assert np.all(np.triu(Lm, 1) == 0)
    R = Kp - Lm @ D @ Lm.T
    growth = np.abs(Lm) @ np.abs(D) @ np.abs(Lm.T)
    assert np.abs(R).max() <= 50 * N * U * max(np.abs(Kp).max(), growth.max())
    # inertia: Sylvester + Proposition 1 (AS: n negative, m positive; NE: m positive)
    st = F.stats()
    ev = np.linalg.eigvalsh(K)
    assert st["nneg"] == (ev < 0).sum() and st["npos"] == (ev > 0).sum()
    if mode == W.AS:
        assert (st["nneg"], st["npos"]) == (lp["n"], lp["m"])
    else:
        assert (st["nneg"], st["npos"]) == (0, lp["m"])


def textbook_block_ldlt(M, ptype):
    """Unpivoted dense block LDL^T with a given 1x1/2x2 partition (no decisions)."""
    M = M.copy()
    N = len(M)
    L = np.eye(N)
    D = np.zeros((N, N))
    k = 0
    while k < N:
        b = 2 if ptype[k] == 1 else 1
        Dk = M[k:k + b, k:k + b].copy()
        D[k:k + b, k:k + b] = Dk
        Lk = np.linalg.solve(Dk, M[k + b:, k:k + b].T).T
        L[k + b:, k:k + b] = Lk
        M[k + b:, k + b:] -= Lk @ Dk @ Lk.T
        k += b
    return L, D


@pytest.mark.parametrize("seed", range(4))
def test_factor_is_the_unique_ldlt_of_its_pivot_sequence(seed):
    lp = random_lp(300 + seed, 30, 60, 0.08, W.AS, trange=(1e-2, 1e2))
    S, F = _factor(lp, opts=O.default_opts(nb=8))
    ex = F.export()
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    fp = ex["fperm"]
    Lt, Dt = textbook_block_ldlt(K[np.ix_(fp, fp)] + np.diag(ex["edyn"]), ex["ptype"])
    scale = np.abs(Lt).max()
    assert np.abs(ex["L"] - Lt).max() <= 1e4 * U * scale * S.N
    assert np.allclose(ex["d"], np.diag(Dt), rtol=1e-10, atol=0)


def test_solution_vs_lapack_small_workload():
    lp = W.ne_random()
    S, F = _factor(lp)
    res = F.solve(lp["r7"], lp["r1"])
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    x = np.linalg.solve(K, lp["r1"][:, 0])
    kappa = np.linalg.cond(K)
    err = np.abs(res["dy"][:, 0] - x).max() / np.abs(x).max()
    assert err <= 10 * kappa * U
    assert res["berr_nw"][0] <= 1e-12
    st = F.stats()
    assert (st["nneg"], st["npos"]) == (0, lp["m"])


def test_small_staircase_vs_lapack_and_berr():
    lp = W.as_staircase(periods=3, rows=40, cols=80, link_cols=8)
    S, F = _factor(lp)
    res = F.solve(lp["r7"], lp["r1"])
    assert res["berr_nw"][0] <= 1e-12
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    b = np.concatenate([lp["r7"][:, 0], lp["r1"][:, 0]])
    xo = np.concatenate([res["dx"][:, 0], res["dy"][:, 0]])
    r = b - K @ xo
    assert np.abs(r).max() / (np.abs(K).sum(1).max() * np.abs(xo).max() + np.abs(b).max()) <= 1e-12
    st = F.stats()
    assert (st["nneg"], st["npos"]) == (lp["n"], lp["m"])


def test_residual_function_matches_dense_definition():
    for mode in (W.AS, W.NE):
        lp = random_lp(400 + mode, 25, 50, 0.1, mode)
        g = W.rng(5, mode)
        N = lp["n"] + lp["m"] if mode == W.AS else lp["m"]
        x = g.standard_normal(N)
        b = g.standard_normal(N)
        r, nw, cw, kn = O.residual(lp, lp["theta"], lp["rho"], lp["delta"], x, b)
        K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
        assert np.allclose(r, b - K @ x, rtol=1e-12, atol=1e-12 * np.abs(K).max())
        assert np.isclose(kn, np.abs(K).sum(axis=0).max(), rtol=1e-13)
        want_nw = np.abs(b - K @ x).max() / (np.abs(K).sum(1).max() * np.abs(x).max() + np.abs(b).max())
        assert np.isclose(nw, want_nw, rtol=1e-10)
        den = np.abs(K) @ np.abs(x) + np.abs(b)
        assert np.isclose(cw, (np.abs(b - K @ x) / den).max(), rtol=1e-10)


def test_componentwise_error_small_denominator_substitution():
    """The componentwise backward error's substitution for tiny denominators (Section 4.5
    cites Arioli, Demmel and Duff; the threshold 1000 N u (||K_i||_1 ||x||_inf + |b_i|) is our
    reading).  K = I (NE, A = I, Theta = 1, rho = delta = 0), b = [1, 0]:
    * x = [1, 1e-300]: r = [0, -1e-300]; row 1's denominator |K||x| + |b| = 1e-300 is below the
      threshold 2000 u, so it becomes |K||x| + ||x||_inf |K|e = 1 + 1e-300 and the row's error is
      1e-300 (it would be 1 without the substitution);
    * x = [1, 1e-12]: the denominator 1e-12 is above the threshold, the row's error is
      1e-12 / 1e-12 = 1.
    The normwise error is ||r||_inf / (||K|| ||x|| + ||b||) = |x_1| / 2 in both cases."""
    lp = lp_from_dense(np.eye(2), W.NE, np.ones(2), 0.0, 0.0)
    b = np.array([1.0, 0.0])
    r, nw, cw, kn = O.residual(lp, lp["theta"], 0.0, 0.0, np.array([1.0, 1e-300]), b)
    assert kn == 1.0
    assert r.tolist() == [0.0, -1e-300]
    assert cw == 1e-300
    assert nw == 1e-300 / 2
    r, nw, cw, kn = O.residual(lp, lp["theta"], 0.0, 0.0, np.array([1.0, 1e-12]), b)
    assert cw == 1.0
    assert nw == 1e-12 / 2


def test_ne_equals_as_for_the_same_regularised_system():
    """Equations (augsys)/(normeq) with (regul_matrix): both give the same (dx, dy)."""
    g = W.rng(11)
    m, n = 30, 70
    lp_ne = random_lp(500, m, n, 0.1, W.NE, trange=(1e-2, 1e2), rho=1e-6, delta=1e-6)
    lp_as = dict(lp_ne)
    lp_as["mode"] = W.AS
    lp_as = W.LP(lp_as)
    r7 = g.standard_normal((n, 1))
    r1 = g.standard_normal((m, 1))
    _, Fn = _factor(lp_ne)
    _, Fa = _factor(lp_as)
    rn = Fn.solve(r7, r1)
    ra = Fa.solve(r7, r1)
    K = dense_K(lp_as, lp_as["theta"], lp_as["rho"], lp_as["delta"])
    kappa = np.linalg.cond(K)
    for key in ("dx", "dy"):
        a, b = rn[key][:, 0], ra[key][:, 0]
        assert np.abs(a - b).max() <= 100 * kappa * U * np.abs(b).max()


def test_no_dynamic_regularisation_on_well_conditioned_qd():
    """Proposition 1: eliminating a QD pivot keeps the Schur complement QD, so neither
    Proposition 3 nor the sign rule fires in (near) exact arithmetic.  The pivot tests read
    unregularised values, so a dual pivot whose diagonal is still exactly 0 (eliminated
    before its primal neighbours) may be lifted; that perturbation is at most eps*||K||_1."""
    for seed in range(4):
        lp = random_lp(600 + seed, 40, 80, 0.08, W.AS, trange=(0.1, 10), rho=1e-2, delta=1e-2)
        _, F = _factor(lp, opts=O.default_opts(nb=8))
        st = F.stats()
        assert st["nprop3"] == 0 and st["nsign"] == 0
        assert st["max_edyn"] <= 2.0 ** -52 * F.knorm()


# ---------------------------------------------------------------- closed forms

def test_closed_form_ne_identity_pair():
    """A = [I I], Theta = I, NE: K = 2I + delta I, so L = I and D = 2 + delta."""
    m = 7
    A = np.hstack([np.eye(m), np.eye(m)])
    delta = 1e-3
    lp = lp_from_dense(A, W.NE, np.ones(2 * m), 0.0, delta)
    S, F = _factor(lp)
    ex = F.export()
    assert np.array_equal(ex["L"], np.eye(m))
    assert np.all(ex["d"] == 2.0 + delta)
    assert F.stats()["npos"] == m


@pytest.mark.parametrize("theta", [0.25, 0.5, 1.0])
def test_closed_form_as_identity_small_theta(theta):
    """A = I, Theta = theta I, AS, theta <= 1: branch (b) on x_j, then y_j.
    D_x = -(1/theta + rho), D_y = delta + theta/(1 + rho theta), L_yx = -theta/(1+rho theta)."""
    m = 5
    rho, delta = 1e-3, 2e-3
    lp = lp_from_dense(np.eye(m), W.AS, np.full(m, theta), rho, delta)
    S, F = _factor(lp)
    ex = F.export()
    assert S.nsuper == m
    st = F.stats()
    assert st["n2x2"] == 0 and (st["nneg"], st["npos"]) == (m, m)
    fp = ex["fperm"]
    for k in range(0, 2 * m, 2):
        assert fp[k] < m and fp[k + 1] >= m  # x_j then y_j
        assert np.isclose(ex["d"][k], -(1 / theta + rho), rtol=1e-15)
        assert np.isclose(ex["d"][k + 1], delta + theta / (1 + rho * theta), rtol=1e-14)
        assert np.isclose(ex["L"][k + 1, k], -theta / (1 + rho * theta), rtol=1e-14)


@pytest.mark.parametrize("theta", [2.0, 10.0, 1e3])
def test_closed_form_as_identity_large_theta(theta):
    """theta >= 2: |1/theta| < alpha, gamma_r = 1, |F_rr| = 0, so branch (e): one 2x2 block
    [[-(1/theta+rho), 1], [1, delta]] per pair with inertia (1 -, 1 +)."""
    m = 4
    rho, delta = 1e-3, 2e-3
    lp = lp_from_dense(np.eye(m), W.AS, np.full(m, theta), rho, delta)
    S, F = _factor(lp)
    ex = F.export()
    st = F.stats()
    assert st["n2x2"] == m and (st["nneg"], st["npos"]) == (m, m)
    for k in range(0, 2 * m, 2):
        assert ex["ptype"][k] == 1 and ex["ptype"][k + 1] == 2
        assert ex["d"][k] == -(1 / theta + rho) and ex["d"][k + 1] == delta
        assert ex["doff"][k] == 1.0


# ---------------------------------------------------------------- Bunch-Kaufman branches (Section 4.5)

ALPHA = (1 + np.sqrt(17)) / 8


def test_alpha_is_the_papers_constant():
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    assert g["bk_alpha"]["value_expr"] == "(sqrt(17)+1)/8"
    assert O.default_opts().alpha == (np.sqrt(17) + 1) / 8


def _ff(F, sigma, knorm=1.0, p=None, **kw):
    F = np.asfortranarray(np.array(F, float))
    f = len(F)
    sigma = np.array(sigma, np.int8)
    shift = np.zeros(f)
    return O.front_factor(F, f if p is None else p, sigma, shift, knorm,
                          O.default_opts(presort=0, **kw))


def test_bk_branch_e_two_by_two():
    r = _ff([[0, 1], [1, 0]], [-1, 1])
    assert r["ptype"].tolist() == [1, 2]
    assert r["d"].tolist() == [0.0, 0.0] and r["doff"][0] == 1.0
    assert r["stats"]["nneg"] == 1 and r["stats"]["npos"] == 1


def test_bk_branch_a_lift():
    tiny = 1e-30
    r = _ff([[tiny, tiny], [tiny, -tiny]], [1, -1], knorm=1.0)
    eps = 2.0 ** -52
    assert r["stats"]["nlift"] >= 1
    assert r["d"][0] == eps  # sigma_0 * eps * ||K||_1
    assert r["edyn"][0] == eps - tiny


def test_bk_branch_b_dominant_diagonal():
    r = _ff([[4, 1, 0.5], [1, 3, 0.2], [0.5, 0.2, 2]], [1, 1, 1])
    assert r["perm"][:3].tolist() == [0, 1, 2]
    assert r["ptype"].tolist() == [0, 0, 0]
    assert r["d"][0] == 4.0


def test_bk_branch_c():
    # |F00|=1 < alpha*2, gamma_r = 10, 1*10 >= alpha*4: 1x1 at k without a swap
    r = _ff([[1, 2, 0], [2, 10, 10], [0, 10, 10]], [1, 1, 1])
    assert r["perm"][0] == 0 and r["ptype"][0] == 0 and r["d"][0] == 1.0


def test_bk_branch_d_swap():
    # gamma_r = 2, 1*2 < alpha*4, |F11| = 10 >= alpha*2: swap r <-> k, 1x1 of value 10
    r = _ff([[1, 2, 0], [2, 10, 1], [0, 1, 3]], [1, 1, 1])
    assert r["perm"][:2].tolist() == [1, 0] and r["d"][0] == 10.0 and r["ptype"][0] == 0
    assert r["stats"]["nbkd"] == 1


def test_two_by_two_with_zero_determinant_falls_back_to_a_lift():
    """Reading of the 2x2 case (the paper gives no rule for a singular block): [[0, 1], [1, 0]]
    with both static shifts +1 reaches branch (e) (|F00| = |F11| = 0 < alpha * 1), and the
    shifted block [[1, 1], [1, 1]] has det = 0 exactly.  By hand: the pivot at 0 is lifted to
    sigma * eps * ||K||_1 = 2^-52, shifted to d0 = 1 + 2^-52 (exact in FP64), E_dyn = 2^-52;
    the second pivot is 1 - 1/(1 + 2^-52) = 2^-52 to first order, positive as its sign."""
    F = np.asfortranarray(np.array([[0.0, 1.0], [1.0, 0.0]]))
    eps = 2.0 ** -52
    r = O.front_factor(F, 2, np.array([1, 1], np.int8), np.array([1.0, 1.0]), 1.0,
                       O.default_opts(presort=0))
    assert r["ptype"].tolist() == [0, 0]
    assert r["stats"]["n2x2"] == 0 and r["stats"]["nlift"] == 1
    assert r["d"][0] == 1.0 + eps
    assert r["edyn"][0] == eps
    assert r["edyn"][1] == 0.0 and 0.0 < r["d"][1] <= 2 * eps
    assert r["stats"]["npos"] == 2 and r["stats"]["nneg"] == 0
    # with a nonzero determinant the same window is a 2x2 block (branch e proper)
    r2 = O.front_factor(F, 2, np.array([1, 1], np.int8), np.array([0.5, 0.5]), 1.0,
                        O.default_opts(presort=0))
    assert r2["ptype"].tolist() == [1, 2] and r2["d"].tolist() == [0.5, 0.5] and r2["doff"][0] == 1.0


def test_bk_branch_e_with_three():
    r = _ff([[1, 2, 0], [2, 1, 0], [0, 0, 3]], [1, -1, 1])
    assert r["ptype"].tolist() == [1, 2, 0]
    assert r["d"][:2].tolist() == [1.0, 1.0] and r["doff"][0] == 2.0


def test_presort_puts_largest_diagonal_first():
    F = [[1, 0.1, 0.1], [0.1, 5, 0.1], [0.1, 0.1, 3]]
    f = np.asfortranarray(np.array(F, float))
    r = O.front_factor(f, 3, np.ones(3, np.int8), np.zeros(3), 1.0, O.default_opts())
    assert r["perm"][0] == 1 and r["d"][0] == 5.0


def test_proposition3_trigger_closed_form():
    """|p| < q^2/|M_jj| for a same-sign j: the pivot becomes sigma*beta exactly."""
    rho = 1e-3
    F = np.asfortranarray(np.array([[-1, 0.1, 0.5], [0.1, -3, 0], [0.5, 0, -0.01]]))
    sig = np.array([-1, -1, -1], np.int8)
    sh = np.full(3, -rho)
    r = O.front_factor(F, 3, sig, sh, 1.0, O.default_opts(presort=0))
    beta = max(0.1 ** 2 / (3 + rho), 0.5 ** 2 / (0.01 + rho))
    assert r["stats"]["nprop3"] >= 1
    assert r["d"][0] == -beta
    assert r["edyn"][0] == -beta - (-1 - rho)


def test_sign_rule_flips_wrong_sign_pivot():
    """A negative-block pivot that comes out positive is forced back to its sign."""
    F = np.asfortranarray(np.array([[2.0]]))
    r = O.front_factor(F, 1, np.array([-1], np.int8), np.zeros(1), 1.0, O.default_opts())
    assert r["stats"]["nsign"] == 1 and r["d"][0] == -2.0


def test_pivot_window_limits_the_search():
    """Section 4.5: only the diagonal block is searched; with nb=1 no 2x2 can form."""
    F = [[0, 1], [1, 0]]
    r = _ff(F, [-1, 1], nb=1)
    assert r["ptype"].tolist() == [0, 0]
    assert r["stats"]["nlift"] == 1 or r["stats"]["nsign"] >= 1


def test_proposition3_threshold_is_exact():
    """beta slightly above |d| must fire; beta slightly below must not."""
    rho = 1e-3
    for q2, fires in ((0.25, True), (0.15, False)):
        F = np.asfortranarray(np.array([[-1.0, np.sqrt(q2)], [np.sqrt(q2), -0.2]]))
        r = O.front_factor(F, 2, np.array([-1, -1], np.int8), np.full(2, -rho), 1.0,
                           O.default_opts(presort=0))
        beta = F[1, 0] ** 2 / (0.2 + rho)
        assert (r["stats"]["nprop3"] == 1) == fires
        assert r["d"][0] == (-beta if fires else -(1 + rho))


def _front_reconstruction(F0, sigma, shift, p, r):
    """P F0 P^T + diag(shift+edyn on pivots) == [L11;L21] D [L11;L21]^T + [0 0; 0 S]."""
    f = len(F0)
    perm = r["perm"]
    Fp = F0[np.ix_(perm, perm)].copy()
    Fp[np.arange(p), np.arange(p)] += shift[perm[:p]] + r["edyn"]
    Lf = np.tril(r["F"][:, :p], -1)
    Lf[np.arange(p), np.arange(p)] = 1.0
    D = np.diag(r["d"])
    for k in np.nonzero(r["ptype"] == 1)[0]:
        D[k + 1, k] = D[k, k + 1] = r["doff"][k]
    S = np.zeros((f, f))
    S[p:, p:] = r["F"][p:, p:]
    R = Fp - (Lf @ D @ Lf.T + S)
    growth = np.abs(Lf) @ np.abs(D) @ np.abs(Lf.T)
    return np.abs(R).max() / max(np.abs(Fp).max(), growth.max())


@pytest.mark.parametrize("seed", range(6))
def test_front_partial_factor_reconstruction_with_2x2(seed):
    """Dense fronts with weak diagonals force 2x2 pivots that have rows below them."""
    f, p = 40, 24
    F0, sigma = W.dense_front(f, p, seed=seed, dmin=1e-3, dmax=1e-2)
    shift = np.where(sigma < 0, -1e-6, 1e-6)
    r = O.front_factor(F0, p, sigma, shift, np.abs(F0).sum(0).max(), O.default_opts(nb=8))
    assert r["stats"]["n2x2"] >= 2
    assert _front_reconstruction(F0, sigma, shift, p, r) <= 100 * f * U
    # the returned signs/shifts are the inputs permuted like the rows
    assert np.array_equal(r["sigma"], sigma[r["perm"]])
